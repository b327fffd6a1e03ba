"""Serving loop with continuous batching.

Requests (a problem, an initial state and a number of SSP-RK3 steps at
CFL 1/2) arrive over time.  The server admits waiting requests in arrival
order as soon as their HBM footprint (state + the handle's two stage
buffers) fits in the budget and, by default, while the admitted requests
hold at most about one GPU-filling solve of nodes (2^21; a larger request
is admitted alone).  Small requests thus batch together, and large ones
are not stretched by sharing every tick with others.  It keeps every
admitted state on the device, and on every tick
advances all admitted requests by one step: the requests of one equation
family form a batch (one HIP graph per step with a work-list launch per
degree and stage), the families' graphs are enqueued back to back on one
stream.  A request leaves as soon as its last step is enqueued; its
completion time is the GPU time of that step's end (HIP event), so
time-to-solution = completion - arrival.

The same request stream can be run FIFO through the plain path (one
request at a time, one solve per launch) for comparison.  Every request's
result is bitwise the same alone and in the mix, because a batched step
equals the plain step of each solve.
"""
import time
from dataclasses import dataclass, field
from typing import Dict, List

import numpy as np

from . import idp_dg
from .workloads import Request, initial_state_device


@dataclass
class Done:
    rid: int
    arrival: float
    admitted: float
    finished: float
    nodes: int
    steps: int
    result: object = None

    @property
    def tts(self) -> float:
        return self.finished - self.arrival


def footprint_bytes(req: Request) -> int:
    prob = req.problem()
    return 3 * 8 * prob.nc * prob.num_nodes + 4096


class Server:
    def __init__(self, hbm_budget: int, cfl: float = 0.5, keep_results: bool = False,
                 max_active: int = 0, max_active_nodes: int = 1 << 21):
        import torch
        self.torch = torch
        self.max_active = int(max_active)   # 0: no cap on concurrently served requests
        # 0: no cap; else a request is admitted only while the admitted
        # requests' nodes stay within it (or nothing else is admitted)
        self.max_active_nodes = int(max_active_nodes)
        self.budget = int(hbm_budget)
        self.cfl = cfl
        self.keep = keep_results
        self.stream = torch.cuda.current_stream()

    def _clock_ms(self, ev):
        return self.ref.elapsed_time(ev) * 1e-3

    def run(self, requests: List[Request]) -> List[Done]:
        torch = self.torch
        pending = sorted(requests, key=lambda r: r.arrival)
        active: Dict[int, dict] = {}
        used = 0
        batches: Dict[int, tuple] = {}     # family -> (member ids, Batch)
        finishing = []                     # (request record, end event)
        out: List[Done] = []
        torch.cuda.synchronize()
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record(self.stream)
        t0 = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - t0
            # admission: FIFO, as long as the footprint fits
            while (pending and pending[0].arrival <= now and used + footprint_bytes(pending[0]) <= self.budget
                   and (self.max_active <= 0 or len(active) < self.max_active)
                   and (self.max_active_nodes <= 0 or not active
                        or sum(a["req"].problem().num_nodes for a in active.values())
                        + pending[0].problem().num_nodes <= self.max_active_nodes)):
                req = pending.pop(0)
                sv = idp_dg.Solver(req.problem(), stream=self.stream, workspace=True)
                u = initial_state_device(req)
                active[req.rid] = {"req": req, "sv": sv, "u": u, "left": req.steps,
                                   "admitted": time.perf_counter() - t0}
                used += footprint_bytes(req)
            if not active:
                if pending:
                    wait = pending[0].arrival - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                continue
            # one step of every admitted request, batched per family
            fams: Dict[int, List[int]] = {}
            for rid, a in active.items():
                fams.setdefault(idp_dg.family_of(a["req"].problem()), []).append(rid)
            for fam, ids in fams.items():
                ids = sorted(ids)
                cur = batches.get(fam)
                members = [active[i]["sv"] for i in ids]
                if cur is None:
                    batches[fam] = [ids, idp_dg.Batch(members, stream=self.stream)]
                elif cur[0] != ids:
                    cur[1].update(members)
                    cur[0] = ids
                batches[fam][1].step_cfl([active[i]["u"] for i in ids], self.cfl)
            # retire requests whose last step is now enqueued
            for rid in [r for r, a in active.items() if a["left"] == 1]:
                a = active.pop(rid)
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(self.stream)
                finishing.append((a, ev))
                used -= footprint_bytes(a["req"])
            for a in active.values():
                a["left"] -= 1
            # record finished requests whose work is complete
            still = []
            for a, ev in finishing:
                if ev.query():
                    out.append(self._done(a, ev))
                else:
                    still.append((a, ev))
            finishing = still
        for a, ev in finishing:
            ev.synchronize()
            out.append(self._done(a, ev))
        for ids, b in batches.values():
            b.close()
        return sorted(out, key=lambda d: d.rid)

    def _done(self, a, ev):
        req = a["req"]
        res = a["u"].cpu() if self.keep else None
        a["sv"].close()
        return Done(rid=req.rid, arrival=req.arrival, admitted=a["admitted"],
                    finished=self._clock_ms(ev), nodes=req.problem().num_nodes,
                    steps=req.steps, result=res)


def run_fifo_plain(requests: List[Request], cfl: float = 0.5, keep_results: bool = False):
    """The same stream, one request at a time through the plain path."""
    import torch
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    ref = torch.cuda.Event(enable_timing=True)
    ref.record(stream)
    t0 = time.perf_counter()
    out = []
    for req in sorted(requests, key=lambda r: r.arrival):
        wait = req.arrival - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        admitted = time.perf_counter() - t0
        sv = idp_dg.Solver(req.problem(), stream=stream, workspace=True)
        u = initial_state_device(req)
        for _ in range(req.steps):
            sv.step_cfl(u, cfl)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(stream)
        ev.synchronize()
        out.append(Done(rid=req.rid, arrival=req.arrival, admitted=admitted,
                        finished=ref.elapsed_time(ev) * 1e-3, nodes=req.problem().num_nodes,
                        steps=req.steps, result=u.cpu() if keep_results else None))
        sv.close()
    return out


def summarize(done: List[Done]) -> dict:
    tts = np.array([d.tts for d in done])
    span = max(d.finished for d in done) - min(d.arrival for d in done)
    dof = sum(3.0 * d.nodes * d.steps for d in done)
    return {"requests": len(done), "tts_s_p50": float(np.percentile(tts, 50)),
            "tts_s_p99": float(np.percentile(tts, 99)), "makespan_s": span,
            "dof_updates_per_s": dof / span}
