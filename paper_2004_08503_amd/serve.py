"""Serving loop with continuous batching.

Requests (a problem, an initial state and a number of SSP-RK3 steps at
CFL 1/2) arrive over time.  The server admits waiting requests in arrival
order as soon as their HBM footprint (state + the handle's two stage
buffers) fits in the budget.  By default a large request is also admitted
only while the admitted large requests hold at most about one GPU-filling
solve of nodes (2^21; a larger request runs alone).  Large requests are
thus not stretched by sharing every tick with each other, and a large
request that must wait holds back the large requests behind it.  Small
requests (at most 1/16 of that many nodes) are admitted as soon as they
fit, past a waiting large request, and are not counted against the cap.

Every admitted state stays on the device.  On every tick, with the
processor-sharing policy ("ps", the default), each admitted request
advances by one step; with the shortest-remaining-work policy ("srw"),
the admitted requests are taken in order of remaining work (nodes times
steps left) until the tick holds about one GPU-filling solve of nodes,
and only those advance (the others keep their state on the device and
wait); age_weight lowers a request's remaining work by that many seconds
per second since its arrival, so that a long wait raises its rank (pure
shortest-remaining-work first starves the largest requests under high
load).  In both:
- the requests of one equation family form a batch (a work-list launch
  per degree and stage);
- a family with one admitted request takes the plain path's graph;
- the families' steps are enqueued back to back on one stream.

A request leaves as soon as its last step is enqueued.  Its completion time
is the GPU time at the end of that step (HIP event), so time-to-solution =
completion - arrival.

The same request stream can be run FIFO through the plain path (one
request at a time, one solve per launch) for comparison.  Every request's
result is bitwise the same alone and in the mix, because a batched step
equals the plain step of each solve.
"""
import time
from dataclasses import dataclass, field
from typing import Dict, List

import numpy as np

from . import idp_dg, tuning
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
    """Device bytes a served request holds: its state and the workspace of
    its handle as Solver(workspace=True) allocates it (the library's
    workspace size for the problem plus 256 bytes of alignment slack)."""
    import ctypes
    prob = req.problem()
    ws = idp_dg.lib.idp_dg_workspace_bytes(ctypes.byref(idp_dg.make_desc(prob)))
    if ws < 0:
        raise ValueError("bad request problem: %s" % idp_dg.lib.idp_dg_last_error(None).decode())
    return 8 * prob.nc * prob.num_nodes + ws + 256


class Server:
    def __init__(self, hbm_budget: int, cfl: float = 0.5, keep_results: bool = False,
                 max_active: int = 0, max_active_nodes: int = 1 << 21, small_nodes: int = -1,
                 policy: str = "ps", tick_nodes: int = 1 << 21, age_weight: float = 0.0,
                 node_rate: float = 1.5e10):
        import torch
        self.torch = torch
        if policy not in ("ps", "srw"):
            raise ValueError("policy must be 'ps' or 'srw'")
        self.policy = policy
        # srw: the requests stepped in one tick hold about this many nodes
        self.tick_nodes = int(tick_nodes)
        # srw: a request's remaining work, in seconds at node_rate node-steps
        # per second (three stages per step), is lowered by age_weight times
        # the seconds since its arrival, so that a long wait raises its rank
        self.age_weight = float(age_weight)
        self.node_rate = float(node_rate)
        self.max_active = int(max_active)   # 0: no cap on concurrently served requests
        # 0: no cap; else a large request is admitted only while the admitted
        # large requests' nodes stay within it (or no other large one is
        # admitted)
        self.max_active_nodes = int(max_active_nodes)
        # requests of at most this many nodes are small: admitted as soon as
        # their footprint fits, past a large request that waits, and not
        # counted against max_active_nodes (-1: max_active_nodes / 16; 0: no
        # small class, every request waits its turn in arrival order)
        self.small_nodes = (self.max_active_nodes // 16 if small_nodes < 0 else int(small_nodes))
        self.budget = int(hbm_budget)
        self.cfl = cfl
        self.keep = keep_results
        self.stream = torch.cuda.current_stream()
        self.table = tuning.load_table()   # tile shapes measured on this device, if any

    def _clock_ms(self, ev):
        return self.ref.elapsed_time(ev) * 1e-3

    def run(self, requests: List[Request]) -> List[Done]:
        torch = self.torch
        pending = sorted(requests, key=lambda r: r.arrival)
        nxt = 0                            # next request to arrive
        waiting: List[Request] = []        # arrived, not admitted (arrival order)
        active: Dict[int, dict] = {}
        used = 0                           # bytes of the admitted requests
        large = 0                          # nodes of the admitted large requests
        groups: Dict[int, list] = {}       # family -> [member ids, Batch, state pointers]
        dirty = set()                      # families whose membership changed
        tick = 0
        self.peak_used = 0                 # most device bytes admitted at once
        finishing = []                     # (request record, end event)
        out: List[Done] = []
        torch.cuda.synchronize()
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record(self.stream)
        t0 = time.perf_counter()
        while nxt < len(pending) or waiting or active:
            now = time.perf_counter() - t0
            while nxt < len(pending) and pending[nxt].arrival <= now:
                waiting.append(pending[nxt])
                nxt += 1
            # admission in arrival order while the footprint and the caps
            # allow; a large request that must wait holds back the large
            # requests behind it, not the small ones
            large_blocked = False
            keep = []
            for req in waiting:
                prob = req.problem()
                fp = footprint_bytes(req)
                small = prob.num_nodes <= self.small_nodes
                ok = used + fp <= self.budget and not (0 < self.max_active <= len(active))
                if not small:
                    ok = ok and not large_blocked and not (
                        self.max_active_nodes > 0 and large > 0
                        and large + prob.num_nodes > self.max_active_nodes)
                    large_blocked = large_blocked or not ok
                if not ok:
                    keep.append(req)
                    continue
                sv = idp_dg.Solver(prob, stream=self.stream, workspace=True)
                if self.table:
                    tuning.apply_solver(sv, self.table)
                u = initial_state_device(req)
                fam = idp_dg.family_of(prob)
                active[req.rid] = {"req": req, "sv": sv, "u": u, "fam": fam, "fp": fp,
                                   "large": 0 if small else prob.num_nodes,
                                   "nodes": prob.num_nodes, "left": req.steps,
                                   "admitted": time.perf_counter() - t0}
                used += fp
                self.peak_used = max(self.peak_used, used)
                large += active[req.rid]["large"]
                dirty.add(fam)
            waiting = keep
            if not active and waiting and not any(
                    footprint_bytes(r) <= self.budget for r in waiting):
                raise ValueError("request %d needs %d bytes, more than the HBM budget"
                                 % (waiting[0].rid, footprint_bytes(waiting[0])))
            if not active:
                if nxt < len(pending):
                    wait = pending[nxt].arrival - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                continue
            # the requests that step this tick: all (ps), or those with the
            # least remaining work up to the tick's node budget (srw)
            if self.policy == "ps":
                run = set(active)
            else:
                run, held = set(), 0

                def rank(r):
                    a = active[r]
                    work = 3.0 * a["nodes"] * a["left"] / self.node_rate
                    return (work - self.age_weight * (now - a["req"].arrival), r)

                for rid in sorted(active, key=rank):
                    if run and held + active[rid]["nodes"] > self.tick_nodes:
                        continue
                    run.add(rid)
                    held += active[rid]["nodes"]
                for fam in {a["fam"] for a in active.values()} | set(groups):
                    g = groups.get(fam)
                    if g is None or g[0] != sorted(r for r in run if active[r]["fam"] == fam):
                        dirty.add(fam)
            # batches of the families whose membership changed
            for fam in dirty:
                ids = sorted(r for r in run if active[r]["fam"] == fam)
                g = groups.get(fam)
                if not ids:
                    if g is not None:
                        g[0], g[2] = [], None
                    continue
                members = [active[i]["sv"] for i in ids]
                if g is None:
                    g = groups[fam] = [ids, idp_dg.Batch(members, stream=self.stream), None]
                elif g[0] != ids:
                    g[1].update(members)
                    g[0] = ids
                g[2] = g[1].prepare([active[i]["u"] for i in ids])
            dirty.clear()
            # one step of every admitted request, batched per family; a
            # family with one admitted request takes the plain path (the
            # same step, bitwise, without the work-list indirection)
            for ids, b, ptrs in groups.values():
                if len(ids) == 1:
                    a = active[ids[0]]
                    a["sv"].step_cfl(a["u"], self.cfl)
                elif ids:
                    b.step_cfl_prepared(ptrs, self.cfl)
            # retire requests whose last step is now enqueued
            for rid in sorted(run):
                active[rid]["left"] -= 1
                if active[rid]["left"] > 0:
                    continue
                a = active.pop(rid)
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(self.stream)
                finishing.append((a, ev))
                used -= a["fp"]
                large -= a["large"]
                dirty.add(a["fam"])
            tick += 1
            # record finished requests whose work is complete
            if finishing:
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
        for ids, b, ptrs in groups.values():
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
    table = tuning.load_table()
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
        if table:
            tuning.apply_solver(sv, table)
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
