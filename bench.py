"""Benchmark of the limited SSP-RK3 stage: 2-D Euler, 256 x 256 elements,
p = 4 (1 638 400 Gauss-Lobatto nodes, 4 conserved components, FP64).

One step = the whole hot path: the low-order CFL bound reduced on the
device (dt = 1/2 of it, as in the paper's runs), then the three limited
stages.  K steps are timed between device synchronisations; every kernel is
bracketed by HIP events on the stream it runs on, which gives the stage
kernel's average duration for the roofline and the p50/p99 stage latency.

value = DOF (node) updates per second over the timed region:
3 * Nn * K / elapsed.  The rocprofv3 counter figures under profiles/ supply
the measured HBM traffic when they match the current kernel source.  The
benchmark solve uses its degree's default tile shape (config.tile_shape and
config.elements_per_workgroup; --tune runs the tile-shape tuner first).

Further legs on the same JSON line:
- the other limiter modes on the same workload (modes);
- the widened workloads (workloads): the same set-up at 512^2, the
  solid-body rotation, the double Mach reflection set-up, 1-D Euler;
- 64 uneven Euler solves, batched against one solve per launch (batched;
  the batch tunes its tile shapes per degree);
- the served stream of 1000 requests against FIFO through the plain path,
  at offered loads 0.5, 0.8 and 0.95 of the plain path's capacity
  (serving);
- the oracle on the host (cpu_baseline).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64 DOF-updates/s per limited RK stage (p=4 Euler); batched vs plain; p99"
HBM_PEAK_GBS = 8000.0
PMC_SUMMARY = os.path.join(ROOT, "profiles", "stage_kernel_euler2d_p4_256x256_pmc.md")
SQ_SUMMARY = os.path.join(ROOT, "profiles", "stage_kernel_euler2d_p4_256x256_sq.md")
SIMDS, CLOCK_GHZ = 1024, 2.4     # 256 CUs x 4 SIMDs, peak engine clock
KERNEL_SOURCES = ["paper_2004_08503_amd/csrc/stage_kernel.hpp",
                  "paper_2004_08503_amd/csrc/common.hpp",
                  "paper_2004_08503_amd/csrc/kernels_euler75_2.hip"]


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per stage launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    text = open(PMC_SUMMARY).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    t = re.search(r"hbm_bytes_per_stage_launch:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != kernel_hash():
        return None
    return float(t.group(1))


def measured_valu():
    """VALU wave-instructions per stage launch from the committed SQ counter
    summary, if it was taken on the current kernel source."""
    if not os.path.exists(SQ_SUMMARY):
        return None
    text = open(SQ_SUMMARY).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    v = re.search(r"valu_wave_instructions_per_stage_launch:\s*([0-9.eE+]+)", text)
    if not m or not v or m.group(1) != kernel_hash():
        return None
    return float(v.group(1))


def cpu_model():
    """The host's CPU model name (lscpu, else /proc/cpuinfo) and nproc."""
    import subprocess
    name = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                name = line.split(":", 1)[1].strip()
    except Exception:
        pass
    if name is None and os.path.exists("/proc/cpuinfo"):
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    return name, os.cpu_count()


def cpu_baseline(threads):
    """The oracle (plain C, as it stands; its node and element loops on
    `threads` OpenMP threads, results independent of the count) timed on the
    host on bounded samples of the workloads, in node-updates per second per
    stage (3 per SSP-RK3 step):
      - the benchmark's 256^2 p = 4 Euler state, 18 steps (about 10 s) on
        `threads` threads (the headline baseline);
      - the same recipe at 64^2 (1/16 of the nodes), 10 steps on one thread;
      - 2-D Burgers 128^2 p = 3, 3 steps on `threads` threads;
      - 1-D advection 64 elements p = 3, its 200 steps on one thread;
      - the 512^2 p = 4 Euler state, 1 step on `threads` threads."""
    import oracle
    from paper_2004_08503_amd import workloads as W

    def timed(wl, steps, nthreads):
        oracle.set_threads(nthreads)
        dt = wl.cfl * oracle.max_dt(wl.prob, wl.u0)
        u = wl.u0
        t0 = time.perf_counter()
        for _ in range(steps):
            u = oracle.step(wl.prob, u, dt)
        el = time.perf_counter() - t0
        return {"value": 3 * wl.prob.num_nodes * steps / el, "seconds": el, "steps": steps,
                "threads": nthreads}

    name, nproc = cpu_model()
    try:
        c3 = timed(W.euler_2d(), 18, threads)
        c3_1 = timed(W.euler_2d(n=64), 10, 1)
        c2 = timed(W.burgers_2d(), 3, threads)
        c1 = timed(W.advection_1d(), 200, 1)
        c3b = timed(W.euler_2d(n=512), 1, threads)
    finally:
        oracle.set_threads(1)
    return {"value": c3["value"], "unit": "DOF-updates/s", "cores": threads, "kind": "oracle",
            "sample": "18 SSP-RK3 steps (54 limited stages) of the benchmark's 256x256 p=4 Euler "
                      "state, %.1f s on %d OpenMP threads" % (c3["seconds"], threads),
            "cpu_model": name, "nproc": nproc,
            "single_thread": dict(c3_1, sample="64x64 p=4 Euler, same recipe, 10 steps"),
            "configs": {"euler_2d_256x256_p4": c3, "burgers_2d_128x128_p3": c2,
                        "advection_1d_64_p3": c1, "euler_2d_512x512_p4": c3b}}


def batched_leg(steps, count=64):
    """The batched workload: `count` independent Euler solves (n in
    [32, 256], p in {2..6}, seeded quadrant data), stepped (a) one solve per
    launch, each through its own cached graph, and (b) all together, one
    work-list launch per degree and stage, through one cached graph, with
    the tile shape of each degree chosen by the batch's tuner.  Per-round (one
    step of every solve) latencies from HIP events."""
    import torch
    from paper_2004_08503_amd import idp_dg, workloads as W

    mix = W.batch_mix(count)
    solvers = [idp_dg.Solver(w.prob) for w in mix]
    u_plain = [torch.from_numpy(w.u0).to("cuda") for w in mix]
    u_batch = [t.clone() for t in u_plain]
    nodes = sum(w.prob.num_nodes for w in mix)
    batch = idp_dg.Batch(solvers)
    batch.tune(u_batch, 0.5, reps=3)   # tile shape per degree (states only read)
    n_items = batch.num_items
    stream = torch.cuda.current_stream()

    def run(fn, k):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(k)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e0, e1 in evs:
            e0.record(stream)
            fn()
            e1.record(stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        return el, np.array([a.elapsed_time(b) for a, b in evs])

    def plain_round():
        for sv, u in zip(solvers, u_plain):
            sv.step_cfl(u, 0.5)

    def batch_round():
        batch.step_cfl(u_batch, 0.5)

    for _ in range(2):
        plain_round()
        batch_round()
    el_p, ms_p = run(plain_round, steps)
    el_b, ms_b = run(batch_round, steps)
    same = all(torch.equal(a, b) for a, b in zip(u_plain, u_batch))
    batch.close()
    for sv in solvers:
        sv.close()
    return {
        "workload": "euler_2d_batch_%d_solves_n32-256_p2-6" % count,
        "solves": count, "nodes": nodes, "work_items": n_items,
        "value": 3 * nodes * steps / el_b, "unit": "DOF-updates/s",
        "plain_value": 3 * nodes * steps / el_p,
        "speedup_vs_plain": el_p / el_b,
        "round_ms_p50": float(np.percentile(ms_b, 50)), "round_ms_p99": float(np.percentile(ms_b, 99)),
        "plain_round_ms_p50": float(np.percentile(ms_p, 50)),
        "plain_round_ms_p99": float(np.percentile(ms_p, 99)),
        "steps": steps, "bitwise_equal_to_plain": bool(same),
    }


def mode_leg(wl, prob, steps, u0=None):
    """Device-timestepped steps of prob (the benchmark workload in another
    limiter mode, or another workload with its own initial state u0):
    stage latency from HIP events around each stage, the limited fractions,
    and the bandwidth the stage's algorithmic bytes reach (read the stage
    input, and u^n on stages 2-3, write the output: nc * 8 * 8/3 bytes per
    node and stage, plus the 9 metric terms, 72 bytes, on a curved mesh)."""
    import torch
    from paper_2004_08503_amd import idp_dg
    sv = idp_dg.Solver(prob)
    if torch.is_tensor(u0):   # a device state, stepped in place
        u = u0
    else:
        u = torch.from_numpy((wl.u0 if u0 is None else u0).copy()).to("cuda")
    b1, b2 = sv.empty(), sv.empty()
    dtd = torch.empty(1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    for k in range(steps + 5):
        e = ev[k - 5] if k >= 5 else None
        if k == 5:
            torch.cuda.synchronize()
            sv.diagnostics()
        sv.max_dt_async(u, dtd)
        for st, (a, b, c) in enumerate(((None, u, b1), (u, b1, b2), (u, b2, u))):
            if e is not None:
                e[st].record(stream)
            sv.stage_dt(a, b, c, dtd, wl.cfl, st)
        if e is not None:
            e[3].record(stream)
    torch.cuda.synchronize()
    d = sv.diagnostics()
    ms = np.array([[x[j].elapsed_time(x[j + 1]) for j in range(3)] for x in ev]).reshape(-1)
    nn = prob.num_nodes
    curved = getattr(prob, "coords", None) is not None
    sv.close()
    return {"stage_ms_p50": float(np.percentile(ms, 50)), "stage_ms_p99": float(np.percentile(ms, 99)),
            "stage_dof_updates_per_s": float(nn / (ms.mean() * 1e-3)),
            "algorithmic_gb_per_s": float((prob.nc * 8.0 * 8.0 / 3.0 + (72.0 if curved else 0.0)) * nn
                                          / (ms.mean() * 1e-3) / 1e9),
            "limited_node_fraction": d["limited_nodes"] / (3.0 * nn * steps),
            "entropy_node_fraction": d["entropy_nodes"] / (3.0 * nn * steps), "steps": steps}


def repeated_leg(wl, rep, steps):
    """mode_leg on the workload's periodic state repeated rep x rep times
    (the domain grown with it, so the elements keep their size): the same
    per-node work on a mesh rep^2 times larger, built on the device.  It
    needs about five state arrays of device memory (the state, the leg's
    two stage buffers and the handle's two); skipped where that is not
    free."""
    import torch
    pr = wl.prob
    big = pr.replace(nx=pr.nx * rep, ny=pr.ny * rep, lx=pr.lx * rep, ly=pr.ly * rep)
    state_bytes = 8 * pr.nc * big.num_nodes
    free, _ = torch.cuda.mem_get_info()
    if free < 5.5 * state_bytes:
        return {"skipped": "needs %.0f GB of free device memory" % (5.5 * state_bytes / 1e9)}
    npe = pr.nodes_per_element
    u0 = torch.from_numpy(wl.u0).to("cuda").view(pr.nc, pr.ny, pr.nx, npe)
    u = u0.repeat(1, rep, rep, 1).reshape(pr.nc, big.num_nodes)
    del u0
    out = mode_leg(wl, big, steps, u0=u)
    del u
    torch.cuda.empty_cache()
    out["nodes"] = big.num_nodes
    return out


def double_mach_state(nx=2400, ny=600, p=3):
    """The double Mach reflection set-up on [0, 4] x [0, 1] (Mach 10 shock at
    60 degrees, rho = 1.4 and p = 1 ahead): the problem with its open sides
    (post-shock inflow at x = 0 and on the bottom for x < 1/6, slip wall on
    the rest of the bottom, outflow at x = 4, the initial shock position on
    the top, held fixed for timing) and its initial state."""
    from paper_2004_08503_amd import workloads as W
    g = 1.4
    post = np.array([8.0, 8.0 * 8.25 * np.cos(np.pi / 6), -8.0 * 8.25 * np.sin(np.pi / 6), 0.0])
    post[3] = 116.5 / (g - 1) + 0.5 * (post[1] ** 2 + post[2] ** 2) / post[0]
    pre = np.array([1.4, 0.0, 0.0, 1.0 / (g - 1)])
    prob = W.Problem(dim=2, nx=nx, ny=ny, p=p, eq=W.EULER, lx=4.0, ly=1.0, bc=(1, 1))
    xc, yc = W._element_centres(prob)
    behind = xc < 1.0 / 6.0 + yc / np.sqrt(3.0)
    u0 = np.where(behind[None, :], post[:, None], pre[:, None])
    xs = ((np.arange(nx)[:, None] + W.gl_points(p)[None, :]) * (4.0 / nx)).reshape(-1)
    n = [W.side_nodes(prob, s) for s in range(4)]
    types = [np.full(n[0], W.BC_STATE, np.int8), np.full(n[1], W.BC_OUTFLOW, np.int8),
             np.where(xs < 1.0 / 6.0, W.BC_STATE, W.BC_SLIP).astype(np.int8),
             np.full(n[3], W.BC_STATE, np.int8)]
    top = np.where((xs < 1.0 / 6.0 + 1.0 / np.sqrt(3.0))[None, :], post[:, None], pre[:, None])
    states = [np.repeat(post[:, None], n[0], axis=1), None, np.repeat(post[:, None], n[2], axis=1), top]
    return prob.replace(bnd=W.Boundary(types, states)), u0


def workload_legs(wl):
    """The widened paths measured like the benchmark: the benchmark's own
    Euler set-up at 512^2 (6.6 M nodes: its 630 MB of stage arrays exceed
    the 256 MB last-level cache that the 256^2 arrays fit in, so this is the
    HBM-resident point), the paper's solid-body rotation (velocity field,
    64^2 and 512^2, p = 3), its double Mach reflection set-up at the paper's
    own resolution (open boundaries, 2400 x 600, p = 3, 23 M nodes) and a
    large 1-D Euler problem (2^20 elements, p = 3, the Sod path), the
    benchmark set-up on a smoothly curved mesh (the Cartesian nodes moved
    by 0.05 sin(2 pi x) sin(2 pi y): metric terms and the corrected
    low-order terms per node), and the benchmark's state repeated 18 x 18
    times (4608^2 elements, 531 M nodes, 17 GB per state)."""
    from paper_2004_08503_amd import workloads as W
    out = {}
    curved = wl.prob.replace(coords=W.perturbed_coords(wl.prob, 0.05))
    out["euler_2d_%dx%d_p%d_curved" % (wl.prob.nx, wl.prob.ny, wl.prob.p)] = mode_leg(wl, curved, 30)
    del curved
    big = W.euler_2d(n=512, p=4)
    out["euler_2d_512x512_p4"] = mode_leg(big, big.prob, 20)
    del big
    out["euler_2d_4608x4608_p4"] = repeated_leg(wl, 18, 5)
    for n in (64, 512):
        sb = W.solid_body(n=n, p=3)
        out["solid_body_%dx%d_p3" % (n, n)] = mode_leg(sb, sb.prob, 30)
    prob, u0 = double_mach_state()
    out["double_mach_2400x600_p3"] = mode_leg(wl, prob, 10, u0=u0)
    e1 = W.euler_1d(n=1 << 20, p=3)
    out["euler_1d_1048576_p3"] = mode_leg(e1, e1.prob, 30)
    return out


def progress(msg):
    """One line on stderr per finished leg (the JSON line stays alone on stdout)."""
    print("bench: %s" % msg, file=sys.stderr, flush=True)


# The server's tick policy for the served leg: the admitted requests with
# the least remaining work (less 0.5 s per second waited) step each tick, up
# to about one GPU-filling solve of nodes; admission by footprint only.
SERVE_POLICY = {"policy": "srw", "age_weight": 0.5, "max_active_nodes": 0}


def fifo_from_service(reqs, service):
    """A single server taking the requests in arrival order, each for its
    measured plain-path service time: completion = max(arrival, previous
    completion) + service."""
    from paper_2004_08503_amd import serve
    t = 0.0
    done = []
    for r in sorted(reqs, key=lambda r: r.arrival):
        start = max(r.arrival, t)
        t = start + service[r.rid]
        done.append(serve.Done(rid=r.rid, arrival=r.arrival, admitted=start, finished=t,
                               nodes=r.problem().num_nodes, steps=r.steps))
    return done


def serving_leg(count, loads, budget_gb=64.0):
    """The served workload: a seeded Poisson stream of `count` requests (half
    Burgers, half Euler; n in [16, 512], p in 2..6, 20..200 steps).  The
    same requests are first run back to back through the plain path, one at
    a time: that makespan is the plain path's capacity, and the gaps between
    consecutive completions are each request's service time.  For each
    offered load the arrival rate is load * count / makespan; the stream
    runs through the continuous-batching server (shortest remaining work
    first with aging, SERVE_POLICY), and FIFO through the plain path is the
    single-server queue over the measured service times."""
    from paper_2004_08503_amd import serve, workloads as W
    back_to_back = W.request_stream(count, rate=1e9, seed=5)
    b2b = sorted(serve.run_fifo_plain(back_to_back), key=lambda d: d.finished)
    busy = b2b[-1].finished
    progress("serving: %d requests back to back through the plain path, %.1f s" % (count, busy))
    service, prev = {}, 0.0
    for d in b2b:
        service[d.rid] = d.finished - prev
        prev = d.finished
    out = {"workload": "served_stream_%d_requests_burgers_euler_n16-512_p2-6_steps20-200" % count,
           "plain_service_s": busy, "hbm_budget_gb": budget_gb, "policy": dict(SERVE_POLICY),
           "loads": {}}
    for load in loads:
        rate = load * count / busy
        reqs = W.request_stream(count, rate=rate, seed=5)   # same requests, new arrivals
        srv = serve.Server(hbm_budget=int(budget_gb * 2 ** 30), **SERVE_POLICY)
        served = serve.summarize(srv.run(reqs))
        fifo = serve.summarize(fifo_from_service(reqs, service))
        out["loads"]["%.2f" % load] = {"rate_per_s": rate, "served": served, "fifo_plain": fifo,
                                       "p99_served_over_fifo": served["tts_s_p99"] / fifo["tts_s_p99"]}
        progress("serving: load %.2f, makespan %.1f s" % (load, served["makespan_s"]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256, help="elements per direction")
    ap.add_argument("--p", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 64-solve leg")
    ap.add_argument("--no-modes", action="store_true", help="skip the other limiter modes")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the solid-body, double Mach and 1-D Euler legs")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests in the served stream (0 skips the serving leg)")
    ap.add_argument("--serve-loads", type=str, default="0.5,0.8,0.95",
                    help="offered loads of the served stream (fractions of the plain path's capacity)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="oracle threads for the CPU baseline (0: all host cores, at most 16)")
    ap.add_argument("--tune", action="store_true",
                    help="run the tile-shape tuner on the benchmark solve first (default: the "
                         "tuned default shape of the degree)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of 512 MiB (4 times), the reference "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the path is single-GPU; "
              "--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2004_08503_amd import idp_dg, workloads as W

    if args.copy_calibration:
        n = 64 * 1024 * 1024    # doubles: 512 MiB read + 512 MiB written per copy
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": 8 * n, "copy_bytes_written_per_launch": 8 * n}))
        return

    wl = W.euler_2d(n=args.n, p=args.p)
    prob = wl.prob
    nn = prob.num_nodes
    sv = idp_dg.Solver(prob)
    u = torch.from_numpy(wl.u0.copy()).to("cuda")
    b1, b2 = sv.empty(), sv.empty()
    dtd = torch.empty(1, dtype=torch.float64, device="cuda")
    cfl = wl.cfl
    stream = torch.cuda.current_stream()
    if args.tune:   # tile-shape autotuning on the workload itself (u is only read)
        sv.tune(u, cfl, reps=5)
    shape, epb = sv.tile_shape, sv.tile_elems
    tx, ty = sv.tile_dims

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        sv.max_dt_async(u, dtd)
        if ev is not None:
            ev[1].record(stream)
        sv.stage_dt(None, u, b1, dtd, cfl, 0)
        if ev is not None:
            ev[2].record(stream)
        sv.stage_dt(u, b1, b2, dtd, cfl, 1)
        if ev is not None:
            ev[3].record(stream)
        sv.stage_dt(u, b2, u, dtd, cfl, 2)
        if ev is not None:
            ev[4].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    sv.diagnostics()  # reset counters
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    diag = sv.diagnostics()
    dt_last = sv.max_dt(u) * cfl

    ms = np.array([[evs[k][j].elapsed_time(evs[k][j + 1]) for j in range(4)]
                   for k in range(args.steps)])          # [step][maxdt, s0, s1, s2]
    stage_ms = ms[:, 1:].reshape(-1)
    # algorithmic bytes: stage 0 reads U and writes the output (64 B/node),
    # stages 1 and 2 also read u^n (96 B/node)
    bytes_stage = np.array([64.0, 96.0, 96.0]) * nn
    achieved = bytes_stage.sum() / (ms[:, 1:].mean(axis=0).sum() * 1e-3) / 1e9   # GB/s
    traffic = measured_traffic()
    valu = measured_valu()
    value = 3 * nn * args.steps / elapsed

    assert np.isfinite(u.cpu().numpy()).all()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "euler_2d_%dx%d_p%d" % (args.n, args.n, args.p),
                   "elements": prob.nx * prob.ny, "p": prob.p, "nodes": nn, "components": prob.nc,
                   "cfl": cfl, "limiter": "subcell convex (density Zalesak + entropy)",
                   "path": "plain (one solve per launch)", "parallelism": "single GPU",
                   "tile_shape": shape, "tile_elements": [tx, ty], "elements_per_workgroup": epb},
        "stage_ms_p50": float(np.percentile(stage_ms, 50)),
        "stage_ms_p99": float(np.percentile(stage_ms, 99)),
        "maxdt_ms_mean": float(ms[:, 0].mean()),
        "stage_ms_mean": [float(x) for x in ms[:, 1:].mean(axis=0)],
        "stage_dof_updates_per_s": float(nn / (stage_ms.mean() * 1e-3)),
        "limited_node_fraction": diag["limited_nodes"] / (3.0 * nn * args.steps),
        "entropy_node_fraction": diag["entropy_nodes"] / (3.0 * nn * args.steps),
        "dt_last": dt_last,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "stage_kernel<EULER75,2,%d,%d,%d>" % (prob.p, tx, ty),
                     "algorithmic_bytes_per_node_stage": float(bytes_stage.mean() / nn),
                     # the kernel is bound by VALU issue, not HBM: at least 4 cycles
                     # per counted wave64 instruction over the SIMDs' cycles in
                     # this run's mean stage time
                     "valu_issue_busy": (None if valu is None else
                                         valu * 4.0 / (SIMDS * stage_ms.mean() * 1e6 * CLOCK_GHZ))},
    }
    sv.close()
    del u, b1, b2
    progress("headline leg: stage p50 %.4f ms" % out["stage_ms_p50"])
    # the other limiter modes on the same workload (the smoothness-indicator
    # mode with the initial density range as global bounds)
    rho0 = wl.u0[0]
    out["modes"] = {} if args.no_modes else {
        "subcell_si": mode_leg(wl, prob.replace(limiter=W.SUBCELL_SI, gmin=float(rho0.min()),
                                                gmax=float(rho0.max())), 50),
        "elementwise": mode_leg(wl, prob.replace(limiter=W.ELEMENTWISE), 50),
        "target_only": mode_leg(wl, prob.replace(limiter=W.TARGET), 50),
        "low_only": mode_leg(wl, prob.replace(limiter=W.LOW), 50),
    }
    progress("limiter modes done")
    if not args.no_workloads:
        out["workloads"] = workload_legs(wl)
        progress("workload legs done")
    if not args.no_batch:
        out["batched"] = batched_leg(args.batch_steps)
        progress("batched leg done")
    if args.serve_requests > 0:
        out["serving"] = serving_leg(args.serve_requests,
                                     [float(x) for x in args.serve_loads.split(",") if x])
    if not args.no_cpu:
        threads = args.cpu_threads or max(1, min(16, os.cpu_count() or 1))
        out["cpu_baseline"] = cpu_baseline(threads)
        progress("cpu baseline done")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
