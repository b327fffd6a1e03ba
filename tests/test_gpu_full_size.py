"""The configurations at their full sizes:

- the benchmark's 2-D Euler workload, 256^2 elements, p = 4 (1.64 M
  nodes), over its whole run of 50 device-timestepped SSP-RK3 steps at
  CFL 1/2, against the oracle stepped with the device's time steps: every
  step's time step to 1e-12 and every node after 50 steps to 1e-9 (the
  oracle's loops run on all host cores; its results do not depend on the
  thread count);

- 2-D Burgers on a 128^2 mesh, p = 3 (262 144 nodes), 100 device-timestepped
  SSP-RK3 steps at CFL 1/2 against the oracle stepped with the same time
  steps, on every node, to 1e-9;
- the same Euler set-up at 512^2 (6.6 M nodes): one device-timestepped
  step against the oracle, every node to 1e-12;
- the bench's limiter-mode legs (the same 256^2 state in the four other
  limiter modes), one step each, every node to 1e-12;
- the bench's other workload legs at full size (solid body 512^2, the
  double Mach set-up at 2400 x 600, 1-D Euler with 2^20 elements), one
  step each, every node to 1e-12;
- the bench's 4608^2 leg (the 256^2 state repeated 18 x 18 times, 531 M
  nodes), too large for the oracle: one step bitwise equal to the 256^2
  step repeated, which is checked against the oracle;
- the same Euler workload on the bench's curved mesh (the nodes moved by
  0.05 sin 2 pi x sin 2 pi y), 10 device-timestepped steps against the
  oracle stepped with the device's time steps (each to 1e-12, every node
  after 10 steps to 1e-10);
- the batched mix of 64 independent Euler solves (32^2 to 256^2 elements,
  p = 2..6, 49.6 M nodes), too large for the oracle: one batched step
  must equal every solve's own plain step bitwise (a property that holds
  at any size; the plain path is pinned to the oracle elsewhere), and the
  three smallest solves of the mix are also compared with the oracle
  directly."""
import numpy as np
import pytest

import oracle
from paper_2004_08503_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_08503_amd import idp_dg
    return idp_dg


def rel_err(a, b):
    a = np.asarray(a).reshape(b.shape)
    return (np.abs(a - b).max(axis=1) / np.maximum(np.abs(b).max(axis=1), 1e-300)).max()


def test_burgers_128_p3_full_run():
    idp_dg = _gpu()
    wl = W.burgers_2d()
    prob = wl.prob
    assert (prob.nx, prob.ny, prob.p, wl.steps) == (128, 128, 3, 100)
    sv = idp_dg.Solver(prob)
    u = torch.from_numpy(wl.u0.copy()).cuda()
    ref = wl.u0.copy()
    for _ in range(wl.steps):
        dt_ref = wl.cfl * oracle.max_dt(prob, ref)
        sv.step_cfl(u, wl.cfl)
        assert sv.last_dt() == pytest.approx(dt_ref, rel=1e-12)
        ref = oracle.step(prob, ref, sv.last_dt())
    sv.close()
    err = rel_err(u.cpu().numpy(), ref)
    print("Burgers 128^2 p = 3, 100 steps: max relative error %.2e" % err)
    assert err <= 1e-9, err


def test_euler_256_p4_full_run():
    idp_dg = _gpu()
    import os
    wl = W.euler_2d()
    prob = wl.prob
    assert (prob.nx, prob.ny, prob.p, wl.steps) == (256, 256, 4, 50)
    oracle.set_threads(max(1, min(16, os.cpu_count() or 1)))
    try:
        sv = idp_dg.Solver(prob)
        u = torch.from_numpy(wl.u0.copy()).cuda()
        ref = wl.u0.copy()
        for n in range(wl.steps):
            sv.step_cfl(u, wl.cfl)
            dt = sv.last_dt()
            assert dt == pytest.approx(wl.cfl * oracle.max_dt(prob, ref), rel=1e-12)
            ref = oracle.step(prob, ref, dt)
            if n % 10 == 9:
                print("Euler 256^2 p = 4: step %d of %d" % (n + 1, wl.steps), flush=True)
        sv.close()
    finally:
        oracle.set_threads(1)
    err = rel_err(u.cpu().numpy(), ref)
    print("Euler 256^2 p = 4, 50 steps: max relative error %.2e" % err)
    assert err <= 1e-9, err


def test_euler_512_p4_one_step():
    """The benchmark's Euler set-up at 512^2 (6.6 M nodes, the bench's
    HBM-resident leg): one device-timestepped step against the oracle
    stepped with the device's time step, every node to 1e-12."""
    idp_dg = _gpu()
    import os
    wl = W.euler_2d(n=512, p=4)
    prob = wl.prob
    oracle.set_threads(max(1, min(16, os.cpu_count() or 1)))
    try:
        sv = idp_dg.Solver(prob)
        u = torch.from_numpy(wl.u0.copy()).cuda()
        sv.step_cfl(u, wl.cfl)
        dt = sv.last_dt()
        assert dt == pytest.approx(wl.cfl * oracle.max_dt(prob, wl.u0), rel=1e-12)
        ref = oracle.step(prob, wl.u0, dt)
        sv.close()
    finally:
        oracle.set_threads(1)
    err = rel_err(u.cpu().numpy(), ref)
    print("Euler 512^2 p = 4, one step: max relative error %.2e" % err)
    assert err <= 1e-12, err


@pytest.mark.parametrize("mode", ["subcell_si", "elementwise", "target_only", "low_only"])
def test_euler_256_p4_limiter_modes_one_step(mode):
    """The bench's limiter-mode legs at full size (the 256^2 p = 4 Euler
    state; the smoothness-indicator mode with the initial density range as
    global bounds): one device-timestepped step against the oracle, every
    node to 1e-12."""
    idp_dg = _gpu()
    import os
    wl = W.euler_2d()
    rho0 = wl.u0[0]
    prob = {"subcell_si": wl.prob.replace(limiter=W.SUBCELL_SI, gmin=float(rho0.min()), gmax=float(rho0.max())),
            "elementwise": wl.prob.replace(limiter=W.ELEMENTWISE),
            "target_only": wl.prob.replace(limiter=W.TARGET),
            "low_only": wl.prob.replace(limiter=W.LOW)}[mode]
    oracle.set_threads(max(1, min(16, os.cpu_count() or 1)))
    try:
        sv = idp_dg.Solver(prob)
        u = torch.from_numpy(wl.u0.copy()).cuda()
        sv.step_cfl(u, wl.cfl)
        dt = sv.last_dt()
        ref = oracle.step(prob, wl.u0, dt)
        sv.close()
    finally:
        oracle.set_threads(1)
    err = rel_err(u.cpu().numpy(), ref)
    print("Euler 256^2 p = 4 %s, one step: max relative error %.2e" % (mode, err))
    assert err <= 1e-12, err


@pytest.mark.parametrize("leg", ["solid_body_512", "double_mach_2400x600", "euler_1d_2e20"])
def test_bench_workload_legs_one_step(leg):
    """The bench's other workload legs at their full sizes: the solid-body
    rotation at 512^2, p = 3 (velocity field), the double Mach reflection
    set-up at 2400 x 600, p = 3 (23 M nodes, open boundaries) and 1-D Euler
    with 2^20 elements, p = 3: one device-timestepped step each against the
    oracle stepped with the device's time step, every node to 1e-12."""
    idp_dg = _gpu()
    import os
    import sys
    if leg == "solid_body_512":
        wl = W.solid_body(n=512, p=3)
        prob, u0, cfl = wl.prob, wl.u0, wl.cfl
    elif leg == "euler_1d_2e20":
        wl = W.euler_1d(n=1 << 20, p=3)
        prob, u0, cfl = wl.prob, wl.u0, wl.cfl
    else:
        sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        import bench
        prob, u0 = bench.double_mach_state()
        cfl = 0.5
    oracle.set_threads(max(1, min(16, os.cpu_count() or 1)))
    try:
        sv = idp_dg.Solver(prob)
        u = torch.from_numpy(np.ascontiguousarray(u0)).cuda()
        sv.step_cfl(u, cfl)
        dt = sv.last_dt()
        assert dt == pytest.approx(cfl * oracle.max_dt(prob, u0), rel=1e-12)
        ref = oracle.step(prob, u0, dt)
        sv.close()
    finally:
        oracle.set_threads(1)
    err = rel_err(u.cpu().numpy(), ref)
    print("%s, one step: max relative error %.2e" % (leg, err))
    assert err <= 1e-12, err


def test_bench_repeated_leg_one_step():
    """The bench's 4608^2 leg (the 256^2 p = 4 Euler state repeated 18 x 18
    times, 531 M nodes), too large for the oracle: its device-timestepped
    step equals, bitwise, the 256^2 step repeated (a node's arithmetic does
    not depend on its position, tile or mesh size; the elements keep their
    size), with the same time step, and the 256^2 step is checked against
    the oracle."""
    idp_dg = _gpu()
    import os
    wl = W.euler_2d()
    small, rep = wl.prob, 18
    big = small.replace(nx=small.nx * rep, ny=small.ny * rep, lx=small.lx * rep, ly=small.ly * rep)
    nc, npe = small.nc, small.nodes_per_element
    free, _ = torch.cuda.mem_get_info()
    if free < 3.3 * 8 * nc * big.num_nodes:
        pytest.skip("needs %.0f GB of free device memory" % (3.3 * 8 * nc * big.num_nodes / 1e9))
    oracle.set_threads(max(1, min(16, os.cpu_count() or 1)))
    try:
        sv = idp_dg.Solver(small)
        us = torch.from_numpy(wl.u0.copy()).cuda()
        sv.step_cfl(us, wl.cfl)
        dt = sv.last_dt()
        sv.close()
        ref = oracle.step(small, wl.u0, dt)
    finally:
        oracle.set_threads(1)
    err = rel_err(us.cpu().numpy(), ref)
    assert err <= 1e-12, err
    u0 = torch.from_numpy(wl.u0).cuda().view(nc, small.ny, small.nx, npe)
    ub = u0.repeat(1, rep, rep, 1).reshape(nc, big.num_nodes)
    del u0
    sv = idp_dg.Solver(big)
    sv.step_cfl(ub, wl.cfl)
    assert sv.last_dt() == dt
    sv.close()
    ndiff = int((ub.view(nc, rep, small.ny, rep, small.nx, npe)
                 != us.view(nc, 1, small.ny, 1, small.nx, npe)).sum().item())
    del ub
    torch.cuda.empty_cache()
    print("Euler 4608^2 p = 4 (256^2 repeated), one step: %d nodes differ from the repeated 256^2 step "
          "(256^2 against the oracle: %.2e)" % (ndiff, err))
    assert ndiff == 0


def test_euler_256_p4_curved_steps():
    idp_dg = _gpu()
    import os
    wl = W.euler_2d()
    prob = wl.prob.replace(coords=W.perturbed_coords(wl.prob, 0.05))
    assert (prob.nx, prob.ny, prob.p) == (256, 256, 4)
    oracle.set_threads(max(1, min(16, os.cpu_count() or 1)))
    try:
        sv = idp_dg.Solver(prob)
        u = torch.from_numpy(wl.u0.copy()).cuda()
        ref = wl.u0.copy()
        for n in range(10):
            sv.step_cfl(u, wl.cfl)
            dt = sv.last_dt()
            assert dt == pytest.approx(wl.cfl * oracle.max_dt(prob, ref), rel=1e-12)
            ref = oracle.step(prob, ref, dt)
            print("curved Euler 256^2 p = 4: step %d of 10" % (n + 1), flush=True)
        sv.close()
    finally:
        oracle.set_threads(1)
    err = rel_err(u.cpu().numpy(), ref)
    print("curved Euler 256^2 p = 4, 10 steps: max relative error %.2e" % err)
    assert err <= 1e-10, err


def test_batched_64_solve_mix_one_step():
    idp_dg = _gpu()
    mix = W.batch_mix(64)
    assert sum(w.prob.num_nodes for w in mix) > 40_000_000
    solvers = [idp_dg.Solver(w.prob) for w in mix]
    u_plain = [torch.from_numpy(w.u0).cuda() for w in mix]
    u_batch = [t.clone() for t in u_plain]
    batch = idp_dg.Batch(solvers)
    batch.step_cfl(u_batch, 0.5)
    for sv, u in zip(solvers, u_plain):
        sv.step_cfl(u, 0.5)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(u_plain, u_batch))
    dts = batch.last_dt()
    for i in sorted(range(len(mix)), key=lambda i: mix[i].prob.num_nodes)[:3]:
        prob = mix[i].prob
        assert dts[i] == pytest.approx(0.5 * oracle.max_dt(prob, mix[i].u0), rel=1e-13)
        ref = oracle.step(prob, mix[i].u0, dts[i])
        err = rel_err(u_batch[i].cpu().numpy(), ref)
        assert err <= 1e-12, (i, prob.nx, prob.p, err)
    batch.close()
    for sv in solvers:
        sv.close()
