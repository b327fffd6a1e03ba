"""Batched path: many Euler solves of uneven mesh size and degree stepped
together (one work-list launch per degree and stage).  Each solve's result
must be bitwise identical to the plain one-solve-per-launch path, which is
itself parity-checked against the oracle."""
import numpy as np
import pytest

import oracle
from paper_2004_08503_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_08503_amd import idp_dg
    return idp_dg


def mix(count=7, seed=21):
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        n = int(rng.integers(5, 23))
        p = [2, 3, 4, 5, 6, 7, 8, 1][s % 8]
        prob = W.Problem(dim=2, nx=n, ny=int(rng.integers(4, 20)), p=p, eq=W.EULER)
        out.append((prob, W.euler_quadrants(prob, np.random.default_rng([seed, s]))))
    return out


def test_batch_step_bitwise_equals_plain():
    idp_dg = _lib()
    cases = mix()
    solvers = [idp_dg.Solver(p) for p, _ in cases]
    ub = [torch.from_numpy(u.copy()).cuda() for _, u in cases]
    up = [torch.from_numpy(u.copy()).cuda() for _, u in cases]
    dts = [0.4 * oracle.max_dt(p, u) for p, u in cases]
    batch = idp_dg.Batch(solvers)
    assert batch.num_items > 0
    for _ in range(3):
        batch.step(ub, dts)
        for sv, u, dt in zip(solvers, up, dts):
            sv.step(u, dt)
    torch.cuda.synchronize()
    for a, b in zip(ub, up):
        assert torch.equal(a, b)
    # and the plain path itself agrees with the oracle
    prob, u0 = cases[0]
    ref = u0
    for _ in range(3):
        ref = oracle.step(prob, ref, dts[0])
    got = ub[0].cpu().numpy()
    err = (np.abs(got - ref).max(axis=1) / np.abs(ref).max(axis=1)).max()
    assert err < 1e-12
    batch.close()


def test_batch_step_cfl_bitwise_equals_plain():
    idp_dg = _lib()
    cases = mix(count=10, seed=5)
    solvers = [idp_dg.Solver(p) for p, _ in cases]
    ub = [torch.from_numpy(u.copy()).cuda() for _, u in cases]
    up = [torch.from_numpy(u.copy()).cuda() for _, u in cases]
    batch = idp_dg.Batch(solvers)
    for _ in range(4):
        batch.step_cfl(ub, 0.5)
        for sv, u in zip(solvers, up):
            sv.step_cfl(u, 0.5)
        dts_b = batch.last_dt()
        dts_p = [sv.last_dt() for sv in solvers]
        assert dts_b == dts_p
    torch.cuda.synchronize()
    for a, b in zip(ub, up):
        assert torch.equal(a, b)


def test_batch_alone_vs_in_mix():
    """A solve's result does not depend on which other solves share the
    launch."""
    idp_dg = _lib()
    cases = mix(count=6, seed=8)
    solvers = [idp_dg.Solver(p) for p, _ in cases]
    u_mix = [torch.from_numpy(u.copy()).cuda() for _, u in cases]
    u_one = torch.from_numpy(cases[2][1].copy()).cuda()
    dts = [0.4 * oracle.max_dt(p, u) for p, u in cases]
    idp_dg.Batch(solvers).step(u_mix, dts)
    idp_dg.Batch([solvers[2]]).step([u_one], [dts[2]])
    torch.cuda.synchronize()
    assert torch.equal(u_mix[2], u_one)


def test_batch_rejects_bad_input():
    idp_dg = _lib()
    e1 = idp_dg.Solver(W.Problem(dim=2, nx=4, ny=4, p=3, eq=W.EULER))
    e2 = idp_dg.Solver(W.Problem(dim=2, nx=4, ny=4, p=3, eq=W.EULER, gamma=5.0 / 3.0))
    b2 = idp_dg.Solver(W.Problem(dim=2, nx=4, ny=4, p=3, eq=W.BURGERS))
    for group in ([e1, e2], [e1, b2], [e1, e1]):
        with pytest.raises(idp_dg.IdpError):
            idp_dg.Batch(group)
    batch = idp_dg.Batch([e1])
    u = e1.empty()
    with pytest.raises(idp_dg.IdpError):
        batch.step([u], [-1.0])


def test_batch_scalar_family():
    """Burgers solves of different degree and velocity in one batch."""
    idp_dg = _lib()
    rng = np.random.default_rng(3)
    cases = []
    for k, p in enumerate([2, 3, 3, 5]):
        prob = W.Problem(dim=2, nx=7 + k, ny=5 + 2 * k, p=p, eq=W.BURGERS, vel=(1.0, 0.5 * k))
        cases.append((prob, rng.uniform(-1, 1, (1, prob.num_nodes))))
    solvers = [idp_dg.Solver(p) for p, _ in cases]
    ub = [torch.from_numpy(u.copy()).cuda() for _, u in cases]
    up = [torch.from_numpy(u.copy()).cuda() for _, u in cases]
    batch = idp_dg.Batch(solvers)
    for _ in range(3):
        batch.step_cfl(ub, 0.5)
        for sv, u in zip(solvers, up):
            sv.step_cfl(u, 0.5)
    torch.cuda.synchronize()
    for a, b in zip(ub, up):
        assert torch.equal(a, b)


@pytest.mark.skip(reason="aborted the host process once on the MI355X box (inside Batch.update, no GPU "
                         "fault) while batch step graphs were captured and retired on every membership "
                         "change; the cause is not established, batch graphs are switched off, and this "
                         "case stays off the GPU until a cause is shown")
def test_batch_membership_changes_while_graphs_run():
    """Alternating memberships without host synchronisation: each change
    retires a step graph whose launch is still queued.  Every solve must
    still equal its plain run, step for step."""
    idp_dg = _lib()
    cases = mix(count=6, seed=9)
    solvers = [idp_dg.Solver(p) for p, _ in cases]
    ub = [torch.from_numpy(u.copy()).cuda() for _, u in cases]
    up = [torch.from_numpy(u.copy()).cuda() for _, u in cases]
    counts = [0] * len(cases)
    batch = idp_dg.Batch(solvers)
    subsets = [list(range(6)), list(range(6)), [0, 2, 4], [0, 2, 4], [0, 2, 4], [1, 5]]
    prev = subsets[0]
    for rnd in range(5):
        for ids in subsets:
            if ids != prev:   # same membership twice in a row: the step runs as a graph
                batch.update([solvers[i] for i in ids])
                prev = ids
            batch.step_cfl([ub[i] for i in ids], 0.5)
            for i in ids:
                counts[i] += 1
    for sv, u, k in zip(solvers, up, counts):
        for _ in range(k):
            sv.step_cfl(u, 0.5)
    torch.cuda.synchronize()
    for a, b in zip(ub, up):
        assert torch.equal(a, b)
    batch.close()
    for sv in solvers:
        sv.close()


def test_batch_smoothness_indicator_bitwise_equals_plain():
    idp_dg = _lib()
    cases = []
    for (prob, u) in mix(count=5, seed=13):
        cases.append((prob.replace(limiter=W.SUBCELL_SI, gmin=float(u[0].min()), gmax=float(u[0].max())), u))
    solvers = [idp_dg.Solver(p) for p, _ in cases]
    ub = [torch.from_numpy(u.copy()).cuda() for _, u in cases]
    up = [torch.from_numpy(u.copy()).cuda() for _, u in cases]
    batch = idp_dg.Batch(solvers)
    for _ in range(3):
        batch.step_cfl(ub, 0.5)
        for sv, u in zip(solvers, up):
            sv.step_cfl(u, 0.5)
    torch.cuda.synchronize()
    for a, b in zip(ub, up):
        assert torch.equal(a, b)
    batch.close()


def test_batch_elementwise_bitwise_equals_plain():
    idp_dg = _lib()
    cases = [(prob.replace(limiter=W.ELEMENTWISE), u) for prob, u in mix(count=5, seed=17)]
    solvers = [idp_dg.Solver(p) for p, _ in cases]
    ub = [torch.from_numpy(u.copy()).cuda() for _, u in cases]
    up = [torch.from_numpy(u.copy()).cuda() for _, u in cases]
    batch = idp_dg.Batch(solvers)
    for _ in range(3):
        batch.step_cfl(ub, 0.5)
        for sv, u in zip(solvers, up):
            sv.step_cfl(u, 0.5)
    torch.cuda.synchronize()
    for a, b in zip(ub, up):
        assert torch.equal(a, b)
    batch.close()
