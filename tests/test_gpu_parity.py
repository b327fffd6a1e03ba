"""GPU parity: the HIP stage (through the C ABI) against the CPU oracle on
the same seeded inputs.

Tolerance (the stated target of the build): per component,
max |u_gpu - u_ref| / max |u_ref| <= 1e-12 for one stage and <= 1e-9 after
100 SSP-RK3 steps.  Both sides compute in binary64; they differ by the
order of rounding (the GPU contracts multiply-adds, forms the high-order
subcell flux directly instead of by prefix sums, and finds the entropy
root by a bracketed Newton search instead of bisection; both land within
rounding of the supremum).  The smoothness-indicator mode (SUBCELL_SI) is
checked the same way, with the global bounds set to the range of the
initial limited component, as in the paper's examples.
"""
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
    scale = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return (np.abs(a - b).max(axis=1) / scale).max()


def alpha_effect(prob, tr, dt, da, m=None):
    """Largest change that nodal-coefficient differences da can make in an
    updated state: per node |da_i| dt/m_i times the sum of |rbar| over its
    subcell faces (its face coefficients are min(alpha_i, alpha_j)), per
    component relative to that component's largest stage input.  The
    coefficient of a node whose corrections are tiny is ill-conditioned
    (a ratio of rounding-size terms) while its effect is not, so this is
    what parity fixes at the state tolerance."""
    n1 = prob.p + 1
    _, w = oracle.gl(prob.p)
    ne = prob.nx * prob.ny
    hx = prob.lx / prob.nx
    if prob.dim == 2:
        hy = prob.ly / prob.ny
        if m is None:   # Cartesian masses (a curved mesh passes its own)
            m = np.tile((np.outer(w, w) * hx * hy).reshape(-1), ne)   # node (a, b) -> w_b w_a
        shape = (-1, ne, n1, n1)
    else:
        m = np.tile(w * hx, ne)
        shape = (-1, ne, 1, n1)
    rb = np.abs(tr["rbar"])                              # [k][c][node]
    tot = np.zeros(rb.shape[1:])
    for k in range(prob.dim):
        plus = rb[k].reshape(shape)
        minus = np.zeros_like(plus)
        if k == 0:
            minus[..., 1:] = plus[..., :-1]
        else:
            minus[:, :, 1:, :] = plus[:, :, :-1, :]
        tot += (plus + minus).reshape(rb.shape[1:])
    return np.abs(da)[None, :] * dt / m[None, :] * tot


def to_dev(u):
    return torch.from_numpy(np.ascontiguousarray(u)).to("cuda")


def stage_parity(prob, u, dt, tol=1e-12):
    idp_dg = _gpu()
    sv = idp_dg.Solver(prob)
    un = to_dev(u)
    cur_ref = u
    cur = un
    worst = 0.0
    for s in range(3):
        ref = oracle.stage(prob, None if s == 0 else u, cur_ref, dt, s)
        out = sv.empty()
        sv.stage(None if s == 0 else un, cur, out, dt, s)
        torch.cuda.synchronize()
        err = rel_err(out.cpu().numpy(), ref)
        worst = max(worst, err)
        assert err <= tol, (s, err)
        # feed the oracle's own output to both sides for the next stage
        cur_ref = ref
        cur = to_dev(ref)
    sv.close()
    return worst


def small_problems():
    out = []
    out.append(("adv1d-C1", W.advection_1d()))
    out.append(("burgers2d-16", W.burgers_2d(n=16, p=3)))
    out.append(("euler2d-16", W.euler_2d(n=16, p=4)))
    out.append(("euler1d-24", W.euler_1d(n=24, p=3)))
    wl = W.euler_2d(n=16, p=4)
    # ragged: element count not a multiple of the tile, nx != ny, lx != ly
    prob = wl.prob.replace(nx=11, ny=7, ly=0.7)
    out.append(("euler2d-11x7", W.Workload("e", prob, W.euler_quadrants(prob, np.random.default_rng(9)), 0.5, 1)))
    prob = W.Problem(dim=2, nx=13, ny=5, p=2, eq=W.BURGERS, vel=(1.0, -0.5))
    x, y, _ = W.node_coords(prob)
    u = (0.3 + np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y))[None, :]
    out.append(("burgers2d-13x5", W.Workload("b", prob, u, 0.5, 1)))
    prob = W.Problem(dim=2, nx=9, ny=10, p=3, eq=W.ADVECTION, vel=(0.8, -0.3))
    x, y, _ = W.node_coords(prob)
    u = ((x > 0.3) & (x < 0.6) & (y > 0.2)).astype(float)[None, :] + 0.1 * np.sin(2 * np.pi * y)[None, :]
    out.append(("adv2d-9x10", W.Workload("a", prob, u, 0.5, 1)))
    return out


SMALL = small_problems()


@pytest.mark.parametrize("name,wl", SMALL, ids=[s[0] for s in SMALL])
@pytest.mark.parametrize("limiter", [W.SUBCELL, W.TARGET, W.LOW], ids=["subcell", "target", "low"])
def test_stage_parity_small(name, wl, limiter):
    prob = wl.prob.replace(limiter=limiter)
    dt = wl.cfl * oracle.max_dt(prob, wl.u0)
    stage_parity(prob, wl.u0, dt)


@pytest.mark.parametrize("p", range(1, 9))
@pytest.mark.parametrize("eq", ["advection", "burgers", "euler"])
@pytest.mark.parametrize("dim", [1, 2])
def test_stage_parity_every_degree(p, eq, dim):
    rng = np.random.default_rng(100 * p + dim)
    if dim == 1:
        prob = W.Problem(dim=1, nx=7, ny=1, p=p, eq=W.EQ_NAMES[eq], vel=(-0.7, 0.0))
    else:
        prob = W.Problem(dim=2, nx=5, ny=3, p=p, eq=W.EQ_NAMES[eq], vel=(0.6, 1.1))
    if prob.eq == W.EULER:
        u = W.euler_quadrants(prob, rng)
    else:
        u = rng.uniform(-1.0, 1.0, (1, prob.num_nodes))
    dt = 0.5 * oracle.max_dt(prob, u)
    stage_parity(prob, u, dt)


def test_max_dt_parity():
    idp_dg = _gpu()
    for name, wl in SMALL:
        sv = idp_dg.Solver(wl.prob)
        got = sv.max_dt(to_dev(wl.u0))
        ref = oracle.max_dt(wl.prob, wl.u0)
        assert got == pytest.approx(ref, rel=1e-14), name
        sv.close()


@pytest.mark.parametrize("wl,steps", [
    (W.advection_1d(), 200),
    (W.burgers_2d(n=24, p=3), 100),
    (W.euler_2d(n=24, p=4), 100),
], ids=["adv1d-200", "burgers2d-24-100", "euler2d-24-100"])
def test_many_steps_parity(wl, steps):
    """Fixed dt from the initial state (C1 uses CFL 0.2), both sides step
    independently."""
    idp_dg = _gpu()
    prob = wl.prob
    dt = wl.cfl * oracle.max_dt(prob, wl.u0)
    if prob.eq == W.EULER:
        dt *= 0.5   # the speeds grow as the Riemann fans open
    ref = wl.u0.copy()
    for _ in range(steps):
        ref = oracle.step(prob, ref, dt)
    sv = idp_dg.Solver(prob)
    u = to_dev(wl.u0)
    for _ in range(steps):
        sv.step(u, dt)
    torch.cuda.synchronize()
    err = rel_err(u.cpu().numpy(), ref)
    assert err <= 1e-9, err
    d = sv.diagnostics()
    assert not d["low_order_violation"] and not d["bad_input"]


def test_step_cfl_matches_oracle_rk3():
    """Device-timestepped steps (graph replay) against the oracle with
    dt = 0.5 * max_dt recomputed from u^n every step."""
    idp_dg = _gpu()
    wl = W.euler_2d(n=20, p=3)
    prob = wl.prob
    ref = wl.u0.copy()
    sv = idp_dg.Solver(prob)
    u = to_dev(wl.u0)
    for _ in range(10):
        dt_ref = 0.5 * oracle.max_dt(prob, ref)
        sv.step_cfl(u, 0.5)
        assert sv.last_dt() == pytest.approx(dt_ref, rel=1e-12)
        ref = oracle.step(prob, ref, sv.last_dt())
    err = rel_err(u.cpu().numpy(), ref)
    assert err <= 1e-11, err


def test_euler_full_size_one_step():
    """The benchmarked workload (Euler, 256^2 elements, p = 4) in the
    benchmark's launch configuration: one device-timestepped step against
    the oracle on every node."""
    idp_dg = _gpu()
    wl = W.euler_2d()
    prob = wl.prob
    sv = idp_dg.Solver(prob)
    u = to_dev(wl.u0)
    sv.step_cfl(u, wl.cfl)
    dt = sv.last_dt()
    assert dt == pytest.approx(wl.cfl * oracle.max_dt(prob, wl.u0), rel=1e-13)
    ref = oracle.step(prob, wl.u0, dt)
    err = rel_err(u.cpu().numpy(), ref)
    assert err <= 1e-12, err
    d = sv.diagnostics()
    assert d["limited_nodes"] > 0 and not d["low_order_violation"]


def test_edge_cases():
    idp_dg = _gpu()
    # one element per direction: an element is its own neighbour
    prob = W.Problem(dim=2, nx=1, ny=1, p=4, eq=W.EULER)
    u = W.euler_quadrants(prob, np.random.default_rng(1))
    stage_parity(prob, u, 0.5 * oracle.max_dt(prob, u))
    prob = W.Problem(dim=1, nx=1, ny=1, p=5, eq=W.BURGERS, vel=(1.0, 0.0))
    u = np.random.default_rng(2).uniform(-1, 1, (1, prob.num_nodes))
    stage_parity(prob, u, 0.5 * oracle.max_dt(prob, u))
    # dt = 0 is the identity; a constant state is preserved
    wl = W.euler_2d(n=8, p=3)
    sv = idp_dg.Solver(wl.prob)
    u = to_dev(wl.u0)
    out = sv.empty()
    sv.stage(None, u, out, 0.0, 0)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), wl.u0)
    c = np.repeat(wl.u0[:, :1], wl.prob.num_nodes, axis=1)
    uc = to_dev(c)
    sv.step(uc, 0.5 * oracle.max_dt(wl.prob, c))
    torch.cuda.synchronize()
    np.testing.assert_allclose(uc.cpu().numpy(), c, rtol=1e-14, atol=1e-14)
    # in-place third stage (u_out == u_n) is allowed, overlapping u_s is not
    v = to_dev(wl.u0)
    w = to_dev(wl.u0)
    dt = 0.5 * oracle.max_dt(wl.prob, wl.u0)
    sv.stage(v, w, v, dt, 2)
    with pytest.raises(idp_dg.IdpError):
        sv.stage(v, w, w, dt, 1)
    with pytest.raises(idp_dg.IdpError):
        sv.stage(None, w, v, -1.0, 0)
    with pytest.raises(idp_dg.IdpError):
        sv.stage(None, w, v, dt, 3)
    torch.cuda.synchronize()
    ref = oracle.stage(wl.prob, wl.u0, wl.u0, dt, 2)
    assert rel_err(v.cpu().numpy(), ref) <= 1e-12
    sv.close()


def test_zero_state_burgers_step_cfl():
    """No dissipation anywhere (u = 0): max_dt is +inf and the step keeps
    the state."""
    idp_dg = _gpu()
    prob = W.Problem(dim=2, nx=4, ny=4, p=2, eq=W.BURGERS)
    sv = idp_dg.Solver(prob)
    u = torch.zeros((1, prob.num_nodes), dtype=torch.float64, device="cuda")
    assert sv.max_dt(u) == float("inf")
    sv.step_cfl(u, 0.5)
    torch.cuda.synchronize()
    assert torch.count_nonzero(u).item() == 0
    sv.close()


@pytest.mark.parametrize("wl", [W.euler_2d(n=16, p=4), W.burgers_2d(n=16, p=3), W.euler_1d(n=30, p=4),
                                W.euler_2d(n=12, p=6)],
                         ids=["euler2d", "burgers2d", "euler1d", "euler2d-p6"])
def test_limiter_intermediates_match_oracle(wl):
    """Bounds, entropy bound and limiting coefficients themselves, not only
    the updated state."""
    idp_dg = _gpu()
    prob = wl.prob
    dt = wl.cfl * oracle.max_dt(prob, wl.u0)
    ref, tr = oracle.fe(prob, wl.u0, dt, trace=True)
    sv = idp_dg.Solver(prob)
    out = sv.empty()
    g = sv.stage_trace(None, to_dev(wl.u0), out, dt, 0).cpu().numpy()
    sc = np.abs(wl.u0[0]).max()
    np.testing.assert_allclose(g[0], tr["umin"], rtol=0, atol=1e-14 * sc)
    np.testing.assert_allclose(g[1], tr["umax"], rtol=0, atol=1e-14 * sc)
    if prob.eq == W.EULER:
        np.testing.assert_allclose(g[2], tr["kmin"], rtol=1e-14, atol=0)
    np.testing.assert_allclose(g[3], tr["alpha_z"], rtol=0, atol=1e-9)
    np.testing.assert_allclose(g[4], tr["alpha"], rtol=0, atol=1e-9)
    # the coefficients' effect on the update, at the state tolerance
    scale = np.abs(wl.u0).max(axis=1)[:, None]
    for q, key in ((3, "alpha_z"), (4, "alpha")):
        eff = alpha_effect(prob, tr, dt, g[q] - tr[key]) / scale
        assert eff.max() <= 1e-12, (key, eff.max())
    assert (tr["alpha"] < 1).any()
    sv.close()


@pytest.mark.parametrize("gamma", [5.0 / 3.0, 1.3], ids=["gamma5/3", "gamma1.3"])
@pytest.mark.parametrize("dim,p", [(1, 3), (2, 2), (2, 4), (2, 7)])
def test_stage_parity_other_gamma(gamma, dim, p):
    """The gamma = 5/3 instantiation (integer powers of rho^-1/3) and the
    generic-gamma one (pow)."""
    rng = np.random.default_rng(7 * p + dim)
    if dim == 1:
        prob = W.Problem(dim=1, nx=9, ny=1, p=p, eq=W.EULER, gamma=gamma)
    else:
        prob = W.Problem(dim=2, nx=6, ny=5, p=p, eq=W.EULER, gamma=gamma)
    u = W.euler_quadrants(prob, rng)
    stage_parity(prob, u, 0.5 * oracle.max_dt(prob, u))


def si(prob, u):
    """The problem in SUBCELL_SI mode with the global bounds of the limited
    component taken from u."""
    return prob.replace(limiter=W.SUBCELL_SI, gmin=float(u[0].min()), gmax=float(u[0].max()))


@pytest.mark.parametrize("name,wl", SMALL, ids=[s[0] for s in SMALL])
def test_stage_parity_smoothness_indicator(name, wl):
    prob = si(wl.prob, wl.u0)
    dt = wl.cfl * oracle.max_dt(prob, wl.u0)
    stage_parity(prob, wl.u0, dt)


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("eq", ["burgers", "euler"])
@pytest.mark.parametrize("dim", [1, 2])
def test_smoothness_indicator_every_degree(p, eq, dim):
    """Smooth data with a jump, so that the tile holds smooth, partly rough
    and rough elements."""
    if dim == 1:
        prob = W.Problem(dim=1, nx=9, ny=1, p=p, eq=W.EQ_NAMES[eq], vel=(0.9, 0.0))
    else:
        prob = W.Problem(dim=2, nx=6, ny=5, p=p, eq=W.EQ_NAMES[eq], vel=(0.6, 1.1))
    x, y, _ = W.node_coords(prob)
    smooth = 1.0 + 0.3 * np.sin(2 * np.pi * x) * (np.cos(2 * np.pi * y) if dim == 2 else 1.0)
    f = smooth + 2.0 * (x > 0.55)
    if prob.eq == W.EULER:
        nc = prob.nc
        u = np.zeros((nc, prob.num_nodes))
        u[0] = f
        u[1] = 0.2 * f
        if dim == 2:
            u[2] = -0.1 * f
        vel2 = (u[1] ** 2 + (u[2] ** 2 if dim == 2 else 0.0)) / f ** 2
        u[nc - 1] = 1.0 / (prob.gamma - 1.0) + 0.5 * f * vel2
    else:
        u = f[None, :]
    prob = si(prob, u)
    eps = oracle.smoothness(prob, u)
    if p > 1:
        assert (eps == 0).any() and (eps > 0).any()
    dt = 0.5 * oracle.max_dt(prob, u)
    stage_parity(prob, u, dt)


@pytest.mark.parametrize("wl", [W.euler_2d(n=16, p=4), W.burgers_2d(n=16, p=3), W.advection_1d()],
                         ids=["euler2d", "burgers2d", "adv1d"])
def test_smoothness_indicator_relaxed_bounds_match_oracle(wl):
    idp_dg = _gpu()
    prob = si(wl.prob, wl.u0)
    dt = wl.cfl * oracle.max_dt(prob, wl.u0)
    ref, tr = oracle.fe(prob, wl.u0, dt, trace=True)
    sv = idp_dg.Solver(prob)
    out = sv.empty()
    g = sv.stage_trace(None, to_dev(wl.u0), out, dt, 0).cpu().numpy()
    sc = np.abs(wl.u0[0]).max()
    np.testing.assert_allclose(g[0], tr["umin"], rtol=0, atol=1e-14 * sc)
    np.testing.assert_allclose(g[1], tr["umax"], rtol=0, atol=1e-14 * sc)
    np.testing.assert_allclose(g[4], tr["alpha"], rtol=0, atol=1e-9)
    eff = alpha_effect(prob, tr, dt, g[4] - tr["alpha"]) / np.abs(wl.u0).max(axis=1)[:, None]
    assert eff.max() <= 1e-12, eff.max()
    # the relaxation changed the bounds somewhere (elements that are not
    # rough): they are not the strict local ones
    _, trs = oracle.fe(wl.prob, wl.u0, dt, trace=True)
    assert (np.abs(tr["umax"] - trs["umax"]) > 1e-6 * sc).any()
    assert rel_err(out.cpu().numpy(), ref) <= 1e-12
    sv.close()


def test_smoothness_indicator_rejects_bad_bounds():
    idp_dg = _gpu()
    prob = W.Problem(dim=1, nx=4, ny=1, p=3, eq=W.BURGERS, limiter=W.SUBCELL_SI, gmin=1.0, gmax=0.0)
    with pytest.raises(idp_dg.IdpError):
        idp_dg.Solver(prob)


@pytest.mark.parametrize("name,wl", SMALL, ids=[s[0] for s in SMALL])
def test_stage_parity_elementwise(name, wl):
    prob = wl.prob.replace(limiter=W.ELEMENTWISE)
    dt = wl.cfl * oracle.max_dt(prob, wl.u0)
    stage_parity(prob, wl.u0, dt)


@pytest.mark.parametrize("p", [1, 2, 4, 6, 8])
@pytest.mark.parametrize("eq", ["advection", "burgers", "euler"])
@pytest.mark.parametrize("dim", [1, 2])
def test_elementwise_every_degree(p, eq, dim):
    rng = np.random.default_rng(300 * p + dim)
    if dim == 1:
        prob = W.Problem(dim=1, nx=7, ny=1, p=p, eq=W.EQ_NAMES[eq], vel=(-0.7, 0.0), limiter=W.ELEMENTWISE)
    else:
        prob = W.Problem(dim=2, nx=5, ny=3, p=p, eq=W.EQ_NAMES[eq], vel=(0.6, 1.1), limiter=W.ELEMENTWISE)
    if prob.eq == W.EULER:
        u = W.euler_quadrants(prob, rng)
    else:
        u = rng.uniform(-1.0, 1.0, (1, prob.num_nodes))
    dt = 0.5 * oracle.max_dt(prob, u)
    stage_parity(prob, u, dt)


def test_elementwise_intermediates_match_oracle():
    idp_dg = _gpu()
    wl = W.euler_2d(n=12, p=4)
    prob = wl.prob.replace(limiter=W.ELEMENTWISE)
    dt = wl.cfl * oracle.max_dt(prob, wl.u0)
    ref, tr = oracle.fe(prob, wl.u0, dt, trace=True)
    sv = idp_dg.Solver(prob)
    out = sv.empty()
    g = sv.stage_trace(None, to_dev(wl.u0), out, dt, 0).cpu().numpy()
    np.testing.assert_allclose(g[3], tr["alpha_z"], rtol=0, atol=1e-9)
    np.testing.assert_allclose(g[4], tr["alpha"], rtol=0, atol=1e-9)
    # elementwise: the element's coefficient scales its nodes' whole
    # corrections u^H - u^L
    corr = np.abs(tr["uH"] - tr["uL"]).reshape(prob.nc, -1, 25).max(axis=2)
    da = np.abs(g[4] - tr["alpha"]).reshape(-1, 25).max(axis=1)
    eff = (da[None, :] * corr) / np.abs(wl.u0).max(axis=1)[:, None]
    assert eff.max() <= 1e-12, eff.max()
    a = g[4].reshape(-1, 25)
    assert np.all(a == a[:, :1]) and (a < 1).any()
    assert rel_err(out.cpu().numpy(), ref) <= 1e-12
    sv.close()


@pytest.mark.parametrize("limiter", [W.SUBCELL, W.SUBCELL_SI, W.ELEMENTWISE],
                         ids=["subcell", "subcell_si", "elementwise"])
def test_diagnostics_count_the_traced_coefficients(limiter):
    """The limiter counters of one stage against the stage's own trace:
    limited nodes are those with alpha < 1; entropy nodes are those whose
    own coefficient the entropy search lowered below alpha_z (read from the
    trace where it holds node coefficients; for elementwise limiting, where
    it holds the element minimum, bracketed from the oracle's u^L, u^H and
    K_min: at least the nodes whose state at alpha_z is clearly inadmissible,
    at most those not clearly admissible.  The bracket is needed: with the
    velocity and pressure uniform in a quadrant every flux is linear in the
    density, the update keeps them uniform, K >= K_min is then the same
    constraint as the density's upper bound, and where Zalesak clips the
    density to that bound the state at alpha_z lies on Phi = 0 up to
    rounding)."""
    idp_dg = _gpu()
    wl = W.euler_2d(n=12, p=4)
    # 1 % noise on the energy too, so that the pressure is not uniform in a
    # quadrant and the entropy bound binds clearly at some nodes
    u = wl.u0.copy()
    u[3] *= 1 + 0.01 * np.random.default_rng(7).uniform(-1, 1, u.shape[1])
    prob = wl.prob.replace(limiter=limiter, gmin=float(u[0].min()), gmax=float(u[0].max()))
    dt = wl.cfl * oracle.max_dt(prob, u)
    sv = idp_dg.Solver(prob)
    sv.diagnostics()   # reset
    out = sv.empty()
    g = sv.stage_trace(None, to_dev(u), out, dt, 0).cpu().numpy()
    d = sv.diagnostics()
    assert d["limited_nodes"] == int((g[4] < 1.0).sum()) > 0
    if limiter != W.ELEMENTWISE:
        assert d["entropy_nodes"] == int((g[4] < g[3]).sum()) > 0
    else:
        _, tr = oracle.fe(prob, u, dt, trace=True)
        v = tr["uL"] + tr["alpha_z"] * (tr["uH"] - tr["uL"])
        rhoe = v[3] - 0.5 * (v[1] ** 2 + v[2] ** 2) / v[0]
        r = (rhoe - tr["kmin"] * v[0] ** prob.gamma / (prob.gamma - 1.0)) / np.abs(rhoe)
        lo = int(((v[0] <= 0) | (r < -1e-12)).sum())
        hi = int(((v[0] <= 0) | (r < 1e-12)).sum())
        assert 0 < lo <= d["entropy_nodes"] <= hi, (lo, d["entropy_nodes"], hi)
    sv.close()
