"""Pins of the oracle's variable-velocity advection (ADVECTION_FIELD,
Sec. 3.3: u_t + div(beta u) = 0 with the modified bar states and graph
viscosity), against what the paper and the mathematics fix:
* a constant field gives exactly the constant-velocity scheme (itself pinned
  against dense assembly, the convergence table and the limiter pins);
* the discrete divergence-free identity: the rotation field of the paper's
  solid-body test passes, a divergence-free field that is not line-separable
  fails it and is rejected;
* a constant state stays constant (the property the modified bar states are
  introduced for), mass is conserved, the low-order and limited updates stay
  within the data's range and the limited one within its local bounds;
* a smooth bump carried an eighth of a revolution converges to the exactly
  rotated bump at the target scheme's order.
"""
import numpy as np
import pytest

import oracle
from paper_2004_08503_amd import workloads as W

MODES = [W.SUBCELL, W.TARGET, W.LOW, W.ELEMENTWISE]


def field_problem(nx, ny, p, bx, by, limiter=W.SUBCELL):
    return W.Problem(dim=2, nx=nx, ny=ny, p=p, eq=W.ADVECTION_FIELD, limiter=limiter,
                     vrows=tuple(np.broadcast_to(bx, (ny * (p + 1),))),
                     vcols=tuple(np.broadcast_to(by, (nx * (p + 1),))))


def masses(prob):
    _, w = oracle.gl(prob.p)
    hx, hy = prob.lx / prob.nx, prob.ly / prob.ny
    return np.tile(np.outer(w, w).reshape(-1), prob.nx * prob.ny) * hx * hy


@pytest.mark.parametrize("limiter", MODES)
def test_constant_field_is_the_constant_velocity_scheme(limiter):
    rng = np.random.default_rng(11)
    vx, vy = -0.7, 1.3
    pf = field_problem(5, 3, 3, vx, vy, limiter)
    pc = W.Problem(dim=2, nx=5, ny=3, p=3, eq=W.ADVECTION, vel=(vx, vy), limiter=limiter)
    u = rng.uniform(0.0, 1.0, (1, pf.num_nodes))
    assert oracle.max_dt(pf, u) == pytest.approx(oracle.max_dt(pc, u), rel=1e-14)
    dt = 0.5 * oracle.max_dt(pc, u)
    of, tf = oracle.fe(pf, u, dt, trace=True)
    oc, tc = oracle.fe(pc, u, dt, trace=True)
    np.testing.assert_allclose(of, oc, rtol=0, atol=1e-14)
    for k in ("uL", "uH", "umin", "umax", "alpha"):
        np.testing.assert_allclose(tf[k], tc[k], rtol=0, atol=1e-13, err_msg=k)


def test_divergence_free_identity_decides_admission():
    wl = W.solid_body(n=6, p=4)
    assert oracle.check(wl.prob) == 0
    # a divergence-free field from the stream function sin^2(pi x) sin^2(pi y):
    # beta_x varies along x-lines, so the identity fails on the mesh
    x, y, _ = W.node_coords(wl.prob)
    bx = 2 * np.pi * np.sin(np.pi * x) ** 2 * np.sin(np.pi * y) * np.cos(np.pi * y)
    by = -2 * np.pi * np.sin(np.pi * x) * np.cos(np.pi * x) * np.sin(np.pi * y) ** 2
    bad = wl.prob.replace()
    bad.beta = np.stack([bx, by])
    assert oracle.check(bad) != 0
    # the same nodal arrays expanded from the line samples pass
    ok = wl.prob.replace()
    ok.beta = oracle.nodal_velocity(wl.prob)
    assert oracle.check(ok) == 0
    # a one-dimensional problem cannot carry a field
    assert oracle.check(W.Problem(dim=1, nx=4, ny=1, p=2, eq=W.ADVECTION_FIELD)) != 0


@pytest.mark.parametrize("limiter", MODES)
def test_constant_state_is_preserved(limiter):
    wl = W.solid_body(n=6, p=3, limiter=limiter)
    u = np.full_like(wl.u0, 0.7)
    dt = 0.5 * oracle.max_dt(wl.prob, u)
    out, tr = oracle.fe(wl.prob, u, dt, trace=True)
    np.testing.assert_allclose(tr["uL"], 0.7, rtol=0, atol=1e-14)
    np.testing.assert_allclose(tr["uH"], 0.7, rtol=0, atol=1e-13)
    np.testing.assert_allclose(out, 0.7, rtol=0, atol=1e-13)


@pytest.mark.parametrize("limiter", MODES)
def test_conservation_and_bounds(limiter):
    wl = W.solid_body(n=7, p=3, limiter=limiter)
    rng = np.random.default_rng(3)
    u = rng.uniform(0.0, 1.0, wl.u0.shape)
    m = masses(wl.prob)
    dt = oracle.max_dt(wl.prob, u)     # the CFL limit itself
    out, tr = oracle.fe(wl.prob, u, dt, trace=True)
    total = (m * u[0]).sum()
    for v in (out[0], tr["uL"][0], tr["uH"][0]):
        assert abs((m * v).sum() - total) <= 1e-14 * total
    assert tr["uL"].min() >= u.min() - 1e-14 and tr["uL"].max() <= u.max() + 1e-14
    if limiter in (W.SUBCELL, W.ELEMENTWISE):
        assert np.all(out[0] >= tr["umin"] - 1e-13) and np.all(out[0] <= tr["umax"] + 1e-13)
        assert (tr["alpha"] < 1).any()


def rotated_bump(prob, t):
    """A Gaussian of width 0.05 centred at (0.5, 0.25), rotated by 2 pi t
    about (0.5, 0.5)."""
    x, y, _ = W.node_coords(prob)
    th = -2 * np.pi * t
    xr = 0.5 + np.cos(th) * (x - 0.5) - np.sin(th) * (y - 0.5)
    yr = 0.5 + np.sin(th) * (x - 0.5) + np.cos(th) * (y - 0.5)
    return np.exp(-((xr - 0.5) ** 2 + (yr - 0.25) ** 2) / (2 * 0.05 ** 2))[None, :]


def rotation_error(n, limiter, t_end=0.125):
    wl = W.solid_body(n=n, p=3, limiter=limiter)
    prob = wl.prob
    u = rotated_bump(prob, 0.0)
    dt0 = 0.5 * oracle.max_dt(prob, u)
    t = 0.0
    while t < t_end - 1e-14:
        dt = min(dt0, t_end - t)
        u = oracle.step(prob, u, dt)
        t += dt
    return (masses(prob) * np.abs(u[0] - rotated_bump(prob, t_end)[0])).sum()


def test_rotation_converges():
    e8, e16 = rotation_error(8, W.TARGET), rotation_error(16, W.TARGET)
    assert e16 < e8 / 8, (e8, e16)          # order p + 1 = 4 expected
    l8, l16 = rotation_error(8, W.SUBCELL), rotation_error(16, W.SUBCELL)
    assert l16 < l8 / 3, (l8, l16)
    assert e16 <= l16 <= 3 * e16, (e16, l16)
