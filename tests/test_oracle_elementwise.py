"""Pins of the oracle's elementwise limiting (ELEMENTWISE mode; Sec. 4.1.2
for linear constraints, eq. convex-provisional-elementwise for the Euler
entropy), checked against its definition recomputed here from the traced
u^H, u^L and bounds:
* each node's provisional coefficient is the Zalesak factor of its single
  correction u^H_i - u^L_i (scalar laws exactly; for Euler the entropy
  search can only lower it, and the state at the found coefficient is
  admissible while a slightly larger one is not, when it was lowered);
* the element applies the minimum over its nodes, and the update is
  u^L + alpha_K (u^H - u^L);
* conservation, the local bounds and positivity hold;
* it is more diffusive than subcell limiting on the smooth advection
  problem (the paper's comparison).
"""
import numpy as np
import pytest

import oracle
from paper_2004_08503_amd import workloads as W


def masses(prob):
    _, w = oracle.gl(prob.p)
    if prob.dim == 1:
        return np.tile(w, prob.nx) * (prob.lx / prob.nx)
    return np.tile(np.outer(w, w).ravel(), prob.nx * prob.ny) * (prob.lx / prob.nx) * (prob.ly / prob.ny)


def phi(V, kmin, gamma, dim):
    rho = V[0]
    mm = sum(V[1 + k] ** 2 for k in range(dim))
    return rho, V[dim + 1] - 0.5 * mm / rho - kmin * rho ** gamma / (gamma - 1.0)


CASES = [
    ("adv1d", W.advection_1d(nx=24, p=3)),
    ("burgers2d", W.burgers_2d(n=10, p=3)),
    ("euler2d", W.euler_2d(n=10, p=4)),
    ("euler1d", W.euler_1d(n=20, p=3)),
]


@pytest.mark.parametrize("name,wl", CASES, ids=[c[0] for c in CASES])
def test_elementwise_definition(name, wl):
    prob = wl.prob.replace(limiter=W.ELEMENTWISE)
    u = wl.u0
    dt = wl.cfl * oracle.max_dt(prob, u)
    out, tr = oracle.fe(prob, u, dt, trace=True)
    uH, uL = tr["uH"], tr["uL"]
    m = masses(prob)
    np_el = (prob.p + 1) ** prob.dim
    # Zalesak with the node's single correction
    f = m / dt * (uH[0] - uL[0])
    Qp = np.maximum(0.0, m / dt * (tr["umax"] - uL[0]))
    Qm = np.minimum(0.0, m / dt * (tr["umin"] - uL[0]))
    with np.errstate(divide="ignore", invalid="ignore"):
        az = np.where(f > 0, np.minimum(1.0, Qp / f), np.where(f < 0, np.minimum(1.0, Qm / f), 1.0))
    assert np.array_equal(tr["alpha_z"], az)
    a = tr["alpha"].reshape(-1, np_el)
    assert np.all(a == a[:, :1])                     # constant per element
    aK = a[:, 0]
    if prob.eq != W.EULER:
        assert np.array_equal(aK, az.reshape(-1, np_el).min(axis=1))
    else:
        assert np.all(aK <= az.reshape(-1, np_el).min(axis=1))
    # the update
    assert np.array_equal(out, uL + tr["alpha"] * (uH - uL))
    # conservation per component
    for c in range(prob.nc):
        assert abs(np.sum(m * (out[c] - u[c]))) <= 1e-14 * np.sum(m * np.abs(u[c]))
    # local bounds of the limited component (IDP)
    sc = np.abs(u[0]).max()
    assert np.all(out[0] <= tr["umax"] + 1e-13 * sc) and np.all(out[0] >= tr["umin"] - 1e-13 * sc)
    assert (aK < 1).any()
    if prob.eq == W.EULER:
        rho, ph = phi(out, tr["kmin"], prob.gamma, prob.dim)
        assert np.all(rho > 0)
        assert np.all(ph >= -1e-12 * np.abs(out[prob.dim + 1]))


def test_elementwise_entropy_search_is_the_supremum():
    wl = W.euler_2d(n=10, p=4)
    prob = wl.prob.replace(limiter=W.ELEMENTWISE)
    dt = wl.cfl * oracle.max_dt(prob, wl.u0)
    _, tr = oracle.fe(prob, wl.u0, dt, trace=True)
    # node-level provisional coefficients: rerun the definition per node with
    # the element minimum removed: for nodes whose element minimum is set by
    # the entropy (alpha_K below every Zalesak factor of the element), the
    # element's limiting node sits on the admissible set's boundary
    np_el = 25
    uH, uL = tr["uH"], tr["uL"]
    a = tr["alpha"].reshape(-1, np_el)[:, 0]
    azm = tr["alpha_z"].reshape(-1, np_el).min(axis=1)
    ent = np.nonzero(a < azm - 1e-12)[0]
    assert len(ent) > 0
    for e in ent[:20]:
        idx = np.arange(e * np_el, (e + 1) * np_el)
        P = uH[:, idx] - uL[:, idx]
        Va = uL[:, idx] + a[e] * P
        Vb = uL[:, idx] + (a[e] + 1e-10) * P
        _, pa = phi(Va, tr["kmin"][idx], prob.gamma, 2)
        _, pb = phi(Vb, tr["kmin"][idx], prob.gamma, 2)
        assert np.all(pa >= -1e-13 * np.abs(Va[3]))      # admissible at alpha_K
        assert (pb < 0).any()                             # some node fails just above


def test_elementwise_more_diffusive_than_subcell():
    def err(limiter, p=3, nx=16):
        prob = W.Problem(dim=1, nx=nx, ny=1, p=p, eq=W.ADVECTION, vel=(1.0, 0.0), limiter=limiter)
        x, _, _ = W.node_coords(prob)
        u = np.sin(2 * np.pi * x)[None, :].copy()
        n = int(np.ceil(0.25 / (0.5 * oracle.max_dt(prob, u))))
        for _ in range(n):
            u = oracle.step(prob, u, 0.25 / n)
        _, w = oracle.gl(p)
        return float(np.sum(np.tile(w, nx) / nx * np.abs(u[0] - np.sin(2 * np.pi * (x - 0.25)))))
    e_el, e_sc = err(W.ELEMENTWISE), err(W.SUBCELL)
    assert e_el > 1.5 * e_sc, (e_el, e_sc)
