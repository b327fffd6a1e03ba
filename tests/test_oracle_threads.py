"""The oracle's OpenMP loops change nothing: every node's arithmetic is the
same on any number of threads, so a step, a traced forward-Euler sub-step
and the time-step bound are bitwise equal on one thread and on several."""
import numpy as np
import pytest

import oracle
from paper_2004_08503_amd import workloads as W


def cases():
    rng = np.random.default_rng(43)
    out = [W.euler_2d(n=10, p=4), W.burgers_2d(n=9, p=3), W.euler_1d(n=40, p=3),
           W.advection_1d(), W.solid_body(n=8, p=3)]
    for wl in list(out[:2]):
        for lim in (W.ELEMENTWISE, W.SUBCELL_SI):
            prob = wl.prob.replace(limiter=lim)
            if lim == W.SUBCELL_SI:
                prob = prob.replace(gmin=float(wl.u0[0].min()), gmax=float(wl.u0[0].max()))
            out.append(W.Workload(wl.name + "-lim%d" % lim, prob, wl.u0, wl.cfl, 1))
    prob = W.Problem(dim=2, nx=6, ny=5, p=3, eq=W.EULER, bc=(1, 1))
    codes = [W.BC_STATE, W.BC_OUTFLOW, W.BC_SLIP, W.BC_SLIP]
    st = np.array([1.1, 0.2, -0.1, 2.4])
    prob = prob.replace(bnd=W.uniform_boundary(prob, codes, [st, None, None, None]))
    out.append(W.Workload("euler-open", prob, W.euler_quadrants(prob, rng), 0.5, 1))
    return out


@pytest.mark.parametrize("wl", cases(), ids=lambda w: w.name)
def test_threads_do_not_change_results(wl):
    prob, u = wl.prob, wl.u0
    res = {}
    try:
        for n in (1, 8):
            oracle.set_threads(n)
            dt = oracle.max_dt(prob, u)
            step = oracle.step(prob, u, wl.cfl * dt)
            _, tr = oracle.fe(prob, u, wl.cfl * dt, trace=True)
            res[n] = (dt, step, tr)
    finally:
        oracle.set_threads(1)
    assert res[1][0] == res[8][0]
    np.testing.assert_array_equal(res[1][1], res[8][1])
    for k in res[1][2]:
        np.testing.assert_array_equal(res[1][2][k], res[8][2][k])
