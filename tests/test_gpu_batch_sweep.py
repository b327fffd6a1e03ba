"""Seeded random batches: each case draws one equation family (dimension,
equation, and for Euler the gamma kind: 7/5, 5/3, or another gamma per
solve) and two to six member solves that differ in everything else the
batch allows: degree 1..8, mesh 1..12 x 1..9 elements with random side
lengths, limiter mode, velocity (constant or a rotation field), periodic or
open directions with per-node boundary codes and states, and, for 2-D
periodic flux problems, a curved mesh.  Two device-timestepped steps of
the batch must equal, bitwise, each member's own two steps on the plain
path (which the other parity tests pin to the oracle), with the same time
steps."""
import os

import numpy as np
import pytest

from paper_2004_08503_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# 60 batches from seed 9000 in the suite; more with IDP_BATCH_SWEEP_CASES
# and IDP_BATCH_SWEEP_SEED
CASES = int(os.environ.get("IDP_BATCH_SWEEP_CASES", "60"))
SEED0 = int(os.environ.get("IDP_BATCH_SWEEP_SEED", "9000"))


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_08503_amd import idp_dg
    return idp_dg


def member(rng, dim, eq, gamma):
    p = int(rng.integers(1, 9))
    nx = int(rng.integers(1, 13))
    ny = int(rng.integers(1, 10)) if dim == 2 else 1
    lx = float(rng.uniform(0.5, 2.0))
    ly = float(rng.uniform(0.5, 2.0)) if dim == 2 else 1.0
    lim = int(rng.integers(0, 5))
    vel = tuple(float(v) for v in rng.uniform(-1.5, 1.5, 2))
    curved = dim == 2 and eq != W.ADVECTION_FIELD and rng.random() < 0.3
    bc = (0, 0) if curved else (int(rng.integers(0, 2)), int(rng.integers(0, 2)) if dim == 2 else 0)
    prob = W.Problem(dim=dim, nx=nx, ny=ny, p=p, eq=eq, lx=lx, ly=ly, gamma=gamma, limiter=lim,
                     vel=vel, bc=bc)
    if eq == W.ADVECTION_FIELD:
        vr, vc = W.rotation_lines(prob, omega=float(rng.uniform(-7, 7)),
                                  centre=(float(rng.uniform(0, lx)), float(rng.uniform(0, ly))))
        prob = prob.replace(vrows=vr, vcols=vc)
    if curved:
        prob = prob.replace(coords=W.perturbed_coords(prob, float(rng.uniform(0.0, 0.05))))
    u = W.euler_quadrants(prob, rng) if eq == W.EULER else rng.uniform(-1.0, 1.0, (1, prob.num_nodes))
    if any(bc):
        types, states = [None] * 4, [None] * 4
        codes = np.array([W.BC_STATE, W.BC_OUTFLOW, W.BC_SLIP], dtype=np.int8)
        for side in range(4):
            if not bc[side // 2]:
                continue
            n = W.side_nodes(prob, side)
            types[side] = rng.choice(codes, n)
            if rng.random() < 0.8:
                states[side] = np.ascontiguousarray(u[:, rng.integers(0, u.shape[1], n)])
        prob = prob.replace(bnd=W.Boundary(types, states))
    lo, hi = float(u[0].min()), float(u[0].max())
    return prob.replace(gmin=lo - 0.1 * abs(lo), gmax=hi + 0.1 * abs(hi)), u


def random_batch(rng):
    dim = int(rng.integers(1, 3))
    eqs = [W.ADVECTION, W.BURGERS, W.EULER] + ([W.ADVECTION_FIELD] if dim == 2 else [])
    eq = int(rng.choice(eqs))
    kind = int(rng.integers(0, 3))
    n = int(rng.integers(2, 7))
    out = []
    for _ in range(n):
        gamma = [1.4, 5.0 / 3.0, float(rng.choice([1.3, 1.2, 1.55]))][kind]
        out.append(member(rng, dim, eq, gamma))
    return out


@pytest.mark.parametrize("seed", range(CASES))
def test_random_batch_bitwise_equals_plain(seed):
    idp_dg = _gpu()
    cases = random_batch(np.random.default_rng(SEED0 + seed))
    desc = ", ".join("p%d %dx%d lim%d%s%s" % (pr.p, pr.nx, pr.ny, pr.limiter, " open" if any(pr.bc) else "",
                                              " curved" if pr.coords is not None else "") for pr, _ in cases)
    print("seed %d: dim %d eq %d gamma %s: %s" % (SEED0 + seed, cases[0][0].dim, cases[0][0].eq,
                                                  sorted({pr.gamma for pr, _ in cases}), desc), flush=True)
    plain = [idp_dg.Solver(pr) for pr, _ in cases]
    members = [idp_dg.Solver(pr) for pr, _ in cases]
    up = [torch.from_numpy(u.copy()).cuda() for _, u in cases]
    ub = [torch.from_numpy(u.copy()).cuda() for _, u in cases]
    batch = idp_dg.Batch(members)
    try:
        for _ in range(2):
            cfl = 0.5
            batch.step_cfl(ub, cfl)
            for sv, u in zip(plain, up):
                sv.step_cfl(u, cfl)
            assert batch.last_dt() == [sv.last_dt() for sv in plain]
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(ub, up)):
            assert torch.equal(a, b), "member %d" % k
    finally:
        batch.close()
        for sv in plain + members:
            sv.close()
