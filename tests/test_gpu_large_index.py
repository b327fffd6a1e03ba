"""Meshes whose arrays pass 2^31 elements: 64-bit addressing end to end.

A state that repeats a small periodic pattern of elements is periodic on
every multiple of that pattern, and the scheme's arithmetic at a node
depends only on the values it reads, not on where the node sits, which
tile or workgroup runs it, or how many elements the mesh has (the element
size lx/nx is the same correctly rounded number).  So one device-timestepped
SSP-RK3 step on the large mesh must equal, bitwise, the step of the small
pattern mesh repeated, and its time step must equal the pattern's (a
minimum over the same values); the same holds for the large mesh stepped
in a batch beside the pattern.  The pattern's own step is checked against
the oracle.  Two cases:

- 2-D Euler at p = 4 on 4640^2 elements (538 M nodes): the flattened state
  index c Nn + node passes 2^31 in the last component;
- 2-D Burgers at p = 8 on 5152^2 elements (2.15 G nodes): the node index
  itself passes 2^31.

Each needs about 55 GB of device memory (state 17 GB, the handle's two
stage buffers 34 GB)."""
import numpy as np
import pytest

import oracle
from paper_2004_08503_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu(need_bytes):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    free, _ = torch.cuda.mem_get_info()
    if free < need_bytes:
        pytest.skip("needs %.0f GB of free device memory" % (need_bytes / 1e9))
    from paper_2004_08503_amd import idp_dg
    return idp_dg


CASES = {
    # name: (pattern workload, repeats per direction)
    "euler_p4_4640": (lambda: W.euler_2d(n=20, p=4, seed=11), 232),
    "burgers_p8_5152": (lambda: W.burgers_2d(n=16, p=8, seed=12), 322),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_repeated_pattern_beyond_2_31(name):
    make, rep = CASES[name]
    wl = make()
    small = wl.prob
    big = small.replace(nx=small.nx * rep, ny=small.ny * rep, lx=small.lx * rep, ly=small.ly * rep)
    nc, npe = small.nc, small.nodes_per_element
    n_big = big.num_nodes
    assert nc * n_big > 2 ** 31
    if name.startswith("burgers"):
        assert n_big > 2 ** 31
    idp_dg = _gpu(int(3.3 * 8 * nc * n_big))

    # the pattern: one step on the device, checked against the oracle
    sv = idp_dg.Solver(small)
    us = torch.from_numpy(wl.u0.copy()).cuda()
    sv.step_cfl(us, wl.cfl)
    dt_small = sv.last_dt()
    sv.close()
    ref = oracle.step(small, wl.u0, dt_small)
    err = np.abs(us.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err <= 1e-12, err
    assert dt_small == pytest.approx(wl.cfl * oracle.max_dt(small, wl.u0), rel=1e-12)

    def repeated():
        # the pattern repeated rep x rep times (state order u[c][ey][ex][node])
        u0 = torch.from_numpy(wl.u0).cuda().view(nc, small.ny, small.nx, npe)
        return u0.repeat(1, rep, rep, 1).reshape(nc, n_big)

    def differing(ub):
        got = ub.view(nc, rep, small.ny, rep, small.nx, npe)
        want = us.view(nc, 1, small.ny, 1, small.nx, npe)
        return int((got != want).sum().item())

    print("%s: %d x %d elements, %d nodes, %d doubles per state" % (name, big.nx, big.ny, n_big, nc * n_big),
          flush=True)
    ub = repeated()
    sv = idp_dg.Solver(big)
    sv.step_cfl(ub, wl.cfl)
    dt_big = sv.last_dt()
    sv.close()
    assert dt_big == dt_small, (dt_big, dt_small)
    ndiff = differing(ub)
    del ub
    torch.cuda.empty_cache()
    print("%s: one step, nodes differing from the repeated pattern: %d" % (name, ndiff), flush=True)
    assert ndiff == 0

    # the same step of the large mesh in a batch beside the pattern itself
    # (one work list over both solves' tiles)
    ub = repeated()
    u1 = torch.from_numpy(wl.u0.copy()).cuda()
    sb, ss = idp_dg.Solver(big), idp_dg.Solver(small)
    bt = idp_dg.Batch([sb, ss])
    bt.step_cfl([ub, u1], wl.cfl)
    dts = bt.last_dt()
    bt.close()
    sb.close()
    ss.close()
    assert dts == [dt_small, dt_small], dts
    assert torch.equal(u1, us)
    ndiff = differing(ub)
    del ub
    torch.cuda.empty_cache()
    print("%s: batched step, nodes differing from the repeated pattern: %d" % (name, ndiff))
    assert ndiff == 0
