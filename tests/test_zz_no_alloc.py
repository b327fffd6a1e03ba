"""idp_dg_step_noalloc (the step without a handle, on the library's static
stage buffers) against idp_dg_step on a handle: bitwise equal, on two calls
in a row, the second with a smaller input, and within 1e-12 of the oracle;
sizes beyond the static buffers are refused with a message."""
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
    scale = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return (np.abs(a - b).max(axis=1) / scale).max()


def one_case(idp_dg, wl, check_oracle):
    prob, u0 = wl.prob, wl.u0
    dt = wl.cfl * oracle.max_dt(prob, u0)
    print("noalloc case %s %dx%d p=%d nc*Nn=%d" % (wl.name, prob.nx, prob.ny, prob.p,
                                                    prob.nc * prob.num_nodes), flush=True)
    sv = idp_dg.Solver(prob)
    ref = torch.from_numpy(u0.copy()).to("cuda")
    sv.step(ref, dt)
    got = torch.from_numpy(u0.copy()).to("cuda")
    idp_dg.step_noalloc(prob, got, dt)
    torch.cuda.synchronize()
    sv.close()
    a, b = got.cpu().numpy(), ref.cpu().numpy()
    assert np.array_equal(a, b), np.abs(a - b).max()
    if check_oracle:
        assert rel_err(a, oracle.step(prob, u0, dt)) <= 1e-12


def test_noalloc_step_equals_handle_step():
    idp_dg = _gpu()
    big = W.euler_2d(n=40, p=4)                  # 4 * 40000 doubles
    small = W.burgers_2d(n=12, p=3)              # 2304 doubles
    one_case(idp_dg, big, check_oracle=False)
    one_case(idp_dg, small, check_oracle=True)
    one_case(idp_dg, W.euler_1d(n=24, p=5), check_oracle=True)


def test_noalloc_refuses_what_it_cannot_hold():
    idp_dg = _gpu()
    prob = W.euler_2d(n=8, p=4).prob.replace(nx=256, ny=256)   # 6.5 M doubles
    u = torch.zeros((1, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        idp_dg.step_noalloc(prob, u, 1e-3)      # the binding checks the tensor first
    d = idp_dg.make_desc(prob)
    import ctypes
    rc = idp_dg.lib.idp_dg_step_noalloc(ctypes.byref(d), ctypes.c_void_p(u.data_ptr()), 1e-3, None)
    assert rc == idp_dg.EINVAL
    assert "exceeds" in idp_dg.lib.idp_dg_last_error(None).decode()
    wall = W.euler_2d(n=8, p=2).prob.replace(bc=(1, 0))
    d = idp_dg.make_desc(wall)
    rc = idp_dg.lib.idp_dg_step_noalloc(ctypes.byref(d), ctypes.c_void_p(u.data_ptr()), 1e-3, None)
    assert rc == idp_dg.EINVAL and "periodic" in idp_dg.lib.idp_dg_last_error(None).decode()
