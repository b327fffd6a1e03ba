"""The library's curved-mesh set-up (idp_dg_mesh_metric, the host
computation behind idp_dg_set_mesh) against the oracle's metric terms
(oracle.metric), on the CPU: the high-order terms det(J) J^-1, the
corrected terms of eq. metric-perturbation and det(J), degrees 1..8, on
smoothly perturbed and on rotated meshes.

Tolerance 1e-12 of the terms' scale: both sides form the derivatives
along node lines from their own Gauss-Lobatto tables, and a derivative
sum cancels terms up to |D| |x| / |J| (several hundred at p = 8 with the
coordinates' offset) times larger than its result; the corrected terms
also come from different factorisations of the minimum-norm problem
(measured up to 1.6e-13 here).  Also the rejected inputs."""
import numpy as np
import pytest

from oracle import metric as ometric
from paper_2004_08503_amd import idp_dg, workloads as W


@pytest.mark.parametrize("kind", ["perturbed", "rotated"])
@pytest.mark.parametrize("p", range(1, 9))
def test_library_metric_matches_oracle(p, kind):
    prob = W.Problem(dim=2, nx=5, ny=3, p=p, eq=W.EULER, ly=0.7)
    coords = W.perturbed_coords(prob, 0.05) if kind == "perturbed" else W.rotated_coords(prob, 0.7)
    prob = prob.replace(coords=coords)
    got = idp_dg.mesh_metric(prob)
    ref = np.asarray(ometric.metric_terms(prob))
    scale = np.abs(ref[:8]).max()
    assert np.abs(got[:8] - ref[:8]).max() <= 1e-12 * scale
    assert np.abs(got[8] - ref[8]).max() <= 1e-12 * np.abs(ref[8]).max()
    if kind == "perturbed" and p > 1:   # a real correction to compare
        assert np.abs(ref[4:8] - ref[:4]).max() > 1e-6 * scale


def test_rejected_meshes():
    prob = W.Problem(dim=2, nx=3, ny=2, p=3, eq=W.BURGERS)
    xy = W.perturbed_coords(prob, 0.05)
    flipped = xy.copy()
    flipped[0] = -flipped[0]                      # orientation reversed
    for bad in (flipped, np.zeros_like(xy), np.full_like(xy, np.nan)):
        with pytest.raises(idp_dg.IdpError):
            idp_dg.mesh_metric(prob, bad)
    with pytest.raises(idp_dg.IdpError):          # open directions stay Cartesian
        idp_dg.mesh_metric(prob.replace(bc=(1, 0)), xy)
    p1 = W.Problem(dim=1, nx=4, ny=1, p=3, eq=W.BURGERS)
    with pytest.raises(idp_dg.IdpError):          # 2-D only
        idp_dg.mesh_metric(p1, np.zeros((2, p1.num_nodes)))
