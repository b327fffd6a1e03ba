"""Pins of the oracle's tables (Sec. 2.1-2.2 and eq. didp) against closed
forms, quadrature exactness and the properties P1/P2 the paper states."""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("p,xi_ref,w_ref", [
    (1, [0.0, 1.0], [0.5, 0.5]),
    (2, [0.0, 0.5, 1.0], [1 / 6, 2 / 3, 1 / 6]),
    (3, [0.0, (1 - 1 / np.sqrt(5)) / 2, (1 + 1 / np.sqrt(5)) / 2, 1.0],
     [1 / 12, 5 / 12, 5 / 12, 1 / 12]),
    (4, [0.0, (1 - np.sqrt(3 / 7)) / 2, 0.5, (1 + np.sqrt(3 / 7)) / 2, 1.0],
     [1 / 20, 49 / 180, 16 / 45, 49 / 180, 1 / 20]),
])
def test_gl_closed_forms(p, xi_ref, w_ref):
    xi, w = oracle.gl(p)
    np.testing.assert_allclose(xi, xi_ref, rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, w_ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("p", range(1, 9))
def test_gl_quadrature_exactness(p):
    """Gauss-Lobatto with p+1 points integrates degree 2p-1 exactly and not
    degree 2p; end weights are 1/(p(p+1))."""
    xi, w = oracle.gl(p)
    assert abs(w.sum() - 1.0) < 1e-14
    for k in range(2 * p):
        assert abs(np.dot(w, xi ** k) - 1.0 / (k + 1)) < 1e-14
    assert abs(np.dot(w, xi ** (2 * p)) - 1.0 / (2 * p + 1)) > 1e-12
    assert abs(w[0] - 1.0 / (p * (p + 1))) < 1e-15
    assert abs(w[-1] - 1.0 / (p * (p + 1))) < 1e-15
    assert np.all(np.diff(xi) > 0)


def test_dmat_explicit_small():
    np.testing.assert_allclose(oracle.dmat(1), [[-0.5, 0.5], [-0.5, 0.5]], atol=1e-15)
    np.testing.assert_allclose(
        oracle.dmat(2),
        [[-0.5, 2 / 3, -1 / 6], [-2 / 3, 0.0, 2 / 3], [1 / 6, -2 / 3, 0.5]], atol=1e-15)


@pytest.mark.parametrize("p", range(1, 9))
def test_dmat_properties(p):
    """P1 (row sums vanish), P2 (SBP column sums) and exact differentiation
    of monomials up to degree p: D xi^k = w * k xi^(k-1)."""
    D = oracle.dmat(p)
    xi, w = oracle.gl(p)
    np.testing.assert_allclose(D.sum(axis=1), 0.0, atol=1e-13)
    col = np.zeros(p + 1)
    col[0], col[-1] = -1.0, 1.0
    np.testing.assert_allclose(D.sum(axis=0), col, atol=1e-13)
    for k in range(1, p + 1):
        np.testing.assert_allclose(D @ xi ** k, w * k * xi ** (k - 1), atol=1e-13)
    # summation by parts: D + D^T = B (the boundary matrix)
    B = np.zeros((p + 1, p + 1))
    B[0, 0], B[-1, -1] = -1.0, 1.0
    np.testing.assert_allclose(D + D.T, B, atol=1e-13)


def test_dhat_printed_block():
    ref = np.loadtxt(os.path.join(GOLDEN, "dhat_printed.txt"))
    for p in range(3, 9):
        np.testing.assert_allclose(oracle.dhat(p)[:3, :4], ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("p", range(1, 9))
def test_dhat_properties(p):
    """Dhat keeps P1 and P2 (Sec. 3) and is first-order exact: it
    differentiates linear functions like D does."""
    Dh = oracle.dhat(p)
    np.testing.assert_allclose(Dh.sum(axis=1), 0.0, atol=1e-15)
    col = np.zeros(p + 1)
    col[0], col[-1] = -1.0, 1.0
    np.testing.assert_allclose(Dh.sum(axis=0), col, atol=1e-15)
    # tridiagonal with +-1/2 off the diagonal
    assert np.count_nonzero(np.triu(Dh, 2)) == 0
    assert np.count_nonzero(np.tril(Dh, -2)) == 0
    np.testing.assert_allclose(np.diag(Dh, 1), 0.5, rtol=0, atol=1e-15)
    np.testing.assert_allclose(np.diag(Dh, -1), -0.5, rtol=0, atol=1e-15)
