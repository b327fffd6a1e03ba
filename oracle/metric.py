"""Metric terms of curved meshes for the CPU oracle (TEST INFRASTRUCTURE
ONLY; part of the oracle, independent of the HIP library).

From the node coordinates of every element (the isoparametric map of the
reference square [0,1]^2):
- the metric terms det(J) J^-1 (Sec. 2.3), rows xi, eta and columns x, y:
  (y_eta, -x_eta) and (-y_xi, x_xi), with the derivatives taken by the
  Gauss-Lobatto derivative matrix along the element's node lines.  In 2-D
  this form satisfies the discrete metric identities (eq. metric) exactly up
  to rounding, since the one-dimensional derivatives along xi and eta
  commute (the freestream-preserving evaluation the paper cites);
- det(J) = x_xi y_eta - x_eta y_xi;
- the conservative correction C (Sec. 3.1, eq. idp-sbp / eq.
  metric-perturbation): per element and physical direction j, the
  minimum-norm solution of
      [Dhat_1^T Dhat_2^T] [C_1j 1; C_2j 1]
          = sum_e B_e n_ej 1 - [Dhat_1^T Dhat_2^T] [Jinv_1j 1; Jinv_2j 1],
  with Dhat_k^T the Kronecker operators of eq. kronecker built from Dhat,
  computed with numpy's pseudo-inverse (a singular value decomposition of
  the reference operator, once per degree), as the paper describes.

Returns the (9, Nn) array of idp_ref_desc.metric: the four high-order
terms, the four modified terms det(J) J^-1 + C, and det(J).  The last two
results are kept (read-only) and returned again for the same degree, mesh
and coordinates, so that stepping a large curved mesh does not recompute
them for every oracle call.
"""
import hashlib

import numpy as np

_CACHE = []   # [(key, array)], most recent last, at most two entries


def _tables(p):
    import oracle
    D = oracle.dmat(p)          # weighted: D[a][c] = w_a l_c'(xi_a)
    Dh = oracle.dhat(p)
    _, w = oracle.gl(p)
    return D, Dh, w


def _lo_operator(p, Dh, w):
    """A = [Dhat_xi^T, Dhat_eta^T] on the nodes (a, b) of an element (node
    index b*(p+1) + a): (Dhat_xi^T g)_(a,b) = w_b sum_c Dhat[c][a] g_(c,b)
    and (Dhat_eta^T g)_(a,b) = w_a sum_c Dhat[c][b] g_(a,c)."""
    n1 = p + 1
    N = n1 * n1
    A = np.zeros((N, 2 * N))
    for b in range(n1):
        for a in range(n1):
            i = b * n1 + a
            for c in range(n1):
                A[i, b * n1 + c] += w[b] * Dh[c, a]
                A[i, N + c * n1 + a] += w[a] * Dh[c, b]
    return A


def metric_terms(prob):
    """The (9, Nn) metric array of a 2-D curved mesh given by prob.coords."""
    xy = np.ascontiguousarray(prob.coords, dtype=np.float64)
    key = (prob.p, prob.nx, prob.ny, xy.shape, hashlib.sha1(xy.tobytes()).hexdigest())
    for k, a in _CACHE:
        if k == key:
            return a
    out = _metric_terms(prob)
    out.setflags(write=False)
    _CACHE.append((key, out))
    del _CACHE[:-2]
    return out


def _metric_terms(prob):
    p, n1 = prob.p, prob.p + 1
    D, Dh, w = _tables(p)
    Dn = D / w[:, None]                      # plain derivative matrix l_c'(xi_a)
    X = np.asarray(prob.coords, dtype=np.float64).reshape(2, -1, n1, n1)   # [comp][e][b][a]
    x, y = X[0], X[1]
    x_xi = np.einsum("ac,ebc->eba", Dn, x)
    y_xi = np.einsum("ac,ebc->eba", Dn, y)
    x_eta = np.einsum("bc,eca->eba", Dn, x)
    y_eta = np.einsum("bc,eca->eba", Dn, y)
    J = np.stack([y_eta, -x_eta, -y_xi, x_xi])              # rows xi, eta; columns x, y
    det = x_xi * y_eta - x_eta * y_xi
    A = _lo_operator(p, Dh, w)
    Ap = np.linalg.pinv(A)
    ne = X.shape[1]
    N = n1 * n1
    Jidp = J.copy()
    for e in range(ne):
        for j in range(2):
            g_xi = J[0 + j, e].reshape(N)                   # Jinv_{xi, j}
            g_eta = J[2 + j, e].reshape(N)                  # Jinv_{eta, j}
            bnd = np.zeros((n1, n1))                        # sum_e B_e n_ej at node [b][a]
            bnd[:, 0] -= w * J[0 + j, e][:, 0]
            bnd[:, p] += w * J[0 + j, e][:, p]
            bnd[0, :] -= w * J[2 + j, e][0, :]
            bnd[p, :] += w * J[2 + j, e][p, :]
            rhs = bnd.reshape(N) - A @ np.concatenate([g_xi, g_eta])
            C = Ap @ rhs
            Jidp[0 + j, e] = (g_xi + C[:N]).reshape(n1, n1)
            Jidp[2 + j, e] = (g_eta + C[N:]).reshape(n1, n1)
    out = np.concatenate([J.reshape(4, -1), Jidp.reshape(4, -1), det.reshape(1, -1)])
    return np.ascontiguousarray(out)
