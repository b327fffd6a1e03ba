// Curved meshes: the metric terms of the isoparametric map (Sec. 2.3) and
// the conservative correction of the low-order operator's metric terms
// (Sec. 3.1, eq. idp-sbp, eq. metric-perturbation), computed on the host
// once per mesh from the node coordinates and kept on the device in the
// layout the stage and time-step kernels read: metric[q * Nn + node] with
// q = 0..3 the high-order terms (xi, x), (xi, y), (eta, x), (eta, y),
// q = 4..7 the corrected terms in the same order, q = 8 det(J).
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/idp_dg.h"
#include "common.hpp"
#include "handle.hpp"

using namespace idp;
using idp_host::desc_ok;
using idp_host::fail;

namespace {

constexpr int MAXN2 = (MAXP + 1) * (MAXP + 1);

// The element operator of eq. metric-perturbation, [Dhat_xi^T  Dhat_eta^T],
// as a dense N x 2N matrix on the nodes (a, b) -> b (p+1) + a of one
// element (eq. kronecker with the one-dimensional low-order matrix Dhat of
// eq. didp and the Gauss-Lobatto weights of the other direction).
// Dhat: -1/2 and +1/2 on the first and last diagonal entries, +1/2 above
// and -1/2 below the diagonal.
struct LoOperator {
  int n1 = 0, N = 0;
  std::vector<double> dh;   // [n1][n1]
  std::vector<double> A;    // [N][2N]
  std::vector<double> L;    // Cholesky factor of A A^T + 1 1^T, [N][N] lower

  bool build(int p, const double* w) {
    n1 = p + 1;
    N = n1 * n1;
    dh.assign(n1 * n1, 0.0);
    for (int m = 0; m < p; ++m) {   // the linear hat functions of subcell m
      dh[m * n1 + m] -= 0.5;
      dh[m * n1 + m + 1] += 0.5;
      dh[(m + 1) * n1 + m] -= 0.5;
      dh[(m + 1) * n1 + m + 1] += 0.5;
    }
    A.assign((size_t)N * 2 * N, 0.0);
    for (int b = 0; b < n1; ++b)
      for (int a = 0; a < n1; ++a) {
        double* row = &A[(size_t)(b * n1 + a) * 2 * N];
        for (int c = 0; c < n1; ++c) {
          row[b * n1 + c] += w[b] * dh[c * n1 + a];       // Dhat_xi^T acting on g(c, b)
          row[N + c * n1 + a] += w[a] * dh[c * n1 + b];   // Dhat_eta^T acting on g(a, c)
        }
      }
    // Every row of Dhat sums to zero, so 1^T A = 0: the constants span the
    // operator's left null space (its rank is N - 1), A A^T + 1 1^T is
    // symmetric positive definite, and on right-hand sides orthogonal to
    // the constants its inverse acts as the pseudo-inverse of A A^T.  So
    // A^T (A A^T + 1 1^T)^-1 r is the minimum-norm solution of A C = r
    // (any rounding component of r along the constants is annihilated by
    // A^T).  A singular factor (rank below N - 1) is reported.
    L.assign((size_t)N * N, 0.0);
    for (int i = 0; i < N; ++i)
      for (int j = 0; j <= i; ++j) {
        double s = 1.0;
        const double* ri = &A[(size_t)i * 2 * N];
        const double* rj = &A[(size_t)j * 2 * N];
        for (int k = 0; k < 2 * N; ++k) s += ri[k] * rj[k];
        L[(size_t)i * N + j] = s;
      }
    for (int j = 0; j < N; ++j) {   // in-place Cholesky, lower triangle
      double d = L[(size_t)j * N + j];
      for (int k = 0; k < j; ++k) d -= L[(size_t)j * N + k] * L[(size_t)j * N + k];
      if (!(d > 0.0)) return false;
      d = std::sqrt(d);
      L[(size_t)j * N + j] = d;
      for (int i = j + 1; i < N; ++i) {
        double s = L[(size_t)i * N + j];
        for (int k = 0; k < j; ++k) s -= L[(size_t)i * N + k] * L[(size_t)j * N + k];
        L[(size_t)i * N + j] = s / d;
      }
    }
    return true;
  }

  // r <- (A A^T + 1 1^T)^-1 r
  void solve(double* r) const {
    for (int i = 0; i < N; ++i) {
      double s = r[i];
      for (int k = 0; k < i; ++k) s -= L[(size_t)i * N + k] * r[k];
      r[i] = s / L[(size_t)i * N + i];
    }
    for (int i = N - 1; i >= 0; --i) {
      double s = r[i];
      for (int k = i + 1; k < N; ++k) s -= L[(size_t)k * N + i] * r[k];
      r[i] = s / L[(size_t)i * N + i];
    }
  }
};

// Metric terms of element e into met (layout above).  false when det(J) is
// not positive or a value is not finite.
bool element_metric(const LoOperator& lo, const double* w, const double* Dn, const double* coords,
                    long long nn, long long e, double* met) {
  const int n1 = lo.n1, N = lo.N;
  const long long g0 = e * N;
  const double* x = coords + g0;
  const double* y = coords + nn + g0;
  double J[4][MAXN2], xdet[MAXN2];
  for (int b = 0; b < n1; ++b)
    for (int a = 0; a < n1; ++a) {
      double x_xi = 0.0, y_xi = 0.0, x_eta = 0.0, y_eta = 0.0;
      for (int c = 0; c < n1; ++c) {
        x_xi += Dn[a * n1 + c] * x[b * n1 + c];
        y_xi += Dn[a * n1 + c] * y[b * n1 + c];
        x_eta += Dn[b * n1 + c] * x[c * n1 + a];
        y_eta += Dn[b * n1 + c] * y[c * n1 + a];
      }
      const int k = b * n1 + a;
      J[0][k] = y_eta;
      J[1][k] = -x_eta;
      J[2][k] = -y_xi;
      J[3][k] = x_xi;
      xdet[k] = x_xi * y_eta - x_eta * y_xi;
      if (!(xdet[k] > 0.0) || !std::isfinite(xdet[k])) return false;
    }
  const int p = n1 - 1;
  for (int j = 0; j < 2; ++j) {   // physical direction
    const double* gx = J[j];       // row xi, column j
    const double* ge = J[2 + j];   // row eta, column j
    // right-hand side: the boundary term sum_e B_e n_ej 1 (the outward
    // scaled normals are the metric rows on the element's faces) minus the
    // low-order operator applied to the high-order terms
    double r[MAXN2];
    for (int b = 0; b < n1; ++b)
      for (int a = 0; a < n1; ++a) {
        const int k = b * n1 + a;
        double s = 0.0;
        if (a == 0) s -= w[b] * gx[k];
        if (a == p) s += w[b] * gx[k];
        if (b == 0) s -= w[a] * ge[k];
        if (b == p) s += w[a] * ge[k];
        const double* row = &lo.A[(size_t)k * 2 * N];
        for (int m = 0; m < N; ++m) s -= row[m] * gx[m] + row[N + m] * ge[m];
        r[k] = s;
      }
    lo.solve(r);
    for (int m = 0; m < N; ++m) {   // C = A^T r, added to the high-order terms
      double cx = 0.0, ce = 0.0;
      for (int k = 0; k < N; ++k) {
        cx += lo.A[(size_t)k * 2 * N + m] * r[k];
        ce += lo.A[(size_t)k * 2 * N + N + m] * r[k];
      }
      met[(4 + j) * nn + g0 + m] = gx[m] + cx;
      met[(6 + j) * nn + g0 + m] = ge[m] + ce;
    }
  }
  for (int k = 0; k < N; ++k) {
    for (int q = 0; q < 4; ++q) met[q * nn + g0 + k] = J[q][k];
    met[8 * nn + g0 + k] = xdet[k];
  }
  for (int q = 4; q < 8; ++q)
    for (int k = 0; k < N; ++k)
      if (!std::isfinite(met[q * nn + g0 + k])) return false;
  return true;
}

// The metric array of a mesh of ne elements of degree p into met (9 nn
// doubles); on failure the message goes to *why.
bool mesh_metric(int p, long long ne, long long nn, const double* coords, double* met, std::string* why) {
  double w[MAXP + 1], Dn[(MAXP + 1) * (MAXP + 1)];
  idp_host::gl_derivative(p, w, Dn);
  LoOperator lo;
  if (!lo.build(p, w)) {
    *why = "curved meshes: singular correction system";
    return false;
  }
  for (long long e = 0; e < ne; ++e)
    if (!element_metric(lo, w, Dn, coords, nn, e, met)) {
      *why = "curved meshes: det(J) not positive or a non-finite value in element " + std::to_string(e);
      return false;
    }
  return true;
}

// The problems a curved mesh supports; false with the reason otherwise.
bool curved_ok(const idp_dg_desc* d, std::string* why) {
  if (d->dim != 2) *why = "curved meshes: 2-D problems only";
  else if (d->eq == IDP_DG_ADVECTION_FIELD) *why = "curved meshes: not with an advection velocity field";
  else if (d->bc[0] != IDP_DG_BC_PERIODIC || d->bc[1] != IDP_DG_BC_PERIODIC)
    *why = "curved meshes: periodic directions only";
  else return true;
  return false;
}

}  // namespace

extern "C" int idp_dg_mesh_metric(const idp_dg_desc* desc, const double* coords, double* metric) {
  std::string why;
  if (!desc_ok(desc, &why) || !curved_ok(desc, &why)) return fail(nullptr, IDP_DG_EINVAL, why);
  if (!coords || !metric) return fail(nullptr, IDP_DG_EINVAL, "coords or metric is NULL");
  const long long n1 = desc->p + 1, ne = (long long)desc->nx * desc->ny;
  if (!mesh_metric(desc->p, ne, ne * n1 * n1, coords, metric, &why)) return fail(nullptr, IDP_DG_EINVAL, why);
  return 0;
}

extern "C" int idp_dg_set_mesh(idp_dg* h, const double* coords) {
  const idp_host::Range trace_range("idp_dg_set_mesh");
  if (!h) return IDP_DG_EINVAL;
  if (!coords) return fail(h, IDP_DG_EINVAL, "coords is NULL");
  std::string why;
  if (!curved_ok(&h->d, &why)) return fail(h, IDP_DG_EINVAL, why);
  if (!h->owns) return fail(h, IDP_DG_EINVAL, "curved meshes: the handle lives in a caller workspace");
  std::vector<double> met((size_t)9 * h->nn);
  if (!mesh_metric(h->d.p, h->ne, h->nn, coords, met.data(), &why)) return fail(h, IDP_DG_EINVAL, why);
  // queued work may read the previous mesh: the handle's own, and a
  // batch's that holds the handle on another stream
  hipError_t err = hipDeviceSynchronize();
  if (err == hipSuccess && !h->metric) err = hipMalloc(&h->metric, sizeof(double) * met.size());
  if (err == hipSuccess)
    err = hipMemcpyAsync(h->metric, met.data(), sizeof(double) * met.size(), hipMemcpyHostToDevice, h->stream);
  if (err == hipSuccess) err = hipStreamSynchronize(h->stream);
  if (err != hipSuccess) return fail(h, IDP_DG_EHIP, std::string("idp_dg_set_mesh: ") + hipGetErrorString(err));
  idp_host::drop_graph(h);   // a captured step holds the Cartesian kernels
  ++h->mesh_version;         // a batch holding the handle re-plans its groups
  return 0;
}
