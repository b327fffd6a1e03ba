// Host runtime of the C ABI declared in include/idp_dg.h: argument checks,
// Gauss-Lobatto tables, launch configuration, device buffers, the cached
// HIP graph of a device-timestepped SSP-RK3 step, diagnostics and the
// batched driver.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/idp_dg.h"
#include "common.hpp"
#include "handle.hpp"

using namespace idp;

namespace {

thread_local std::string g_create_error = "no error";

// ---------------------------------------------------------------------
// tables: Gauss-Lobatto points as the roots of P_{p+1} - P_{p-1}, which
// vanishes at +-1 and at the roots of P_p' (Newton from Chebyshev-Lobatto
// guesses, derivative (2p+1) P_p); weights 2/(p(p+1) P_p^2) on [-1,1];
// the derivative matrix from barycentric weights with its diagonal set by
// the exact row sum (derivative of a constant).
// ---------------------------------------------------------------------
void legendre_pair(int n, double x, double* pn, double* pnm1) {
  double a = 1.0, b = x;  // P_0, P_1
  if (n == 0) { *pn = 1.0; *pnm1 = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    const double c = ((2 * k - 1) * x * b - (k - 1) * a) / k;
    a = b;
    b = c;
  }
  *pn = b;
  *pnm1 = a;
}

void gl_tables(int p, double* xi01, double* w01, double* D) {
  const int n = p + 1;
  double x[MAXP + 1];
  x[0] = -1.0;
  x[p] = 1.0;
  for (int k = 1; k < p; ++k) {
    double t = -std::cos(M_PI * k / p);
    for (int it = 0; it < 60; ++it) {
      double pp1, pp, pm1, dummy;
      legendre_pair(p + 1, t, &pp1, &pp);
      legendre_pair(p - 1, t, &pm1, &dummy);
      const double f = pp1 - pm1;
      const double df = (2.0 * p + 1.0) * pp;
      const double dx = f / df;
      t -= dx;
      if (std::fabs(dx) <= 1e-16) break;
    }
    x[k] = t;
  }
  double w[MAXP + 1], bw[MAXP + 1];
  for (int k = 0; k < n; ++k) {
    double pk, pkm1;
    legendre_pair(p, x[k], &pk, &pkm1);
    w[k] = 1.0 / (p * (p + 1.0) * pk * pk);  // on [0,1]
    xi01[k] = 0.5 * (x[k] + 1.0);
  }
  xi01[0] = 0.0;
  xi01[p] = 1.0;
  for (int j = 0; j < n; ++j) {
    double prod = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != j) prod *= xi01[j] - xi01[m];
    bw[j] = 1.0 / prod;
  }
  for (int i = 0; i < n; ++i) {
    double rs = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      const double dij = bw[j] / bw[i] / (xi01[i] - xi01[j]);
      D[i * n + j] = w[i] * dij;
      rs += dij;
    }
    D[i * n + i] = -w[i] * rs;
  }
  for (int k = 0; k < n; ++k) w01[k] = w[k];
}

}  // namespace

namespace idp_host {

void gl_derivative(int p, double* w01, double* Dn) {
  const int n = p + 1;
  double xi[MAXP + 1], D[(MAXP + 1) * (MAXP + 1)];
  gl_tables(p, xi, w01, D);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Dn[i * n + j] = D[i * n + j] / w01[i];
}

int fail(idp_dg* h, int code, const std::string& msg) {
  if (h) h->err = msg; else g_create_error = msg;
  return code;
}

int hip_fail(idp_dg* h, hipError_t e, const char* where) {
  return fail(h, IDP_DG_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Nodal -> Legendre modal map on the Gauss-Lobatto points: the points'
// quadrature is exact for P_j P_k with j + k <= 2p - 1, so the Legendre
// polynomials are orthogonal in the discrete inner product and
// c_k = sum_a w_a u_a P_k(x_a) / sum_a w_a P_k(x_a)^2 recovers the modal
// coefficients of the interpolating polynomial exactly (for k = p too, with
// the discrete norm in the denominator).  Also the L2 norms 2/(2k+1) on
// [-1,1] and the smoothness indicator centre log10(p^-4) (Sec. 4.4).
void modal_tables(int p, const double* xi01, const double* w01, Tables* T) {
  const int n = p + 1;
  for (int k = 0; k < n; ++k) {
    double g = 0.0;
    double pk[MAXP + 1];
    for (int a = 0; a < n; ++a) {
      double pn, pm;
      legendre_pair(k, 2.0 * xi01[a] - 1.0, &pn, &pm);
      pk[a] = pn;
      g += w01[a] * pn * pn;
    }
    for (int a = 0; a < n; ++a) T->M[k * n + a] = w01[a] * pk[a] / g;
    T->nk[k] = 2.0 / (2.0 * k + 1.0);
  }
  T->s0 = std::log10(std::pow((double)p, -4.0));
}

bool desc_ok(const idp_dg_desc* d, std::string* why) {
  if (!d) { *why = "desc is NULL"; return false; }
  if (d->dim != 1 && d->dim != 2) { *why = "dim must be 1 or 2"; return false; }
  if (d->nx < 1 || d->ny < 1) { *why = "nx, ny must be >= 1"; return false; }
  if (d->dim == 1 && d->ny != 1) { *why = "ny must be 1 when dim = 1"; return false; }
  if (!(d->lx > 0.0) || (d->dim == 2 && !(d->ly > 0.0))) { *why = "lx, ly must be > 0"; return false; }
  if (d->p < 1 || d->p > MAXP) { *why = "p must be in [1, 8]"; return false; }
  if (d->eq < IDP_DG_ADVECTION || d->eq > IDP_DG_ADVECTION_FIELD) { *why = "unknown equation"; return false; }
  if (d->limiter < IDP_DG_SUBCELL || d->limiter > IDP_DG_ELEMENTWISE) { *why = "unknown limiter"; return false; }
  if (d->limiter == IDP_DG_SUBCELL_SI && !(std::isfinite(d->gmin) && std::isfinite(d->gmax) && d->gmin <= d->gmax)) {
    *why = "gmin, gmax must be finite with gmin <= gmax";
    return false;
  }
  if (d->eq == IDP_DG_EULER && !(d->gamma > 1.0 && d->gamma <= 5.0 / 3.0)) {
    *why = "gamma must be in (1, 5/3]";
    return false;
  }
  const long long n1 = d->p + 1;
  const long long nn = (long long)d->nx * d->ny * (d->dim == 2 ? n1 * n1 : n1);
  if ((long long)d->nx * d->ny > 0x7fffffffLL || nn > (1LL << 40)) { *why = "mesh too large"; return false; }
  for (int k = 0; k < 2; ++k)
    if (d->bc[k] != IDP_DG_BC_PERIODIC && d->bc[k] != IDP_DG_BC_OPEN) { *why = "bc must be periodic or open"; return false; }
  if (d->dim == 1 && d->bc[1] != IDP_DG_BC_PERIODIC) { *why = "bc[1] must be periodic when dim = 1"; return false; }
  if (d->eq == IDP_DG_ADVECTION_FIELD) {
    if (d->dim != 2) { *why = "a velocity field needs dim = 2"; return false; }
    if (!d->vel_rows || !d->vel_cols) { *why = "vel_rows and vel_cols must be non-NULL"; return false; }
    for (long long i = 0; i < d->ny * n1; ++i)
      if (!std::isfinite(d->vel_rows[i])) { *why = "vel_rows must be finite"; return false; }
    for (long long i = 0; i < d->nx * n1; ++i)
      if (!std::isfinite(d->vel_cols[i])) { *why = "vel_cols must be finite"; return false; }
  }
  return true;
}

bool bnd_ready(const idp_dg* h) {
  for (int k = 0; k < 2; ++k)
    if (((h->bnd.open >> k) & 1) && (!h->bnd.type[2 * k] || !h->bnd.type[2 * k + 1])) return false;
  return true;
}

// kernel family: equation code (with the gamma specialisation) and dimension
int family(const idp_dg* h) { return h->kcode * 2 + (h->d.dim - 1); }

hipError_t launch_stage(const idp_dg* h, const StageArgs& a, hipStream_t s) {
  const int p = h->d.p;
  if (h->metric) {   // curved mesh: the first tile shape
    switch (family(h)) {
      case 1: return launch_stage_curved_adv2(p, a, s);
      case 3: return launch_stage_curved_burg2(p, a, s);
      case 5: return launch_stage_curved_euler2(p, a, s);
      case 7: return launch_stage_curved_euler53_2(p, a, s);
      case 9: return launch_stage_curved_euler75_2(p, a, s);
    }
    return hipErrorInvalidValue;
  }
  switch (family(h)) {
    case 0: return launch_stage_adv1(p, h->variant, a, s);
    case 1: return launch_stage_adv2(p, h->variant, a, s);
    case 2: return launch_stage_burg1(p, h->variant, a, s);
    case 3: return launch_stage_burg2(p, h->variant, a, s);
    case 4: return launch_stage_euler1(p, h->variant, a, s);
    case 5: return launch_stage_euler2(p, h->variant, a, s);
    case 6: return launch_stage_euler53_1(p, h->variant, a, s);
    case 7: return launch_stage_euler53_2(p, h->variant, a, s);
    case 8: return launch_stage_euler75_1(p, h->variant, a, s);
    case 9: return launch_stage_euler75_2(p, h->variant, a, s);
    case 11: return launch_stage_advv2(p, h->variant, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_maxdt(const idp_dg* h, const MaxDtArgs& a, hipStream_t s) {
  const int p = h->d.p;
  if (h->metric) {
    switch (family(h)) {
      case 1: return launch_maxdt_curved_adv2(p, a, s);
      case 3: return launch_maxdt_curved_burg2(p, a, s);
      case 5: return launch_maxdt_curved_euler2(p, a, s);
      case 7: return launch_maxdt_curved_euler53_2(p, a, s);
      case 9: return launch_maxdt_curved_euler75_2(p, a, s);
    }
    return hipErrorInvalidValue;
  }
  switch (family(h)) {
    case 0: return launch_maxdt_adv1(p, h->variant, a, s);
    case 1: return launch_maxdt_adv2(p, h->variant, a, s);
    case 2: return launch_maxdt_burg1(p, h->variant, a, s);
    case 3: return launch_maxdt_burg2(p, h->variant, a, s);
    case 4: return launch_maxdt_euler1(p, h->variant, a, s);
    case 5: return launch_maxdt_euler2(p, h->variant, a, s);
    case 6: return launch_maxdt_euler53_1(p, h->variant, a, s);
    case 7: return launch_maxdt_euler53_2(p, h->variant, a, s);
    case 8: return launch_maxdt_euler75_1(p, h->variant, a, s);
    case 9: return launch_maxdt_euler75_2(p, h->variant, a, s);
    case 11: return launch_maxdt_advv2(p, h->variant, a, s);
  }
  return hipErrorInvalidValue;
}

void tile_dims(const idp_dg* h, int* tx, int* ty) {
  const int p = h->d.p;
  const int v = h->metric ? 0 : h->variant;   // curved meshes: the first shape only
  *tx = *ty = 1;
  switch (family(h)) {
    case 0: return tile_dims_adv1(p, v, tx, ty);
    case 1: return tile_dims_adv2(p, v, tx, ty);
    case 2: return tile_dims_burg1(p, v, tx, ty);
    case 3: return tile_dims_burg2(p, v, tx, ty);
    case 4: return tile_dims_euler1(p, v, tx, ty);
    case 5: return tile_dims_euler2(p, v, tx, ty);
    case 6: return tile_dims_euler53_1(p, v, tx, ty);
    case 7: return tile_dims_euler53_2(p, v, tx, ty);
    case 8: return tile_dims_euler75_1(p, v, tx, ty);
    case 9: return tile_dims_euler75_2(p, v, tx, ty);
    case 11: return tile_dims_advv2(p, v, tx, ty);
  }
}

int tile_elems(const idp_dg* h) {
  int tx, ty;
  tile_dims(h, &tx, &ty);
  return tx * ty;
}

// tiles of the handle's mesh, and tiles per row of tiles
int tiles_of(const idp_dg* h, int* ntx) {
  int tx, ty;
  tile_dims(h, &tx, &ty);
  *ntx = (h->d.nx + tx - 1) / tx;
  return *ntx * ((h->d.ny + ty - 1) / ty);
}

StageArgs make_stage_args(const idp_dg* h, const double* u_n, const double* u_s, double* u_out,
                          double dt, const double* dt_dev, double dt_scale, int stage) {
  static const double As[3] = {0.0, 0.75, 1.0 / 3.0};
  static const double Bs[3] = {1.0, 0.25, 2.0 / 3.0};
  StageArgs a;
  std::memset(&a, 0, sizeof(a));
  a.S.u_n = u_n;
  a.S.u_s = u_s;
  a.S.u_out = u_out;
  a.S.dt_dev = dt_dev;
  a.S.dt = dt;
  a.S.dt_scale = dt_scale;
  a.S.nn = h->nn;
  a.S.p = h->d.p;
  a.S.nx = h->d.nx;
  a.S.ny = h->d.ny;
  a.S.ne = h->ne;
  a.S.ntiles = tiles_of(h, &a.S.ntx);
  a.S.hx = h->d.lx / h->d.nx;
  a.S.hy = h->d.dim == 2 ? h->d.ly / h->d.ny : 1.0;
  a.S.ihx = 1.0 / a.S.hx;
  a.S.ihy = 1.0 / a.S.hy;
  a.ph = h->ph;
  a.T = h->T;
  a.a_s = As[stage];
  a.b_s = Bs[stage];
  a.use_un = stage > 0;
  a.limiter = h->d.limiter;
  a.diag = h->diag;
  a.gmin = h->d.gmin;
  a.gmax = h->d.gmax;
  a.bnd = h->bnd;
  a.S.metric = h->metric;
  return a;
}

MaxDtArgs make_dt_args(const idp_dg* h, const double* u) {
  MaxDtArgs a;
  std::memset(&a, 0, sizeof(a));
  a.u = u;
  a.partial = h->partial;
  a.nn = h->nn;
  a.p = h->d.p;
  a.nx = h->d.nx;
  a.ny = h->d.ny;
  a.ne = h->ne;
  a.ntiles = tiles_of(h, &a.ntx);
  a.hx = h->d.lx / h->d.nx;
  a.hy = h->d.dim == 2 ? h->d.ly / h->d.ny : 1.0;
  a.ph = h->ph;
  a.T = h->T;
  a.bnd = h->bnd;
  a.metric = h->metric;
  return a;
}

void retire_graph(std::vector<RetiredGraph>* list, hipGraph_t* g, hipGraphExec_t* e, hipEvent_t* ev) {
  if (*e || *g) list->push_back(RetiredGraph{*g, *e, *ev});
  else if (*ev) (void)hipEventDestroy(*ev);
  *g = nullptr;
  *e = nullptr;
  *ev = nullptr;
  reap_graphs(list, false);
}

void reap_graphs(std::vector<RetiredGraph>* list, bool wait) {
  size_t keep = 0;
  for (size_t i = 0; i < list->size(); ++i) {
    RetiredGraph& r = (*list)[i];
    if (r.done) {
      if (wait) (void)hipEventSynchronize(r.done);
      else if (hipEventQuery(r.done) == hipErrorNotReady) {
        (*list)[keep++] = r;
        continue;
      }
    }
    if (r.exec) (void)hipGraphExecDestroy(r.exec);
    if (r.graph) (void)hipGraphDestroy(r.graph);
    if (r.done) (void)hipEventDestroy(r.done);
  }
  list->resize(keep);
}

int batch_kernels(int fam, int p, int variant, BatchKernels* k) {
  switch (fam) {
    case 0: return batch_kernels_adv1(p, variant, k);
    case 1: return batch_kernels_adv2(p, variant, k);
    case 2: return batch_kernels_burg1(p, variant, k);
    case 3: return batch_kernels_burg2(p, variant, k);
    case 4: return batch_kernels_euler1(p, variant, k);
    case 5: return batch_kernels_euler2(p, variant, k);
    case 6: return batch_kernels_euler53_1(p, variant, k);
    case 7: return batch_kernels_euler53_2(p, variant, k);
    case 8: return batch_kernels_euler75_1(p, variant, k);
    case 9: return batch_kernels_euler75_2(p, variant, k);
    case 11: return batch_kernels_advv2(p, variant, k);
  }
  return -1;
}

int batch_kernels_curved(int fam, int p, BatchKernels* k) {
  switch (fam) {
    case 1: return batch_kernels_curved_adv2(p, k);
    case 3: return batch_kernels_curved_burg2(p, k);
    case 5: return batch_kernels_curved_euler2(p, k);
    case 7: return batch_kernels_curved_euler53_2(p, k);
    case 9: return batch_kernels_curved_euler75_2(p, k);
  }
  return -1;
}

void drop_graph(idp_dg* h) {
  retire_graph(&h->retired, &h->graph, &h->exec, &h->g_done);
  h->g_u = nullptr;
}

}  // namespace idp_host

using namespace idp_host;

namespace {

bool overlaps(const double* a, const double* b, long long n) {
  return a < b + n && b < a + n;
}

}  // namespace
namespace idp {
// per workgroup b of the grid: min over its contiguous chunk of
// partial[0..n) -> out[b] (1024 threads)
__global__ void chunk_min_kernel(const double* partial, int n, double* out);
}  // namespace idp
namespace {

// Minima per workgroup that one 1024-thread workgroup folds (256 KB, a few
// microseconds); past that a first launch of kChunks workgroups folds
// contiguous chunks into the kChunks slots that follow the minima (the
// array holds ne + 64 >= tiles + 64 doubles), and one workgroup folds
// those.  The minimum does not depend on the grouping.
constexpr int kOneGroupMinima = 32768, kChunks = 64;

// the low-order CFL bound of u into out[0] (device), two or three launches
hipError_t enqueue_max_dt(const idp_dg* h, const double* u, double* out, hipStream_t s) {
  hipError_t e = launch_maxdt(h, make_dt_args(h, u), s);
  if (e != hipSuccess) return e;
  int ntx;
  const int nb = tiles_of(h, &ntx);
  if (nb <= kOneGroupMinima) {
    hipLaunchKernelGGL(min_reduce_kernel, dim3(1), dim3(1024), 0, s, h->partial, nb, out);
  } else {
    hipLaunchKernelGGL(chunk_min_kernel, dim3(kChunks), dim3(1024), 0, s, h->partial, nb, h->partial + nb);
    hipLaunchKernelGGL(min_reduce_kernel, dim3(1), dim3(1024), 0, s, h->partial + nb, kChunks, out);
  }
  return hipGetLastError();
}

// enqueue one device-timestepped step on stream s
hipError_t enqueue_step_cfl(idp_dg* h, double* u, double cfl, hipStream_t s) {
  hipError_t e = enqueue_max_dt(h, u, h->dtdev, s);
  if (e != hipSuccess) return e;
  const double* dtp = h->dtdev;
  e = launch_stage(h, make_stage_args(h, nullptr, u, h->buf1, 0.0, dtp, cfl, 0), s);
  if (e != hipSuccess) return e;
  e = launch_stage(h, make_stage_args(h, u, h->buf1, h->buf2, 0.0, dtp, cfl, 1), s);
  if (e != hipSuccess) return e;
  return launch_stage(h, make_stage_args(h, u, h->buf2, u, 0.0, dtp, cfl, 2), s);
}

}  // namespace

namespace idp {
__global__ __launch_bounds__(256) void segmented_min_kernel(const double* partial, const int* range,
                                                             double* out) {
  __shared__ double red[4];
  const int s = blockIdx.x;
  double v = wave_min63(strided_min<256>(partial, range[2 * s], range[2 * s + 1]));
  if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) out[s] = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

__global__ __launch_bounds__(1024) void chunk_min_kernel(const double* partial, int n, double* out) {
  __shared__ double red[16];
  const int chunk = (n + gridDim.x - 1) / gridDim.x;
  const int b = (int)blockIdx.x * chunk, e = min(n, b + chunk);
  double v = wave_min63(strided_min<1024>(partial, b, e));
  if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    v = red[0];
    for (int i = 1; i < 16; ++i) v = fmin(v, red[i]);
    out[blockIdx.x] = v;
  }
}

__global__ __launch_bounds__(1024) void min_reduce_kernel(const double* partial, int n, double* out) {
  __shared__ double red[16];
  double v = wave_min63(strided_min<1024>(partial, 0, n));
  if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    v = red[0];
    for (int i = 1; i < 16; ++i) v = fmin(v, red[i]);
    out[0] = v;
  }
}
}  // namespace idp

extern "C" {

namespace {
constexpr long long kWsAlign = 256;
long long ws_up(long long x) { return (x + kWsAlign - 1) / kWsAlign * kWsAlign; }

// Offsets of the handle's device buffers in one workspace.
struct WsLayout {
  long long buf1, buf2, diag, dtdev, partial, vel, total;
};

WsLayout ws_layout(const idp_dg_desc* d) {
  const long long n1 = d->p + 1;
  const long long ne = (long long)d->nx * d->ny;
  const long long nn = ne * (d->dim == 2 ? n1 * n1 : n1);
  const long long nc = d->eq == IDP_DG_EULER ? d->dim + 2 : 1;
  WsLayout L;
  L.buf1 = 0;
  L.buf2 = ws_up(L.buf1 + 8 * nc * nn);
  L.diag = ws_up(L.buf2 + 8 * nc * nn);
  L.dtdev = ws_up(L.diag + (long long)sizeof(Diag));
  L.partial = ws_up(L.dtdev + 64);
  L.vel = ws_up(L.partial + 8 * (ne + 64));
  L.total = ws_up(L.vel + (d->eq == IDP_DG_ADVECTION_FIELD ? 8 * n1 * (d->nx + d->ny) : 0));
  return L;
}

int create_impl(const idp_dg_desc* desc, void* hip_stream, char* ws, long long ws_bytes, idp_dg** out);
}  // namespace

int idp_dg_create(const idp_dg_desc* desc, void* hip_stream, idp_dg** out) {
  const idp_host::Range trace_range("idp_dg_create");
  return create_impl(desc, hip_stream, nullptr, 0, out);
}

long long idp_dg_workspace_bytes(const idp_dg_desc* desc) {
  std::string why;
  if (!desc_ok(desc, &why)) return fail(nullptr, IDP_DG_EINVAL, why);
  return ws_layout(desc).total;
}

int idp_dg_create_in(const idp_dg_desc* desc, void* hip_stream, void* workspace, long long bytes,
                     idp_dg** out) {
  const idp_host::Range trace_range("idp_dg_create_in");
  if (!out) return fail(nullptr, IDP_DG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kWsAlign)
    return fail(nullptr, IDP_DG_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  std::string why;
  if (!desc_ok(desc, &why)) return fail(nullptr, IDP_DG_EINVAL, why);
  if (bytes < ws_layout(desc).total) return fail(nullptr, IDP_DG_EINVAL, "workspace too small");
  return create_impl(desc, hip_stream, static_cast<char*>(workspace), bytes, out);
}

namespace {
// Copy a velocity field's row and column samples to h->vel on the handle's
// stream and wait for the copy (the caller's arrays are only borrowed for
// the create call); point the physics constants at them.
hipError_t upload_field(idp_dg* h, const idp_dg_desc* desc) {
  h->d.vel_rows = nullptr;
  h->d.vel_cols = nullptr;
  if (desc->eq != IDP_DG_ADVECTION_FIELD) return hipSuccess;
  const size_t nr = (size_t)desc->ny * (desc->p + 1), ncol = (size_t)desc->nx * (desc->p + 1);
  hipError_t e = hipMemcpyAsync(h->vel, desc->vel_rows, sizeof(double) * nr, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->vel + nr, desc->vel_cols, sizeof(double) * ncol, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  h->ph.vrow = h->vel;
  h->ph.vcol = h->vel + nr;
  return e;
}

}  // namespace

extern "C++" {
namespace idp_host {
// Host-side set-up of a handle from a checked descriptor: sizes, tables,
// physics constants and the kernel family (no device calls, no allocation).
void init_host(idp_dg* h, const idp_dg_desc* desc, void* hip_stream) {
  h->d = *desc;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  h->nc = desc->eq == IDP_DG_EULER ? desc->dim + 2 : 1;
  h->ne = desc->nx * desc->ny;
  const long long n1 = desc->p + 1;
  h->nn = (long long)h->ne * (desc->dim == 2 ? n1 * n1 : n1);
  double xi[MAXP + 1], D[(MAXP + 1) * (MAXP + 1)];
  gl_tables(desc->p, xi, h->T.w, D);
  for (int a = 0; a < desc->p; ++a) {
    for (int e = 0; e <= desc->p; ++e) {
      double acc = 0.0;
      for (int c = 0; c <= a; ++c) acc += D[c * (desc->p + 1) + e];
      h->T.Q[a * (desc->p + 1) + e] = acc;
    }
  }
  h->ph.vel0 = desc->velocity[0];
  h->ph.vel1 = desc->dim == 2 ? desc->velocity[1] : 0.0;
  h->ph.gamma = desc->eq == IDP_DG_EULER ? desc->gamma : 1.4;
  h->ph.g1 = 0.5 * (h->ph.gamma - 1.0);
  h->ph.igm1 = 1.0 / (h->ph.gamma - 1.0);
  h->ph.fac = (h->ph.gamma + 1.0) / (2.0 * h->ph.gamma);
  h->ph.ex = (h->ph.gamma - 1.0) / (2.0 * h->ph.gamma);
  h->ph.inv_ex = 1.0 / h->ph.ex;
  const double r = std::nearbyint(h->ph.inv_ex);
  h->ph.inv_ex_int = (std::fabs(h->ph.inv_ex - r) < 1e-12 && r > 0 && r < 64) ? (int)r : 0;
  h->kcode = desc->eq == IDP_DG_ADVECTION_FIELD ? EQ_ADVV : desc->eq;
  h->bnd.open = (desc->bc[0] == IDP_DG_BC_OPEN ? 1 : 0) | (desc->bc[1] == IDP_DG_BC_OPEN ? 2 : 0);
  if (desc->eq == IDP_DG_EULER) {
    const double gn = std::nearbyint(2.0 / (h->ph.gamma - 1.0));
    const bool exact = std::fabs(h->ph.gamma - (1.0 + 2.0 / gn)) <= 4e-16 * h->ph.gamma;
    if (exact && gn == 5.0) h->kcode = EQ_EULER75;
    if (exact && gn == 3.0) h->kcode = EQ_EULER53;
  }
  for (int k = 0; k <= desc->p; ++k) h->T.iw[k] = 1.0 / h->T.w[k];
  modal_tables(desc->p, xi, h->T.w, &h->T);
}
}  // namespace idp_host
}  // extern "C++"

namespace {
int create_impl(const idp_dg_desc* desc, void* hip_stream, char* ws, long long ws_bytes, idp_dg** out) {
  (void)ws_bytes;
  if (!out) return fail(nullptr, IDP_DG_EINVAL, "out is NULL");
  *out = nullptr;
  std::string why;
  if (!desc_ok(desc, &why)) return fail(nullptr, IDP_DG_EINVAL, why);
  idp_dg* h = new (std::nothrow) idp_dg;
  if (!h) return fail(nullptr, IDP_DG_ENOMEM, "host allocation failed");
  init_host(h, desc, hip_stream);
  const long long n1 = desc->p + 1;
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) { int rc = hip_fail(nullptr, e, "hipGetDevice"); delete h; return rc; }
  if (ws) {  // caller workspace: no allocation, diagnostics cleared on the stream
    const WsLayout L = ws_layout(desc);
    h->owns = false;
    h->buf1 = reinterpret_cast<double*>(ws + L.buf1);
    h->buf2 = reinterpret_cast<double*>(ws + L.buf2);
    h->diag = reinterpret_cast<Diag*>(ws + L.diag);
    h->dtdev = reinterpret_cast<double*>(ws + L.dtdev);
    h->partial = reinterpret_cast<double*>(ws + L.partial);
    if (desc->eq == IDP_DG_ADVECTION_FIELD) h->vel = reinterpret_cast<double*>(ws + L.vel);
    e = hipMemsetAsync(h->diag, 0, sizeof(Diag), h->stream);
    if (e == hipSuccess) e = upload_field(h, desc);
    if (e != hipSuccess) {
      fail(nullptr, IDP_DG_EHIP, std::string("workspace set-up: ") + hipGetErrorString(e));
      delete h;
      return IDP_DG_EHIP;
    }
    *out = h;
    return 0;
  }
  const size_t bytes = sizeof(double) * h->nc * h->nn;
  e = hipMalloc(&h->buf1, bytes);
  if (e == hipSuccess) e = hipMalloc(&h->buf2, bytes);
  if (e == hipSuccess) e = hipMalloc(&h->diag, sizeof(Diag) + 64);
  if (e == hipSuccess) e = hipMalloc(&h->dtdev, 64);
  if (e == hipSuccess) e = hipMalloc(&h->partial, sizeof(double) * ((size_t)h->ne + 64));
  if (e == hipSuccess && desc->eq == IDP_DG_ADVECTION_FIELD)
    e = hipMalloc(&h->vel, sizeof(double) * n1 * (desc->nx + desc->ny));
  if (e == hipSuccess) e = hipMemset(h->diag, 0, sizeof(Diag));
  if (e == hipSuccess) e = upload_field(h, desc);
  if (e != hipSuccess) {
    const int code = e == hipErrorOutOfMemory ? IDP_DG_ENOMEM : IDP_DG_EHIP;
    fail(nullptr, code, std::string("device allocation: ") + hipGetErrorString(e));
    hipFree(h->buf1); hipFree(h->buf2); hipFree(h->diag); hipFree(h->dtdev); hipFree(h->partial);
    hipFree(h->vel);
    delete h;
    return code;
  }
  *out = h;
  return 0;
}
}  // namespace

void idp_dg_destroy(idp_dg* h) {
  if (!h) return;
  drop_graph(h);
  reap_graphs(&h->retired, true);
  if (h->cap) hipStreamDestroy(h->cap);
  hipFree(h->metric);   // allocated by idp_dg_set_mesh
  if (h->owns) {
    hipFree(h->buf1);
    hipFree(h->buf2);
    hipFree(h->diag);
    hipFree(h->dtdev);
    hipFree(h->partial);
    hipFree(h->vel);
  }
  delete h;
}

long idp_dg_num_nodes(const idp_dg* h) { return h ? (long)h->nn : -1; }
int idp_dg_num_comp(const idp_dg* h) { return h ? h->nc : -1; }

int idp_dg_stage(idp_dg* h, const double* u_n, const double* u_s, double* u_out, double dt,
                 int stage) {
  const idp_host::Range trace_range("idp_dg_stage");
  if (!h) return IDP_DG_EINVAL;
  if (!bnd_ready(h)) return fail(h, IDP_DG_EINVAL, "an open side has no boundary conditions (idp_dg_set_boundary)");
  if (stage < 0 || stage > 2) return fail(h, IDP_DG_EINVAL, "stage must be 0, 1 or 2");
  if (!u_s || !u_out || (stage > 0 && !u_n)) return fail(h, IDP_DG_EINVAL, "NULL state pointer");
  if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(h, IDP_DG_EINVAL, "dt must be finite and >= 0");
  const long long n = (long long)h->nc * h->nn;
  if (overlaps(u_out, u_s, n)) return fail(h, IDP_DG_EINVAL, "u_out overlaps u_s");
  if (stage > 0 && u_n != u_out && overlaps(u_out, u_n, n))
    return fail(h, IDP_DG_EINVAL, "u_out partially overlaps u_n");
  hipError_t e = launch_stage(h, make_stage_args(h, u_n, u_s, u_out, dt, nullptr, 1.0, stage), h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "stage launch");
  return 0;
}

int idp_dg_stage_trace(idp_dg* h, const double* u_n, const double* u_s, double* u_out,
                       double dt, int stage, double* trace) {
  const idp_host::Range trace_range("idp_dg_stage_trace");
  if (!h) return IDP_DG_EINVAL;
  if (!bnd_ready(h)) return fail(h, IDP_DG_EINVAL, "an open side has no boundary conditions (idp_dg_set_boundary)");
  if (!trace) return fail(h, IDP_DG_EINVAL, "NULL trace pointer");
  if (stage < 0 || stage > 2) return fail(h, IDP_DG_EINVAL, "stage must be 0, 1 or 2");
  if (!u_s || !u_out || (stage > 0 && !u_n)) return fail(h, IDP_DG_EINVAL, "NULL state pointer");
  if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(h, IDP_DG_EINVAL, "dt must be finite and >= 0");
  const long long n = (long long)h->nc * h->nn;
  if (overlaps(u_out, u_s, n)) return fail(h, IDP_DG_EINVAL, "u_out overlaps u_s");
  if (overlaps(trace, u_out, n) || overlaps(trace, u_s, n) || (u_n && overlaps(trace, u_n, n)))
    return fail(h, IDP_DG_EINVAL, "trace overlaps a state");
  StageArgs a = make_stage_args(h, u_n, u_s, u_out, dt, nullptr, 1.0, stage);
  a.trace = trace;
  hipError_t e = launch_stage(h, a, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "stage launch");
  return 0;
}

int idp_dg_step(idp_dg* h, double* u, double dt) {
  const idp_host::Range trace_range("idp_dg_step");
  if (!h) return IDP_DG_EINVAL;
  if (!u) return fail(h, IDP_DG_EINVAL, "NULL state pointer");
  const long long n = (long long)h->nc * h->nn;
  if (overlaps(u, h->buf1, n) || overlaps(u, h->buf2, n))
    return fail(h, IDP_DG_EINVAL, "u overlaps the handle's buffers");
  int rc = idp_dg_stage(h, nullptr, u, h->buf1, dt, 0);
  if (!rc) rc = idp_dg_stage(h, u, h->buf1, h->buf2, dt, 1);
  if (!rc) rc = idp_dg_stage(h, u, h->buf2, u, dt, 2);
  return rc;
}

int idp_dg_step_cfl(idp_dg* h, double* u, double cfl) {
  const idp_host::Range trace_range("idp_dg_step_cfl");
  if (!h) return IDP_DG_EINVAL;
  if (!bnd_ready(h)) return fail(h, IDP_DG_EINVAL, "an open side has no boundary conditions (idp_dg_set_boundary)");
  if (!u) return fail(h, IDP_DG_EINVAL, "NULL state pointer");
  if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(h, IDP_DG_EINVAL, "cfl must be finite and > 0");
  const long long n = (long long)h->nc * h->nn;
  if (overlaps(u, h->buf1, n) || overlaps(u, h->buf2, n))
    return fail(h, IDP_DG_EINVAL, "u overlaps the handle's buffers");
  hipError_t e;
  if (!h->exec || h->g_u != u || h->g_cfl != cfl) {
    drop_graph(h);
    if (!h->cap) {
      e = hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_fail(h, e, "hipStreamCreate");
    }
    e = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamBeginCapture");
    hipError_t le = enqueue_step_cfl(h, u, cfl, h->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(h->cap, &g);
    if (le != hipSuccess) { if (g) hipGraphDestroy(g); return hip_fail(h, le, "step capture"); }
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamEndCapture");
    h->graph = g;
    e = hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) { drop_graph(h); return hip_fail(h, e, "hipGraphInstantiate"); }
    h->g_u = u;
    h->g_cfl = cfl;
    e = hipEventCreateWithFlags(&h->g_done, hipEventDisableTiming);
    if (e != hipSuccess) { drop_graph(h); return hip_fail(h, e, "hipEventCreate"); }
  }
  e = hipGraphLaunch(h->exec, h->stream);
  if (e == hipSuccess) e = hipEventRecord(h->g_done, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "hipGraphLaunch");
  return 0;
}

int idp_dg_last_dt(idp_dg* h, double* dt) {
  if (!h || !dt) return IDP_DG_EINVAL;
  double v = 0.0;
  hipError_t e = hipMemcpyAsync(&v, h->dtdev, sizeof(v), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "last dt copy");
  if (!(v < INFINITY)) v = INFINITY;
  *dt = h->g_cfl * v;  // the same product the stage kernels form
  if (!(*dt < INFINITY)) *dt = 0.0;  // no dissipation anywhere: the step kept the state
  return 0;
}

int idp_dg_max_dt(idp_dg* h, const double* u, double* dt) {
  const idp_host::Range trace_range("idp_dg_max_dt");
  if (!h) return IDP_DG_EINVAL;
  if (!bnd_ready(h)) return fail(h, IDP_DG_EINVAL, "an open side has no boundary conditions (idp_dg_set_boundary)");
  if (!u || !dt) return fail(h, IDP_DG_EINVAL, "NULL pointer");
  double* slot = h->dtdev + 1;   // keep the step's dt slot intact
  hipError_t e = enqueue_max_dt(h, u, slot, h->stream);
  double v = 0.0;
  if (e == hipSuccess) e = hipMemcpyAsync(&v, slot, sizeof(v), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "max_dt");
  *dt = v;
  return 0;
}

int idp_dg_max_dt_async(idp_dg* h, const double* u, double* dt_dev) {
  const idp_host::Range trace_range("idp_dg_max_dt_async");
  if (!h) return IDP_DG_EINVAL;
  if (!bnd_ready(h)) return fail(h, IDP_DG_EINVAL, "an open side has no boundary conditions (idp_dg_set_boundary)");
  if (!u || !dt_dev) return fail(h, IDP_DG_EINVAL, "NULL pointer");
  if (reinterpret_cast<uintptr_t>(dt_dev) % 8) return fail(h, IDP_DG_EINVAL, "dt_dev not 8-byte aligned");
  hipError_t e = enqueue_max_dt(h, u, dt_dev, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "max_dt_async");
  return 0;
}

int idp_dg_stage_dt(idp_dg* h, const double* u_n, const double* u_s, double* u_out,
                    const double* dt_dev, double cfl, int stage) {
  const idp_host::Range trace_range("idp_dg_stage_dt");
  if (!h) return IDP_DG_EINVAL;
  if (!bnd_ready(h)) return fail(h, IDP_DG_EINVAL, "an open side has no boundary conditions (idp_dg_set_boundary)");
  if (stage < 0 || stage > 2) return fail(h, IDP_DG_EINVAL, "stage must be 0, 1 or 2");
  if (!u_s || !u_out || !dt_dev || (stage > 0 && !u_n)) return fail(h, IDP_DG_EINVAL, "NULL pointer");
  if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(h, IDP_DG_EINVAL, "cfl must be finite and > 0");
  const long long n = (long long)h->nc * h->nn;
  if (overlaps(u_out, u_s, n)) return fail(h, IDP_DG_EINVAL, "u_out overlaps u_s");
  if (stage > 0 && u_n != u_out && overlaps(u_out, u_n, n))
    return fail(h, IDP_DG_EINVAL, "u_out partially overlaps u_n");
  hipError_t e = launch_stage(h, make_stage_args(h, u_n, u_s, u_out, 0.0, dt_dev, cfl, stage), h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "stage launch");
  return 0;
}

static_assert(kNumVariants == IDP_DG_NUM_TILE_SHAPES, "tile shapes compiled per degree");

int idp_dg_tile_shape(const idp_dg* h) { return h ? h->variant : -1; }

int idp_dg_tile_elems(const idp_dg* h) { return h ? tile_elems(h) : -1; }

int idp_dg_tile_dims(const idp_dg* h, int* tx, int* ty) {
  if (!h || !tx || !ty) return IDP_DG_EINVAL;
  tile_dims(h, tx, ty);
  return 0;
}

int idp_dg_set_tile_shape(idp_dg* h, int shape) {
  if (!h) return IDP_DG_EINVAL;
  if (shape < 0 || shape >= kNumVariants) return fail(h, IDP_DG_EINVAL, "tile shape out of range");
  if (shape != h->variant) {
    h->variant = shape;
    drop_graph(h);   // the cached step holds the other shape's kernels
  }
  return 0;
}

int idp_dg_tune(idp_dg* h, const double* u, double cfl, int reps, int* shape) {
  const idp_host::Range trace_range("idp_dg_tune");
  if (!h) return IDP_DG_EINVAL;
  if (!bnd_ready(h)) return fail(h, IDP_DG_EINVAL, "an open side has no boundary conditions (idp_dg_set_boundary)");
  if (!u) return fail(h, IDP_DG_EINVAL, "NULL state pointer");
  if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(h, IDP_DG_EINVAL, "cfl must be finite and > 0");
  if (reps < 1 || reps > 100) return fail(h, IDP_DG_EINVAL, "reps must be in 1..100");
  const long long n = (long long)h->nc * h->nn;
  if (overlaps(u, h->buf1, n) || overlaps(u, h->buf2, n))
    return fail(h, IDP_DG_EINVAL, "u overlaps the handle's buffers");
  if (h->metric) {   // curved meshes run one tile shape: nothing to choose
    if (shape) *shape = h->variant;
    return 0;
  }
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  const int keep = h->variant;
  double* dtp = h->dtdev + 1;   // the spare slot: idp_dg_last_dt reads dtdev[0]
  float best_ms = 0.0f;
  int best = keep;
  // one step of u into the handle's buffers: u -> buf1 -> buf2 -> buf1
  auto step = [&]() -> hipError_t {
    hipError_t r = enqueue_max_dt(h, u, dtp, h->stream);
    if (r == hipSuccess) r = launch_stage(h, make_stage_args(h, nullptr, u, h->buf1, 0.0, dtp, cfl, 0), h->stream);
    if (r == hipSuccess) r = launch_stage(h, make_stage_args(h, u, h->buf1, h->buf2, 0.0, dtp, cfl, 1), h->stream);
    if (r == hipSuccess) r = launch_stage(h, make_stage_args(h, u, h->buf2, h->buf1, 0.0, dtp, cfl, 2), h->stream);
    return r;
  };
  // the shapes take turns, twice, so that drifts of the clock or of the
  // machine's load affect them alike; a shape replaces the current one only
  // if it is at least 2 % faster
  float total[kNumVariants] = {};
  for (int v = 0; v < kNumVariants && e == hipSuccess; ++v) {
    h->variant = v;
    e = step();   // warm-up (first launch of this shape's kernels)
  }
  for (int round = 0; round < 2 && e == hipSuccess; ++round) {
    for (int v = 0; v < kNumVariants && e == hipSuccess; ++v) {
      h->variant = v;
      e = hipEventRecord(ev[0], h->stream);
      for (int r = 0; r < reps && e == hipSuccess; ++r) e = step();
      if (e == hipSuccess) e = hipEventRecord(ev[1], h->stream);
      if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
      total[v] += ms;
    }
  }
  if (ev[0]) hipEventDestroy(ev[0]);
  if (ev[1]) hipEventDestroy(ev[1]);
  h->variant = keep;
  if (e != hipSuccess) return hip_fail(h, e, "tune");
  best_ms = total[keep];
  for (int v = 0; v < kNumVariants; ++v)
    if (total[v] < 0.98f * best_ms) {
      best_ms = total[v];
      best = v;
    }
  if (best != keep) {
    h->variant = best;
    drop_graph(h);
  }
  if (shape) *shape = best;
  return 0;
}

int idp_dg_set_boundary(idp_dg* h, int side, const signed char* type, const double* state) {
  if (!h) return IDP_DG_EINVAL;
  if (side < 0 || side >= 2 * h->d.dim) return fail(h, IDP_DG_EINVAL, "side must be in [0, 2 dim)");
  if (!((h->bnd.open >> (side >> 1)) & 1)) return fail(h, IDP_DG_EINVAL, "the side's direction is periodic");
  if (!type) return fail(h, IDP_DG_EINVAL, "type is NULL");
  h->bnd.type[side] = type;
  h->bnd.state[side] = state;
  ++h->bnd_version;
  drop_graph(h);   // a captured step holds the previous pointers
  return 0;
}

int idp_dg_diagnostics(idp_dg* h, idp_dg_diag* out) {
  if (!h || !out) return IDP_DG_EINVAL;
  std::vector<unsigned char> buf(sizeof(Diag));
  Diag* d = reinterpret_cast<Diag*>(buf.data());
  hipError_t e = hipMemcpyAsync(d, h->diag, sizeof(Diag), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->diag, 0, sizeof(Diag), h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "diagnostics");
  long long nl = 0, ne = 0;
  for (int i = 0; i < DIAG_SLOTS; ++i) {
    nl += (long long)d->limited[i];
    ne += (long long)d->entropy[i];
  }
  out->limited_nodes = nl;
  out->entropy_nodes = ne;
  out->bad_input = d->bad_input ? 1 : 0;
  out->low_order_violation = d->lo_violation ? 1 : 0;
  return 0;
}

const char* idp_dg_last_error(const idp_dg* h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

#ifndef IDP_DG_SOURCE_HASH
#define IDP_DG_SOURCE_HASH "unknown"
#endif
const char* idp_dg_build_hash(void) { return IDP_DG_SOURCE_HASH; }

}  // extern "C"
