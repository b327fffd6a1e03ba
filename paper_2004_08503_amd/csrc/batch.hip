// Batched execution: many independent solves of one equation family (any
// mix of mesh sizes and degrees) advance together.  Every RK stage is one
// persistent launch over a work list of (solve, tile) items; the work list
// is cut into eight contiguous chunks, one per XCD, so that each XCD sweeps
// the tiles of a few solves in order and their face traces stay in its L2.
// The time-step bounds of all solves come from one persistent launch plus a
// segmented minimum.  A device-timestepped batched step is captured once in
// a HIP graph per (pointer set, cfl) and replayed.
//
// Results are bitwise identical to the plain path: a tile's arithmetic does
// not depend on how many elements share its workgroup, and the only
// reductions (alpha over faces, dt over nodes) are minima.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/idp_dg.h"
#include "common.hpp"
#include "handle.hpp"

using namespace idp;
using namespace idp_host;

namespace {
constexpr int kRing = 32;  // pinned staging slots for host time steps
}

struct idp_dg_batch {
  std::vector<idp_dg*> s;
  hipStream_t stream = nullptr;
  int fam = 0;
  int n = 0;
  int nitems = 0;
  int grid = 8;
  int lds = 0;   // dynamic LDS bytes of the persistent kernels
  int chunk[9] = {};
  // device
  StageArgs* d_args = nullptr;     // [3][n]
  MaxDtArgs* d_dtargs = nullptr;   // [n]
  int* d_item_solve = nullptr;
  int* d_item_tile = nullptr;
  int* d_begin = nullptr;          // [n+1]
  double* d_partial = nullptr;     // [nitems]
  double* d_dt = nullptr;          // [0,n) host time steps, [n,2n) device bounds
  // host mirrors of what d_args / d_dtargs hold
  std::vector<StageArgs> h_args;
  std::vector<MaxDtArgs> h_dtargs;
  std::vector<double*> cur_u;
  double cur_scale = -1.0;
  int cur_mode = -1;               // 0: host time steps, 1: device bounds
  // pinned ring of host time steps
  double* h_ring = nullptr;
  hipEvent_t ring_ev[kRing] = {};
  int ring_next = 0;
  // graph of one device-timestepped step
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string err = "no error";
};

namespace {

thread_local std::string g_batch_create_error = "no error";

int bfail(idp_dg_batch* b, int code, const std::string& msg) {
  if (b) b->err = msg; else g_batch_create_error = msg;
  return code;
}

int bhip(idp_dg_batch* b, hipError_t e, const char* where) {
  return bfail(b, IDP_DG_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

void drop_batch_graph(idp_dg_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

bool overlap(const double* a, long long na, const double* c, long long nc) {
  return a < c + nc && c < a + na;
}

// Point the per-stage arguments of every solve at u[i] and at the time
// steps in dt_dev (+ i) scaled by dt_scale, and upload them if they changed.
int set_args(idp_dg_batch* b, double* const* u, double* dt_dev, double dt_scale, int mode) {
  bool same = b->cur_scale == dt_scale && b->cur_mode == mode;
  for (int i = 0; same && i < b->n; ++i) same = b->cur_u[i] == u[i];
  if (same) return 0;
  for (int i = 0; i < b->n; ++i) {
    idp_dg* h = b->s[i];
    const double* dtp = dt_dev + i;
    b->h_args[0 * b->n + i] = make_stage_args(h, nullptr, u[i], h->buf1, 0.0, dtp, dt_scale, 0);
    b->h_args[1 * b->n + i] = make_stage_args(h, u[i], h->buf1, h->buf2, 0.0, dtp, dt_scale, 1);
    b->h_args[2 * b->n + i] = make_stage_args(h, u[i], h->buf2, u[i], 0.0, dtp, dt_scale, 2);
    b->h_dtargs[i] = make_dt_args(h, u[i]);
    b->h_dtargs[i].partial = b->d_partial;  // tiles write partial[item]
  }
  hipError_t e = hipMemcpyAsync(b->d_args, b->h_args.data(), sizeof(StageArgs) * 3 * b->n,
                                hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_dtargs, b->h_dtargs.data(), sizeof(MaxDtArgs) * b->n,
                       hipMemcpyHostToDevice, b->stream);
  // the mirrors are rewritten on the next change: let the copies finish
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bhip(b, e, "batch argument upload");
  for (int i = 0; i < b->n; ++i) b->cur_u[i] = u[i];
  b->cur_scale = dt_scale;
  b->cur_mode = mode;
  drop_batch_graph(b);
  return 0;
}

BatchArgs stage_args_of(const idp_dg_batch* b, int stage) {
  BatchArgs a;
  a.args = b->d_args + stage * b->n;
  a.item_solve = b->d_item_solve;
  a.item_tile = b->d_item_tile;
  for (int x = 0; x < 9; ++x) a.chunk[x] = b->chunk[x];
  return a;
}

hipError_t enqueue_batch_stages(const idp_dg_batch* b, hipStream_t s) {
  for (int st = 0; st < 3; ++st) {
    hipError_t e = launch_batch_stage(b->fam, stage_args_of(b, st), b->grid, b->lds, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t enqueue_batch_maxdt(const idp_dg_batch* b, double* out, hipStream_t s) {
  BatchDtArgs a;
  a.args = b->d_dtargs;
  a.item_solve = b->d_item_solve;
  a.item_tile = b->d_item_tile;
  a.partial = b->d_partial;
  for (int x = 0; x < 9; ++x) a.chunk[x] = b->chunk[x];
  hipError_t e = launch_batch_maxdt(b->fam, a, b->grid, b->lds, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(segmented_min_kernel, dim3(b->n), dim3(256), 0, s, b->d_partial, b->d_begin, out);
  return hipGetLastError();
}

int check_states(idp_dg_batch* b, double* const* u) {
  if (!u) return bfail(b, IDP_DG_EINVAL, "u is NULL");
  for (int i = 0; i < b->n; ++i) {
    idp_dg* h = b->s[i];
    const long long ni = (long long)h->nc * h->nn;
    if (!u[i]) return bfail(b, IDP_DG_EINVAL, "u[i] is NULL");
    for (idp_dg* o : b->s) {
      const long long no = (long long)o->nc * o->nn;
      if (overlap(u[i], ni, o->buf1, no) || overlap(u[i], ni, o->buf2, no))
        return bfail(b, IDP_DG_EINVAL, "a state overlaps a solve's stage buffers");
    }
    for (int j = 0; j < i; ++j) {
      const long long nj = (long long)b->s[j]->nc * b->s[j]->nn;
      if (overlap(u[i], ni, u[j], nj)) return bfail(b, IDP_DG_EINVAL, "two states overlap");
    }
  }
  return 0;
}

}  // namespace

extern "C" {

int idp_dg_batch_create(idp_dg* const* solves, int n, void* hip_stream, idp_dg_batch** out) {
  if (!out) return bfail(nullptr, IDP_DG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!solves || n < 1) return bfail(nullptr, IDP_DG_EINVAL, "need at least one solve");
  for (int i = 0; i < n; ++i) {
    if (!solves[i]) return bfail(nullptr, IDP_DG_EINVAL, "NULL solve handle");
    for (int j = 0; j < i; ++j)
      if (solves[j] == solves[i]) return bfail(nullptr, IDP_DG_EINVAL, "a handle appears twice");
  }
  const int fam = family(solves[0]);
  for (int i = 1; i < n; ++i)
    if (family(solves[i]) != fam || solves[i]->device != solves[0]->device)
      return bfail(nullptr, IDP_DG_EINVAL, "solves of one batch must share equation, gamma kind, dimension and device");
  int lds = 0;
  for (int i = 0; i < n; ++i) {
    const int l = batch_lds_bytes(fam, solves[i]->d.p);
    if (l < 0) return bfail(nullptr, IDP_DG_EINVAL, "batched solves need p >= 2 (use the plain path for p = 1)");
    lds = l > lds ? l : lds;
  }
  idp_dg_batch* b = new (std::nothrow) idp_dg_batch;
  if (!b) return bfail(nullptr, IDP_DG_ENOMEM, "host allocation failed");
  b->s.assign(solves, solves + n);
  b->stream = reinterpret_cast<hipStream_t>(hip_stream);
  b->fam = fam;
  b->n = n;
  b->lds = lds;
  std::vector<int> item_solve, item_tile, begin(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    const int epb = batch_tile_elems(fam, solves[i]->d.p);
    const int nt = (solves[i]->ne + epb - 1) / epb;
    begin[i] = (int)item_solve.size();
    for (int t = 0; t < nt; ++t) {
      item_solve.push_back(i);
      item_tile.push_back(t);
    }
  }
  begin[n] = (int)item_solve.size();
  b->nitems = begin[n];
  // tiles of 128 threads carry about the same work: equal counts per XCD
  for (int x = 0; x <= 8; ++x) b->chunk[x] = (int)((long long)b->nitems * x / 8);
  int cus = 0;
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, solves[0]->device);
  const int per_cu = batch_blocks_per_cu(fam, lds);
  int grid = (cus > 0 ? cus : 256) * per_cu;
  const int cap_items = ((b->nitems + 7) / 8) * 8;
  if (grid > cap_items) grid = cap_items;
  b->grid = grid < 8 ? 8 : (grid / 8) * 8;
  b->h_args.resize(3 * n);
  b->h_dtargs.resize(n);
  b->cur_u.assign(n, nullptr);
  hipError_t e = hipMalloc(&b->d_args, sizeof(StageArgs) * 3 * n);
  if (e == hipSuccess) e = hipMalloc(&b->d_dtargs, sizeof(MaxDtArgs) * n);
  if (e == hipSuccess) e = hipMalloc(&b->d_item_solve, sizeof(int) * b->nitems);
  if (e == hipSuccess) e = hipMalloc(&b->d_item_tile, sizeof(int) * b->nitems);
  if (e == hipSuccess) e = hipMalloc(&b->d_begin, sizeof(int) * (n + 1));
  if (e == hipSuccess) e = hipMalloc(&b->d_partial, sizeof(double) * b->nitems);
  if (e == hipSuccess) e = hipMalloc(&b->d_dt, sizeof(double) * 2 * n);
  if (e == hipSuccess) e = hipHostMalloc(&b->h_ring, sizeof(double) * kRing * n, hipHostMallocDefault);
  for (int r = 0; e == hipSuccess && r < kRing; ++r) e = hipEventCreateWithFlags(&b->ring_ev[r], hipEventDisableTiming);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_item_solve, item_solve.data(), sizeof(int) * b->nitems, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_item_tile, item_tile.data(), sizeof(int) * b->nitems, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_begin, begin.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    const int code = e == hipErrorOutOfMemory ? IDP_DG_ENOMEM : IDP_DG_EHIP;
    bfail(nullptr, code, std::string("batch allocation: ") + hipGetErrorString(e));
    idp_dg_batch_destroy(b);
    return code;
  }
  *out = b;
  return 0;
}

void idp_dg_batch_destroy(idp_dg_batch* b) {
  if (!b) return;
  drop_batch_graph(b);
  if (b->cap) hipStreamDestroy(b->cap);
  for (int r = 0; r < kRing; ++r)
    if (b->ring_ev[r]) hipEventDestroy(b->ring_ev[r]);
  hipFree(b->d_args);
  hipFree(b->d_dtargs);
  hipFree(b->d_item_solve);
  hipFree(b->d_item_tile);
  hipFree(b->d_begin);
  hipFree(b->d_partial);
  hipFree(b->d_dt);
  if (b->h_ring) hipHostFree(b->h_ring);
  delete b;
}

int idp_dg_batch_num_items(const idp_dg_batch* b) { return b ? b->nitems : -1; }

int idp_dg_batch_step(idp_dg_batch* b, double* const* u, const double* dt) {
  if (!b) return IDP_DG_EINVAL;
  if (!dt) return bfail(b, IDP_DG_EINVAL, "dt is NULL");
  for (int i = 0; i < b->n; ++i)
    if (!(dt[i] >= 0.0) || !std::isfinite(dt[i])) return bfail(b, IDP_DG_EINVAL, "dt must be finite and >= 0");
  int rc = check_states(b, u);
  if (rc) return rc;
  // stage the time steps through a pinned ring slot (the slot is reused
  // only after its copy has run)
  const int r = b->ring_next;
  b->ring_next = (r + 1) % kRing;
  hipError_t e = hipEventSynchronize(b->ring_ev[r]);
  if (e != hipSuccess) return bhip(b, e, "ring event");
  double* slot = b->h_ring + (size_t)r * b->n;
  std::memcpy(slot, dt, sizeof(double) * b->n);
  rc = set_args(b, u, b->d_dt, 1.0, 0);
  if (rc) return rc;
  e = hipMemcpyAsync(b->d_dt, slot, sizeof(double) * b->n, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipEventRecord(b->ring_ev[r], b->stream);
  if (e != hipSuccess) return bhip(b, e, "dt upload");
  e = enqueue_batch_stages(b, b->stream);
  if (e != hipSuccess) return bhip(b, e, "batch stage launch");
  return 0;
}

int idp_dg_batch_step_cfl(idp_dg_batch* b, double* const* u, double cfl) {
  if (!b) return IDP_DG_EINVAL;
  if (!(cfl > 0.0) || !std::isfinite(cfl)) return bfail(b, IDP_DG_EINVAL, "cfl must be finite and > 0");
  int rc = check_states(b, u);
  if (rc) return rc;
  double* bounds = b->d_dt + b->n;
  rc = set_args(b, u, bounds, cfl, 1);
  if (rc) return rc;
  hipError_t e;
  if (!b->exec) {
    if (!b->cap) {
      e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
      if (e != hipSuccess) return bhip(b, e, "hipStreamCreate");
    }
    e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bhip(b, e, "hipStreamBeginCapture");
    hipError_t le = enqueue_batch_maxdt(b, bounds, b->cap);
    if (le == hipSuccess) le = enqueue_batch_stages(b, b->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->cap, &g);
    if (le != hipSuccess) { if (g) hipGraphDestroy(g); return bhip(b, le, "batch capture"); }
    if (e != hipSuccess) return bhip(b, e, "hipStreamEndCapture");
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) { drop_batch_graph(b); return bhip(b, e, "hipGraphInstantiate"); }
  }
  e = hipGraphLaunch(b->exec, b->stream);
  if (e != hipSuccess) return bhip(b, e, "hipGraphLaunch");
  return 0;
}

int idp_dg_batch_last_dt(idp_dg_batch* b, double* dt) {
  if (!b || !dt) return IDP_DG_EINVAL;
  std::vector<double> v(b->n);
  const double* bounds = b->d_dt + b->n;
  hipError_t e = hipMemcpyAsync(v.data(), bounds, sizeof(double) * b->n, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bhip(b, e, "batch dt copy");
  for (int i = 0; i < b->n; ++i) {
    double d = b->cur_scale * v[i];  // the product the stage kernels form
    dt[i] = d < INFINITY ? d : 0.0;
  }
  return 0;
}

const char* idp_dg_batch_last_error(const idp_dg_batch* b) {
  return b ? b->err.c_str() : g_batch_create_error.c_str();
}

}  // extern "C"
