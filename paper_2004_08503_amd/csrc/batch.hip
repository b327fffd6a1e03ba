// Batched execution: many independent solves of one equation family (any
// mix of mesh sizes and degrees) advance together.  The solves are grouped
// by degree; each group has a work list of (solve, element tile) items over
// all its solves and one work-list kernel per RK stage (the plain path's
// tile shape, mapped XCD-aware over the list).  A batched step is one HIP
// graph, built once per (pointer set, time-step mode, cfl): the groups'
// kernels of a stage are parallel branches, the stages follow each other,
// and in the device-timestepped mode the groups' time-step kernels and one
// segmented minimum come first.  Host time steps reach the device through
// a pinned ring before the graph launch.
//
// Results are bitwise identical to the plain path: a tile's arithmetic does
// not depend on which workgroup or launch runs it, and the only reductions
// (alpha over faces, dt over nodes) are minima.
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

struct BatchGroup {
  int p = 0;
  BatchKernels k{};
  int nitems = 0;
  int ofs = 0;        // first item of the group in the item arrays / partials
};

struct idp_dg_batch {
  std::vector<idp_dg*> s;
  hipStream_t stream = nullptr;
  int fam = 0;
  int n = 0;
  int nitems = 0;
  std::vector<BatchGroup> groups;
  // device
  StageArgs* d_args = nullptr;     // [3][n]
  MaxDtArgs* d_dtargs = nullptr;   // [n]
  int* d_item_solve = nullptr;     // [nitems], grouped by degree
  int* d_item_tile = nullptr;
  int* d_range = nullptr;          // [2n] item range of each solve
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
  // graph of one step in the current mode
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

hipError_t add_kernel(hipGraph_t g, hipGraphNode_t* node, const std::vector<hipGraphNode_t>& deps,
                      const void* func, dim3 grid, dim3 block, void** args) {
  hipKernelNodeParams kp;
  std::memset(&kp, 0, sizeof(kp));
  kp.func = const_cast<void*>(func);
  kp.gridDim = grid;
  kp.blockDim = block;
  kp.sharedMemBytes = 0;
  kp.kernelParams = args;
  kp.extra = nullptr;
  return hipGraphAddKernelNode(node, g, deps.empty() ? nullptr : deps.data(), deps.size(), &kp);
}

// One batched step as a graph: [time-step kernels of every group ->
// segmented min ->] stage 0 of every group -> stage 1 -> stage 2.
hipError_t build_graph(idp_dg_batch* b, bool device_dt) {
  hipGraph_t g = nullptr;
  hipError_t e = hipGraphCreate(&g, 0);
  if (e != hipSuccess) return e;
  std::vector<hipGraphNode_t> prev;
  if (device_dt) {
    std::vector<hipGraphNode_t> dts;
    for (const BatchGroup& gr : b->groups) {
      BatchDtArgs a;
      a.args = b->d_dtargs;
      a.item_solve = b->d_item_solve + gr.ofs;
      a.item_tile = b->d_item_tile + gr.ofs;
      a.partial = b->d_partial + gr.ofs;
      a.nitems = gr.nitems;
      void* args[] = {&a};
      hipGraphNode_t nd;
      e = add_kernel(g, &nd, {}, gr.k.maxdt, dim3(gr.nitems), dim3(gr.k.block), args);
      if (e != hipSuccess) break;
      dts.push_back(nd);
    }
    if (e == hipSuccess) {
      const double* part = b->d_partial;
      const int* range = b->d_range;
      double* out = b->d_dt + b->n;
      void* args[] = {&part, &range, &out};
      hipGraphNode_t nd;
      e = add_kernel(g, &nd, dts, reinterpret_cast<const void*>(&segmented_min_kernel), dim3(b->n),
                     dim3(256), args);
      prev.assign(1, nd);
    }
  }
  for (int st = 0; st < 3 && e == hipSuccess; ++st) {
    std::vector<hipGraphNode_t> cur;
    for (const BatchGroup& gr : b->groups) {
      BatchArgs a;
      a.args = b->d_args + st * b->n;
      a.item_solve = b->d_item_solve + gr.ofs;
      a.item_tile = b->d_item_tile + gr.ofs;
      a.nitems = gr.nitems;
      void* args[] = {&a};
      hipGraphNode_t nd;
      e = add_kernel(g, &nd, prev, gr.k.stage, dim3(gr.nitems), dim3(gr.k.block), args);
      if (e != hipSuccess) break;
      cur.push_back(nd);
    }
    prev.swap(cur);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(g);
    b->exec = nullptr;
    return e;
  }
  b->graph = g;
  return hipSuccess;
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
  idp_dg_batch* b = new (std::nothrow) idp_dg_batch;
  if (!b) return bfail(nullptr, IDP_DG_ENOMEM, "host allocation failed");
  b->s.assign(solves, solves + n);
  b->stream = reinterpret_cast<hipStream_t>(hip_stream);
  b->fam = fam;
  b->n = n;
  std::vector<int> item_solve, item_tile, range(2 * n, 0);
  for (int p = 1; p <= MAXP; ++p) {
    BatchGroup gr;
    gr.p = p;
    gr.ofs = (int)item_solve.size();
    for (int i = 0; i < n; ++i) {
      if (solves[i]->d.p != p) continue;
      if (batch_kernels(fam, p, &gr.k)) {
        delete b;
        return bfail(nullptr, IDP_DG_EINVAL, "no batched kernel for this degree");
      }
      const int epb = gr.k.tile_elems;
      const int nt = (solves[i]->ne + epb - 1) / epb;
      range[2 * i] = (int)item_solve.size();
      for (int t = 0; t < nt; ++t) {
        item_solve.push_back(i);
        item_tile.push_back(t);
      }
      range[2 * i + 1] = (int)item_solve.size();
    }
    gr.nitems = (int)item_solve.size() - gr.ofs;
    if (gr.nitems > 0) b->groups.push_back(gr);
  }
  b->nitems = (int)item_solve.size();
  b->h_args.resize(3 * n);
  b->h_dtargs.resize(n);
  b->cur_u.assign(n, nullptr);
  hipError_t e = hipMalloc(&b->d_args, sizeof(StageArgs) * 3 * n);
  if (e == hipSuccess) e = hipMalloc(&b->d_dtargs, sizeof(MaxDtArgs) * n);
  if (e == hipSuccess) e = hipMalloc(&b->d_item_solve, sizeof(int) * b->nitems);
  if (e == hipSuccess) e = hipMalloc(&b->d_item_tile, sizeof(int) * b->nitems);
  if (e == hipSuccess) e = hipMalloc(&b->d_range, sizeof(int) * 2 * n);
  if (e == hipSuccess) e = hipMalloc(&b->d_partial, sizeof(double) * b->nitems);
  if (e == hipSuccess) e = hipMalloc(&b->d_dt, sizeof(double) * 2 * n);
  if (e == hipSuccess) e = hipHostMalloc(&b->h_ring, sizeof(double) * kRing * n, hipHostMallocDefault);
  for (int r = 0; e == hipSuccess && r < kRing; ++r) e = hipEventCreateWithFlags(&b->ring_ev[r], hipEventDisableTiming);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_item_solve, item_solve.data(), sizeof(int) * b->nitems, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_item_tile, item_tile.data(), sizeof(int) * b->nitems, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_range, range.data(), sizeof(int) * 2 * n, hipMemcpyHostToDevice);
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
  for (int r = 0; r < kRing; ++r)
    if (b->ring_ev[r]) hipEventDestroy(b->ring_ev[r]);
  hipFree(b->d_args);
  hipFree(b->d_dtargs);
  hipFree(b->d_item_solve);
  hipFree(b->d_item_tile);
  hipFree(b->d_range);
  hipFree(b->d_partial);
  hipFree(b->d_dt);
  if (b->h_ring) (void)hipHostFree(b->h_ring);
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
  if (!b->exec) {
    e = build_graph(b, false);
    if (e != hipSuccess) return bhip(b, e, "batch graph");
  }
  e = hipGraphLaunch(b->exec, b->stream);
  if (e != hipSuccess) return bhip(b, e, "hipGraphLaunch");
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
    e = build_graph(b, true);
    if (e != hipSuccess) return bhip(b, e, "batch graph");
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
