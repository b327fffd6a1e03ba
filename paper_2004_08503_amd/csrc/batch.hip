// Batched execution: many independent solves of one equation family (any
// mix of mesh sizes and degrees) advance together.  The solves are grouped
// by degree; each group has a work list of (solve, element tile) items over
// all its solves and one work-list kernel per RK stage (the plain path's
// tile shape, mapped XCD-aware over the list).  A batched step runs, per
// stage, the groups' kernels; in the device-timestepped mode the groups'
// time-step kernels and one segmented minimum come first.
//
// Everything a launch reads (per-solve stage arguments, work lists, item
// ranges) lives in one device blob that is rewritten by a single
// asynchronous copy from a pinned staging ring whenever the membership, the
// state pointers or the time-step mode change, so changing a batch never
// synchronises the host with the device.  The kernels of a step are
// launched directly on the batch's stream (a few launches per degree
// present; at the batch sizes this path is for, the launches cost well
// under one per cent of a step).  A batch does not capture its step as a
// HIP graph: capturing on repeated configurations and retiring the graph
// on every membership change (with its launch still queued) is the one
// pattern common to the host aborts seen under serving loads, whose cause
// in the runtime or in this code is not established.
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
constexpr int kRing = 4;   // pinned staging slots
constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
}  // namespace

struct BatchGroup {
  int p = 0;
  BatchKernels k{};
  int nitems = 0;
  int ofs = 0;        // first item of the group in the work-list arrays
};

struct idp_dg_batch {
  std::vector<idp_dg*> s;
  hipStream_t stream = nullptr;
  int fam = 0;
  int n = 0;
  int nitems = 0;
  std::vector<BatchGroup> groups;
  int shape[MAXP + 1] = {};        // tile shape of each degree's kernels
  bool dirty = true;               // membership (or a tile shape) changed since the last upload
  // blob layout (offsets in bytes) for the current n / nitems
  size_t o_args = 0, o_dtargs = 0, o_isolve = 0, o_itile = 0, o_range = 0, o_partial = 0,
         o_dt = 0, blob_bytes = 0, stage_bytes = 0;
  char* d_blob = nullptr;
  size_t d_cap = 0;
  char* h_ring = nullptr;          // kRing pinned slots of h_cap bytes
  size_t h_cap = 0;
  hipEvent_t ring_ev[kRing] = {};
  int ring_next = 0;
  // what the device blob currently describes
  std::vector<double*> cur_u;
  std::vector<unsigned> cur_bv;    // the solves' boundary versions
  std::vector<unsigned> cur_mv;    // the solves' mesh versions
  double cur_scale = -1.0;
  int cur_mode = -1;               // 0: host time steps, 1: device bounds
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

bool overlap(const double* a, long long na, const double* c, long long nc) {
  return a < c + nc && c < a + na;
}

template <class T>
T* at(char* base, size_t off) { return reinterpret_cast<T*>(base + off); }

// the work-list kernels of member h: its degree's tile shape, or on a
// curved mesh the curved kernels of the first shape
int member_kernels(const idp_dg_batch* b, const idp_dg* h, BatchKernels* k) {
  return h->metric ? batch_kernels_curved(b->fam, h->d.p, k) : batch_kernels(b->fam, h->d.p, b->shape[h->d.p], k);
}

// Work lists and blob layout for the current membership: one group per
// degree and mesh kind (Cartesian, curved).
int plan(idp_dg_batch* b, std::vector<int>* isolve, std::vector<int>* itile, std::vector<int>* range) {
  b->groups.clear();
  isolve->clear();
  itile->clear();
  range->assign(2 * b->n, 0);
  for (int p = 1; p <= MAXP; ++p)
  for (int curved = 0; curved < 2; ++curved) {
    BatchGroup gr;
    gr.p = p;
    gr.ofs = (int)isolve->size();
    for (int i = 0; i < b->n; ++i) {
      if (b->s[i]->d.p != p || (b->s[i]->metric != nullptr) != (curved == 1)) continue;
      if (member_kernels(b, b->s[i], &gr.k))
        return bfail(b, IDP_DG_EINVAL, "no batched kernel for this degree");
      const int nt = ((b->s[i]->d.nx + gr.k.tile_x - 1) / gr.k.tile_x) *
                     ((b->s[i]->d.ny + gr.k.tile_y - 1) / gr.k.tile_y);
      if ((long long)isolve->size() + nt > 0x7fffffffLL)   // item indices and grids are int
        return bfail(b, IDP_DG_EINVAL, "batch too large: more than 2^31 - 1 work items");
      (*range)[2 * i] = (int)isolve->size();
      for (int t = 0; t < nt; ++t) {
        isolve->push_back(i);
        itile->push_back(t);
      }
      (*range)[2 * i + 1] = (int)isolve->size();
    }
    gr.nitems = (int)isolve->size() - gr.ofs;
    if (gr.nitems > 0) b->groups.push_back(gr);
  }
  b->nitems = (int)isolve->size();
  const size_t n = b->n, ni = b->nitems;
  b->o_args = 0;
  b->o_dtargs = up(b->o_args + sizeof(StageArgs) * 3 * n);
  b->o_isolve = up(b->o_dtargs + sizeof(MaxDtArgs) * n);
  b->o_itile = up(b->o_isolve + sizeof(int) * ni);
  b->o_range = up(b->o_itile + sizeof(int) * ni);
  b->stage_bytes = up(b->o_range + sizeof(int) * 2 * n);   // the part uploaded from the host
  b->o_partial = b->stage_bytes;
  b->o_dt = up(b->o_partial + sizeof(double) * ni);
  b->blob_bytes = up(b->o_dt + sizeof(double) * 2 * n);
  return 0;
}

// Rewrite the device blob for (membership, u, mode, scale) through a pinned
// staging slot with one asynchronous copy.
int upload(idp_dg_batch* b, double* const* u, int mode, double scale) {
  std::vector<int> isolve, itile, range;
  int rc = plan(b, &isolve, &itile, &range);
  if (rc) return rc;
  hipError_t e = hipSuccess;
  if (b->blob_bytes > b->d_cap) {
    // growing: the old blob may still be read by queued launches
    if (b->d_blob) {
      e = hipStreamSynchronize(b->stream);
      if (e == hipSuccess) e = hipFree(b->d_blob);
      b->d_blob = nullptr;
      b->d_cap = 0;
    }
    const size_t cap = b->blob_bytes + b->blob_bytes / 2;
    if (e == hipSuccess) e = hipMalloc(&b->d_blob, cap);
    if (e != hipSuccess) return bhip(b, e, "batch blob");
    b->d_cap = cap;
  }
  const size_t need = b->stage_bytes > sizeof(double) * b->n ? b->stage_bytes : sizeof(double) * b->n;
  if (need > b->h_cap) {
    if (b->h_ring) {
      for (int r = 0; r < kRing; ++r) (void)hipEventSynchronize(b->ring_ev[r]);
      (void)hipHostFree(b->h_ring);
      b->h_ring = nullptr;
    }
    const size_t cap = up(need + need / 2);
    e = hipHostMalloc(&b->h_ring, cap * kRing, hipHostMallocDefault);
    if (e != hipSuccess) return bhip(b, e, "batch staging");
    b->h_cap = cap;
  }
  const int r = b->ring_next;
  b->ring_next = (r + 1) % kRing;
  e = hipEventSynchronize(b->ring_ev[r]);   // the slot's previous copy has run
  if (e != hipSuccess) return bhip(b, e, "staging event");
  char* h = b->h_ring + (size_t)r * b->h_cap;
  char* d = b->d_blob;
  double* dt_dev = at<double>(d, b->o_dt) + (mode == 1 ? b->n : 0);
  StageArgs* a = at<StageArgs>(h, b->o_args);
  MaxDtArgs* m = at<MaxDtArgs>(h, b->o_dtargs);
  for (int i = 0; i < b->n; ++i) {
    idp_dg* hd = b->s[i];
    const double* dtp = dt_dev + i;
    a[0 * b->n + i] = make_stage_args(hd, nullptr, u[i], hd->buf1, 0.0, dtp, scale, 0);
    a[1 * b->n + i] = make_stage_args(hd, u[i], hd->buf1, hd->buf2, 0.0, dtp, scale, 1);
    a[2 * b->n + i] = make_stage_args(hd, u[i], hd->buf2, u[i], 0.0, dtp, scale, 2);
    m[i] = make_dt_args(hd, u[i]);
    m[i].partial = at<double>(d, b->o_partial);
    // the tiles are those of the degree's batched kernels, whose shape may
    // differ from the member's own
    BatchKernels k;
    if (member_kernels(b, hd, &k)) return bfail(b, IDP_DG_EINVAL, "no batched kernel");
    const int ntx = (hd->d.nx + k.tile_x - 1) / k.tile_x;
    const int nt = ntx * ((hd->d.ny + k.tile_y - 1) / k.tile_y);
    for (int st = 0; st < 3; ++st) {
      a[st * b->n + i].S.ntx = ntx;
      a[st * b->n + i].S.ntiles = nt;
    }
    m[i].ntx = ntx;
    m[i].ntiles = nt;
  }
  if (b->nitems) {
    std::memcpy(h + b->o_isolve, isolve.data(), sizeof(int) * b->nitems);
    std::memcpy(h + b->o_itile, itile.data(), sizeof(int) * b->nitems);
  }
  std::memcpy(h + b->o_range, range.data(), sizeof(int) * 2 * b->n);
  e = hipMemcpyAsync(d, h, b->stage_bytes, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipEventRecord(b->ring_ev[r], b->stream);
  if (e != hipSuccess) return bhip(b, e, "batch upload");
  b->cur_u.assign(u, u + b->n);
  b->cur_bv.resize(b->n);
  b->cur_mv.resize(b->n);
  for (int i = 0; i < b->n; ++i) {
    b->cur_bv[i] = b->s[i]->bnd_version;
    b->cur_mv[i] = b->s[i]->mesh_version;
  }
  b->cur_mode = mode;
  b->cur_scale = scale;
  b->dirty = false;
  return 0;
}

int prepare(idp_dg_batch* b, double* const* u, int mode, double scale) {
  bool same = !b->dirty && b->cur_mode == mode && b->cur_scale == scale;
  for (int i = 0; same && i < b->n; ++i)
    same = b->cur_u[i] == u[i] && b->cur_bv[i] == b->s[i]->bnd_version && b->cur_mv[i] == b->s[i]->mesh_version;
  if (same) return 0;
  return upload(b, u, mode, scale);
}

BatchArgs group_args(const idp_dg_batch* b, const BatchGroup& gr, int stage) {
  BatchArgs a;
  a.args = at<StageArgs>(b->d_blob, b->o_args) + stage * b->n;
  a.item_solve = at<int>(b->d_blob, b->o_isolve) + gr.ofs;
  a.item_tile = at<int>(b->d_blob, b->o_itile) + gr.ofs;
  a.nitems = gr.nitems;
  return a;
}

BatchDtArgs group_dt_args(const idp_dg_batch* b, const BatchGroup& gr) {
  BatchDtArgs a;
  a.args = at<MaxDtArgs>(b->d_blob, b->o_dtargs);
  a.item_solve = at<int>(b->d_blob, b->o_isolve) + gr.ofs;
  a.item_tile = at<int>(b->d_blob, b->o_itile) + gr.ofs;
  a.partial = at<double>(b->d_blob, b->o_partial) + gr.ofs;
  a.nitems = gr.nitems;
  return a;
}

// The launches of one step on the batch's stream: per stage, every degree
// group's work-list kernel (stream order puts each stage after the one
// before).
hipError_t run_step(idp_dg_batch* b, int mode) {
  if (b->nitems == 0) return hipSuccess;
  hipError_t e = hipSuccess;
  if (mode == 1) {
    for (const BatchGroup& gr : b->groups) {
      BatchDtArgs a = group_dt_args(b, gr);
      void* args[] = {&a};
      e = hipLaunchKernel(gr.k.maxdt, dim3(gr.nitems), dim3(gr.k.block), args, 0, b->stream);
      if (e != hipSuccess) return e;
    }
    const double* part = at<double>(b->d_blob, b->o_partial);
    const int* range = at<int>(b->d_blob, b->o_range);
    double* out = at<double>(b->d_blob, b->o_dt) + b->n;
    void* args[] = {&part, &range, &out};
    e = hipLaunchKernel(reinterpret_cast<const void*>(&segmented_min_kernel), dim3(b->n), dim3(256), args, 0,
                        b->stream);
    if (e != hipSuccess) return e;
  }
  for (int st = 0; st < 3; ++st) {
    for (const BatchGroup& gr : b->groups) {
      BatchArgs a = group_args(b, gr, st);
      void* args[] = {&a};
      e = hipLaunchKernel(gr.k.stage, dim3(gr.nitems), dim3(gr.k.block), args, 0, b->stream);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

int check_members(idp_dg* const* solves, int n, idp_dg_batch* b) {
  if (!solves || n < 1) return bfail(b, IDP_DG_EINVAL, "need at least one solve");
  for (int i = 0; i < n; ++i) {
    if (!solves[i]) return bfail(b, IDP_DG_EINVAL, "NULL solve handle");
    for (int j = 0; j < i; ++j)
      if (solves[j] == solves[i]) return bfail(b, IDP_DG_EINVAL, "a handle appears twice");
  }
  for (int i = 1; i < n; ++i)
    if (family(solves[i]) != family(solves[0]) || solves[i]->device != solves[0]->device)
      return bfail(b, IDP_DG_EINVAL, "solves of one batch must share equation, gamma kind, dimension and device");
  return 0;
}

int check_states(idp_dg_batch* b, double* const* u) {
  if (!u) return bfail(b, IDP_DG_EINVAL, "u is NULL");
  for (int i = 0; i < b->n; ++i) {
    idp_dg* h = b->s[i];
    const long long ni = (long long)h->nc * h->nn;
    if (!u[i]) return bfail(b, IDP_DG_EINVAL, "u[i] is NULL");
    if (!bnd_ready(h)) return bfail(b, IDP_DG_EINVAL, "a solve has an open side without boundary conditions");
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
  const idp_host::Range trace_range("idp_dg_batch_create");
  if (!out) return bfail(nullptr, IDP_DG_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_members(solves, n, nullptr);
  if (rc) return rc;
  idp_dg_batch* b = new (std::nothrow) idp_dg_batch;
  if (!b) return bfail(nullptr, IDP_DG_ENOMEM, "host allocation failed");
  b->stream = reinterpret_cast<hipStream_t>(hip_stream);
  hipError_t e = hipSuccess;
  for (int r = 0; e == hipSuccess && r < kRing; ++r)
    e = hipEventCreateWithFlags(&b->ring_ev[r], hipEventDisableTiming);
  if (e != hipSuccess) {
    bfail(nullptr, IDP_DG_EHIP, std::string("batch events: ") + hipGetErrorString(e));
    idp_dg_batch_destroy(b);
    return IDP_DG_EHIP;
  }
  rc = idp_dg_batch_update(b, solves, n);
  if (rc) {
    g_batch_create_error = b->err;
    idp_dg_batch_destroy(b);
    return rc;
  }
  *out = b;
  return 0;
}

int idp_dg_batch_update(idp_dg_batch* b, idp_dg* const* solves, int n) {
  const idp_host::Range trace_range("idp_dg_batch_update");
  if (!b) return IDP_DG_EINVAL;
  int rc = check_members(solves, n, b);
  if (rc) return rc;
  b->s.assign(solves, solves + n);
  b->fam = family(solves[0]);
  b->n = n;
  std::vector<int> isolve, itile, range;
  rc = plan(b, &isolve, &itile, &range);   // validates the degrees, sizes the blob
  if (rc) return rc;
  b->dirty = true;
  return 0;
}

void idp_dg_batch_destroy(idp_dg_batch* b) {
  if (!b) return;
  if (b->stream || b->d_blob) (void)hipStreamSynchronize(b->stream);   // queued steps read the blob
  for (int r = 0; r < kRing; ++r)
    if (b->ring_ev[r]) {
      (void)hipEventSynchronize(b->ring_ev[r]);
      (void)hipEventDestroy(b->ring_ev[r]);
    }
  if (b->d_blob) (void)hipFree(b->d_blob);
  if (b->h_ring) (void)hipHostFree(b->h_ring);
  delete b;
}

int idp_dg_batch_num_items(const idp_dg_batch* b) { return b ? b->nitems : -1; }

int idp_dg_batch_step(idp_dg_batch* b, double* const* u, const double* dt) {
  const idp_host::Range trace_range("idp_dg_batch_step");
  if (!b) return IDP_DG_EINVAL;
  if (!dt) return bfail(b, IDP_DG_EINVAL, "dt is NULL");
  for (int i = 0; i < b->n; ++i)
    if (!(dt[i] >= 0.0) || !std::isfinite(dt[i])) return bfail(b, IDP_DG_EINVAL, "dt must be finite and >= 0");
  int rc = check_states(b, u);
  if (rc) return rc;
  rc = prepare(b, u, 0, 1.0);
  if (rc) return rc;
  // the time steps go through a staging slot of their own
  const int r = b->ring_next;
  b->ring_next = (r + 1) % kRing;
  hipError_t e = hipEventSynchronize(b->ring_ev[r]);
  if (e != hipSuccess) return bhip(b, e, "staging event");
  double* h = reinterpret_cast<double*>(b->h_ring + (size_t)r * b->h_cap);
  std::memcpy(h, dt, sizeof(double) * b->n);
  e = hipMemcpyAsync(at<double>(b->d_blob, b->o_dt), h, sizeof(double) * b->n, hipMemcpyHostToDevice,
                     b->stream);
  if (e == hipSuccess) e = hipEventRecord(b->ring_ev[r], b->stream);
  if (e == hipSuccess) e = run_step(b, 0);
  if (e != hipSuccess) return bhip(b, e, "batch step");
  return 0;
}

int idp_dg_batch_step_cfl(idp_dg_batch* b, double* const* u, double cfl) {
  const idp_host::Range trace_range("idp_dg_batch_step_cfl");
  if (!b) return IDP_DG_EINVAL;
  if (!(cfl > 0.0) || !std::isfinite(cfl)) return bfail(b, IDP_DG_EINVAL, "cfl must be finite and > 0");
  int rc = check_states(b, u);
  if (rc) return rc;
  rc = prepare(b, u, 1, cfl);
  if (rc) return rc;
  hipError_t e = run_step(b, 1);
  if (e != hipSuccess) return bhip(b, e, "batch step");
  return 0;
}

int idp_dg_batch_tune(idp_dg_batch* b, double* const* u, double cfl, int reps) {
  const idp_host::Range trace_range("idp_dg_batch_tune");
  if (!b) return IDP_DG_EINVAL;
  int rc = check_states(b, u);
  if (rc) return rc;
  // a member's timed steps write its stage buffers, which queued batch steps
  // also use: let the batch's work finish first (a member may run on
  // another stream)
  hipError_t e0 = hipStreamSynchronize(b->stream);
  if (e0 != hipSuccess) return bhip(b, e0, "batch tune");
  for (int p = 1; p <= MAXP; ++p) {
    int big = -1;
    for (int i = 0; i < b->n; ++i)
      if (b->s[i]->d.p == p && !b->s[i]->metric && (big < 0 || b->s[i]->nn > b->s[big]->nn)) big = i;
    if (big < 0) continue;
    idp_dg* h = b->s[big];
    const int keep = h->variant;
    int shape = 0;
    rc = idp_dg_tune(h, u[big], cfl, reps, &shape);
    if (rc) return bfail(b, rc, std::string("tuning a member: ") + h->err);
    rc = idp_dg_set_tile_shape(h, keep);   // the member's own shape is its own business
    if (rc) return bfail(b, rc, h->err);
    if (shape != b->shape[p]) {
      b->shape[p] = shape;
      b->dirty = true;
    }
  }
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bhip(b, e, "batch tune");
  return 0;
}

int idp_dg_batch_last_dt(idp_dg_batch* b, double* dt) {
  if (!b || !dt) return IDP_DG_EINVAL;
  if (!b->d_blob || b->cur_mode != 1) return bfail(b, IDP_DG_EINVAL, "no device-timestepped step has run");
  std::vector<double> v(b->n);
  const double* bounds = at<double>(b->d_blob, b->o_dt) + b->n;
  hipError_t e = hipMemcpyAsync(v.data(), bounds, sizeof(double) * b->n, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bhip(b, e, "batch dt copy");
  for (int i = 0; i < b->n; ++i) {
    const double d = b->cur_scale * v[i];  // the product the stage kernels form
    dt[i] = d < INFINITY ? d : 0.0;
  }
  return 0;
}

const char* idp_dg_batch_last_error(const idp_dg_batch* b) {
  return b ? b->err.c_str() : g_batch_create_error.c_str();
}

}  // extern "C"
