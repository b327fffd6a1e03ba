// Host-side lifetime check of libidp_dg against the runtime stand-in
// (hip_mock.cpp), under AddressSanitizer.
//  1. The call pattern of a serving loop whose ticks run nested sub-steps:
//     per tick each admitted request takes k steps (k from its step cost),
//     each sub-step updates the per-family batch to the requests that still
//     step and calls idp_dg_batch_step_cfl, without host synchronisation;
//     requests retire on an event recorded after their last sub-step and
//     are destroyed once it completes.
//  2. The plain path: device-timestepped steps whose graph is re-captured
//     whenever the state pointer or the CFL number changes, then destroyed
//     with launches pending.
//  3. A curved mesh: idp_dg_set_mesh between queued steps.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <vector>
#include <algorithm>
#include <random>
#include "idp_dg.h"

extern "C" {
int hipMalloc(void** p, size_t n);
int hipFree(void* p);
int hipEventCreateWithFlags(void** e, unsigned f);
int hipEventRecord(void* e, void* s);
int hipEventQuery(void* e);
int hipEventSynchronize(void* e);
int hipEventDestroy(void* e);
int hipStreamSynchronize(void* s);
void mock_report();
}

struct Req { int id, kind, n, p, steps, left; double arrival_tick; idp_dg* h = nullptr; void* ws = nullptr; double* u = nullptr; int fam = 0; double cost = 0; };

static int fam_of(const Req& r) { return r.kind; }

int main(int argc, char** argv) {
  int nreq = argc > 1 ? atoi(argv[1]) : 80;
  int maxsub = argc > 2 ? atoi(argv[2]) : 16;
  unsigned seed = argc > 3 ? atoi(argv[3]) : 5;
  std::mt19937 rng(seed);
  std::vector<Req> reqs;
  for (int i = 0; i < nreq; ++i) {
    Req r; r.id = i; r.kind = rng() % 2; r.n = 4 + rng() % 60; r.p = 2 + rng() % 5;
    r.steps = 20 + rng() % 181; r.left = r.steps; r.arrival_tick = i * 1.5;
    double nodes = double(r.n) * r.n * (r.p + 1) * (r.p + 1);
    r.cost = 3.0 * nodes / (r.kind ? 5e9 : 4e10);
    reqs.push_back(r);
  }
  std::map<int, std::pair<std::vector<int>, idp_dg_batch*>> batches;
  std::map<int, Req*> active;
  std::vector<std::pair<Req*, void*>> finishing;
  size_t next = 0; int tick = 0, done = 0;
  while (done < nreq) {
    while (next < reqs.size() && reqs[next].arrival_tick <= tick) {
      Req& r = reqs[next++];
      idp_dg_desc d{}; d.dim = 2; d.nx = r.n; d.ny = r.n; d.lx = 1; d.ly = 1; d.p = r.p;
      d.eq = r.kind ? IDP_DG_EULER : IDP_DG_BURGERS; d.velocity[0] = 1; d.velocity[1] = 1; d.gamma = 1.4;
      d.limiter = IDP_DG_SUBCELL;
      long long bytes = idp_dg_workspace_bytes(&d);
      hipMalloc(&r.ws, bytes + 256);
      if (idp_dg_create_in(&d, nullptr, r.ws, bytes, &r.h)) { fprintf(stderr, "create_in: %s\n", idp_dg_last_error(nullptr)); return 1; }
      hipMalloc((void**)&r.u, sizeof(double) * idp_dg_num_comp(r.h) * idp_dg_num_nodes(r.h));
      active[r.id] = &r;
    }
    ++tick;
    if (active.empty()) continue;
    double quantum = 0; for (auto& kv : active) quantum = std::max(quantum, kv.second->cost);
    std::map<int, int> take; int maxk = 0;
    for (auto& kv : active) {
      int k = std::max(1, std::min(std::min(kv.second->left, maxsub), int(quantum / kv.second->cost)));
      take[kv.first] = k; maxk = std::max(maxk, k);
    }
    for (int sub = 0; sub < maxk; ++sub) {
      std::map<int, std::vector<int>> fams;
      for (auto& kv : take) if (kv.second > sub) fams[fam_of(*active[kv.first])].push_back(kv.first);
      for (auto& fv : fams) {
        std::vector<int> ids = fv.second; std::sort(ids.begin(), ids.end());
        std::vector<idp_dg*> hs; std::vector<double*> us;
        for (int id : ids) { hs.push_back(active[id]->h); us.push_back(active[id]->u); }
        auto it = batches.find(fv.first);
        if (it == batches.end()) {
          idp_dg_batch* b = nullptr;
          if (idp_dg_batch_create(hs.data(), (int)hs.size(), nullptr, &b)) { fprintf(stderr, "batch_create: %s\n", idp_dg_batch_last_error(nullptr)); return 1; }
          batches[fv.first] = {ids, b};
        } else if (it->second.first != ids) {
          if (idp_dg_batch_update(it->second.second, hs.data(), (int)hs.size())) { fprintf(stderr, "update: %s\n", idp_dg_batch_last_error(it->second.second)); return 1; }
          it->second.first = ids;
        }
        idp_dg_batch* b = batches[fv.first].second;
        if (idp_dg_batch_step_cfl(b, us.data(), 0.5)) { fprintf(stderr, "step_cfl: %s\n", idp_dg_batch_last_error(b)); return 1; }
      }
      std::vector<int> done_now;
      for (auto& kv : take) if (kv.second == sub + 1 && active[kv.first]->left == kv.second) done_now.push_back(kv.first);
      if (!done_now.empty()) {
        void* ev; hipEventCreateWithFlags(&ev, 0); hipEventRecord(ev, nullptr);
        for (int id : done_now) finishing.push_back({active[id], ev});
      }
    }
    std::vector<int> gone;
    for (auto& kv : active) if (kv.second->left == take[kv.first]) gone.push_back(kv.first);
    for (int id : gone) active.erase(id);
    for (auto& kv : active) kv.second->left -= take[kv.first];
    std::vector<std::pair<Req*, void*>> still;
    for (auto& f : finishing) {
      if (hipEventQuery(f.second) == 0) {
        idp_dg_destroy(f.first->h); f.first->h = nullptr;
        hipFree(f.first->ws); hipFree(f.first->u); ++done;
      } else still.push_back(f);
    }
    finishing = still;
    if (active.empty() && next >= reqs.size()) {
      for (auto& f : finishing) { hipEventSynchronize(f.second); idp_dg_destroy(f.first->h); hipFree(f.first->ws); hipFree(f.first->u); ++done; }
      finishing.clear();
    }
  }
  for (auto& kv : batches) idp_dg_batch_destroy(kv.second.second);
  hipStreamSynchronize(nullptr);
  printf("served %d requests over %d ticks\n", nreq, tick);

  // 2. plain path
  idp_dg_desc d{}; d.dim = 2; d.nx = 9; d.ny = 7; d.lx = 1; d.ly = 1; d.p = 4;
  d.eq = IDP_DG_EULER; d.gamma = 1.4; d.limiter = IDP_DG_SUBCELL;
  idp_dg* h = nullptr;
  if (idp_dg_create(&d, nullptr, &h)) { fprintf(stderr, "create: %s\n", idp_dg_last_error(nullptr)); return 1; }
  const size_t nb = sizeof(double) * idp_dg_num_comp(h) * idp_dg_num_nodes(h);
  double* u[2];
  hipMalloc((void**)&u[0], nb);
  hipMalloc((void**)&u[1], nb);
  for (int it = 0; it < 200; ++it) {
    const double cfl = (it / 7) % 2 ? 0.5 : 0.4;
    if (idp_dg_step_cfl(h, u[(it / 3) % 2], cfl)) { fprintf(stderr, "step_cfl: %s\n", idp_dg_last_error(h)); return 1; }
    if (it % 50 == 49 && idp_dg_step(h, u[0], 1e-4)) { fprintf(stderr, "step: %s\n", idp_dg_last_error(h)); return 1; }
    // the tile-shape tuner between queued steps: it may retire the cached graph
    if (it % 40 == 20) {
      int shape = -1;
      if (idp_dg_tune(h, u[(it / 3) % 2], cfl, 2, &shape)) { fprintf(stderr, "tune: %s\n", idp_dg_last_error(h)); return 1; }
      if (idp_dg_set_tile_shape(h, (it / 40) % 2)) { fprintf(stderr, "shape: %s\n", idp_dg_last_error(h)); return 1; }
    }
  }
  idp_dg_destroy(h);
  hipFree(u[0]);
  hipFree(u[1]);
  printf("plain path done\n");

  // 3. curved mesh: metric set-up, replaced while steps are queued; the
  // rejected cases leave the handle usable
  d.nx = 5; d.ny = 4; d.p = 3;
  if (idp_dg_create(&d, nullptr, &h)) { fprintf(stderr, "create: %s\n", idp_dg_last_error(nullptr)); return 1; }
  const long nn = idp_dg_num_nodes(h);
  std::vector<double> xy(2 * nn, 0.0);
  if (idp_dg_set_mesh(h, xy.data()) != IDP_DG_EINVAL) { fprintf(stderr, "degenerate mesh accepted\n"); return 1; }
  hipMalloc((void**)&u[0], sizeof(double) * idp_dg_num_comp(h) * nn);
  for (int rep = 0; rep < 3; ++rep) {
    const double amp = 0.01 * (rep + 1);
    for (int e = 0; e < d.nx * d.ny; ++e)
      for (int b = 0; b <= d.p; ++b)
        for (int a = 0; a <= d.p; ++a) {
          const long g = (long)e * (d.p + 1) * (d.p + 1) + b * (d.p + 1) + a;
          const double X = ((e % d.nx) + a / (double)d.p) / d.nx, Y = ((e / d.nx) + b / (double)d.p) / d.ny;
          const double s2 = std::sin(6.283185307179586 * X) * std::sin(6.283185307179586 * Y);
          xy[g] = X + amp * s2;
          xy[nn + g] = Y + amp * s2;
        }
    if (idp_dg_set_mesh(h, xy.data())) { fprintf(stderr, "set_mesh: %s\n", idp_dg_last_error(h)); return 1; }
    for (int it = 0; it < 4; ++it)
      if (idp_dg_step_cfl(h, u[0], 0.4)) { fprintf(stderr, "curved step_cfl: %s\n", idp_dg_last_error(h)); return 1; }
  }
  // a batch holding the curved handle, and the mesh replaced between its
  // unsynchronised steps
  idp_dg_batch* cb = nullptr;
  if (idp_dg_batch_create(&h, 1, nullptr, &cb)) { fprintf(stderr, "curved batch: %s\n", idp_dg_batch_last_error(nullptr)); return 1; }
  for (int it = 0; it < 4; ++it) {
    if (idp_dg_batch_step_cfl(cb, &u[0], 0.4)) { fprintf(stderr, "curved batch step: %s\n", idp_dg_batch_last_error(cb)); return 1; }
    if (it == 1 && idp_dg_set_mesh(h, xy.data())) { fprintf(stderr, "set_mesh: %s\n", idp_dg_last_error(h)); return 1; }
  }
  idp_dg_batch_destroy(cb);
  idp_dg_destroy(h);
  hipFree(u[0]);
  printf("curved path done\n");
  mock_report();
  return 0;
}
