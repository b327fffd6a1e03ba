// Private host-side definitions shared by the translation units of the
// runtime (plain and batched paths).
#pragma once
#include <rocprofiler-sdk-roctx/roctx.h>
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/idp_dg.h"
#include "common.hpp"

using idp::Tables;
using idp::Phys;
using idp::Diag;

struct idp_dg {
  idp_dg_desc d{};
  hipStream_t stream = nullptr;
  int device = 0;
  int nc = 1;
  long long nn = 0;
  int ne = 0;
  int variant = 0;
  int kcode = 0;   // kernel equation code (EQ_*), Euler split by gamma
  Tables T{};
  Phys ph{};
  double* buf1 = nullptr;   // stage buffers of idp_dg_step
  double* buf2 = nullptr;
  Diag* diag = nullptr;
  double* dtdev = nullptr;     // [0] bound of the last step_cfl, [1] of max_dt
  double* partial = nullptr;   // per-workgroup minima of the time-step kernel
  double* vel = nullptr;       // IDP_DG_ADVECTION_FIELD: row then column velocities
  double* metric = nullptr;    // curved meshes (idp_dg_set_mesh): [9][nn] metric terms
  unsigned mesh_version = 0;   // bumped by every idp_dg_set_mesh
  idp::Bnd bnd{};              // open sides: per-node conditions (idp_dg_set_boundary)
  unsigned bnd_version = 0;    // bumped by every idp_dg_set_boundary
  // cached graph of one device-timestepped step
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t g_done = nullptr;   // recorded after every launch of exec
  double* g_u = nullptr;
  double g_cfl = 0.0;
  std::vector<idp::RetiredGraph> retired;
  bool owns = true;             // device buffers allocated by the handle (not a workspace)
  std::string err = "no error";
};


namespace idp_host {
// A roctx range over one C-ABI call (visible to rocprofv3 --marker-trace;
// a few tens of nanoseconds when no tool is attached).
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};
int family(const idp_dg* h);
int tile_elems(const idp_dg* h);
void tile_dims(const idp_dg* h, int* tx, int* ty);
// tiles of the handle's mesh; *ntx receives the tiles per row of tiles
int tiles_of(const idp_dg* h, int* ntx);
idp::StageArgs make_stage_args(const idp_dg* h, const double* u_n, const double* u_s, double* u_out,
                               double dt, const double* dt_dev, double dt_scale, int stage);
idp::MaxDtArgs make_dt_args(const idp_dg* h, const double* u);
int fail(idp_dg* h, int code, const std::string& msg);
// Gauss-Lobatto weights on [0,1] and the plain derivative matrix
// Dn[i*(p+1)+j] = l_j'(xi_i) of the Lagrange basis on those points
void gl_derivative(int p, double* w01, double* Dn);
void drop_graph(idp_dg* h);
bool desc_ok(const idp_dg_desc* d, std::string* why);
void init_host(idp_dg* h, const idp_dg_desc* desc, void* hip_stream);
hipError_t launch_stage(const idp_dg* h, const idp::StageArgs& a, hipStream_t s);
// Every side of an open direction has its conditions.
bool bnd_ready(const idp_dg* h);
// the work-list kernels of family fam, degree p, tile shape `variant`
int batch_kernels(int fam, int p, int variant, idp::BatchKernels* k);
// the curved-mesh work-list kernels of family fam and degree p (first tile shape)
int batch_kernels_curved(int fam, int p, idp::BatchKernels* k);
// tile shapes compiled per degree
constexpr int kNumVariants = 2;
// Retire (graph, exec, event) and destroy retired graphs whose launches
// have completed; with wait, block until all have completed.
void retire_graph(std::vector<idp::RetiredGraph>* list, hipGraph_t* g, hipGraphExec_t* e, hipEvent_t* ev);
void reap_graphs(std::vector<idp::RetiredGraph>* list, bool wait);
}  // namespace idp_host
