// Shared declarations of the gfx950 stage kernels and the host runtime.
#pragma once
#include <hip/hip_runtime.h>

namespace idp {

// Equation codes of the kernels.  Euler comes in three instantiations:
// generic gamma, and gamma = 1 + 2/n with n = 3 (5/3) or n = 5 (7/5), where
// the fractional powers become integer powers of one inverse root.
// EQ_ADVV is advection by a velocity field beta = (beta_x(y), beta_y(x))
// given per node row and column (2-D only).
enum { EQ_ADV = 0, EQ_BURG = 1, EQ_EULER = 2, EQ_EULER53 = 3, EQ_EULER75 = 4, EQ_ADVV = 5 };
constexpr bool is_euler(int eq) { return eq >= EQ_EULER && eq <= EQ_EULER75; }
constexpr int gn_of(int eq) { return eq == EQ_EULER53 ? 3 : eq == EQ_EULER75 ? 5 : 0; }
enum { LIM_SUBCELL = 0, LIM_TARGET = 1, LIM_LOW = 2, LIM_SUBCELL_SI = 3, LIM_ELEMENTWISE = 4 };
constexpr int MAXP = 8;

// Per-degree constants, passed by value in the kernel arguments.
struct Tables {
  double w[MAXP + 1];             // Gauss-Lobatto weights on [0,1]
  double Q[MAXP * (MAXP + 1)];    // Q[a][e] = sum_{c<=a} D[c][e], a < p; rows of p+1
  double iw[MAXP + 1];            // 1 / w
  double M[(MAXP + 1) * (MAXP + 1)];  // nodal -> Legendre modal: c_k = sum_a M[k][a] u_a
  double nk[MAXP + 1];            // ||P_k||^2 on [-1,1] = 2/(2k+1)
  double s0;                      // smoothness indicator centre log10(p^-4)
};

// Physics constants of one problem.
struct Phys {
  double vel0, vel1;   // advection velocity / Burgers direction
  const double* vrow;  // EQ_ADVV: beta_x of every node row (ny*(p+1), device)
  const double* vcol;  // EQ_ADVV: beta_y of every node column (nx*(p+1), device)
  double gamma;        // Euler
  double g1;           // (gamma-1)/2
  double igm1;         // 1/(gamma-1)
  double fac;          // (gamma+1)/(2 gamma)
  double ex;           // (gamma-1)/(2 gamma)
  double inv_ex;       // 2 gamma/(gamma-1)
  int inv_ex_int;      // inv_ex when it is an integer (7 for gamma = 1.4), else 0
};

// Open boundaries.  Per side (x = 0, x = lx, y = 0, y = ly) the condition
// of every boundary node (node-row order on x-sides, node-column order on
// y-sides, one node per side in 1-D) and the prescribed states [c][node]
// (device arrays, caller-owned).  A face trace on an open side holds the
// exterior state: the prescribed state, the node's own state (outflow), or
// the own state with the normal momentum reversed (slip; outflow for the
// scalar laws).  Other codes, and STATE without a state array, act as
// outflow.
enum { BC_STATE = 1, BC_OUTFLOW = 2, BC_SLIP = 3 };
struct Bnd {
  const signed char* type[4];
  const double* state[4];
  int open;   // bit k set: direction k is open (not periodic)
};

// Diagnostics words in device memory.  Counters are spread over slots
// (indexed by workgroup) so that concurrent workgroups rarely meet on one
// address; the host sums them.
constexpr int DIAG_SLOTS = 1024;
struct Diag {
  unsigned long long limited[DIAG_SLOTS];   // nodes with final alpha < 1
  unsigned long long entropy[DIAG_SLOTS];   // nodes where the entropy search bound alpha
  unsigned int bad_input;                   // rho <= 0 or p <= 0 seen in a stage input
  unsigned int lo_violation;                // u^L outside its bounds (dt above CFL)
};

// Geometry of one solve and where its arrays are.
struct Solve {
  const double* u_n;    // read when use_un
  const double* u_s;    // stage input
  double* u_out;        // stage output
  const double* dt_dev; // when non-null: dt = dt_scale * dt_dev[0]
  double dt, dt_scale;
  long long nn;         // nodes
  int p;                // polynomial degree
  int nx, ny, ne;       // elements
  int ntiles;           // element tiles of this solve
  int ntx;              // tiles per row of tiles
  double hx, hy;
  double ihx, ihy;      // 1/hx, 1/hy
  const double* metric; // curved meshes: per node [q][nn] (q < 4 det(J) J^-1, q < 8 the
                        // corrected terms, q = 8 det(J)); NULL on Cartesian meshes
};

struct StageArgs {
  Solve S;
  Phys ph;
  Tables T;
  double a_s, b_s;
  int use_un;
  int limiter;
  Diag* diag;
  double* trace;   // optional per-node [umin, umax, kmin, alpha_z, alpha] x Nn
  double gmin, gmax;   // global bounds (LIM_SUBCELL_SI)
  Bnd bnd;
};

struct MaxDtArgs {
  const double* u;
  double* partial;           // one minimum per workgroup
  long long nn;
  int p;
  int nx, ny, ne, ntiles;
  int ntx;                   // tiles per row of tiles
  double hx, hy;
  Phys ph;
  Tables T;
  Bnd bnd;
  const double* metric;      // curved meshes (as Solve::metric), else NULL
};

// Batched execution: per degree, a work list of (solve, tile) items over
// every solve of that degree.
struct BatchArgs {
  const StageArgs* args;     // per solve (this stage's pointers and dt)
  const int* item_solve;
  const int* item_tile;
  int nitems;
};
struct BatchDtArgs {
  const MaxDtArgs* args;     // per solve
  const int* item_solve;
  const int* item_tile;
  double* partial;           // one minimum per item
  int nitems;
};
// The work-list kernels of one degree, for building graph nodes.
struct BatchKernels {
  const void* stage;         // __global__ void(BatchArgs)
  const void* maxdt;         // __global__ void(BatchDtArgs)
  int block;                 // threads per workgroup
  int tile_x, tile_y;        // elements per tile in x and y
};

// A graph whose last launch may still run: destroyed only once its event
// has completed (destroying a graph exec that is executing would free
// runtime objects the launch still uses).
struct RetiredGraph {
  hipGraph_t graph;
  hipGraphExec_t exec;
  hipEvent_t done;
};

// Kernel launchers, one translation unit per (equation, dimension).
// Return hipSuccess or the launch error; variant selects elements-per-block.
#define IDP_DECLARE_LAUNCHERS(NAME)                                               \
  hipError_t launch_stage_##NAME(int p, int variant, const StageArgs& a,          \
                                 hipStream_t s);                                  \
  hipError_t launch_maxdt_##NAME(int p, int variant, const MaxDtArgs& a,          \
                                 hipStream_t s);                                  \
  hipError_t launch_stage_curved_##NAME(int p, const StageArgs& a, hipStream_t s); \
  hipError_t launch_maxdt_curved_##NAME(int p, const MaxDtArgs& a, hipStream_t s); \
  void tile_dims_##NAME(int p, int variant, int* tx, int* ty);                    \
  int num_variants_##NAME(int p);                                                 \
  int batch_kernels_##NAME(int p, int variant, BatchKernels* k);                  \
  int batch_kernels_curved_##NAME(int p, BatchKernels* k);

IDP_DECLARE_LAUNCHERS(adv1)
IDP_DECLARE_LAUNCHERS(adv2)
IDP_DECLARE_LAUNCHERS(burg1)
IDP_DECLARE_LAUNCHERS(burg2)
IDP_DECLARE_LAUNCHERS(euler1)
IDP_DECLARE_LAUNCHERS(euler2)
IDP_DECLARE_LAUNCHERS(euler53_1)
IDP_DECLARE_LAUNCHERS(euler53_2)
IDP_DECLARE_LAUNCHERS(euler75_1)
IDP_DECLARE_LAUNCHERS(euler75_2)
IDP_DECLARE_LAUNCHERS(advv2)

// min over partial[b..e) by one thread at stride BS: eight independent loads
// in flight per wait (a single chain waits on every load; large meshes have
// hundreds of thousands of partial minima)
template <int BS>
__device__ inline double strided_min(const double* __restrict__ partial, int b, int e) {
  double v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = INFINITY;
  int i = b + (int)threadIdx.x;
  for (; i + 7 * BS < e; i += 8 * BS) {
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = fmin(v[j], partial[i + j * BS]);
  }
  for (; i < e; i += BS) v[0] = fmin(v[0], partial[i]);
#pragma unroll
  for (int j = 1; j < 8; ++j) v[0] = fmin(v[0], v[j]);
  return v[0];
}

// One step of a wave-wide minimum of doubles by data-parallel-primitive
// lane moves: x = min(x, x of the lane the DPP control CTRL selects), the
// move done on the two 32-bit halves; lanes of rows outside ROWS (and lanes
// whose source is outside the row) keep x.
template <int CTRL, int ROWS>
__device__ inline double dpp_min(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false);
  const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false);
  return fmin(x, __hiloint2double(hi2, lo2));
}

// Minimum over the 64 lanes of a wave, valid in lane 63: quad permutations
// [1,0,3,2] and [2,3,0,1], the half-row and row mirrors (every lane then
// holds the minimum of its row of 16), lane 15 of each row broadcast into
// rows 1 and 3, then lane 31 into rows 2 and 3.
__device__ inline double wave_min63(double x) {
  x = dpp_min<0xB1, 0xF>(x);
  x = dpp_min<0x4E, 0xF>(x);
  x = dpp_min<0x141, 0xF>(x);
  x = dpp_min<0x140, 0xF>(x);
  x = dpp_min<0x142, 0xA>(x);
  x = dpp_min<0x143, 0xC>(x);
  return x;
}

// min over partial[0..n) -> out[0] (one workgroup of 1024 threads)
__global__ void min_reduce_kernel(const double* partial, int n, double* out);
// per solve s: min over partial[range[2s]..range[2s+1]) -> out[s] (one workgroup per solve)
__global__ void segmented_min_kernel(const double* partial, const int* range, double* out);

}  // namespace idp
