/*
 * idp_dg.h -- C ABI of the MI355X (gfx950) library for one explicit,
 * limited SSP Runge-Kutta stage of the sparse invariant-domain-preserving
 * (IDP) nodal discontinuous Galerkin method with subcell convex limiting of
 * Pazner, "Sparse invariant domain preserving discontinuous Galerkin
 * methods with subcell convex limiting" (arXiv 2004.08503).
 *
 * One stage computes, for every node i of a Cartesian mesh of tensor-product
 * Gauss-Lobatto elements (periodic, or with open sides, see
 * idp_dg_set_boundary):
 *   - the high-order target residual r^H: the strong-form DG spectral
 *     element operator with the local Lax-Friedrichs flux (Sec. 2,
 *     eq. dg-strong, eq. ho-update);
 *   - the sparse low-order residual r^L with graph viscosity (Sec. 3,
 *     eq. dg-idp, eq. lo-update) and the low-order state u^L;
 *   - the antidiffusive subcell fluxes rbar on the interior subcell faces of
 *     each line of nodes (Sec. 4.1.3);
 *   - the local bounds from the bar states (eq. bar-states) and the nodal
 *     limiting coefficients: Zalesak for scalar laws and for the Euler
 *     density, then the entropy line search of eq. convex-provisional;
 *   - the flux-corrected update (eq. convex-fct) combined into the SSP-RK3
 *     stage.
 *
 * Conventions shared by every call:
 *   - Arithmetic is IEEE binary64 throughout.
 *   - A state is a device array of nc * Nn doubles in structure-of-arrays
 *     layout u[c][e][b][a]: component c outermost, element e = ey*nx + ex,
 *     node index b in y, node index a in x fastest.  nc = 1 (advection,
 *     Burgers) or d+2 (Euler: rho, rho v, rho E).  Nn = nx*ny*(p+1)^d.
 *   - Device pointers are caller-owned; the library never frees them.
 *   - Work is enqueued asynchronously on the HIP stream given at creation
 *     (borrowed, not owned); of the calls on a created handle only
 *     idp_dg_max_dt, idp_dg_last_dt, idp_dg_diagnostics and idp_dg_tune
 *     synchronise that stream, and idp_dg_set_mesh the whole device.
 *   - A batch (below) steps its handles on the batch's stream, in the
 *     handles' own stage buffers: while such work is queued, the caller
 *     orders any other work on those handles after it (stream events or
 *     a synchronisation).
 *   - Return codes: 0 success; IDP_DG_EINVAL (-1) bad argument, state left
 *     untouched; IDP_DG_ENOMEM (-2) allocation failure; IDP_DG_EHIP (-3) a
 *     HIP runtime error.  No call aborts or throws; idp_dg_last_error gives
 *     a message for the last failure on a handle.
 *   - A handle is used from one host thread at a time.
 */
#ifndef IDP_DG_H
#define IDP_DG_H

#ifdef __cplusplus
extern "C" {
#endif

#define IDP_DG_EINVAL (-1)
#define IDP_DG_ENOMEM (-2)
#define IDP_DG_EHIP (-3)

/* equations (Sec. 2, Sec. 4.3 for Euler, Sec. 5 for the scalar tests) */
enum {
  IDP_DG_ADVECTION = 0, /* u_t + div(v u) = 0, constant v = velocity */
  IDP_DG_BURGERS = 1,   /* u_t + div(u^2/2 v) = 0, constant direction v */
  IDP_DG_EULER = 2,     /* compressible Euler, ideal gas with gamma */
  IDP_DG_ADVECTION_FIELD = 3 /* u_t + div(beta(x) u) = 0 with a prescribed
                             velocity field (Sec. 3.3: modified bar states
                             and graph viscosity dhat_ij = max(|chat_ij .
                             beta_i|, |chat_ji . beta_j|)); dim = 2, and the
                             field has the form beta = (beta_x(y), beta_y(x))
                             (desc.vel_rows, desc.vel_cols), which satisfies
                             the discrete divergence-free identity sum_j
                             chat_ij . beta_j = 0 the method needs on
                             Cartesian meshes; the solid-body rotation
                             field is of this form */
};

/* limiter modes */
enum {
  IDP_DG_SUBCELL = 0,     /* subcell convex limiting (Sec. 4.1.3, 4.2.2) */
  IDP_DG_TARGET_ONLY = 1, /* alpha = 1: the unlimited high-order update */
  IDP_DG_LOW_ONLY = 2,    /* alpha = 0: the low-order IDP update */
  IDP_DG_SUBCELL_SI = 3,  /* SUBCELL with the local bounds of the limited
                             component (u, or rho for Euler) relaxed by the
                             subcell-resolution smoothness indicator towards
                             the global bounds [gmin, gmax] (Sec. 4.4,
                             eq. relaxed-bounds): per element, s_K = log10
                             of the L2 energy fraction of the degree-p
                             Legendre modes (any variable), eps_K rising on
                             1/2 + 1/2 sin(pi (s_K - s0)/2) from 0 at
                             s0 - 1 to 1 at s0 + 1, s0 = log10(p^-4); p = 1
                             keeps the strict bounds */
  IDP_DG_ELEMENTWISE = 4  /* elementwise limiting (Sec. 4.1.2 and the convex
                             counterpart, eq. convex-provisional-elementwise):
                             every node limits its whole correction
                             u^H_i - u^L_i (Zalesak, then the Euler entropy
                             line search), and each element applies the
                             minimum over its nodes, u = u^L + alpha_K
                             (u^H - u^L) */
};

/* Boundaries, per direction (desc.bc): periodic, or open with per-node
 * conditions on its two sides given by idp_dg_set_boundary. */
enum { IDP_DG_BC_PERIODIC = 0, IDP_DG_BC_OPEN = 1 };

/* Condition of a boundary node on an open side: the state on the far side
 * of the boundary face (the exterior state, which enters the
 * Lax-Friedrichs flux, the graph viscosity, the bar states and the local
 * bounds like a neighbour's) is a prescribed state (STATE), the node's own
 * state (OUTFLOW), or its own state with the normal momentum reversed
 * (SLIP, a reflecting wall; for the scalar laws the same as OUTFLOW).  Any
 * other code, and STATE on a side given no state array, act as OUTFLOW.
 * The paper leaves the boundary treatment open; the low-order update stays
 * a convex combination of admissible bar states when the exterior states
 * are admissible. */
enum { IDP_DG_BC_STATE = 1, IDP_DG_BC_OUTFLOW = 2, IDP_DG_BC_SLIP = 3 };

/* Problem description.  Box [0,lx) x [0,ly) of nx x ny elements
 * (ny = 1 and ly ignored when dim = 1); p in [1, 8]; velocity is the
 * advection velocity or the Burgers direction vector; gamma in (1, 5/3]
 * for Euler (the range where the wave-speed bound used is proven).
 * For IDP_DG_ADVECTION_FIELD, vel_rows and vel_cols are host arrays read
 * (and copied to the device) during idp_dg_create / idp_dg_create_in only:
 * vel_rows[ey*(p+1) + b] = beta_x on the node row y = (ey + xi_b) hy and
 * vel_cols[ex*(p+1) + a] = beta_y on the node column x = (ex + xi_a) hx,
 * xi the Gauss-Lobatto points on [0,1]; ny*(p+1) and nx*(p+1) finite
 * doubles.  Other equations ignore them (NULL is fine). */
typedef struct {
  int dim;
  int nx, ny;
  double lx, ly;
  int p;
  int eq;
  double velocity[2];
  double gamma;
  int limiter;
  double gmin, gmax;  /* global bounds of the limited component, used by
                         IDP_DG_SUBCELL_SI (finite, gmin <= gmax) */
  const double* vel_rows; /* IDP_DG_ADVECTION_FIELD: beta_x per node row */
  const double* vel_cols; /* IDP_DG_ADVECTION_FIELD: beta_y per node column */
  int bc[2];              /* x, y: IDP_DG_BC_PERIODIC or IDP_DG_BC_OPEN
                             (bc[1] periodic when dim = 1) */
} idp_dg_desc;

typedef struct idp_dg idp_dg;

/* Diagnostics accumulated since the last idp_dg_diagnostics call. */
typedef struct {
  long long limited_nodes;  /* nodes whose final coefficient was < 1 */
  long long entropy_nodes;  /* Euler nodes where the entropy search bound */
  int bad_input;            /* a stage input had rho <= 0 or p <= 0 */
  int low_order_violation;  /* u^L left its bounds: dt above the CFL bound */
} idp_dg_diag;

/* Create a handle for one problem.  Builds the Gauss-Lobatto tables, picks
 * the launch configuration and allocates two state-sized device buffers
 * for idp_dg_step.  hip_stream is a hipStream_t (0 for the null stream).
 * *out receives the handle, or NULL on failure. */
int idp_dg_create(const idp_dg_desc* desc, void* hip_stream, idp_dg** out);

/* Device bytes idp_dg_create_in needs for desc: the two stage buffers,
 * the diagnostics and the time-step partial minima.  Negative
 * (IDP_DG_EINVAL) for a bad desc. */
long long idp_dg_workspace_bytes(const idp_dg_desc* desc);

/* idp_dg_create with every device buffer of the handle placed in the
 * caller's workspace (device memory of at least idp_dg_workspace_bytes
 * bytes, 256-byte aligned, caller-owned, kept alive until idp_dg_destroy
 * has returned and the handle's queued work has run).  The handle then
 * allocates and frees no device memory, so a caller that creates and drops
 * many handles (a serving loop) can take the memory from its own
 * stream-ordered allocator.  The diagnostics are cleared with an
 * asynchronous memset on hip_stream. */
int idp_dg_create_in(const idp_dg_desc* desc, void* hip_stream,
                     void* workspace, long long bytes, idp_dg** out);

/* Conditions of one side of an open direction: side 0 (x = 0), 1 (x = lx),
 * 2 (y = 0), 3 (y = ly).  type holds one IDP_DG_BC_* code per boundary node
 * and state (NULL allowed) the prescribed states [c][node] of STATE nodes;
 * boundary nodes are ordered by node row ey*(p+1) + b on x-sides (ny*(p+1)
 * of them) and by node column ex*(p+1) + a on y-sides (nx*(p+1)); one node
 * per side in 1-D.  Both are device arrays, borrowed: every later launch
 * on the handle reads them, so the caller may rewrite their contents
 * between launches (time-dependent data) and keeps them alive while work
 * that reads them is queued.  Every side of an open direction must be set
 * before the handle steps (IDP_DG_EINVAL otherwise).  New pointers drop
 * the handle's captured idp_dg_step_cfl graph; a batch holding the handle
 * picks them up at its next step.  IDP_DG_EINVAL for a bad side, a
 * periodic direction or a NULL type. */
int idp_dg_set_boundary(idp_dg* h, int side, const signed char* type, const double* state);

/* Curved mesh (Sec. 2.3 isoparametric elements, Sec. 3.1 conservative
 * correction): coords is a host array [2][Nn] of the physical node
 * coordinates (x then y, state order u[c][e][b][a]), read during the call
 * only.  Each element is the image of the reference square under the
 * polynomial interpolant of its nodes; neighbouring elements must agree on
 * their shared face nodes up to the periodic shift (not checked).  From
 * them the call computes, per node, the metric terms det(J) J^-1 of the
 * high-order operator (rows xi, eta = (y_eta, -x_eta), (-y_xi, x_xi), the
 * derivatives by the Gauss-Lobatto derivative matrix along node lines),
 * det(J), and the corrected terms of the low-order operator: per element
 * and physical direction the minimum-norm solution C of eq.
 * metric-perturbation, added to the high-order terms.  They are uploaded to
 * a device array of 9 Nn doubles that the handle allocates (hipMalloc) and
 * frees at idp_dg_destroy; every later stage and time-step launch uses the
 * curved operators (one tile shape; idp_dg_set_tile_shape has no effect).
 * A second call replaces the mesh in place.  Waits for all work queued on
 * the device (a batch holding the handle may run on another stream).
 * IDP_DG_EINVAL: NULL coords, a non-2-D problem, an advection field, an open
 * direction (curved meshes are periodic), a handle created in a caller
 * workspace (which must not allocate), or a node with det(J) not positive
 * or a non-finite coordinate.  A batch may mix curved and Cartesian
 * solves (its curved members step with the curved work-list kernels); a
 * member given a new mesh after joining is picked up at the batch's next
 * step. */
int idp_dg_set_mesh(idp_dg* h, const double* coords);

/* The metric array idp_dg_set_mesh computes, written to the host array
 * metric (9 * Nn doubles, caller-owned): metric[q * Nn + node] with
 * q = 0..3 the high-order terms det(J) J^-1 (rows xi, eta; columns x, y),
 * q = 4..7 the corrected terms (eq. metric-perturbation), q = 8 det(J).
 * Host only: no device, no handle.  coords as for idp_dg_set_mesh.
 * IDP_DG_EINVAL for a bad desc, a desc a curved mesh does not support, NULL
 * arrays or a mesh idp_dg_set_mesh would refuse (idp_dg_last_error(NULL)
 * gives the message; metric is then partly written). */
int idp_dg_mesh_metric(const idp_dg_desc* desc, const double* coords, double* metric);

/* Release the handle and the buffers it allocated.  NULL-safe. */
void idp_dg_destroy(idp_dg* h);

/* Number of nodes Nn and of components nc of the handle's problem. */
long idp_dg_num_nodes(const idp_dg* h);
int idp_dg_num_comp(const idp_dg* h);

/* One SSP-RK3 stage in Shu-Osher form (Sec. 5: third-order SSP RK):
 *   u_out = a_s * u_n + b_s * FE(u_s, dt),
 *   (a_s, b_s) = (0, 1), (3/4, 1/4), (1/3, 2/3) for stage = 0, 1, 2,
 * FE the limited forward-Euler sub-step.  u_n is not read for stage 0 and
 * may then be NULL.  u_out may equal u_n but must not overlap u_s
 * (neighbouring elements read u_s).  dt >= 0; dt above idp_dg_max_dt
 * loses the IDP guarantee and is reported by the diagnostics. */
int idp_dg_stage(idp_dg* h, const double* u_n, const double* u_s,
                 double* u_out, double dt, int stage);

/* idp_dg_stage that also writes the limiter's per-node intermediates to
 * the device array trace (5 * Nn doubles, caller-owned, not overlapping a
 * state): trace[0..Nn) the lower bound and [Nn..2Nn) the upper bound of
 * the limited component (u, or rho for Euler; eq. bar-states), [2Nn..3Nn)
 * the Euler entropy bound K_min = min p rho^-gamma over the stencil (0 for
 * scalar laws), [3Nn..4Nn) the Zalesak coefficient and [4Nn..5Nn) the
 * final nodal coefficient (eq. convex-provisional).  For inspection and
 * testing of the limiter; the state update is the same as idp_dg_stage. */
int idp_dg_stage_trace(idp_dg* h, const double* u_n, const double* u_s,
                       double* u_out, double dt, int stage, double* trace);

/* One SSP-RK3 step in place: three stages through the handle's buffers. */
int idp_dg_step(idp_dg* h, double* u, double dt);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the step
 * of idp_dg_step without a handle.  Nothing is allocated, here or earlier.
 * The two stage buffers are one static device array of the library
 * (2 * IDP_DG_NOALLOC_MAX_DOUBLES doubles = 64 MiB), present on every GPU
 * the library runs on until the process ends; the first call on a device
 * only looks up that array's address there.
 *   - desc: as for idp_dg_create; periodic directions only (bc = 0) and
 *     any equation but IDP_DG_ADVECTION_FIELD, else IDP_DG_EINVAL;
 *     nc * Nn <= IDP_DG_NOALLOC_MAX_DOUBLES, else IDP_DG_EINVAL with a
 *     message giving both sizes;
 *   - u: device state (layout as for idp_dg_stage), updated in place by
 *     dt >= 0 on hip_stream (a hipStream_t, 0 for the null stream) of the
 *     current device; asynchronous;
 *   - the result is bitwise that of idp_dg_step on a handle of desc (the
 *     same kernels); no diagnostics are counted;
 *   - every call on one GPU shares the array: calls whose work may overlap
 *     on one GPU (other streams, other host threads) race and must be
 *     ordered by the caller.
 * Errors: idp_dg_last_error(NULL) gives the message. */
#define IDP_DG_NOALLOC_MAX_DOUBLES (4LL << 20)
int idp_dg_step_noalloc(const idp_dg_desc* desc, double* u, double dt, void* hip_stream);

/* One SSP-RK3 step in place with dt = cfl * idp_dg_max_dt(u) computed on
 * the device from u at the start of the step (eq. cfl-low; the paper runs
 * cfl = 1/2).  Nothing is copied to the host: the four kernels replay from
 * a HIP graph cached for (u, cfl).  The dt used is kept on the device and
 * can be read with idp_dg_last_dt. */
int idp_dg_step_cfl(idp_dg* h, double* u, double cfl);

/* dt of the last idp_dg_step_cfl (synchronises the stream). */
int idp_dg_last_dt(idp_dg* h, double* dt);

/* Largest dt allowed by the low-order CFL condition (eq. cfl-low):
 * min over nodes of m_i / (2 sum_{j != i} dhat_ij), written to *dt (host).
 * +inf when no node has dissipation.  Synchronises the stream. */
int idp_dg_max_dt(idp_dg* h, const double* u, double* dt);

/* The low-order CFL bound of idp_dg_max_dt written to device memory
 * (dt_dev: one caller-owned double, 8-byte aligned) without synchronising:
 * for callers that keep the whole step on the device or capture it in a
 * graph. */
int idp_dg_max_dt_async(idp_dg* h, const double* u, double* dt_dev);

/* idp_dg_stage with dt = cfl * dt_dev[0] read on the device (dt_dev as
 * written by idp_dg_max_dt_async; cfl > 0).  A bound of +inf (no
 * dissipation anywhere) is taken as dt = 0. */
int idp_dg_stage_dt(idp_dg* h, const double* u_n, const double* u_s,
                    double* u_out, const double* dt_dev, double cfl, int stage);

/* Tile-shape autotuning.  The stage and time-step kernels are compiled
 * for IDP_DG_NUM_TILE_SHAPES tile shapes per degree: a workgroup owns a
 * tile of tx x ty elements (tx in 1-D) and evaluates every subcell face of
 * the tile once.  A new handle uses shape 0.  Every shape gives bitwise the
 * same results: a face's and a node's arithmetic does not depend on which
 * tile, workgroup or launch runs it.
 *
 * idp_dg_tune times `reps` (1..100) device-timestepped SSP-RK3 steps (as
 * idp_dg_step_cfl; cfl > 0) of the device state u under each shape, the
 * shapes taking turns twice, and moves to another shape only if it is at
 * least 2 % faster than the current one; the shape kept is written to
 * *shape (may be NULL).  u is only read: the timed steps write the
 * handle's own stage buffers and a spare time-step slot (idp_dg_last_dt is
 * unchanged).  Enqueued on the handle's stream after its earlier work;
 * synchronises that stream.  A cached idp_dg_step_cfl graph is rebuilt on
 * its next call if the shape changed.  Returns 0, IDP_DG_EINVAL (NULL u,
 * bad cfl or reps, u overlapping the handle's buffers, an open side
 * without conditions) or IDP_DG_EHIP.  On a curved mesh (idp_dg_set_mesh),
 * which runs the first shape whatever the setting, it times nothing and
 * reports the current setting.
 *
 * idp_dg_tile_shape: the current shape (-1 for NULL).
 * idp_dg_set_tile_shape: 0 <= shape < IDP_DG_NUM_TILE_SHAPES, else
 * IDP_DG_EINVAL. */
#define IDP_DG_NUM_TILE_SHAPES 2
int idp_dg_tune(idp_dg* h, const double* u, double cfl, int reps, int* shape);
int idp_dg_tile_shape(const idp_dg* h);
/* Elements per workgroup of the current tile shape (-1 for NULL). */
int idp_dg_tile_elems(const idp_dg* h);
/* The current tile shape's elements per tile in x (*tx) and y (*ty; 1 in
 * 1-D).  Returns 0, or IDP_DG_EINVAL for a NULL argument. */
int idp_dg_tile_dims(const idp_dg* h, int* tx, int* ty);
int idp_dg_set_tile_shape(idp_dg* h, int shape);

/* Copy out and reset the diagnostics (synchronises the stream). */
int idp_dg_diagnostics(idp_dg* h, idp_dg_diag* out);

/* Message of the last failure on h (or of the last failed create when h is
 * NULL).  Never NULL. */
const char* idp_dg_last_error(const idp_dg* h);

/* Provenance: the first 16 hex digits of the SHA-256 of the sources this
 * library was built from (every file of its source directory and this
 * header, in name order), or "unknown" for a build that did not set it.
 * Static string, never NULL. */
const char* idp_dg_build_hash(void);

/* ------------------------------------------------------------------ */
/* Batched execution: many independent solves of uneven mesh size and  */
/* degree advance together.  Per degree present, one work-list launch  */
/* per RK stage covers the element tiles of all solves of that degree; */
/* the launches of a step go directly to the batch's stream.          */
/* ------------------------------------------------------------------ */

typedef struct idp_dg_batch idp_dg_batch;

/* Group n >= 1 distinct handles for batched stepping on hip_stream.  The
 * handles are borrowed (they must outlive the batch) and must share the
 * equation, dimension, gamma kind (7/5, 5/3 or other) and device; mesh
 * size, p, limiter mode and velocity may differ.  Each solve keeps using
 * its handle's stage buffers and diagnostics. */
int idp_dg_batch_create(idp_dg* const* solves, int n, void* hip_stream,
                        idp_dg_batch** out);
void idp_dg_batch_destroy(idp_dg_batch* b);

/* Replace the batch's solves by solves[0..n) (same rules as for create),
 * keeping its device storage: for a serving loop whose set of running
 * solves changes from step to step.  Takes effect at the next step; work
 * already enqueued is unaffected. */
int idp_dg_batch_update(idp_dg_batch* b, idp_dg* const* solves, int n);

/* Work items (element tiles over all solves) of the current membership. */
int idp_dg_batch_num_items(const idp_dg_batch* b);

/* One SSP-RK3 step of every solve i: u[i] (device, in place, layout as for
 * idp_dg_stage) advanced by dt[i] (host array of n values >= 0).  The
 * result of each solve is bitwise identical to idp_dg_step on its own.
 * States must not overlap each other or any solve's stage buffers. */
int idp_dg_batch_step(idp_dg_batch* b, double* const* u, const double* dt);

/* One step of every solve with dt_i = cfl * (CFL bound of u[i]) computed
 * on the device (no host synchronisation).  Bitwise identical to
 * idp_dg_step_cfl per solve. */
int idp_dg_batch_step_cfl(idp_dg_batch* b, double* const* u, double cfl);

/* Tile shape per degree for the batch: each degree's work-list kernels
 * take the tile shape of its member with the most nodes after idp_dg_tune
 * on that member's state u[i] (states only read; n device pointers as for
 * the steps), with `reps` steps per shape.  Results are unchanged; the
 * batch re-plans its work lists before its next step.  Synchronises the
 * batch's stream. */
int idp_dg_batch_tune(idp_dg_batch* b, double* const* u, double cfl, int reps);

/* The n time steps used by the last idp_dg_batch_step_cfl (host array;
 * synchronises the stream). */
int idp_dg_batch_last_dt(idp_dg_batch* b, double* dt);

/* Message of the last failure on b (or of the last failed batch create
 * when b is NULL).  Never NULL. */
const char* idp_dg_batch_last_error(const idp_dg_batch* b);

#ifdef __cplusplus
}
#endif
#endif
