/*
 * idp_ref.h -- CPU oracle for one limited SSP-RK stage of the sparse
 * invariant-domain-preserving (IDP) nodal DG method with subcell convex
 * limiting (Pazner, "Sparse invariant domain preserving discontinuous
 * Galerkin methods with subcell convex limiting", arXiv 2004.08503).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, FP64
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Every routine allocates with malloc, works on host pointers and is
 * compiled with -ffp-contract=off (no fused multiply-add).  The loops over
 * nodes and element rows may run on several OpenMP threads
 * (idp_ref_set_threads); every node's arithmetic is the same on any number
 * of threads, so results do not depend on it.
 *
 * Mesh: Cartesian box [0,lx) x [0,ly) split into nx x ny elements (ny = 1
 * in 1-D), periodic in each direction unless that direction is open.  Each element carries the (p+1)^d tensor Gauss-Lobatto
 * nodes.  State layout: u[c][e][b][a], i.e. component c outermost, element
 * e = ey*nx + ex, then the y node index b, then the x node index a fastest.
 * The number of nodes is Nn = nx*ny*(p+1)^d and an array holds nc*Nn
 * doubles, nc = 1 for the scalar laws and d+2 for Euler.
 */
#ifndef IDP_REF_H
#define IDP_REF_H

#ifdef __cplusplus
extern "C" {
#endif

/* ADVECTION_FIELD is u_t + div(beta(x) u) = 0 with a prescribed,
 * divergence-free velocity field given by its nodal values (Sec. 3.3; 2-D
 * only: a divergence-free field in 1-D is constant). */
enum { IDP_REF_ADVECTION = 0, IDP_REF_BURGERS = 1, IDP_REF_EULER = 2,
       IDP_REF_ADVECTION_FIELD = 3 };

/* Conditions of a boundary node of an open direction: the state on the
 * far side of the boundary face (the exterior, or "ghost", state) is a
 * prescribed state (STATE), the node's own state (OUTFLOW), or its own state
 * with the normal momentum reversed (SLIP: a reflecting wall for Euler; the
 * same as OUTFLOW for the scalar laws).  Any other code acts as OUTFLOW. */
enum { IDP_REF_BC_STATE = 1, IDP_REF_BC_OUTFLOW = 2, IDP_REF_BC_SLIP = 3 };

/* Limiter modes: SUBCELL is the subcell convex limiter (Sec. 4.1.3 and
 * 4.2.2); TARGET returns the unlimited high-order update (eq. ho-update);
 * LOW returns the low-order IDP update (eq. lo-update / idp-fe); SUBCELL_SI
 * is SUBCELL with the local bounds of the limited component relaxed towards
 * the global bounds [gmin, gmax] by the subcell-resolution smoothness
 * indicator (Sec. 4.4, eq. relaxed-bounds); ELEMENTWISE limits every node's
 * whole correction u^H_i - u^L_i (Zalesak, then for Euler the entropy line
 * search of eq. convex-provisional-elementwise) and applies the minimum over
 * the element (Sec. 4.1.2 and 4.2.1). */
enum { IDP_REF_SUBCELL = 0, IDP_REF_TARGET = 1, IDP_REF_LOW = 2, IDP_REF_SUBCELL_SI = 3,
       IDP_REF_ELEMENTWISE = 4 };

typedef struct {
  int dim;          /* 1 or 2 */
  int nx, ny;       /* elements per direction (ny = 1 when dim = 1) */
  double lx, ly;    /* box lengths */
  int p;            /* polynomial degree, 1..8 */
  int eq;           /* IDP_REF_ADVECTION / _BURGERS / _EULER */
  double vel[2];    /* advection velocity, or Burgers direction vector v */
  double gamma;     /* ratio of specific heats (Euler) */
  int limiter;      /* IDP_REF_SUBCELL / _TARGET / _LOW / _SUBCELL_SI / _ELEMENTWISE */
  double gmin, gmax; /* global bounds of the limited component (SUBCELL_SI) */
  const double* beta; /* ADVECTION_FIELD: nodal velocity beta[k*Nn + i],
                         k < dim (host, read during each call); the field
                         must satisfy the discrete divergence-free identity
                         sum_j chat_ij . beta_j = 0 at every node (checked,
                         1e-12 relative), which fields with beta_x = beta_x(y)
                         and beta_y = beta_y(x) meet on Cartesian meshes */
  int bc[2];          /* per direction x, y: 0 periodic, 1 open (bc[1] = 0
                         in 1-D) */
  const signed char* bc_type[4]; /* open sides x = 0, x = lx, y = 0, y = ly:
                         the condition of every boundary node, ny*(p+1)
                         (x-sides, node row ey*(p+1) + b) or nx*(p+1)
                         (y-sides, node column ex*(p+1) + a) entries; one
                         entry per side in 1-D */
  const double* bc_state[4];     /* the prescribed states of STATE nodes,
                         [c*n + q] for n boundary nodes (NULL: STATE acts
                         as OUTFLOW) */
  const double* metric; /* curved meshes (2-D, periodic, not a velocity
                         field): per node i, metric[q*Nn + i] with
                         q = 0..3 the metric terms det(J) J^-1 of Sec. 2.3,
                         row-major (row k: reference direction xi_k,
                         column l: physical direction x_l), evaluated
                         freestream-preservingly; q = 4..7 the modified
                         terms det(J) J^-1 + C of Sec. 3.1 (eq.
                         metric-perturbation); q = 8 det(J).  The mapping
                         is from the reference square [0,1]^2.  NULL: the
                         affine Cartesian elements of lx/nx x ly/ny. */
} idp_ref_desc;

/* Optional per-node outputs of one forward-Euler sub-step.  Any pointer may
 * be NULL.  Sizes: nc*Nn for uL and uH; dim*nc*Nn for rH, rL and rbar laid
 * out [k][c][node]; Nn for the rest.  rbar[k][c][i] is the antidiffusive
 * subcell flux at the subcell face on the +e_k side of node i (zero when
 * that face is an element face).  umin/umax bound the limited component
 * (u for scalar laws, rho for Euler); kmin is the Euler entropy bound
 * K_min = min p*rho^-gamma over the stencil; alpha_z is the Zalesak
 * coefficient; alpha is the final nodal provisional coefficient. */
typedef struct {
  double *uL, *uH, *rH, *rL, *rbar;
  double *umin, *umax, *kmin, *alpha_z, *alpha;
} idp_ref_trace;

/* Threads of the node and element loops (n >= 1; OpenMP's default when
 * never called).  Returns the number in use after the call (1 when built
 * without OpenMP). */
int idp_ref_set_threads(int n);

/* Returns 0 on success, -1 on a bad argument. */
int idp_ref_check(const idp_ref_desc* d);
long idp_ref_num_nodes(const idp_ref_desc* d);
int idp_ref_num_comp(const idp_ref_desc* d);

/* O0 tables: Gauss-Lobatto nodes/weights on [0,1] (sum w = 1), the weighted
 * differentiation matrix D[a][c] = w_a phi_c'(xi_a) and the sparsified
 * first-order matrix Dhat, both (p+1)x(p+1) row-major. */
int idp_ref_gl(int p, double* xi, double* w);
int idp_ref_dmat(int p, double* D);
int idp_ref_dhat(int p, double* Dh);

/* Pointwise physics: F[k*nc + c] for k < dim; lambda for the 1-D Riemann
 * problem with left state uL, right state uR along the unit vector n.
 * Both need a state-only flux: -1 / NaN for ADVECTION_FIELD. */
int idp_ref_flux(const idp_ref_desc* d, const double* u, double* F);
double idp_ref_lambda(const idp_ref_desc* d, const double* uL,
                      const double* uR, const double* n);

/* Smoothness factor eps_K in [0, 1] of every element (Sec. 4.4) for the
 * limited component of u (u for scalar laws, rho for Euler): the element's
 * polynomial in the Legendre basis, s_K = log10 of the L2 energy fraction in
 * the modes of degree p in any variable, and eps_K rising from 0 at
 * s_K = s0 - kappa to 1 at s0 + kappa, s0 = log10(p^-4), kappa = 1.
 * eps has nx*ny entries.  Returns 0, or -1 on a bad argument. */
int idp_ref_smoothness(const idp_ref_desc* d, const double* u, double* eps);

/* One forward-Euler sub-step out = FE(u, dt) with the limiter mode of d. */
int idp_ref_fe(const idp_ref_desc* d, const double* u, double* out,
               double dt, idp_ref_trace* tr);

/* One SSP-RK3 stage (Shu-Osher form): out = a_s*u_n + b_s*FE(u_s, dt) with
 * (a_s, b_s) = (0,1), (3/4,1/4), (1/3,2/3) for stage = 0, 1, 2.  u_n may be
 * NULL for stage 0.  out may alias u_n but not u_s. */
int idp_ref_stage(const idp_ref_desc* d, const double* u_n, const double* u_s,
                  double* out, double dt, int stage);

/* Three stages in place. */
int idp_ref_step(const idp_ref_desc* d, double* u, double dt);

/* Largest dt allowed by the low-order CFL condition (eq. cfl-low):
 * min_i m_i / (2 sum_{j != i} dhat_ij).  +inf when no dissipation. */
int idp_ref_max_dt(const idp_ref_desc* d, const double* u, double* dt);

#ifdef __cplusplus
}
#endif
#endif
