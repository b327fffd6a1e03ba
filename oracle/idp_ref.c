/*
 * idp_ref.c -- CPU oracle (TEST INFRASTRUCTURE ONLY) for one limited SSP-RK
 * stage of the sparse IDP nodal DG method with subcell convex limiting
 * (Pazner, arXiv 2004.08503).  Plain FP64 loops over elements, lines and
 * nodes, in the order the paper states the method:
 *
 *   O0 tables          Sec. 2.1-2.2 (Gauss-Lobatto basis, eq. P1/P2),
 *                      Sec. 3 (eq. didp)
 *   O1 pointwise flux  eq. cons-law, eq. euler-eos / euler-flux; for a
 *                      velocity field the nodal flux beta_i u_i (Sec. 3.3)
 *   O2 wave speeds     eq. riemann-problem, eq. lax-friedrichs
 *   O3/O4 residuals    eq. ho-update (strong form, eq. dg-strong) and
 *                      eq. lo-update (weak form with Dhat + graph viscosity,
 *                      eq. dij), split per direction (Prop. line-zero-sum)
 *   O5 low-order state eq. lo-update
 *   O6 subcell fluxes  Sec. 4.1.3 (rbar as sums of nodal antidiffusive
 *                      fluxes on one side of a subcell face)
 *   O7 bounds          eq. bar-states, Sec. 4.1.1, Sec. 4.3 (Euler); the
 *                      modified bar states of Sec. 3.3 for a velocity field
 *   O8 Zalesak         Sec. 4.1.2-4.1.3
 *   O9 entropy search  eq. convex-provisional, Sec. 4.3
 *   O10 update         eq. subcell-fct / convex-fct
 *   time step          eq. cfl-low, SSP-RK3 (Shu-Osher form)
 *
 * Built with -ffp-contract=off.  Readings of places where the paper is
 * silent or garbled are marked "reading:" in the comments.
 */
#include "idp_ref.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXP 8
#define MAXN (MAXP + 1)
#define MAXC 4

typedef struct {
  idp_ref_desc d;
  int nc, n1, np;   /* components, nodes per line, nodes per element */
  long ne, nn;      /* elements, nodes */
  double hx, hy;    /* element sizes */
  double xi[MAXN], w[MAXN];
  double D[MAXN * MAXN], Dh[MAXN * MAXN];
} ref_t;

/* ------------------------------------------------------------------ */
/* argument checks                                                     */
/* ------------------------------------------------------------------ */

static int field_check(const idp_ref_desc* d);

int idp_ref_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

int idp_ref_check(const idp_ref_desc* d) {
  if (!d) return -1;
  if (d->dim != 1 && d->dim != 2) return -1;
  if (d->nx < 1 || d->ny < 1) return -1;
  if (d->dim == 1 && d->ny != 1) return -1;
  if (!(d->lx > 0.0) || (d->dim == 2 && !(d->ly > 0.0))) return -1;
  if (d->p < 1 || d->p > MAXP) return -1;
  if (d->eq < IDP_REF_ADVECTION || d->eq > IDP_REF_ADVECTION_FIELD) return -1;
  if (d->limiter < IDP_REF_SUBCELL || d->limiter > IDP_REF_ELEMENTWISE) return -1;
  if (d->limiter == IDP_REF_SUBCELL_SI && !(d->gmin <= d->gmax && isfinite(d->gmin) && isfinite(d->gmax)))
    return -1;
  /* the two-rarefaction wave-speed bound holds for 1 < gamma <= 5/3 */
  if (d->eq == IDP_REF_EULER && !(d->gamma > 1.0 && d->gamma <= 5.0 / 3.0))
    return -1;
  if (d->eq == IDP_REF_ADVECTION_FIELD && field_check(d)) return -1;
  for (int k = 0; k < 2; ++k) {
    if (d->bc[k] != 0 && d->bc[k] != 1) return -1;
    if (d->bc[k] && (!d->bc_type[2 * k] || !d->bc_type[2 * k + 1])) return -1;
  }
  if (d->dim == 1 && d->bc[1]) return -1;
  if (d->metric) {
    /* curved meshes: 2-D, periodic, flux F(u) (not a velocity field) */
    if (d->dim != 2 || d->eq == IDP_REF_ADVECTION_FIELD || d->bc[0] || d->bc[1]) return -1;
    long nn = idp_ref_num_nodes(d);
    for (long q = 0; q < 9 * nn; ++q)
      if (!isfinite(d->metric[q])) return -1;
    for (long i = 0; i < nn; ++i)
      if (!(d->metric[8 * nn + i] > 0.0)) return -1;
  }
  return 0;
}

int idp_ref_num_comp(const idp_ref_desc* d) {
  return d->eq == IDP_REF_EULER ? d->dim + 2 : 1;
}

long idp_ref_num_nodes(const idp_ref_desc* d) {
  long n1 = d->p + 1;
  long np = d->dim == 2 ? n1 * n1 : n1;
  return (long)d->nx * (long)d->ny * np;
}

/* ------------------------------------------------------------------ */
/* O0: tables                                                          */
/* ------------------------------------------------------------------ */

/* Legendre polynomial P_n and its first two derivatives at x, from the
 * three-term recurrence (k+1)P_{k+1} = (2k+1) x P_k - k P_{k-1} and the
 * identities P'_{k+1} = P'_{k-1} + (2k+1) P_k, P''_{k+1} = P''_{k-1} +
 * (2k+1) P'_k. */
static void legendre(int n, double x, double* P, double* dP, double* d2P) {
  double p0 = 1.0, p1 = x, q0 = 0.0, q1 = 1.0, s0 = 0.0, s1 = 0.0;
  if (n == 0) {
    *P = 1.0; *dP = 0.0; *d2P = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    double q2 = q0 + (2.0 * k + 1.0) * p1;
    double s2 = s0 + (2.0 * k + 1.0) * q1;
    p0 = p1; p1 = p2;
    q0 = q1; q1 = q2;
    s0 = s1; s1 = s2;
  }
  *P = p1; *dP = q1; *d2P = s1;
}

/* Gauss-Lobatto points of degree p on [0,1]: the end points and the roots
 * of P_p' (Sec. 2.1), found by Newton's method from the Chebyshev-Lobatto
 * points.  Weights: w = 1/(p(p+1) P_p(x)^2) on [0,1] (half the classical
 * weights on [-1,1]). */
int idp_ref_gl(int p, double* xi, double* w) {
  if (p < 1 || p > MAXP || !xi || !w) return -1;
  double x[MAXN];
  x[0] = -1.0;
  x[p] = 1.0;
  for (int k = 1; k < p; ++k) {
    double t = -cos(M_PI * k / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP, d2P;
      legendre(p, t, &P, &dP, &d2P);
      double dx = dP / d2P;
      t -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    x[k] = t;
  }
  for (int k = 0; k <= p; ++k) {
    double P, dP, d2P;
    legendre(p, x[k], &P, &dP, &d2P);
    xi[k] = 0.5 * (x[k] + 1.0);
    w[k] = 1.0 / (p * (p + 1.0) * P * P);
  }
  xi[0] = 0.0;
  xi[p] = 1.0;
  return 0;
}

/* Weighted differentiation matrix (Sec. 2.2): D[a][c] = w_a phi_c'(xi_a),
 * phi_c the Lagrange polynomial through the Gauss-Lobatto points, its
 * derivative written out from the product form. */
int idp_ref_dmat(int p, double* D) {
  double xi[MAXN], w[MAXN];
  if (idp_ref_gl(p, xi, w)) return -1;
  for (int a = 0; a <= p; ++a) {
    for (int c = 0; c <= p; ++c) {
      double dphi;
      if (a == c) {
        dphi = 0.0;
        for (int m = 0; m <= p; ++m)
          if (m != a) dphi += 1.0 / (xi[a] - xi[m]);
      } else {
        double num = 1.0, den = 1.0;
        for (int m = 0; m <= p; ++m) {
          if (m != c) den *= (xi[c] - xi[m]);
          if (m != c && m != a) num *= (xi[a] - xi[m]);
        }
        dphi = num / den;
      }
      D[a * (p + 1) + c] = w[a] * dphi;
    }
  }
  return 0;
}

/* Sparsified matrix (eq. didp): Dhat[i][j] is the integral over [0,1] of
 * psi_i psi_j', psi the piecewise-linear hat functions on the subgrid of
 * Gauss-Lobatto points.  On the subinterval [xi_m, xi_{m+1}] of width h,
 * psi_m' = -1/h, psi_{m+1}' = +1/h and each of psi_m, psi_{m+1} integrates
 * to h/2, so each pair contributes +-1/2. */
int idp_ref_dhat(int p, double* Dh) {
  double xi[MAXN], w[MAXN];
  if (idp_ref_gl(p, xi, w)) return -1;
  int n = p + 1;
  for (int i = 0; i < n * n; ++i) Dh[i] = 0.0;
  for (int m = 0; m < p; ++m) {
    double h = xi[m + 1] - xi[m];
    int idx[2] = {m, m + 1};
    double dpsi[2] = {-1.0 / h, 1.0 / h};
    for (int ii = 0; ii < 2; ++ii)
      for (int jj = 0; jj < 2; ++jj)
        Dh[idx[ii] * n + idx[jj]] += dpsi[jj] * (0.5 * h);
  }
  return 0;
}

static int setup(ref_t* R, const idp_ref_desc* d) {
  if (idp_ref_check(d)) return -1;
  memset(R, 0, sizeof(*R));
  R->d = *d;
  R->nc = idp_ref_num_comp(d);
  R->n1 = d->p + 1;
  R->np = d->dim == 2 ? R->n1 * R->n1 : R->n1;
  R->ne = (long)d->nx * d->ny;
  R->nn = R->ne * R->np;
  R->hx = d->lx / d->nx;
  R->hy = d->dim == 2 ? d->ly / d->ny : 1.0;
  idp_ref_gl(d->p, R->xi, R->w);
  idp_ref_dmat(d->p, R->D);
  idp_ref_dhat(d->p, R->Dh);
  return 0;
}

/* ------------------------------------------------------------------ */
/* O1, O2: pointwise physics                                           */
/* ------------------------------------------------------------------ */

static double euler_pressure(const ref_t* R, const double* u) {
  double g = R->d.gamma, kin = 0.0;
  for (int k = 0; k < R->d.dim; ++k) kin += u[1 + k] * u[1 + k];
  return (g - 1.0) * (u[R->d.dim + 1] - 0.5 * kin / u[0]);
}

/* flux F(u) (eq. cons-law): F[k*nc + c] */
static void flux(const ref_t* R, const double* u, double* F) {
  int dim = R->d.dim, nc = R->nc;
  if (R->d.eq == IDP_REF_ADVECTION) {
    for (int k = 0; k < dim; ++k) F[k] = R->d.vel[k] * u[0];
  } else if (R->d.eq == IDP_REF_BURGERS) {
    for (int k = 0; k < dim; ++k) F[k] = 0.5 * u[0] * u[0] * R->d.vel[k];
  } else {
    /* eq. euler-flux: (rho v, rho v v^T + p I, rho H v), rho H = rho E + p */
    double rho = u[0], pr = euler_pressure(R, u), rE = u[dim + 1];
    for (int k = 0; k < dim; ++k) {
      double vk = u[1 + k] / rho;
      F[k * nc + 0] = u[1 + k];
      for (int l = 0; l < dim; ++l)
        F[k * nc + 1 + l] = u[1 + l] * vk + (k == l ? pr : 0.0);
      F[k * nc + dim + 1] = vk * (rE + pr);
    }
  }
}

/* Upper bound of the maximum wave speed of the 1-D Riemann problem (eq.
 * riemann-problem) with uL at x<0 and uR at x>0 along the unit vector n.
 * Scalar laws: max |f'(u) . n| over the states of the fan (exact, the
 * fluxes are linear or convex).  Euler, reading: the paper only asks for
 * lambda >= lambda_max; we use the two-rarefaction pressure bound of
 * Guermond & Popov (J. Comput. Phys. 2016), an upper bound for
 * 1 < gamma <= 5/3. */
static double lambda(const ref_t* R, const double* uL, const double* uR,
                     const double* n) {
  int dim = R->d.dim;
  if (R->d.eq == IDP_REF_ADVECTION) {
    double an = 0.0;
    for (int k = 0; k < dim; ++k) an += R->d.vel[k] * n[k];
    return fabs(an);
  }
  if (R->d.eq == IDP_REF_BURGERS) {
    double vn = 0.0;
    for (int k = 0; k < dim; ++k) vn += R->d.vel[k] * n[k];
    return fmax(fabs(uL[0]), fabs(uR[0])) * fabs(vn);
  }
  double g = R->d.gamma;
  double rl = uL[0], rr = uR[0];
  double vl = 0.0, vr = 0.0;
  for (int k = 0; k < dim; ++k) {
    vl += uL[1 + k] * n[k];
    vr += uR[1 + k] * n[k];
  }
  vl /= rl;
  vr /= rr;
  double pl = euler_pressure(R, uL), pr = euler_pressure(R, uR);
  double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
  double ex = (g - 1.0) / (2.0 * g);
  double num = cl + cr - 0.5 * (g - 1.0) * (vr - vl);
  if (num < 0.0) num = 0.0;
  double den = cl * pow(pl, -ex) + cr * pow(pr, -ex);
  double pstar = pow(num / den, 1.0 / ex);
  double fac = (g + 1.0) / (2.0 * g);
  double lam_l = vl - cl * sqrt(1.0 + fac * fmax(pstar - pl, 0.0) / pl);
  double lam_r = vr + cr * sqrt(1.0 + fac * fmax(pstar - pr, 0.0) / pr);
  return fmax(fmax(-lam_l, 0.0), fmax(lam_r, 0.0));
}

int idp_ref_flux(const idp_ref_desc* d, const double* u, double* F) {
  ref_t R;
  if (setup(&R, d) || d->eq == IDP_REF_ADVECTION_FIELD) return -1;
  flux(&R, u, F);
  return 0;
}

double idp_ref_lambda(const idp_ref_desc* d, const double* uL,
                      const double* uR, const double* n) {
  ref_t R;
  if (setup(&R, d) || d->eq == IDP_REF_ADVECTION_FIELD) return NAN;
  return lambda(&R, uL, uR, n);
}

/* The flux at node i with state ui: F(ui), or beta_i ui for a velocity
 * field (the collocated flux of Sec. 3.3). */
static void flux_node(const ref_t* R, const double* ui, long i, double* F) {
  if (R->d.eq == IDP_REF_ADVECTION_FIELD) {
    for (int k = 0; k < R->d.dim; ++k) F[k] = R->d.beta[(long)k * R->nn + i] * ui[0];
    return;
  }
  flux(R, ui, F);
}

/* Lax-Friedrichs numerical flux (eq. lax-friedrichs) between node im
 * (state um) and node ip (state up) on an element face: Fh = 1/2 (F_m +
 * F_p) . n - lambda/2 (up - um).  Reading for a velocity field: lambda =
 * max(|beta_m . n|, |beta_p . n|); the two nodes sit at one point, where
 * the field has one value. */
static void lax_friedrichs(const ref_t* R, const double* um, long im, const double* up,
                           long ip, const double* n, double* Fh) {
  double Fm[2 * MAXC], Fp[2 * MAXC];
  int nc = R->nc;
  flux_node(R, um, im, Fm);
  flux_node(R, up, ip, Fp);
  double lam;
  if (R->d.eq == IDP_REF_ADVECTION_FIELD) {
    double bm = 0.0, bp = 0.0;
    for (int k = 0; k < R->d.dim; ++k) {
      bm += R->d.beta[(long)k * R->nn + im] * n[k];
      bp += R->d.beta[(long)k * R->nn + ip] * n[k];
    }
    lam = fmax(fabs(bm), fabs(bp));
  } else {
    lam = lambda(R, um, up, n);
  }
  for (int c = 0; c < nc; ++c) {
    double fn = 0.0;
    for (int k = 0; k < R->d.dim; ++k)
      fn += 0.5 * (Fm[k * nc + c] + Fp[k * nc + c]) * n[k];
    Fh[c] = fn - 0.5 * lam * (up[c] - um[c]);
  }
}

/* ------------------------------------------------------------------ */
/* mesh helpers                                                        */
/* ------------------------------------------------------------------ */

static long node_index(const ref_t* R, long ex, long ey, int a, int b) {
  long e = ey * R->d.nx + ex;
  return e * R->np + (long)b * R->n1 + a;
}

/* local coordinates of node i */
static void node_coords(const ref_t* R, long i, long* ex, long* ey, int* a,
                        int* b) {
  long e = i / R->np;
  int loc = (int)(i % R->np);
  *ex = e % R->d.nx;
  *ey = e / R->d.nx;
  *a = loc % R->n1;
  *b = loc / R->n1;
}

/* The neighbour of node i one node away in direction k on side s (+1 or
 * -1), across the element face (periodic) when i lies on that face.
 * *across is set when the pair straddles an element face. */
static long neighbour(const ref_t* R, long i, int k, int s, int* across) {
  long ex, ey;
  int a, b, p = R->d.p;
  node_coords(R, i, &ex, &ey, &a, &b);
  *across = 0;
  if (k == 0) {
    a += s;
    if (a < 0) { a = p; ex = (ex - 1 + R->d.nx) % R->d.nx; *across = 1; }
    if (a > p) { a = 0; ex = (ex + 1) % R->d.nx; *across = 1; }
  } else {
    b += s;
    if (b < 0) { b = p; ey = (ey - 1 + R->d.ny) % R->d.ny; *across = 1; }
    if (b > p) { b = 0; ey = (ey + 1) % R->d.ny; *across = 1; }
  }
  return node_index(R, ex, ey, a, b);
}

/* the position of node i along a k-line and the transverse index */
static int line_pos(const ref_t* R, long i, int k, int* t) {
  long ex, ey;
  int a, b;
  node_coords(R, i, &ex, &ey, &a, &b);
  if (k == 0) { *t = b; return a; }
  *t = a;
  return b;
}

/* Metric factor of a k-line (Sec. 2.3 on an affine Cartesian element):
 * GJ^-1 = diag(hy, hx); the Kronecker structure (eq. kronecker) puts the
 * transverse quadrature weight on each line.  In 1-D it is 1. */
static double line_scale(const ref_t* R, int k, int t) {
  if (R->d.dim == 1) return 1.0;
  return k == 0 ? R->w[t] * R->hy : R->w[t] * R->hx;
}

/* metric term q of node i on a curved mesh (see idp_ref_desc.metric) */
static double met(const ref_t* R, int q, long i) { return R->d.metric[(long)q * R->nn + i]; }

/* node mass m_i: diagonal of M_K = M_ref G (Sec. 2.3), G = det(J) */
static double node_mass(const ref_t* R, long i) {
  long ex, ey;
  int a, b;
  node_coords(R, i, &ex, &ey, &a, &b);
  if (R->d.dim == 1) return R->w[a] * R->hx;
  if (R->d.metric) return R->w[a] * R->w[b] * met(R, 8, i);
  return R->w[a] * R->w[b] * R->hx * R->hy;
}

/* Row k of the metric terms of node i (curved meshes): the high-order
 * det(J) J^-1 (corr = 0) or the modified terms with the conservative
 * correction (corr = 1). */
static void metric_row(const ref_t* R, long i, int k, int corr, double* v) {
  v[0] = met(R, 4 * corr + 2 * k, i);
  v[1] = met(R, 4 * corr + 2 * k + 1, i);
}

/* the contravariant flux (eq. contravariant) of component c of node i
 * along reference direction k: sum_l (row k of the metric)_l F_l(u_i) */
static double contra(const ref_t* R, const double* F, long i, int k, int c, int corr) {
  double v[2];
  metric_row(R, i, k, corr, v);
  const long nn = R->nn;
  const int nc = R->nc;
  return v[0] * F[((long)0 * nc + c) * nn + i] + v[1] * F[((long)1 * nc + c) * nn + i];
}

/* The scaled normal (pointing in +xi_k) of the element face between the
 * k-neighbours jl (on the lower side) and jr: row k of the high-order
 * metric terms at the face node of the lower element, so that both
 * elements use one normal and the face flux is single-valued (reading:
 * the paper evaluates the face normals from the metric terms at the face
 * nodes; for a continuous mesh the two sides agree up to rounding). */
static void face_normal(const ref_t* R, long jl, int k, double* n) {
  metric_row(R, jl, k, 0, n);
}

static void get_state(const ref_t* R, const double* u, long i, double* ui) {
  for (int c = 0; c < R->nc; ++c) ui[c] = u[(long)c * R->nn + i];
}

/* The neighbour of node i in direction k on side s when the pair may cross
 * the boundary of an open direction.  Returns the neighbour's index, or i
 * itself for a boundary face of an open direction (*ghost set): the
 * exterior state then stands in for the neighbour, at the same point as
 * node i. */
static long nbr(const ref_t* R, long i, int k, int s, int* across, int* ghost) {
  long j = neighbour(R, i, k, s, across);
  *ghost = 0;
  if (*across && R->d.bc[k]) {
    long ex, ey;
    int a, b;
    node_coords(R, i, &ex, &ey, &a, &b);
    long e = k == 0 ? ex : ey, n = k == 0 ? R->d.nx : R->d.ny;
    if ((s < 0 && e == 0) || (s > 0 && e == n - 1)) {
      *ghost = 1;
      return i;
    }
  }
  return j;
}

/* The state of that neighbour: u_j, or the exterior state of the boundary
 * node i (reading: the paper leaves the boundary treatment open; the
 * exterior state enters the Lax-Friedrichs flux, the graph viscosity and
 * the bar states like a neighbour, so the low-order update stays a convex
 * combination of admissible bar states when the exterior state is
 * admissible). */
static void nbr_state(const ref_t* R, const double* u, long i, int k, int s, int ghost, long j,
                      double* uj) {
  get_state(R, u, j, uj);
  if (!ghost) return;
  long ex, ey;
  int a, b;
  node_coords(R, i, &ex, &ey, &a, &b);
  int side = 2 * k + (s > 0);
  long q = k == 0 ? ey * R->n1 + b : ex * R->n1 + a;
  long n = R->d.dim == 1 ? 1 : (k == 0 ? R->d.ny : R->d.nx) * R->n1;
  int type = R->d.bc_type[side][q];
  if (type == IDP_REF_BC_STATE && R->d.bc_state[side]) {
    for (int c = 0; c < R->nc; ++c) uj[c] = R->d.bc_state[side][(long)c * n + q];
  } else if (type == IDP_REF_BC_SLIP && R->d.eq == IDP_REF_EULER) {
    uj[1 + k] = -uj[1 + k];
  }
}

/* Graph coefficients of the low-order scheme in the form eq. dg-idp for
 * the neighbour j of i in direction k on side s: chat_ij (the k-th
 * component; the others vanish on Cartesian elements) and dhat_ij.
 *  - j in the same element: chat_ij = c_ij, the coefficient of F_j in row
 *    i of Dhat_k^T GJ^-1 (eq. dg-lo-cij), and dhat_ij = d_ij (eq. dij).
 *  - j across an element face: chat_ij = b_ij, the coefficient of F_j in
 *    -B_e Fhat_e, i.e. -1/2 times the weighted outward normal, and
 *    dhat_ij = lambda/2 |wn_ij| (the Lax-Friedrichs dissipation).
 * Reading: lambda_max(u_i, u_j, n) is taken for the Riemann problem with
 * u_i on the left and u_j on the right along the unit vector pointing
 * from node i to node j. */
static void graph_coeffs(const ref_t* R, const double* u, long i, int k, int s,
                         long* j_out, double* chat, double* dhat, double* uj_out) {
  int across, ghost, t;
  long j = nbr(R, i, k, s, &across, &ghost);
  if (u && uj_out) nbr_state(R, u, i, k, s, ghost, j, uj_out);
  double scale = line_scale(R, k, (line_pos(R, i, k, &t), t));
  double e_ij[2] = {0.0, 0.0}, e_ji[2] = {0.0, 0.0};
  e_ij[k] = (double)s;
  e_ji[k] = (double)-s;
  if (R->d.eq == IDP_REF_ADVECTION_FIELD) {
    /* Sec. 3.3: dhat_ij = max(|chat_ij . beta_i|, |chat_ji . beta_j|) */
    double bi = R->d.beta[(long)k * R->nn + i], bj = R->d.beta[(long)k * R->nn + j];
    double cij, cji;
    if (across) {
      cij = -0.5 * scale * (double)s;
      cji = 0.5 * scale * (double)s;
    } else {
      int ai = line_pos(R, i, k, &t);
      cij = scale * R->Dh[(ai + s) * R->n1 + ai];
      cji = scale * R->Dh[ai * R->n1 + ai + s];
    }
    double d1 = fabs(cij * bi), d2 = fabs(cji * bj);
    *chat = cij;
    *dhat = d1 > d2 ? d1 : d2;
    *j_out = j;
    return;
  }
  double ui[MAXC], uj[MAXC];
  get_state(R, u, i, ui);
  nbr_state(R, u, i, k, s, ghost, j, uj);
  if (across) {
    double wn = scale; /* |wn_ij|: face weight times face metric */
    *chat = -0.5 * wn * (double)s;
    *dhat = 0.5 * lambda(R, ui, uj, e_ij) * wn;
  } else {
    int n1 = R->n1;
    int ai = line_pos(R, i, k, &t);
    int aj = ai + s;
    double cij = scale * R->Dh[aj * n1 + ai]; /* (Dhat^T)_{ai,aj} */
    double cji = scale * R->Dh[ai * n1 + aj];
    *chat = cij;
    double d1 = lambda(R, ui, uj, e_ij) * fabs(cij);
    double d2 = lambda(R, uj, ui, e_ji) * fabs(cji);
    *dhat = d1 > d2 ? d1 : d2;
  }
  *j_out = j;
}

/* Graph coefficients on a curved mesh (vector chat_ij, and dhat_ij) for
 * the neighbour j of i in direction k on side s.
 *  - j in the same element: chat_ij = w_t Dhat[aj][ai] (row k of the
 *    modified metric terms at j), the coefficient of F_j in row i of
 *    Dhat_k^T Jinvidp_k. (eq. dg-lo-cij, eq. dg-lo-modified), and
 *    dhat_ij = max(lambda(u_i, u_j, n_ij) |chat_ij|, lambda(u_j, u_i,
 *    n_ji) |chat_ji|) (eq. dij).
 *  - j across an element face: chat_ij = -1/2 w_t n (n the outward scaled
 *    normal of i's element) and dhat_ij = lambda/2 |n| w_t.
 * Reading (as on Cartesian meshes): n_ij is the unit vector pointing from
 * node i to node j, -chat_ij / |chat_ij|, and lambda_max(u_i, u_j, n) is
 * taken for u_i on the left and u_j on the right along it. */
static void graph_coeffs_m(const ref_t* R, const double* u, long i, int k, int s,
                           long* j_out, double* chat, double* dhat, double* uj_out) {
  int across, t;
  long j = neighbour(R, i, k, s, &across);
  double ui[MAXC], uj[MAXC];
  get_state(R, u, i, ui);
  get_state(R, u, j, uj);
  if (uj_out) memcpy(uj_out, uj, sizeof(double) * R->nc);
  int ai = line_pos(R, i, k, &t);
  double wt = R->w[t];
  if (across) {
    double n[2];
    face_normal(R, s > 0 ? i : j, k, n);
    n[0] *= (double)s;
    n[1] *= (double)s;
    double nm = sqrt(n[0] * n[0] + n[1] * n[1]);
    double nu[2] = {n[0] / nm, n[1] / nm};
    chat[0] = -0.5 * wt * n[0];
    chat[1] = -0.5 * wt * n[1];
    *dhat = 0.5 * lambda(R, ui, uj, nu) * nm * wt;
  } else {
    int n1 = R->n1, aj = ai + s;
    double vj[2], vi[2];
    metric_row(R, j, k, 1, vj);
    metric_row(R, i, k, 1, vi);
    double cij[2] = {wt * R->Dh[aj * n1 + ai] * vj[0], wt * R->Dh[aj * n1 + ai] * vj[1]};
    double cji[2] = {wt * R->Dh[ai * n1 + aj] * vi[0], wt * R->Dh[ai * n1 + aj] * vi[1]};
    double mij = sqrt(cij[0] * cij[0] + cij[1] * cij[1]);
    double mji = sqrt(cji[0] * cji[0] + cji[1] * cji[1]);
    double nij[2] = {-cij[0] / mij, -cij[1] / mij};
    double nji[2] = {-cji[0] / mji, -cji[1] / mji};
    double d1 = lambda(R, ui, uj, nij) * mij;
    double d2 = lambda(R, uj, ui, nji) * mji;
    chat[0] = cij[0];
    chat[1] = cij[1];
    *dhat = d1 > d2 ? d1 : d2;
  }
  *j_out = j;
}

/* The discrete divergence-free identity of a velocity field (Sec. 3.3):
 * per node and direction, sum_{j != i} chat_ij beta_{j,k} = 0 within 1e-12
 * of sum |chat_ij beta_{j,k}|.  Reading: the paper requires this identity
 * for the low-order update to be conservative and the bar states to be
 * the update's convex decomposition, and says that the conservative
 * correction must be adapted to enforce it without giving the adaptation;
 * fields that miss it are rejected rather than corrected.  Fields with
 * beta_x depending on y only and beta_y on x only meet it on Cartesian
 * meshes (beta_{j,k} is constant along a k-line and the chat_ij of a line
 * sum to zero). */
static int field_check(const idp_ref_desc* d) {
  if (d->dim != 2 || !d->beta) return -1;
  ref_t Rs, *R = &Rs;
  memset(R, 0, sizeof(*R));
  R->d = *d;
  R->nc = 1;
  R->n1 = d->p + 1;
  R->np = R->n1 * R->n1;
  R->ne = (long)d->nx * d->ny;
  R->nn = R->ne * R->np;
  R->hx = d->lx / d->nx;
  R->hy = d->ly / d->ny;
  if (idp_ref_gl(d->p, R->xi, R->w) || idp_ref_dhat(d->p, R->Dh)) return -1;
  for (long q = 0; q < 2 * R->nn; ++q)
    if (!isfinite(d->beta[q])) return -1;
  for (long i = 0; i < R->nn; ++i) {
    for (int k = 0; k < 2; ++k) {
      double sum = 0.0, mag = 0.0;
      for (int sd = -1; sd <= 1; sd += 2) {
        long j;
        double chat, dhat;
        graph_coeffs(R, NULL, i, k, sd, &j, &chat, &dhat, NULL);
        double t = chat * d->beta[(long)k * R->nn + j];
        sum += t;
        mag += fabs(t);
      }
      if (fabs(sum) > 1e-12 * mag) return -1;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* O9: entropy line search                                             */
/* ------------------------------------------------------------------ */

/* Phi(V) = rho e - K_min rho^gamma/(gamma-1), rho e = E - |m|^2/(2 rho).
 * For rho > 0, Phi >= 0 <=> p rho^-gamma >= K_min <=> s >= s_min (the
 * specific entropy of Sec. 4.3 is increasing in p rho^-gamma), and Phi is
 * concave, so {Phi >= 0, rho > 0} is convex. */
static int admissible(const ref_t* R, const double* V, double kmin) {
  int dim = R->d.dim;
  double g = R->d.gamma;
  if (!(V[0] > 0.0)) return 0;
  double kin = 0.0;
  for (int k = 0; k < dim; ++k) kin += V[1 + k] * V[1 + k];
  double rhoe = V[dim + 1] - 0.5 * kin / V[0];
  double phi = rhoe - kmin * pow(V[0], g) / (g - 1.0);
  return phi >= 0.0;
}

/* sup { t in [0, tmax] : uL + t P admissible }, by bisection on the convex
 * feasible set; returns the admissible end of a bracket no wider than
 * 1e-15 (reading: the paper asks for a line search, by Newton's method,
 * without a tolerance). */
static double entropy_search(const ref_t* R, const double* uL, const double* P,
                             double tmax, double kmin) {
  double V[MAXC];
  int nc = R->nc;
  for (int c = 0; c < nc; ++c) V[c] = uL[c] + tmax * P[c];
  if (admissible(R, V, kmin)) return tmax;
  if (!admissible(R, uL, kmin)) return 0.0;
  double lo = 0.0, hi = tmax;
  for (int it = 0; it < 200 && hi - lo > 1e-15; ++it) {
    double mid = 0.5 * (lo + hi);
    for (int c = 0; c < nc; ++c) V[c] = uL[c] + mid * P[c];
    if (admissible(R, V, kmin))
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

/* ------------------------------------------------------------------ */
/* O7b: subcell-resolution smoothness indicator (Sec. 4.4)             */
/* ------------------------------------------------------------------ */

/* Inverse of the Legendre Vandermonde matrix V[a][k] = P_k(2 xi_a - 1) on
 * the Gauss-Lobatto points (nodal values -> modal coefficients), by
 * Gauss-Jordan elimination with partial pivoting. */
static int legendre_vandermonde_inverse(int p, const double* xi, double* Vi) {
  int n = p + 1;
  double A[MAXN][2 * MAXN];
  for (int a = 0; a < n; ++a) {
    for (int k = 0; k < n; ++k) {
      double P, dP, d2P;
      legendre(k, 2.0 * xi[a] - 1.0, &P, &dP, &d2P);
      A[a][k] = P;
      A[a][n + k] = a == k ? 1.0 : 0.0;
    }
  }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
    if (A[piv][c] == 0.0) return -1;
    for (int k = 0; k < 2 * n; ++k) {
      double t = A[c][k];
      A[c][k] = A[piv][k];
      A[piv][k] = t;
    }
    double inv = 1.0 / A[c][c];
    for (int k = 0; k < 2 * n; ++k) A[c][k] *= inv;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = A[r][c];
      for (int k = 0; k < 2 * n; ++k) A[r][k] -= f * A[c][k];
    }
  }
  for (int a = 0; a < n; ++a)
    for (int k = 0; k < n; ++k) Vi[a * n + k] = A[a][n + k];
  return 0;
}

/* Readings (the printed ramp 1/2 - 1/2 sin(.) contradicts its own end
 * values, 0 below s0 - kappa and 1 above s0 + kappa, and the text, which
 * keeps the local bounds where the solution is rough): eps rises as
 * 1/2 + 1/2 sin(pi (s - s0) / (2 kappa)).  s0 = log10(p^-4) and kappa = 1,
 * the choices the paper states for p > 1; for p = 1 the indicator is off
 * (eps = 1, the strict local bounds), as in the paper's table where both
 * columns agree for p <= 1.  An element whose polynomial is zero is smooth
 * (eps = 0).  The L2 norms are those of the element's interpolating
 * polynomial, exact through the orthogonality of the Legendre modes
 * (||P_k||^2 = 2/(2k+1) on [-1,1]; the element's size cancels in the
 * ratio). */
int idp_ref_smoothness(const idp_ref_desc* d, const double* u, double* eps) {
  if (idp_ref_check(d) || !u || !eps) return -1;
  const int p = d->p, n1 = p + 1, dim = d->dim;
  const long ne = (long)d->nx * d->ny;
  const long np = dim == 2 ? (long)n1 * n1 : n1;
  if (p == 1) {
    for (long e = 0; e < ne; ++e) eps[e] = 1.0;
    return 0;
  }
  double xi[MAXN], w[MAXN], Vi[MAXN * MAXN], nk[MAXN];
  if (idp_ref_gl(p, xi, w) || legendre_vandermonde_inverse(p, xi, Vi)) return -1;
  for (int k = 0; k < n1; ++k) nk[k] = 2.0 / (2.0 * k + 1.0);
  const double s0 = log10(pow((double)p, -4.0)), kappa = 1.0;
  for (long e = 0; e < ne; ++e) {
    const double* ue = u + e * np;   /* component 0: u, or rho for Euler */
    double total = 0.0, high = 0.0;
    if (dim == 1) {
      for (int k = 0; k < n1; ++k) {
        double c = 0.0;
        for (int a = 0; a < n1; ++a) c += Vi[k * n1 + a] * ue[a];
        total += c * c * nk[k];
        if (k == p) high += c * c * nk[k];
      }
    } else {
      for (int l = 0; l < n1; ++l) {
        for (int k = 0; k < n1; ++k) {
          double c = 0.0;
          for (int b = 0; b < n1; ++b)
            for (int a = 0; a < n1; ++a) c += Vi[l * n1 + b] * Vi[k * n1 + a] * ue[b * n1 + a];
          total += c * c * nk[k] * nk[l];
          if (k == p || l == p) high += c * c * nk[k] * nk[l];
        }
      }
    }
    if (!(total > 0.0)) {
      eps[e] = 0.0;
      continue;
    }
    const double sk = log10(high / total);
    if (sk < s0 - kappa)
      eps[e] = 0.0;
    else if (sk > s0 + kappa)
      eps[e] = 1.0;
    else
      eps[e] = 0.5 + 0.5 * sin(M_PI * (sk - s0) / (2.0 * kappa));
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* forward-Euler sub-step                                              */
/* ------------------------------------------------------------------ */

/* O3/O4/O6 on one k-line of element (ex, ey) of a curved mesh: the
 * transverse weight w_t of the Kronecker structure (eq. kronecker) times
 *  - high order (eq. dg-strong): -sum_m D[a][m] Ft_m with Ft the
 *    contravariant flux of the high-order metric terms, and on the element
 *    faces -(Fhat - F . n) with n the outward scaled normal;
 *  - low order (eq. dg-lo-modified): sum_m Dhat[m][a] Gt_m with Gt the
 *    contravariant flux of the modified metric terms, -Fhat on the element
 *    faces, and the graph viscosity d_ij (u_j - u_i) of eq. dij inside;
 *  - the subcell sums rbar of the line (zero on the element faces).
 * The face flux is the Lax-Friedrichs flux of eq. lax-friedrichs with the
 * scaled normal n: |n| Fhat(u^-, u^+, n/|n|). */
static void curved_line(const ref_t* R, const double* u, const double* F, double* rH, double* rL,
                        double* rbar, long ex, long ey, int k, int t) {
  const int nc = R->nc, p = R->d.p, n1 = R->n1;
  const long nn = R->nn;
  long line[MAXN];
  for (int a = 0; a <= p; ++a) line[a] = k == 0 ? node_index(R, ex, ey, a, t) : node_index(R, ex, ey, t, a);
  const double wt = R->w[t];
  int across;
  long jl = neighbour(R, line[0], k, -1, &across);
  long jr = neighbour(R, line[p], k, +1, &across);
  double nL[2], nR[2];
  face_normal(R, jl, k, nL);        /* +xi_k normal of the left face */
  face_normal(R, line[p], k, nR);   /* of the right face */
  double u0[MAXC], up[MAXC], ujl[MAXC], ujr[MAXC], FhL[MAXC], FhR[MAXC];
  get_state(R, u, line[0], u0);
  get_state(R, u, line[p], up);
  get_state(R, u, jl, ujl);
  get_state(R, u, jr, ujr);
  {
    /* outward normals of this element: -nL on the left, +nR on the right */
    double mL = sqrt(nL[0] * nL[0] + nL[1] * nL[1]), mR = sqrt(nR[0] * nR[0] + nR[1] * nR[1]);
    double oL[2] = {-nL[0] / mL, -nL[1] / mL}, oR[2] = {nR[0] / mR, nR[1] / mR};
    lax_friedrichs(R, u0, line[0], ujl, jl, oL, FhL);
    lax_friedrichs(R, up, line[p], ujr, jr, oR, FhR);
    for (int c = 0; c < nc; ++c) {
      FhL[c] *= mL;
      FhR[c] *= mR;
    }
  }
#define IDX3(kk, cc, ii) (((long)(kk) * nc + (cc)) * nn + (ii))
  for (int a = 0; a <= p; ++a) {
    long i = line[a];
    for (int c = 0; c < nc; ++c) {
      double vol = 0.0;
      for (int m = 0; m <= p; ++m) vol += R->D[a * n1 + m] * contra(R, F, line[m], k, c, 0);
      double rh = -wt * vol;
      if (a == 0) {
        double fn = F[IDX3(0, c, i)] * (-nL[0]) + F[IDX3(1, c, i)] * (-nL[1]);
        rh -= wt * (FhL[c] - fn);
      }
      if (a == p) {
        double fn = F[IDX3(0, c, i)] * nR[0] + F[IDX3(1, c, i)] * nR[1];
        rh -= wt * (FhR[c] - fn);
      }
      rH[IDX3(k, c, i)] = rh;
      double volh = 0.0;
      for (int m = 0; m <= p; ++m) volh += R->Dh[m * n1 + a] * contra(R, F, line[m], k, c, 1);
      double rl = wt * volh;
      if (a == 0) rl -= wt * FhL[c];
      if (a == p) rl -= wt * FhR[c];
      rL[IDX3(k, c, i)] = rl;
    }
    for (int sd = -1; sd <= 1; sd += 2) {
      int aj = a + sd;
      if (aj < 0 || aj > p) continue;
      long j;
      double chat[2], dij, ui[MAXC], uj[MAXC];
      graph_coeffs_m(R, u, i, k, sd, &j, chat, &dij, uj);
      get_state(R, u, i, ui);
      for (int c = 0; c < nc; ++c) rL[IDX3(k, c, i)] += dij * (uj[c] - ui[c]);
    }
  }
  for (int c = 0; c < nc; ++c) {
    double acc = 0.0;
    for (int a = 0; a < p; ++a) {
      acc += rH[IDX3(k, c, line[a])] - rL[IDX3(k, c, line[a])];
      rbar[IDX3(k, c, line[a])] = acc;
    }
    rbar[IDX3(k, c, line[p])] = 0.0;
  }
#undef IDX3
}

int idp_ref_fe(const idp_ref_desc* dsc, const double* u, double* out,
               double dt, idp_ref_trace* tr) {
  ref_t Rs, *R = &Rs;
  if (setup(R, dsc)) return -1;
  if (!u || !out || !(dt >= 0.0)) return -1;
  const int dim = R->d.dim, nc = R->nc, p = R->d.p, n1 = R->n1;
  const long nn = R->nn;
  const int lim = 0; /* limited component: u (scalar) or rho (Euler) */
  const int euler = R->d.eq == IDP_REF_EULER;
  const int field = R->d.eq == IDP_REF_ADVECTION_FIELD;

  if (dt == 0.0) { /* a zero step leaves the state unchanged */
    memcpy(out, u, sizeof(double) * nc * nn);
    return 0;
  }

  double* F = malloc(sizeof(double) * dim * nc * nn);
  double* rH = calloc((size_t)dim * nc * nn, sizeof(double));
  double* rL = calloc((size_t)dim * nc * nn, sizeof(double));
  double* rbar = calloc((size_t)dim * nc * nn, sizeof(double));
  double* uL = malloc(sizeof(double) * nc * nn);
  double* uH = malloc(sizeof(double) * nc * nn);
  double* umin = malloc(sizeof(double) * nn);
  double* umax = malloc(sizeof(double) * nn);
  double* kmin = malloc(sizeof(double) * nn);
  double* az = malloc(sizeof(double) * nn);
  double* al = malloc(sizeof(double) * nn);
  if (!F || !rH || !rL || !rbar || !uL || !uH || !umin || !umax || !kmin ||
      !az || !al) {
    free(F); free(rH); free(rL); free(rbar); free(uL); free(uH);
    free(umin); free(umax); free(kmin); free(az); free(al);
    return -2;
  }
#define IDX3(k, c, i) (((long)(k) * nc + (c)) * nn + (i))

  /* O1: nodal fluxes */
#pragma omp parallel for schedule(static)
  for (long i = 0; i < nn; ++i) {
    double ui[MAXC], Fi[2 * MAXC];
    get_state(R, u, i, ui);
    flux_node(R, ui, i, Fi);
    for (int k = 0; k < dim; ++k)
      for (int c = 0; c < nc; ++c) F[IDX3(k, c, i)] = Fi[k * nc + c];
  }

  /* O3/O4: per-direction residuals along every line of every element
   * (each line writes only its own nodes' entries) */
#pragma omp parallel for schedule(static)
  for (long ey = 0; ey < R->d.ny; ++ey) {
    for (long ex = 0; ex < R->d.nx; ++ex) {
      for (int k = 0; k < dim; ++k) {
        for (int t = 0; t < (dim == 2 ? n1 : 1); ++t) {
          if (R->d.metric) {
            curved_line(R, u, F, rH, rL, rbar, ex, ey, k, t);
            continue;
          }
          long line[MAXN];
          for (int a = 0; a <= p; ++a)
            line[a] = k == 0 ? node_index(R, ex, ey, a, t)
                             : node_index(R, ex, ey, t, a);
          double s = line_scale(R, k, t);
          int across, gl, gr;
          long jl = nbr(R, line[0], k, -1, &across, &gl);
          long jr = nbr(R, line[p], k, +1, &across, &gr);
          double u0[MAXC], up[MAXC], ujl[MAXC], ujr[MAXC];
          double FhL[MAXC], FhR[MAXC];
          double nm[2] = {0.0, 0.0}, np_[2] = {0.0, 0.0};
          nm[k] = -1.0;
          np_[k] = 1.0;
          get_state(R, u, line[0], u0);
          get_state(R, u, line[p], up);
          nbr_state(R, u, line[0], k, -1, gl, jl, ujl);
          nbr_state(R, u, line[p], k, +1, gr, jr, ujr);
          /* numerical fluxes on the two element faces of this line, with
           * the outward unit normal of this element */
          lax_friedrichs(R, u0, line[0], ujl, jl, nm, FhL);
          lax_friedrichs(R, up, line[p], ujr, jr, np_, FhR);

          for (int a = 0; a <= p; ++a) {
            long i = line[a];
            for (int c = 0; c < nc; ++c) {
              /* high order, eq. ho-update: -(D_k GJ^-1 F + B (Fhat - F.n)) */
              double vol = 0.0;
              for (int m = 0; m <= p; ++m)
                vol += R->D[a * n1 + m] * F[IDX3(k, c, line[m])];
              double rh = -s * vol;
              if (a == 0) rh -= s * (FhL[c] - (-F[IDX3(k, c, i)]));
              if (a == p) rh -= s * (FhR[c] - F[IDX3(k, c, i)]);
              rH[IDX3(k, c, i)] = rh;

              /* low order, eq. lo-update: Dhat_k^T GJ^-1 F - B Fhat + sum
               * d_ij (u_j - u_i).  Reading: the viscosity enters with the
               * dissipative sign of eq. idp-fe. */
              double volh = 0.0;
              for (int m = 0; m <= p; ++m)
                volh += R->Dh[m * n1 + a] * F[IDX3(k, c, line[m])];
              double rl = s * volh;
              if (a == 0) rl -= s * FhL[c];
              if (a == p) rl -= s * FhR[c];
              rL[IDX3(k, c, i)] = rl;
            }
            if (field) {
              /* Sec. 3.3: the low-order update as the convex combination
               * of the modified bar states, sum_j 2 dhat_ij (ubar_ij - u_i)
               * = sum_j (dhat_ij + chat_ij . beta_j) (u_j - u_i), over
               * the two neighbours of i on this line (inside the element
               * or across its face) */
              double ui[MAXC];
              get_state(R, u, i, ui);
              double rl = 0.0;
              for (int sd = -1; sd <= 1; sd += 2) {
                long j;
                double chat, dhat, uj[MAXC];
                graph_coeffs(R, u, i, k, sd, &j, &chat, &dhat, uj);
                rl += (dhat + chat * R->d.beta[(long)k * nn + j]) * (uj[0] - ui[0]);
              }
              rL[IDX3(k, 0, i)] = rl;
              continue;
            }
            /* graph viscosity d_ij (eq. dij) between i and its neighbours
             * on the same line inside the element */
            for (int sd = -1; sd <= 1; sd += 2) {
              int aj = a + sd;
              if (aj < 0 || aj > p) continue;
              long j = line[aj];
              double ui[MAXC], uj[MAXC];
              get_state(R, u, i, ui);
              get_state(R, u, j, uj);
              double cij = s * R->Dh[aj * n1 + a];
              double cji = s * R->Dh[a * n1 + aj];
              double eij[2] = {0.0, 0.0}, eji[2] = {0.0, 0.0};
              eij[k] = (double)sd;
              eji[k] = (double)-sd;
              double d1 = lambda(R, ui, uj, eij) * fabs(cij);
              double d2 = lambda(R, uj, ui, eji) * fabs(cji);
              double dij = d1 > d2 ? d1 : d2;
              for (int c = 0; c < nc; ++c)
                rL[IDX3(k, c, i)] += dij * (uj[c] - ui[c]);
            }
          }

          /* O6: subcell fluxes rbar_{a+1/2} = sum_{c<=a} (rH - rL) over the
           * nodes on the left of the interior subcell face; zero on the
           * element faces (reading: only interior subcell faces carry an
           * antidiffusive flux, and the total over the line vanishes by
           * Prop. line-zero-sum). */
          for (int c = 0; c < nc; ++c) {
            double acc = 0.0;
            for (int a = 0; a < p; ++a) {
              acc += rH[IDX3(k, c, line[a])] - rL[IDX3(k, c, line[a])];
              rbar[IDX3(k, c, line[a])] = acc;
            }
            rbar[IDX3(k, c, line[p])] = 0.0;
          }
        }
      }
    }
  }

  /* O5: low-order and high-order provisional states */
#pragma omp parallel for schedule(static)
  for (long i = 0; i < nn; ++i) {
    double m = node_mass(R, i);
    for (int c = 0; c < nc; ++c) {
      double sl = 0.0, sh = 0.0;
      for (int k = 0; k < dim; ++k) {
        sl += rL[IDX3(k, c, i)];
        sh += rH[IDX3(k, c, i)];
      }
      uL[(long)c * nn + i] = u[(long)c * nn + i] + dt / m * sl;
      uH[(long)c * nn + i] = u[(long)c * nn + i] + dt / m * sh;
    }
  }

  /* O7: local bounds from the bar states (eq. bar-states, Sec. 4.1.1) and,
   * for Euler, the entropy bound s_min = min over the stencil (Sec. 4.3).
   * Reading: the stencil N(i) includes i itself. */
#pragma omp parallel for schedule(static)
  for (long i = 0; i < nn; ++i) {
    double ui[MAXC], Fi[2 * MAXC];
    get_state(R, u, i, ui);
    flux_node(R, ui, i, Fi);
    double lo = ui[lim], hi = ui[lim];
    double km = 0.0;
    if (euler) km = euler_pressure(R, ui) * pow(ui[0], -R->d.gamma);
    for (int k = 0; k < dim; ++k) {
      for (int sd = -1; sd <= 1; sd += 2) {
        long j;
        double chat, dhat;
        double uj[MAXC], Fj[2 * MAXC];
        if (R->d.metric) {
          /* eq. bar-states with the vector chat_ij of a curved mesh */
          double cv[2];
          graph_coeffs_m(R, u, i, k, sd, &j, cv, &dhat, uj);
          flux_node(R, uj, j, Fj);
          double bar = 0.5 * (ui[lim] + uj[lim]);
          double dF = cv[0] * (Fj[lim] - Fi[lim]) + cv[1] * (Fj[nc + lim] - Fi[nc + lim]);
          if (dhat > 0.0) bar += dF / (2.0 * dhat);
          if (bar < lo) lo = bar;
          if (bar > hi) hi = bar;
          if (euler) {
            double kj = euler_pressure(R, uj) * pow(uj[0], -R->d.gamma);
            if (kj < km) km = kj;
          }
          continue;
        }
        graph_coeffs(R, u, i, k, sd, &j, &chat, &dhat, uj);
        flux_node(R, uj, j, Fj);
        double bar = 0.5 * (ui[lim] + uj[lim]);
        /* eq. bar-states; for a velocity field the modified bar state of
         * Sec. 3.3, with chat_ij . beta_j (u_j - u_i) in place of
         * chat_ij . (F_j - F_i).  Reading: with dhat_ij = 0 the flux term
         * is 0/0; the bar state is then the plain average */
        double dF = field ? R->d.beta[(long)k * nn + j] * (uj[lim] - ui[lim])
                          : Fj[k * nc + lim] - Fi[k * nc + lim];
        if (dhat > 0.0) bar += chat * dF / (2.0 * dhat);
        if (bar < lo) lo = bar;
        if (bar > hi) hi = bar;
        if (euler) {
          double kj = euler_pressure(R, uj) * pow(uj[0], -R->d.gamma);
          if (kj < km) km = kj;
        }
      }
    }
    umin[i] = lo;
    umax[i] = hi;
    kmin[i] = euler ? km : 0.0;
  }

  /* O7b: eq. relaxed-bounds, u_hat = eps_K u + (1 - eps_K) g, on the bounds
   * of the limited component (the entropy bound of Euler is not relaxed) */
  if (R->d.limiter == IDP_REF_SUBCELL_SI) {
    double* eps = malloc(sizeof(double) * R->ne);
    if (!eps || idp_ref_smoothness(&R->d, u, eps)) {
      free(eps);
      free(F); free(rH); free(rL); free(rbar); free(uL); free(uH);
      free(umin); free(umax); free(kmin); free(az); free(al);
      return -1;
    }
    const long np = nn / R->ne;
    for (long i = 0; i < nn; ++i) {
      double ek = eps[i / np];
      umin[i] = ek * umin[i] + (1.0 - ek) * R->d.gmin;
      umax[i] = ek * umax[i] + (1.0 - ek) * R->d.gmax;
    }
    free(eps);
  }

  /* O8e/O9e: elementwise limiting (Sec. 4.1.2, eq. convex-provisional-
   * elementwise).  Every node limits its whole correction u^H_i - u^L_i =
   * dt/m_i (r^H_i - r^L_i): Zalesak with that single contribution on the
   * limited component, then for Euler the largest t in [0, alpha_z] with
   * u^L_i + t (u^H_i - u^L_i) admissible; the element applies the minimum
   * over its nodes, u = u^L + alpha_K (u^H - u^L). */
  if (R->d.limiter == IDP_REF_ELEMENTWISE) {
    const long np = nn / R->ne;
#pragma omp parallel for schedule(dynamic, 256)
    for (long i = 0; i < nn; ++i) {
      double m = node_mass(R, i);
      double ul = uL[(long)lim * nn + i];
      double f = m / dt * (uH[(long)lim * nn + i] - ul);
      double Qp = m / dt * (umax[i] - ul);
      double Qm = m / dt * (umin[i] - ul);
      if (Qp < 0.0) Qp = 0.0;
      if (Qm > 0.0) Qm = 0.0;
      double a = 1.0;
      if (f > 0.0) a = fmin(1.0, Qp / f);
      if (f < 0.0) a = fmin(1.0, Qm / f);
      az[i] = a;
      if (euler) {
        double uli[MAXC], P[MAXC];
        for (int c = 0; c < nc; ++c) {
          uli[c] = uL[(long)c * nn + i];
          P[c] = uH[(long)c * nn + i] - uli[c];
        }
        a = entropy_search(R, uli, P, a, kmin[i]);
      }
      al[i] = a;
    }
#pragma omp parallel for schedule(static)
    for (long e = 0; e < R->ne; ++e) {
      double aK = 1.0;
      for (long q = 0; q < np; ++q) aK = fmin(aK, al[e * np + q]);
      for (long q = 0; q < np; ++q) al[e * np + q] = aK;
    }
#pragma omp parallel for schedule(static)
    for (long i = 0; i < nn; ++i)
      for (int c = 0; c < nc; ++c) {
        long ic = (long)c * nn + i;
        out[ic] = uL[ic] + al[i] * (uH[ic] - uL[ic]);
      }
  }

  /* O8: nodal Zalesak coefficients on the limited component */
  const long nz_ = R->d.limiter == IDP_REF_ELEMENTWISE ? 0 : nn;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < nz_; ++i) {
    double m = node_mass(R, i);
    double Pp = 0.0, Pm = 0.0;
    for (int k = 0; k < dim; ++k) {
      int t;
      int a = line_pos(R, i, k, &t);
      double cp = a < p ? rbar[IDX3(k, lim, i)] : 0.0;
      double cm = 0.0;
      if (a > 0) {
        int across;
        long jm = neighbour(R, i, k, -1, &across);
        cm = -rbar[IDX3(k, lim, jm)];
      }
      Pp += (cp > 0.0 ? cp : 0.0) + (cm > 0.0 ? cm : 0.0);
      Pm += (cp < 0.0 ? cp : 0.0) + (cm < 0.0 ? cm : 0.0);
    }
    double ul = uL[(long)lim * nn + i];
    double Qp = m / dt * (umax[i] - ul);
    double Qm = m / dt * (umin[i] - ul);
    if (Qp < 0.0) Qp = 0.0;
    if (Qm > 0.0) Qm = 0.0;
    double Rp = Pp == 0.0 ? 1.0 : fmin(1.0, Qp / Pp);
    double Rm = Pm == 0.0 ? 1.0 : fmin(1.0, Qm / Pm);
    az[i] = fmin(Rp, Rm);
    al[i] = az[i];
  }

  /* O9: Euler, convex limiting of the specific entropy (eq.
   * convex-provisional with gamma = 2d): every partial state
   * uL + t 2d dt/m (+-rbar) must stay admissible, t <= alpha_z.  Reading:
   * the search runs on [0, alpha_z] and also keeps rho > 0. */
  if (euler && R->d.limiter != IDP_REF_ELEMENTWISE) {
#pragma omp parallel for schedule(dynamic, 256)
    for (long i = 0; i < nn; ++i) {
      double m = node_mass(R, i);
      double uli[MAXC];
      get_state(R, uL, i, uli);
      double a_i = az[i];
      for (int k = 0; k < dim; ++k) {
        int t;
        int a = line_pos(R, i, k, &t);
        for (int sd = -1; sd <= 1; sd += 2) {
          double cf[MAXC];
          int nz = 0;
          if (sd > 0) {
            if (a == p) continue;
            for (int c = 0; c < nc; ++c) cf[c] = rbar[IDX3(k, c, i)];
          } else {
            if (a == 0) continue;
            int across;
            long jm = neighbour(R, i, k, -1, &across);
            for (int c = 0; c < nc; ++c) cf[c] = -rbar[IDX3(k, c, jm)];
          }
          double P[MAXC];
          for (int c = 0; c < nc; ++c) {
            P[c] = 2.0 * dim * dt / m * cf[c];
            if (cf[c] != 0.0) nz = 1;
          }
          if (!nz) continue;
          double tf = entropy_search(R, uli, P, az[i], kmin[i]);
          if (tf < a_i) a_i = tf;
        }
      }
      al[i] = a_i;
    }
  }

  /* O10: subcell face coefficients alpha_{m,k} = min of the two adjacent
   * nodal coefficients and the flux-corrected update (eq. subcell-fct /
   * convex-fct).  Limiter modes TARGET and LOW return the unlimited
   * high-order and the low-order updates. */
#pragma omp parallel for schedule(static)
  for (long i = 0; i < nz_; ++i) {
    if (R->d.limiter == IDP_REF_TARGET) {
      for (int c = 0; c < nc; ++c) out[(long)c * nn + i] = uH[(long)c * nn + i];
      continue;
    }
    if (R->d.limiter == IDP_REF_LOW) {
      for (int c = 0; c < nc; ++c) out[(long)c * nn + i] = uL[(long)c * nn + i];
      continue;
    }
    double m = node_mass(R, i);
    double corr[MAXC] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < dim; ++k) {
      int t, across;
      int a = line_pos(R, i, k, &t);
      if (a < p) {
        long jp = neighbour(R, i, k, +1, &across);
        double ap = fmin(al[i], al[jp]);
        for (int c = 0; c < nc; ++c) corr[c] += ap * rbar[IDX3(k, c, i)];
      }
      if (a > 0) {
        long jm = neighbour(R, i, k, -1, &across);
        double am = fmin(al[i], al[jm]);
        for (int c = 0; c < nc; ++c) corr[c] -= am * rbar[IDX3(k, c, jm)];
      }
    }
    for (int c = 0; c < nc; ++c)
      out[(long)c * nn + i] = uL[(long)c * nn + i] + dt / m * corr[c];
  }

  if (tr) {
    size_t s1 = sizeof(double) * nc * nn, s2 = sizeof(double) * dim * nc * nn;
    size_t s0 = sizeof(double) * nn;
    if (tr->uL) memcpy(tr->uL, uL, s1);
    if (tr->uH) memcpy(tr->uH, uH, s1);
    if (tr->rH) memcpy(tr->rH, rH, s2);
    if (tr->rL) memcpy(tr->rL, rL, s2);
    if (tr->rbar) memcpy(tr->rbar, rbar, s2);
    if (tr->umin) memcpy(tr->umin, umin, s0);
    if (tr->umax) memcpy(tr->umax, umax, s0);
    if (tr->kmin) memcpy(tr->kmin, kmin, s0);
    if (tr->alpha_z) memcpy(tr->alpha_z, az, s0);
    if (tr->alpha) {
      for (long i = 0; i < nn; ++i)
        tr->alpha[i] = R->d.limiter == IDP_REF_TARGET ? 1.0
                     : R->d.limiter == IDP_REF_LOW    ? 0.0
                                                      : al[i];
    }
  }
#undef IDX3
  free(F); free(rH); free(rL); free(rbar); free(uL); free(uH);
  free(umin); free(umax); free(kmin); free(az); free(al);
  return 0;
}

/* ------------------------------------------------------------------ */
/* SSP-RK3 and the time-step bound                                     */
/* ------------------------------------------------------------------ */

int idp_ref_stage(const idp_ref_desc* d, const double* u_n, const double* u_s,
                  double* out, double dt, int stage) {
  static const double A[3] = {0.0, 0.75, 1.0 / 3.0};
  static const double B[3] = {1.0, 0.25, 2.0 / 3.0};
  if (idp_ref_check(d) || stage < 0 || stage > 2 || !u_s || !out) return -1;
  if (out == u_s) return -1;
  if (stage > 0 && !u_n) return -1;
  long n = idp_ref_num_nodes(d) * idp_ref_num_comp(d);
  double* fe = malloc(sizeof(double) * n);
  if (!fe) return -2;
  int rc = idp_ref_fe(d, u_s, fe, dt, NULL);
  if (rc) { free(fe); return rc; }
  if (stage == 0) {
    memcpy(out, fe, sizeof(double) * n);
  } else {
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) out[i] = A[stage] * u_n[i] + B[stage] * fe[i];
  }
  free(fe);
  return 0;
}

int idp_ref_step(const idp_ref_desc* d, double* u, double dt) {
  if (idp_ref_check(d) || !u) return -1;
  long n = idp_ref_num_nodes(d) * idp_ref_num_comp(d);
  double* u1 = malloc(sizeof(double) * n);
  double* u2 = malloc(sizeof(double) * n);
  if (!u1 || !u2) { free(u1); free(u2); return -2; }
  int rc = idp_ref_stage(d, NULL, u, u1, dt, 0);
  if (!rc) rc = idp_ref_stage(d, u, u1, u2, dt, 1);
  if (!rc) rc = idp_ref_stage(d, u, u2, u, dt, 2);
  free(u1);
  free(u2);
  return rc;
}

int idp_ref_max_dt(const idp_ref_desc* dsc, const double* u, double* dt) {
  ref_t Rs, *R = &Rs;
  if (setup(R, dsc) || !u || !dt) return -1;
  double best = INFINITY;
#pragma omp parallel for schedule(static) reduction(min : best)
  for (long i = 0; i < R->nn; ++i) {
    double sum = 0.0;
    for (int k = 0; k < R->d.dim; ++k) {
      for (int sd = -1; sd <= 1; sd += 2) {
        long j;
        double chat, dhat, cv[2];
        if (R->d.metric) graph_coeffs_m(R, u, i, k, sd, &j, cv, &dhat, NULL);
        else graph_coeffs(R, u, i, k, sd, &j, &chat, &dhat, NULL);
        sum += dhat;
      }
    }
    /* eq. cfl-low, reading: the denominator is |dhat_ii| = sum_{j!=i}
     * dhat_ij, which makes every weight of eq. convex-combination >= 0 */
    double dti = node_mass(R, i) / (2.0 * sum);
    if (dti < best) best = dti;
  }
  *dt = best;
  return 0;
}
