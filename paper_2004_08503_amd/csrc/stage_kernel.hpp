// Fused limited SSP-RK stage for gfx950: one workgroup owns a tile of EPB
// consecutive elements, one thread per node, and runs every step of the
// stage out of LDS.  Global memory is touched once per node for the stage
// input (plus the face traces of the 2d neighbouring elements), once for
// u^n on the second and third stages, and once for the output.
//
// Phases (LDS barriers between them):
//   1. load the tile's states and the neighbours' face traces;
//   2. pointwise physics: fluxes F^x, F^y and, for Euler, 1/rho, p, c,
//      p^{-(gamma-1)/(2 gamma)} and K = p rho^{-gamma};
//   3. one work item per subcell face of every line (element faces
//      included): wave-speed bound, low-order flux f^L (eq. lax-friedrichs
//      on the subgrid), bar state of the limited component (eq.
//      bar-states), the entropy bound over the pair, and on interior
//      subcell faces the high-order subcell flux f^H and the antidiffusive
//      flux rbar = s (f^L - f^H);
//   4. per node: u^L, local bounds, Zalesak coefficient and, for Euler,
//      the entropy line search of eq. convex-provisional;
//   5. per node: subcell-face coefficients min(alpha_i, alpha_j), the
//      flux-corrected update (eq. convex-fct) and the RK combination.
//
// The high-order subcell flux uses the cumulative derivative matrix
// Q[a][e] = sum_{c<=a} D[c][e]: on an interior subcell face a+1/2 of a
// line, f^H_{a+1/2} = F_0 + sum_e Q[a][e] F_e is the flux whose
// differences reproduce the strong-form residual (eq. dg-strong), so the
// prefix sums of r^H - r^L of Sec. 4.1.3 become one short contraction per
// face and rbar = s (f^L - f^H) is the difference of the two fluxes.
#pragma once
#include "common.hpp"

namespace idp {

template <int EQ, int DIM, int P, int EPB>
struct Cfg {
  static constexpr int N1 = P + 1;
  static constexpr int NP = DIM == 2 ? N1 * N1 : N1;   // own nodes per element
  static constexpr int TJ = DIM == 2 ? N1 : 1;          // nodes per face trace
  static constexpr int NT = 2 * DIM * TJ;               // trace nodes per element
  static constexpr int NS = NP + NT;                    // LDS slots per element
  static constexpr int NC = is_euler(EQ) ? DIM + 2 : 1;
  // per-slot auxiliaries: Euler 1/rho, p, c, p^-ex, K; EQ_ADVV beta_x, beta_y
  static constexpr int NAUX = is_euler(EQ) ? 5 : EQ == EQ_ADVV ? 2 : 0;
  static constexpr int NAUXF = is_euler(EQ) ? 4 : NAUX;   // those fluxes and speeds read
  static constexpr int NFL = P + 2;                     // subcell faces per line
  static constexpr int NL = DIM == 2 ? N1 : 1;          // lines per direction
  static constexpr int NF = NFL * NL;                   // faces per direction
  static constexpr int BS = ((EPB * NP + 63) / 64) * 64;
  // phase 3 work: per direction, the element faces (f = 0 or p + 1) and the
  // interior faces form two groups, each cut into chunks of 64 items; a wave
  // takes whole chunks, so each of its passes runs one body specialised for
  // a direction and a face kind
  static constexpr int NW = BS / 64;                   // waves per workgroup
  static constexpr int GE = EPB * 2 * NL;              // element-face items per direction
  static constexpr int GI = EPB * P * NL;              // interior items per direction
  static constexpr int CE = (GE + 63) / 64;            // chunks per group
  static constexpr int CI = (GI + 63) / 64;
  static constexpr int NCHUNK = DIM * (CE + CI);
  static constexpr int NITEM = (NCHUNK + NW - 1) / NW;  // chunks per wave
  // region A: phase 1-2 results, read in phase 3 (fluxes of own nodes only:
  // the face-trace fluxes are formed where a face needs them)
  static constexpr int A_U = 0;
  static constexpr int A_X = A_U + NC * EPB * NS;
  static constexpr int A_F = A_X + NAUX * EPB * NS;
  static constexpr int A_END = A_F + DIM * NC * EPB * NP;
  // region B (aliases A): phase 3 results, read in phases 4-5
  static constexpr int B_FL = 0;
  static constexpr int B_RB = B_FL + DIM * NC * EPB * NF;
  static constexpr int B_UB = B_RB + DIM * NC * EPB * NF;
  static constexpr int B_END = B_UB + DIM * EPB * NF;
  // region C: Euler search data, written once the low-order fluxes are
  // consumed; it overwrites them where it fits
  static constexpr int C_SIZE = is_euler(EQ) ? (NC + 2 + DIM) * EPB * NP : 0;
  static constexpr int C_UL = C_SIZE <= DIM * NC * EPB * NF ? B_FL : B_END;   // [NC][EPB*NP]
  static constexpr int C_KM = C_UL + (is_euler(EQ) ? NC * EPB * NP : 0);
  static constexpr int C_AZ = C_KM + (is_euler(EQ) ? EPB * NP : 0);   // bound U of the node
  static constexpr int C_LIST = C_AZ + (is_euler(EQ) ? EPB * NP : 0);  // int[2*DIM*EPB*NP]
  static constexpr int C_END = C_LIST + (is_euler(EQ) ? DIM * EPB * NP : 0);
  static constexpr int AB0 = A_END > B_END ? A_END : B_END;
  static constexpr int AB = AB0 > C_END ? AB0 : C_END;
  static constexpr int S_AL = AB;                       // nodal alpha
  static constexpr int S_W = S_AL + EPB * NP;           // weights
  static constexpr int S_Q = S_W + N1;                  // cumulative D
  static constexpr int S_IW = S_Q + P * N1;             // 1/w
  static constexpr int S_M = S_IW + N1;                 // nodal -> modal map [k][a]
  static constexpr int S_NK = S_M + N1 * N1;            // Legendre norms
  static constexpr int S_LN = S_NK + N1;                // search list length (int)
  static constexpr int LDS = S_LN + 1;
  static_assert(LDS * 8 <= 160 * 1024, "tile does not fit in LDS");
};

// Workgroups are dealt round-robin to the eight XCDs; give every XCD a
// contiguous range of tiles so that the face traces a tile reads from the
// element rows above and below were fetched into the same XCD's L2.
__device__ inline int xcd_tile(int b, int nb) {
  const int x = b & 7, i = b >> 3;
  const int q = nb >> 3, r = nb & 7;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// Global node index of trace t of element e: face 0/1 = the x-neighbours'
// facing node columns, 2/3 = the y-neighbours' facing rows (periodic).
template <int DIM, int P>
__device__ inline long long trace_node(int e, int t, int nx, int ny) {
  constexpr int N1 = P + 1;
  const int ex = e % nx, ey = e / nx;
  if constexpr (DIM == 1) {
    const int exn = t == 0 ? (ex == 0 ? nx - 1 : ex - 1) : (ex == nx - 1 ? 0 : ex + 1);
    return (long long)exn * N1 + (t == 0 ? P : 0);
  } else {
    constexpr int NP = N1 * N1;
    const int face = t / N1, j = t - face * N1;
    int exn = ex, eyn = ey, loc;
    if (face == 0) { exn = ex == 0 ? nx - 1 : ex - 1; loc = j * N1 + P; }
    else if (face == 1) { exn = ex == nx - 1 ? 0 : ex + 1; loc = j * N1; }
    else if (face == 2) { eyn = ey == 0 ? ny - 1 : ey - 1; loc = P * N1 + j; }
    else { eyn = ey == ny - 1 ? 0 : ey + 1; loc = j; }
    return ((long long)eyn * nx + exn) * NP + loc;
  }
}

// Whether trace t of element e lies on an open side of the box; if so the
// side, the boundary node's index along that side and the global index of
// the element's own node at that point.
template <int DIM, int P>
__device__ inline bool boundary_trace(int e, int t, int nx, int ny, int open, int* side, int* q,
                                      long long* own) {
  constexpr int N1 = P + 1;
  const int face = DIM == 2 ? t / N1 : t, j = DIM == 2 ? t - face * N1 : 0;
  const int k = face >> 1;
  if (!((open >> k) & 1)) return false;
  const int ex = e % nx, ey = e / nx;
  const bool edge = k == 0 ? ((face & 1) ? ex == nx - 1 : ex == 0)
                           : ((face & 1) ? ey == ny - 1 : ey == 0);
  if (!edge) return false;
  *side = face;
  *q = DIM == 1 ? 0 : (k == 0 ? ey * N1 + j : ex * N1 + j);
  if constexpr (DIM == 1) {
    *own = (long long)e * N1 + ((face & 1) ? P : 0);
  } else {
    const int loc = face == 0 ? j * N1 : face == 1 ? j * N1 + P : face == 2 ? j : P * N1 + j;
    *own = (long long)e * (N1 * N1) + loc;
  }
  return true;
}

// The advection velocity / Burgers direction component k, selected between
// two values already loaded (a select between two fields of the argument
// struct could otherwise become a load from a run-time address, which moves
// a local copy of the struct to scratch memory).
__device__ inline double vel_k(int k, const Phys& ph) {
  const unsigned long long v0 = __double_as_longlong(ph.vel0), v1 = __double_as_longlong(ph.vel1);
  return __longlong_as_double(k == 0 ? v0 : v1);
}

__device__ inline double ipow(double x, int n) {
  double r = 1.0;
  while (n) {
    if (n & 1) r *= x;
    x *= x;
    n >>= 1;
  }
  return r;
}

template <int N>
__device__ inline double ipow_c(double x) {
  if constexpr (N == 1) return x;
  else if constexpr (N % 2 == 0) { const double h = ipow_c<N / 2>(x); return h * h; }
  else return x * ipow_c<N - 1>(x);
}

// x^(-1/N) in binary64 for x > 0, without branches.  Range reduction:
// x = m 2^e with m in [1/2, 1) and e = N q + r (0 <= r < N), so that
// x^(-1/N) = 2^-q (m 2^r)^(-1/N) with m 2^r in [1/2, 2^(N-1)).  On that
// range the single-precision log2/exp2 seed is within 1e-6 (relative), and
// two Newton steps y <- y (1 + (1 - x y^N)/N) bring the error to
// ((N+1)/2)^3 1e-24, below the binary64 rounding of the last step.
// Non-positive, infinite or NaN x give NaN or infinity.
template <int N>
__device__ inline double inv_root(double x) {
  int e;
  const double m = frexp(x, &e);
  const int q = (e + 1100 * N) / N - 1100;   // floor(e / N) for e >= -1100 N
  const double xr = ldexp(m, e - N * q);
  double y = (double)__builtin_amdgcn_exp2f(__builtin_amdgcn_logf((float)xr) * (-1.0f / N));
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double r = fma(-xr, ipow_c<N>(y), 1.0);
    y = fma(y * r, 1.0 / N, y);
  }
  return ldexp(y, -q);
}

// Euler auxiliaries of one state: X = (1/rho, p, c, p^-(gamma-1)/(2gamma),
// K = p rho^-gamma) (K only when WITHK).  For gamma = 1 + 2/n (GN = n = 5:
// 7/5, n = 3: 5/3) every fractional power is an integer power of
// z = rho^(-1/n) or of p^(-1/(n+2)): 1/rho = z^n, K = p z^(n+2); otherwise
// pow and a division are used.  Without K (the time-step pass) 1/rho is a
// plain division, cheaper than the root.
template <int DIM, int GN, bool WITHK = true>
__device__ inline void euler_aux(const double* U, const Phys& ph, double* X, bool& bad) {
  double rinv, z = 0.0;
  if constexpr (GN > 0 && WITHK) {   // z = rho^(-1/n) also gives K below
    z = inv_root<GN>(U[0]);
    rinv = ipow_c<GN>(z);
  } else {
    rinv = 1.0 / U[0];
  }
  double mm = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) mm += U[1 + k] * U[1 + k];
  const double p = (ph.gamma - 1.0) * (U[DIM + 1] - 0.5 * mm * rinv);
  bad = !(U[0] > 0.0) || !(p > 0.0);
  X[0] = rinv;
  X[1] = p;
  X[2] = sqrt(ph.gamma * p * rinv);
  if constexpr (GN > 0) {
    X[3] = inv_root<GN + 2>(p);
    if constexpr (WITHK) X[4] = p * ipow_c<GN + 2>(z);
  } else {
    X[3] = pow(p, -ph.ex);
    if constexpr (WITHK) X[4] = p * pow(U[0], -ph.gamma);
  }
}

// flux in direction k of one state (X: Euler auxiliaries)
template <int EQ, int DIM>
__device__ inline void flux_k(int k, const double* U, const double* X, const Phys& ph, double* F) {
  if constexpr (EQ == EQ_ADV) {
    F[0] = (vel_k(k, ph)) * U[0];
  } else if constexpr (EQ == EQ_ADVV) {
    F[0] = X[k] * U[0];
  } else if constexpr (EQ == EQ_BURG) {
    F[0] = 0.5 * U[0] * U[0] * (vel_k(k, ph));
  } else {
    const double vk = U[1 + k] * X[0];
    const double p = X[1];
    F[0] = U[1 + k];
#pragma unroll
    for (int l = 0; l < DIM; ++l) F[1 + l] = U[1 + l] * vk + (l == k ? p : 0.0);
    F[DIM + 1] = vk * (U[DIM + 1] + p);
  }
}

// The two-rarefaction bound of the Euler wave speeds (Guermond and Popov,
// J. Comput. Phys. 2016, valid for 1 < gamma <= 5/3) from the normal
// velocities, pressures, sound speeds and p^-(gamma-1)/(2 gamma) of the
// left and right states.
template <int GN>
__device__ inline double euler_lambda(double vl, double vr, double pl, double pr, double cl, double cr,
                                      double xl3, double xr3, const Phys& ph) {
  const double g = ph.gamma;
  double num = cl + cr - 0.5 * (g - 1.0) * (vr - vl);
  num = num < 0.0 ? 0.0 : num;
  const double den = cl * xl3 + cr * xr3;
  const double base = num / den;
  double pstar, ipl, ipr;
  if constexpr (GN > 0) {  // 2 gamma/(gamma-1) = n + 2; 1/p = (p^-1/(n+2))^(n+2)
    pstar = ipow_c<GN + 2>(base);
    ipl = ipow_c<GN + 2>(xl3);
    ipr = ipow_c<GN + 2>(xr3);
  } else {
    pstar = ph.inv_ex_int ? ipow(base, ph.inv_ex_int) : pow(base, ph.inv_ex);
    ipl = 1.0 / pl;
    ipr = 1.0 / pr;
  }
  const double fac = (g + 1.0) / (2.0 * g);
  const double lam_l = vl - cl * sqrt(1.0 + fac * fmax(pstar - pl, 0.0) * ipl);
  const double lam_r = vr + cr * sqrt(1.0 + fac * fmax(pstar - pr, 0.0) * ipr);
  return fmax(fmax(-lam_l, 0.0), fmax(lam_r, 0.0));
}

// Upper bound of the maximum wave speed of the Riemann problem (UL | UR)
// along +e_k.  Euler: the two-rarefaction pressure bound (Guermond and
// Popov, J. Comput. Phys. 2016), valid for 1 < gamma <= 5/3.
template <int EQ, int DIM>
__device__ inline double lambda_k(int k, const double* UL, const double* XL, const double* UR,
                                  const double* XR, const Phys& ph) {
  if constexpr (EQ == EQ_ADV) {
    return fabs(vel_k(k, ph));
  } else if constexpr (EQ == EQ_ADVV) {
    // Sec. 3.3: dhat_ij = max(|chat_ij . beta_i|, |chat_ji . beta_j|)
    return fmax(fabs(XL[k]), fabs(XR[k]));
  } else if constexpr (EQ == EQ_BURG) {
    return fmax(fabs(UL[0]), fabs(UR[0])) * fabs(vel_k(k, ph));
  } else {
    const double vl = UL[1 + k] * XL[0], vr = UR[1 + k] * XR[0];
    return euler_lambda<gn_of(EQ)>(vl, vr, XL[1], XR[1], XL[2], XR[2], XL[3], XR[3], ph);
  }
}

// lambda_k of an element face from its own-side state O and its trace T:
// side 1 is the element's right face (O on the left), side 0 its left face
// (T on the left).  The Euler bound selects the values it reads into
// left/right order and then forms the same expressions as lambda_k (so the
// result is identical to the bound of the pair in that order).
template <int EQ, int DIM>
__device__ inline double lambda_face(int k, const double* UO, const double* XO, const double* UT,
                                     const double* XT, int side, const Phys& ph) {
  if constexpr (is_euler(EQ)) {
    const bool r = side != 0;
    double ul[DIM + 2] = {}, ur[DIM + 2] = {}, xl[4], xr[4];
    ul[1 + k] = r ? UO[1 + k] : UT[1 + k];
    ur[1 + k] = r ? UT[1 + k] : UO[1 + k];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      xl[q] = r ? XO[q] : XT[q];
      xr[q] = r ? XT[q] : XO[q];
    }
    return lambda_k<EQ, DIM>(k, ul, xl, ur, xr, ph);
  } else {
    // symmetric in the two states
    return lambda_k<EQ, DIM>(k, UO, XO, UT, XT, ph);
  }
}

// Phi(V) = rho e - K_min rho^gamma / (gamma - 1) along V = uL + t P, with
// its t-derivative.  Phi >= 0 with rho > 0 is the specific-entropy minimum
// principle of Sec. 4.3; Phi is concave.
struct PhiVal {
  double rho, phi, dphi;
};

template <int DIM, int GN>
__device__ inline PhiVal phi_at(double t, const double* uL, const double* P, double kmin,
                                const Phys& ph) {
  // straight-line code (no branches), so that independent evaluations
  // interleave; a non-positive density gives phi = -infinity
  PhiVal r;
  r.rho = fma(t, P[0], uL[0]);
  const bool pos = r.rho > 0.0;
  const double rho = pos ? r.rho : 1.0;
  const double g = ph.gamma;
  double rinv, rg;
  if constexpr (GN > 0) {  // z = rho^(-1/n): 1/rho = z^n, rho^gamma = rho^2 z^(n-2)
    const double z = inv_root<GN>(rho);
    rinv = ipow_c<GN>(z);
    rg = (rho * rho) * ipow_c<GN - 2>(z);
  } else {
    rinv = 1.0 / rho;
    rg = pow(rho, g);
  }
  double mm = 0.0, mp = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const double m = fma(t, P[1 + k], uL[1 + k]);
    mm += m * m;
    mp += m * P[1 + k];
  }
  const double E = fma(t, P[DIM + 1], uL[DIM + 1]);
  const double kg = kmin / (g - 1.0);
  const double phi = E - 0.5 * mm * rinv - kg * rg;
  const double dphi = P[DIM + 1] - mp * rinv + 0.5 * mm * rinv * rinv * P[0] - kg * g * rg * rinv * P[0];
  r.phi = pos ? phi : -INFINITY;
  r.dphi = pos ? dphi : 0.0;
  return r;
}

__device__ inline bool admissible(const PhiVal& e) { return e.rho > 0.0 && e.phi >= 0.0; }

// Whether V = uL + t P is admissible beyond doubt, from integer powers
// only; false means "not certain" and leaves the decision to phi_at.  For
// gamma = 1 + 2/n and rho > 0, with W = rho (rho e) = E rho - |m|^2 / 2 and
// w = W (gamma - 1) / K_min:  Phi >= 0  <=>  w^n >= rho^(2n+2).  W is
// lowered by 32 ulps of the terms it is formed from (twice a bound on its
// own rounding, and on that of a direct evaluation of rho e), the powers
// carry a relative margin of 1e-12, and densities or w outside the ranges
// where the powers neither overflow nor underflow are never certain.  For
// other gamma the test is the direct evaluation itself.
template <int DIM, int GN>
__device__ inline bool surely_admissible(double t, const double* uL, const double* P, double kmin,
                                         double ikg, const Phys& ph) {
  if constexpr (GN == 5 || GN == 3) {
    const double rho = fma(t, P[0], uL[0]);
    double mm = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const double m = fma(t, P[1 + k], uL[1 + k]);
      mm = fma(m, m, mm);
    }
    const double E = fma(t, P[DIM + 1], uL[DIM + 1]);
    const double W = fma(E, rho, -0.5 * mm);
    const double err = 0x1p-48 * fma(fabs(E), rho, 0.5 * mm);
    const double w = (W - err) * ikg;
    const double r2 = rho * rho, r4 = r2 * r2;
    const double rhs = GN == 5 ? r4 * r4 * r4 : r4 * r4;   // rho^12 or rho^8
    const double lhs = ipow_c<GN>(w);
    return rho >= 1e-20 && rho <= 1e20 && w >= 1e-50 && w <= 1e50 && lhs >= rhs * (1.0 + 1e-12);
  } else {
    return admissible(phi_at<DIM, GN>(t, uL, P, kmin, ph));
  }
}

// sup { t in [0, U] : uL + t P admissible }, for uL admissible.  U is the
// node's alpha for a subcell face, and for elementwise limiting the
// tangent bound from alpha (tang = true).
//  - the first point is U itself: an admissible U is the answer; otherwise
//    it is the first infeasible end (for a subcell face, the exact value
//    at alpha that the screen could not certify);
//  - then Newton steps from the infeasible end hi (Phi is concave wherever
//    rho > 0, so the tangent at hi cuts zero at or above the root), each a
//    single evaluation; a tangent step that lands admissible is within
//    rounding of the root and ends the search; without a usable tangent
//    (rho <= 0 at hi), or after three Newton steps in a row that do not
//    halve (convergence slower than quadratic), one bisection; once the
//    Newton step is below half the tolerance, hi sits on the root and the
//    next points are probes under hi at half the tolerance, doubling the
//    distance after each inadmissible probe;
//  - the search stops once the bracket is narrower than 1e-15 or than
//    RTOL max|uL| / max(|P|, pscale), and returns the admissible end.
// The node's t scales more than this P: a subcell node's coefficient limits
// every face of the node (through min(alpha_i, alpha_j)), so pscale is the
// largest |P| over the node's faces, and the answer moves every face's
// contribution to the state by less than RTOL of its largest component
// from any point of the bracket, the supremum included.  RTOL: 1e-14 for
// subcell faces; 1e-16 for elementwise limiting, where one node's t is
// applied to every node of the element, so that nodes of other scales (the
// small momentum of a gas near rest next to a node of large energy) still
// land within rounding.
template <int DIM, int GN, int RTOL_EXP>
__device__ double entropy_root(const double* uL, const double* P, double U, bool tang, double kmin,
                               double pscale, const Phys& ph) {
  constexpr double RTOL = RTOL_EXP == 16 ? 1e-16 : 1e-14;
  static_assert(RTOL_EXP == 14 || RTOL_EXP == 16, "search tolerance 1e-14 or 1e-16");
  double us = 0.0, ps = pscale;
#pragma unroll
  for (int c = 0; c < DIM + 2; ++c) {
    us = fmax(us, fabs(uL[c]));
    ps = fmax(ps, fabs(P[c]));
  }
  const double tol = fmax(1e-15, RTOL * us / ps);
  double lo = 0.0, hi = U, fhi = -INFINITY, dhi = 0.0, rhi = 0.0;
  double t = U, prev = INFINITY, probe = 0.5 * tol;
  int slow = 0;
  for (int it = 0; it < 64; ++it) {
    const PhiVal e = phi_at<DIM, GN>(t, uL, P, kmin, ph);
    if (admissible(e)) {
      if (tang || t >= U) return t;
      lo = t;
    } else {
      hi = t;
      fhi = e.phi;
      dhi = e.dphi;
      rhi = e.rho;
    }
    if (!(hi - lo > tol)) break;
    tang = false;
    if (rhi > 0.0 && dhi < 0.0) {
      const double step = fhi / dhi;  // the Newton step from hi, >= 0
      if (step < 0.5 * tol) {         // hi sits on the root: probe under it
        t = hi - probe;
        probe *= 2.0;
      } else if (slow >= 3) {
        t = 0.5 * (lo + hi);
        slow = 0;
      } else {
        t = hi - step;
        tang = true;
        slow = step > 0.5 * prev ? slow + 1 : 0;
        prev = step;
      }
    } else {
      t = 0.5 * (lo + hi);
    }
    if (!(t > lo && t < hi)) {
      t = 0.5 * (lo + hi);
      tang = false;
    }
  }
  return lo;
}

__device__ inline const Phys& ph_of(const StageArgs& A) { return A.ph; }

// local slot of the node at position pos of line l in direction k
template <int DIM, int P>
__device__ inline int own_slot(int k, int l, int pos) {
  if constexpr (DIM == 1) return pos;
  return k == 0 ? l * (P + 1) + pos : pos * (P + 1) + l;
}

// One element face of a tile for phase 3: item -> element le, line l and
// side (0: f = 0, the trace on the left; 1: f = p + 1, the trace on the
// right).  Writes the low-order flux, the bar state of the limited
// component and the face's index in the phase-3 arrays (o < 0: no face).
template <int EQ, int DIM, int P, int EPB, int K>
__device__ __forceinline__ void element_face(const double* lds, const Phys& ph, int item, int nel,
                                             double* FLo, double& UBo, int& o) {
  using C = Cfg<EQ, DIM, P, EPB>;
  constexpr int NC = C::NC, NS = C::NS, NP = C::NP, NL = C::NL;
  constexpr int NX = C::NAUX > 0 ? C::NAUX : 1;
  const int le = item / (2 * NL);
  if (le >= nel) return;
  const int r = item - le * (2 * NL);
  const int l = r >> 1, side = r & 1;
  const int base = le * NS;
  const int st = base + NP + (2 * K + side) * C::TJ + l;             // trace slot
  const int so = base + own_slot<DIM, P>(K, l, side ? P : 0);       // own slot
  double UO[NC], UT[NC], XO[NX], XT[NX], FO[NC], FT[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    UO[c] = lds[C::A_U + c * EPB * NS + so];
    UT[c] = lds[C::A_U + c * EPB * NS + st];
    FO[c] = lds[C::A_F + (K * NC + c) * EPB * NP + le * NP + (so - base)];
  }
#pragma unroll
  for (int q = 0; q < C::NAUXF; ++q) {
    XO[q] = lds[C::A_X + q * EPB * NS + so];
    XT[q] = lds[C::A_X + q * EPB * NS + st];
  }
  flux_k<EQ, DIM>(K, UT, XT, ph, FT);
  const double lam = lambda_face<EQ, DIM>(K, UO, XO, UT, XT, side, ph);
  // (F_L + F_R) / 2 - lam (U_R - U_L) / 2 with U_R - U_L = sg (U_T - U_O),
  // sg = +-1 (exact).  The trace flux enters its sums rounded, not fused
  // into them, as an interior face's fluxes do.
  const double sg = side ? 1.0 : -1.0;
  double fs[NC], df0;
  {
#pragma clang fp contract(off)
#pragma unroll
    for (int c = 0; c < NC; ++c) fs[c] = FO[c] + FT[c];
    df0 = FT[0] - FO[0];
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) FLo[c] = 0.5 * fs[c] - 0.5 * lam * (sg * (UT[c] - UO[c]));
  const double avg = 0.5 * (UO[0] + UT[0]);
  UBo = lam > 0.0 ? avg - (sg * df0) / (2.0 * lam) : avg;
  o = le * C::NF + l * C::NFL + (side ? P + 1 : 0);
}

// One interior subcell face (1 <= f <= p) of a tile for phase 3: also the
// high-order subcell flux and the antidiffusive flux.
template <int EQ, int DIM, int P, int EPB, int K>
__device__ __forceinline__ void interior_face(const double* lds, const Phys& ph, const Solve& S, int item,
                                              int nel, double* FLo, double* RBo, double& UBo, int& o) {
  using C = Cfg<EQ, DIM, P, EPB>;
  constexpr int NC = C::NC, NS = C::NS, NP = C::NP, NL = C::NL, N1 = C::N1;
  constexpr int NX = C::NAUX > 0 ? C::NAUX : 1;
  const int le = item / (P * NL);
  if (le >= nel) return;
  const int r = item - le * (P * NL);
  const int l = r / P;
  const int f = 1 + (r - l * P);
  const int base = le * NS;
  const int sl = base + own_slot<DIM, P>(K, l, f - 1);
  const int sr = base + own_slot<DIM, P>(K, l, f);
  double UL[NC], UR[NC], FL[NC], FR[NC], XL[NX], XR[NX];
  const double* Fo = lds + C::A_F + K * NC * EPB * NP + le * NP;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    UL[c] = lds[C::A_U + c * EPB * NS + sl];
    UR[c] = lds[C::A_U + c * EPB * NS + sr];
    FL[c] = Fo[c * EPB * NP + sl - base];
    FR[c] = Fo[c * EPB * NP + sr - base];
  }
#pragma unroll
  for (int q = 0; q < C::NAUXF; ++q) {
    XL[q] = lds[C::A_X + q * EPB * NS + sl];
    XR[q] = lds[C::A_X + q * EPB * NS + sr];
  }
  const double lam = lambda_k<EQ, DIM>(K, UL, XL, UR, XR, ph);
#pragma unroll
  for (int c = 0; c < NC; ++c) FLo[c] = 0.5 * (FL[c] + FR[c]) - 0.5 * lam * (UR[c] - UL[c]);
  const double avg = 0.5 * (UL[0] + UR[0]);
  UBo = lam > 0.0 ? avg - (FR[0] - FL[0]) / (2.0 * lam) : avg;
  const double sc = DIM == 2 ? lds[C::S_W + l] * (K == 0 ? S.hy : S.hx) : 1.0;
  const double* q = lds + C::S_Q + (f - 1) * N1;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double* Fl = Fo + c * EPB * NP;
    double fh = Fl[own_slot<DIM, P>(K, l, 0)];
#pragma unroll
    for (int e = 0; e <= P; ++e) fh += q[e] * Fl[own_slot<DIM, P>(K, l, e)];
    RBo[c] = sc * (FLo[c] - fh);
  }
  o = le * C::NF + l * C::NFL + f;
}

// Phase-3 chunk ch (wave-uniform) of a tile: chunks of the element-face
// groups (direction 0, then 1) come first, then those of the interior
// groups; lane picks the item within the chunk.
template <int EQ, int DIM, int P, int EPB>
__device__ __forceinline__ void face_chunk(const double* lds, const Phys& ph, const Solve& S, int ch, int lane,
                                           int nel, double* FLo, double* RBo, double& UBo, int& o) {
  using C = Cfg<EQ, DIM, P, EPB>;
  if (ch < DIM * C::CE) {
    const int k = ch / C::CE;
    const int item = (ch - k * C::CE) * 64 + lane;
    if (k == 0) element_face<EQ, DIM, P, EPB, 0>(lds, ph, item, nel, FLo, UBo, o);
    else if constexpr (DIM == 2) element_face<EQ, DIM, P, EPB, 1>(lds, ph, item, nel, FLo, UBo, o);
  } else if (ch < C::NCHUNK) {
    const int c2 = ch - DIM * C::CE;
    const int k = c2 / C::CI;
    const int item = (c2 - k * C::CI) * 64 + lane;
    if (k == 0) interior_face<EQ, DIM, P, EPB, 0>(lds, ph, S, item, nel, FLo, RBo, UBo, o);
    else if constexpr (DIM == 2) interior_face<EQ, DIM, P, EPB, 1>(lds, ph, S, item, nel, FLo, RBo, UBo, o);
  }
}

// direction of phase-3 chunk ch
template <int EQ, int DIM, int P, int EPB>
__device__ inline int chunk_dir(int ch) {
  using C = Cfg<EQ, DIM, P, EPB>;
  if constexpr (DIM == 1) return 0;
  return ch < DIM * C::CE ? ch / C::CE : (ch - DIM * C::CE) / C::CI;
}

// ----------------------------------------------------------------------
// phases 1-2 shared by the stage and the time-step kernels
// ----------------------------------------------------------------------
template <int EQ, int DIM, int P, int EPB, bool FLUX>
__device__ inline void load_tile(double* lds, const double* __restrict__ u, long long nn, int e0,
                                 int ne, int nx, int ny, const Phys& ph, const Bnd& bnd, double* Uown,
                                 unsigned int* bad_flag) {
  using C = Cfg<EQ, DIM, P, EPB>;
  constexpr int NC = C::NC, NS = C::NS, NP = C::NP, NT = C::NT;
  const int tid = threadIdx.x;
  const int nel = min(EPB, ne - e0);
  bool bad = false;
  // own nodes: one per thread, contiguous in global memory
  if (tid < nel * NP) {
    const int le = tid / NP, s = tid - le * NP;
    const long long g = (long long)e0 * NP + tid;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      Uown[c] = u[c * nn + g];
      lds[C::A_U + c * EPB * NS + le * NS + s] = Uown[c];
    }
  }
  // face traces of the neighbouring elements, or exterior states on the
  // open sides of the box
  for (int t = tid; t < nel * NT; t += C::BS) {
    const int le = t / NT, j = t - le * NT;
    int side, q;
    long long own;
    if (bnd.open && boundary_trace<DIM, P>(e0 + le, j, nx, ny, bnd.open, &side, &q, &own)) {
      double v[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) v[c] = u[c * nn + own];
      const int ty = bnd.type[side][q];
      if (ty == BC_STATE && bnd.state[side]) {
        const int n = DIM == 1 ? 1 : (side < 2 ? ny : nx) * (P + 1);
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = bnd.state[side][c * n + q];
      } else if (ty == BC_SLIP && is_euler(EQ)) {
        v[1 + (side >> 1)] = -v[1 + (side >> 1)];
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) lds[C::A_U + c * EPB * NS + le * NS + NP + j] = v[c];
    } else {
      const long long g = trace_node<DIM, P>(e0 + le, j, nx, ny);
#pragma unroll
      for (int c = 0; c < NC; ++c) lds[C::A_U + c * EPB * NS + le * NS + NP + j] = u[c * nn + g];
    }
  }
  __syncthreads();
  // pointwise physics on every slot: the tile's own slots first, then its
  // face traces, so that most waves agree on forming their slot's fluxes
  for (int i = tid; i < nel * NS; i += C::BS) {
    int le, s;
    if (i < nel * NP) {
      le = i / NP;
      s = i - le * NP;
    } else {
      const int j = i - nel * NP;
      le = j / NT;
      s = NP + (j - le * NT);
    }
    const int t = le * NS + s;
    double U[NC], X[C::NAUX > 0 ? C::NAUX : 1];
#pragma unroll
    for (int c = 0; c < NC; ++c) U[c] = lds[C::A_U + c * EPB * NS + t];
    if constexpr (is_euler(EQ)) {
      bool b;
      euler_aux<DIM, gn_of(EQ), FLUX>(U, ph, X, b);
      bad |= b;
#pragma unroll
      for (int q = 0; q < (FLUX ? C::NAUX : C::NAUXF); ++q) lds[C::A_X + q * EPB * NS + t] = X[q];
    } else if constexpr (EQ == EQ_ADVV) {
      // the velocity of the slot's node: beta_x of its row, beta_y of its
      // column (own slot or face trace; an exterior state sits at the
      // element's own face node)
      int side, q;
      long long g;
      if (s < NP)
        g = (long long)(e0 + le) * NP + s;
      else if (!(bnd.open && boundary_trace<DIM, P>(e0 + le, s - NP, nx, ny, bnd.open, &side, &q, &g)))
        g = trace_node<DIM, P>(e0 + le, s - NP, nx, ny);
      const int e = (int)(g / NP), sn = (int)(g - (long long)e * NP);
      const int ey = e / nx, ex = e - ey * nx;
      X[0] = ph.vrow[ey * C::N1 + sn / C::N1];
      X[1] = ph.vcol[ex * C::N1 + sn % C::N1];
      lds[C::A_X + t] = X[0];
      lds[C::A_X + EPB * NS + t] = X[1];
    }
    if constexpr (FLUX) {
      if (s < NP) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          double F[NC];
          flux_k<EQ, DIM>(k, U, X, ph, F);
#pragma unroll
          for (int c = 0; c < NC; ++c) lds[C::A_F + (k * NC + c) * EPB * NP + le * NP + s] = F[c];
        }
      }
    }
  }
  if (bad && bad_flag) atomicOr(bad_flag, 1u);
}

// copy the per-degree tables into LDS (sm, snk: the modal map and norms,
// or NULL)
template <int P>
__device__ inline void load_tables(double* sw, double* sq, double* siw, double* sm, double* snk,
                                   const Tables& T, int nthreads) {
  constexpr int N1 = P + 1;
  for (int t = threadIdx.x; t < N1; t += nthreads) {
    sw[t] = T.w[t];
    siw[t] = T.iw[t];
    if (snk) snk[t] = T.nk[t];
  }
  for (int t = threadIdx.x; t < P * N1; t += nthreads) sq[t] = T.Q[t];
  if (sm)
    for (int t = threadIdx.x; t < N1 * N1; t += nthreads) sm[t] = T.M[t];
}

// Subcell-resolution smoothness factor of every element of the tile
// (Sec. 4.4) from the limited component in LDS (own slots): modal
// coefficients c = M u (tensor product in 2-D), the energy fraction of the
// modes of degree p in any variable, s_K = log10 of it and eps_K on the
// ramp 1/2 + 1/2 sin(pi (s_K - s0)/2) between s0 - 1 (0) and s0 + 1 (1).
// An element whose polynomial is zero is smooth (0).  Uses scr (2-D:
// 2 EPB (p+1) + EPB doubles, 1-D: EPB) as scratch; returns the factor of the
// calling thread's element (own nodes), 1 for the others.  Sums run in a
// fixed order, so the result does not depend on the launch.
template <int DIM, int P, int EPB, int NS, int BS>
__device__ inline double smoothness_tile(const double* u0, const double* M, const double* nk, double s0,
                                         int nel, double* scr) {
  // no multiply-add contraction: the result must not depend on how the
  // kernel that inlines this is compiled (plain and batched agree bitwise)
#pragma clang fp contract(off)
  constexpr int N1 = P + 1, NP = DIM == 2 ? N1 * N1 : N1;
  const int tid = threadIdx.x;
  double* tot_h = scr;                                  // [2][EPB*N1] row sums (2-D)
  double* eps_e = scr + (DIM == 2 ? 2 * EPB * N1 : 0);  // [EPB]
  if constexpr (DIM == 2) {
    // thread (element, x-mode k): the k-th x-modes of every row, then their
    // y-transforms, squared and weighted
    if (tid < nel * N1) {
      const int le = tid / N1, k = tid - le * N1;
      const double* ue = u0 + le * NS;
      double t[N1];
#pragma unroll
      for (int b = 0; b < N1; ++b) {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < N1; ++a) acc += M[k * N1 + a] * ue[b * N1 + a];
        t[b] = acc;
      }
      double tot = 0.0, hi = 0.0;
#pragma unroll
      for (int l = 0; l < N1; ++l) {
        double c = 0.0;
#pragma unroll
        for (int b = 0; b < N1; ++b) c += M[l * N1 + b] * t[b];
        const double e = c * c * nk[k] * nk[l];
        tot += e;
        if (k == P || l == P) hi += e;
      }
      tot_h[tid] = tot;
      tot_h[EPB * N1 + tid] = hi;
    }
    __syncthreads();
  }
  if (tid < nel) {
    double tot = 0.0, hi = 0.0;
    if constexpr (DIM == 2) {
#pragma unroll
      for (int k = 0; k < N1; ++k) {
        tot += tot_h[tid * N1 + k];
        hi += tot_h[EPB * N1 + tid * N1 + k];
      }
    } else {
      const double* ue = u0 + tid * NS;
#pragma unroll
      for (int k = 0; k < N1; ++k) {
        double c = 0.0;
#pragma unroll
        for (int a = 0; a < N1; ++a) c += M[k * N1 + a] * ue[a];
        const double e = c * c * nk[k];
        tot += e;
        if (k == P) hi += e;
      }
    }
    double eps = 0.0;
    if (tot > 0.0) {
      const double sk = log10(hi / tot);
      eps = sk < s0 - 1.0 ? 0.0 : (sk > s0 + 1.0 ? 1.0 : 0.5 + 0.5 * sin(M_PI * 0.5 * (sk - s0)));
    }
    eps_e[tid] = eps;
  }
  __syncthreads();
  return tid < nel * NP ? eps_e[tid / NP] : 1.0;
}

// ----------------------------------------------------------------------
// the fused stage kernel
// ----------------------------------------------------------------------
// One tile of EPB elements of one solve, run by one workgroup of C::BS
// threads on C::LDS doubles of LDS, with the degree tables T.  Shared by
// the plain kernel (the tiles of one solve) and the batched work-list
// kernel (the tiles of every solve of one degree).
template <int EQ, int DIM, int P, int EPB>
__device__ __forceinline__ void stage_tile(double* lds, const StageArgs& A, const Tables& T, const Bnd& bnd,
                                           int tile) {
  using C = Cfg<EQ, DIM, P, EPB>;
  constexpr int NC = C::NC, NS = C::NS, NP = C::NP, NF = C::NF, NFL = C::NFL, N1 = C::N1;
  constexpr int NX = C::NAUX > 0 ? C::NAUX : 1;
  const int tid = threadIdx.x;
  const Solve& S = A.S;
  const int e0 = tile * EPB;
  if (e0 >= S.ne) return;  // whole workgroup
  const int nel = min(EPB, S.ne - e0);
  const long long nn = S.nn;

  double dt = S.dt_dev ? S.dt_scale * S.dt_dev[0] : S.dt;
  if (!(dt < INFINITY)) dt = 0.0;  // no dissipation anywhere: nothing moves

  load_tables<P>(lds + C::S_W, lds + C::S_Q, lds + C::S_IW, lds + C::S_M, lds + C::S_NK, T, C::BS);
  if (tid == 0) *reinterpret_cast<int*>(lds + C::S_LN) = 0;
  double U[NC], Un[NC];
  load_tile<EQ, DIM, P, EPB, true>(lds, S.u_s, nn, e0, S.ne, S.nx, S.ny, A.ph, bnd, U,
                                   A.diag ? &A.diag->bad_input : nullptr);
  const bool own = tid < nel * NP;
  if (A.use_un && own) {
#pragma unroll
    for (int c = 0; c < NC; ++c) Un[c] = S.u_n[c * nn + (long long)e0 * NP + tid];
  }
  __syncthreads();

  // smoothness factor of the node's element (SUBCELL_SI; p = 1 keeps the
  // strict bounds); the nodal-alpha array is free scratch until phase 4
  double eps = 1.0;
  if constexpr (P > 1) {
    static_assert(DIM == 1 || 2 * EPB * N1 + EPB <= EPB * NP, "scratch for the smoothness factor");
    if (A.limiter == LIM_SUBCELL_SI)
      eps = smoothness_tile<DIM, P, EPB, NS, C::BS>(lds + C::A_U, lds + C::S_M, lds + C::S_NK, T.s0, nel,
                                                   lds + C::S_AL);
  }

  // ---- phase 3: subcell faces ----
  // K_min over the node and its 2d face neighbours (Euler)
  double kmin = INFINITY;
  if constexpr (is_euler(EQ)) {
    if (own) {
      const int le = tid / NP, s = tid - le * NP;
      const int a = DIM == 2 ? s % N1 : s;
      const int b = DIM == 2 ? s / N1 : 0;
      const double* K = lds + C::A_X + 4 * EPB * NS + le * NS;
      kmin = K[s];
      kmin = fmin(kmin, K[a > 0 ? s - 1 : NP + b]);
      kmin = fmin(kmin, K[a < P ? s + 1 : NP + C::TJ + b]);
      if constexpr (DIM == 2) {
        kmin = fmin(kmin, K[b > 0 ? s - N1 : NP + 2 * C::TJ + a]);
        kmin = fmin(kmin, K[b < P ? s + N1 : NP + 3 * C::TJ + a]);
      }
    }
  }
  // one work item per subcell face of every line (element faces included,
  // formed by both adjacent elements), in wave-uniform chunks
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  double rFL[C::NITEM][NC], rRB[C::NITEM][NC], rUB[C::NITEM];
  int rO[C::NITEM];
#pragma unroll
  for (int it = 0; it < C::NITEM; ++it) {
    rUB[it] = 0.0;
    rO[it] = -1;
#pragma unroll
    for (int c = 0; c < NC; ++c) rFL[it][c] = rRB[it][c] = 0.0;
    face_chunk<EQ, DIM, P, EPB>(lds, A.ph, S, wv + it * C::NW, lane, nel, rFL[it], rRB[it], rUB[it], rO[it]);
  }
  __syncthreads();  // region A is dead from here on
#pragma unroll
  for (int it = 0; it < C::NITEM; ++it) {
    const int k = chunk_dir<EQ, DIM, P, EPB>(wv + it * C::NW);
    const int o = rO[it];
    if (o >= 0) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        lds[C::B_FL + (k * NC + c) * EPB * NF + o] = rFL[it][c];
        lds[C::B_RB + (k * NC + c) * EPB * NF + o] = rRB[it][c];
      }
      lds[C::B_UB + k * EPB * NF + o] = rUB[it];
    }
  }
  __syncthreads();

  // ---- phase 4a: low-order state, bounds, Zalesak, entropy checks ----
  const int le = tid / NP, s = tid - le * NP;
  const int a = DIM == 2 ? s % N1 : s;
  const int b = DIM == 2 ? s / N1 : 0;
  double uL[NC], alpha = 1.0, m = 1.0;
  int fl[DIM], fr[DIM];
  fl[0] = le * NF + b * NFL + a;
  fr[0] = fl[0] + 1;
  if constexpr (DIM == 2) {
    fl[1] = le * NF + a * NFL + b;
    fr[1] = fl[1] + 1;
  }
  bool lov = false;
  double kmin_dbg = 0.0, az_dbg = 1.0, umin = 0.0, umax = 0.0;
  int search = 0, check0 = 0;   // faces of this node for the search list; check u^L first
  double ubound = 0.0;
  const double idt = dt > 0.0 ? 1.0 / dt : 0.0;
  double dtm = 0.0;
  if (own) {
    const double wa = lds[C::S_W + a];
    const double wb = DIM == 2 ? lds[C::S_W + b] : 1.0;
    m = DIM == 2 ? wa * wb * S.hx * S.hy : wa * S.hx;
    const double cx = dt * (lds[C::S_IW + a] * S.ihx);
    const double cy = DIM == 2 ? dt * (lds[C::S_IW + b] * S.ihy) : 0.0;
    dtm = DIM == 2 ? cx * (lds[C::S_IW + b] * S.ihy) : cx;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double d = (lds[C::B_FL + c * EPB * NF + fl[0]] - lds[C::B_FL + c * EPB * NF + fr[0]]) * cx;
      if constexpr (DIM == 2)
        d += (lds[C::B_FL + (NC + c) * EPB * NF + fl[1]] - lds[C::B_FL + (NC + c) * EPB * NF + fr[1]]) * cy;
      uL[c] = U[c] + d;
    }
    umin = U[0];
    umax = U[0];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const double b1 = lds[C::B_UB + k * EPB * NF + fl[k]];
      const double b2 = lds[C::B_UB + k * EPB * NF + fr[k]];
      umin = fmin(umin, fmin(b1, b2));
      umax = fmax(umax, fmax(b1, b2));
    }
    const double tol = 1e-12 * fmax(fabs(umin), fabs(umax));
    lov = uL[0] > umax + tol || uL[0] < umin - tol;
    if (A.limiter == LIM_SUBCELL_SI) {  // eq. relaxed-bounds
#pragma clang fp contract(off)
      umin = eps * umin + (1.0 - eps) * A.gmin;
      umax = eps * umax + (1.0 - eps) * A.gmax;
    }
    if (A.limiter == LIM_TARGET) {
      alpha = 1.0;
    } else if (A.limiter == LIM_LOW) {
      alpha = 0.0;
    } else if (A.limiter == LIM_ELEMENTWISE) {
      if (dt > 0.0) {
        // elementwise limiting (Sec. 4.1.2, eq. convex-provisional-
        // elementwise): the node's whole correction d = u^H - u^L, the sum
        // of its subcell-face antidiffusive fluxes; Zalesak with that single
        // contribution, then the entropy line search along d; the element
        // minimum is taken in phase 5
        double d[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          double acc = 0.0;
          const int pos[2] = {a, b};
#pragma unroll
          for (int k = 0; k < DIM; ++k) {
            if (pos[k] < P) acc += lds[C::B_RB + (k * NC + c) * EPB * NF + fr[k]];
            if (pos[k] > 0) acc -= lds[C::B_RB + (k * NC + c) * EPB * NF + fl[k]];
          }
          d[c] = dtm * acc;
        }
        const double mdt = m * idt;
        const double f = mdt * d[0];
        const double Qp = fmax(0.0, mdt * (umax - uL[0]));
        const double Qm = fmin(0.0, mdt * (umin - uL[0]));
        alpha = f > 0.0 ? fmin(1.0, Qp / f) : (f < 0.0 ? fmin(1.0, Qm / f) : 1.0);
        az_dbg = alpha;
        if constexpr (is_euler(EQ)) {
          kmin_dbg = kmin;
          const PhiVal ea = phi_at<DIM, gn_of(EQ)>(alpha, uL, d, kmin, ph_of(A));
          if (!admissible(ea)) {
            const double zero[NC] = {};
            const PhiVal e0 = phi_at<DIM, gn_of(EQ)>(0.0, uL, zero, kmin, ph_of(A));
            if (!admissible(e0)) {
              alpha = 0.0;
            } else {
              double tn = ea.rho > 0.0 && ea.dphi < 0.0 ? alpha - ea.phi / ea.dphi : alpha;
              tn = fmin(fmax(tn, 0.0), alpha);
              alpha = entropy_root<DIM, gn_of(EQ), 16>(uL, d, tn, true, kmin, 0.0, ph_of(A));
            }
          }
        }
        alpha = alpha > 0.0 ? alpha : 0.0;
      }
    } else if (dt > 0.0) {
      double Pp = 0.0, Pm = 0.0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        const double cp = lds[C::B_RB + (k * NC) * EPB * NF + fr[k]];
        const double cm = -lds[C::B_RB + (k * NC) * EPB * NF + fl[k]];
        Pp += fmax(cp, 0.0) + fmax(cm, 0.0);
        Pm += fmin(cp, 0.0) + fmin(cm, 0.0);
      }
      const double mdt = m * idt;
      const double Qp = fmax(0.0, mdt * (umax - uL[0]));
      const double Qm = fmin(0.0, mdt * (umin - uL[0]));
      const double Rp = Pp == 0.0 ? 1.0 : fmin(1.0, Qp / Pp);
      const double Rm = Pm == 0.0 ? 1.0 : fmin(1.0, Qm / Pm);
      alpha = fmin(Rp, Rm);
      alpha = alpha > 0.0 ? alpha : 0.0;  // no negative zero: alpha is ordered as a u64 below
      az_dbg = alpha;
      if constexpr (is_euler(EQ)) {
        // every partial state uL + t 2d dt/m (+-rbar) must stay admissible
        // for t <= alpha (eq. convex-provisional).  A face whose partial
        // state at t = alpha is not admissible beyond doubt goes to the
        // workgroup's search list, which finds its root on [0, alpha]
        // starting from the exact value at alpha; most faces pass here
        // with integer powers only.  If u^L itself is not certain, the
        // search first checks it exactly (u^L off the set by rounding
        // leaves the node at alpha = 0).  A node whose partial-state
        // corrections are all below the search tolerance (max|P| over its
        // faces <= 1e-14 max|u^L|) needs no search: any t in [0, alpha]
        // moves its state by less than that, which is as close as a search
        // would get (in a uniform region the antidiffusive fluxes are of
        // rounding size and Phi at alpha is zero to rounding, which no test
        // could settle).
        kmin_dbg = kmin;
        const double g2 = 2.0 * DIM * dtm;
        const double ikg = (ph_of(A).gamma - 1.0) / kmin;
        double us = 0.0, rmax = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) us = fmax(us, fabs(uL[c]));
#pragma unroll
        for (int k = 0; k < DIM; ++k)
#pragma unroll
          for (int c = 0; c < NC; ++c)
            rmax = fmax(rmax, fmax(fabs(lds[C::B_RB + (k * NC + c) * EPB * NF + fl[k]]),
                                   fabs(lds[C::B_RB + (k * NC + c) * EPB * NF + fr[k]])));
        int act = 0;
        if (g2 * rmax > 1e-14 * us) {
#pragma unroll
          for (int k = 0; k < DIM; ++k) {
#pragma unroll
            for (int sd = 0; sd < 2; ++sd) {
              const int fidx = sd ? fr[k] : fl[k];
              const double sg = sd ? 1.0 : -1.0;
              double Pv[NC];
              bool nz = false;
#pragma unroll
              for (int c = 0; c < NC; ++c) {
                Pv[c] = g2 * (sg * lds[C::B_RB + (k * NC + c) * EPB * NF + fidx]);
                nz |= Pv[c] != 0.0;
              }
              if (nz && !surely_admissible<DIM, gn_of(EQ)>(alpha, uL, Pv, kmin, ikg, ph_of(A)))
                act |= 1 << (2 * k + sd);
            }
          }
        }
        if (act) {
          const double zero[NC] = {};
          search = act;
          ubound = alpha;
          check0 = !surely_admissible<DIM, gn_of(EQ)>(0.0, uL, zero, kmin, ikg, ph_of(A));
        }
      }
    }
    lds[C::S_AL + tid] = alpha;
  }
  if constexpr (is_euler(EQ)) {
    __syncthreads();  // the low-order fluxes are consumed: region C may overwrite them
    if (search) {
#pragma unroll
      for (int c = 0; c < NC; ++c) lds[C::C_UL + c * EPB * NP + tid] = uL[c];
      lds[C::C_KM + tid] = kmin;
      lds[C::C_AZ + tid] = ubound;
      int* list = reinterpret_cast<int*>(lds + C::C_LIST);
      int* count = reinterpret_cast<int*>(lds + C::S_LN);
#pragma unroll
      for (int f = 0; f < 2 * DIM; ++f)
        if (search & (1 << f)) list[atomicAdd(count, 1)] = tid * 8 + f * 2 + check0;
    }
    __syncthreads();
    // ---- phase 4b: entropy line searches, spread over the workgroup ----
    const int nact = *reinterpret_cast<const int*>(lds + C::S_LN);
    const int* list = reinterpret_cast<const int*>(lds + C::C_LIST);
    for (int w = tid; w < nact; w += C::BS) {
      const int item = list[w];
      const int node = item >> 3, f = (item >> 1) & 3, k = f >> 1, sd = f & 1;
      const int nle = node / NP, ns = node - nle * NP;
      const int na = DIM == 2 ? ns % N1 : ns;
      const int nb = DIM == 2 ? ns / N1 : 0;
      const double cxn = dt * (lds[C::S_IW + na] * S.ihx);
      const double g2 = 2.0 * DIM * (DIM == 2 ? cxn * (lds[C::S_IW + nb] * S.ihy) : cxn);
      const int fidx = k == 0 ? nle * NF + nb * NFL + na + sd : nle * NF + na * NFL + nb + sd;
      double ul[NC], Pv[NC], rmax = 0.0;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        ul[c] = lds[C::C_UL + c * EPB * NP + node];
        Pv[c] = g2 * (sd ? 1.0 : -1.0) * lds[C::B_RB + (k * NC + c) * EPB * NF + fidx];
      }
      // the node's largest face correction scales the search tolerance
      const int fx = nle * NF + nb * NFL + na, fy = nle * NF + na * NFL + nb;
#pragma unroll
      for (int kk = 0; kk < DIM; ++kk)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const double* rb = lds + C::B_RB + (kk * NC + c) * EPB * NF + (kk == 0 ? fx : fy);
          rmax = fmax(rmax, fmax(fabs(rb[0]), fabs(rb[1])));
        }
      const double km = lds[C::C_KM + node];
      bool feasible = true;
      if (item & 1) {
        const double zero[NC] = {};
        feasible = admissible(phi_at<DIM, gn_of(EQ)>(0.0, ul, zero, km, ph_of(A)));
      }
      const double t = feasible ? entropy_root<DIM, gn_of(EQ), 14>(ul, Pv, lds[C::C_AZ + node], false, km,
                                                                   g2 * rmax, ph_of(A))
                                : 0.0;
      atomicMin(reinterpret_cast<unsigned long long*>(lds + C::S_AL + node),
                (unsigned long long)__double_as_longlong(t));
    }
  }
  __syncthreads();

  // ---- phase 5: subcell-face coefficients, corrected update, RK stage ----
  bool limited = false, ent = false;
  if (own) {
    alpha = lds[C::S_AL + tid];
    // the node's own coefficient was lowered by the entropy search
    ent = is_euler(EQ) && A.limiter != LIM_TARGET && A.limiter != LIM_LOW && alpha < az_dbg;
    const bool elementwise = A.limiter == LIM_ELEMENTWISE;
    if (elementwise) {  // one coefficient per element: the minimum over its nodes
      const double* ae = lds + C::S_AL + le * NP;
      for (int q = 0; q < NP; ++q) alpha = fmin(alpha, ae[q]);
    }
    limited = alpha < 1.0;
    if (A.trace) {
      const long long g = (long long)e0 * NP + tid;
      A.trace[g] = umin;
      A.trace[nn + g] = umax;
      A.trace[2 * nn + g] = kmin_dbg;
      A.trace[3 * nn + g] = az_dbg;
      A.trace[4 * nn + g] = alpha;
    }
    double corr[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) corr[c] = 0.0;
    const int pos[2] = {a, b};
    const int stride[2] = {1, N1};
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      if (pos[k] < P) {
        const double ap = elementwise ? alpha : fmin(alpha, lds[C::S_AL + tid + stride[k]]);
#pragma unroll
        for (int c = 0; c < NC; ++c) corr[c] += ap * lds[C::B_RB + (k * NC + c) * EPB * NF + fr[k]];
      }
      if (pos[k] > 0) {
        const double am = elementwise ? alpha : fmin(alpha, lds[C::S_AL + tid - stride[k]]);
#pragma unroll
        for (int c = 0; c < NC; ++c) corr[c] -= am * lds[C::B_RB + (k * NC + c) * EPB * NF + fl[k]];
      }
    }
    const long long g = (long long)e0 * NP + tid;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double fe = uL[c] + dtm * corr[c];
      S.u_out[c * nn + g] = A.use_un ? A.a_s * Un[c] + A.b_s * fe : fe;
    }
  }
  if (A.diag) {
    const unsigned long long bl = __ballot(limited), be = __ballot(ent), bv = __ballot(lov);
    if ((tid & 63) == 0) {
      const int slot = (blockIdx.x * (C::BS / 64) + (tid >> 6)) & (DIAG_SLOTS - 1);
      if (bl) atomicAdd(&A.diag->limited[slot], (unsigned long long)__popcll(bl));
      if (be) atomicAdd(&A.diag->entropy[slot], (unsigned long long)__popcll(be));
      if (bv) atomicOr(&A.diag->lo_violation, 1u);
    }
  }
}

template <int EQ, int DIM, int P, int EPB>
__global__ __launch_bounds__((Cfg<EQ, DIM, P, EPB>::BS)) void stage_kernel(StageArgs A) {
  __shared__ double lds[Cfg<EQ, DIM, P, EPB>::LDS];
  stage_tile<EQ, DIM, P, EPB>(lds, A, A.T, A.bnd, xcd_tile(blockIdx.x, gridDim.x));
}

// ----------------------------------------------------------------------
// low-order CFL bound (eq. cfl-low): min over nodes of m_i/(2 sum dhat_ij)
// ----------------------------------------------------------------------
template <int EQ, int DIM, int P, int EPB>
struct DtCfg {
  using C = Cfg<EQ, DIM, P, EPB>;
  static constexpr int L = C::A_X + C::NAUXF * EPB * C::NS;  // [DIM][EPB*NF] wave speeds
  static constexpr int W = L + DIM * EPB * C::NF;
  static constexpr int R = W + C::N1;
  static constexpr int LDS = R + C::BS / 64;
  static constexpr int CH = (EPB * C::NF + 63) / 64;   // chunks of faces per direction
};

// Wave speed of face w (element le, line l, position f in 0..p+1) of
// direction K of a tile, into the time-step kernel's array.
template <int EQ, int DIM, int P, int EPB, int K>
__device__ __forceinline__ void dt_face(double* lds, const Phys& ph, int w, int nel) {
  using C = Cfg<EQ, DIM, P, EPB>;
  using D = DtCfg<EQ, DIM, P, EPB>;
  constexpr int NC = C::NC, NS = C::NS, NP = C::NP, NF = C::NF, NFL = C::NFL;
  constexpr int NX = C::NAUX > 0 ? C::NAUX : 1;
  const int le = w / NF;
  if (le >= nel) return;
  const int fi = w - le * NF;
  const int l = fi / NFL;
  const int f = fi - l * NFL;
  const int base = le * NS;
  const int sl = base + (f == 0 ? NP + (2 * K) * C::TJ + l : own_slot<DIM, P>(K, l, f - 1));
  const int sr = base + (f == P + 1 ? NP + (2 * K + 1) * C::TJ + l : own_slot<DIM, P>(K, l, f));
  double UL[NC], UR[NC], XL[NX], XR[NX];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    UL[c] = lds[C::A_U + c * EPB * NS + sl];
    UR[c] = lds[C::A_U + c * EPB * NS + sr];
  }
#pragma unroll
  for (int q = 0; q < C::NAUXF; ++q) {
    XL[q] = lds[C::A_X + q * EPB * NS + sl];
    XR[q] = lds[C::A_X + q * EPB * NS + sr];
  }
  lds[D::L + K * EPB * NF + le * NF + fi] = lambda_k<EQ, DIM>(K, UL, XL, UR, XR, ph);
}

// the minimum of one tile into *out
template <int EQ, int DIM, int P, int EPB>
__device__ __forceinline__ void maxdt_tile(double* lds, const MaxDtArgs& A, const Tables& T, const Bnd& bnd, int tile,
                                           double* out) {
  using C = Cfg<EQ, DIM, P, EPB>;
  using D = DtCfg<EQ, DIM, P, EPB>;
  constexpr int NC = C::NC, NS = C::NS, NP = C::NP, NF = C::NF, NFL = C::NFL, N1 = C::N1;
  constexpr int NX = C::NAUX > 0 ? C::NAUX : 1;
  const int tid = threadIdx.x;
  const int e0 = tile * EPB;
  if (e0 >= A.ne) return;
  const int nel = min(EPB, A.ne - e0);
  for (int t = tid; t < N1; t += C::BS) lds[D::W + t] = T.w[t];
  double U[NC];
  load_tile<EQ, DIM, P, EPB, false>(lds, A.u, A.nn, e0, A.ne, A.nx, A.ny, A.ph, bnd, U, nullptr);
  __syncthreads();
  // wave-uniform chunks of 64 faces of one direction (D::CH per direction)
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  for (int ch = wv; ch < DIM * D::CH; ch += C::NW) {
    const int k = ch / D::CH;
    const int w = (ch - k * D::CH) * 64 + lane;
    if (k == 0) dt_face<EQ, DIM, P, EPB, 0>(lds, A.ph, w, nel);
    else if constexpr (DIM == 2) dt_face<EQ, DIM, P, EPB, 1>(lds, A.ph, w, nel);
  }
  __syncthreads();
  double dti = INFINITY;
  if (tid < nel * NP) {
    const int le = tid / NP, s = tid - le * NP;
    const int a = DIM == 2 ? s % N1 : s;
    const int b = DIM == 2 ? s / N1 : 0;
    const double wa = lds[D::W + a];
    const double wb = DIM == 2 ? lds[D::W + b] : 1.0;
    const int fx = le * NF + b * NFL + a;
    double den = (lds[D::L + fx] + lds[D::L + fx + 1]) * (DIM == 2 ? wb * A.hy : 1.0);
    if constexpr (DIM == 2) {
      const int fy = le * NF + a * NFL + b;
      den += (lds[D::L + EPB * NF + fy] + lds[D::L + EPB * NF + fy + 1]) * (wa * A.hx);
    }
    const double m = DIM == 2 ? wa * wb * A.hx * A.hy : wa * A.hx;
    dti = den > 0.0 ? m / den : INFINITY;
  }
  for (int off = 32; off > 0; off >>= 1) dti = fmin(dti, __shfl_xor(dti, off));
  if ((tid & 63) == 0) lds[D::R + (tid >> 6)] = dti;
  __syncthreads();
  if (tid == 0) {
    double v = lds[D::R];
    for (int i = 1; i < C::BS / 64; ++i) v = fmin(v, lds[D::R + i]);
    *out = v;
  }
}

template <int EQ, int DIM, int P, int EPB>
__global__ __launch_bounds__((Cfg<EQ, DIM, P, EPB>::BS)) void maxdt_kernel(MaxDtArgs A) {
  __shared__ double lds[DtCfg<EQ, DIM, P, EPB>::LDS];
  maxdt_tile<EQ, DIM, P, EPB>(lds, A, A.T, A.bnd, xcd_tile(blockIdx.x, gridDim.x), A.partial + blockIdx.x);
}

// ----------------------------------------------------------------------
// elements per workgroup: variant 0 fills 64-lane multiples best
// ----------------------------------------------------------------------
constexpr int epb_for(int dim, int p, int variant) {
  if (dim == 1) return (variant == 0 ? 128 : 256) / (p + 1);
  // shape 0 (a new handle's): the faster of the two on 2-D Euler (256^2 for
  // p = 1..4, 40^2..128^2 for p = 3..8), measured with both shapes taking
  // turns on the same state; shape 1 the alternative for idp_dg_tune
  constexpr int v0[9] = {0, 16, 14, 8, 5, 7, 5, 2, 3};
  constexpr int v1[9] = {0, 32, 7, 16, 10, 3, 2, 4, 6};
  return variant == 0 ? v0[p] : v1[p];
}

#define IDP_NUM_VARIANTS 2

// ----------------------------------------------------------------------
// batched work-list kernels: one kernel per degree, its work list holding
// the element tiles of every solve of that degree (same tile shape as the
// plain kernel), one workgroup per item, mapped XCD-aware.  The item's
// arguments are read once at entry, before any store, so that they can live
// in scalar registers; the degree tables go straight from global memory to
// LDS.
// ----------------------------------------------------------------------
template <int EQ, int DIM, int P, int EPB>
__global__ __launch_bounds__((Cfg<EQ, DIM, P, EPB>::BS)) void batch_stage_kernel(BatchArgs B) {
  __shared__ double lds[Cfg<EQ, DIM, P, EPB>::LDS];
  const int it = xcd_tile(blockIdx.x, gridDim.x);
  if (it >= B.nitems) return;
  const StageArgs* pa = B.args + B.item_solve[it];
  StageArgs A;
  A.S = pa->S;
  A.ph = pa->ph;
  A.a_s = pa->a_s;
  A.b_s = pa->b_s;
  A.use_un = pa->use_un;
  A.limiter = pa->limiter;
  A.diag = pa->diag;
  A.trace = pa->trace;
  A.gmin = pa->gmin;
  A.gmax = pa->gmax;
  // the boundary arrays are indexed at run time: read them where they are
  // (a copy in this local struct would move it to scratch memory)
  stage_tile<EQ, DIM, P, EPB>(lds, A, pa->T, pa->bnd, B.item_tile[it]);
}

template <int EQ, int DIM, int P, int EPB>
__global__ __launch_bounds__((Cfg<EQ, DIM, P, EPB>::BS)) void batch_maxdt_kernel(BatchDtArgs B) {
  __shared__ double lds[DtCfg<EQ, DIM, P, EPB>::LDS];
  const int it = xcd_tile(blockIdx.x, gridDim.x);
  if (it >= B.nitems) return;
  const MaxDtArgs* pa = B.args + B.item_solve[it];
  MaxDtArgs A;
  A.u = pa->u;
  A.partial = pa->partial;
  A.nn = pa->nn;
  A.p = pa->p;
  A.nx = pa->nx;
  A.ny = pa->ny;
  A.ne = pa->ne;
  A.ntiles = pa->ntiles;
  A.hx = pa->hx;
  A.hy = pa->hy;
  A.ph = pa->ph;
  maxdt_tile<EQ, DIM, P, EPB>(lds, A, pa->T, pa->bnd, B.item_tile[it], B.partial + it);
}

template <int EQ, int DIM, int P, int EPB>
void batch_kernels_e(BatchKernels* k) {
  k->stage = reinterpret_cast<const void*>(&batch_stage_kernel<EQ, DIM, P, EPB>);
  k->maxdt = reinterpret_cast<const void*>(&batch_maxdt_kernel<EQ, DIM, P, EPB>);
  k->block = Cfg<EQ, DIM, P, EPB>::BS;
  k->tile_elems = EPB;
}

template <int EQ, int DIM, int P>
void batch_kernels_t(int variant, BatchKernels* k) {
#if IDP_NUM_VARIANTS > 1
  if (variant == 1) return batch_kernels_e<EQ, DIM, P, epb_for(DIM, P, 1)>(k);
#endif
  (void)variant;
  batch_kernels_e<EQ, DIM, P, epb_for(DIM, P, 0)>(k);
}

template <int EQ, int DIM, int P, int EPB>
hipError_t launch_stage_t(const StageArgs& a, hipStream_t s) {
  using C = Cfg<EQ, DIM, P, EPB>;
  const int nb = (a.S.ne + EPB - 1) / EPB;
  hipLaunchKernelGGL((stage_kernel<EQ, DIM, P, EPB>), dim3(nb), dim3(C::BS), 0, s, a);
  return hipGetLastError();
}

template <int EQ, int DIM, int P, int EPB>
hipError_t launch_maxdt_t(const MaxDtArgs& a, hipStream_t s) {
  using C = Cfg<EQ, DIM, P, EPB>;
  const int nb = (a.ne + EPB - 1) / EPB;
  hipLaunchKernelGGL((maxdt_kernel<EQ, DIM, P, EPB>), dim3(nb), dim3(C::BS), 0, s, a);
  return hipGetLastError();
}

template <int EQ, int DIM, int P>
hipError_t launch_stage_v(int variant, const StageArgs& a, hipStream_t s) {
#if IDP_NUM_VARIANTS > 1
  if (variant == 1) return launch_stage_t<EQ, DIM, P, epb_for(DIM, P, 1)>(a, s);
#endif
  (void)variant;
  return launch_stage_t<EQ, DIM, P, epb_for(DIM, P, 0)>(a, s);
}

template <int EQ, int DIM, int P>
hipError_t launch_maxdt_v(int variant, const MaxDtArgs& a, hipStream_t s) {
#if IDP_NUM_VARIANTS > 1
  if (variant == 1) return launch_maxdt_t<EQ, DIM, P, epb_for(DIM, P, 1)>(a, s);
#endif
  (void)variant;
  return launch_maxdt_t<EQ, DIM, P, epb_for(DIM, P, 0)>(a, s);
}

#define IDP_DEFINE_LAUNCHERS(NAME, EQ, DIM)                                              \
  hipError_t launch_stage_##NAME(int p, int variant, const StageArgs& a, hipStream_t s) { \
    switch (p) {                                                                         \
      case 1: return launch_stage_v<EQ, DIM, 1>(variant, a, s);                          \
      case 2: return launch_stage_v<EQ, DIM, 2>(variant, a, s);                          \
      case 3: return launch_stage_v<EQ, DIM, 3>(variant, a, s);                          \
      case 4: return launch_stage_v<EQ, DIM, 4>(variant, a, s);                          \
      case 5: return launch_stage_v<EQ, DIM, 5>(variant, a, s);                          \
      case 6: return launch_stage_v<EQ, DIM, 6>(variant, a, s);                          \
      case 7: return launch_stage_v<EQ, DIM, 7>(variant, a, s);                          \
      case 8: return launch_stage_v<EQ, DIM, 8>(variant, a, s);                          \
    }                                                                                    \
    return hipErrorInvalidValue;                                                         \
  }                                                                                      \
  hipError_t launch_maxdt_##NAME(int p, int variant, const MaxDtArgs& a, hipStream_t s) { \
    switch (p) {                                                                         \
      case 1: return launch_maxdt_v<EQ, DIM, 1>(variant, a, s);                          \
      case 2: return launch_maxdt_v<EQ, DIM, 2>(variant, a, s);                          \
      case 3: return launch_maxdt_v<EQ, DIM, 3>(variant, a, s);                          \
      case 4: return launch_maxdt_v<EQ, DIM, 4>(variant, a, s);                          \
      case 5: return launch_maxdt_v<EQ, DIM, 5>(variant, a, s);                          \
      case 6: return launch_maxdt_v<EQ, DIM, 6>(variant, a, s);                          \
      case 7: return launch_maxdt_v<EQ, DIM, 7>(variant, a, s);                          \
      case 8: return launch_maxdt_v<EQ, DIM, 8>(variant, a, s);                          \
    }                                                                                    \
    return hipErrorInvalidValue;                                                         \
  }                                                                                      \
  int tile_elems_##NAME(int p, int variant) { return epb_for(DIM, p, variant); }         \
  int batch_kernels_##NAME(int p, int variant, BatchKernels* k) {                        \
    switch (p) {                                                                         \
      case 1: batch_kernels_t<EQ, DIM, 1>(variant, k); return 0;                         \
      case 2: batch_kernels_t<EQ, DIM, 2>(variant, k); return 0;                         \
      case 3: batch_kernels_t<EQ, DIM, 3>(variant, k); return 0;                         \
      case 4: batch_kernels_t<EQ, DIM, 4>(variant, k); return 0;                         \
      case 5: batch_kernels_t<EQ, DIM, 5>(variant, k); return 0;                         \
      case 6: batch_kernels_t<EQ, DIM, 6>(variant, k); return 0;                         \
      case 7: batch_kernels_t<EQ, DIM, 7>(variant, k); return 0;                         \
      case 8: batch_kernels_t<EQ, DIM, 8>(variant, k); return 0;                         \
    }                                                                                    \
    return -1;                                                                           \
  }                                                                                      \
  int num_variants_##NAME(int p) {                                                       \
    (void)p;                                                                             \
    return IDP_NUM_VARIANTS;                                                             \
  }

}  // namespace idp
