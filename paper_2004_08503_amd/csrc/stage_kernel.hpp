// Fused limited SSP-RK stage for gfx950.  One workgroup owns a tile of
// TX x TY elements (TX elements in 1-D), one thread per node, and runs every
// step of the stage out of LDS.  Global memory is touched once per node for
// the stage input (plus one ring of face-trace nodes around the tile), once
// for u^n on the second and third stages, and once for the output.
//
// The tile's nodes form one grid of GX = TX (p+1) columns and GY = TY (p+1)
// rows (one row in 1-D), surrounded by a ring of halo slots holding the
// facing nodes of the neighbouring elements (or, on an open side of the
// box, the exterior states).  Along a grid row, consecutive columns are
// neighbours whether they belong to one element (an interior subcell face)
// or to two (an element face), so every subcell face of the tile is one
// pair of adjacent slots and is evaluated once, left state first: element
// faces inside the tile are not duplicated, and a face on the tile's edge,
// which the neighbouring tile evaluates too, gives bitwise the same values
// in both (a face's arithmetic does not depend on which tile runs it).
//
// Phases (LDS barriers between them):
//   1-2. load the tile's own nodes and its halo ring; pointwise physics on
//        every slot: fluxes (own nodes: both directions, halo slots: the
//        direction of their face) and, for Euler, 1/rho, the sound speed c,
//        c p^{-(gamma-1)/(2 gamma)}, (gamma+1)/(2 gamma p) (the inputs of the
//        wave-speed bound) and K = p rho^{-gamma};
//   3. one work item per subcell face: wave-speed bound, low-order flux f^L
//      (eq. lax-friedrichs on the subgrid), bar state of the limited
//      component (eq. bar-states) and on interior subcell faces the
//      high-order subcell flux f^H and the antidiffusive flux
//      rbar = s (f^L - f^H);
//   4. per node: u^L, local bounds (K_min over the node and its four grid
//      neighbours), Zalesak coefficient and, for Euler, the entropy line
//      search of eq. convex-provisional;
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

template <int EQ, int DIM, int P, int TX, int TY, int PAD, bool CURV = false>
struct CfgP {
  static constexpr int N1 = P + 1;
  static constexpr int NP = DIM == 2 ? N1 * N1 : N1;    // nodes per element
  static constexpr int TYE = DIM == 2 ? TY : 1;         // elements per tile in y
  static constexpr int NE = TX * TYE;                   // elements per tile
  static constexpr int GX = TX * N1;                    // node columns of the tile
  static constexpr int GY = DIM == 2 ? TYE * N1 : 1;    // node rows
  static constexpr int NOWN = NE * NP;                  // own nodes (= GX GY)
  static constexpr int BS = ((NOWN + 63) / 64) * 64;
  static constexpr int NW = BS / 64;                    // waves per workgroup
  static constexpr int NC = is_euler(EQ) ? DIM + 2 : 1;
  // per-slot auxiliaries the faces read: Euler 1/rho, c, c p^-ex,
  // (gamma+1)/(2 gamma p); EQ_ADVV beta_x, beta_y.  The Euler K = p rho^-gamma
  // of every slot goes to the nodal-alpha array, free until phase 4.
  static constexpr int NAUX = is_euler(EQ) ? 4 : EQ == EQ_ADVV ? 2 : 0;
  static constexpr int NAUXF = NAUX;
  // slot grid: own nodes (i, j), 0 <= i < GX, 0 <= j < GY, and the halo ring
  // i = -1, i = GX (x-neighbours) and j = -1, j = GY (y-neighbours)
  static constexpr int RP = GX + 2;                     // row pitch
  static constexpr int NSL = DIM == 2 ? RP * (GY + 2) : RP;
  static constexpr int NH = 2 * GY + (DIM == 2 ? 2 * GX : 0);   // halo slots
  // flux grids: F^x on rows 0..GY-1 and columns -1..GX, F^y on rows
  // -1..GY and columns 0..GX-1
  static constexpr int NFX = GY * RP;
  static constexpr int NFY = DIM == 2 ? (GY + 2) * GX : 0;
  // face grids: x-face i (between columns i-1 and i) of row j, i = 0..GX;
  // y-face j (between rows j-1 and j) of column i, j = 0..GY
  static constexpr int FXP = GX + 1;
  static constexpr int NOX = GY * FXP;
  static constexpr int NOY = DIM == 2 ? (GY + 1) * GX : 0;
  // Consecutive arrays of a multi-component (or multi-auxiliary) field
  // start PAD doubles past a multiple of 64, so that the components of one
  // slot fall into different LDS banks (with PAD = 0 every pair of them
  // would share a bank).
  static constexpr int up64(int n) { return (n + 63) / 64 * 64 + PAD; }
  static constexpr int CSU = up64(NSL), CSX = up64(NFX), CSY = up64(NFY);
  static constexpr int COX = up64(NOX), COY = up64(NOY), CSO = up64(NOWN);
  // phase-3 work: per direction the element faces and the interior faces
  // form two groups, each cut into chunks of 64 items; a wave takes whole
  // chunks, so each of its passes runs one body specialised for a direction
  // and a face kind
  static constexpr int GEX = GY * (TX + 1);
  static constexpr int GIX = GY * TX * P;
  static constexpr int GEY = DIM == 2 ? GX * (TYE + 1) : 0;
  static constexpr int GIY = DIM == 2 ? GX * TYE * P : 0;
  static constexpr int CEX = (GEX + 63) / 64, CEY = (GEY + 63) / 64;
  static constexpr int CIX = (GIX + 63) / 64, CIY = (GIY + 63) / 64;
  static constexpr int NCHUNK = CEX + CEY + CIX + CIY;
  static constexpr int NITEM = (NCHUNK + NW - 1) / NW;  // chunks per wave
  // region A: phase 1-2 results, read in phase 3
  static constexpr int A_U = 0;
  static constexpr int A_X = A_U + NC * CSU;
  static constexpr int A_FX = A_X + NAUX * CSU;
  static constexpr int A_FY = A_FX + NC * CSX;
  // curved meshes: the flux grids A_FX / A_FY hold the contravariant fluxes
  // of the high-order metric terms, A_GX / A_GY those of the modified
  // (corrected) terms, and A_M the eight metric terms of every slot
  static constexpr int A_GX = A_FY + NC * CSY;
  static constexpr int A_GY = A_GX + (CURV ? NC * CSX : 0);
  static constexpr int A_M = A_GY + (CURV ? NC * CSY : 0);
  static constexpr int A_END = A_M + (CURV ? 8 * CSU : 0);
  // region B (aliases A): phase 3 results, read in phases 4-5
  static constexpr int B_FLX = 0;
  static constexpr int B_FLY = B_FLX + NC * COX;
  static constexpr int B_UBX = B_FLY + NC * COY;
  static constexpr int B_UBY = B_UBX + COX;
  // curved meshes: the bar state of the right (upper) node of each face
  // (B_UBX / B_UBY hold the left (lower) node's)
  static constexpr int B_UBX2 = B_UBY + COY;
  static constexpr int B_UBY2 = B_UBX2 + (CURV ? COX : 0);
  static constexpr int B_RBX = B_UBY2 + (CURV ? COY : 0);
  static constexpr int B_RBY = B_RBX + NC * COX;
  static constexpr int B_END = B_RBY + NC * COY;
  // region C: Euler search data, written once the low-order fluxes are
  // consumed; it overwrites them where it fits
  static constexpr int C_SIZE = is_euler(EQ) ? (NC + 4 + DIM) * CSO : 0;
  static constexpr int C_UL = C_SIZE <= (NC + (CURV ? 2 : 1)) * (COX + COY) ? B_FLX : B_END;   // [NC][CSO]
  static constexpr int C_KM = C_UL + (is_euler(EQ) ? NC * CSO : 0);
  static constexpr int C_AZ = C_KM + (is_euler(EQ) ? CSO : 0);   // bound U of the node
  static constexpr int C_G2 = C_AZ + (is_euler(EQ) ? CSO : 0);   // 2d dt/m of the node
  static constexpr int C_PS = C_G2 + (is_euler(EQ) ? CSO : 0);   // largest |P| over the node's faces
  static constexpr int C_LIST = C_PS + (is_euler(EQ) ? CSO : 0);  // int[2*DIM*CSO]
  static constexpr int C_END = C_LIST + (is_euler(EQ) ? DIM * CSO : 0);
  static constexpr int AB0 = A_END > B_END ? A_END : B_END;
  static constexpr int AB = AB0 > C_END ? AB0 : C_END;
  // nodal alpha [NOWN] (grid order); before phase 4 the Euler K of every
  // slot [NSL] (slot order), and the smoothness indicator's scratch
  static constexpr int S_AL = AB;
  static constexpr int S_W = S_AL + (is_euler(EQ) ? CSU : NOWN);   // weights
  static constexpr int S_Q = S_W + N1;                  // cumulative D
  static constexpr int S_IW = S_Q + P * N1;             // 1/w
  static constexpr int S_M = S_IW + N1;                 // nodal -> modal map [k][a]
  static constexpr int S_NK = S_M + N1 * N1;            // Legendre norms
  static constexpr int S_LN = S_NK + N1;                // search list length (int)
  static constexpr int LDS = S_LN + 1;
  static_assert(LDS * 8 <= 160 * 1024, "tile does not fit in LDS");

  // slot of grid point (i, j), -1 <= i <= GX, -1 <= j <= GY
  static __device__ __forceinline__ int sl(int i, int j) { return DIM == 2 ? (j + 1) * RP + i + 1 : i + 1; }
  // flux-grid entries
  static __device__ __forceinline__ int fx(int i, int j) { return j * RP + i + 1; }
  static __device__ __forceinline__ int fy(int i, int j) { return (j + 1) * GX + i; }
  // face-grid entries
  static __device__ __forceinline__ int ox(int i, int j) { return j * FXP + i; }
  static __device__ __forceinline__ int oy(int i, int j) { return j * GX + i; }
};

// The bank padding is 4 doubles unless it would lower the number of
// workgroups whose LDS fits in a CU's 160 KB.
template <int EQ, int DIM, int P, int TX, int TY, bool CURV>
constexpr int lds_pad() {
  constexpr int k0 = 160 * 1024 / (CfgP<EQ, DIM, P, TX, TY, 0, CURV>::LDS * 8);
  constexpr int k4 = 160 * 1024 / (CfgP<EQ, DIM, P, TX, TY, 4, CURV>::LDS * 8);
  return k4 == k0 ? 4 : 0;
}
template <int EQ, int DIM, int P, int TX, int TY, bool CURV = false>
using Cfg = CfgP<EQ, DIM, P, TX, TY, lds_pad<EQ, DIM, P, TX, TY, CURV>(), CURV>;

// Where a tile lies: its first element column and row, and how many of its
// TX x TY elements exist (tiles on the high edges of the mesh are ragged).
struct TileGeo {
  int ex0, ey0, tw, th;
};
template <int DIM, int TX, int TY>
__device__ inline TileGeo tile_geo(int tile, int ntx, int nx, int ny) {
  TileGeo t;
  const int ty = DIM == 2 ? tile / ntx : 0;
  const int tx = tile - ty * ntx;
  t.ex0 = tx * TX;
  t.ey0 = DIM == 2 ? ty * TY : 0;
  t.tw = min(TX, nx - t.ex0);
  t.th = DIM == 2 ? min(TY, ny - t.ey0) : 1;
  return t;
}

// Workgroups are dealt round-robin to the eight XCDs; give every XCD a
// contiguous range of tiles so that the halo nodes a tile reads from the
// tile rows above and below were fetched into the same XCD's L2.
__device__ inline int xcd_tile(int b, int nb) {
  const int x = b & 7, i = b >> 3;
  const int q = nb >> 3, r = nb & 7;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
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

// sqrt(x) for x >= 1 (or +infinity): the hardware reciprocal square root
// refined by Goldschmidt's iteration and two residual corrections, which
// brings it to within an ulp; no scaling is needed in this range.
__device__ inline double sqrt_ge1(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  g = fma(d, h, g);
  return x < INFINITY ? g : x;
}

// 1/x for x of normal magnitude: the hardware approximation refined by two
// Newton steps, within an ulp (infinity gives 0, NaN gives NaN).
__device__ inline double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

// ----------------------------------------------------------------------
// pointwise physics
// ----------------------------------------------------------------------

// Euler auxiliaries of one state: X = (1/rho, c, c p^-ex, (gamma+1)/(2 gamma
// p), and with WITHK K = p rho^-gamma), ex = (gamma-1)/(2 gamma); p is
// returned for the fluxes.  For gamma = 1 + 2/n (GN = n = 5: 7/5, n = 3:
// 5/3) every fractional power is an integer power of z = rho^(-1/n) or of
// x3 = p^(-1/(n+2)): 1/rho = z^n, K = p z^(n+2), 1/p = x3^(n+2); otherwise
// pow and divisions are used.  Without K (the time-step pass) 1/rho is a
// plain division, cheaper than the root.
template <int DIM, int GN, bool WITHK>
__device__ inline void euler_aux(const double* U, const Phys& ph, double* X, double& p, bool& bad) {
  double rinv, z = 0.0;
  if constexpr (GN > 0 && WITHK) {
    z = inv_root<GN>(U[0]);
    rinv = ipow_c<GN>(z);
  } else {
    rinv = 1.0 / U[0];
  }
  double mm = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) mm += U[1 + k] * U[1 + k];
  p = (ph.gamma - 1.0) * (U[DIM + 1] - 0.5 * mm * rinv);
  bad = !(U[0] > 0.0) || !(p > 0.0);
  const double c = sqrt(ph.gamma * p * rinv);
  double x3, ip;
  if constexpr (GN > 0) {
    x3 = inv_root<GN + 2>(p);
    ip = ipow_c<GN + 2>(x3);
  } else {
    x3 = pow(p, -ph.ex);
    ip = 1.0 / p;
  }
  X[0] = rinv;
  X[1] = c;
  X[2] = c * x3;
  X[3] = ph.fac * ip;
  if constexpr (WITHK) {
    if constexpr (GN > 0) X[4] = p * ipow_c<GN + 2>(z);
    else X[4] = p * pow(U[0], -ph.gamma);
  }
}

// flux in direction k (k known at compile time where the caller unrolls;
// otherwise the components are selected, never indexed at run time).
// X: Euler auxiliaries (X[0] = 1/rho) with the pressure p, or beta for EQ_ADVV.
template <int EQ, int DIM>
__device__ inline void flux_k(int k, const double* U, const double* X, double p, const Phys& ph, double* F) {
  if constexpr (EQ == EQ_ADV) {
    F[0] = vel_k(k, ph) * U[0];
  } else if constexpr (EQ == EQ_ADVV) {
    F[0] = (k == 0 ? X[0] : X[1]) * U[0];
  } else if constexpr (EQ == EQ_BURG) {
    F[0] = 0.5 * U[0] * U[0] * vel_k(k, ph);
  } else {
    const double mk = DIM == 2 && k == 1 ? U[2] : U[1];
    const double vk = mk * X[0];
    F[0] = mk;
#pragma unroll
    for (int l = 0; l < DIM; ++l) F[1 + l] = U[1 + l] * vk + (l == k ? p : 0.0);
    F[DIM + 1] = vk * (U[DIM + 1] + p);
  }
}

// The two-rarefaction bound of the Euler wave speeds (Guermond and Popov,
// J. Comput. Phys. 2016, valid for 1 < gamma <= 5/3) from the normal
// velocities and the auxiliaries X = (1/rho, c, c p^-ex, (gamma+1)/(2 gamma
// p)) of the left and right states: with
// p* = ((c_L + c_R - (gamma-1)/2 (v_R - v_L))_+ / (c_L p_L^-ex + c_R p_R^-ex))^(1/ex),
// lambda = max((v_L - c_L sqrt(1 + (gamma+1)/(2 gamma) (p* - p_L)_+ / p_L))_-,
//              (v_R + c_R sqrt(1 + (gamma+1)/(2 gamma) (p* - p_R)_+ / p_R))_+).
template <int GN>
__device__ inline double euler_lambda(double vl, double vr, const double* XL, const double* XR, const Phys& ph) {
  const double num = fmax(fma(-ph.g1, vr - vl, XL[1] + XR[1]), 0.0);
  const double base = num * rcp_nr(XL[2] + XR[2]);   // c p^-ex > 0 on both sides
  double pstar;
  if constexpr (GN > 0) pstar = ipow_c<GN + 2>(base);
  else pstar = ph.inv_ex_int ? ipow(base, ph.inv_ex_int) : pow(base, ph.inv_ex);
  const double tl = fmax(fma(pstar, XL[3], -ph.fac), 0.0);
  const double tr = fmax(fma(pstar, XR[3], -ph.fac), 0.0);
  const double lam_l = fma(-XL[1], sqrt_ge1(1.0 + tl), vl);
  const double lam_r = fma(XR[1], sqrt_ge1(1.0 + tr), vr);
  return fmax(fmax(-lam_l, lam_r), 0.0);
}

// Upper bound of the maximum wave speed of the Riemann problem (UL | UR)
// along +e_K.
template <int EQ, int DIM, int K>
__device__ inline double lambda_k(const double* UL, const double* XL, const double* UR, const double* XR,
                                  const Phys& ph) {
  if constexpr (EQ == EQ_ADV) {
    return fabs(vel_k(K, ph));
  } else if constexpr (EQ == EQ_ADVV) {
    // Sec. 3.3: dhat_ij = max(|chat_ij . beta_i|, |chat_ji . beta_j|)
    return fmax(fabs(XL[K]), fabs(XR[K]));
  } else if constexpr (EQ == EQ_BURG) {
    return fmax(fabs(UL[0]), fabs(UR[0])) * fabs(vel_k(K, ph));
  } else {
    return euler_lambda<gn_of(EQ)>(UL[1 + K] * XL[0], UR[1 + K] * XR[0], XL, XR, ph);
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
  const double kg = kmin * ph.igm1;
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

// sup { t in [0, U] : uL + t P admissible } for one subcell face of a node
// whose u^L is admissible, to within tol (as for entropy_root).  The first
// point is U.  Then Newton steps from the infeasible end hi; Phi is concave
// along the segment, so a Newton point tn lies at or above the root, and the
// point evaluated is tn - tol/2 instead of tn: if it is admissible, the root
// lies in [tn - tol/2, tn] and the search ends there; if not, it is the new
// infeasible end.  Without a usable tangent, or after three Newton steps in
// a row that do not halve, one bisection; a Newton step below tol/4 means
// hi sits on the root, and the next points are probes under hi at tol/2,
// doubling the distance after each inadmissible probe.
template <int DIM, int GN>
__device__ double entropy_root_face(const double* uL, const double* P, double U, double kmin, double pscale,
                                    const Phys& ph) {
  double us = 0.0, ps = pscale;
#pragma unroll
  for (int c = 0; c < DIM + 2; ++c) {
    us = fmax(us, fabs(uL[c]));
    ps = fmax(ps, fabs(P[c]));
  }
  const double tol = fmax(1e-15, 1e-14 * us / ps);
  double lo = 0.0, hi = U, fhi = -INFINITY, dhi = 0.0, rhi = 0.0;
  double t = U, prev = INFINITY, probe = 0.5 * tol;
  int slow = 0;
  bool below = false;   // t = tn - tol/2 under a Newton point tn
  for (int it = 0; it < 64; ++it) {
    const PhiVal e = phi_at<DIM, GN>(t, uL, P, kmin, ph);
    if (admissible(e)) {
      if (below || t >= U) return t;
      lo = t;
    } else {
      hi = t;
      fhi = e.phi;
      dhi = e.dphi;
      rhi = e.rho;
    }
    if (!(hi - lo > tol)) break;
    below = false;
    if (rhi > 0.0 && dhi < 0.0) {
      const double step = fhi / dhi;  // the Newton step from hi, >= 0
      if (step < 0.25 * tol) {        // hi sits on the root: probe under it
        t = hi - probe;
        probe *= 2.0;
      } else if (slow >= 3) {
        t = 0.5 * (lo + hi);
        slow = 0;
      } else {
        t = (hi - step) - 0.5 * tol;
        below = true;
        slow = step > 0.5 * prev ? slow + 1 : 0;
        prev = step;
      }
    } else {
      t = 0.5 * (lo + hi);
    }
    if (!(t > lo && t < hi)) {
      t = 0.5 * (lo + hi);
      below = false;
    }
  }
  return lo;
}

__device__ inline const Phys& ph_of(const StageArgs& A) { return A.ph; }

// ----------------------------------------------------------------------
// phases 1-2 shared by the stage and the time-step kernels
// ----------------------------------------------------------------------

// Halo slot h of a tile: its grid point (hi, hj) and the direction of the
// face it serves (x-halos: h < 2 GY, left then right; y-halos: bottom then
// top), and where its state comes from: the facing node of the
// neighbouring element (periodic wrap), or, on an open side of the box,
// the tile's own boundary node (ext), with the side and the boundary node's
// index along it.
struct Halo {
  int hi, hj, k, side, q;
  bool ext;
  long long g;
};
template <int DIM, int P, int TX, int TY>
__device__ inline bool halo_of(int h, const TileGeo& t, int nx, int ny, int open, Halo* r) {
  constexpr int N1 = P + 1, NP = DIM == 2 ? N1 * N1 : N1;
  constexpr int GX = TX * N1, GY = DIM == 2 ? TY * N1 : 1;
  if (h < 2 * GY) {
    const bool hiside = h >= GY;
    const int j = hiside ? h - GY : h;
    if (j >= (DIM == 2 ? t.th * N1 : 1)) return false;
    const int ey = t.ey0 + (DIM == 2 ? j / N1 : 0), b = DIM == 2 ? j % N1 : 0;
    r->hj = j;
    r->k = 0;
    r->side = hiside ? 1 : 0;
    r->q = DIM == 2 ? ey * N1 + b : 0;
    if (!hiside) {
      r->hi = -1;
      r->ext = (open & 1) && t.ex0 == 0;
      const int ex = r->ext ? t.ex0 : (t.ex0 == 0 ? nx - 1 : t.ex0 - 1);
      r->g = ((long long)ey * nx + ex) * NP + b * N1 + (r->ext ? 0 : P);
    } else {
      r->hi = t.tw * N1;
      const int exh = t.ex0 + t.tw;
      r->ext = (open & 1) && exh == nx;
      const int ex = r->ext ? exh - 1 : (exh == nx ? 0 : exh);
      r->g = ((long long)ey * nx + ex) * NP + b * N1 + (r->ext ? P : 0);
    }
    return true;
  }
  if constexpr (DIM == 2) {
    const bool hiside = h >= 2 * GY + GX;
    const int i = h - 2 * GY - (hiside ? GX : 0);
    if (i >= t.tw * N1) return false;
    const int ex = t.ex0 + i / N1, a = i % N1;
    r->hi = i;
    r->k = 1;
    r->side = hiside ? 3 : 2;
    r->q = ex * N1 + a;
    if (!hiside) {
      r->hj = -1;
      r->ext = (open & 2) && t.ey0 == 0;
      const int ey = r->ext ? t.ey0 : (t.ey0 == 0 ? ny - 1 : t.ey0 - 1);
      r->g = ((long long)ey * nx + ex) * NP + (r->ext ? 0 : P * N1) + a;
    } else {
      r->hj = t.th * N1;
      const int eyh = t.ey0 + t.th;
      r->ext = (open & 2) && eyh == ny;
      const int ey = r->ext ? eyh - 1 : (eyh == ny ? 0 : eyh);
      r->g = ((long long)ey * nx + ex) * NP + (r->ext ? P * N1 : 0) + a;
    }
    return true;
  }
  return false;
}

// Velocity of the node at global index g (EQ_ADVV): beta_x of its node row,
// beta_y of its node column.
template <int DIM, int P>
__device__ inline void field_at(long long g, int nx, const Phys& ph, double* X) {
  constexpr int N1 = P + 1, NP = N1 * N1;
  const int e = (int)(g / NP), s = (int)(g - (long long)e * NP);
  const int ey = e / nx, ex = e - ey * nx;
  X[0] = ph.vrow[ey * N1 + s / N1];
  X[1] = ph.vcol[ex * N1 + s % N1];
}

// The exterior state of an open side for halo slot hs (V holds the own
// boundary node's state on entry): the prescribed state, the own state
// (outflow) or the own state with the normal momentum reversed (slip).  The
// side's arrays are selected between the four pointers already loaded: an
// index into the argument struct at run time would move it to scratch.
template <int EQ, int DIM, int NC>
__device__ inline void exterior_state(const Bnd& bnd, const Halo& hs, int n, double* V) {
  const unsigned long long t0 = (unsigned long long)bnd.type[0], t1 = (unsigned long long)bnd.type[1];
  const unsigned long long t2 = (unsigned long long)bnd.type[2], t3 = (unsigned long long)bnd.type[3];
  const unsigned long long s0 = (unsigned long long)bnd.state[0], s1 = (unsigned long long)bnd.state[1];
  const unsigned long long s2 = (unsigned long long)bnd.state[2], s3 = (unsigned long long)bnd.state[3];
  const int sd = hs.side;
  const signed char* type = (const signed char*)(sd == 0 ? t0 : sd == 1 ? t1 : sd == 2 ? t2 : t3);
  const double* state = (const double*)(sd == 0 ? s0 : sd == 1 ? s1 : sd == 2 ? s2 : s3);
  const int ty = type[hs.q];
  if (ty == BC_STATE && state) {
#pragma unroll
    for (int c = 0; c < NC; ++c) V[c] = state[c * n + hs.q];
  } else if (ty == BC_SLIP && is_euler(EQ)) {
    if (hs.k == 0) V[1] = -V[1];
    else if constexpr (DIM == 2) V[2] = -V[2];
  }
}

// Phases 1-2: own nodes (one per thread, into Uown) and the halo ring
// (threads h < NH) into the slot grid, with their auxiliaries and, with
// FLUX, their fluxes.  Returns after the stores; the caller synchronises.
// On a curved mesh (CURV) every slot also stages its eight metric terms,
// the own nodes' flux grids hold the contravariant fluxes of the high-order
// terms (A_FX, A_FY) and of the corrected terms (A_GX, A_GY), halo slots
// store no flux (an element face takes the flux of both states along its
// normal), and *det receives det(J) of the own node.
template <int EQ, int DIM, int P, int TX, int TY, bool FLUX, bool CURV = false>
__device__ inline void load_tile(double* lds, const double* __restrict__ u, long long nn, const TileGeo& tg,
                                 int nx, int ny, const Phys& ph, const Bnd& bnd, double* Uown,
                                 unsigned int* bad_flag, const double* __restrict__ metric = nullptr,
                                 double* det = nullptr) {
  using C = Cfg<EQ, DIM, P, TX, TY, CURV>;
  constexpr int NC = C::NC, NP = C::NP, N1 = C::N1, NX = is_euler(EQ) ? 5 : C::NAUX > 0 ? C::NAUX : 1;
  constexpr int NXW = C::NAUX;   // auxiliaries stored in the slot arrays
  const int tid = threadIdx.x;
  const int j = tid / C::GX, i = tid - j * C::GX;
  const int lex = i / N1, ley = DIM == 2 ? j / N1 : 0;
  const bool own = tid < C::NOWN && lex < tg.tw && ley < tg.th;
  const int s = DIM == 2 ? (j - ley * N1) * N1 + (i - lex * N1) : i - lex * N1;
  const long long g = ((long long)(tg.ey0 + ley) * nx + tg.ex0 + lex) * NP + s;
  Halo hs;
  const bool halo = tid < C::NH && halo_of<DIM, P, TX, TY>(tid, tg, nx, ny, bnd.open, &hs);
  // both loads in flight before any use
  double V[NC], Mo[CURV ? 9 : 1], Mh[CURV ? 8 : 1];
  if (own) {
#pragma unroll
    for (int c = 0; c < NC; ++c) Uown[c] = u[c * nn + g];
    if constexpr (CURV) {
#pragma unroll
      for (int q = 0; q < 9; ++q) Mo[q] = metric[q * nn + g];
    }
  }
  if (halo) {
#pragma unroll
    for (int c = 0; c < NC; ++c) V[c] = u[c * nn + hs.g];
    if constexpr (CURV) {
#pragma unroll
      for (int q = 0; q < 8; ++q) Mh[q] = metric[q * nn + hs.g];
    }
  }
  bool bad = false;
  if (own) {
    const int t = C::sl(i, j);
    double X[NX], pr = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) lds[C::A_U + c * C::CSU + t] = Uown[c];
    if constexpr (is_euler(EQ)) {
      bool b;
      euler_aux<DIM, gn_of(EQ), FLUX>(Uown, ph, X, pr, b);
      bad |= b;
    } else if constexpr (EQ == EQ_ADVV) {
      field_at<DIM, P>(g, nx, ph, X);
    }
#pragma unroll
    for (int q = 0; q < NXW; ++q) lds[C::A_X + q * C::CSU + t] = X[q];
    if constexpr (FLUX && is_euler(EQ)) lds[C::S_AL + t] = X[4];
    if constexpr (CURV) {
#pragma clang fp contract(off)
      double Fx[NC], Fy[NC];
      flux_k<EQ, DIM>(0, Uown, X, pr, ph, Fx);
      flux_k<EQ, DIM>(1, Uown, X, pr, ph, Fy);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        lds[C::A_FX + c * C::CSX + C::fx(i, j)] = Mo[0] * Fx[c] + Mo[1] * Fy[c];
        lds[C::A_FY + c * C::CSY + C::fy(i, j)] = Mo[2] * Fx[c] + Mo[3] * Fy[c];
        lds[C::A_GX + c * C::CSX + C::fx(i, j)] = Mo[4] * Fx[c] + Mo[5] * Fy[c];
        lds[C::A_GY + c * C::CSY + C::fy(i, j)] = Mo[6] * Fx[c] + Mo[7] * Fy[c];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) lds[C::A_M + q * C::CSU + t] = Mo[q];
      *det = Mo[8];
    } else if constexpr (FLUX) {
      double F[NC];
      flux_k<EQ, DIM>(0, Uown, X, pr, ph, F);
#pragma unroll
      for (int c = 0; c < NC; ++c) lds[C::A_FX + c * C::CSX + C::fx(i, j)] = F[c];
      if constexpr (DIM == 2) {
        flux_k<EQ, DIM>(1, Uown, X, pr, ph, F);
#pragma unroll
        for (int c = 0; c < NC; ++c) lds[C::A_FY + c * C::CSY + C::fy(i, j)] = F[c];
      }
    }
  }
  if (halo) {
    if (hs.ext)   // exterior state of an open side
      exterior_state<EQ, DIM, NC>(bnd, hs, DIM == 1 ? 1 : (hs.side < 2 ? ny : nx) * N1, V);
    const int t = C::sl(hs.hi, hs.hj);
    double X[NX], pr = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) lds[C::A_U + c * C::CSU + t] = V[c];
    if constexpr (is_euler(EQ)) {
      bool b;
      euler_aux<DIM, gn_of(EQ), FLUX>(V, ph, X, pr, b);
      bad |= b;
    } else if constexpr (EQ == EQ_ADVV) {
      field_at<DIM, P>(hs.g, nx, ph, X);   // an exterior state sits at the own boundary node
    }
#pragma unroll
    for (int q = 0; q < NXW; ++q) lds[C::A_X + q * C::CSU + t] = X[q];
    if constexpr (FLUX && is_euler(EQ)) lds[C::S_AL + t] = X[4];
    if constexpr (CURV) {
#pragma unroll
      for (int q = 0; q < 8; ++q) lds[C::A_M + q * C::CSU + t] = Mh[q];
    } else if constexpr (FLUX) {
      double F[NC];
      flux_k<EQ, DIM>(hs.k, V, X, pr, ph, F);
      const int o = hs.k == 0 ? C::A_FX + C::fx(hs.hi, hs.hj) : C::A_FY + C::fy(hs.hi, hs.hj);
      const int cs = hs.k == 0 ? C::CSX : C::CSY;
#pragma unroll
      for (int c = 0; c < NC; ++c) lds[o + c * cs] = F[c];
    }
  }
  if (bad && bad_flag) atomicOr(bad_flag, 1u);
}

// The per-degree tables, fetched into registers by the first threads of
// the workgroup (thread t holds entry t of each table it covers) before the
// state loads are issued, and stored to LDS once the state has arrived, so
// that their latency hides under that of the state.
template <int P>
struct TableRegs {
  static constexpr int N1 = P + 1;
  double w, iw, nk, q, m;
  __device__ inline void fetch(const Tables& T, bool modal) {
    const int t = threadIdx.x;
    if (t < N1) {
      w = T.w[t];
      iw = T.iw[t];
      if (modal) nk = T.nk[t];
    }
    if (t < P * N1) q = T.Q[t];
    if (modal && t < N1 * N1) m = T.M[t];
  }
  // sm, snk: the modal map and norms (smoothness indicator), or NULL
  __device__ inline void store(double* sw, double* sq, double* siw, double* sm, double* snk) const {
    const int t = threadIdx.x;
    if (t < N1) {
      sw[t] = w;
      siw[t] = iw;
      if (snk) snk[t] = nk;
    }
    if (t < P * N1) sq[t] = q;
    if (sm && t < N1 * N1) sm[t] = m;
  }
};

// ----------------------------------------------------------------------
// phase 3: subcell faces
// ----------------------------------------------------------------------

// Face item q of direction K, kind INT (interior subcell faces) or element
// faces, of a tile.  Writes the low-order flux, the bar state of the
// limited component, on interior faces the antidiffusive flux, and the
// face's index in its face grid (o < 0: no face).
template <int EQ, int DIM, int P, int TX, int TY, int K, bool INT>
__device__ __forceinline__ void face_item(const double* lds, const Phys& ph, const Solve& S, int q,
                                          const TileGeo& tg, double* FLo, double* RBo, double& UBo, int& o) {
  using C = Cfg<EQ, DIM, P, TX, TY>;
  constexpr int NC = C::NC, N1 = C::N1, GX = C::GX, NX = C::NAUX > 0 ? C::NAUX : 1;
  int i, j, f = 0, el;
  if constexpr (K == 0) {
    const int jmax = DIM == 2 ? tg.th * N1 : 1;
    if constexpr (INT) {
      j = q / (TX * P);
      const int r = q - j * (TX * P);
      el = r / P;
      f = r - el * P + 1;
      i = el * N1 + f;
      if (!(j < jmax && el < tg.tw)) return;
    } else {
      j = q / (TX + 1);
      el = q - j * (TX + 1);
      i = el * N1;
      if (!(j < jmax && el <= tg.tw)) return;
    }
  } else {
    const int r = q / GX;
    i = q - r * GX;
    if constexpr (INT) {
      el = r / P;
      f = r - el * P + 1;
      j = el * N1 + f;
      if (!(i < tg.tw * N1 && el < tg.th)) return;
    } else {
      el = r;
      j = el * N1;
      if (!(i < tg.tw * N1 && el <= tg.th)) return;
    }
  }
  // The right state's slot is the left one's plus an offset the compiler
  // cannot see through, so it does not pair the left and right reads of a
  // component into one two-address LDS read (which measured slower: the
  // stage takes about 2 % longer with the pairs).
  int dR = K == 0 ? 1 : C::RP, dF = K == 0 ? 1 : GX;
  asm volatile("" : "+s"(dR), "+s"(dF));
  const int sL = K == 0 ? C::sl(i, j) - 1 : C::sl(i, j) - C::RP, sR = sL + dR;
  const double* Fg = lds + (K == 0 ? C::A_FX : C::A_FY);
  constexpr int FS = K == 0 ? C::CSX : C::CSY;
  const int fL = K == 0 ? C::fx(i, j) - 1 : C::fy(i, j) - GX, fR = fL + dF;
  double UL[NC], UR[NC], FL[NC], FR[NC], XL[NX], XR[NX];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    UL[c] = lds[C::A_U + c * C::CSU + sL];
    UR[c] = lds[C::A_U + c * C::CSU + sR];
    FL[c] = Fg[c * FS + fL];
    FR[c] = Fg[c * FS + fR];
  }
#pragma unroll
  for (int x = 0; x < C::NAUXF; ++x) {
    XL[x] = lds[C::A_X + x * C::CSU + sL];
    XR[x] = lds[C::A_X + x * C::CSU + sR];
  }
  const double lam = lambda_k<EQ, DIM, K>(UL, XL, UR, XR, ph);
#pragma unroll
  for (int c = 0; c < NC; ++c) FLo[c] = 0.5 * (FL[c] + FR[c]) - 0.5 * lam * (UR[c] - UL[c]);
  const double avg = 0.5 * (UL[0] + UR[0]);
  UBo = lam > 0.0 ? avg - (FR[0] - FL[0]) * (0.5 * rcp_nr(lam)) : avg;
  if constexpr (INT) {
    // f^H of the element line through this face, and rbar = s (f^L - f^H)
    const int tr = K == 0 ? j % N1 : i % N1;   // the line's transverse node index
    const double sc = DIM == 2 ? lds[C::S_W + tr] * (K == 0 ? S.hy : S.hx) : 1.0;
    const double* qr = lds + C::S_Q + (f - 1) * N1;
    const int base = K == 0 ? C::fx(el * N1, j) : C::fy(i, el * N1);
    constexpr int st = K == 0 ? 1 : GX;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double* Fl = Fg + c * FS + base;
      double fh = Fl[0];
#pragma unroll
      for (int e = 0; e <= P; ++e) fh += qr[e] * Fl[e * st];
      RBo[c] = sc * (FLo[c] - fh);
    }
  }
  o = K == 0 ? C::ox(i, j) : C::oy(i, j);
}

// Phase-3 chunk ch (wave-uniform) of a tile: element faces of x, interior
// faces of x, element faces of y, interior faces of y; the lane picks the
// item within the chunk.  Wave w takes chunks w, w + NW, ...: at p = 4 on
// 3 x 3 elements (eight chunks, four waves) wave 0, which also formed the
// halo slots in phase 2, gets the two cheaper element-face chunks.
template <int EQ, int DIM, int P, int TX, int TY>
__device__ __forceinline__ void face_chunk(const double* lds, const Phys& ph, const Solve& S, int ch, int lane,
                                           const TileGeo& tg, double* FLo, double* RBo, double& UBo, int& o) {
  using C = Cfg<EQ, DIM, P, TX, TY>;
  constexpr int X1 = C::CEX, X2 = X1 + C::CIX, Y1 = X2 + C::CEY;
  if (ch < X1) {
    face_item<EQ, DIM, P, TX, TY, 0, false>(lds, ph, S, ch * 64 + lane, tg, FLo, RBo, UBo, o);
  } else if (ch < X2) {
    face_item<EQ, DIM, P, TX, TY, 0, true>(lds, ph, S, (ch - X1) * 64 + lane, tg, FLo, RBo, UBo, o);
  } else if (ch < Y1) {
    if constexpr (DIM == 2)
      face_item<EQ, DIM, P, TX, TY, 1, false>(lds, ph, S, (ch - X2) * 64 + lane, tg, FLo, RBo, UBo, o);
  } else if (ch < C::NCHUNK) {
    if constexpr (DIM == 2)
      face_item<EQ, DIM, P, TX, TY, 1, true>(lds, ph, S, (ch - Y1) * 64 + lane, tg, FLo, RBo, UBo, o);
  }
}

// direction of phase-3 chunk ch
template <int EQ, int DIM, int P, int TX, int TY>
__device__ inline int chunk_dir(int ch) {
  using C = Cfg<EQ, DIM, P, TX, TY>;
  if constexpr (DIM == 1) return 0;
  return ch >= C::CEX + C::CIX ? 1 : 0;
}

// ----------------------------------------------------------------------
// curved meshes (Sec. 2.3 metric terms, Sec. 3.1 corrected terms)
// ----------------------------------------------------------------------
// The curved-only code below (and the curved blocks of load_tile and
// dt_face) is compiled without multiply-add contraction: the compiler
// otherwise fuses its products of metric terms and fluxes differently in
// the plain and the batched kernels, whose results must agree bitwise.

// The flux along a (scaled) normal n, F(U) . n.  X: the auxiliaries (Euler
// 1/rho first).
template <int EQ, int DIM>
__device__ inline void flux_dot(const double* U, const double* X, const Phys& ph, const double* n,
                                double* Fn) {
#pragma clang fp contract(off)
  if constexpr (EQ == EQ_ADV) {
    Fn[0] = (ph.vel0 * n[0] + ph.vel1 * n[1]) * U[0];
  } else if constexpr (EQ == EQ_BURG) {
    Fn[0] = 0.5 * U[0] * U[0] * (ph.vel0 * n[0] + ph.vel1 * n[1]);
  } else {
    const double mn = U[1] * n[0] + U[2] * n[1];
    const double vn = mn * X[0];
    const double pr = (ph.gamma - 1.0) * (U[3] - 0.5 * (U[1] * U[1] + U[2] * U[2]) * X[0]);
    Fn[0] = mn;
    Fn[1] = U[1] * vn + pr * n[0];
    Fn[2] = U[2] * vn + pr * n[1];
    Fn[3] = vn * (U[3] + pr);
  }
}

// Upper bound of the wave speeds of the Riemann problem (UL | UR) along
// the unit vector nh.
template <int EQ, int DIM>
__device__ inline double lambda_n(const double* UL, const double* XL, const double* UR, const double* XR,
                                  const double* nh, const Phys& ph) {
#pragma clang fp contract(off)
  if constexpr (EQ == EQ_ADV) {
    return fabs(ph.vel0 * nh[0] + ph.vel1 * nh[1]);
  } else if constexpr (EQ == EQ_BURG) {
    return fmax(fabs(UL[0]), fabs(UR[0])) * fabs(ph.vel0 * nh[0] + ph.vel1 * nh[1]);
  } else {
    return euler_lambda<gn_of(EQ)>((UL[1] * nh[0] + UL[2] * nh[1]) * XL[0],
                                   (UR[1] * nh[0] + UR[2] * nh[1]) * XR[0], XL, XR, ph);
  }
}

// The difference of the limited component's flux, F_0(UR) - F_0(UL), as a
// vector (the momentum for Euler).
template <int EQ>
__device__ inline void flux_diff0(const double* UL, const double* UR, const Phys& ph, double* d) {
#pragma clang fp contract(off)
  if constexpr (is_euler(EQ)) {
    d[0] = UR[1] - UL[1];
    d[1] = UR[2] - UL[2];
  } else {
    const double f = EQ == EQ_BURG ? 0.5 * (UR[0] * UR[0] - UL[0] * UL[0]) : UR[0] - UL[0];
    d[0] = f * ph.vel0;
    d[1] = f * ph.vel1;
  }
}

// Face item q of direction K (kind INT or element faces) of a tile on a
// curved mesh, the counterpart of face_item.  With J the corrected metric
// row K of a node (|J| its length, Jh = J/|J|):
//  - interior subcell face (L, R): the viscosity coefficient of eq. dij,
//    2 d_LR / w_t = max(|J_R| lambda(L, R, Jh_R), |J_L| lambda(L, R, Jh_L))
//    =: lt (the two wave speeds of eq. dij along n_LR and n_RL), the
//    low-order flux 1/2 (G_L + G_R) - lt/2 (U_R - U_L) from the corrected
//    contravariant fluxes G, the bar states of L and R,
//    1/2 (U_L + U_R) - J_R . (F_R - F_L) / (2 lt) and the same with J_L,
//    and rbar = w_t (f^L - f^H) with f^H from the high-order contravariant
//    fluxes;
//  - element face: the high-order metric row K of the lower node is the
//    face's scaled normal n, the flux is |n| times the Lax-Friedrichs flux
//    along n/|n| (F(U) . n taken from both states), and both bar states are
//    1/2 (U_L + U_R) - (n/|n|) . (F_R - F_L) / (2 lambda).
template <int EQ, int DIM, int P, int TX, int TY, int K, bool INT>
__device__ __forceinline__ void face_item_c(const double* lds, const Phys& ph, int q, const TileGeo& tg,
                                            double* FLo, double* RBo, double& UBo, double& UBo2, int& o) {
#pragma clang fp contract(off)
  using C = Cfg<EQ, DIM, P, TX, TY, true>;
  constexpr int NC = C::NC, N1 = C::N1, GX = C::GX, NX = C::NAUX > 0 ? C::NAUX : 1;
  int i, j, f = 0, el;
  if constexpr (K == 0) {
    const int jmax = tg.th * N1;
    if constexpr (INT) {
      j = q / (TX * P);
      const int r = q - j * (TX * P);
      el = r / P;
      f = r - el * P + 1;
      i = el * N1 + f;
      if (!(j < jmax && el < tg.tw)) return;
    } else {
      j = q / (TX + 1);
      el = q - j * (TX + 1);
      i = el * N1;
      if (!(j < jmax && el <= tg.tw)) return;
    }
  } else {
    const int r = q / GX;
    i = q - r * GX;
    if constexpr (INT) {
      el = r / P;
      f = r - el * P + 1;
      j = el * N1 + f;
      if (!(i < tg.tw * N1 && el < tg.th)) return;
    } else {
      el = r;
      j = el * N1;
      if (!(i < tg.tw * N1 && el <= tg.th)) return;
    }
  }
  const int sR = C::sl(i, j), sL = K == 0 ? sR - 1 : sR - C::RP;
  const int fR = K == 0 ? C::fx(i, j) : C::fy(i, j), fL = K == 0 ? fR - 1 : fR - GX;
  double UL[NC], UR[NC], XL[NX], XR[NX];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    UL[c] = lds[C::A_U + c * C::CSU + sL];
    UR[c] = lds[C::A_U + c * C::CSU + sR];
  }
#pragma unroll
  for (int x = 0; x < C::NAUXF; ++x) {
    XL[x] = lds[C::A_X + x * C::CSU + sL];
    XR[x] = lds[C::A_X + x * C::CSU + sR];
  }
  const double* M = lds + C::A_M;
  const double avg = 0.5 * (UL[0] + UR[0]);
  double dF[2];
  flux_diff0<EQ>(UL, UR, ph, dF);
  if constexpr (INT) {
    const double JL[2] = {M[(4 + 2 * K) * C::CSU + sL], M[(5 + 2 * K) * C::CSU + sL]};
    const double JR[2] = {M[(4 + 2 * K) * C::CSU + sR], M[(5 + 2 * K) * C::CSU + sR]};
    const double mL = sqrt(JL[0] * JL[0] + JL[1] * JL[1]), mR = sqrt(JR[0] * JR[0] + JR[1] * JR[1]);
    const double hL[2] = {JL[0] / mL, JL[1] / mL}, hR[2] = {JR[0] / mR, JR[1] / mR};
    const double lt = fmax(mR * lambda_n<EQ, DIM>(UL, XL, UR, XR, hR, ph),
                           mL * lambda_n<EQ, DIM>(UL, XL, UR, XR, hL, ph));
    const double* G = lds + (K == 0 ? C::A_GX : C::A_GY);
    constexpr int FS = K == 0 ? C::CSX : C::CSY;
#pragma unroll
    for (int c = 0; c < NC; ++c) FLo[c] = 0.5 * (G[c * FS + fL] + G[c * FS + fR]) - 0.5 * lt * (UR[c] - UL[c]);
    UBo = lt > 0.0 ? avg - (JR[0] * dF[0] + JR[1] * dF[1]) / (2.0 * lt) : avg;
    UBo2 = lt > 0.0 ? avg - (JL[0] * dF[0] + JL[1] * dF[1]) / (2.0 * lt) : avg;
    // f^H of the element line through this face, and rbar = w_t (f^L - f^H)
    const int tr = K == 0 ? j % N1 : i % N1;
    const double sc = lds[C::S_W + tr];
    const double* qr = lds + C::S_Q + (f - 1) * N1;
    const double* Fg = lds + (K == 0 ? C::A_FX : C::A_FY);
    const int base = K == 0 ? C::fx(el * N1, j) : C::fy(i, el * N1);
    constexpr int st = K == 0 ? 1 : GX;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double* Fl = Fg + c * FS + base;
      double fh = Fl[0];
#pragma unroll
      for (int e = 0; e <= P; ++e) fh += qr[e] * Fl[e * st];
      RBo[c] = sc * (FLo[c] - fh);
    }
  } else {
    const double n[2] = {M[(2 * K) * C::CSU + sL], M[(2 * K + 1) * C::CSU + sL]};
    const double mn = sqrt(n[0] * n[0] + n[1] * n[1]);
    const double nh[2] = {n[0] / mn, n[1] / mn};
    const double lam = lambda_n<EQ, DIM>(UL, XL, UR, XR, nh, ph);
    double FnL[NC], FnR[NC];
    flux_dot<EQ, DIM>(UL, XL, ph, n, FnL);
    flux_dot<EQ, DIM>(UR, XR, ph, n, FnR);
#pragma unroll
    for (int c = 0; c < NC; ++c) FLo[c] = 0.5 * (FnL[c] + FnR[c]) - 0.5 * (mn * lam) * (UR[c] - UL[c]);
    UBo = lam > 0.0 ? avg - (nh[0] * dF[0] + nh[1] * dF[1]) / (2.0 * lam) : avg;
    UBo2 = UBo;
  }
  o = K == 0 ? C::ox(i, j) : C::oy(i, j);
}

template <int EQ, int DIM, int P, int TX, int TY>
__device__ __forceinline__ void face_chunk_c(const double* lds, const Phys& ph, int ch, int lane,
                                             const TileGeo& tg, double* FLo, double* RBo, double& UBo,
                                             double& UBo2, int& o) {
  using C = Cfg<EQ, DIM, P, TX, TY, true>;
  constexpr int X1 = C::CEX, X2 = X1 + C::CIX, Y1 = X2 + C::CEY;
  if (ch < X1) {
    face_item_c<EQ, DIM, P, TX, TY, 0, false>(lds, ph, ch * 64 + lane, tg, FLo, RBo, UBo, UBo2, o);
  } else if (ch < X2) {
    face_item_c<EQ, DIM, P, TX, TY, 0, true>(lds, ph, (ch - X1) * 64 + lane, tg, FLo, RBo, UBo, UBo2, o);
  } else if (ch < Y1) {
    face_item_c<EQ, DIM, P, TX, TY, 1, false>(lds, ph, (ch - X2) * 64 + lane, tg, FLo, RBo, UBo, UBo2, o);
  } else if (ch < C::NCHUNK) {
    face_item_c<EQ, DIM, P, TX, TY, 1, true>(lds, ph, (ch - Y1) * 64 + lane, tg, FLo, RBo, UBo, UBo2, o);
  }
}

// Subcell-resolution smoothness factor of every element of the tile
// (Sec. 4.4) from the limited component in the slot grid: modal
// coefficients c = M u (tensor product in 2-D), the energy fraction of the
// modes of degree p in any variable, s_K = log10 of it and eps_K on the
// ramp 1/2 + 1/2 sin(pi (s_K - s0)/2) between s0 - 1 (0) and s0 + 1 (1).
// An element whose polynomial is zero is smooth (0).  Uses scr (2-D:
// 2 NE (p+1) + NE doubles, 1-D: NE) as scratch; returns the factor of the
// calling thread's element (own nodes), 1 for the others.  Sums run in a
// fixed order, so the result does not depend on the launch.
template <int EQ, int DIM, int P, int TX, int TY>
__device__ inline double smoothness_tile(const double* u0, const double* M, const double* nk, double s0,
                                         const TileGeo& tg, double* scr) {
  // no multiply-add contraction: the result must not depend on how the
  // kernel that inlines this is compiled (plain and batched agree bitwise)
#pragma clang fp contract(off)
  using C = Cfg<EQ, DIM, P, TX, TY>;
  constexpr int N1 = P + 1, NP = C::NP, NE = C::NE;
  const int tid = threadIdx.x;
  double* tot_h = scr;                                 // [2][NE*N1] row sums (2-D)
  double* eps_e = scr + (DIM == 2 ? 2 * NE * N1 : 0);  // [NE]
  auto valid = [&](int le) { return le < NE && le % TX < tg.tw && le / TX < tg.th; };
  auto at = [&](int le, int a, int b) { return u0[C::sl((le % TX) * N1 + a, (le / TX) * N1 + b)]; };
  if constexpr (DIM == 2) {
    // thread (element, x-mode k): the k-th x-modes of every row, then their
    // y-transforms, squared and weighted
    if (tid < NE * N1 && valid(tid / N1)) {
      const int le = tid / N1, k = tid - le * N1;
      double t[N1];
#pragma unroll
      for (int b = 0; b < N1; ++b) {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < N1; ++a) acc += M[k * N1 + a] * at(le, a, b);
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
      tot_h[NE * N1 + tid] = hi;
    }
    __syncthreads();
  }
  if (valid(tid)) {
    double tot = 0.0, hi = 0.0;
    if constexpr (DIM == 2) {
#pragma unroll
      for (int k = 0; k < N1; ++k) {
        tot += tot_h[tid * N1 + k];
        hi += tot_h[NE * N1 + tid * N1 + k];
      }
    } else {
#pragma unroll
      for (int k = 0; k < N1; ++k) {
        double c = 0.0;
#pragma unroll
        for (int a = 0; a < N1; ++a) c += M[k * N1 + a] * at(tid, a, 0);
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
  const int j = tid / C::GX, i = tid - j * C::GX;
  return tid < C::NOWN ? eps_e[(DIM == 2 ? (j / N1) * TX : 0) + i / N1] : 1.0;
}

// ----------------------------------------------------------------------
// the fused stage kernel
// ----------------------------------------------------------------------
// One tile of one solve, run by one workgroup of C::BS threads on C::LDS
// doubles of LDS, with the degree tables T.  Shared by the plain kernel
// (the tiles of one solve) and the batched work-list kernel (the tiles of
// every solve of one degree).
template <int EQ, int DIM, int P, int TX, int TY, bool CURV = false>
__device__ __forceinline__ void stage_tile(double* lds, const StageArgs& A, const Tables& T, const Bnd& bnd,
                                           int tile) {
  using C = Cfg<EQ, DIM, P, TX, TY, CURV>;
  static_assert(!CURV || (DIM == 2 && EQ != EQ_ADVV), "curved meshes: 2-D, flux F(u)");
  constexpr int NC = C::NC, NP = C::NP, N1 = C::N1, GX = C::GX;
  const int tid = threadIdx.x;
  const Solve& S = A.S;
  const TileGeo tg = tile_geo<DIM, TX, TY>(tile, S.ntx, S.nx, S.ny);
  if (tg.tw <= 0 || tg.th <= 0) return;  // whole workgroup
  const long long nn = S.nn;

  double dt = S.dt_dev ? S.dt_scale * S.dt_dev[0] : S.dt;
  if (!(dt < INFINITY)) dt = 0.0;  // no dissipation anywhere: nothing moves

  // the calling thread's own node: grid point (i, j) in row-major order
  // (consecutive lanes read consecutive LDS words: no bank conflicts), in
  // element (lex, ley) of the tile at local position (a, b)
  const int j = tid / GX, i = tid - j * GX;
  const int lex = i / N1, ley = DIM == 2 ? j / N1 : 0;
  const int a = i - lex * N1, b = DIM == 2 ? j - ley * N1 : 0;
  const int s = DIM == 2 ? b * N1 + a : a;
  const bool own = tid < C::NOWN && lex < tg.tw && ley < tg.th;
  const long long g = ((long long)(tg.ey0 + ley) * S.nx + tg.ex0 + lex) * NP + s;

  static_assert(P * (P + 1) <= C::BS && (P + 1) * (P + 1) <= C::BS, "one table entry per thread");
  const bool modal = A.limiter == LIM_SUBCELL_SI;
  TableRegs<P> tr;
  tr.fetch(T, modal);
  double U[NC], Un[NC];
  if (A.use_un && own) {
#pragma unroll
    for (int c = 0; c < NC; ++c) Un[c] = S.u_n[c * nn + g];
  }
  double detn = 1.0;   // det(J) of the own node (curved meshes)
  load_tile<EQ, DIM, P, TX, TY, true, CURV>(lds, S.u_s, nn, tg, S.nx, S.ny, A.ph, bnd, U,
                                            A.diag ? &A.diag->bad_input : nullptr, S.metric, &detn);
  tr.store(lds + C::S_W, lds + C::S_Q, lds + C::S_IW, modal ? lds + C::S_M : nullptr, modal ? lds + C::S_NK : nullptr);
  if (tid == 0) *reinterpret_cast<int*>(lds + C::S_LN) = 0;
  __syncthreads();

  // K_min over the node and its 2d grid neighbours (Euler), from the K of
  // every slot in the nodal-alpha array
  double kmin = INFINITY;
  if constexpr (is_euler(EQ)) {
    if (own) {
      const double* K = lds + C::S_AL;
      const int t = C::sl(i, j);
      kmin = fmin(K[t], fmin(K[t - 1], K[t + 1]));
      if constexpr (DIM == 2) kmin = fmin(kmin, fmin(K[t - C::RP], K[t + C::RP]));
    }
  }

  // smoothness factor of the node's element (SUBCELL_SI; p = 1 keeps the
  // strict bounds); the nodal-alpha array is free scratch until phase 4
  // once every K_min is formed
  double eps = 1.0;
  if constexpr (P > 1) {
    static_assert(DIM == 1 || 2 * C::NE * N1 + C::NE <= C::NOWN, "scratch for the smoothness factor");
    if (A.limiter == LIM_SUBCELL_SI) {
      if constexpr (is_euler(EQ)) __syncthreads();
      eps = smoothness_tile<EQ, DIM, P, TX, TY>(lds + C::A_U, lds + C::S_M, lds + C::S_NK, T.s0, tg,
                                                lds + C::S_AL);
    }
  }

  // ---- phase 3: subcell faces ----
  // one work item per subcell face, in wave-uniform chunks
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  double rFL[C::NITEM][NC], rRB[C::NITEM][NC], rUB[C::NITEM], rUB2[CURV ? C::NITEM : 1];
  int rO[C::NITEM];
#pragma unroll
  for (int it = 0; it < C::NITEM; ++it) {
    rUB[it] = 0.0;
    rO[it] = -1;
#pragma unroll
    for (int c = 0; c < NC; ++c) rFL[it][c] = rRB[it][c] = 0.0;
    if constexpr (CURV) {
      rUB2[it] = 0.0;
      face_chunk_c<EQ, DIM, P, TX, TY>(lds, A.ph, wv + it * C::NW, lane, tg, rFL[it], rRB[it], rUB[it],
                                       rUB2[it], rO[it]);
    } else {
      face_chunk<EQ, DIM, P, TX, TY>(lds, A.ph, S, wv + it * C::NW, lane, tg, rFL[it], rRB[it], rUB[it], rO[it]);
    }
  }
  __syncthreads();  // region A is dead from here on
#pragma unroll
  for (int it = 0; it < C::NITEM; ++it) {
    const int o = rO[it];
    if (o >= 0) {
      if (chunk_dir<EQ, DIM, P, TX, TY>(wv + it * C::NW) == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          lds[C::B_FLX + c * C::COX + o] = rFL[it][c];
          lds[C::B_RBX + c * C::COX + o] = rRB[it][c];
        }
        lds[C::B_UBX + o] = rUB[it];
        if constexpr (CURV) lds[C::B_UBX2 + o] = rUB2[it];
      } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          lds[C::B_FLY + c * C::COY + o] = rFL[it][c];
          lds[C::B_RBY + c * C::COY + o] = rRB[it][c];
        }
        lds[C::B_UBY + o] = rUB[it];
        if constexpr (CURV) lds[C::B_UBY2 + o] = rUB2[it];
      }
    }
  }
  __syncthreads();

  // ---- phase 4a: low-order state, bounds, Zalesak, entropy checks ----
  // the node's faces: x-faces i, i+1 of row j; y-faces j, j+1 of column i
  const int ox0 = C::ox(i, j), oy0 = C::oy(i, j);
  auto FLk = [&](int k, int c, int side) -> double {
    return k == 0 ? lds[C::B_FLX + c * C::COX + ox0 + side] : lds[C::B_FLY + c * C::COY + oy0 + side * GX];
  };
  auto RBk = [&](int k, int c, int side) -> double {
    return k == 0 ? lds[C::B_RBX + c * C::COX + ox0 + side] : lds[C::B_RBY + c * C::COY + oy0 + side * GX];
  };
  // the bar state of the node toward its neighbour on side `side` of
  // direction k (on a curved mesh the node is the right node of its side-0
  // face and the left node of its side-1 face)
  auto UBk = [&](int k, int side) -> double {
    if constexpr (CURV) {
      if (side == 0) return k == 0 ? lds[C::B_UBX2 + ox0] : lds[C::B_UBY2 + oy0];
    }
    return k == 0 ? lds[C::B_UBX + ox0 + side] : lds[C::B_UBY + oy0 + side * GX];
  };
  double uL[NC], alpha = 1.0, m = 1.0;
  bool lov = false;
  double kmin_dbg = 0.0, az_dbg = 1.0, umin = 0.0, umax = 0.0;
  int search = 0, check0 = 0;   // faces of this node for the search list; check u^L first
  double ubound = 0.0, g2s = 0.0, pss = 0.0;
  const double idt = dt > 0.0 ? 1.0 / dt : 0.0;
  double dtm = 0.0;
  if (own) {
    const double wa = lds[C::S_W + a];
    const double wb = DIM == 2 ? lds[C::S_W + b] : 1.0;
    double cx, cy;
    if constexpr (CURV) {
      // m = w_a w_b det(J); the line scale of the fluxes is w_b (x-lines)
      // or w_a (y-lines), so dt w_b / m = dt / (w_a det(J))
      m = wa * wb * detn;
      const double idet = 1.0 / detn;
      cx = dt * (lds[C::S_IW + a] * idet);
      cy = dt * (lds[C::S_IW + b] * idet);
      dtm = cx * lds[C::S_IW + b];
    } else {
      m = DIM == 2 ? wa * wb * S.hx * S.hy : wa * S.hx;
      cx = dt * (lds[C::S_IW + a] * S.ihx);
      cy = DIM == 2 ? dt * (lds[C::S_IW + b] * S.ihy) : 0.0;
      dtm = DIM == 2 ? cx * (lds[C::S_IW + b] * S.ihy) : cx;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double d = (FLk(0, c, 0) - FLk(0, c, 1)) * cx;
      if constexpr (DIM == 2) d += (FLk(1, c, 0) - FLk(1, c, 1)) * cy;
      uL[c] = U[c] + d;
    }
    umin = U[0];
    umax = U[0];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const double b1 = UBk(k, 0), b2 = UBk(k, 1);
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
        // of its subcell-face antidiffusive fluxes (zero on element faces);
        // Zalesak with that single contribution, then the entropy line
        // search along d; the element minimum is taken in phase 5
        double d[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < DIM; ++k) acc += RBk(k, c, 1) - RBk(k, c, 0);
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
        const double cp = RBk(k, 0, 1);
        const double cm = -RBk(k, 0, 0);
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
        const double ikg = (ph_of(A).gamma - 1.0) * rcp_nr(kmin);
        double us = 0.0, rmax = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) us = fmax(us, fabs(uL[c]));
#pragma unroll
        for (int k = 0; k < DIM; ++k)
#pragma unroll
          for (int c = 0; c < NC; ++c) rmax = fmax(rmax, fmax(fabs(RBk(k, c, 0)), fabs(RBk(k, c, 1))));
        int act = 0;
        if (g2 * rmax > 1e-14 * us) {
#pragma unroll
          for (int k = 0; k < DIM; ++k) {
#pragma unroll
            for (int sd = 0; sd < 2; ++sd) {
              // the partial state at alpha, uL + (alpha 2d dt/m) (+-rbar): the
              // screen only certifies with margins, so how its scale is
              // rounded does not matter (an uncertified face is searched
              // from the exact value at alpha)
              double R[NC];
              bool nz = false;
#pragma unroll
              for (int c = 0; c < NC; ++c) {
                R[c] = RBk(k, c, sd);
                nz |= R[c] != 0.0;
              }
              const double sc = (sd ? alpha : -alpha) * g2;
              if (nz && !surely_admissible<DIM, gn_of(EQ)>(sc, uL, R, kmin, ikg, ph_of(A)))
                act |= 1 << (2 * k + sd);
            }
          }
        }
        if (act) {
          const double zero[NC] = {};
          search = act;
          ubound = alpha;
          g2s = g2;
          pss = g2 * rmax;
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
      for (int c = 0; c < NC; ++c) lds[C::C_UL + c * C::CSO + tid] = uL[c];
      lds[C::C_KM + tid] = kmin;
      lds[C::C_AZ + tid] = ubound;
      lds[C::C_G2 + tid] = g2s;
      lds[C::C_PS + tid] = pss;
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
      const int nj = node / GX, ni = node - nj * GX;
      const double g2 = lds[C::C_G2 + node];
      const int nox = C::ox(ni, nj), noy = C::oy(ni, nj);
      auto rb = [&](int kk, int c, int side) -> double {
        return kk == 0 ? lds[C::B_RBX + c * C::COX + nox + side] : lds[C::B_RBY + c * C::COY + noy + side * GX];
      };
      double ul[NC], Pv[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        ul[c] = lds[C::C_UL + c * C::CSO + node];
        Pv[c] = g2 * (sd ? 1.0 : -1.0) * rb(k, c, sd);
      }
      const double km = lds[C::C_KM + node];
      bool feasible = true;
      if (item & 1) {
        const double zero[NC] = {};
        feasible = admissible(phi_at<DIM, gn_of(EQ)>(0.0, ul, zero, km, ph_of(A)));
      }
      const double t = feasible ? entropy_root_face<DIM, gn_of(EQ)>(ul, Pv, lds[C::C_AZ + node], km,
                                                                     lds[C::C_PS + node], ph_of(A))
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
      const double* ae = lds + C::S_AL + (ley * N1) * GX * (DIM == 2 ? 1 : 0) + lex * N1;
      for (int bb = 0; bb < (DIM == 2 ? N1 : 1); ++bb)
        for (int aa = 0; aa < N1; ++aa) alpha = fmin(alpha, ae[bb * GX + aa]);
    }
    limited = alpha < 1.0;
    if (A.trace) {
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
    const int stride[2] = {1, GX};
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      if (pos[k] < P) {
        const double ap = elementwise ? alpha : fmin(alpha, lds[C::S_AL + tid + stride[k]]);
#pragma unroll
        for (int c = 0; c < NC; ++c) corr[c] += ap * RBk(k, c, 1);
      }
      if (pos[k] > 0) {
        const double am = elementwise ? alpha : fmin(alpha, lds[C::S_AL + tid - stride[k]]);
#pragma unroll
        for (int c = 0; c < NC; ++c) corr[c] -= am * RBk(k, c, 0);
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double fe = uL[c] + dtm * corr[c];
      S.u_out[c * nn + g] = A.use_un ? A.a_s * Un[c] + A.b_s * fe : fe;
    }
  }
  if (A.diag) {
    const unsigned long long bl = __ballot(limited), be = __ballot(ent), bv = __ballot(lov);
    if ((tid & 63) == 0) {
      const int slot = (blockIdx.x * C::NW + (tid >> 6)) & (DIAG_SLOTS - 1);
      if (bl) atomicAdd(&A.diag->limited[slot], (unsigned long long)__popcll(bl));
      if (be) atomicAdd(&A.diag->entropy[slot], (unsigned long long)__popcll(be));
      if (bv) atomicOr(&A.diag->lo_violation, 1u);
    }
  }
}

template <int EQ, int DIM, int P, int TX, int TY, bool CURV = false>
__global__ __launch_bounds__((Cfg<EQ, DIM, P, TX, TY, CURV>::BS)) void stage_kernel(StageArgs A) {
  __shared__ double lds[Cfg<EQ, DIM, P, TX, TY, CURV>::LDS];
  stage_tile<EQ, DIM, P, TX, TY, CURV>(lds, A, A.T, A.bnd, xcd_tile(blockIdx.x, gridDim.x));
}

// ----------------------------------------------------------------------
// low-order CFL bound (eq. cfl-low): min over nodes of m_i/(2 sum dhat_ij)
// ----------------------------------------------------------------------
// The time-step kernel stages per slot only what the wave-speed bounds read:
// for Euler the velocity components and the auxiliaries c, c p^-ex,
// (gamma+1)/(2 gamma p); for Burgers the state; for a velocity field beta.
// Each quantity is one array of the slot grid (padded as the stage kernel's).
// On a curved mesh the slot also stages its eight metric terms.
template <int EQ, int DIM, int P, int TX, int TY, bool CURV = false>
struct DtCfg {
  using C = Cfg<EQ, DIM, P, TX, TY>;
  static constexpr int NWS = is_euler(EQ) ? DIM + 3 : EQ == EQ_BURG ? 1 : EQ == EQ_ADVV ? 2 : 0;
  static constexpr int WS = 0;                             // [NWS][CSU]
  static constexpr int WM = WS + NWS * C::CSU;             // curved: metric terms [8][CSU]
  static constexpr int LX = WM + (CURV ? 8 * C::CSU : 0);  // wave speeds of the x-faces [NOX]
  static constexpr int LY = LX + C::NOX;                   // of the y-faces [NOY]
  static constexpr int W = LY + C::NOY;                    // Gauss-Lobatto weights
  static constexpr int R = W + C::N1;                      // per-thread bounds [BS]
  static constexpr int LDS = R + C::BS;
  static constexpr int CX = (C::NOX + 63) / 64;            // chunks of x-faces
  static constexpr int CY = (C::NOY + 63) / 64;
  static constexpr int NWS1 = NWS > 0 ? NWS : 1;
};

// The wave-speed inputs of one state (the node at global index g for a
// velocity field); sets bad for a non-physical Euler state.
template <int EQ, int DIM, int P>
__device__ inline void wave_inputs(const double* U, long long g, int nx, const Phys& ph, double* ws) {
  if constexpr (is_euler(EQ)) {
    double X[5], pr;
    bool bad;
    euler_aux<DIM, gn_of(EQ), false>(U, ph, X, pr, bad);
#pragma unroll
    for (int k = 0; k < DIM; ++k) ws[k] = U[1 + k] * X[0];
    ws[DIM] = X[1];
    ws[DIM + 1] = X[2];
    ws[DIM + 2] = X[3];
  } else if constexpr (EQ == EQ_BURG) {
    ws[0] = U[0];
  } else if constexpr (EQ == EQ_ADVV) {
    field_at<DIM, P>(g, nx, ph, ws);
  }
}

// Wave-speed bound of the pair (left, right) along +e_K from the staged
// inputs: the same arithmetic as lambda_k.
template <int EQ, int DIM, int K>
__device__ inline double lambda_ws(const double* wl, const double* wr, const Phys& ph) {
  if constexpr (EQ == EQ_ADV) {
    return fabs(vel_k(K, ph));
  } else if constexpr (EQ == EQ_ADVV) {
    return fmax(fabs(wl[K]), fabs(wr[K]));
  } else if constexpr (EQ == EQ_BURG) {
    return fmax(fabs(wl[0]), fabs(wr[0])) * fabs(vel_k(K, ph));
  } else {
    const double XL[4] = {0.0, wl[DIM], wl[DIM + 1], wl[DIM + 2]};
    const double XR[4] = {0.0, wr[DIM], wr[DIM + 1], wr[DIM + 2]};
    return euler_lambda<gn_of(EQ)>(wl[K], wr[K], XL, XR, ph);
  }
}

// Wave speed of the pair (left, right) along the unit vector nh from the
// staged inputs (Euler: velocity components first, then c, c p^-ex,
// (gamma+1)/(2 gamma p)).
template <int EQ, int DIM>
__device__ inline double lambda_ws_n(const double* wl, const double* wr, const double* nh, const Phys& ph) {
#pragma clang fp contract(off)
  if constexpr (EQ == EQ_ADV) {
    return fabs(ph.vel0 * nh[0] + ph.vel1 * nh[1]);
  } else if constexpr (EQ == EQ_BURG) {
    return fmax(fabs(wl[0]), fabs(wr[0])) * fabs(ph.vel0 * nh[0] + ph.vel1 * nh[1]);
  } else {
    const double XL[4] = {0.0, wl[DIM], wl[DIM + 1], wl[DIM + 2]};
    const double XR[4] = {0.0, wr[DIM], wr[DIM + 1], wr[DIM + 2]};
    return euler_lambda<gn_of(EQ)>(wl[0] * nh[0] + wl[1] * nh[1], wr[0] * nh[0] + wr[1] * nh[1], XL, XR, ph);
  }
}

// Wave speed of face item q of direction K of a tile into the time-step
// kernel's arrays (every face of the tile: element faces and interior ones).
// On a curved mesh (CURV) the face's value is the one the stage kernel uses
// in its graph viscosity: max(|J_R| lambda(Jh_R), |J_L| lambda(Jh_L)) with
// the corrected metric rows J on an interior subcell face, and |n| lambda(n/|n|)
// with the high-order row of the lower node on an element face.
template <int EQ, int DIM, int P, int TX, int TY, int K, bool CURV = false>
__device__ __forceinline__ void dt_face(double* lds, const Phys& ph, int q, const TileGeo& tg) {
  using C = Cfg<EQ, DIM, P, TX, TY>;
  using D = DtCfg<EQ, DIM, P, TX, TY, CURV>;
  constexpr int N1 = C::N1;
  int i, j;
  if constexpr (K == 0) {
    j = q / C::FXP;
    i = q - j * C::FXP;
    if (!(j < (DIM == 2 ? tg.th * N1 : 1) && i <= tg.tw * N1)) return;
  } else {
    j = q / C::GX;
    i = q - j * C::GX;
    if (!(i < tg.tw * N1 && j <= tg.th * N1)) return;
  }
  int dR = K == 0 ? 1 : C::RP;   // opaque to the compiler, as in face_item
  asm volatile("" : "+s"(dR));
  const int sL = K == 0 ? C::sl(i, j) - 1 : C::sl(i, j) - C::RP, sR = sL + dR;
  double wl[D::NWS1], wr[D::NWS1];
#pragma unroll
  for (int x = 0; x < D::NWS; ++x) {
    wl[x] = lds[D::WS + x * C::CSU + sL];
    wr[x] = lds[D::WS + x * C::CSU + sR];
  }
  double lam;
  if constexpr (CURV) {
#pragma clang fp contract(off)
    const double* M = lds + D::WM;
    const bool elem = (K == 0 ? i : j) % N1 == 0;   // an element face
    if (elem) {
      const double n[2] = {M[(2 * K) * C::CSU + sL], M[(2 * K + 1) * C::CSU + sL]};
      const double mn = sqrt(n[0] * n[0] + n[1] * n[1]);
      const double nh[2] = {n[0] / mn, n[1] / mn};
      lam = mn * lambda_ws_n<EQ, DIM>(wl, wr, nh, ph);
    } else {
      const double JL[2] = {M[(4 + 2 * K) * C::CSU + sL], M[(5 + 2 * K) * C::CSU + sL]};
      const double JR[2] = {M[(4 + 2 * K) * C::CSU + sR], M[(5 + 2 * K) * C::CSU + sR]};
      const double mL = sqrt(JL[0] * JL[0] + JL[1] * JL[1]), mR = sqrt(JR[0] * JR[0] + JR[1] * JR[1]);
      const double hL[2] = {JL[0] / mL, JL[1] / mL}, hR[2] = {JR[0] / mR, JR[1] / mR};
      lam = fmax(mR * lambda_ws_n<EQ, DIM>(wl, wr, hR, ph), mL * lambda_ws_n<EQ, DIM>(wl, wr, hL, ph));
    }
  } else {
    lam = lambda_ws<EQ, DIM, K>(wl, wr, ph);
  }
  if constexpr (K == 0) lds[D::LX + C::ox(i, j)] = lam;
  else lds[D::LY + C::oy(i, j)] = lam;
}

// the minimum of one tile into *out
template <int EQ, int DIM, int P, int TX, int TY, bool CURV = false>
__device__ __forceinline__ void maxdt_tile(double* lds, const MaxDtArgs& A, const Tables& T, const Bnd& bnd,
                                           int tile, double* out) {
  using C = Cfg<EQ, DIM, P, TX, TY>;
  using D = DtCfg<EQ, DIM, P, TX, TY, CURV>;
  constexpr int NC = C::NC, NP = C::NP, N1 = C::N1, GX = C::GX;
  const int tid = threadIdx.x;
  const int nx = A.nx, ny = A.ny;
  const TileGeo tg = tile_geo<DIM, TX, TY>(tile, A.ntx, nx, ny);
  if (tg.tw <= 0 || tg.th <= 0) {   // whole workgroup
    if (tid == 0) *out = INFINITY;
    return;
  }
  const double wt = tid < N1 ? T.w[tid] : 0.0;   // stored once the state has arrived
  // own nodes (one per thread) and the halo ring (threads h < NH), as in
  // the stage kernel's load, but only the wave-speed inputs are staged
  const int j = tid / GX, i = tid - j * GX;
  const int lex = i / N1, ley = DIM == 2 ? j / N1 : 0;
  const bool own = tid < C::NOWN && lex < tg.tw && ley < tg.th;
  const int a = i - lex * N1, b = DIM == 2 ? j - ley * N1 : 0;
  const long long g = ((long long)(tg.ey0 + ley) * nx + tg.ex0 + lex) * NP + (DIM == 2 ? b * N1 + a : a);
  Halo hs;
  const bool halo = tid < C::NH && halo_of<DIM, P, TX, TY>(tid, tg, nx, ny, bnd.open, &hs);
  double Uo[NC], V[NC], Mo[CURV ? 9 : 1], Mh[CURV ? 8 : 1];
  if (own) {
#pragma unroll
    for (int c = 0; c < NC; ++c) Uo[c] = A.u[c * A.nn + g];
    if constexpr (CURV) {
#pragma unroll
      for (int q = 0; q < 9; ++q) Mo[q] = A.metric[q * A.nn + g];
    }
  }
  if (halo) {
#pragma unroll
    for (int c = 0; c < NC; ++c) V[c] = A.u[c * A.nn + hs.g];
    if constexpr (CURV) {
#pragma unroll
      for (int q = 0; q < 8; ++q) Mh[q] = A.metric[q * A.nn + hs.g];
    }
  }
  if (own) {
    double ws[D::NWS1];
    wave_inputs<EQ, DIM, P>(Uo, g, nx, A.ph, ws);
    const int t = C::sl(i, j);
#pragma unroll
    for (int x = 0; x < D::NWS; ++x) lds[D::WS + x * C::CSU + t] = ws[x];
    if constexpr (CURV) {
#pragma unroll
      for (int q = 0; q < 8; ++q) lds[D::WM + q * C::CSU + t] = Mo[q];
    }
  }
  if (halo) {
    if (hs.ext)   // exterior state of an open side
      exterior_state<EQ, DIM, NC>(bnd, hs, DIM == 1 ? 1 : (hs.side < 2 ? ny : nx) * N1, V);
    double ws[D::NWS1];
    wave_inputs<EQ, DIM, P>(V, hs.g, nx, A.ph, ws);
    const int t = C::sl(hs.hi, hs.hj);
#pragma unroll
    for (int x = 0; x < D::NWS; ++x) lds[D::WS + x * C::CSU + t] = ws[x];
    if constexpr (CURV) {
#pragma unroll
      for (int q = 0; q < 8; ++q) lds[D::WM + q * C::CSU + t] = Mh[q];
    }
  }
  if (tid < N1) lds[D::W + tid] = wt;
  __syncthreads();
  // wave-uniform chunks of 64 faces of one direction
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  for (int ch = wv; ch < D::CX + D::CY; ch += C::NW) {
    if (ch < D::CX) dt_face<EQ, DIM, P, TX, TY, 0, CURV>(lds, A.ph, ch * 64 + lane, tg);
    else if constexpr (DIM == 2) dt_face<EQ, DIM, P, TX, TY, 1, CURV>(lds, A.ph, (ch - D::CX) * 64 + lane, tg);
  }
  __syncthreads();
  double dti = INFINITY;
  if (own) {
    const double wa = lds[D::W + a];
    const double wb = DIM == 2 ? lds[D::W + b] : 1.0;
    const int o = C::ox(i, j);
    // curved: the wave speeds carry the metric scale; the line weight is
    // w_b (x-faces) or w_a (y-faces) and m = w_a w_b det(J)
    double den = (lds[D::LX + o] + lds[D::LX + o + 1]) * (DIM == 2 ? (CURV ? wb : wb * A.hy) : 1.0);
    if constexpr (DIM == 2) {
      const int oy = C::oy(i, j);
      den += (lds[D::LY + oy] + lds[D::LY + oy + GX]) * (CURV ? wa : wa * A.hx);
    }
    const double m = CURV ? wa * wb * Mo[8] : DIM == 2 ? wa * wb * A.hx * A.hy : wa * A.hx;
    dti = den > 0.0 ? m / den : INFINITY;
  }
  // every thread's bound to LDS; the first wave folds them, then across
  // its lanes
  lds[D::R + tid] = dti;
  __syncthreads();
  if (tid < 64) {
    double v = lds[D::R + tid];
#pragma unroll
    for (int w = 1; w < C::NW; ++w) v = fmin(v, lds[D::R + tid + 64 * w]);
    v = wave_min63(v);
    if (tid == 63) *out = v;
  }
}

template <int EQ, int DIM, int P, int TX, int TY, bool CURV = false>
__global__ __launch_bounds__((Cfg<EQ, DIM, P, TX, TY>::BS)) void maxdt_kernel(MaxDtArgs A) {
  __shared__ double lds[DtCfg<EQ, DIM, P, TX, TY, CURV>::LDS];
  maxdt_tile<EQ, DIM, P, TX, TY, CURV>(lds, A, A.T, A.bnd, xcd_tile(blockIdx.x, gridDim.x),
                                       A.partial + blockIdx.x);
}

// ----------------------------------------------------------------------
// tile shapes (TX x TY elements) per degree: variant 0 is a new handle's,
// variant 1 the alternative the tuner may pick
// ----------------------------------------------------------------------
constexpr int tile_x_for(int dim, int p, int variant) {
  if (dim == 1) return (variant == 0 ? 128 : 256) / (p + 1);
  constexpr int v0[9] = {0, 8, 5, 4, 3, 3, 5, 2, 3};
  constexpr int v1[9] = {0, 8, 7, 4, 5, 7, 2, 4, 2};
  return variant == 0 ? v0[p] : v1[p];
}
constexpr int tile_y_for(int dim, int p, int variant) {
  if (dim == 1) return 1;
  constexpr int v0[9] = {0, 8, 5, 4, 3, 2, 1, 2, 1};
  constexpr int v1[9] = {0, 4, 4, 2, 2, 1, 2, 1, 1};
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
template <int EQ, int DIM, int P, int TX, int TY, bool CURV = false>
__global__ __launch_bounds__((Cfg<EQ, DIM, P, TX, TY, CURV>::BS)) void batch_stage_kernel(BatchArgs B) {
  __shared__ double lds[Cfg<EQ, DIM, P, TX, TY, CURV>::LDS];
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
  stage_tile<EQ, DIM, P, TX, TY, CURV>(lds, A, pa->T, pa->bnd, B.item_tile[it]);
}

template <int EQ, int DIM, int P, int TX, int TY, bool CURV = false>
__global__ __launch_bounds__((Cfg<EQ, DIM, P, TX, TY>::BS)) void batch_maxdt_kernel(BatchDtArgs B) {
  __shared__ double lds[DtCfg<EQ, DIM, P, TX, TY, CURV>::LDS];
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
  A.ntx = pa->ntx;
  A.hx = pa->hx;
  A.hy = pa->hy;
  A.ph = pa->ph;
  A.metric = pa->metric;
  maxdt_tile<EQ, DIM, P, TX, TY, CURV>(lds, A, pa->T, pa->bnd, B.item_tile[it], B.partial + it);
}

template <int EQ, int DIM, int P, int TX, int TY, bool CURV = false>
void batch_kernels_e(BatchKernels* k) {
  k->stage = reinterpret_cast<const void*>(&batch_stage_kernel<EQ, DIM, P, TX, TY, CURV>);
  k->maxdt = reinterpret_cast<const void*>(&batch_maxdt_kernel<EQ, DIM, P, TX, TY, CURV>);
  k->block = Cfg<EQ, DIM, P, TX, TY>::BS;
  k->tile_x = TX;
  k->tile_y = DIM == 2 ? TY : 1;
}

template <int EQ, int DIM, int P>
void batch_kernels_t(int variant, BatchKernels* k) {
#if IDP_NUM_VARIANTS > 1
  if (variant == 1)
    return batch_kernels_e<EQ, DIM, P, tile_x_for(DIM, P, 1), tile_y_for(DIM, P, 1)>(k);
#endif
  (void)variant;
  batch_kernels_e<EQ, DIM, P, tile_x_for(DIM, P, 0), tile_y_for(DIM, P, 0)>(k);
}

// curved meshes: the work-list kernels of the first tile shape
template <int EQ, int DIM, int P>
int batch_kernels_curved_t(BatchKernels* k) {
  if constexpr (DIM == 2 && EQ != EQ_ADVV) {
    batch_kernels_e<EQ, DIM, P, tile_x_for(DIM, P, 0), tile_y_for(DIM, P, 0), true>(k);
    return 0;
  } else {
    (void)k;
    return -1;
  }
}

// tiles of a mesh of nx x ny elements
inline int num_tiles(int nx, int ny, int tx, int ty) { return ((nx + tx - 1) / tx) * ((ny + ty - 1) / ty); }

template <int EQ, int DIM, int P, int TX, int TY>
hipError_t launch_stage_t(const StageArgs& a, hipStream_t s) {
  using C = Cfg<EQ, DIM, P, TX, TY>;
  const int nb = num_tiles(a.S.nx, a.S.ny, TX, DIM == 2 ? TY : 1);
  hipLaunchKernelGGL((stage_kernel<EQ, DIM, P, TX, TY>), dim3(nb), dim3(C::BS), 0, s, a);
  return hipGetLastError();
}

template <int EQ, int DIM, int P, int TX, int TY>
hipError_t launch_maxdt_t(const MaxDtArgs& a, hipStream_t s) {
  using C = Cfg<EQ, DIM, P, TX, TY>;
  const int nb = num_tiles(a.nx, a.ny, TX, DIM == 2 ? TY : 1);
  hipLaunchKernelGGL((maxdt_kernel<EQ, DIM, P, TX, TY>), dim3(nb), dim3(C::BS), 0, s, a);
  return hipGetLastError();
}

template <int EQ, int DIM, int P>
hipError_t launch_stage_v(int variant, const StageArgs& a, hipStream_t s) {
#if IDP_NUM_VARIANTS > 1
  if (variant == 1) return launch_stage_t<EQ, DIM, P, tile_x_for(DIM, P, 1), tile_y_for(DIM, P, 1)>(a, s);
#endif
  (void)variant;
  return launch_stage_t<EQ, DIM, P, tile_x_for(DIM, P, 0), tile_y_for(DIM, P, 0)>(a, s);
}

template <int EQ, int DIM, int P>
hipError_t launch_maxdt_v(int variant, const MaxDtArgs& a, hipStream_t s) {
#if IDP_NUM_VARIANTS > 1
  if (variant == 1) return launch_maxdt_t<EQ, DIM, P, tile_x_for(DIM, P, 1), tile_y_for(DIM, P, 1)>(a, s);
#endif
  (void)variant;
  return launch_maxdt_t<EQ, DIM, P, tile_x_for(DIM, P, 0), tile_y_for(DIM, P, 0)>(a, s);
}

// Curved meshes: one kernel per degree, on the first tile shape.
template <int EQ, int DIM, int P>
hipError_t launch_stage_curved_t(const StageArgs& a, hipStream_t s) {
  if constexpr (DIM == 2 && EQ != EQ_ADVV) {
    constexpr int TX = tile_x_for(DIM, P, 0), TY = tile_y_for(DIM, P, 0);
    using C = Cfg<EQ, DIM, P, TX, TY, true>;
    const int nb = num_tiles(a.S.nx, a.S.ny, TX, TY);
    hipLaunchKernelGGL((stage_kernel<EQ, DIM, P, TX, TY, true>), dim3(nb), dim3(C::BS), 0, s, a);
    return hipGetLastError();
  } else {
    (void)a;
    (void)s;
    return hipErrorInvalidValue;
  }
}

template <int EQ, int DIM, int P>
hipError_t launch_maxdt_curved_t(const MaxDtArgs& a, hipStream_t s) {
  if constexpr (DIM == 2 && EQ != EQ_ADVV) {
    constexpr int TX = tile_x_for(DIM, P, 0), TY = tile_y_for(DIM, P, 0);
    using C = Cfg<EQ, DIM, P, TX, TY>;
    const int nb = num_tiles(a.nx, a.ny, TX, TY);
    hipLaunchKernelGGL((maxdt_kernel<EQ, DIM, P, TX, TY, true>), dim3(nb), dim3(C::BS), 0, s, a);
    return hipGetLastError();
  } else {
    (void)a;
    (void)s;
    return hipErrorInvalidValue;
  }
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
  hipError_t launch_stage_curved_##NAME(int p, const StageArgs& a, hipStream_t s) {       \
    switch (p) {                                                                         \
      case 1: return launch_stage_curved_t<EQ, DIM, 1>(a, s);                            \
      case 2: return launch_stage_curved_t<EQ, DIM, 2>(a, s);                            \
      case 3: return launch_stage_curved_t<EQ, DIM, 3>(a, s);                            \
      case 4: return launch_stage_curved_t<EQ, DIM, 4>(a, s);                            \
      case 5: return launch_stage_curved_t<EQ, DIM, 5>(a, s);                            \
      case 6: return launch_stage_curved_t<EQ, DIM, 6>(a, s);                            \
      case 7: return launch_stage_curved_t<EQ, DIM, 7>(a, s);                            \
      case 8: return launch_stage_curved_t<EQ, DIM, 8>(a, s);                            \
    }                                                                                    \
    return hipErrorInvalidValue;                                                         \
  }                                                                                      \
  hipError_t launch_maxdt_curved_##NAME(int p, const MaxDtArgs& a, hipStream_t s) {       \
    switch (p) {                                                                         \
      case 1: return launch_maxdt_curved_t<EQ, DIM, 1>(a, s);                            \
      case 2: return launch_maxdt_curved_t<EQ, DIM, 2>(a, s);                            \
      case 3: return launch_maxdt_curved_t<EQ, DIM, 3>(a, s);                            \
      case 4: return launch_maxdt_curved_t<EQ, DIM, 4>(a, s);                            \
      case 5: return launch_maxdt_curved_t<EQ, DIM, 5>(a, s);                            \
      case 6: return launch_maxdt_curved_t<EQ, DIM, 6>(a, s);                            \
      case 7: return launch_maxdt_curved_t<EQ, DIM, 7>(a, s);                            \
      case 8: return launch_maxdt_curved_t<EQ, DIM, 8>(a, s);                            \
    }                                                                                    \
    return hipErrorInvalidValue;                                                         \
  }                                                                                      \
  void tile_dims_##NAME(int p, int variant, int* tx, int* ty) {                          \
    *tx = tile_x_for(DIM, p, variant);                                                   \
    *ty = tile_y_for(DIM, p, variant);                                                   \
  }                                                                                      \
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
  int batch_kernels_curved_##NAME(int p, BatchKernels* k) {                             \
    switch (p) {                                                                         \
      case 1: return batch_kernels_curved_t<EQ, DIM, 1>(k);                              \
      case 2: return batch_kernels_curved_t<EQ, DIM, 2>(k);                              \
      case 3: return batch_kernels_curved_t<EQ, DIM, 3>(k);                              \
      case 4: return batch_kernels_curved_t<EQ, DIM, 4>(k);                              \
      case 5: return batch_kernels_curved_t<EQ, DIM, 5>(k);                              \
      case 6: return batch_kernels_curved_t<EQ, DIM, 6>(k);                              \
      case 7: return batch_kernels_curved_t<EQ, DIM, 7>(k);                              \
      case 8: return batch_kernels_curved_t<EQ, DIM, 8>(k);                              \
    }                                                                                    \
    return -1;                                                                           \
  }                                                                                      \
  int num_variants_##NAME(int p) {                                                       \
    (void)p;                                                                             \
    return IDP_NUM_VARIANTS;                                                             \
  }

}  // namespace idp
