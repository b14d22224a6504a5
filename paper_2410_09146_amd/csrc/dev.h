// Device math for the gfx950 GRMHD stage: analytic metric, Valencia
// conserved/flux/speed evaluation, reconstruction, inversion.  Every function
// is inlined into the kernels of grmhd.hip.
//
// The metric family covered has gamma_12 = gamma_23 = 0 and shift only along
// x1: Minkowski-Cartesian and Kerr-Schild in (ln r, theta, phi).  The code is
// written for exactly that structure (11 scalars per point) to keep FP64
// register pressure down.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace grmhd {

enum { MK_MINK = 0, MK_KS = 1 };
enum { RC_CONST = 0, RC_PLM_MC = 1, RC_WENO = 2, RC_PLM_MINMOD = 3, RC_MP5 = 4 };
enum { RS_HLL = 0, RS_LLF = 1 };

// ------------------------------------------------------------------ layout

struct BlockInfo {
  int n[3];          // interior cells
  int s[3];          // padded extent n + 2 ng
  long long off;     // cell offset of the block in every variable plane
  double dx[3];
  int tab1, tab2;    // offsets of the block's rows in the 1-D coordinate tables
  int pole_lo, pole_hi;  // local x2 face index of a polar face, or -1
  int pad[2];
};

struct Tables {      // Kerr-Schild 1-D coordinate tables (ghost rows mirrored)
  const double *rc, *rf;          // r at x1 centres / lower faces
  const double *sc, *cc, *sf, *cf;  // sin, cos theta at x2 centres / lower faces
};

struct MetricP { double M, a; };

struct EosP {
  double gam, rho_flr0, rho_flr_pow, u_flr0, u_flr_pow, W_max, tol;
  int max_iter;
};

// Tabulated EOS (Sec. 2.2 tabulated EOS, Sec. 3.2 table bounds): nodes
// uniform in (ln rho, ln eps, Y_e), node (i, j, k) at d[i + nx (j + ny k)]
// holding (ln p, Gamma_1), Gamma_1 = d ln p / d ln rho at constant entropy
// (rho h c_s^2 = Gamma_1 p).  Trilinear between nodes; coordinates outside
// the table are clamped onto it.  d == nullptr: the ideal gas of EosP.
struct EosTab {
  const double2 *d;
  int nx, ny, nz;
  double lo[3], hi[3], ih[3];            // first / last node, 1 / spacing per axis
  double rho_min, rho_max, eps_min, eps_max;
};

// ------------------------------------------------------------------ metric
//
// Everything below is templated on the arithmetic type T: FP64 everywhere in
// the default path; the mixed-precision flux path instantiates the geometry,
// reconstruction and Riemann solve with float (the densitization by sqrt(-g),
// U, the face field, the RK accumulation and the inversion stay FP64).

template <typename T> struct Lim;
template <> struct Lim<double> {
  static constexpr double weno_eps = 1e-40;
  static constexpr bool clamp = false;
  static constexpr double rmax = 0.0;
};
template <> struct Lim<float> {
  // (tau/(beta+eps))^2 must stay finite in FP32
  static constexpr float weno_eps = 1e-20f;
  static constexpr bool clamp = true;
  static constexpr float rmax = 1e15f;
};

// 1/d for finite d != 0: the hardware reciprocal estimate refined by two
// Newton-Raphson steps r <- r + r (1 - d r), each squaring the relative error
// (within an ulp or two of the rounded quotient; not for zero, infinite or
// subnormal d).
__device__ __forceinline__ double rcp_nr(double d)
{
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// 1/x in arithmetic T: FP64 through rcp_nr (x finite, normal, nonzero);
// FP32 through the hardware division; the operation counter sees a division.
template <typename T>
__device__ __forceinline__ T inv(T x)
{
#ifndef GRMHD_OPCOUNT
  if constexpr (sizeof(T) == sizeof(double)) return rcp_nr(x);
#endif
  return T(1) / x;
}

template <typename T>
struct GeoT {
  T alpha, ialpha, beta1;       // lapse, its inverse, shift (x1 component only)
  T g11, g13, g22, g33;         // gamma_ij
  T gi11, gi13, gi22, gi33;     // gamma^ij
  T sqrtg;                      // sqrt(gamma)
};
using Geo = GeoT<double>;

template <typename T = double>
__device__ __forceinline__ GeoT<T> geo_mink()
{
  GeoT<T> G;
  G.alpha = T(1); G.ialpha = T(1); G.beta1 = T(0);
  G.g11 = T(1); G.g13 = T(0); G.g22 = T(1); G.g33 = T(1);
  G.gi11 = T(1); G.gi13 = T(0); G.gi22 = T(1); G.gi33 = T(1);
  G.sqrtg = T(1);
  return G;
}

// Kerr-Schild at (r, sin theta, cos theta), x1 = ln r.  With Sigma = r^2 +
// a^2 cos^2, z = 2 M r / Sigma:  alpha = (1+z)^-1/2, beta^1 = z/((1+z) r),
// gamma_11 = r^2 (1+z), gamma_13 = -a (1+z) sin^2 r, gamma_22 = Sigma,
// gamma_33 = sin^2 (Sigma + a^2 (1+z) sin^2); the (1,3) block has
// determinant r^2 (1+z) sin^2 Sigma, so sqrt(gamma) = r Sigma sin sqrt(1+z).
template <typename T = double>
__device__ __forceinline__ GeoT<T> geo_ks(T r, T s, T c, T M, T a)
{
  const T a2 = a * a, s2 = s * s;
  const T Sig = fma(a2 * c, c, r * r);
  const T iSig = inv(Sig);
  const T z = T(2) * M * r * iSig;
  const T opz = T(1) + z;
  const T sq = sqrt(opz);
  GeoT<T> G;
  // 1/r, 1/sqrt(1+z) and 1/((1+z) sin^2) from one division (sin^2 = 0 only
  // on pole faces, whose fluxes are zero and never evaluated)
  const T s2q = s2 > T(0) ? s2 : T(1);
  const T osq = opz * s2q;
  const T Q = inv(r * sq * osq);
  const T ir = Q * sq * osq;
  G.alpha = Q * r * osq;
  G.ialpha = sq;
  G.beta1 = z * G.alpha * G.alpha * ir;
  G.g11 = r * r * opz;
  G.g13 = -a * opz * s2 * r;
  G.g22 = Sig;
  G.g33 = s2 * fma(a2 * opz, s2, Sig);
  const T idet = iSig * ir * ir * (Q * r * sq);
  G.gi11 = G.g33 * idet;
  G.gi13 = -G.g13 * idet;
  G.gi33 = G.g11 * idet;
  G.gi22 = iSig;
  G.sqrtg = r * Sig * s * sq;
  return G;
}

__device__ __forceinline__ Geo geo_ks(double r, double s, double c, const MetricP &m)
{
  return geo_ks<double>(r, s, c, m.M, m.a);
}

template <int MK, typename T = double>
__device__ __forceinline__ GeoT<T> geo_at(const Tables &Tb, const MetricP &m, int ir, bool rface,
                                          int it, bool tface)
{
  if constexpr (MK == MK_MINK) {
    return geo_mink<T>();
  } else {
    const double r = rface ? Tb.rf[ir] : Tb.rc[ir];
    const double s = tface ? Tb.sf[it] : Tb.sc[it];
    const double c = tface ? Tb.cf[it] : Tb.cc[it];
    return geo_ks<T>(T(r), T(s), T(c), T(m.M), T(m.a));
  }
}

// ------------------------------------------------------------------ physics

template <typename T> struct PrimT { T rho, u1, u2, u3, ie, B1, B2, B3, ye; };
using Prim = PrimT<double>;

// Auxiliary 4-vector quantities of a primitive state (Sec. 2.1 kinematics and
// the b^mu / B^i relation).
template <typename T>
struct AuxT {
  T W, ut2, v1, v2, v3, vl1, vl2, vl3, Bv;
  T iW, iW1;              // 1 / W, 1 / (W + 1)
  T uc1, uc2, uc3;        // u^i (contravariant four-velocity)
  T b0, bc1, bc2, bc3;    // b^mu
  T bl1, bl2, bl3;        // b_i
  T b2, p, w;             // b^2, pressure, rho h
  T gp;                   // Gamma_1 p = rho h c_s^2
};
using Aux = AuxT<double>;

// Kinematics of q with the thermodynamics (p, Gamma_1 p) supplied.
template <typename T>
__device__ __forceinline__ AuxT<T> aux_th(const GeoT<T> &G, const PrimT<T> &q, T p, T gp)
{
  AuxT<T> A;
  A.ut2 = G.g11 * q.u1 * q.u1 + T(2) * G.g13 * q.u1 * q.u3 + G.g22 * q.u2 * q.u2 +
          G.g33 * q.u3 * q.u3;
  A.W = sqrt(T(1) + A.ut2);
  // 1/W and 1/(W + 1) from one division
  const T iWW1 = inv(A.W * (A.W + T(1)));
  const T iW = (A.W + T(1)) * iWW1;
  A.iW = iW;
  A.iW1 = A.W * iWW1;
  A.v1 = q.u1 * iW; A.v2 = q.u2 * iW; A.v3 = q.u3 * iW;
  A.vl1 = G.g11 * A.v1 + G.g13 * A.v3;
  A.vl2 = G.g22 * A.v2;
  A.vl3 = G.g13 * A.v1 + G.g33 * A.v3;
  A.Bv = q.B1 * A.vl1 + q.B2 * A.vl2 + q.B3 * A.vl3;
  const T Bl1 = G.g11 * q.B1 + G.g13 * q.B3;
  const T Bl2 = G.g22 * q.B2;
  const T Bl3 = G.g13 * q.B1 + G.g33 * q.B3;
  const T BB = q.B1 * Bl1 + q.B2 * Bl2 + q.B3 * Bl3;
  const T ia = G.ialpha;
  // u^i = W v^i - W beta^i / alpha;  b^i = B^i / W + (alpha b^0 / W) u^i,
  // alpha b^0 = W (B . v)
  A.uc1 = q.u1 - A.W * G.beta1 * ia;
  A.uc2 = q.u2;
  A.uc3 = q.u3;
  A.b0 = A.W * A.Bv * ia;
  A.bc1 = q.B1 * iW + A.Bv * A.uc1;
  A.bc2 = q.B2 * iW + A.Bv * A.uc2;
  A.bc3 = q.B3 * iW + A.Bv * A.uc3;
  // b_i = beta_i b^0 + gamma_ij b^j  (beta_1 = g11 beta^1, beta_3 = g13 beta^1)
  A.bl1 = G.g11 * (G.beta1 * A.b0 + A.bc1) + G.g13 * A.bc3;
  A.bl2 = G.g22 * A.bc2;
  A.bl3 = G.g13 * (G.beta1 * A.b0 + A.bc1) + G.g33 * A.bc3;
  A.b2 = BB * iW * iW + A.Bv * A.Bv;
  A.p = p;
  A.gp = gp;
  A.w = q.rho + q.ie + A.p;
  return A;
}

// Ideal gas: p = (gam - 1) u, Gamma_1 = gam.
template <typename T>
__device__ __forceinline__ AuxT<T> aux_of(const GeoT<T> &G, T gam, const PrimT<T> &q)
{
  const T p = (gam - T(1)) * q.ie;
  return aux_th(G, q, p, gam * p);
}

// ------------------------------------------------------------- tabulated EOS

// One axis of the table lookup: cell i in [0, n-2] and weight w of x clamped
// into [lo, hi]; inside = x strictly within (the derivative along the axis
// is zero on the clamped part).  A NaN coordinate lands on lo (fmax / fmin
// return the non-NaN operand), so the cell index is always in range.
__device__ __forceinline__ void tab_axis(double x, double lo, double hi, double ih, int n, int &i,
                                         double &w, bool &inside)
{
  inside = x > lo && x < hi;
  const double t = (fmin(fmax(x, lo), hi) - lo) * ih;
  const int k = min((int)t, n - 2);
  i = k;
  w = t - (double)k;
}

struct TabV { double L, G1, Lx, Ly; };   // ln p, Gamma_1, d ln p / d ln rho, d ln p / d ln eps

// Trilinear lookup at (x, y, z) = (ln rho, ln eps, Y_e); with DER also the
// two partial derivatives of the interpolant of ln p.
template <bool DER>
__device__ __forceinline__ TabV tab_eval(const EosTab &t, double x, double y, double z)
{
  int i, j, k;
  double wx, wy, wz;
  bool inx, iny, inz;
  tab_axis(x, t.lo[0], t.hi[0], t.ih[0], t.nx, i, wx, inx);
  tab_axis(y, t.lo[1], t.hi[1], t.ih[1], t.ny, j, wy, iny);
  tab_axis(z, t.lo[2], t.hi[2], t.ih[2], t.nz, k, wz, inz);
  const long long sy = t.nx, sz = (long long)t.nx * t.ny;
  const double2 *b = t.d + (i + sy * j + sz * k);
  const double2 c000 = b[0], c100 = b[1], c010 = b[sy], c110 = b[sy + 1];
  const double2 c001 = b[sz], c101 = b[sz + 1], c011 = b[sz + sy], c111 = b[sz + sy + 1];
  auto lerp = [](double a, double c, double w) { return fma(w, c - a, a); };
  TabV v;
  const double l00 = lerp(c000.x, c100.x, wx), l10 = lerp(c010.x, c110.x, wx);
  const double l01 = lerp(c001.x, c101.x, wx), l11 = lerp(c011.x, c111.x, wx);
  const double l0 = lerp(l00, l10, wy), l1 = lerp(l01, l11, wy);
  v.L = lerp(l0, l1, wz);
  const double g00 = lerp(c000.y, c100.y, wx), g10 = lerp(c010.y, c110.y, wx);
  const double g01 = lerp(c001.y, c101.y, wx), g11 = lerp(c011.y, c111.y, wx);
  v.G1 = lerp(lerp(g00, g10, wy), lerp(g01, g11, wy), wz);
  v.Lx = v.Ly = 0.0;
  if constexpr (DER) {
    if (inx) {
      const double d0 = lerp(c100.x - c000.x, c110.x - c010.x, wy);
      const double d1 = lerp(c101.x - c001.x, c111.x - c011.x, wy);
      v.Lx = lerp(d0, d1, wz) * t.ih[0];
    }
    if (iny) v.Ly = lerp(l10 - l00, l11 - l01, wz) * t.ih[1];
  }
  (void)inz;
  return v;
}

// p and Gamma_1 p of (rho, u, Y_e) from the table (rho, u > 0).
__device__ __forceinline__ void tab_thermo(const EosTab &t, double rho, double u, double ye,
                                           double &p, double &gp)
{
  const double x = log(rho);
  const TabV v = tab_eval<false>(t, x, log(u) - x, ye);
  p = exp(v.L);
  gp = v.G1 * p;
}

// Undensitized conserved vector (D, S_j, tau, B^k).
template <typename T>
__device__ __forceinline__ void cons_of(const GeoT<T> &G, const PrimT<T> &q, const AuxT<T> &A,
                                        T U[8])
{
  const T W2 = A.W * A.W;
  const T D = q.rho * A.W;
  const T wt = A.w + A.b2;
  const T ab0 = A.W * A.Bv;     // alpha b^0
  U[0] = D;
  U[1] = wt * W2 * A.vl1 - ab0 * A.bl1;
  U[2] = wt * W2 * A.vl2 - ab0 * A.bl2;
  U[3] = wt * W2 * A.vl3 - ab0 * A.bl3;
  // tau with the rest-mass part rho (W^2 - W) = D ut2 / (W + 1)
  U[4] = D * A.ut2 * A.iW1 + (q.ie + A.p + A.b2) * W2 - (A.p + T(0.5) * A.b2) - ab0 * ab0;
  U[5] = q.B1; U[6] = q.B2; U[7] = q.B3;
}

// Undensitized flux along direction DIR (0,1,2) given U.
template <int DIR, typename T>
__device__ __forceinline__ void flux_of(const GeoT<T> &G, const PrimT<T> &q, const AuxT<T> &A,
                                        const T U[8], T F[8])
{
  const T ia = G.ialpha;
  const T vt1 = G.alpha * A.v1 - G.beta1, vt2 = G.alpha * A.v2, vt3 = G.alpha * A.v3;
  const T vtd = DIR == 0 ? vt1 : (DIR == 1 ? vt2 : vt3);
  const T vd = DIR == 0 ? A.v1 : (DIR == 1 ? A.v2 : A.v3);
  const T Bd = DIR == 0 ? q.B1 : (DIR == 1 ? q.B2 : q.B3);
  const T pt = A.p + T(0.5) * A.b2;
  const T iW = A.iW;
  const T adv = vtd * ia;
  F[0] = U[0] * adv;
  F[1] = U[1] * adv - A.bl1 * Bd * iW + (DIR == 0 ? pt : T(0));
  F[2] = U[2] * adv - A.bl2 * Bd * iW + (DIR == 1 ? pt : T(0));
  F[3] = U[3] * adv - A.bl3 * Bd * iW + (DIR == 2 ? pt : T(0));
  F[4] = U[4] * adv + pt * vd - A.Bv * Bd;
  F[5] = (q.B1 * vtd - Bd * vt1) * ia;
  F[6] = (q.B2 * vtd - Bd * vt2) * ia;
  F[7] = (q.B3 * vtd - Bd * vt3) * ia;
}

// Fast-wave coordinate speeds along DIR from (k.u)^2 (1 - c^2) = c^2 k.k,
// k_mu = (-lambda, e_DIR), c^2 = cs^2 + ca^2 - cs^2 ca^2.
template <int DIR, typename T>
__device__ __forceinline__ void speeds_of(const GeoT<T> &G, const AuxT<T> &A, T &lm, T &lp)
{
  // c^2 = cs^2 + ca^2 - cs^2 ca^2 = 1 - (1 - cs^2)(1 - ca^2), with
  // cs^2 = Gamma_1 p / w and ca^2 = b^2 / (w + b^2), is N / Dn with
  // N = Gamma_1 p + b^2, Dn = w + b^2.  The roots of the quadratic do not
  // change when all three coefficients are multiplied by Dn > 0, so c^2
  // enters as (1 - c^2) Dn = Dn - N and c^2 Dn = N, with no division.
  const T Nc = A.gp + A.b2;
  const T omc = (A.w + A.b2) - Nc;
  const T ia = G.ialpha;
  const T ia2 = ia * ia;
  const T u0 = A.W * ia;
  const T ud = DIR == 0 ? A.uc1 : (DIR == 1 ? A.uc2 : A.uc3);
  const T g00 = -ia2;
  const T g0d = DIR == 0 ? G.beta1 * ia2 : T(0);
  const T gdd = DIR == 0 ? G.gi11 - G.beta1 * G.beta1 * ia2 : (DIR == 1 ? G.gi22 : G.gi33);
  const T qa = omc * u0 * u0 - Nc * g00;
  const T qb = T(-2) * (omc * u0 * ud - Nc * g0d);
  const T qc = omc * ud * ud - Nc * gdd;
  T disc = qb * qb - T(4) * qa * qc;
  disc = disc > T(0) ? disc : T(0);
  const T sq = sqrt(disc);
  const T i2a = T(0.5) * inv(qa);
  const T l1 = (-qb + sq) * i2a, l2 = (-qb - sq) * i2a;
  lp = fmax(l1, l2);
  lm = fmin(l1, l2);
}

// The operation counter counts the plain definitions (both roots, then the
// largest magnitude), not the shortcuts below.
#ifdef GRMHD_OPCOUNT
constexpr bool COUNTING = true;
#else
constexpr bool COUNTING = false;
#endif

// max(|lambda_-|, |lambda_+|) of speeds_of: (|qb| + sqrt(disc)) |1 / (2 qa)|,
// the same number as the larger magnitude of the two roots computed there.
template <int DIR, typename T>
__device__ __forceinline__ T speed_absmax(const GeoT<T> &G, const AuxT<T> &A)
{
  const T Nc = A.gp + A.b2;
  const T omc = (A.w + A.b2) - Nc;
  const T ia = G.ialpha;
  const T ia2 = ia * ia;
  const T u0 = A.W * ia;
  const T ud = DIR == 0 ? A.uc1 : (DIR == 1 ? A.uc2 : A.uc3);
  const T g00 = -ia2;
  const T g0d = DIR == 0 ? G.beta1 * ia2 : T(0);
  const T gdd = DIR == 0 ? G.gi11 - G.beta1 * G.beta1 * ia2 : (DIR == 1 ? G.gi22 : G.gi33);
  const T qa = omc * u0 * u0 - Nc * g00;
  const T qb = T(-2) * (omc * u0 * ud - Nc * g0d);
  const T qc = omc * ud * ud - Nc * gdd;
  T disc = qb * qb - T(4) * qa * qc;
  disc = disc > T(0) ? disc : T(0);
  const T sq = sqrt(disc);
  const T i2a = T(0.5) * inv(qa);
  return (fabs(qb) + sq) * fabs(i2a);
}

// Face flux of the law d_t(sqrt(gamma) U) + d_i(sqrt(-g) F^i) = ..., returned
// as two undensitized parts: the densitized flux is sqrt(-g) A + sqrt(gamma) B
// (the speeds are eigenvalues of d(sqrt(-g)F)/d(sqrt(gamma)U), so the
// dissipation B acts on sqrt(gamma) U).  The caller densitizes in FP64.
// (pL, gpL), (pR, gpR): pressure and Gamma_1 p of the two states.  NSC = 1
// adds the passive scalar as component 8: conserved D Y_e, flux Y_e F_D.
template <int DIR, int RS, typename T, int NSC = 0>
__device__ __forceinline__ void riemann_parts(const GeoT<T> &G, const PrimT<T> &L,
                                              const PrimT<T> &R, T pL, T gpL, T pR, T gpR,
                                              T A[8 + NSC], T B[8 + NSC])
{
  constexpr int NC = 8 + NSC;
  T UL[NC], UR[NC], FL[NC], FR[NC], lmL, lpL, lmR, lpR;
  {
    const AuxT<T> X = aux_th(G, L, pL, gpL);
    cons_of(G, L, X, UL);
    flux_of<DIR>(G, L, X, UL, FL);
    if constexpr (RS == RS_HLL || COUNTING) speeds_of<DIR>(G, X, lmL, lpL);
    else lpL = speed_absmax<DIR>(G, X), lmL = T(0);
    if constexpr (NSC != 0) { UL[8] = UL[0] * L.ye; FL[8] = FL[0] * L.ye; }
  }
#ifndef GRMHD_OPCOUNT
  // the right state after the left: interleaved by the scheduler, the two
  // states' temporaries pushed the x2 tiles past 128 VGPRs (2 spilled)
  __builtin_amdgcn_sched_barrier(0);
#endif
  {
    const AuxT<T> X = aux_th(G, R, pR, gpR);
    cons_of(G, R, X, UR);
    flux_of<DIR>(G, R, X, UR, FR);
    if constexpr (RS == RS_HLL || COUNTING) speeds_of<DIR>(G, X, lmR, lpR);
    else lpR = speed_absmax<DIR>(G, X), lmR = T(0);
    if constexpr (NSC != 0) { UR[8] = UR[0] * R.ye; FR[8] = FR[0] * R.ye; }
  }
  if constexpr (RS == RS_HLL) {
    const T cm = fmin(T(0), fmin(lmL, lmR));
    const T cp = fmax(T(0), fmax(lpL, lpR));
    const T den = cp - cm;
    if (den > T(0)) {
      const T id = T(1) / den;
      const T a = cp * id, b = cm * id, c = cp * cm * id;
#pragma unroll
      for (int v = 0; v < NC; ++v) { A[v] = a * FL[v] - b * FR[v]; B[v] = c * (UR[v] - UL[v]); }
    } else {
#pragma unroll
      for (int v = 0; v < NC; ++v) { A[v] = T(0.5) * (FL[v] + FR[v]); B[v] = T(0); }
    }
  } else {
    const T c = COUNTING ? fmax(fmax(fabs(lmL), fabs(lpL)), fmax(fabs(lmR), fabs(lpR)))
                         : fmax(lpL, lpR);      // the largest |lambda| of either state
    const T hc = T(-0.5) * c;
#pragma unroll
    for (int v = 0; v < NC; ++v) { A[v] = T(0.5) * (FL[v] + FR[v]); B[v] = hc * (UR[v] - UL[v]); }
  }
}

// FP64 densitized face flux, ideal gas.
template <int DIR, int RS>
__device__ __forceinline__ void riemann(const Geo &G, double gam, const Prim &L, const Prim &R,
                                        double out[8])
{
  double A[8], B[8];
  const double pL = (gam - 1.0) * L.ie, pR = (gam - 1.0) * R.ie;
  riemann_parts<DIR, RS, double>(G, L, R, pL, gam * pL, pR, gam * pR, A, B);
  const double smg = G.alpha * G.sqrtg, sg = G.sqrtg;
#pragma unroll
  for (int v = 0; v < 8; ++v) out[v] = smg * A[v] + sg * B[v];
}

// ---------------------------------------------------------- reconstruction

template <typename T>
__device__ __forceinline__ T mc_slope(T dm, T dp)
{
  if (dm * dp <= T(0)) return T(0);
  const T a = fmin(fmin(T(2) * fabs(dm), T(2) * fabs(dp)), T(0.5) * fabs(dm + dp));
  return dm > T(0) ? a : -a;
}

template <typename T>
__device__ __forceinline__ T minmod_slope(T dm, T dp)
{
  if (dm * dp <= T(0)) return T(0);
  const T a = fmin(fabs(dm), fabs(dp));
  return dm > T(0) ? a : -a;
}

// One WENO5-Z face value at x_{j+1/2} from f0..f4 = f_{j-2..j+2}; also the
// per-face measure 3 w0 w1 w2 / (g2 w0 w1 + g1 w0 w2 + g0 w1 w2).
template <int FV, typename T>
__device__ __forceinline__ T weno_z_face(T f0, T f1, T f2, T f3, T f4, T &sig)
{
  constexpr T g0 = FV ? T(0.1) : T(1.0 / 16.0);
  constexpr T g1 = FV ? T(0.6) : T(10.0 / 16.0);
  constexpr T g2 = FV ? T(0.3) : T(5.0 / 16.0);
  const T t0 = f0 - T(2) * f1 + f2, s0 = f0 - T(4) * f1 + T(3) * f2;
  const T t1 = f1 - T(2) * f2 + f3, s1 = f1 - f3;
  const T t2 = f2 - T(2) * f3 + f4, s2 = T(3) * f2 - T(4) * f3 + f4;
  constexpr T c13 = T(13.0 / 12.0);
  const T b0 = c13 * t0 * t0 + T(0.25) * s0 * s0;
  const T b1 = c13 * t1 * t1 + T(0.25) * s1 * s1;
  const T b2 = c13 * t2 * t2 + T(0.25) * s2 * s2;
  const T tau = fabs(b0 - b2);
  constexpr T eps = Lim<T>::weno_eps;
  T r0 = tau / (b0 + eps), r1 = tau / (b1 + eps), r2 = tau / (b2 + eps);
  if constexpr (Lim<T>::clamp) {
    r0 = fmin(r0, Lim<T>::rmax); r1 = fmin(r1, Lim<T>::rmax); r2 = fmin(r2, Lim<T>::rmax);
  }
  const T a0 = g0 * (T(1) + r0 * r0), a1 = g1 * (T(1) + r1 * r1), a2 = g2 * (T(1) + r2 * r2);
  const T is = T(1) / (a0 + a1 + a2);
  const T w0 = a0 * is, w1 = a1 * is, w2 = a2 * is;
  T p0, p1, p2;
  if constexpr (FV) {
    p0 = (T(2) * f0 - T(7) * f1 + T(11) * f2) * T(1.0 / 6.0);
    p1 = (-f1 + T(5) * f2 + T(2) * f3) * T(1.0 / 6.0);
    p2 = (T(2) * f2 + T(5) * f3 - f4) * T(1.0 / 6.0);
  } else {
    p0 = (T(3) * f0 - T(10) * f1 + T(15) * f2) * T(0.125);
    p1 = (-f1 + T(6) * f2 + T(3) * f3) * T(0.125);
    p2 = (T(3) * f2 + T(6) * f3 - f4) * T(0.125);
  }
  const T w01 = w0 * w1;
  sig = T(3) * w01 * w2 / (g2 * w01 + g1 * w0 * w2 + g0 * w1 * w2);
  return w0 * p0 + w1 * p1 + w2 * p2;
}

// Both WENO5-Z faces of cell j in FP64 with three divisions instead of
// eleven.  The smoothness indicators of the left face are those of the right
// face mirrored (beta_0 <-> beta_2), and with q_k = beta_k + eps the weights
// alpha_k = gamma_k (1 + (tau/q_k)^2) are proportional to the homogeneous
//   a_k = gamma_k (q_k^2 + tau^2) prod_{m != k} q_m^2,
// so one division normalises each face (q >= eps = 1e-40 keeps every a_k a
// normal number for |f| below ~1e25).  The blend sigma = 2 s+ s- / (s+ + s-)
// of the per-face measures s = N / D (N = 3 w0 w1 w2, D = g2 w0 w1 + g1 w0 w2
// + g0 w1 w2) is 2 N+ N- / (N+ D- + N- D+): the third division.  Returns
// false (and nothing) if a normalising sum is not a finite positive number.
template <int FV>
__device__ __forceinline__ bool weno_pair(double f0, double f1, double f2, double f3, double f4,
                                          double &pl, double &pr, double &sigma)
{
  constexpr double g0 = FV ? 0.1 : 1.0 / 16.0;
  constexpr double g1 = FV ? 0.6 : 10.0 / 16.0;
  constexpr double g2 = FV ? 0.3 : 5.0 / 16.0;
  const double t0 = f0 - 2.0 * f1 + f2, s0 = f0 - 4.0 * f1 + 3.0 * f2;
  const double t1 = f1 - 2.0 * f2 + f3, s1 = f1 - f3;
  const double t2 = f2 - 2.0 * f3 + f4, s2 = 3.0 * f2 - 4.0 * f3 + f4;
  constexpr double c13 = 13.0 / 12.0;
  const double b0 = c13 * t0 * t0 + 0.25 * s0 * s0;
  const double b1 = c13 * t1 * t1 + 0.25 * s1 * s1;
  const double b2 = c13 * t2 * t2 + 0.25 * s2 * s2;
  const double tau = fabs(b0 - b2), tt = tau * tau;
  constexpr double eps = Lim<double>::weno_eps;
  const double q0 = b0 + eps, q1 = b1 + eps, q2 = b2 + eps;
  const double E0 = q0 * q0 + tt, E1 = q1 * q1 + tt, E2 = q2 * q2 + tt;
  const double m01 = q0 * q1, m02 = q0 * q2, m12 = q1 * q2;
  const double Q01 = m01 * m01, Q02 = m02 * m02, Q12 = m12 * m12;
  // right face j+1/2 and its mirror j-1/2
  const double ar0 = g0 * E0 * Q12, ar1 = g1 * E1 * Q02, ar2 = g2 * E2 * Q01;
  const double al0 = g0 * E2 * Q01, al1 = g1 * E1 * Q02, al2 = g2 * E0 * Q12;
  const double Sr = ar0 + ar1 + ar2, Sl = al0 + al1 + al2;
  if (!(Sr > 1e-300 && Sr <= 1e300 && Sl > 1e-300 && Sl <= 1e300)) return false;
  const double ir = rcp_nr(Sr), il = rcp_nr(Sl);
  const double wr0 = ar0 * ir, wr1 = ar1 * ir, wr2 = ar2 * ir;
  const double wl0 = al0 * il, wl1 = al1 * il, wl2 = al2 * il;
  // the candidates without their common factor (1/8, or 1/6 for cell
  // averages), applied once to each weighted sum: for 1/8 a power of two, so
  // the result is the same number as with the factor inside
  double pr0, pr1, pr2, pl0, pl1, pl2;
  constexpr double cs = FV ? 1.0 / 6.0 : 0.125;
  if constexpr (FV) {
    pr0 = 2.0 * f0 - 7.0 * f1 + 11.0 * f2;
    pr1 = -f1 + 5.0 * f2 + 2.0 * f3;
    pr2 = 2.0 * f2 + 5.0 * f3 - f4;
    pl0 = 2.0 * f4 - 7.0 * f3 + 11.0 * f2;
    pl1 = -f3 + 5.0 * f2 + 2.0 * f1;
    pl2 = 2.0 * f2 + 5.0 * f1 - f0;
  } else {
    pr0 = 3.0 * f0 - 10.0 * f1 + 15.0 * f2;
    pr1 = -f1 + 6.0 * f2 + 3.0 * f3;
    pr2 = 3.0 * f2 + 6.0 * f3 - f4;
    pl0 = 3.0 * f4 - 10.0 * f3 + 15.0 * f2;
    pl1 = -f3 + 6.0 * f2 + 3.0 * f1;
    pl2 = 3.0 * f2 + 6.0 * f1 - f0;
  }
  pr = (wr0 * pr0 + wr1 * pr1 + wr2 * pr2) * cs;
  pl = (wl0 * pl0 + wl1 * pl1 + wl2 * pl2) * cs;
  const double Nr = 3.0 * wr0 * wr1 * wr2, Dr = g2 * wr0 * wr1 + g1 * wr0 * wr2 + g0 * wr1 * wr2;
  const double Nl = 3.0 * wl0 * wl1 * wl2, Dl = g2 * wl0 * wl1 + g1 * wl0 * wl2 + g0 * wl1 * wl2;
  const double den = Nr * Dl + Nl * Dr;
  sigma = den > 1e-300 ? 2.0 * Nr * Nl * rcp_nr(den) : 0.0;
  return true;
}

// Monotonicity-preserving fifth-order face value at x_{j+1/2} (Suresh &
// Huynh 1997) from f0..f4 = f_{j-2..j+2}, alpha = 4: the unlimited value is
// kept when it lies between f_j and the monotone bound f_MP; otherwise it is
// moved into [f_min, f_max] built from the M4-limited curvatures.
template <typename T>
__device__ __forceinline__ T minmod4(T a, T b, T c, T d)
{
  const bool pos = a > T(0) && b > T(0) && c > T(0) && d > T(0);
  const bool neg = a < T(0) && b < T(0) && c < T(0) && d < T(0);
  const T m = fmin(fmin(fabs(a), fabs(b)), fmin(fabs(c), fabs(d)));
  return pos ? m : (neg ? -m : T(0));
}

template <int FV, typename T>
__device__ __forceinline__ T mp5_face(T fm2, T fm1, T f0, T fp1, T fp2)
{
  constexpr T alpha = T(4);
  const T f5 = FV ? (T(2) * fm2 - T(13) * fm1 + T(47) * f0 + T(27) * fp1 - T(3) * fp2) * T(1.0 / 60.0)
                  : (T(3) * fm2 - T(20) * fm1 + T(90) * f0 + T(60) * fp1 - T(5) * fp2) * T(1.0 / 128.0);
  const T fmp = f0 + minmod_slope(fp1 - f0, alpha * (f0 - fm1));
  if ((f5 - f0) * (f5 - fmp) <= T(0)) return f5;
  const T dm = fm2 - T(2) * fm1 + f0, d0 = fm1 - T(2) * f0 + fp1, dp = f0 - T(2) * fp1 + fp2;
  const T dM4p = minmod4(T(4) * d0 - dp, T(4) * dp - d0, d0, dp);
  const T dM4m = minmod4(T(4) * d0 - dm, T(4) * dm - d0, d0, dm);
  const T fUL = f0 + alpha * (f0 - fm1);
  const T fAV = T(0.5) * (f0 + fp1);
  const T fMD = fAV - T(0.5) * dM4p;
  const T fLC = f0 + T(0.5) * (f0 - fm1) + T(4.0 / 3.0) * dM4m;
  const T lo = fmax(fmin(fmin(f0, fp1), fMD), fmin(fmin(f0, fUL), fLC));
  const T hi = fmin(fmax(fmax(f0, fp1), fMD), fmax(fmax(f0, fUL), fLC));
  return f5 + minmod_slope(lo - f5, hi - f5);     // median(f5, lo, hi)
}

// WENO5-Z-AOAH without the per-face fallback: false (and nothing) where the
// shared-divisor pair cannot be normalised (then recon5 must be used); every
// other reconstruction is complete here.
template <int RECON, int FV, typename T>
__device__ __forceinline__ bool recon5_fast(T f0, T f1, T f2, T f3, T f4, T &fl, T &fr);

// Left (j-1/2) and right (j+1/2) face values of cell j.
template <int RECON, int FV, typename T>
__device__ __forceinline__ void recon5(T f0, T f1, T f2, T f3, T f4, T &fl, T &fr)
{
  if constexpr (RECON == RC_MP5) {
    fr = mp5_face<FV>(f0, f1, f2, f3, f4);
    fl = mp5_face<FV>(f4, f3, f2, f1, f0);
  } else if constexpr (RECON == RC_CONST) {
    fl = f2; fr = f2;
  } else if constexpr (RECON == RC_PLM_MINMOD) {
    const T s = minmod_slope(f2 - f1, f3 - f2);
    fl = f2 - T(0.5) * s; fr = f2 + T(0.5) * s;
  } else if constexpr (RECON == RC_PLM_MC) {
    const T s = mc_slope(f2 - f1, f3 - f2);
    fl = f2 - T(0.5) * s; fr = f2 + T(0.5) * s;
  } else {
    const T s = mc_slope(f2 - f1, f3 - f2);
    T pr = T(0), pl = T(0), sigma = T(0);
    bool done = false;
#ifndef GRMHD_OPCOUNT   // the operation count is taken on the per-face definition
    if constexpr (sizeof(T) == sizeof(double)) done = weno_pair<FV>(f0, f1, f2, f3, f4, pl, pr, sigma);
#endif
    if (!done) {
      T sp, sm;
      pr = weno_z_face<FV>(f0, f1, f2, f3, f4, sp);
      pl = weno_z_face<FV>(f4, f3, f2, f1, f0, sm);   // mirror x -> -x
      sigma = T(2) * sp * sm / (sp + sm);
    }
    sigma = sigma > T(0) ? sigma : T(0);                     // also maps NaN to 0
    sigma = sigma < T(1) ? sigma : T(1);
    fr = sigma * pr + (T(1) - sigma) * (f2 + T(0.5) * s);
    fl = sigma * pl + (T(1) - sigma) * (f2 - T(0.5) * s);
  }
}

template <int RECON, int FV, typename T>
__device__ __forceinline__ bool recon5_fast(T f0, T f1, T f2, T f3, T f4, T &fl, T &fr)
{
#ifndef GRMHD_OPCOUNT
  if constexpr (RECON == RC_WENO && sizeof(T) == sizeof(double)) {
    T pr, pl, sigma;
    if (!weno_pair<FV>(f0, f1, f2, f3, f4, pl, pr, sigma)) return false;
    const T s = mc_slope(f2 - f1, f3 - f2);
    sigma = sigma > T(0) ? sigma : T(0);                     // also maps NaN to 0
    sigma = sigma < T(1) ? sigma : T(1);
    fr = sigma * pr + (T(1) - sigma) * (f2 + T(0.5) * s);
    fl = sigma * pl + (T(1) - sigma) * (f2 - T(0.5) * s);
    return true;
  }
#endif
  recon5<RECON, FV, T>(f0, f1, f2, f3, f4, fl, fr);
  return true;
}

// --------------------------------------------------------- sources (KS)

struct Sym4 { double t00, t01, t02, t03, t11, t12, t13, t22, t23, t33; };

// sqrt(-g) (S_1, S_2, S_tau) at a cell centre of Kerr-Schild (x1 = ln r).
// S_j = T^{mu nu} d_j g_{mu nu} / 2;
// S_tau = alpha (T^{mu 0} d_mu ln alpha - T^{mu nu} Gamma^0_{mu nu}),
// Gamma^0_{mu nu} = (g^00 (d_mu g_0nu + d_nu g_0mu) + g^01 (d_mu g_1nu + d_nu g_1mu - d_1 g_mu nu))/2
// (KS: g^02 = g^03 = 0; stationary and axisymmetric, so only d_1, d_2 act).
__device__ __forceinline__ void ks_sources(double r, double s, double cth, const MetricP &m,
                                           const Geo &G, const Sym4 &T, double &S1, double &S2,
                                           double &St)
{
  const double a = m.a, a2 = a * a, s2 = s * s, ds2 = 2.0 * s * cth;
  const double Sig = r * r + a2 * cth * cth;
  const double iSig = 1.0 / Sig;
  const double z = 2.0 * m.M * r * iSig;
  const double opz = 1.0 + z;
  const double r2 = r * r;
  const double dz1 = z * (1.0 - 2.0 * r2 * iSig);
  const double dz2 = z * 2.0 * a2 * cth * s * iSig;
  // d_1 g
  const double a00 = dz1, a01 = r * dz1 + z * r, a03 = -a * s2 * dz1;
  const double a11 = r2 * dz1 + 2.0 * opz * r2, a13 = -a * s2 * (r * dz1 + opz * r);
  const double a22 = 2.0 * r2, a33 = s2 * (2.0 * r2 + a2 * s2 * dz1);
  // d_2 g
  const double dSig2 = -2.0 * a2 * cth * s;
  const double c00 = dz2, c01 = r * dz2, c03 = -a * (dz2 * s2 + z * ds2);
  const double c11 = r2 * dz2, c13 = -a * r * (dz2 * s2 + opz * ds2);
  const double c22 = dSig2;
  const double c33 = ds2 * (Sig + a2 * opz * s2) + s2 * (dSig2 + a2 * (dz2 * s2 + opz * ds2));
  S1 = 0.5 * (T.t00 * a00 + 2.0 * T.t01 * a01 + 2.0 * T.t03 * a03 + T.t11 * a11 +
              2.0 * T.t13 * a13 + T.t22 * a22 + T.t33 * a33);
  S2 = 0.5 * (T.t00 * c00 + 2.0 * T.t01 * c01 + 2.0 * T.t03 * c03 + T.t11 * c11 +
              2.0 * T.t13 * c13 + T.t22 * c22 + T.t33 * c33);
  // Gamma^0 components (symmetric), X = g^00, Y = g^01
  const double X = -opz, Y = z / r;
  // Gamma^0_{mu nu} = X/2 (d_mu g_0nu + d_nu g_0mu) + Y/2 (d_mu g_1nu + d_nu g_1mu - d_1 g_mu nu)
  const double G00 = 0.5 * Y * (-a00);
  const double G01 = 0.5 * X * (a00) + 0.5 * Y * (a01 - a01);
  const double G02 = 0.5 * X * (c00) + 0.5 * Y * (c01);
  const double G03 = 0.5 * Y * (-a03);
  const double G11 = 0.5 * X * (2.0 * a01) + 0.5 * Y * (2.0 * a11 - a11);
  const double G12 = 0.5 * X * (c01) + 0.5 * Y * (c11);
  const double G13 = 0.5 * X * (a03) + 0.5 * Y * (a13 - a13);
  const double G22 = 0.5 * Y * (-a22);
  const double G23 = 0.5 * X * (c03) + 0.5 * Y * (c13);
  const double G33 = 0.5 * Y * (-a33);
  const double TG = T.t00 * G00 + 2.0 * (T.t01 * G01 + T.t02 * G02 + T.t03 * G03 +
                                         T.t12 * G12 + T.t13 * G13 + T.t23 * G23) +
                    T.t11 * G11 + T.t22 * G22 + T.t33 * G33;
  const double dla1 = -0.5 * dz1 / opz, dla2 = -0.5 * dz2 / opz;
  St = G.alpha * (T.t01 * dla1 + T.t02 * dla2 - TG);
  const double smg = G.alpha * G.sqrtg;
  S1 *= smg; S2 *= smg; St *= smg;
}

__device__ __forceinline__ Sym4 tmunu(const Geo &G, const Aux &A)
{
  const double wt = A.w + A.b2, pt = A.p + 0.5 * A.b2;
  const double ia2 = G.ialpha * G.ialpha;
  const double u0 = A.W * G.ialpha;
  const double gi00 = -ia2, gi01 = G.beta1 * ia2, gi11 = G.gi11 - G.beta1 * G.beta1 * ia2;
  Sym4 T;
  T.t00 = wt * u0 * u0 + pt * gi00 - A.b0 * A.b0;
  T.t01 = wt * u0 * A.uc1 + pt * gi01 - A.b0 * A.bc1;
  T.t02 = wt * u0 * A.uc2 - A.b0 * A.bc2;
  T.t03 = wt * u0 * A.uc3 - A.b0 * A.bc3;
  T.t11 = wt * A.uc1 * A.uc1 + pt * gi11 - A.bc1 * A.bc1;
  T.t12 = wt * A.uc1 * A.uc2 - A.bc1 * A.bc2;
  T.t13 = wt * A.uc1 * A.uc3 + pt * G.gi13 - A.bc1 * A.bc3;
  T.t22 = wt * A.uc2 * A.uc2 + pt * G.gi22 - A.bc2 * A.bc2;
  T.t23 = wt * A.uc2 * A.uc3 - A.bc2 * A.bc3;
  T.t33 = wt * A.uc3 * A.uc3 + pt * G.gi33 - A.bc3 * A.bc3;
  return T;
}

// ---------------------------------------------------------------- inversion

struct C2P { double q, r2, b2, rb, gam, v2max; };

// Master function f(mu) = mu - 1/(h/W + mu rbar^2) and its derivative.
__device__ __forceinline__ double master(const C2P &m, double mu, double &df)
{
  const double x = inv(1.0 + mu * m.b2);
  const double dx = -m.b2 * x * x;
  const double rb2 = m.rb * m.rb;
  const double rbar2 = m.r2 * x * x + mu * x * (1.0 + x) * rb2;
  const double drbar2 = 2.0 * m.r2 * x * dx + rb2 * (x * (1.0 + x) + mu * (1.0 + 2.0 * x) * dx);
  const double K = m.b2 * m.r2 - rb2;
  const double qbar = m.q - 0.5 * m.b2 - 0.5 * mu * mu * x * x * K;
  const double dqbar = -K * (mu * x * x + mu * mu * x * dx);
  double v2 = mu * mu * rbar2, dv2 = 2.0 * mu * rbar2 + mu * mu * drbar2;
  if (v2 > m.v2max) { v2 = m.v2max; dv2 = 0.0; }
  const double iW = sqrt(1.0 - v2);
  const double W = inv(iW);
  const double dW = 0.5 * W * W * W * dv2;
  double eps = W * (qbar - mu * rbar2) + v2 * W * W * inv(1.0 + W);
  double deps = dW * (1.0 + qbar - mu * rbar2) + W * (dqbar - rbar2 - mu * drbar2);
  if (eps < 0.0) { eps = 0.0; deps = 0.0; }
  const double hh = 1.0 + m.gam * eps, dh = m.gam * deps;
  const double nu = hh * iW, dnu = dh * iW - hh * dW * iW * iW;
  const double den = nu + mu * rbar2;
  const double iden = inv(den);
  df = 1.0 + (dnu + rbar2 + mu * drbar2) * iden * iden;
  return mu - iden;
}

__device__ __forceinline__ double master_f(const C2P &m, double mu)
{
  double d;
  return master(m, mu, d);
}

// General-EOS master function (the inversion of Kastaun, Kalinani & Ciolfi
// 2021 that Sec. 3.1 uses) over the table: rho = D/W and eps clamped into
// the table, a = p / (rho (1 + eps)),
//   nu = max((1 + a)(1 + eps)/W, (1 + a)(1 + qbar - mu rbar^2)),
//   f(mu) = mu - 1/(nu + mu rbar^2),
// with df/dmu from the derivatives of the trilinear interpolant.
struct C2PT { double q, r2, b2, rb, v2max, D, ye; };

__device__ __forceinline__ double master_tab(const C2PT &m, const EosTab &t, double mu,
                                             double &df)
{
  const double x = inv(1.0 + mu * m.b2);
  const double dx = -m.b2 * x * x;
  const double rb2 = m.rb * m.rb;
  const double rbar2 = m.r2 * x * x + mu * x * (1.0 + x) * rb2;
  const double drbar2 = 2.0 * m.r2 * x * dx + rb2 * (x * (1.0 + x) + mu * (1.0 + 2.0 * x) * dx);
  const double K = m.b2 * m.r2 - rb2;
  const double qbar = m.q - 0.5 * m.b2 - 0.5 * mu * mu * x * x * K;
  const double dqbar = -K * (mu * x * x + mu * mu * x * dx);
  double v2 = mu * mu * rbar2, dv2 = 2.0 * mu * rbar2 + mu * mu * drbar2;
  if (v2 > m.v2max) { v2 = m.v2max; dv2 = 0.0; }
  const double iW = sqrt(1.0 - v2);
  const double W = inv(iW);
  const double dW = 0.5 * W * W * W * dv2;
  double rho = m.D * iW, drho = -rho * iW * dW;
  if (rho < t.rho_min) { rho = t.rho_min; drho = 0.0; }
  if (rho > t.rho_max) { rho = t.rho_max; drho = 0.0; }
  const double s = 1.0 + qbar - mu * rbar2, ds = dqbar - rbar2 - mu * drbar2;
  // eps = W (qbar - mu rbar^2) + v^2 W^2/(1 + W) (= W s - 1, without its cancellation)
  double eps = W * (qbar - mu * rbar2) + v2 * W * W * inv(1.0 + W), deps = dW * s + W * ds;
  if (eps < t.eps_min) { eps = t.eps_min; deps = 0.0; }
  if (eps > t.eps_max) { eps = t.eps_max; deps = 0.0; }
  const double irho = inv(rho), iope = inv(1.0 + eps);
  const TabV v = tab_eval<true>(t, log(rho), log(eps), m.ye);
  const double p = exp(v.L);
  const double dp = p * (v.Lx * drho * irho + v.Ly * deps * inv(eps));
  const double a = p * irho * iope;
  const double da = (dp - p * (drho * irho + deps * iope)) * irho * iope;
  const double nuA = (1.0 + a) * (1.0 + eps) * iW;
  const double nuB = (1.0 + a) * s;
  double nu, dnu;
  if (nuA > nuB) {
    nu = nuA;
    dnu = (da * (1.0 + eps) + (1.0 + a) * deps) * iW - nuA * dW * iW;
  } else {
    nu = nuB;
    dnu = da * s + (1.0 + a) * ds;
  }
  const double iden = inv(nu + mu * rbar2);
  df = 1.0 + (dnu + rbar2 + mu * drbar2) * iden * iden;
  return mu - iden;
}

}  // namespace grmhd
