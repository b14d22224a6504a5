// Gray M1 moments on gfx950: the closure and the implicit (backward-Euler)
// update of the collision sources of each cell (Phoebus Sec. 2.4, moments).
// Included once, by grmhd.hip (after kernels.h).
//
// Per species the Eulerian moments X = (E, F_1, F_2, F_3) of one cell solve
//   X - X* = dt S(X),  S_E = alpha^2 G^0,  S_Fi = alpha G_i,
//   G^nu = kappa_J u^nu (J_eq - J) - kappa_H H^nu,
// with the opacities and J_eq fixed.  In 3+1 form, with the fluid's W, v^i
// (v_i = gamma_ij v^j), F.v = F_i v^i, q = P^jk v_j v_k and
// p_i = gamma_ik P^kl v_l:
//   J   = W^2 (E - 2 F.v + q),
//   S_E = alpha W [kappa_J (J_eq - J) + kappa_H (J - E + F.v)],
//   S_Fi = alpha W [kappa_J v_i (J_eq - J) - kappa_H (F_i - p_i - v_i J)].
// Closure: f = |F|/E clamped to [0, 1], chi = (1 - 2f + 4f^2)/3 (maximum-
// entropy Fermi-Dirac closure at maximum packing),
//   P = (3 chi - 1)/2 E F^i F^j / F^2 + 3 (1 - chi)/2 P_thick,
// and P_thick the projection of the fluid-frame-isotropic tensor with the
// same E and F_i:
//   J_t = 3 [(2W^2 - 1) E - 2 W^2 F.v] / (2W^2 + 1),
//   W s = [E - J_t (4W^2 - 1)/3] / 2,   h_i = [F_i - (4/3) J_t W^2 v_i - W s v_i] / W,
//   P_thick^ij = (4/3) J_t W^2 v^i v^j + (J_t / 3) gamma^ij + W (h^i v^j + v^i h^j).
// The root is found by Newton's method (started from the root of the
// thick-closure problem where that is closer, steps halved while they do not
// reduce the residual); the residual and its exact Jacobian come from one
// evaluation in forward-mode dual numbers.
#pragma once
#include "dev.h"

namespace grmhd {

// value + gradient with respect to the 4 unknowns
struct D4 {
  double v, d[4];
};
__device__ __forceinline__ D4 dc(double x)
{
  D4 r;
  r.v = x;
#pragma unroll
  for (int k = 0; k < 4; ++k) r.d[k] = 0.0;
  return r;
}
__device__ __forceinline__ D4 operator+(const D4 &a, const D4 &b)
{
  D4 r; r.v = a.v + b.v;
#pragma unroll
  for (int k = 0; k < 4; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
__device__ __forceinline__ D4 operator-(const D4 &a, const D4 &b)
{
  D4 r; r.v = a.v - b.v;
#pragma unroll
  for (int k = 0; k < 4; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
__device__ __forceinline__ D4 operator*(const D4 &a, const D4 &b)
{
  D4 r; r.v = a.v * b.v;
#pragma unroll
  for (int k = 0; k < 4; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
__device__ __forceinline__ D4 operator*(double s, const D4 &a)
{
  D4 r; r.v = s * a.v;
#pragma unroll
  for (int k = 0; k < 4; ++k) r.d[k] = s * a.d[k];
  return r;
}
__device__ __forceinline__ D4 operator+(double s, const D4 &a)
{
  D4 r = a; r.v += s;
  return r;
}
__device__ __forceinline__ D4 inv(const D4 &a)
{
  const double i = inv(a.v);
  D4 r; r.v = i;
  const double m = -i * i;
#pragma unroll
  for (int k = 0; k < 4; ++k) r.d[k] = m * a.d[k];
  return r;
}
__device__ __forceinline__ D4 dsqrt(const D4 &a)
{
  const double s = sqrt(a.v);
  D4 r; r.v = s;
  const double h = 0.5 * inv(s);
#pragma unroll
  for (int k = 0; k < 4; ++k) r.d[k] = h * a.d[k];
  return r;
}

// Per-cell geometry and fluid for the solve.
struct M1Cell {
  Geo G;
  double W, vu[3], vl[3];      // Lorentz factor, v^i, v_i
  double vv;                   // v^i v_i
};

// Lower / raise a spatial vector with gamma_ij / gamma^ij (the metric family
// of dev.h: gamma_12 = gamma_23 = 0).
template <typename T>
__device__ __forceinline__ void lower(const Geo &G, const T u[3], T l[3])
{
  l[0] = G.g11 * u[0] + G.g13 * u[2];
  l[1] = G.g22 * u[1];
  l[2] = G.g13 * u[0] + G.g33 * u[2];
}
template <typename T>
__device__ __forceinline__ void raise(const Geo &G, const T l[3], T u[3])
{
  u[0] = G.gi11 * l[0] + G.gi13 * l[2];
  u[1] = G.gi22 * l[1];
  u[2] = G.gi13 * l[0] + G.gi33 * l[2];
}

// Residual R = X - Xs - dt S(X) of one species, with its Jacobian; THICK
// evaluates it with the optically thick closure alone (then R is affine in X).
template <bool THICK = false>
__device__ __forceinline__ void m1_residual(const M1Cell &c, const double X[4], const double Xs[4],
                                            double kJ, double kH, double Jeq, double dt, D4 R[4])
{
  D4 E = dc(X[0]), F[3];
  E.d[0] = 1.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    F[i] = dc(X[1 + i]);
    F[i].d[1 + i] = 1.0;
  }
  D4 Fu[3];
  {
    Fu[0] = c.G.gi11 * F[0] + c.G.gi13 * F[2];
    Fu[1] = c.G.gi22 * F[1];
    Fu[2] = c.G.gi13 * F[0] + c.G.gi33 * F[2];
  }
  const D4 F2 = Fu[0] * F[0] + Fu[1] * F[1] + Fu[2] * F[2];
  const D4 Fv = c.vu[0] * F[0] + c.vu[1] * F[1] + c.vu[2] * F[2];
  const double W = c.W, W2 = W * W;
  // flux factor and the closure weights
  D4 f = dc(0.0);
  if (!THICK && F2.v > 0.0 && E.v > 0.0) {
    f = dsqrt(F2) * inv(E);
    if (f.v > 1.0) f = dc(1.0);
  }
  const D4 chi = (1.0 / 3.0) * (1.0 + (-2.0) * f + 4.0 * (f * f));
  const D4 wa = 0.5 * (3.0 * chi + dc(-1.0));
  const D4 wb = 1.5 * (1.0 + (-1.0) * chi);
  // thick part from the lab moments
  const D4 Jt = (3.0 * inv(dc(2.0 * W2 + 1.0))) * ((2.0 * W2 - 1.0) * E + (-2.0 * W2) * Fv);
  const D4 Ws = 0.5 * (E + (-(4.0 * W2 - 1.0) / 3.0) * Jt);
  D4 hl[3], hu[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    hl[i] = (1.0 / W) * (F[i] + (-(4.0 / 3.0) * W2 * c.vl[i]) * Jt + (-c.vl[i]) * Ws);
  raise(c.G, hl, hu);
  // the two contractions of P the sources need: q = P^jk v_j v_k and
  // Pv^k = P^kl v_l (p_i = gamma_ik Pv^k)
  //   thin:  E F^k (F.v) / F^2 ,  E (F.v)^2 / F^2
  //   thick: (4/3) J_t W^2 v^k vv + (J_t/3) v^k + W (h^k vv + v^k (h.v))
  D4 thinq = dc(0.0), thinP[3] = {dc(0.0), dc(0.0), dc(0.0)};
  if (!THICK && F2.v > 0.0) {
    const D4 r = E * inv(F2) * Fv;
    thinq = r * Fv;
#pragma unroll
    for (int k = 0; k < 3; ++k) thinP[k] = r * Fu[k];
  }
  const D4 hv = c.vu[0] * hl[0] + c.vu[1] * hl[1] + c.vu[2] * hl[2];
  const D4 thkc = ((4.0 / 3.0) * W2 * c.vv + 1.0 / 3.0) * Jt + W * hv;
  D4 thkP[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) thkP[k] = c.vu[k] * thkc + (W * c.vv) * hu[k];
  const D4 thkq = c.vl[0] * thkP[0] + c.vl[1] * thkP[1] + c.vl[2] * thkP[2];
  const D4 q = wa * thinq + wb * thkq;
  D4 Pv[3], pl[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) Pv[k] = wa * thinP[k] + wb * thkP[k];
  lower(c.G, Pv, pl);
  // fluid-frame energy and the sources
  const D4 J = W2 * (E + (-2.0) * Fv + q);
  const D4 dJ = dc(Jeq) - J;
  const double aW = c.G.alpha * W;
  const D4 SE = aW * (kJ * dJ + kH * (J - E + Fv));
  R[0] = E - dc(Xs[0]) - dt * SE;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const D4 SF = aW * ((kJ * c.vl[i]) * dJ + (-kH) * (F[i] - pl[i] + (-c.vl[i]) * J));
    R[1 + i] = F[i] - dc(Xs[1 + i]) - dt * SF;
  }
}

// Solve A x = b (4x4, partial pivoting); false if singular.
__device__ __forceinline__ bool solve4(double A[4][4], double b[4], double x[4])
{
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    int p = c;
    double best = fabs(A[c][c]);
#pragma unroll
    for (int r = c + 1; r < 4; ++r)
      if (fabs(A[r][c]) > best) { best = fabs(A[r][c]); p = r; }
    if (!(best > 0.0)) return false;
    if (p != c) {
#pragma unroll
      for (int k = 0; k < 4; ++k) { const double t = A[c][k]; A[c][k] = A[p][k]; A[p][k] = t; }
      const double t = b[c]; b[c] = b[p]; b[p] = t;
    }
    const double id = 1.0 / A[c][c];
#pragma unroll
    for (int r = c + 1; r < 4; ++r) {
      const double m = A[r][c] * id;
#pragma unroll
      for (int k = c; k < 4; ++k) A[r][k] -= m * A[c][k];
      b[r] -= m * b[c];
    }
  }
#pragma unroll
  for (int c = 3; c >= 0; --c) {
    double s = b[c];
#pragma unroll
    for (int k = c + 1; k < 4; ++k) s -= A[c][k] * x[k];
    x[c] = s / A[c][c];
  }
  return true;
}

__device__ __forceinline__ double rnorm(const D4 R[4])
{
  return fabs(R[0].v) + fabs(R[1].v) + fabs(R[2].v) + fabs(R[3].v);
}

// Newton on one species; returns the iteration count (negative: not
// converged within max_it, X left at the last iterate).  Start: the better
// (smaller residual) of X* and the root of the thick-closure problem (one
// linear solve, as that residual is affine); steps are halved while they do
// not reduce the residual (at most 6 times).
__device__ __forceinline__ int m1_newton(const M1Cell &c, const double Xs[4], double kJ,
                                         double kH, double Jeq, double dt, double tol,
                                         int max_it, double X[4])
{
#pragma unroll
  for (int k = 0; k < 4; ++k) X[k] = Xs[k];
  if (kJ == 0.0 && kH == 0.0) return 0;
  const double scale0 = fabs(Xs[0]) + fabs(Xs[1]) + fabs(Xs[2]) + fabs(Xs[3]) + fabs(dt * Jeq);
  D4 R[4];
  double A[4][4], b[4], d[4];
  m1_residual(c, X, Xs, kJ, kH, Jeq, dt, R);
  {
    D4 Rt[4];
    m1_residual<true>(c, Xs, Xs, kJ, kH, Jeq, dt, Rt);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      b[r] = -Rt[r].v;
#pragma unroll
      for (int k = 0; k < 4; ++k) A[r][k] = Rt[r].d[k];
    }
    if (solve4(A, b, d)) {
      double Xt[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) Xt[k] = Xs[k] + d[k];
      D4 R2[4];
      m1_residual(c, Xt, Xs, kJ, kH, Jeq, dt, R2);
      if (Xt[0] > 0.0 && rnorm(R2) < rnorm(R)) {
#pragma unroll
        for (int k = 0; k < 4; ++k) { X[k] = Xt[k]; R[k] = R2[k]; }
      }
    }
  }
  for (int it = 1; it <= max_it; ++it) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      b[r] = -R[r].v;
#pragma unroll
      for (int k = 0; k < 4; ++k) A[r][k] = R[r].d[k];
    }
    if (!solve4(A, b, d)) return -it;
    const double r0 = rnorm(R);
    double xn0 = fabs(X[0]) + fabs(X[1]) + fabs(X[2]) + fabs(X[3]);
    double dn = fabs(d[0]) + fabs(d[1]) + fabs(d[2]) + fabs(d[3]);
    double lam = 1.0, Xn[4];
    for (int bt = 0; bt < 7; ++bt) {
#pragma unroll
      for (int k = 0; k < 4; ++k) Xn[k] = X[k] + lam * d[k];
      m1_residual(c, Xn, Xs, kJ, kH, Jeq, dt, R);
      // accept a decrease, any step already at rounding size, or the last try
      if ((Xn[0] > 0.0 && rnorm(R) < r0) || lam * dn <= 1e3 * tol * (scale0 + xn0) || bt == 6) break;
      lam *= 0.5;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) X[k] = Xn[k];
    const double xn = fabs(X[0]) + fabs(X[1]) + fabs(X[2]) + fabs(X[3]);
    if (lam * dn <= tol * (scale0 + xn)) return it;
  }
  return -max_it;
}

// One interior cell, every species: R[s][4] densitized in place; with
// couple the fluid's tau and S_i take the opposite of the exchanged energy
// and momentum.
__global__ __launch_bounds__(256) void k_m1_source(KArgs a, const int2 *__restrict__ chunks,
                                                   int nsp, double *__restrict__ R,
                                                   const double *__restrict__ kap, double dt,
                                                   double tol, int max_it, int couple,
                                                   uint8_t *__restrict__ iters, int mk)
{
  const int2 ch = chunks[blockIdx.x];
  const BlockInfo b = a.blocks[ch.x];
  const int e = ch.y + threadIdx.x;
  if (e >= b.n[0] * b.n[1] * b.n[2]) return;
  const int ng = a.ng;
  const int i = ng + e % b.n[0], j = ng + (e / b.n[0]) % b.n[1], k = ng + e / (b.n[0] * b.n[1]);
  const long long c = b.off + i + (long long)b.s[0] * (j + (long long)b.s[1] * k);
  const long long n = a.nct;
  M1Cell m;
  m.G = mk == MK_KS ? geo_at<MK_KS>(a.tab, a.met, b.tab1 + i, false, b.tab2 + j, false)
                    : geo_mink<double>();
  const double ut[3] = {a.P[n + c], a.P[2 * n + c], a.P[3 * n + c]};
  double utl[3];
  lower(m.G, ut, utl);
  m.W = sqrt(1.0 + ut[0] * utl[0] + ut[1] * utl[1] + ut[2] * utl[2]);
  const double iW = 1.0 / m.W;
#pragma unroll
  for (int q = 0; q < 3; ++q) { m.vu[q] = ut[q] * iW; m.vl[q] = utl[q] * iW; }
  m.vv = m.vu[0] * m.vl[0] + m.vu[1] * m.vl[1] + m.vu[2] * m.vl[2];
  const double sg = m.G.sqrtg, isg = 1.0 / sg;
  double dE = 0.0, dF[3] = {0.0, 0.0, 0.0};
  int worst = 0;
  bool fail = false;
  for (int s = 0; s < nsp; ++s) {
    double Xs[4], X[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) Xs[v] = R[(s * 4 + v) * n + c] * isg;
    const double kJ = kap[(s * 3) * n + c], kH = kap[(s * 3 + 1) * n + c];
    const double Jeq = kap[(s * 3 + 2) * n + c];
    const int it = m1_newton(m, Xs, kJ, kH, Jeq, dt, tol, max_it, X);
    if (it == 0) continue;                 // no coupling: the moments stay as they are
    fail |= it < 0;
    worst = max(worst, it < 0 ? -it : it);
#pragma unroll
    for (int v = 0; v < 4; ++v) R[(s * 4 + v) * n + c] = sg * X[v];
    dE += X[0] - Xs[0];
#pragma unroll
    for (int q = 0; q < 3; ++q) dF[q] += X[1 + q] - Xs[1 + q];
  }
  if (couple) {
    a.U[4 * n + c] -= sg * dE;
#pragma unroll
    for (int q = 0; q < 3; ++q) a.U[(1 + q) * n + c] -= sg * dF[q];
  }
  if (iters) iters[c] = (uint8_t)(fail ? 255 : min(worst, 254));
}

}  // namespace grmhd
