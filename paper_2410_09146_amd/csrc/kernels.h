// gfx950 kernels of the GRMHD stage.  Included once, by grmhd.hip.
//
//   k_ghost_P / k_ghost_B   gather ghost zones through precomputed maps
//   k_bcc                   cell-centred B from the face field
//   k_flux<D>               LDS-staged 16x16 face tiles: reconstruct -> Riemann
//   k_flux_planes           the last face plane of every direction (one thread per face)
//   k_update                flux divergence + sources + CT (edge-averaged EMF)
//                           + Runge-Kutta combination, one thread per cell
//   k_c2p                   safeguarded Newton inversion + floors
//   k_p2c                   U from P (initialisation)
//   k_reduce / k_reduce_fin CFL dt, div B, conserved totals, inversion stats
#pragma once
#include "dev.h"
#include "mlp.h"

namespace grmhd {

struct KArgs {
  double *P, *Bf, *U, *U0, *Bf0;
  double *F;            // [3][8][nct] densitized face fluxes
  double *Bcc;          // [3][nct] cell-centred undensitized B
  int8_t *flags;
  uint8_t *iters;
  const BlockInfo *blocks;
  Tables tab;
  MetricP met;
  EosP eos;
  long long nct;
  int ng;
  int active[3];        // directions with more than one cell (CFL sum)
  double *SP, *SB;      // staged coarse-view rows of P [5][nsp] and face B [nsb]
  long long nsp;
  double *E;            // two-level meshes: edge EMFs [3][nct] (corrected at level boundaries)
  EosTab et;            // tabulated EOS (et.d == nullptr: ideal gas)
  int npv;              // primitive planes: 5, or 6 with the Y_e scalar in P[5]
  unsigned long long *nfail;  // failed inversions since the pack was created
  // Kerr-Schild: the density and energy floors of every radial table entry
  // (rho_flr0 r^-rho_flr_pow, u_flr0 r^-u_flr_pow), written by k_floor_tab
  // whenever an inversion asks for other floors than the table holds
  double *flr_rho, *flr_u;
};

// Runge-Kutta coefficients of a stage (U = c0 U0 + c1 U + cdt dt L); dt <= 0:
// the device-resident dt at dtd.  save: U0 <- U first (the stage's base).
struct RkArgs {
  double dt;
  const double *dtd;
  double c0, c1, cdt;
  int save;
};

// p and Gamma_1 p of a cell or face state: the table when one is bound (only
// packs with the scalar, NSC = 1, can bind one), else the ideal gas.
template <int NSC>
__device__ __forceinline__ void thermo_of(const KArgs &a, double rho, double u, double ye,
                                          double &p, double &gp)
{
  if constexpr (NSC != 0) {
    if (a.et.d) { tab_thermo(a.et, rho, u, ye, p, gp); return; }
  }
  p = (a.eos.gam - 1.0) * u;
  gp = a.eos.gam * p;
}

template <int NSC>
__device__ __forceinline__ Aux aux_cell(const KArgs &a, const Geo &G, const Prim &q)
{
  double p, gp;
  thermo_of<NSC>(a, q.rho, q.ie, q.ye, p, gp);
  return aux_th(G, q, p, gp);
}

struct GhostP { long long dst, src; int flags, pad; };
struct GhostB { long long dst, src; int comp, flip; };
// Two-level meshes.  A coarse-view value is the mean of n = 1 cell or of the
// n = 8 children src + {0,1} + {0,sj} + {0,sk} of a coarse cell; tgt = 0
// writes a ghost cell of P (restriction), tgt = 1 a row of the staging
// buffer that the prolongation reads.
struct GhostR { long long dst, src, sk; int flags, n, sj, tgt; };
// Fine ghost cell from staged coarse values: s = parent, parent -/+ x1,
// -/+ x2, -/+ x3; oct bit d set = the child lies on the upper side along d.
struct GhostPro { long long dst; int s[7]; int flags, oct, pad; };
// Face field: mean of n = 1 face or of the 4 child faces src + {0,st1} +
// {0,st2} (tgt as above), and fine ghost faces from one staged coarse face
// (sb < 0) or the mean of two.
struct GhostBR { long long dst, src, st1, st2; int comp, flip, n, tgt; };
struct GhostBPro { long long dst; int sa, sb, comp, flip; };
// Level-boundary corrections of a coarse block: a face along D takes the
// mean of the 4 fine faces src + {0, st1} + {0, st2} (hydro fluxes); an edge
// along e the mean of the fine edges src and src + st (EMFs).
struct FixF { long long dst, src, st1, st2; int D, pad; };
struct FixE { long long dst, src, st; int e, pad; };

// ------------------------------------------------------------------ ghosts

__device__ __forceinline__ void bc_flags(int flags, double *v);

// flags: bit d = polar mirror along d (velocity d flips); 8 << 2d / 16 << 2d
// = low / high outflow along d (inflow velocity zeroed); the scalar plane
// (npv = 6) is copied as it is
__global__ __launch_bounds__(256) void k_ghost_P(KArgs a, const GhostP *__restrict__ map, int n)
{
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const GhostP g = map[e];
  double v[6];
#pragma unroll
  for (int q = 0; q < 6; ++q)
    if (q < a.npv) v[q] = a.P[q * a.nct + g.src];
  bc_flags(g.flags, v);
#pragma unroll
  for (int q = 0; q < 6; ++q)
    if (q < a.npv) a.P[q * a.nct + g.dst] = v[q];
}

__global__ __launch_bounds__(256) void k_ghost_B(KArgs a, const GhostB *__restrict__ map, int n)
{
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const GhostB g = map[e];
  const double v = a.Bf[g.comp * a.nct + g.src];
  a.Bf[g.comp * a.nct + g.dst] = g.flip ? -v : v;
}

__device__ __forceinline__ void bc_flags(int flags, double *v)
{
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (flags & (8 << (2 * d))) v[1 + d] = v[1 + d] > 0.0 ? 0.0 : v[1 + d];
    if (flags & (16 << (2 * d))) v[1 + d] = v[1 + d] < 0.0 ? 0.0 : v[1 + d];
    if (flags & (1 << d)) v[1 + d] = -v[1 + d];
  }
}

// restriction into coarse ghosts and coarse-view staging rows
__global__ __launch_bounds__(256) void k_ghost_avg(KArgs a, const GhostR *__restrict__ map, int n)
{
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const GhostR g = map[e];
  double v[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const double *p = a.P + q * a.nct + g.src;
    if (g.n == 1) {
      v[q] = p[0];
    } else {
      double acc = 0.0;
      for (int z = 0; z < 2; ++z)
        for (int y = 0; y < 2; ++y)
          for (int x = 0; x < 2; ++x) acc += p[x + y * (long long)g.sj + z * g.sk];
      v[q] = 0.125 * acc;
    }
  }
  bc_flags(g.flags, v);
  if (g.tgt) {
#pragma unroll
    for (int q = 0; q < 5; ++q) a.SP[q * a.nsp + g.dst] = v[q];
  } else {
#pragma unroll
    for (int q = 0; q < 5; ++q) a.P[q * a.nct + g.dst] = v[q];
  }
}

__device__ __forceinline__ double mc_lim(double dm, double dp)
{
  if (dm * dp <= 0.0) return 0.0;
  const double s = fmin(fmin(2.0 * fabs(dm), 2.0 * fabs(dp)), 0.5 * fabs(dm + dp));
  return dm > 0.0 ? s : -s;
}

// fine ghost cells: parent + MC-limited slopes toward the child's octant;
// a non-positive density or internal energy keeps the parent value
__global__ __launch_bounds__(256) void k_prolong_P(KArgs a, const GhostPro *__restrict__ map, int n)
{
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const GhostPro g = map[e];
  double v[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const double *S = a.SP + q * a.nsp;
    const double c0 = S[g.s[0]];
    double sum = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double sl = mc_lim(c0 - S[g.s[1 + 2 * d]], S[g.s[2 + 2 * d]] - c0);
      sum += ((g.oct >> d) & 1) ? sl : -sl;
    }
    v[q] = c0 + 0.25 * sum;
    if ((q == 0 || q == 4) && (!(v[q] > 0.0) || !isfinite(v[q]))) v[q] = c0;
  }
  bc_flags(g.flags, v);
#pragma unroll
  for (int q = 0; q < 5; ++q) a.P[q * a.nct + g.dst] = v[q];
}

__global__ __launch_bounds__(256) void k_ghost_bavg(KArgs a, const GhostBR *__restrict__ map, int n)
{
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const GhostBR g = map[e];
  const double *p = a.Bf + g.comp * a.nct + g.src;
  double v;
  if (g.n == 1) {
    v = p[0];
  } else {
    double acc = 0.0;
    for (int t2 = 0; t2 < 2; ++t2)
      for (int t1 = 0; t1 < 2; ++t1) acc += p[t1 * g.st1 + t2 * g.st2];
    v = 0.25 * acc;
  }
  if (g.flip) v = -v;
  if (g.tgt) a.SB[g.dst] = v;
  else a.Bf[g.comp * a.nct + g.dst] = v;
}

__global__ __launch_bounds__(256) void k_prolong_B(KArgs a, const GhostBPro *__restrict__ map, int n)
{
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const GhostBPro g = map[e];
  double v = g.sb < 0 ? a.SB[g.sa] : 0.5 * (a.SB[g.sa] + a.SB[g.sb]);
  if (g.flip) v = -v;
  a.Bf[g.comp * a.nct + g.dst] = v;
}

// ------------------------------------------------------------ cell-centred B

template <int MK>
__device__ __forceinline__ Geo geo_center(const KArgs &a, const BlockInfo &b, int i, int j)
{
  return geo_at<MK>(a.tab, a.met, b.tab1 + i, false, b.tab2 + j, false);
}

template <int MK>
__global__ __launch_bounds__(256) void k_bcc(KArgs a, const int2 *__restrict__ chunks)
{
  const int2 ch = chunks[blockIdx.x];
  const BlockInfo b = a.blocks[ch.x];
  const int e = ch.y + threadIdx.x;
  const int m1 = b.s[0] - 1, m2 = b.s[1] - 1;
  if (e >= m1 * m2 * (b.s[2] - 1)) return;
  const int i = e % m1, j = (e / m1) % m2, k = e / (m1 * m2);
  const long long c = b.off + i + (long long)b.s[0] * (j + (long long)b.s[1] * k);
  const long long sj = b.s[0], sk = (long long)b.s[0] * b.s[1];
  const Geo G = geo_center<MK>(a, b, i, j);
  const double h = 0.5 / G.sqrtg;
  a.Bcc[c] = h * (a.Bf[c] + a.Bf[c + 1]);
  a.Bcc[a.nct + c] = h * (a.Bf[a.nct + c] + a.Bf[a.nct + c + sj]);
  a.Bcc[2 * a.nct + c] = h * (a.Bf[2 * a.nct + c] + a.Bf[2 * a.nct + c + sk]);
}

// ------------------------------------------------------------------- fluxes

// Face-tile shapes: TD faces along the flux direction x TA columns (256 faces);
// the columns run along x1 when the direction is x2 or x3.
template <int SH> struct Shape;
template <> struct Shape<0> { static constexpr int TD = 16, TA = 16; };
template <> struct Shape<1> { static constexpr int TD = 32, TA = 8; };
template <> struct Shape<2> { static constexpr int TD = 8, TA = 32; };
template <> struct Shape<3> { static constexpr int TD = 64, TA = 4; };
template <> struct Shape<4> { static constexpr int TD = 4, TA = 64; };
constexpr int NSHAPE = 5;
__host__ __device__ constexpr int shape_td(int sh) { return sh == 0 ? 16 : sh == 1 ? 32 : sh == 2 ? 8 : sh == 3 ? 64 : 4; }
__host__ __device__ constexpr int shape_ta(int sh) { return 256 / shape_td(sh); }

// transverse field components reconstructed along D
template <int D> __device__ constexpr int tcomp(int w) { return D == 0 ? 1 + w : (D == 1 ? 2 * w : w); }

template <int MK, int D>
__device__ __forceinline__ Geo geo_face(const KArgs &a, const BlockInfo &b, int i, int j)
{
  return geo_at<MK>(a.tab, a.met, b.tab1 + i, D == 0, b.tab2 + j, D == 1);
}

// Reconstructed variables along D: rho, u-tilde^1..3, u, the two transverse
// cell-centred B, and (NSC) Y_e.
template <int D, int NSC, typename T>
__device__ __forceinline__ PrimT<T> make_prim(const T q[7 + NSC], T bn)
{
  PrimT<T> p;
  p.rho = q[0]; p.u1 = q[1]; p.u2 = q[2]; p.u3 = q[3]; p.ie = q[4];
  if constexpr (D == 0) { p.B1 = bn; p.B2 = q[5]; p.B3 = q[6]; }
  if constexpr (D == 1) { p.B1 = q[5]; p.B2 = bn; p.B3 = q[6]; }
  if constexpr (D == 2) { p.B1 = q[5]; p.B2 = q[6]; p.B3 = bn; }
  if constexpr (NSC != 0) p.ye = q[7];
  else p.ye = T(0);
  return p;
}

template <typename T>
__device__ __forceinline__ GeoT<T> geo_cast(const Geo &G)
{
  GeoT<T> g;
  g.alpha = T(G.alpha); g.ialpha = T(G.ialpha); g.beta1 = T(G.beta1);
  g.g11 = T(G.g11); g.g13 = T(G.g13); g.g22 = T(G.g22); g.g33 = T(G.g33);
  g.gi11 = T(G.gi11); g.gi13 = T(G.gi13); g.gi22 = T(G.gi22); g.gi33 = T(G.gi33);
  g.sqrtg = T(G.sqrtg);
  return g;
}

// Riemann solve at one face in arithmetic T; densitization in FP64.  The
// flux of the normal field component vanishes identically, so its slot
// 5 + D carries the passive-scalar flux when NSC = 1 (and is not written
// otherwise).
template <int MK, int D, int RS, typename T, int NSC>
__device__ __forceinline__ void face_flux_geo(const KArgs &a, const Geo &G, double bface,
                                              const T qL[7 + NSC], const T qR[7 + NSC],
                                              double Fo[8]);

template <int MK, int D, int RS, typename T, int NSC>
__device__ __forceinline__ void face_flux(const KArgs &a, const BlockInfo &b, int i, int j,
                                          long long c, const T qL[7 + NSC], const T qR[7 + NSC],
                                          double Fo[8])
{
  if (D == 1 && (j == b.pole_lo || j == b.pole_hi)) {   // sqrt(-g) = 0 on the axis
#pragma unroll
    for (int v = 0; v < 8; ++v) Fo[v] = 0.0;
    return;
  }
  face_flux_geo<MK, D, RS, T, NSC>(a, geo_face<MK, D>(a, b, i, j), a.Bf[D * a.nct + c], qL, qR,
                                   Fo);
}

// The Riemann solve of a face given its metric and the face field
// sqrt(gamma) B^D (bface).
template <int MK, int D, int RS, typename T, int NSC>
__device__ __forceinline__ void face_flux_geo(const KArgs &a, const Geo &G, double bface,
                                              const T qL[7 + NSC], const T qR[7 + NSC],
                                              double Fo[8])
{
  const double bn = bface / G.sqrtg;
  const PrimT<T> L = make_prim<D, NSC>(qL, T(bn)), R = make_prim<D, NSC>(qR, T(bn));
  T A[8 + NSC], B[8 + NSC];
  if constexpr (sizeof(T) == sizeof(double)) {
    double pL, gpL, pR, gpR;
    thermo_of<NSC>(a, L.rho, L.ie, L.ye, pL, gpL);
    thermo_of<NSC>(a, R.rho, R.ie, R.ye, pR, gpR);
    riemann_parts<D, RS, T, NSC>(G, L, R, pL, gpL, pR, gpR, A, B);
  } else {
    static_assert(NSC == 0, "the mixed-precision flux path has no scalar");
    const T gam = T(a.eos.gam);
    const T pL = (gam - T(1)) * L.ie, pR = (gam - T(1)) * R.ie;
    riemann_parts<D, RS, T>(geo_cast<T>(G), L, R, pL, gam * pL, pR, gam * pR, A, B);
  }
  const double smg = G.alpha * G.sqrtg, sg = G.sqrtg;
#pragma unroll
  for (int v = 0; v < 8; ++v)
    Fo[v] = (v != 5 + D) ? smg * (double)A[v] + sg * (double)B[v] : 0.0;
  if constexpr (NSC != 0) Fo[5 + D] = smg * (double)A[8] + sg * (double)B[8];
}

template <int MK, int D, int RS, typename T, int NSC>
__device__ __forceinline__ void face_flux_store(const KArgs &a, const BlockInfo &b, int i, int j,
                                                long long c, const T qL[7 + NSC],
                                                const T qR[7 + NSC])
{
  double Fo[8];
  face_flux<MK, D, RS, T, NSC>(a, b, i, j, c, qL, qR, Fo);
#pragma unroll
  for (int v = 0; v < 8; ++v)
    if (v != 5 + D || NSC) a.F[(D * 8 + v) * a.nct + c] = Fo[v];
}

template <typename T>
__device__ __forceinline__ void positivity(int v, T f2, T &l, T &r)
{
  if (v == 0 || v == 4) {
    if (!(l > T(0)) || !isfinite(l)) l = f2;
    if (!(r > T(0)) || !isfinite(r)) r = f2;
  }
}

// Kerr-Schild geometric source terms of one cell (sqrt(-g) S, Sec. 2.1) added
// to the momentum and energy parts of rhs.
template <int MK, int NSC>
__device__ __forceinline__ void add_sources(const KArgs &a, const BlockInfo &b, int i, int j,
                                            const Prim &q, double *rhs)
{
  if constexpr (MK == MK_KS) {
    const double r = a.tab.rc[b.tab1 + i], s = a.tab.sc[b.tab2 + j], ct = a.tab.cc[b.tab2 + j];
    const Geo G = geo_ks(r, s, ct, a.met);
    const Aux A = aux_cell<NSC>(a, G, q);
    const Sym4 T = tmunu(G, A);
    double S1, S2, St;
    ks_sources(r, s, ct, a.met, G, T, S1, S2, St);
    rhs[1] += S1;
    rhs[2] += S2;
    rhs[4] += St;
  }
}

// The Runge-Kutta combination of one value, by mode:
//   0: cur <- c0 base + c1 cur + h r          1: base <- cur, cur <- c0 cur + h r
//   2: base <- c0 cur + h r (cur kept)        3: base <- c0 base + c1 cur + h r
// Modes 0/1 are a stage that leaves its result in the current array; 2/3 the
// same two stages with the result written over the base array instead, so a
// two-stage step needs no copy of its base (the arithmetic is the same).
__device__ __forceinline__ void rk_value(double *cur, double *base, long long i, double c0,
                                         double c1, double h, int mode, double r)
{
  const double u = cur[i];
  if (mode == 1) {
    base[i] = u;
    cur[i] = c0 * u + h * r;
  } else if (mode == 0) {
    cur[i] = c0 * base[i] + c1 * u + h * r;
  } else if (mode == 2) {
    base[i] = c0 * u + h * r;
  } else {
    base[i] = c0 * base[i] + c1 * u + h * r;
  }
}

// U (and base U0) of one cell by rk_value's mode
template <int NV>
__device__ __forceinline__ void rk_cell(const KArgs &a, long long c, double c0, double c1,
                                        double h, int mode, const double *rhs)
{
  const long long n = a.nct;
#pragma unroll
  for (int v = 0; v < NV; ++v) rk_value(a.U, a.U0, v * n + c, c0, c1, h, mode, rhs[v]);
}

// Main face tiles: TD faces along D x TA columns along A (x2 for D = x1,
// else x1), one row along the third axis.  Tile origin = lower face of the
// tile in block-local (i, j, k).
// Occupancy target: 4 waves per SIMD (128 VGPRs) for the hydro variables;
// with the scalar and the table lookups 3 (up to 168 VGPRs, no spills).
template <int MK, int D, int RECON, int FV, int RS, typename T, int SH, int NSC = 0, int FUSE = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4 - NSC)))
void k_flux(KArgs a, const int4 *__restrict__ tiles, int ntiles, RkArgs rk)
{
  static_assert(FUSE == 0 || NSC == 0, "the fused stage has no scalar");
  constexpr int TD = Shape<SH>::TD, TA = Shape<SH>::TA, NS = TD + 5, NR = TD + 1;
  constexpr int NV = 7 + NSC;
  constexpr int NSTG = NV * TA * NS, NSFR = NV * TA * NR;
  // fused: the hydro face fluxes of the tile (FP64) take the staged window's
  // place once it has been read; FP32 windows are too small, so they get
  // space of their own
  constexpr int NFLX = (FUSE && sizeof(T) != sizeof(double)) ? 10 * TA * TD : 0;
  static_assert(!FUSE || sizeof(T) != sizeof(double) || NSTG >= 5 * TA * TD,
                "the fused hydro fluxes reuse the staging space");
  // staged stencil window, then the right-face states of cells org[D]-1 ..
  // org[D]+TD-1
  __shared__ __align__(16) T lds[NSTG + NSFR + NFLX];
  T *const stg = lds;
  T *const sfr = lds + NSTG;
  double *const flx = (double *)(NFLX ? lds + NSTG + NSFR : lds);
  constexpr int AX = (D == 0) ? 1 : 0;
  constexpr int BX = 3 - D - AX;
  const int tid = threadIdx.x;
  // this thread's face (and cell) within the tile
  int fd, aa;
  if constexpr (D == 0) { fd = tid % TD; aa = tid / TD; }
  else                  { aa = tid % TA; fd = tid / TA; }

  // persistent: the grid strides over the tile work-list (every thread of a
  // workgroup runs the same number of iterations, so the barriers match)
  for (int ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
    const int4 t = tiles[ti];
    const BlockInfo b = a.blocks[t.x];
    const int org[3] = {t.y, t.z, t.w};
    const long long str[3] = {1, b.s[0], (long long)b.s[0] * b.s[1]};

    // stage P and the transverse cell-centred field of cells org[D]-3 ..
    // org[D]+TD+1: one (column, cell) position per thread and pass, all seven
    // variables from one address computation
    for (int p = tid; p < TA * NS; p += 256) {
      int s, pa;
      if constexpr (D == 0) { s = p % NS; pa = p / NS; }
      else                  { pa = p % TA; s = p / TA; }
      int idx[3] = {org[0], org[1], org[2]};
      idx[D] = min(max(org[D] - 3 + s, 0), b.s[D] - 1);
      idx[AX] = min(org[AX] + pa, b.s[AX] - 1);
      const long long c = b.off + idx[0] * str[0] + idx[1] * str[1] + idx[2] * str[2];
      T *dst = &stg[pa * NS + s];
#pragma unroll
      for (int v = 0; v < 5; ++v) dst[v * TA * NS] = T(a.P[v * a.nct + c]);
      dst[5 * TA * NS] = T(a.Bcc[tcomp<D>(0) * a.nct + c]);
      dst[6 * TA * NS] = T(a.Bcc[tcomp<D>(1) * a.nct + c]);
      if constexpr (NSC != 0) dst[7 * TA * NS] = T(a.P[5 * a.nct + c]);
    }
    __syncthreads();

    // reconstruct: each thread its own cell org[D]+fd (all NV variables),
    // keeping the left-face state for its face and publishing the right-face
    // state; the cells org[D]-1 of the TA columns come after (right face only)
    T qR[NV];
    bool redo = false;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T *f = &stg[(v * TA + aa) * NS + fd + 1];
      T l, r;
      redo |= !recon5_fast<RECON, FV, T>(f[0], f[1], f[2], f[3], f[4], l, r);
      positivity(v, f[2], l, r);
      sfr[(v * TA + aa) * NR + fd + 1] = r;
      qR[v] = l;
    }
    if (redo) {           // rare: a WENO pair that could not be normalised
#pragma unroll 1
      for (int v = 0; v < NV; ++v) {
        const T *f = &stg[(v * TA + aa) * NS + fd + 1];
        T l, r;
        recon5<RECON, FV, T>(f[0], f[1], f[2], f[3], f[4], l, r);
        positivity(v, f[2], l, r);
        sfr[(v * TA + aa) * NR + fd + 1] = r;
#pragma unroll
        for (int w = 0; w < NV; ++w)
          if (w == v) qR[w] = l;
      }
    }
    for (int it = tid; it < NV * TA; it += 256) {
      const int v = it / TA, ca = it % TA;
      const T *f = &stg[(v * TA + ca) * NS];
      T l, r;
      // fused: the same reconstruction as the tile's own cells, so that a
      // face shared by two tiles gets the same flux in both
      if (!FUSE || !recon5_fast<RECON, FV, T>(f[0], f[1], f[2], f[3], f[4], l, r))
        recon5<RECON, FV, T>(f[0], f[1], f[2], f[3], f[4], l, r);
      positivity(v, f[2], l, r);
      sfr[(v * TA + ca) * NR] = r;
    }
    __syncthreads();

    int idx[3] = {org[0], org[1], org[2]};
    idx[D] = org[D] + fd;
    idx[AX] = org[AX] + aa;
    const int ng = a.ng;
    const bool tr = idx[AX] <= ng + b.n[AX] && idx[AX] < b.s[AX];
    const long long c = b.off + idx[0] * str[0] + idx[1] * str[1] + idx[2] * str[2];
    if constexpr (!FUSE) {
      // every flux of the faces org[D] .. org[D]+TD-1 to HBM
      if (tr && idx[D] < ng + b.n[D]) {
        T qL[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) qL[v] = sfr[(v * TA + aa) * NR + fd];   // cell idx[D]-1
        face_flux_store<MK, D, RS, T, NSC>(a, b, idx[0], idx[1], c, qL, qR);
      }
    } else {
      // Fused: the tiles overlap by one face (stride TD - 1), so the faces
      // org[D] .. org[D]+TD-1, up to the block's upper face, give the flux
      // difference of the cells org[D] .. org[D]+TD-2 within the tile.  Only
      // the induction fluxes (for the edge EMFs) go to HBM; the hydro flux
      // divergence accumulates in the cell's dU (F[0][0..4]): x1 writes it,
      // x2 adds to it, and x3 adds its own, the sources and does the
      // Runge-Kutta combination, so no hydro flux is stored.
      const bool live = tr && idx[D] <= ng + b.n[D];
      const bool cell = live && fd < TD - 1 && idx[D] < ng + b.n[D] && idx[AX] >= ng &&
                        idx[AX] < ng + b.n[AX] && idx[BX] >= ng && idx[BX] < ng + b.n[BX];
      if (live) {
        T qL[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) qL[v] = sfr[(v * TA + aa) * NR + fd];
        double Fo[8];
        face_flux<MK, D, RS, T, NSC>(a, b, idx[0], idx[1], c, qL, qR, Fo);
        // Each face is stored by one tile; the other tile that computes it
        // (the shared face) writes into the unused normal-field slot.  A
        // select rather than a branch: a conditional store here costs the
        // Riemann solve its registers.
        const bool own = fd > 0 || org[D] == ng;
#pragma unroll
        for (int v = 5; v < 8; ++v)
          if (v != 5 + D) a.F[(D * 8 + (own ? v : 5 + D)) * a.nct + c] = Fo[v];
        // the window is no longer read after the reconstruction barrier
#pragma unroll
        for (int v = 0; v < 5; ++v) flx[(v * TA + aa) * TD + fd] = Fo[v];
      }
      __syncthreads();
      if (cell) {
        const long long n = a.nct;
        const double *f0 = &flx[aa * TD + fd];
        const double id = 1.0 / b.dx[D];
        if constexpr (D == 0) {
#pragma unroll
          for (int v = 0; v < 5; ++v) a.F[v * n + c] = -(f0[v * TA * TD + 1] - f0[v * TA * TD]) * id;
        } else if constexpr (D == 1) {
#pragma unroll
          for (int v = 0; v < 5; ++v)
            a.F[v * n + c] = a.F[v * n + c] - (f0[v * TA * TD + 1] - f0[v * TA * TD]) * id;
        } else {
          double rhs[5];
#pragma unroll
          for (int v = 0; v < 5; ++v)
            rhs[v] = a.F[v * n + c] - (f0[v * TA * TD + 1] - f0[v * TA * TD]) * id;
          if constexpr (MK == MK_KS) {
            Prim q;    // the cell's own state in FP64
            q.rho = a.P[c]; q.u1 = a.P[n + c]; q.u2 = a.P[2 * n + c]; q.u3 = a.P[3 * n + c];
            q.ie = a.P[4 * n + c];
            q.B1 = a.Bcc[c]; q.B2 = a.Bcc[n + c]; q.B3 = a.Bcc[2 * n + c];
            q.ye = 0.0;
            add_sources<MK, 0>(a, b, idx[0], idx[1], q, rhs);
          }
          const double dt = rk.dt > 0.0 ? rk.dt : *rk.dtd;
          rk_cell<5>(a, c, rk.c0, rk.c1, rk.cdt * dt, rk.save, rhs);
        }
      }
    }
    __syncthreads();   // LDS is restaged by the next tile
  }
}

// Persistent face tiles with the next tile's stencil window streamed into LDS
// while the current tile's Riemann solves run (FP64, no scalar).  The window
// goes from global memory straight to LDS (gfx950 global_load_lds_dwordx4: 16
// bytes, two adjacent cells along x1, per lane; consecutive lanes fill
// consecutive LDS), so no registers hold it and the loads stay in flight
// across the solves.  Layouts keep x1 contiguous in LDS as in memory:
//   D = x1: stg[v][column][cell], NW = TD + 6 cells from org - 4 (even, so
//           every pair is 16-byte aligned; the first cell is not used);
//   D = x2, x3: stg[v][cell][column], NS = TD + 5 cells from org - 3, the TA
//           columns from an even x1 (the tile lists start at ng - 2).
// The right-face states use the same orientation.  Each workgroup walks the
// tile list with stride gridDim.x.  Results equal k_flux's to rounding (the
// same reconstruction and Riemann code on the same values; the two kernels
// are compiled apart, so fused multiply-adds may be formed differently).
#ifndef GRMHD_PF_WAVES
#define GRMHD_PF_WAVES 3
#endif
template <int MK, int D, int RECON, int FV, int RS, int SH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GRMHD_PF_WAVES)))
void k_flux_pf(KArgs a, const int4 *__restrict__ tiles, int ntiles)
{
  constexpr int TD = Shape<SH>::TD, TA = Shape<SH>::TA, NR = TD + 1, NV = 7;
  constexpr int NW = (D == 0) ? TD + 6 : TD + 5;      // window cells along D
  static_assert(TA % 2 == 0 && TD % 2 == 0, "pairs of cells along x1");
  __shared__ __align__(16) double stg[NV * TA * NW];
  __shared__ __align__(16) double sfr[NV * TA * NR];
  constexpr int AX = (D == 0) ? 1 : 0;
  constexpr int NCH = NV * TA * NW / 2;                // 16-byte chunks of a window
  constexpr int NIT = (NCH + 255) / 256;
  const int4 *const ctl = tiles;
  const BlockInfo *const cbl = a.blocks;
  const int tid = threadIdx.x;
  int fd, aa;
  if constexpr (D == 0) { fd = tid % TD; aa = tid / TD; }
  else                  { aa = tid % TA; fd = tid / TA; }

  // the window of tile ti into stg (asynchronous; completion: vmcnt)
  auto issue = [&](int ti) {
    const int4 t = ctl[ti];
    const BlockInfo b = cbl[t.x];
    const long long s1 = b.s[0], s12 = (long long)b.s[0] * b.s[1];
    // not unrolled: unrolled, the per-thread chunk offsets are hoisted out of
    // the tile loop and held in registers the Riemann solve needs
#pragma unroll 1
    for (int m = 0; m < NIT; ++m) {
      const int q0 = (tid & ~63) + 256 * m;
      const int q = q0 + (tid & 63);
      if (q < NCH) {
        int v, x1, j2, j3;           // variable, x1 of the pair's first cell, other indices
        if constexpr (D == 0) {
          v = q / (TA * NW / 2);
          const int r = q % (TA * NW / 2);
          const int pa = r / (NW / 2), s2 = r % (NW / 2);
          x1 = min(max(t.y - 4 + 2 * s2, 0), b.s[0] - 2);
          j2 = min(t.z + pa, b.s[1] - 1);
          j3 = t.w;
        } else {
          v = q / (NW * TA / 2);
          const int r = q % (NW * TA / 2);
          const int sd = r / (TA / 2), p2 = r % (TA / 2);
          x1 = min(t.y + 2 * p2, b.s[0] - 2);
          const int jd = min(max((D == 1 ? t.z : t.w) - 3 + sd, 0), b.s[D] - 1);
          j2 = D == 1 ? jd : t.z;
          j3 = D == 2 ? jd : t.w;
        }
        const double *src = v < 5 ? a.P + (long long)v * a.nct
                                  : a.Bcc + (long long)tcomp<D>(v - 5) * a.nct;
        src += b.off + x1 + s1 * j2 + s12 * j3;
        __builtin_amdgcn_global_load_lds((const void *)src,
                                         (__attribute__((address_space(3))) void *)(stg + 2 * q0),
                                         16, 0, 0);
      }
    }
  };

  int ti = blockIdx.x;
  if (ti < ntiles) issue(ti);
  for (; ti < ntiles; ti += gridDim.x) {
    __builtin_amdgcn_s_waitcnt(0);     // this wave's window loads (and stores) done
    __syncthreads();                   // ... and every other wave's
    const int4 t = ctl[ti];
    const BlockInfo b = cbl[t.x];
    const int org[3] = {t.y, t.z, t.w};
    const long long str[3] = {1, b.s[0], (long long)b.s[0] * b.s[1]};

    // reconstruct the own cell org[D]+fd (all variables; left state kept,
    // right state published), then the right faces of the cells org[D]-1
    auto win = [&](int v, int col, int k) -> double {   // stencil value k (0..4) of the own cell
      if constexpr (D == 0) return stg[(v * TA + col) * NW + fd + 2 + k];
      else return stg[(v * NW + fd + 1 + k) * TA + col];
    };
    auto rslot = [&](int v, int col, int f) -> double & {
      if constexpr (D == 0) return sfr[(v * TA + col) * NR + f];
      else return sfr[(v * NR + f) * TA + col];
    };
    double qR[NV];
    bool redo = false;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double f0 = win(v, aa, 0), f1 = win(v, aa, 1), f2 = win(v, aa, 2),
                   f3 = win(v, aa, 3), f4 = win(v, aa, 4);
      double l, r;
      redo |= !recon5_fast<RECON, FV, double>(f0, f1, f2, f3, f4, l, r);
      positivity(v, f2, l, r);
      rslot(v, aa, fd + 1) = r;
      qR[v] = l;
    }
    if (redo) {           // rare: a WENO pair that could not be normalised
#pragma unroll 1
      for (int v = 0; v < NV; ++v) {
        const double f0 = win(v, aa, 0), f1 = win(v, aa, 1), f2 = win(v, aa, 2),
                     f3 = win(v, aa, 3), f4 = win(v, aa, 4);
        double l, r;
        recon5<RECON, FV, double>(f0, f1, f2, f3, f4, l, r);
        positivity(v, f2, l, r);
        rslot(v, aa, fd + 1) = r;
#pragma unroll
        for (int w = 0; w < NV; ++w)
          if (w == v) qR[w] = l;
      }
    }
    for (int it = tid; it < NV * TA; it += 256) {
      const int v = it / TA, ca = it % TA;
      double f[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        if constexpr (D == 0) f[k] = stg[(v * TA + ca) * NW + 1 + k];
        else f[k] = stg[(v * NW + k) * TA + ca];
      }
      double l, r;
      recon5<RECON, FV, double>(f[0], f[1], f[2], f[3], f[4], l, r);
      positivity(v, f[2], l, r);
      rslot(v, ca, 0) = r;
    }

    // this face: position and the values it reads from global memory, loaded
    // before the next window is requested (vector loads complete in order,
    // so a load issued behind the stream would wait for all of it)
    int idx[3] = {org[0], org[1], org[2]};
    idx[D] = org[D] + fd;
    idx[AX] = org[AX] + aa;
    const bool live = idx[D] < a.ng + b.n[D] && idx[AX] >= a.ng - 1 &&
                      idx[AX] <= a.ng + b.n[AX] && idx[AX] < b.s[AX];
    const bool pole = D == 1 && (idx[1] == b.pole_lo || idx[1] == b.pole_hi);
    const long long c = b.off + idx[0] * str[0] + idx[1] * str[1] + idx[2] * str[2];
    double gr = 0.0, gs = 0.0, gc = 0.0, bface = 0.0;
    if (live && !pole) {
      if constexpr (MK == MK_KS) {
        gr = D == 0 ? a.tab.rf[b.tab1 + idx[0]] : a.tab.rc[b.tab1 + idx[0]];
        gs = D == 1 ? a.tab.sf[b.tab2 + idx[1]] : a.tab.sc[b.tab2 + idx[1]];
        gc = D == 1 ? a.tab.cf[b.tab2 + idx[1]] : a.tab.cc[b.tab2 + idx[1]];
      }
      bface = a.Bf[D * a.nct + c];
    }
    // wait for these loads here, while no window load is in flight behind them
    asm volatile("" ::"v"(gr), "v"(gs), "v"(gc), "v"(bface));
    __syncthreads();      // the window is read: stream the next one in
    if (ti + (int)gridDim.x < ntiles) issue(ti + gridDim.x);

    if (live) {
      double qL[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) qL[v] = rslot(v, aa, fd);   // cell idx[D]-1
      double Fo[8];
      if (pole) {     // sqrt(-g) = 0 on the axis
#pragma unroll
        for (int v = 0; v < 8; ++v) Fo[v] = 0.0;
      } else {
        Geo G;
        if constexpr (MK == MK_KS) G = geo_ks<double>(gr, gs, gc, a.met.M, a.met.a);
        else G = geo_mink<double>();
        face_flux_geo<MK, D, RS, double, 0>(a, G, bface, qL, qR, Fo);
      }
#pragma unroll
      for (int v = 0; v < 8; ++v)
        if (v != 5 + D) a.F[(D * 8 + v) * a.nct + c] = Fo[v];
    }
  }
}

// One face on the upper boundary plane along D (index ng + n_D); e indexes
// the (n_A + 2) x (n_B + 2) faces of the plane (transverse ghosts included).
template <int MK, int D, int RECON, int FV, int RS, typename T, int NSC>
__device__ __forceinline__ void plane_face(const KArgs &a, const BlockInfo &b, int e)
{
  constexpr int NV = 7 + NSC;
  constexpr int AX = (D == 0) ? 1 : 0;
  constexpr int BX = (D == 2) ? 1 : 2;
  const int na = b.n[AX] + 2, nb = b.n[BX] + 2;
  if (e >= na * nb) return;
  int idx[3];
  idx[D] = a.ng + b.n[D];
  idx[AX] = a.ng - 1 + e % na;
  idx[BX] = a.ng - 1 + e / na;
  const long long str[3] = {1, b.s[0], (long long)b.s[0] * b.s[1]};
  const long long c = b.off + idx[0] * str[0] + idx[1] * str[1] + idx[2] * str[2];
  const long long sd = str[D];
  T qL[NV], qR[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double *arr = v < 5 ? a.P + v * a.nct
                      : v < 7 ? a.Bcc + tcomp<D>(v - 5) * a.nct : a.P + 5 * a.nct;
    T f[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) f[m] = T(arr[c + (m - 3) * sd]);
    T l, r;
    recon5<RECON, FV, T>(f[0], f[1], f[2], f[3], f[4], l, r);   // cell idx-1
    positivity(v, f[2], l, r);
    qL[v] = r;
    recon5<RECON, FV, T>(f[1], f[2], f[3], f[4], f[5], l, r);   // cell idx
    positivity(v, f[3], l, r);
    qR[v] = l;
  }
  face_flux_store<MK, D, RS, T, NSC>(a, b, idx[0], idx[1], c, qL, qR);
}

// The boundary planes of all three directions in one launch of 64-thread
// workgroups (a plane holds ~1/n of a direction's faces: small grids of
// latency-bound work are better spread thin over the CUs):
// chunk = (3 * block + D, first face of 64).
template <int MK, int RECON, int FV, int RS, typename T, int NSC = 0>
__global__ __launch_bounds__(64) void k_flux_planes(KArgs a, const int2 *__restrict__ chunks)
{
  const int2 ch = chunks[blockIdx.x];
  const int D = ch.x % 3;
  const BlockInfo b = a.blocks[ch.x / 3];
  const int e = ch.y + threadIdx.x;
  if (D == 0) plane_face<MK, 0, RECON, FV, RS, T, NSC>(a, b, e);
  else if (D == 1) plane_face<MK, 1, RECON, FV, RS, T, NSC>(a, b, e);
  else plane_face<MK, 2, RECON, FV, RS, T, NSC>(a, b, e);
}

// ------------------------------------------------- two-level coupling

// Edge EMFs of every cell of the box [ng, ng+n] (the four-point averages the
// update forms itself on single-level packs).
__global__ __launch_bounds__(256) void k_emf(KArgs a, const int2 *__restrict__ chunks)
{
  const int2 ch = chunks[blockIdx.x];
  const BlockInfo b = a.blocks[ch.x];
  const int e = ch.y + threadIdx.x;
  const int m1 = b.n[0] + 1, m2 = b.n[1] + 1;
  if (e >= m1 * m2 * (b.n[2] + 1)) return;
  const int ng = a.ng;
  const int i = ng + e % m1, j = ng + (e / m1) % m2, k = ng + e / (m1 * m2);
  const long long sj = b.s[0], sk = (long long)b.s[0] * b.s[1];
  const long long q = b.off + i + sj * j + sk * k;
  const long long n = a.nct;
  const double *F0 = a.F, *F1 = a.F + 8 * n, *F2 = a.F + 16 * n;
  a.E[q] = 0.25 * (F1[7 * n + q] + F1[7 * n + q - sk] - F2[6 * n + q] - F2[6 * n + q - sj]);
  a.E[n + q] = 0.25 * (F2[5 * n + q] + F2[5 * n + q - 1] - F0[7 * n + q] - F0[7 * n + q - sk]);
  a.E[2 * n + q] = 0.25 * (F0[6 * n + q] + F0[6 * n + q - sj] - F1[5 * n + q] - F1[5 * n + q - 1]);
}

// Coarse hydro fluxes on level boundaries <- mean of the 4 fine fluxes.
__global__ __launch_bounds__(256) void k_flux_fix(KArgs a, const FixF *__restrict__ map, int nfix)
{
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nfix) return;
  const FixF f = map[e];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double *p = a.F + (long long)(f.D * 8 + v) * a.nct + f.src;
    double acc = 0.0;
    for (int bb = 0; bb < 2; ++bb)
      for (int aa = 0; aa < 2; ++aa) acc += p[aa * f.st1 + bb * f.st2];
    a.F[(long long)(f.D * 8 + v) * a.nct + f.dst] = 0.25 * acc;
  }
}

// Coarse EMFs on level boundaries <- mean of the 2 fine EMFs.
__global__ __launch_bounds__(256) void k_emf_fix(KArgs a, const FixE *__restrict__ map, int nfix)
{
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nfix) return;
  const FixE f = map[e];
  const double *p = a.E + (long long)f.e * a.nct;
  a.E[(long long)f.e * a.nct + f.dst] = 0.5 * (p[f.src] + p[f.src + f.st]);
}

// ------------------------------------------------------------------ update

// HYDRO = 0: the constrained-transport part only (the flux tiles have done
// the hydro update).
template <int MK, int EARR, int NSC = 0, int HYDRO = 1>
__global__ __launch_bounds__(256) void k_update(KArgs a, const int2 *__restrict__ chunks,
                                                double dt_in, const double *__restrict__ dt_dev,
                                                double c0, double c1, double cdt, int mode)
{
  const int2 ch = chunks[blockIdx.x];
  const BlockInfo b = a.blocks[ch.x];
  const int e = ch.y + threadIdx.x;
  const int m1 = b.n[0] + 1, m2 = b.n[1] + 1;
  if (e >= m1 * m2 * (b.n[2] + 1)) return;
  const int ng = a.ng;
  const int i = ng + e % m1, j = ng + (e / m1) % m2, k = ng + e / (m1 * m2);
  const long long sj = b.s[0], sk = (long long)b.s[0] * b.s[1];
  const long long c = b.off + i + sj * j + sk * k;
  const long long n = a.nct;
  const double dt = dt_in > 0.0 ? dt_in : *dt_dev;
  const double h = cdt * dt;
  const double i1 = 1.0 / b.dx[0], i2 = 1.0 / b.dx[1], i3 = 1.0 / b.dx[2];
  const double *F0 = a.F, *F1 = a.F + 8 * n, *F2 = a.F + 16 * n;
  const bool in1 = i < ng + b.n[0], in2 = j < ng + b.n[1], in3 = k < ng + b.n[2];

  // Kerr-Schild sources first, then a scheduling barrier: without it the
  // compiler hoists the 30 flux loads above the source arithmetic and holds
  // both (134 VGPRs, 3 waves per SIMD); apart it needs 92 (5 waves).  The
  // sources are added at the same point as before, so the sums are unchanged.
  double S[5 + NSC] = {};
  if constexpr (MK == MK_KS) {
    if (HYDRO && in1 && in2 && in3) {
      Prim q;
      q.rho = a.P[c]; q.u1 = a.P[n + c]; q.u2 = a.P[2 * n + c]; q.u3 = a.P[3 * n + c];
      q.ie = a.P[4 * n + c];
      q.B1 = a.Bcc[c]; q.B2 = a.Bcc[n + c]; q.B3 = a.Bcc[2 * n + c];
      q.ye = NSC ? a.P[5 * n + c] : 0.0;
      add_sources<MK, NSC>(a, b, i, j, q, S);
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  if (HYDRO && in1 && in2 && in3) {
    double rhs[5 + NSC];
#pragma unroll
    for (int v = 0; v < 5; ++v)
      rhs[v] = -(F0[v * n + c + 1] - F0[v * n + c]) * i1 - (F1[v * n + c + sj] - F1[v * n + c]) * i2 -
               (F2[v * n + c + sk] - F2[v * n + c]) * i3;
    if constexpr (NSC != 0)   // scalar fluxes in the normal-field slots 5, 6, 7
      rhs[5] = -(F0[5 * n + c + 1] - F0[5 * n + c]) * i1 -
               (F1[6 * n + c + sj] - F1[6 * n + c]) * i2 - (F2[7 * n + c + sk] - F2[7 * n + c]) * i3;
    if constexpr (MK == MK_KS) {
      rhs[1] += S[1];
      rhs[2] += S[2];
      rhs[4] += S[4];
    }
    rk_cell<5 + NSC>(a, c, c0, c1, h, mode, rhs);
  }

  // edge EMFs: E1 = Omega_23 at (i, j-1/2, k-1/2), E2 = Omega_31 at
  // (i-1/2, j, k-1/2), E3 = Omega_12 at (i-1/2, j-1/2, k); four-point averages
  // (EARR: read from the edge arrays, which two-level meshes correct at level
  // boundaries before the update)
  auto E1 = [&](long long q) {
    if constexpr (EARR != 0) return a.E[q];
    return 0.25 * (F1[7 * n + q] + F1[7 * n + q - sk] - F2[6 * n + q] - F2[6 * n + q - sj]);
  };
  auto E2 = [&](long long q) {
    if constexpr (EARR != 0) return a.E[n + q];
    return 0.25 * (F2[5 * n + q] + F2[5 * n + q - 1] - F0[7 * n + q] - F0[7 * n + q - sk]);
  };
  auto E3 = [&](long long q) {
    if constexpr (EARR != 0) return a.E[2 * n + q];
    return 0.25 * (F0[6 * n + q] + F0[6 * n + q - sj] - F1[5 * n + q] - F1[5 * n + q - 1]);
  };
  double rb[3];
  bool upd[3] = {in2 && in3, in1 && in3, in1 && in2};
  rb[0] = upd[0] ? (E3(c + sj) - E3(c)) * i2 - (E2(c + sk) - E2(c)) * i3 : 0.0;
  rb[1] = upd[1] ? -(E3(c + 1) - E3(c)) * i1 + (E1(c + sk) - E1(c)) * i3 : 0.0;
  rb[2] = upd[2] ? (E2(c + 1) - E2(c)) * i1 - (E1(c + sj) - E1(c)) * i2 : 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d)
    if (upd[d]) rk_value(a.Bf, a.Bf0, d * n + c, c0, c1, h, mode, rb[d]);
}

// ------------------------------------------------------------- reductions

constexpr int NPART = 14;   // smax, divmax, bmax, tot[5], nfail, nfloor, itsum, wavemax, guess fallback, scalar total

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Per-cell diagnostics of the reductions: [0] sum_d max|lambda_d| / dx_d,
// [1] |div B|, [2] max |face B|, [3..7] U dV, [8] failed inversion,
// [9] floor hit, [10] Newton iterations, [12] learned guess rejected,
// [13] scalar U dV.
template <int MK, int NSC = 0>
__device__ __forceinline__ void cell_diag(const KArgs &a, const BlockInfo &b, const Geo &G,
                                          const Prim &q, const double bf[6],
                                          const double U[5 + NSC], int fl, int iters,
                                          double val[NPART])
{
  const Aux A = aux_cell<NSC>(a, G, q);
  double s = 0.0, lm, lp;
  if (a.active[0]) { speeds_of<0>(G, A, lm, lp); s += fmax(fabs(lm), fabs(lp)) / b.dx[0]; }
  if (a.active[1]) { speeds_of<1>(G, A, lm, lp); s += fmax(fabs(lm), fabs(lp)) / b.dx[1]; }
  if (a.active[2]) { speeds_of<2>(G, A, lm, lp); s += fmax(fabs(lm), fabs(lp)) / b.dx[2]; }
  val[0] = s;
  val[1] = fabs((bf[1] - bf[0]) / b.dx[0] + (bf[3] - bf[2]) / b.dx[1] + (bf[5] - bf[4]) / b.dx[2]);
  val[2] = fmax(fmax(fmax(fabs(bf[0]), fabs(bf[1])), fmax(fabs(bf[2]), fabs(bf[3]))),
                fmax(fabs(bf[4]), fabs(bf[5])));
  const double dV = b.dx[0] * b.dx[1] * b.dx[2];
#pragma unroll
  for (int v = 0; v < 5; ++v) val[3 + v] = U[v] * dV;
  val[8] = (fl & 8) ? 1.0 : 0.0;
  val[9] = (fl & 7) ? 1.0 : 0.0;
  val[10] = (double)iters;
  val[11] = 0.0;
  val[12] = (fl & 16) ? 1.0 : 0.0;
  val[13] = NSC ? U[NSC ? 5 : 0] * dV : 0.0;
}

__device__ __forceinline__ int wave_max_i(int v)
{
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_sum_i(int v)
{
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fold the 256 threads' diagnostics (wavefront shuffles, then a fixed order
// over the 4 wavefronts) into part[blockIdx.x]; every thread must call it.
// The 0/1 counters (failures, floors, guess fallbacks) are counted by ballot
// and the Newton iterations summed as integers: the same exact values as
// summing them as doubles, with fewer cross-lane shuffles.
template <int NSC>
__device__ __forceinline__ void block_diag_store(double val[NPART], double *__restrict__ part)
{
  __shared__ double sh[4][NPART];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double nfail = (double)__popcll(__ballot(val[8] != 0.0));
  const double nfloor = (double)__popcll(__ballot(val[9] != 0.0));
  const double nfall = (double)__popcll(__ballot(val[12] != 0.0));
  const int it = (int)val[10];
  const int itsum = wave_sum_i(it), itmax = wave_max_i(it);
#pragma unroll
  for (int q = 0; q < 3; ++q) val[q] = wave_max(val[q]);
#pragma unroll
  for (int q = 3; q < 8; ++q) val[q] = wave_sum(val[q]);
  val[8] = nfail;
  val[9] = nfloor;
  val[10] = (double)itsum;
  val[11] = (double)itmax;
  val[12] = nfall;
  val[13] = NSC ? wave_sum(val[13]) : 0.0;
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NPART; ++q) sh[wv][q] = val[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double o[NPART];
#pragma unroll
    for (int q = 0; q < NPART; ++q) o[q] = sh[0][q];
    for (int w = 1; w < 4; ++w) {
      for (int q = 0; q < 3; ++q) o[q] = fmax(o[q], sh[w][q]);
      for (int q = 3; q < NPART; ++q) o[q] += sh[w][q];
    }
    for (int q = 0; q < NPART; ++q) part[(long long)blockIdx.x * NPART + q] = o[q];
  }
}

template <int MK, int NSC = 0>
__global__ __launch_bounds__(256) void k_reduce(KArgs a, const int2 *__restrict__ chunks,
                                                double *__restrict__ part)
{
  const int2 ch = chunks[blockIdx.x];
  const BlockInfo b = a.blocks[ch.x];
  const int e = ch.y + threadIdx.x;
  double val[NPART];
#pragma unroll
  for (int q = 0; q < NPART; ++q) val[q] = 0.0;
  if (e < b.n[0] * b.n[1] * b.n[2]) {
    const int ng = a.ng;
    const int i = ng + e % b.n[0], j = ng + (e / b.n[0]) % b.n[1], k = ng + e / (b.n[0] * b.n[1]);
    const long long sj = b.s[0], sk = (long long)b.s[0] * b.s[1];
    const long long c = b.off + i + sj * j + sk * k;
    const long long n = a.nct;
    const Geo G = geo_center<MK>(a, b, i, j);
    const double isg = 1.0 / G.sqrtg;
    const double bf[6] = {a.Bf[c], a.Bf[c + 1], a.Bf[n + c], a.Bf[n + c + sj], a.Bf[2 * n + c],
                          a.Bf[2 * n + c + sk]};
    Prim q;
    q.rho = a.P[c]; q.u1 = a.P[n + c]; q.u2 = a.P[2 * n + c]; q.u3 = a.P[3 * n + c];
    q.ie = a.P[4 * n + c];
    q.B1 = 0.5 * (bf[0] + bf[1]) * isg; q.B2 = 0.5 * (bf[2] + bf[3]) * isg;
    q.B3 = 0.5 * (bf[4] + bf[5]) * isg;
    q.ye = NSC ? a.P[5 * n + c] : 0.0;
    double U[5 + NSC];
#pragma unroll
    for (int v = 0; v < 5 + NSC; ++v) U[v] = a.U[v * n + c];
    cell_diag<MK, NSC>(a, b, G, q, bf, U, a.flags[c], a.iters[c], val);
  }
  block_diag_store<NSC>(val, part);
}

// --------------------------------------------------------------- inversion

template <int MK, int NSC = 0>
__device__ __forceinline__ void cons_store(const KArgs &a, long long c, const Geo &G,
                                           const Prim &q, double Uout[5 + NSC])
{
  const Aux A = aux_cell<NSC>(a, G, q);
  double U[8];
  cons_of(G, q, A, U);
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    Uout[v] = G.sqrtg * U[v];
    a.U[v * a.nct + c] = Uout[v];
  }
  if constexpr (NSC != 0) {
    Uout[5] = G.sqrtg * (U[0] * q.ye);
    a.U[5 * a.nct + c] = Uout[5];
  }
}

// One cell's inversion + floors; with RED also its reduction diagnostics.
// NSC = 1: the Y_e scalar (P[5], U[5] = sqrt(gamma) D Y_e) and, when a table
// is bound, the general-EOS master function with the table's bounds
// (Sec. 3.2: rho, eps and Y_e stay inside the table).
template <int MK, int GUESS, int RED, int NSC = 0>
__device__ __forceinline__ void c2p_cell(const KArgs &a, const BlockInfo &b, int e,
                                         float g_mu, float g_W, double val[NPART])
{
  constexpr int NU = 5 + NSC;
  const int ng = a.ng;
  const int i = ng + e % b.n[0], j = ng + (e / b.n[0]) % b.n[1], k = ng + e / (b.n[0] * b.n[1]);
  const long long sj = b.s[0], sk = (long long)b.s[0] * b.s[1];
  const long long c = b.off + i + sj * j + sk * k;
  const long long n = a.nct;
  const Geo G = geo_center<MK>(a, b, i, j);
  const double isg = inv(G.sqrtg);
  double Ur[NU], Ud[NU];
#pragma unroll
  for (int v = 0; v < NU; ++v) {
    Ur[v] = a.U[v * n + c];
    Ud[v] = Ur[v] * isg;
  }
  const double bf[6] = {a.Bf[c], a.Bf[c + 1], a.Bf[n + c], a.Bf[n + c + sj], a.Bf[2 * n + c],
                        a.Bf[2 * n + c + sk]};
  const double B1 = 0.5 * (bf[0] + bf[1]) * isg;
  const double B2 = 0.5 * (bf[2] + bf[3]) * isg;
  const double B3 = 0.5 * (bf[4] + bf[5]) * isg;
  Prim prev;
  prev.rho = a.P[c]; prev.u1 = a.P[n + c]; prev.u2 = a.P[2 * n + c]; prev.u3 = a.P[3 * n + c];
  prev.ie = a.P[4 * n + c];
  prev.B1 = B1; prev.B2 = B2; prev.B3 = B3;
  prev.ye = NSC ? a.P[5 * n + c] : 0.0;
  const bool tab = NSC != 0 && a.et.d != nullptr;

  const double gam = a.eos.gam;
  int flag = 0, iters = 0;
  Prim q = prev;
  bool ok = Ud[0] > 0.0;
#pragma unroll
  for (int v = 0; v < NU; ++v) ok = ok && isfinite(Ud[v]);
  if (ok) {
    const double D = Ud[0], iD = inv(D);
    double ye = 0.0;
    if constexpr (NSC != 0) {
      const double yr = Ud[5] * iD;
      ye = tab ? fmin(fmax(yr, a.et.lo[2]), a.et.hi[2]) : yr;
      if (ye != yr) flag |= 32;            // Y_e held inside the table
    }
    // S^i = gamma^ij S_j ; B_i = gamma_ij B^j
    const double Su1 = G.gi11 * Ud[1] + G.gi13 * Ud[3];
    const double Su2 = G.gi22 * Ud[2];
    const double Su3 = G.gi13 * Ud[1] + G.gi33 * Ud[3];
    const double Bl1 = G.g11 * B1 + G.g13 * B3, Bl2 = G.g22 * B2, Bl3 = G.g13 * B1 + G.g33 * B3;
    C2P m;
    m.gam = gam;
    m.q = Ud[4] * iD;
    m.r2 = (Ud[1] * Su1 + Ud[2] * Su2 + Ud[3] * Su3) * iD * iD;
    m.b2 = (Bl1 * B1 + Bl2 * B2 + Bl3 * B3) * iD;
    const double isD = inv(sqrt(D));
    m.rb = (Ud[1] * B1 + Ud[2] * B2 + Ud[3] * B3) * iD * isD;
    m.v2max = m.r2 / (1.0 + m.r2);
    C2PT mt;
    mt.q = m.q; mt.r2 = m.r2; mt.b2 = m.b2; mt.rb = m.rb; mt.v2max = m.v2max;
    mt.D = D; mt.ye = ye;
    auto F = [&](double mu, double &df) -> double {
      if constexpr (NSC != 0) {
        if (tab) return master_tab(mt, a.et, mu, df);
      }
      return master(m, mu, df);
    };
    double df1;
    if (F(1.0, df1) < 0.0) {
      ok = false;
    } else {
      double mu;
      if constexpr (GUESS == 1 && NSC == 0) {
        const Aux Ap = aux_of(G, gam, prev);
        mu = 1.0 / ((1.0 + gam * prev.ie / prev.rho) * Ap.W);
      } else if constexpr (GUESS == 1) {
        double pp, gpp;
        thermo_of<NSC>(a, prev.rho, prev.ie, prev.ye, pp, gpp);
        const Aux Ap = aux_th(G, prev, pp, gpp);
        mu = 1.0 / ((1.0 + (prev.ie + pp) / prev.rho) * Ap.W);
      } else {
        mu = 1.0 / sqrt(1.0 + m.r2);             // cold guess: no prior state
        if constexpr (GUESS == 2) {
          // learned guess, kept if its W(mu0) agrees with the network's own
          // W output to 50 % (out-of-distribution check); else the cold guess
          const double g = (double)g_mu;
          bool take = g > 0.0 && g <= 1.0;
          if (take) {
            const double x0 = 1.0 / (1.0 + g * m.b2);
            const double rb0 = m.r2 * x0 * x0 + g * x0 * (1.0 + x0) * m.rb * m.rb;
            double v20 = g * g * rb0;
            v20 = v20 > m.v2max ? m.v2max : v20;
            const double W0 = 1.0 / sqrt(1.0 - v20);
            take = fabs((double)g_W - W0) <= 0.5 * W0;
          }
          if (take) mu = g;
          else flag |= 16;
        }
      }
      if (!(mu > 0.0 && mu <= 1.0)) mu = 0.5;
      double lo = 0.0, hi = 1.0;
      const double tol = a.eos.tol;
      for (iters = 1; iters <= a.eos.max_iter; ++iters) {
        double df;
        const double f = F(mu, df);
        if (f == 0.0) break;
        if (f < 0.0) lo = mu; else hi = mu;
        double mn = mu - f / df;
        if (!(mn > lo && mn < hi)) mn = 0.5 * (lo + hi);
        const double dmu = fabs(mn - mu);
        mu = mn;
        if (dmu <= tol * mu) break;
      }
      // no root within the iteration cap: the state counts as not inverted
      if (iters > a.eos.max_iter) ok = false;
      const double x = inv(1.0 + mu * m.b2);
      const double rbar2 = m.r2 * x * x + mu * x * (1.0 + x) * m.rb * m.rb;
      const double qbar = m.q - 0.5 * m.b2 - 0.5 * mu * mu * x * x * (m.b2 * m.r2 - m.rb * m.rb);
      double v2 = mu * mu * rbar2;
      v2 = v2 > m.v2max ? m.v2max : v2;
      const double iW = sqrt(1.0 - v2);
      const double W = inv(iW);
      double eps = W * (qbar - mu * rbar2) + v2 * W * W * inv(1.0 + W);
      eps = eps < 0.0 ? 0.0 : eps;
      if (tab) eps = fmin(fmax(eps, a.et.eps_min), a.et.eps_max);
      q.rho = D * iW;
      q.ie = q.rho * eps;
      q.ye = ye;
      const double f1 = mu * x * W, f2 = mu * m.rb * isD;
      q.u1 = f1 * (Su1 * iD + f2 * B1);
      q.u2 = f1 * (Su2 * iD + f2 * B2);
      q.u3 = f1 * (Su3 * iD + f2 * B3);
      // a root whose primitives are not finite (the v^2 bound rounded to 1,
      // so W overflowed) is no inversion either
      if (!(q.rho > 0.0) || !isfinite(q.rho) || !isfinite(q.ie) || !isfinite(q.u1) ||
          !isfinite(q.u2) || !isfinite(q.u3))
        ok = false;
    }
  }
  if (!ok) {
    q = prev;
    flag = (flag & 16) | 8;
  }
  // floors (Sec. 3.2), never below the table
  double rflr = a.eos.rho_flr0, uflr = a.eos.u_flr0;      // r = 1: no radial factor
  if constexpr (MK == MK_KS) {
    rflr = a.flr_rho[b.tab1 + i];
    uflr = a.flr_u[b.tab1 + i];
  }
  if (tab) rflr = fmax(rflr, a.et.rho_min);
  if (q.rho < rflr) { q.rho = rflr; flag |= 1; }
  if (tab) {
    if (q.rho > a.et.rho_max) { q.rho = a.et.rho_max; flag |= 1; }
    uflr = fmax(uflr, q.rho * a.et.eps_min);
  }
  if (q.ie < uflr) { q.ie = uflr; flag |= 2; }
  if (tab && q.ie > q.rho * a.et.eps_max) { q.ie = q.rho * a.et.eps_max; flag |= 2; }
  const double ut2 = G.g11 * q.u1 * q.u1 + 2.0 * G.g13 * q.u1 * q.u3 + G.g22 * q.u2 * q.u2 +
                     G.g33 * q.u3 * q.u3;
  if (sqrt(1.0 + ut2) > a.eos.W_max) {
    const double sc = sqrt((a.eos.W_max * a.eos.W_max - 1.0) / ut2);
    q.u1 *= sc; q.u2 *= sc; q.u3 *= sc;
    flag |= 4;
  }
  a.P[c] = q.rho; a.P[n + c] = q.u1; a.P[2 * n + c] = q.u2; a.P[3 * n + c] = q.u3;
  a.P[4 * n + c] = q.ie;
  if constexpr (NSC != 0) a.P[5 * n + c] = q.ye;
  if (flag & 47) cons_store<MK, NSC>(a, c, G, q, Ur);
  a.flags[c] = (int8_t)flag;
  a.iters[c] = (uint8_t)min(iters, 255);
  if (flag & 8) atomicAdd(a.nfail, 1ull);
  if constexpr (RED != 0) cell_diag<MK, NSC>(a, b, G, q, bf, Ur, flag, min(iters, 255), val);
}

// The floors of every radial table entry (Sec. 3.2): rho_flr0 r^-rho_flr_pow
// and u_flr0 r^-u_flr_pow, once per entry (and per change of the floors)
// instead of twice per cell and inversion.
__global__ __launch_bounds__(256) void k_floor_tab(KArgs a, int nr)
{
  const int ir = blockIdx.x * 256 + threadIdx.x;
  if (ir >= nr) return;
  const double r = a.tab.rc[ir];
  a.flr_rho[ir] = a.eos.rho_flr0 * pow(r, -a.eos.rho_flr_pow);
  a.flr_u[ir] = a.eos.u_flr0 * pow(r, -a.eos.u_flr_pow);
}

// Inversion of every interior cell; RED = 1 also folds the reduction
// diagnostics of the final state into part[] (the reductions pass fused into
// the last inversion of a step).
template <int MK>
__device__ __forceinline__ void mlp_cell_features(const KArgs &a, const MlpDev &m,
                                                  const BlockInfo &b, int e, float x[5]);

// Inversion of every interior cell; RED = 1 also folds the reduction
// diagnostics of the final state into part[] (the reductions pass fused into
// the last inversion of a step).  GUESS = 2: each wavefront first evaluates
// the learned guess of its 64 cells (features -> LDS -> BF16 matrix-core
// layers with the activations in registers), so the guess never leaves the
// chip.
// Occupancy: 4 waves per SIMD (128 VGPRs, a few spilled) for the plain
// inversion; with the scalar 2 (up to 256 VGPRs, none spilled: at 3 or 4 waves
// the general-EOS inversion spilled 24 or 66 and ran 1.1-1.6x slower); the one
// with the fused reductions keeps the compiler's choice.
template <int MK, int GUESS, int RED, int NSC = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RED ? 1 : (NSC ? 2 : 4))))
void k_c2p(KArgs a, const int2 *__restrict__ chunks, MlpDev md,
                                             double *__restrict__ part)
{
  const int2 ch = chunks[blockIdx.x];
  const BlockInfo b = a.blocks[ch.x];
  const int e = ch.y + threadIdx.x;
  const bool live = e < b.n[0] * b.n[1] * b.n[2];
  double val[NPART];
#pragma unroll
  for (int q = 0; q < NPART; ++q) val[q] = 0.0;
  float g_mu = -1.0f, g_W = 0.0f;
  if constexpr (GUESS == 2) {
    __shared__ __align__(16) unsigned short X[4][64 * 16];
    __shared__ float out[4][64 * MLP_OUT];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float x[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    if (live) mlp_cell_features<MK>(a, md, b, e, x);
#pragma unroll
    for (int q = 0; q < 16; ++q) X[w][lane * 16 + q] = q < 5 ? f2bf(x[q]) : 0;
    __syncthreads();
    mlp_wave(md, X[w], out[w], lane);
    // mu = 1/(hW) <= 1 always: a guess above 1 (log hW output slightly
    // negative near h W = 1) is clamped; a non-finite or non-positive one is
    // marked -1.  The network's own W rides along for the consistency check.
    const float mu = fminf(expf(-out[w][lane * 2 + 1]), 1.0f);
    g_mu = (mu > 0.0f) ? mu : -1.0f;
    g_W = expf(out[w][lane * 2]);
  }
  if (live) c2p_cell<MK, GUESS, RED, NSC>(a, b, e, g_mu, g_W, val);
  if constexpr (RED != 0) block_diag_store<NSC>(val, part);
}

template <int MK, int NSC = 0>
__global__ __launch_bounds__(256) void k_p2c(KArgs a, const int2 *__restrict__ chunks)
{
  const int2 ch = chunks[blockIdx.x];
  const BlockInfo b = a.blocks[ch.x];
  const int e = ch.y + threadIdx.x;
  if (e >= b.n[0] * b.n[1] * b.n[2]) return;
  const int ng = a.ng;
  const int i = ng + e % b.n[0], j = ng + (e / b.n[0]) % b.n[1], k = ng + e / (b.n[0] * b.n[1]);
  const long long sj = b.s[0], sk = (long long)b.s[0] * b.s[1];
  const long long c = b.off + i + sj * j + sk * k;
  const long long n = a.nct;
  const Geo G = geo_center<MK>(a, b, i, j);
  const double isg = 1.0 / G.sqrtg;
  Prim q;
  q.rho = a.P[c]; q.u1 = a.P[n + c]; q.u2 = a.P[2 * n + c]; q.u3 = a.P[3 * n + c];
  q.ie = a.P[4 * n + c];
  q.B1 = 0.5 * (a.Bf[c] + a.Bf[c + 1]) * isg;
  q.B2 = 0.5 * (a.Bf[n + c] + a.Bf[n + c + sj]) * isg;
  q.B3 = 0.5 * (a.Bf[2 * n + c] + a.Bf[2 * n + c + sk]) * isg;
  q.ye = NSC ? a.P[5 * n + c] : 0.0;
  double Uo[5 + NSC];
  cons_store<MK, NSC>(a, c, G, q, Uo);
}

// -------------------------------------------------------------- reductions

// One workgroup folds the per-workgroup partials in a fixed order.
// res: dt, divb_rel, divb_max, tot[5], nfail, nfloor, itsum, wavemax_sum, bmax, smax
__global__ __launch_bounds__(256) void k_reduce_fin(const double *__restrict__ part, int np,
                                                    double cfl, double dxmin, double *res)
{
  __shared__ double sh[256][NPART];
  double o[NPART];
#pragma unroll
  for (int q = 0; q < NPART; ++q) o[q] = 0.0;
  for (int p = threadIdx.x; p < np; p += 256) {
    for (int q = 0; q < 3; ++q) o[q] = fmax(o[q], part[(long long)p * NPART + q]);
    for (int q = 3; q < NPART; ++q) o[q] += part[(long long)p * NPART + q];
  }
  for (int q = 0; q < NPART; ++q) sh[threadIdx.x][q] = o[q];
  __syncthreads();
  // pairwise tree in a fixed order (deterministic)
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const int t = threadIdx.x;
      for (int q = 0; q < 3; ++q) sh[t][q] = fmax(sh[t][q], sh[t + w][q]);
      for (int q = 3; q < NPART; ++q) sh[t][q] += sh[t + w][q];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int q = 0; q < NPART; ++q) o[q] = sh[0][q];
    res[0] = o[0] > 0.0 ? cfl / o[0] : 0.0;
    res[1] = o[2] > 0.0 ? o[1] / (o[2] / dxmin) : o[1];
    res[2] = o[1];
    for (int v = 0; v < 5; ++v) res[3 + v] = o[3 + v];
    res[8] = o[8]; res[9] = o[9]; res[10] = o[10]; res[11] = o[11];
    res[12] = o[2]; res[13] = o[0]; res[14] = o[12]; res[15] = o[13];
  }
}

// ----------------------------------------------------------- learned guess

// The network's standardised features of interior cell e of block b (its
// undensitized conserved state and cell-centred field on the cell's metric).
template <int MK>
__device__ __forceinline__ void mlp_cell_features(const KArgs &a, const MlpDev &m,
                                                  const BlockInfo &b, int e, float x[5])
{
  const int ng = a.ng;
  const int i = ng + e % b.n[0], j = ng + (e / b.n[0]) % b.n[1], k = ng + e / (b.n[0] * b.n[1]);
  const long long sj = b.s[0], sk = (long long)b.s[0] * b.s[1];
  const long long c = b.off + i + sj * j + sk * k;
  const long long n = a.nct;
  const Geo G = geo_center<MK>(a, b, i, j);
  const double isg = 1.0 / G.sqrtg;
  const double D = a.U[c] * isg, S1 = a.U[n + c] * isg, S2 = a.U[2 * n + c] * isg;
  const double S3 = a.U[3 * n + c] * isg, tau = a.U[4 * n + c] * isg;
  const double B1 = 0.5 * (a.Bf[c] + a.Bf[c + 1]) * isg;
  const double B2 = 0.5 * (a.Bf[n + c] + a.Bf[n + c + sj]) * isg;
  const double B3 = 0.5 * (a.Bf[2 * n + c] + a.Bf[2 * n + c + sk]) * isg;
  const double SS = G.gi11 * S1 * S1 + 2.0 * G.gi13 * S1 * S3 + G.gi22 * S2 * S2 + G.gi33 * S3 * S3;
  const double BB = G.g11 * B1 * B1 + 2.0 * G.g13 * B1 * B3 + G.g22 * B2 * B2 + G.g33 * B3 * B3;
  const double SB = S1 * B1 + S2 * B2 + S3 * B3;
  if (D > 0.0) mlp_features(D, SS, tau, BB, SB, m.f + MLPF_MEAN, m.f + MLPF_ISTD, x);
}

}  // namespace grmhd
