// Refinement of the two-level block mesh on gfx950: tagging, and the remap of
// a state from one block layout onto another (blocks copied, refined or
// derefined).  Included once, by grmhd.hip (after kernels.h).
//
// Refined cells: P by parent + monotonized-central slopes toward the
// child's octant (from its filled ghosts; a non-positive rho or u keeps the
// parent value), then U = U(P, B) of each child with the new face field,
// plus the parent's U minus the children's mean (the same for all 8), so the
// totals are kept and each child's U matches its field's energy and
// momentum.
// Refined faces: on a coarse face the fine faces copy the fine neighbour's
// where an existing fine block lies across, else the coarse value; the 12
// faces inside a coarse cell start from the mean of the two outer faces
// along their normal and take the smallest correction (least squares) that
// makes all 8 children divergence-free.  Derefined cells and faces: means of
// the 8 children and of the 4 fine faces.
#pragma once
#include "kernels.h"

namespace grmhd {

// op 0 copy, 1 prolong, 2 restrict; inb (prolongation): bit 2d / 2d+1 set =
// the lower / upper neighbour of the parent along d is an interior cell of
// the source block (U is read there; P, whose ghosts are filled, always)
struct RemapC { long long dst, src; int op, oct, sj, sk, inb, pad; };
struct RemapF { long long dst, src, st1, st2; int comp, op; }; // op 0 copy, 1 mean of 4 faces
struct RemapP { long long dst0, src; int sj, sk; };           // refined parent: child (0,0,0), source cell

struct RemapArgs {
  const double *sP, *sU, *sBf;
  double *dP, *dU, *dBf;
  long long snct, dnct;
};

// Per-chunk maximum of the refinement indicator of P[var]: max over the three
// directions of |q(+1) - q(-1)| / (2 |q|) (a relative first difference; the
// directions with one cell are skipped).
__global__ __launch_bounds__(256) void k_tag(KArgs a, const int2 *__restrict__ chunks, int var,
                                             double *__restrict__ out)
{
  __shared__ double sh[4];
  const int2 ch = chunks[blockIdx.x];
  const BlockInfo b = a.blocks[ch.x];
  const int e = ch.y + threadIdx.x;
  double v = 0.0;
  if (e < b.n[0] * b.n[1] * b.n[2]) {
    const int ng = a.ng;
    const int i = ng + e % b.n[0], j = ng + (e / b.n[0]) % b.n[1], k = ng + e / (b.n[0] * b.n[1]);
    const long long sj = b.s[0], sk = (long long)b.s[0] * b.s[1];
    const long long c = b.off + i + sj * j + sk * k;
    const double *q = a.P + (long long)var * a.nct;
    const double den = 2.0 * fabs(q[c]) + 1e-300;
    const long long st[3] = {1, sj, sk};
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (a.active[d]) v = fmax(v, fabs(q[c + st[d]] - q[c - st[d]]) / den);
  }
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

__global__ __launch_bounds__(256) void k_remap_cells(RemapArgs r, const RemapC *__restrict__ map,
                                                     int n)
{
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const RemapC m = map[e];
  const long long st[3] = {1, m.sj, m.sk};
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const double *sp = r.sP + q * r.snct, *su = r.sU + q * r.snct;
    double vp, vu;
    if (m.op == 0) {
      vp = sp[m.src];
      vu = su[m.src];
    } else if (m.op == 2) {
      double ap = 0.0, au = 0.0;
      for (int z = 0; z < 2; ++z)
        for (int y = 0; y < 2; ++y)
          for (int x = 0; x < 2; ++x) {
            const long long o = m.src + x + y * (long long)m.sj + z * (long long)m.sk;
            ap += sp[o];
            au += su[o];
          }
      vp = 0.125 * ap;
      vu = 0.125 * au;
    } else {
      const double p0 = sp[m.src], u0 = su[m.src];
      double sump = 0.0, sumu = 0.0, absu = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double slp = mc_lim(p0 - sp[m.src - st[d]], sp[m.src + st[d]] - p0);
        const double ul = ((m.inb >> (2 * d)) & 1) ? su[m.src - st[d]] : u0;
        const double uh = ((m.inb >> (2 * d + 1)) & 1) ? su[m.src + st[d]] : u0;
        const double slu = mc_lim(u0 - ul, uh - u0);
        const bool up = (m.oct >> d) & 1;
        sump += up ? slp : -slp;
        sumu += up ? slu : -slu;
        absu += fabs(slu);
      }
      vp = p0 + 0.25 * sump;
      if ((q == 0 || q == 4) && (!(vp > 0.0) || !isfinite(vp))) vp = p0;
      // the smallest child is u0 - |s|_1 / 4: keep every child positive
      vu = ((q == 0 || q == 4) && !(u0 - 0.25 * absu > 0.0)) ? u0 : u0 + 0.25 * sumu;
    }
    r.dP[q * r.dnct + m.dst] = vp;
    if (m.op != 1) r.dU[q * r.dnct + m.dst] = vu;
  }
}

// Refined cells: U = U(P) of each child (computed by k_p2c) plus the
// parent's excess over the children's mean, so that the 8 children keep the
// parent's conserved content.
__global__ __launch_bounds__(256) void k_remap_cons(RemapArgs r, const RemapP *__restrict__ map,
                                                    int n)
{
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const RemapP m = map[e];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    double *u = r.dU + q * r.dnct + m.dst0;
    double acc = 0.0;
    for (int z = 0; z < 2; ++z)
      for (int y = 0; y < 2; ++y)
        for (int x = 0; x < 2; ++x) acc += u[x + y * (long long)m.sj + z * (long long)m.sk];
    const double dlt = r.sU[q * r.snct + m.src] - 0.125 * acc;
    for (int z = 0; z < 2; ++z)
      for (int y = 0; y < 2; ++y)
        for (int x = 0; x < 2; ++x) u[x + y * (long long)m.sj + z * (long long)m.sk] += dlt;
  }
}

__global__ __launch_bounds__(256) void k_remap_faces(RemapArgs r, const RemapF *__restrict__ map,
                                                     int n)
{
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const RemapF m = map[e];
  const double *s = r.sBf + m.comp * r.snct + m.src;
  double v;
  if (m.op == 0) {
    v = s[0];
  } else {
    double acc = 0.0;
    for (int t2 = 0; t2 < 2; ++t2)
      for (int t1 = 0; t1 < 2; ++t1) acc += s[t1 * m.st1 + t2 * m.st2];
    v = 0.25 * acc;
  }
  r.dBf[m.comp * r.dnct + m.dst] = v;
}

// The 12 faces inside each refined parent from its 24 outer fine faces
// (already in place): x = x0 + M (-div(x0)), M = D^T (D D^T + 1 1^T)^-1 the
// minimum-norm solution operator of the 8 children's divergence constraints
// (12 x 8, row-major).  Unknown order: x faces (b, c) -> b + 2c, y faces
// (a, c) -> 4 + a + 2c, z faces (a, b) -> 8 + a + 2b; child (a, b, c) ->
// a + 2b + 4c.
__global__ __launch_bounds__(256) void k_remap_div(RemapArgs r, const RemapP *__restrict__ map,
                                                   int n, const double *__restrict__ M, double idx,
                                                   double idy, double idz)
{
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const RemapP m = map[e];
  const long long sj = m.sj, sk = m.sk, N = r.dnct;
  double *Bx = r.dBf, *By = r.dBf + N, *Bz = r.dBf + 2 * N;
  auto at = [&](int a, int b, int c) { return m.dst0 + a + b * sj + c * sk; };
  double x[12];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b) x[b + 2 * c] = 0.5 * (Bx[at(0, b, c)] + Bx[at(2, b, c)]);
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int a = 0; a < 2; ++a) x[4 + a + 2 * c] = 0.5 * (By[at(a, 0, c)] + By[at(a, 2, c)]);
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a) x[8 + a + 2 * b] = 0.5 * (Bz[at(a, b, 0)] + Bz[at(a, b, 2)]);
  double rhs[8];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const double xl = a ? x[b + 2 * c] : Bx[at(0, b, c)];
        const double xh = a ? Bx[at(2, b, c)] : x[b + 2 * c];
        const double yl = b ? x[4 + a + 2 * c] : By[at(a, 0, c)];
        const double yh = b ? By[at(a, 2, c)] : x[4 + a + 2 * c];
        const double zl = c ? x[8 + a + 2 * b] : Bz[at(a, b, 0)];
        const double zh = c ? Bz[at(a, b, 2)] : x[8 + a + 2 * b];
        rhs[a + 2 * b + 4 * c] = -((xh - xl) * idx + (yh - yl) * idy + (zh - zl) * idz);
      }
  double y[12];
#pragma unroll
  for (int u = 0; u < 12; ++u) {
    double s = x[u];
#pragma unroll
    for (int v = 0; v < 8; ++v) s += M[u * 8 + v] * rhs[v];
    y[u] = s;
  }
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b) Bx[at(1, b, c)] = y[b + 2 * c];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int a = 0; a < 2; ++a) By[at(a, 1, c)] = y[4 + a + 2 * c];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a) Bz[at(a, b, 1)] = y[8 + a + 2 * b];
}

}  // namespace grmhd
