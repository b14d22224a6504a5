/*
 * Oracle ghost fill of a two-level block mesh.  TEST INFRASTRUCTURE ONLY (see
 * orc.h).
 *
 * The paper evolves its meshblocks on Parthenon's block-structured adaptive
 * mesh (Sec. 1 and Sec. 3, the framework's refinement with prolongation and
 * restriction between levels).  It does not spell out the inter-level
 * operators, so this file states one reading and computes it directly, value
 * by value, from the block interiors:
 *
 *   - Levels 0 and 1; a level-l block covers global level-l cells
 *     [lloc, lloc + nx) of a domain of root_nx * 2^l cells.
 *   - Every ghost value is the value of the *composite view* at that level:
 *       same-level owner      -> copy of its interior value;
 *       coarser owner (prolongation into a fine ghost)
 *           cells : parent value plus monotonized-central limited slopes,
 *                   c + (s1 o1 + s2 o2 + s3 o3) / 4 with o = +-1 the child
 *                   octant; the slopes use the coarse view of the six
 *                   neighbours of the parent (a neighbour beyond a FIXED
 *                   boundary counts as the parent itself); a non-positive
 *                   density or internal energy falls back to the parent value;
 *           faces : a fine face lying on a coarse face takes its value, a fine
 *                   face inside a coarse cell the mean of the two coarse faces
 *                   bracketing it (constant across the face, linear along the
 *                   normal, so each fine ghost cell inherits the divergence of
 *                   its parent);
 *       finer owner (restriction into a coarse ghost)
 *           cells : mean of the 8 children;
 *           faces : mean of the 4 child faces (the densitized flux through the
 *                   coarse face).
 *   - Physical boundaries act first, at the level of the value asked for:
 *     periodic wrap, outflow copy with inflow velocity zeroed, polar mirror
 *     with the sign of the x2 velocity (and of the x2 face field) flipped.
 *   - A face belongs to the cell on its upper side (the cell below at the
 *     upper domain edge), except that where the two cells beside it lie on
 *     different levels the finer one owns it.
 *   - Each stage couples the levels conservatively (orc_mesh_correct): coarse
 *     hydro fluxes and EMFs on level boundaries are replaced by the means of
 *     the fine ones.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "orc.h"

typedef struct {
  int nb, ng;
  int root_nx[3];
  int bc[6];
  const int *level, *nx, *lloc;   /* [nb], [3 nb], [3 nb] */
} orc_mesh;

typedef struct {
  const orc_mesh *m;
  double **P, **Bf;
  int *own;                        /* owner block of each level-0 cell */
} ctx_t;

static int lvl_n(const orc_mesh *m, int l, int d) { return m->root_nx[d] << l; }

static size_t blk_ncell(const orc_mesh *m, int b)
{
  size_t c = 1;
  for (int d = 0; d < 3; ++d) c *= (size_t)(m->nx[3 * b + d] + 2 * m->ng);
  return c;
}

static size_t blk_idx(const orc_mesh *m, int b, const int loc[3])
{
  const int s0 = m->nx[3 * b] + 2 * m->ng, s1 = m->nx[3 * b + 1] + 2 * m->ng;
  return (size_t)loc[0] + (size_t)s0 * ((size_t)loc[1] + (size_t)s1 * (size_t)loc[2]);
}

/* Boundary map of global index g at level l along axis d.  Returns 0 if g is
   inside, 1 if mapped to *src, -1 beyond a FIXED boundary.  *flip: polar
   mirror; *ofl: 1 low / 2 high outflow. */
static int bmap(const orc_mesh *m, int l, int d, int g, int normal, int *src, int *flip,
                int *ofl)
{
  const int N = lvl_n(m, l, d), hi = normal ? N : N - 1;
  *flip = 0;
  *ofl = 0;
  if (g >= 0 && g <= hi) { *src = g; return 0; }
  const int low = g < 0;
  switch (m->bc[2 * d + (low ? 0 : 1)]) {
  case ORC_BC_PERIODIC:
    *src = ((g % N) + N) % N;
    return 1;
  case ORC_BC_OUTFLOW:
    *src = low ? 0 : hi;
    *ofl = low ? 1 : 2;
    return 1;
  case ORC_BC_POLAR:
    if (normal) *src = low ? -g : 2 * N - g;
    else        *src = low ? -1 - g : 2 * N - 1 - g;
    *flip = 1;
    return 1;
  default:
    return -1;
  }
}

static int owner(const ctx_t *c, int l, const int G[3])
{
  const orc_mesh *m = c->m;
  const int C[3] = {G[0] >> l, G[1] >> l, G[2] >> l};
  return c->own[C[0] + (size_t)m->root_nx[0] * (C[1] + (size_t)m->root_nx[1] * C[2])];
}

static void local_of(const orc_mesh *m, int b, const int G[3], int loc[3])
{
  for (int d = 0; d < 3; ++d) loc[d] = G[d] - m->lloc[3 * b + d] + m->ng;
}

static double mc_slope(double dm, double dp)
{
  if (dm * dp <= 0.0) return 0.0;
  const double a = fmin(fmin(2.0 * fabs(dm), 2.0 * fabs(dp)), 0.5 * fabs(dm + dp));
  return dm > 0.0 ? a : -a;
}

/* Primitive values of level-l cell G (any index); returns -1 beyond a FIXED
   boundary. */
static int cell_view(const ctx_t *c, int l, const int Gin[3], double v[5])
{
  const orc_mesh *m = c->m;
  int G[3], flip[3], ofl[3];
  for (int d = 0; d < 3; ++d)
    if (bmap(m, l, d, Gin[d], 0, &G[d], &flip[d], &ofl[d]) < 0) return -1;
  const int ob = owner(c, l, G), lo = m->level[ob];
  const size_t nc = blk_ncell(m, ob);
  if (lo == l) {
    int loc[3];
    local_of(m, ob, G, loc);
    const size_t q = blk_idx(m, ob, loc);
    for (int k = 0; k < 5; ++k) v[k] = c->P[ob][k * nc + q];
  } else if (lo < l) {                         /* prolongation from level l-1 */
    const int Pc[3] = {G[0] >> 1, G[1] >> 1, G[2] >> 1};
    double c0[5], s[3][5];
    cell_view(c, l - 1, Pc, c0);
    for (int d = 0; d < 3; ++d) {
      int Q[3] = {Pc[0], Pc[1], Pc[2]};
      double vm[5], vp[5];
      Q[d] = Pc[d] - 1;
      if (cell_view(c, l - 1, Q, vm) < 0) memcpy(vm, c0, sizeof vm);
      Q[d] = Pc[d] + 1;
      if (cell_view(c, l - 1, Q, vp) < 0) memcpy(vp, c0, sizeof vp);
      for (int k = 0; k < 5; ++k) s[d][k] = mc_slope(c0[k] - vm[k], vp[k] - c0[k]);
    }
    for (int k = 0; k < 5; ++k) {
      double sum = 0.0;
      for (int d = 0; d < 3; ++d) sum += (G[d] & 1) ? s[d][k] : -s[d][k];
      v[k] = c0[k] + 0.25 * sum;
    }
    if (!(v[0] > 0.0) || !isfinite(v[0])) v[0] = c0[0];
    if (!(v[4] > 0.0) || !isfinite(v[4])) v[4] = c0[4];
  } else {                                     /* restriction from level l+1 */
    double acc[5] = {0, 0, 0, 0, 0};
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const int Ch[3] = {2 * G[0] + dx, 2 * G[1] + dy, 2 * G[2] + dz};
          double w[5];
          cell_view(c, l + 1, Ch, w);
          for (int k = 0; k < 5; ++k) acc[k] += w[k];
        }
    for (int k = 0; k < 5; ++k) v[k] = 0.125 * acc[k];
  }
  for (int d = 0; d < 3; ++d) {
    if (ofl[d] == 1 && v[1 + d] > 0.0) v[1 + d] = 0.0;   /* no inflow */
    if (ofl[d] == 2 && v[1 + d] < 0.0) v[1 + d] = 0.0;
    if (flip[d]) v[1 + d] = -v[1 + d];
  }
  return 0;
}

/* Densitized field of component cmp on level-l face F (F[cmp] a face index,
   the others cell indices); returns -1 beyond a FIXED boundary. */
static int face_view(const ctx_t *c, int l, int cmp, const int Fin[3], double *v)
{
  const orc_mesh *m = c->m;
  int F[3], flip[3], ofl[3];
  for (int d = 0; d < 3; ++d)
    if (bmap(m, l, d, Fin[d], d == cmp, &F[d], &flip[d], &ofl[d]) < 0) return -1;
  /* owner: the cell above the face (below at the upper domain edge); where
     the two cells beside the face lie on different levels, the finer one */
  const int N = lvl_n(m, l, cmp);
  int Co[3] = {F[0], F[1], F[2]};
  if (Co[cmp] == N) Co[cmp] -= 1;
  int ob = owner(c, l, Co);
  {
    int Ca[3] = {F[0], F[1], F[2]}, alt = -1;
    const int per = m->bc[2 * cmp] == ORC_BC_PERIODIC;
    if (F[cmp] > 0 && F[cmp] < N) { Ca[cmp] = F[cmp] - 1; alt = F[cmp]; }
    else if (F[cmp] == N && per) { Ca[cmp] = 0; alt = 0; }
    else if (F[cmp] == 0 && per) { Ca[cmp] = N - 1; alt = N; }
    if (alt >= 0) {
      const int oa = owner(c, l, Ca);
      if (m->level[oa] > m->level[ob]) { ob = oa; F[cmp] = alt; }
    }
  }
  const int lo = m->level[ob];
  double val;
  if (lo == l) {
    int loc[3];
    local_of(m, ob, F, loc);
    val = c->Bf[ob][cmp * blk_ncell(m, ob) + blk_idx(m, ob, loc)];
  } else if (lo < l) {
    int Q[3] = {F[0] >> 1, F[1] >> 1, F[2] >> 1};
    if ((F[cmp] & 1) == 0) {
      Q[cmp] = F[cmp] / 2;
      face_view(c, l - 1, cmp, Q, &val);
    } else {
      double a, b;
      Q[cmp] = (F[cmp] - 1) / 2;
      face_view(c, l - 1, cmp, Q, &a);
      Q[cmp] = (F[cmp] + 1) / 2;
      face_view(c, l - 1, cmp, Q, &b);
      val = 0.5 * (a + b);
    }
  } else {
    const int t1 = (cmp + 1) % 3, t2 = (cmp + 2) % 3;
    double acc = 0.0;
    for (int e2 = 0; e2 < 2; ++e2)
      for (int e1 = 0; e1 < 2; ++e1) {
        int Ch[3];
        Ch[cmp] = 2 * F[cmp];
        Ch[t1] = 2 * F[t1] + e1;
        Ch[t2] = 2 * F[t2] + e2;
        double w;
        face_view(c, l + 1, cmp, Ch, &w);
        acc += w;
      }
    val = 0.25 * acc;
  }
  *v = flip[cmp] ? -val : val;
  return 0;
}

/* Fill every ghost cell and ghost face of every block.  Returns 0, or -1 if
   the blocks do not tile the domain. */
int orc_mesh_fill_ghosts(const orc_mesh *m, double **P, double **Bf)
{
  const size_t nroot = (size_t)m->root_nx[0] * m->root_nx[1] * m->root_nx[2];
  ctx_t c = {m, P, Bf, malloc(nroot * sizeof(int))};
  for (size_t q = 0; q < nroot; ++q) c.own[q] = -1;
  for (int b = 0; b < m->nb; ++b) {
    const int l = m->level[b];
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = m->lloc[3 * b + d] >> l;
      hi[d] = (m->lloc[3 * b + d] + m->nx[3 * b + d]) >> l;
    }
    for (int z = lo[2]; z < hi[2]; ++z)
      for (int y = lo[1]; y < hi[1]; ++y)
        for (int x = lo[0]; x < hi[0]; ++x) {
          int *o = &c.own[x + (size_t)m->root_nx[0] * (y + (size_t)m->root_nx[1] * z)];
          if (*o >= 0) { free(c.own); return -1; }
          *o = b;
        }
  }
  for (size_t q = 0; q < nroot; ++q)
    if (c.own[q] < 0) { free(c.own); return -1; }

  const int ng = m->ng;
#pragma omp parallel for schedule(dynamic)
  for (int b = 0; b < m->nb; ++b) {
    const int l = m->level[b];
    const int s[3] = {m->nx[3 * b] + 2 * ng, m->nx[3 * b + 1] + 2 * ng, m->nx[3 * b + 2] + 2 * ng};
    const size_t nc = blk_ncell(m, b);
    for (int cmp = -1; cmp < 3; ++cmp)
      for (int k = 0; k < s[2]; ++k)
        for (int j = 0; j < s[1]; ++j)
          for (int i = 0; i < s[0]; ++i) {
            const int loc[3] = {i, j, k};
            int ghost = 0, G[3];
            for (int d = 0; d < 3; ++d) {
              const int top = (cmp == d) ? ng + m->nx[3 * b + d] : ng + m->nx[3 * b + d] - 1;
              if (loc[d] < ng || loc[d] > top) ghost = 1;
              G[d] = m->lloc[3 * b + d] + loc[d] - ng;
            }
            if (!ghost) continue;
            const size_t q = blk_idx(m, b, loc);
            if (cmp < 0) {
              double v[5];
              if (cell_view(&c, l, G, v) < 0) continue;
              for (int k2 = 0; k2 < 5; ++k2) P[b][k2 * nc + q] = v[k2];
            } else {
              double v;
              if (face_view(&c, l, cmp, G, &v) < 0) continue;
              Bf[b][cmp * nc + q] = v;
            }
          }
  }
  free(c.own);
  return 0;
}

/*
 * Conservative coupling of the two levels for one stage (the framework's
 * flux correction and its constrained-transport counterpart, reading of the
 * refinement the paper builds on).  F[b]: face fluxes [3][8][ncell] and E[b]:
 * edge EMFs [3][ncell] of every block (orc_fluxes_emfs).  For each level-0
 * block:
 *   - a face on its boundary whose other side is a level-1 block takes, for
 *     the five hydro fluxes, the mean of the 4 child faces' fluxes of that
 *     block (the fine fluxes are authoritative);
 *   - an edge of its own that coincides with an edge of a level-1 block (two
 *     fine edges) takes the mean of the two fine EMFs; the first such fine
 *     block in block order supplies them.
 * Periodic boundaries are followed; other physical boundaries have no
 * neighbour.  Returns the number of corrected faces + edges.
 */
static int wrap_axis(const orc_mesh *m, int l, int d, int g, int *out)
{
  const int N = lvl_n(m, l, d);
  if (g >= 0 && g < N) { *out = g; return 1; }
  if (m->bc[2 * d] != ORC_BC_PERIODIC) return 0;
  *out = ((g % N) + N) % N;
  return 1;
}

/* does fine block f own the fine edge along e at cell ie, face indices (jf, kf)
   along (e+1)%3, (e+2)%3?  On success sets the local indices. */
static int owns_edge(const orc_mesh *m, int f, int e, int ie, int jf, int kf, int loc[3])
{
  const int a = (e + 1) % 3, b = (e + 2) % 3;
  const int *ll = &m->lloc[3 * f], *nx = &m->nx[3 * f];
  int cand[3][3], nc[3] = {0, 0, 0};
  const int want[3] = {ie, jf, kf}, ax[3] = {e, a, b};
  for (int q = 0; q < 3; ++q) {
    const int d = ax[q], N = lvl_n(m, 1, d);
    cand[q][nc[q]++] = want[q];
    if (m->bc[2 * d] == ORC_BC_PERIODIC) {
      if (q > 0 && want[q] == 0) cand[q][nc[q]++] = N;     /* face N is face 0 */
      if (q > 0 && want[q] == N) cand[q][nc[q]++] = 0;
    }
  }
  for (int x = 0; x < nc[0]; ++x)
    for (int y = 0; y < nc[1]; ++y)
      for (int z = 0; z < nc[2]; ++z) {
        const int v[3] = {cand[0][x], cand[1][y], cand[2][z]};
        int ok = 1, L[3];
        for (int q = 0; q < 3; ++q) {
          const int d = ax[q];
          const int lo = ll[d], hi = ll[d] + nx[d] - (q == 0 ? 1 : 0);
          if (v[q] < lo || v[q] > hi) ok = 0;
          L[d] = v[q] - ll[d] + m->ng;
        }
        if (ok) { loc[0] = L[0]; loc[1] = L[1]; loc[2] = L[2]; return 1; }
      }
  return 0;
}

int orc_mesh_correct(const orc_mesh *m, double **F, double **E)
{
  const size_t nroot = (size_t)m->root_nx[0] * m->root_nx[1] * m->root_nx[2];
  int *own = malloc(nroot * sizeof(int));
  for (size_t q = 0; q < nroot; ++q) own[q] = -1;
  for (int b = 0; b < m->nb; ++b) {
    const int l = m->level[b];
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = m->lloc[3 * b + d] >> l;
      hi[d] = (m->lloc[3 * b + d] + m->nx[3 * b + d]) >> l;
    }
    for (int z = lo[2]; z < hi[2]; ++z)
      for (int y = lo[1]; y < hi[1]; ++y)
        for (int x = lo[0]; x < hi[0]; ++x)
          own[x + (size_t)m->root_nx[0] * (y + (size_t)m->root_nx[1] * z)] = b;
  }
  const int ng = m->ng;
  int count = 0;
  for (int c = 0; c < m->nb; ++c) {
    if (m->level[c] != 0) continue;
    const int *ll = &m->lloc[3 * c], *nx = &m->nx[3 * c];
    const size_t ncC = blk_ncell(m, c);
    /* faces on the block boundary */
    for (int d = 0; d < 3; ++d) {
      const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
      for (int side = 0; side < 2; ++side) {
        const int fl = side ? ng + nx[d] : ng;             /* local face index */
        const int other = side ? ll[d] + nx[d] : ll[d] - 1; /* level-0 cell across */
        int oc;
        if (!wrap_axis(m, 0, d, other, &oc)) continue;
        for (int u2 = 0; u2 < nx[t2]; ++u2)
          for (int u1 = 0; u1 < nx[t1]; ++u1) {
            int C0[3];
            C0[d] = oc; C0[t1] = ll[t1] + u1; C0[t2] = ll[t2] + u2;
            const int f = own[C0[0] + (size_t)m->root_nx[0] * (C0[1] + (size_t)m->root_nx[1] * C0[2])];
            if (m->level[f] != 1) continue;
            /* the interface plane seen from the fine block: its face across */
            int X[3];
            X[d] = side ? 2 * oc : 2 * (oc + 1);
            X[t1] = 2 * C0[t1]; X[t2] = 2 * C0[t2];
            int Lf[3];
            for (int q = 0; q < 3; ++q) Lf[q] = X[q] - m->lloc[3 * f + q] + ng;
            const size_t ncF = blk_ncell(m, f);
            const int s0 = m->nx[3 * f] + 2 * ng, s1 = m->nx[3 * f + 1] + 2 * ng;
            const size_t str[3] = {1, (size_t)s0, (size_t)s0 * s1};
            const size_t src = blk_idx(m, f, Lf);
            int Lc[3];
            Lc[d] = fl; Lc[t1] = ng + u1; Lc[t2] = ng + u2;
            const size_t dst = blk_idx(m, c, Lc);
            for (int v = 0; v < 5; ++v) {
              const double *Ff = F[f] + ((size_t)d * 8 + v) * ncF;
              double acc = 0.0;
              for (int bb = 0; bb < 2; ++bb)
                for (int aa = 0; aa < 2; ++aa) acc += Ff[src + aa * str[t1] + bb * str[t2]];
              F[c][((size_t)d * 8 + v) * ncC + dst] = 0.25 * acc;
            }
            ++count;
          }
      }
    }
    /* own edges on the block surface */
    for (int e = 0; e < 3; ++e) {
      const int a = (e + 1) % 3, bx = (e + 2) % 3;
      for (int kb = 0; kb <= nx[bx]; ++kb)
        for (int ka = 0; ka <= nx[a]; ++ka) {
          if (!(ka == 0 || ka == nx[a] || kb == 0 || kb == nx[bx])) continue;
          for (int ie = 0; ie < nx[e]; ++ie) {
            /* (complex.h owns the name I) */
            const int fe = 2 * (ll[e] + ie), fa = 2 * (ll[a] + ka), fb = 2 * (ll[bx] + kb);
            int f = -1, loc[3];
            for (int q = 0; q < m->nb && f < 0; ++q)
              if (m->level[q] == 1 && owns_edge(m, q, e, fe, fa, fb, loc)) f = q;
            if (f < 0) continue;
            const int s0 = m->nx[3 * f] + 2 * ng, s1 = m->nx[3 * f + 1] + 2 * ng;
            const size_t str[3] = {1, (size_t)s0, (size_t)s0 * s1};
            const size_t ncF = blk_ncell(m, f);
            const size_t sa = blk_idx(m, f, loc);
            const double *Ef = E[f] + (size_t)e * ncF;
            int Lc[3];
            Lc[e] = ng + ie; Lc[a] = ng + ka; Lc[bx] = ng + kb;
            E[c][(size_t)e * ncC + blk_idx(m, c, Lc)] = 0.5 * (Ef[sa] + Ef[sa + str[e]]);
            ++count;
          }
        }
    }
  }
  free(own);
  return count;
}
