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
 *     upper domain edge).
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
  int Co[3] = {F[0], F[1], F[2]};
  if (Co[cmp] == lvl_n(m, l, cmp)) Co[cmp] -= 1;
  const int ob = owner(c, l, Co), lo = m->level[ob];
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
