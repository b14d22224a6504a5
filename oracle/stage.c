/*
 * Oracle block driver: ghost fill, one Runge-Kutta stage, con2prim with
 * floors, reductions.  TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * Stage (Sec. 2.1 conservation law, Sec. 3.1 second-order finite volumes):
 *   dU/dt = -sum_d [Fd(i+1/2) - Fd(i-1/2)]/dx_d + sqrt(-g) S
 *   Uout  = c0 U0 + c1 U + cdt dt dU/dt
 * with face fluxes from reconstruction + LLF/HLL, and face-centred
 * sqrt(gamma) B^k advanced by constrained transport: each edge EMF is the
 * four-point average of the induction fluxes of the faces sharing the edge
 * (Omega_{ik} = sqrt(-g) F^i(B^k) is antisymmetric in i,k), and
 *   d_t B1 = d_2 E3 - d_3 E2,  d_t B2 = -d_1 E3 + d_3 E1,  d_t B3 = d_1 E2 - d_2 E1,
 * with E1 = Omega_23, E2 = Omega_31, E3 = Omega_12.
 * Sources (Sec. 2.1 source vector with G_nu = 0):
 *   S_j   = (1/2) T^{mu nu} d_j g_{mu nu}   (equal to the paper's
 *           T^{mu nu}(g_{nu j,mu} - Gamma^d_{nu mu} g_{dj}) for symmetric T)
 *   S_tau = alpha (T^{mu 0} d_mu ln alpha - T^{mu nu} Gamma^0_{nu mu}).
 * Floors (Sec. 3.2): rho >= rho0 r^-a, u >= u0 r^-b, W <= W_max, then the
 * hydro conserved variables are recomputed from the floored primitives.  With
 * a tabulated EOS the floors never go below the table (rho within its range,
 * eps = u/rho within its range, Y_e within its range).
 * Passive scalar (nscalar = 1): P[5] = Y_e, U[5] = sqrt(gamma) D Y_e, no
 * source; its face flux sits in the slot 5 + d of the direction-d block.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#include "orc.h"

#define S1(g) ((g)->n[0] + 2 * (g)->ng)
#define S2(g) ((g)->n[1] + 2 * (g)->ng)
#define S3(g) ((g)->n[2] + 2 * (g)->ng)

static size_t ncell(const orc_grid *g) { return (size_t)S1(g) * S2(g) * S3(g); }
static size_t IDX(const orc_grid *g, int i, int j, int k)
{
  return (size_t)i + (size_t)S1(g) * ((size_t)j + (size_t)S2(g) * (size_t)k);
}

int orc_version(void) { return 1; }

/* ---------------------------------------------------------------- ghosts */

/*
 * Map one index along axis d to its source.  Returns 0 if the index is not a
 * ghost along d, 1 if it maps to *src, -1 if the boundary is FIXED (leave).
 * normal = the variable lives on d-faces.  *flip = 1 for a polar mirror.
 */
static int map_axis(const orc_grid *g, int d, int idx, int normal, int *src, int *flip,
                    int *side)
{
  const int ng = g->ng, n = g->n[d];
  const int lo = ng, hi = normal ? ng + n : ng + n - 1;   /* inclusive interior */
  *flip = 0;
  if (idx >= lo && idx <= hi) { *src = idx; *side = 0; return 0; }
  const int low = idx < lo;
  const int bc = g->bc[2 * d + (low ? 0 : 1)];
  *side = low ? -1 : 1;
  switch (bc) {
  case ORC_BC_PERIODIC:
    /* wrap modulo n: a direction thinner than the ghost depth still maps
       every ghost to an interior cell (face n is face 0) */
    *src = ng + (((idx - ng) % n) + n) % n;
    return 1;
  case ORC_BC_OUTFLOW:
    *src = low ? lo : hi;
    return 1;
  case ORC_BC_POLAR:
    if (normal) *src = low ? 2 * lo - idx : 2 * (ng + n) - idx;
    else        *src = low ? 2 * lo - 1 - idx : 2 * (ng + n) - 1 - idx;
    *flip = 1;
    return 1;
  default:
    return -1;
  }
}

void orc_fill_ghosts_n(const orc_grid *g, const orc_metric *m, int nv, double *P, double *Bf)
{
  (void)m;
  const size_t nc = ncell(g);
  /* cell-centred primitives */
  for (int k = 0; k < S3(g); ++k)
    for (int j = 0; j < S2(g); ++j)
      for (int i = 0; i < S1(g); ++i) {
        int idx[3] = {i, j, k}, src[3], flip[3], side[3], any = 0, fixed = 0;
        for (int d = 0; d < 3; ++d) {
          int r = map_axis(g, d, idx[d], 0, &src[d], &flip[d], &side[d]);
          if (r < 0) fixed = 1;
          if (r != 0) any = 1;
        }
        if (!any || fixed) continue;
        const size_t s = IDX(g, src[0], src[1], src[2]), t = IDX(g, i, j, k);
        double v[6];
        for (int q = 0; q < nv; ++q) v[q] = P[q * nc + s];
        for (int d = 0; d < 3; ++d) {
          if (side[d] == 0) continue;
          const int bc = g->bc[2 * d + (side[d] < 0 ? 0 : 1)];
          if (bc == ORC_BC_OUTFLOW) {
            /* no inflow through an outflow boundary */
            if (side[d] < 0 && v[1 + d] > 0.0) v[1 + d] = 0.0;
            if (side[d] > 0 && v[1 + d] < 0.0) v[1 + d] = 0.0;
          }
          if (flip[d]) v[1 + d] = -v[1 + d];
        }
        for (int q = 0; q < nv; ++q) P[q * nc + t] = v[q];
      }
  /* face-centred densitized field */
  for (int c = 0; c < 3; ++c)
    for (int k = 0; k < S3(g); ++k)
      for (int j = 0; j < S2(g); ++j)
        for (int i = 0; i < S1(g); ++i) {
          int idx[3] = {i, j, k}, src[3], flip[3], side[3], any = 0, fixed = 0;
          for (int d = 0; d < 3; ++d) {
            int r = map_axis(g, d, idx[d], d == c, &src[d], &flip[d], &side[d]);
            if (r < 0) fixed = 1;
            if (r != 0) any = 1;
          }
          if (!any || fixed) continue;
          double v = Bf[c * nc + IDX(g, src[0], src[1], src[2])];
          if (flip[c]) v = -v;   /* normal component reverses across the pole */
          Bf[c * nc + IDX(g, i, j, k)] = v;
        }
}

void orc_fill_ghosts(const orc_grid *g, const orc_metric *m, double *P, double *Bf)
{
  orc_fill_ghosts_n(g, m, 5, P, Bf);
}

/* Cell-centred undensitized B^i = (Bf_lo + Bf_hi) / (2 sqrt(gamma)). */
void orc_cell_B(const orc_grid *g, const orc_metric *m, const double *Bf, double *Bcc)
{
  const size_t nc = ncell(g);
  memset(Bcc, 0, 3 * nc * sizeof(double));
  for (int k = 0; k < S3(g) - 1; ++k)
    for (int j = 0; j < S2(g) - 1; ++j)
      for (int i = 0; i < S1(g) - 1; ++i) {
        double x[3];
        orc_geom G;
        orc_coord(g, m, ORC_LOC_CENTER, i, j, k, x);
        orc_geom_at(m, x, &G);
        const size_t c = IDX(g, i, j, k);
        const size_t up[3] = {IDX(g, i + 1, j, k), IDX(g, i, j + 1, k), IDX(g, i, j, k + 1)};
        for (int d = 0; d < 3; ++d)
          Bcc[d * nc + c] = 0.5 * (Bf[d * nc + c] + Bf[d * nc + up[d]]) / G.sqrtgam;
      }
}

static void load_prim(const orc_grid *g, const orc_eos *e, const double *P, const double *Bcc,
                      size_t c, orc_prim *q)
{
  const size_t nc = ncell(g);
  q->rho = P[c];
  for (int i = 0; i < 3; ++i) q->ut[i] = P[(1 + i) * nc + c];
  q->u = P[4 * nc + c];
  for (int i = 0; i < 3; ++i) q->B[i] = Bcc[i * nc + c];
  q->ye = e->nscalar ? P[5 * nc + c] : 0.0;
}

/* The conserved planes of a cell from the undensitized vector of 9. */
static void store_cons(const orc_eos *e, double *U, size_t nc, size_t c, double sg,
                       const double Uc[9])
{
  for (int v = 0; v < 5; ++v) U[(size_t)v * nc + c] = sg * Uc[v];
  if (e->nscalar) U[5 * nc + c] = sg * Uc[8];
}

void orc_prim_to_cons_grid(const orc_grid *g, const orc_metric *m, const orc_eos *e,
                           const double *P, const double *Bf, double *U)
{
  const size_t nc = ncell(g);
  double *Bcc = malloc(3 * nc * sizeof(double));
  orc_cell_B(g, m, Bf, Bcc);
  for (int k = g->ng; k < g->ng + g->n[2]; ++k)
    for (int j = g->ng; j < g->ng + g->n[1]; ++j)
      for (int i = g->ng; i < g->ng + g->n[0]; ++i) {
        double x[3], Uc[9];
        orc_geom G;
        orc_prim q;
        orc_coord(g, m, ORC_LOC_CENTER, i, j, k, x);
        orc_geom_at(m, x, &G);
        const size_t c = IDX(g, i, j, k);
        load_prim(g, e, P, Bcc, c, &q);
        orc_prim_to_cons(&G, e, &q, Uc);
        store_cons(e, U, nc, c, G.sqrtgam, Uc);
      }
  free(Bcc);
}

/* ----------------------------------------------------------------- stage */

static int is_pole_face(const orc_grid *g, int d, int j)
{
  if (d != 1) return 0;
  if (g->bc[2] == ORC_BC_POLAR && j == g->ng) return 1;
  if (g->bc[3] == ORC_BC_POLAR && j == g->ng + g->n[1]) return 1;
  return 0;
}

/* Reconstruct the 5 hydro primitives, the 2 transverse B and (nscalar) Y_e
   of cell c along d; entry 8 is Y_e. */
static void recon_cell(const orc_grid *g, int ns, const double *P, const double *Bcc, int d,
                       int i, int j, int k, double lo[9], double hi[9])
{
  const size_t nc = ncell(g);
  const size_t stride = (d == 0) ? 1 : (d == 1) ? (size_t)S1(g) : (size_t)S1(g) * S2(g);
  const size_t c = IDX(g, i, j, k);
  lo[8] = hi[8] = 0.0;
  for (int q = 0; q < 8 + ns; ++q) {
    if (q >= 5 && q < 8 && q - 5 == d) { lo[q] = hi[q] = 0.0; continue; }
    const double *arr = (q < 5) ? P + (size_t)q * nc
                      : (q < 8) ? Bcc + (size_t)(q - 5) * nc : P + 5 * nc;
    double f[5];
    for (int s = -2; s <= 2; ++s) f[s + 2] = arr[c + s * (ptrdiff_t)stride];
    orc_recon1(g->recon, g->weno_fv, f, &lo[q], &hi[q]);
    if (q == 0 || q == 4) {
      /* positivity: fall back to the cell value for a non-positive face */
      if (!(lo[q] > 0.0) || !isfinite(lo[q])) lo[q] = f[2];
      if (!(hi[q] > 0.0) || !isfinite(hi[q])) hi[q] = f[2];
    }
  }
}

static void face_fluxes(const orc_grid *g, const orc_metric *m, const orc_eos *e,
                        const double *P, const double *Bf, const double *Bcc, int d,
                        double *F, int nthreads)
{
  const size_t nc = ncell(g);
  int lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = (a == d) ? g->ng : g->ng - 1;
    hi[a] = g->ng + g->n[a];            /* inclusive */
  }
  #pragma omp parallel for schedule(dynamic) num_threads(nthreads)
  for (int k = lo[2]; k <= hi[2]; ++k)
    for (int j = lo[1]; j <= hi[1]; ++j)
      for (int i = lo[0]; i <= hi[0]; ++i) {
        const size_t f = IDX(g, i, j, k);
        double fl[9];
        if (is_pole_face(g, d, j)) {
          for (int v = 0; v < 8; ++v) F[(size_t)v * nc + f] = 0.0;
          continue;
        }
        int im = i - (d == 0), jm = j - (d == 1), km = k - (d == 2);
        double lL[9], hL[9], lR[9], hR[9];
        recon_cell(g, e->nscalar, P, Bcc, d, im, jm, km, lL, hL);   /* left cell  */
        recon_cell(g, e->nscalar, P, Bcc, d, i, j, k, lR, hR);      /* right cell */
        double x[3];
        orc_geom G;
        orc_coord(g, m, ORC_LOC_FACE1 + d, i, j, k, x);
        orc_geom_at(m, x, &G);
        orc_prim L, R;
        L.rho = hL[0]; R.rho = lR[0];
        for (int a = 0; a < 3; ++a) { L.ut[a] = hL[1 + a]; R.ut[a] = lR[1 + a]; }
        L.u = hL[4]; R.u = lR[4];
        L.ye = hL[8]; R.ye = lR[8];
        for (int a = 0; a < 3; ++a) {
          if (a == d) {
            L.B[a] = R.B[a] = Bf[(size_t)d * nc + f] / G.sqrtgam;
          } else {
            L.B[a] = hL[5 + a]; R.B[a] = lR[5 + a];
          }
        }
        orc_riemann(&G, e, g->riemann, &L, &R, d, fl);
        for (int v = 0; v < 8; ++v) F[(size_t)v * nc + f] = fl[v];
        if (e->nscalar) F[(size_t)(5 + d) * nc + f] = fl[8];   /* normal-field slot */
      }
}

/*
 * One stage.  P, Bf: the state L is evaluated on.  U0/Bf0, U: RK operands.
 * Outputs Uout/Bfout (complete copies of U/Bf with updated entries).
 * flux_out (optional) receives F[3][8][ncell].
 */
/* Face fluxes F[3][8][ncell] and edge EMFs E[3][ncell] of the state (P, Bf):
   E1 at (i, j-1/2, k-1/2), E2 at (i-1/2, j, k-1/2), E3 at (i-1/2, j-1/2, k)
   for every (i, j, k) in the box [ng, ng+n] (four-point averages of the
   induction fluxes).  Both arrays are zeroed first. */
static void emfs_from_fluxes(const orc_grid *g, const double *F, double *E);

int orc_fluxes_emfs(const orc_grid *g, const orc_metric *m, const orc_eos *e,
                    const double *P, const double *Bf, double *F, double *E, int nthreads)
{
  const size_t nc = ncell(g);
  double *Bcc = malloc(3 * nc * sizeof(double));
  if (!Bcc) return -1;
  memset(F, 0, 24 * nc * sizeof(double));
  orc_cell_B(g, m, Bf, Bcc);
  for (int d = 0; d < 3; ++d) face_fluxes(g, m, e, P, Bf, Bcc, d, F + (size_t)d * 8 * nc, nthreads);
  emfs_from_fluxes(g, F, E);
  free(Bcc);
  return 0;
}

static void emfs_from_fluxes(const orc_grid *g, const double *F, double *E)
{
  const size_t nc = ncell(g);
  const int ng = g->ng;
  const double *F1 = F, *F2 = F + 8 * nc, *F3 = F + 16 * nc;
  memset(E, 0, 3 * nc * sizeof(double));
#define FL(Fd, v, i, j, k) (Fd)[(size_t)(v) * nc + IDX(g, i, j, k)]
  for (int k = ng; k <= ng + g->n[2]; ++k)
    for (int j = ng; j <= ng + g->n[1]; ++j)
      for (int i = ng; i <= ng + g->n[0]; ++i) {
        const size_t c = IDX(g, i, j, k);
        E[0 * nc + c] = 0.25 * (FL(F2, 7, i, j, k) + FL(F2, 7, i, j, k - 1)
                              - FL(F3, 6, i, j, k) - FL(F3, 6, i, j - 1, k));
        E[1 * nc + c] = 0.25 * (FL(F3, 5, i, j, k) + FL(F3, 5, i - 1, j, k)
                              - FL(F1, 7, i, j, k) - FL(F1, 7, i, j, k - 1));
        E[2 * nc + c] = 0.25 * (FL(F1, 6, i, j, k) + FL(F1, 6, i, j - 1, k)
                              - FL(F2, 5, i, j, k) - FL(F2, 5, i - 1, j, k));
      }
#undef FL
}

/*
 * One stage from given face fluxes F and edge EMFs E (as orc_fluxes_emfs
 * returns them, possibly corrected at level boundaries): the face field by
 * the discrete curl of E, the hydro state by the flux divergence and the
 * geometric source of (P, Bf).
 */
int orc_stage_from(const orc_grid *g, const orc_metric *m, const orc_eos *e,
                   const double *P, const double *Bf, const double *U0, const double *Bf0,
                   const double *U, double dt, const double rk[3], const double *F,
                   const double *E, double *Uout, double *Bfout, int nthreads);

int orc_stage(const orc_grid *g, const orc_metric *m, const orc_eos *e,
              const double *P, const double *Bf, const double *U0, const double *Bf0,
              const double *U, double dt, const double rk[3], double *Uout,
              double *Bfout, double *flux_out, int nthreads)
{
  const size_t nc = ncell(g);
  double *F = flux_out ? flux_out : malloc(24 * nc * sizeof(double));
  double *E = malloc(3 * nc * sizeof(double));
  if (!F || !E) return -1;
  int r = orc_fluxes_emfs(g, m, e, P, Bf, F, E, nthreads);
  if (!r) r = orc_stage_from(g, m, e, P, Bf, U0, Bf0, U, dt, rk, F, E, Uout, Bfout, nthreads);
  free(E);
  if (!flux_out) free(F);
  return r;
}

int orc_stage_from(const orc_grid *g, const orc_metric *m, const orc_eos *e,
                   const double *P, const double *Bf, const double *U0, const double *Bf0,
                   const double *U, double dt, const double rk[3], const double *F,
                   const double *E, double *Uout, double *Bfout, int nthreads)
{
  const size_t nc = ncell(g);
  const int ng = g->ng;
  double *Bcc = malloc(3 * nc * sizeof(double));
  if (!Bcc) return -1;
  orc_cell_B(g, m, Bf, Bcc);
  const double *F1 = F, *F2 = F + 8 * nc, *F3 = F + 16 * nc;
#define FL(Fd, v, i, j, k) (Fd)[(size_t)(v) * nc + IDX(g, i, j, k)]
#define EE(a, i, j, k) E[(size_t)(a) * nc + IDX(g, i, j, k)]

  const int nv = 5 + e->nscalar;
  memcpy(Uout, U, (size_t)nv * nc * sizeof(double));
  memcpy(Bfout, Bf, 3 * nc * sizeof(double));
  const double c0 = rk[0], c1 = rk[1], cdt = rk[2] * dt;
  const double dx1 = g->dx[0], dx2 = g->dx[1], dx3 = g->dx[2];

  /* face field */
  for (int k = ng; k <= ng + g->n[2]; ++k)
    for (int j = ng; j <= ng + g->n[1]; ++j)
      for (int i = ng; i <= ng + g->n[0]; ++i) {
        const size_t c = IDX(g, i, j, k);
        const int in1 = i < ng + g->n[0], in2 = j < ng + g->n[1], in3 = k < ng + g->n[2];
        if (in2 && in3) {
          double r = (EE(2, i, j + 1, k) - EE(2, i, j, k)) / dx2
                   - (EE(1, i, j, k + 1) - EE(1, i, j, k)) / dx3;
          Bfout[0 * nc + c] = c0 * Bf0[0 * nc + c] + c1 * Bf[0 * nc + c] + cdt * r;
        }
        if (in1 && in3) {
          double r = -(EE(2, i + 1, j, k) - EE(2, i, j, k)) / dx1
                   + (EE(0, i, j, k + 1) - EE(0, i, j, k)) / dx3;
          Bfout[1 * nc + c] = c0 * Bf0[1 * nc + c] + c1 * Bf[1 * nc + c] + cdt * r;
        }
        if (in1 && in2) {
          double r = (EE(1, i + 1, j, k) - EE(1, i, j, k)) / dx1
                   - (EE(0, i, j + 1, k) - EE(0, i, j, k)) / dx2;
          Bfout[2 * nc + c] = c0 * Bf0[2 * nc + c] + c1 * Bf[2 * nc + c] + cdt * r;
        }
      }

  /* hydro: flux divergence + geometric source */
  #pragma omp parallel for schedule(dynamic) num_threads(nthreads)
  for (int k = ng; k < ng + g->n[2]; ++k)
    for (int j = ng; j < ng + g->n[1]; ++j)
      for (int i = ng; i < ng + g->n[0]; ++i) {
        const size_t c = IDX(g, i, j, k);
        double rhs[6];
        for (int v = 0; v < 5; ++v)
          rhs[v] = -(FL(F1, v, i + 1, j, k) - FL(F1, v, i, j, k)) / dx1
                   - (FL(F2, v, i, j + 1, k) - FL(F2, v, i, j, k)) / dx2
                   - (FL(F3, v, i, j, k + 1) - FL(F3, v, i, j, k)) / dx3;
        if (nv > 5)   /* scalar fluxes in the normal-field slots 5, 6, 7 */
          rhs[5] = -(FL(F1, 5, i + 1, j, k) - FL(F1, 5, i, j, k)) / dx1
                   - (FL(F2, 6, i, j + 1, k) - FL(F2, 6, i, j, k)) / dx2
                   - (FL(F3, 7, i, j, k + 1) - FL(F3, 7, i, j, k)) / dx3;
        if (m->kind != ORC_MINKOWSKI) {
          double x[3], dg[4][4][4], Gam[4][4][4], dla[4], T[4][4];
          orc_geom G;
          orc_prim q;
          orc_coord(g, m, ORC_LOC_CENTER, i, j, k, x);
          orc_geom_at(m, x, &G);
          orc_metric_derivs(m, x, dg, Gam, dla);
          load_prim(g, e, P, Bcc, c, &q);
          orc_tmunu(&G, e, &q, T);
          for (int jj = 1; jj <= 3; ++jj) {
            double s = 0.0;
            for (int a = 0; a < 4; ++a)
              for (int b = 0; b < 4; ++b) s += T[a][b] * dg[jj][a][b];
            rhs[jj] += G.sqrtmg * 0.5 * s;
          }
          double s1 = 0.0, s2 = 0.0;
          for (int a = 0; a < 4; ++a) s1 += T[a][0] * dla[a];
          for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) s2 += T[a][b] * Gam[0][b][a];
          rhs[4] += G.sqrtmg * G.alpha * (s1 - s2);
        }
        for (int v = 0; v < nv; ++v)
          Uout[(size_t)v * nc + c] = c0 * U0[(size_t)v * nc + c] + c1 * U[(size_t)v * nc + c]
                                   + cdt * rhs[v];
      }
#undef FL
#undef EE
  free(Bcc);
  return 0;
}

/* ------------------------------------------------------------ con2prim */

static int apply_floors(const orc_eos *e, const orc_geom *G, double r, orc_prim *q)
{
  int flag = 0;
  double rho_flr = e->rho_flr0 * pow(r, -e->rho_flr_pow);
  double u_flr = e->u_flr0 * pow(r, -e->u_flr_pow);
  if (e->tab) {
    const double rmin = exp(e->tab->lo[0]);
    if (rho_flr < rmin) rho_flr = rmin;
  }
  if (q->rho < rho_flr) { q->rho = rho_flr; flag |= ORC_FLAG_RHO_FLOOR; }
  if (e->tab) {
    const double rmax = exp(e->tab->hi[0]);
    if (q->rho > rmax) { q->rho = rmax; flag |= ORC_FLAG_RHO_FLOOR; }
    const double umin = q->rho * exp(e->tab->lo[1]);
    if (u_flr < umin) u_flr = umin;
  }
  if (q->u < u_flr) { q->u = u_flr; flag |= ORC_FLAG_U_FLOOR; }
  if (e->tab) {
    const double umax = q->rho * exp(e->tab->hi[1]);
    if (q->u > umax) { q->u = umax; flag |= ORC_FLAG_U_FLOOR; }
  }
  double ut2 = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) ut2 += G->gam[i][j] * q->ut[i] * q->ut[j];
  const double W = sqrt(1.0 + ut2);
  if (W > e->W_max) {
    const double s = sqrt((e->W_max * e->W_max - 1.0) / ut2);
    for (int i = 0; i < 3; ++i) q->ut[i] *= s;
    flag |= ORC_FLAG_W_CAP;
  }
  return flag;
}

/*
 * U (densitized, interior) -> P.  P holds the previous primitives on entry
 * (used as the fallback of a failed inversion).  Where a floor or the
 * fallback acts, the hydro part of U is rewritten from the final P.
 * Returns the number of failed inversions.
 */
int orc_con2prim(const orc_grid *g, const orc_metric *m, const orc_eos *e, double *U,
                 const double *Bf, double *P, int8_t *flag, int nthreads)
{
  const size_t nc = ncell(g);
  double *Bcc = malloc(3 * nc * sizeof(double));
  orc_cell_B(g, m, Bf, Bcc);
  int nfail = 0;
  #pragma omp parallel for schedule(dynamic) num_threads(nthreads) reduction(+:nfail)
  for (int k = g->ng; k < g->ng + g->n[2]; ++k)
    for (int j = g->ng; j < g->ng + g->n[1]; ++j)
      for (int i = g->ng; i < g->ng + g->n[0]; ++i) {
        const size_t c = IDX(g, i, j, k);
        double x[3], Ud[6] = {0, 0, 0, 0, 0, 0}, B[3];
        orc_geom G;
        orc_prim q;
        orc_coord(g, m, ORC_LOC_CENTER, i, j, k, x);
        orc_geom_at(m, x, &G);
        const int nv = 5 + e->nscalar;
        for (int v = 0; v < nv; ++v) Ud[v] = U[(size_t)v * nc + c] / G.sqrtgam;
        for (int a = 0; a < 3; ++a) B[a] = Bcc[(size_t)a * nc + c];
        int fl = 0;
        if (orc_c2p_point(e, &G, Ud, B, &q, NULL) != 0) {
          load_prim(g, e, P, Bcc, c, &q);
          fl |= ORC_FLAG_C2P_FAIL;
          nfail += 1;
        } else if (e->nscalar && q.ye != Ud[5] / Ud[0]) {
          fl |= ORC_FLAG_YE_CLAMP;           /* Y_e held inside the table */
        }
        fl |= apply_floors(e, &G, orc_radius(m, x), &q);
        P[c] = q.rho;
        for (int a = 0; a < 3; ++a) P[(size_t)(1 + a) * nc + c] = q.ut[a];
        P[4 * nc + c] = q.u;
        if (e->nscalar) P[5 * nc + c] = q.ye;
        if (fl) {
          double Uc[9];
          orc_prim_to_cons(&G, e, &q, Uc);
          store_cons(e, U, nc, c, G.sqrtgam, Uc);
        }
        if (flag) flag[c] = (int8_t)fl;
      }
  free(Bcc);
  return nfail;
}

/* ---------------------------------------------------------- reductions */

/*
 * out[0] = dt = cfl / max_cells sum_d max|lambda_d| / dx_d  (active d only)
 * out[1] = max |div B| / (max |Bf| / min dx)   (or max |div B| if Bf = 0)
 * out[2] = max |div B|
 * out[3..7] = sum over interior of U_v dx1 dx2 dx3
 * out[8] = the same sum of the scalar plane U_5 (0 without a scalar)
 */
void orc_reductions(const orc_grid *g, const orc_metric *m, const orc_eos *e,
                    const double *P, const double *Bf, const double *U, double cfl,
                    double out[9])
{
  const size_t nc = ncell(g);
  const int ng = g->ng;
  double *Bcc = malloc(3 * nc * sizeof(double));
  orc_cell_B(g, m, Bf, Bcc);
  double smax = 0.0, dmax = 0.0, bmax = 0.0, tot[6] = {0, 0, 0, 0, 0, 0};
  double dxmin = 1e300;
  for (int d = 0; d < 3; ++d)
    if (g->n[d] > 1 && g->dx[d] < dxmin) dxmin = g->dx[d];
  const double dV = g->dx[0] * g->dx[1] * g->dx[2];
  for (int k = ng; k < ng + g->n[2]; ++k)
    for (int j = ng; j < ng + g->n[1]; ++j)
      for (int i = ng; i < ng + g->n[0]; ++i) {
        const size_t c = IDX(g, i, j, k);
        double x[3];
        orc_geom G;
        orc_prim q;
        orc_coord(g, m, ORC_LOC_CENTER, i, j, k, x);
        orc_geom_at(m, x, &G);
        load_prim(g, e, P, Bcc, c, &q);
        double s = 0.0;
        for (int d = 0; d < 3; ++d) {
          if (g->n[d] <= 1) continue;
          double lm, lp;
          orc_speeds(&G, e, &q, d, &lm, &lp);
          s += fmax(fabs(lm), fabs(lp)) / g->dx[d];
        }
        if (s > smax) smax = s;
        const size_t up[3] = {IDX(g, i + 1, j, k), IDX(g, i, j + 1, k), IDX(g, i, j, k + 1)};
        double div = 0.0;
        for (int d = 0; d < 3; ++d) {
          div += (Bf[d * nc + up[d]] - Bf[d * nc + c]) / g->dx[d];
          if (fabs(Bf[d * nc + c]) > bmax) bmax = fabs(Bf[d * nc + c]);
          if (fabs(Bf[d * nc + up[d]]) > bmax) bmax = fabs(Bf[d * nc + up[d]]);
        }
        if (fabs(div) > dmax) dmax = fabs(div);
        for (int v = 0; v < 5 + e->nscalar; ++v) tot[v] += U[(size_t)v * nc + c] * dV;
      }
  out[0] = (smax > 0.0) ? cfl / smax : 0.0;
  out[1] = (bmax > 0.0) ? dmax / (bmax / dxmin) : dmax;
  out[2] = dmax;
  for (int v = 0; v < 6; ++v) out[3 + v] = tot[v];
  free(Bcc);
}
