/*
 * Oracle point physics.  TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * Follows the Valencia formulation of the Phoebus paper, Sec. 2.1:
 * kinematics (definitions of v^i, v-tilde^i, W), the b^mu / B^i relation,
 * the conserved vector U, flux vector F^i and stress tensor T^{mu nu}, with
 * the ideal-gas or tabulated EOS of Sec. 2.2 (eos.c).  The characteristic
 * speeds (not given in the paper) are the fast-speed estimate of the isotropic
 * dispersion relation with c_s^2 = Gamma_1 p / (rho h); the Riemann solvers
 * are the LLF and HLL of Sec. 3.1.  The passive scalar of Sec. 2.1 (Y_e) is
 * carried as the ninth component: conserved D Y_e, flux Y_e times the mass
 * flux.
 */
#include <math.h>
#include "orc.h"

void orc_aux_from_prim(const orc_geom *G, const orc_eos *e, const orc_prim *P, orc_aux *A)
{
  double ut2 = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) ut2 += G->gam[i][j] * P->ut[i] * P->ut[j];
  A->W = sqrt(1.0 + ut2);
  for (int i = 0; i < 3; ++i) A->v[i] = P->ut[i] / A->W;          /* W v^i = u-tilde^i */
  for (int i = 0; i < 3; ++i) {
    A->vl[i] = 0.0;
    for (int j = 0; j < 3; ++j) A->vl[i] += G->gam[i][j] * A->v[j];
  }
  /* W = alpha u^0 ;  v^i = u^i / W + beta^i / alpha */
  A->ucon[0] = A->W / G->alpha;
  for (int i = 0; i < 3; ++i) A->ucon[i + 1] = P->ut[i] - A->W * G->beta[i] / G->alpha;
  double Bv = 0.0, B2 = 0.0;
  for (int i = 0; i < 3; ++i) {
    Bv += P->B[i] * A->vl[i];
    for (int j = 0; j < 3; ++j) B2 += G->gam[i][j] * P->B[i] * P->B[j];
  }
  A->bcon[0] = A->W * Bv / G->alpha;
  for (int i = 0; i < 3; ++i)
    A->bcon[i + 1] = (P->B[i] + G->alpha * A->bcon[0] * A->ucon[i + 1]) / A->W;
  A->b2 = (B2 + G->alpha * G->alpha * A->bcon[0] * A->bcon[0]) / (A->W * A->W);
  for (int m = 0; m < 4; ++m) {
    A->bcov[m] = 0.0;
    for (int n = 0; n < 4; ++n) A->bcov[m] += G->g[m][n] * A->bcon[n];
  }
  orc_thermo(e, P->rho, P->u, P->ye, &A->p, &A->gp);
  A->w = P->rho + P->u + A->p;
}

/* Undensitized U = (D, S_1, S_2, S_3, tau, B^1, B^2, B^3, D Y_e). */
void orc_prim_to_cons(const orc_geom *G, const orc_eos *e, const orc_prim *P, double U[9])
{
  orc_aux A;
  orc_aux_from_prim(G, e, P, &A);
  const double W2 = A.W * A.W;
  const double D = P->rho * A.W;
  const double wtot = A.w + A.b2;
  U[0] = D;
  for (int j = 0; j < 3; ++j)
    U[1 + j] = wtot * W2 * A.vl[j] - G->alpha * A.bcon[0] * A.bcov[j + 1];
  /*
   * tau = (rho h + b^2) W^2 - (p + b^2/2) - alpha^2 (b^0)^2 - D, with the
   * rest-mass part rho W^2 - rho W written as D (W^2 - 1)/(W + 1) so that
   * slow flows keep the internal energy exact.  Algebraically identical.
   */
  double ut2 = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) ut2 += G->gam[i][j] * P->ut[i] * P->ut[j];
  U[4] = D * ut2 / (A.W + 1.0) + (P->u + A.p) * W2 + A.b2 * W2
       - (A.p + 0.5 * A.b2) - G->alpha * G->alpha * A.bcon[0] * A.bcon[0];
  for (int k = 0; k < 3; ++k) U[5 + k] = P->B[k];
  U[8] = D * P->ye;
}

/* Undensitized flux F^dir (dir = 0, 1, 2 for x1, x2, x3). */
void orc_flux(const orc_geom *G, const orc_eos *e, const orc_prim *P, int dir, double F[9])
{
  orc_aux A;
  orc_aux_from_prim(G, e, P, &A);
  double U[9];
  orc_prim_to_cons(G, e, P, U);
  double vt[3];
  for (int i = 0; i < 3; ++i) vt[i] = G->alpha * A.v[i] - G->beta[i];
  const double ptot = A.p + 0.5 * A.b2;
  const double a = G->alpha, W = A.W, Bd = P->B[dir];
  F[0] = U[0] * vt[dir] / a;
  for (int j = 0; j < 3; ++j)
    F[1 + j] = U[1 + j] * vt[dir] / a + (j == dir ? ptot : 0.0) - A.bcov[j + 1] * Bd / W;
  F[4] = U[4] * vt[dir] / a + ptot * A.v[dir] - a * A.bcon[0] * Bd / W;
  for (int k = 0; k < 3; ++k) F[5 + k] = (P->B[k] * vt[dir] - Bd * vt[k]) / a;
  F[8] = U[8] * vt[dir] / a;
}

/*
 * Coordinate speeds dx^dir/dt of the fast wave: roots of
 * (k_mu u^mu)^2 (1 - c^2) = c^2 k_mu k^mu with k_mu = (-lambda, e_dir) and
 * c^2 = cs^2 + ca^2 - cs^2 ca^2.
 */
void orc_speeds(const orc_geom *G, const orc_eos *e, const orc_prim *P, int dir,
                double *lm, double *lp)
{
  orc_aux A;
  orc_aux_from_prim(G, e, P, &A);
  const double cs2 = A.gp / A.w;
  const double ca2 = A.b2 / (A.w + A.b2);
  const double c2 = cs2 + ca2 - cs2 * ca2;
  const double u0 = A.ucon[0], ui = A.ucon[dir + 1];
  const double g00 = G->gi[0][0], g0i = G->gi[0][dir + 1], gii = G->gi[dir + 1][dir + 1];
  const double qa = (1.0 - c2) * u0 * u0 - c2 * g00;
  const double qb = -2.0 * ((1.0 - c2) * u0 * ui - c2 * g0i);
  const double qc = (1.0 - c2) * ui * ui - c2 * gii;
  double disc = qb * qb - 4.0 * qa * qc;
  if (disc < 0.0) disc = 0.0;
  const double sq = sqrt(disc);
  const double l1 = (-qb + sq) / (2.0 * qa), l2 = (-qb - sq) / (2.0 * qa);
  *lp = fmax(l1, l2);
  *lm = fmin(l1, l2);
}

/*
 * Densitized numerical flux at a face of the law
 *   d_t (sqrt(gamma) U) + d_i (sqrt(-g) F^i) = ...
 * The wave speeds are eigenvalues of d(sqrt(-g)F)/d(sqrt(gamma)U), so the
 * dissipation acts on sqrt(gamma) U and the flux is sqrt(-g) F.
 */
void orc_riemann(const orc_geom *G, const orc_eos *e, int solver, const orc_prim *L,
                 const orc_prim *R, int dir, double flux[9])
{
  double UL[9], UR[9], FL[9], FR[9];
  double lmL, lpL, lmR, lpR;
  orc_prim_to_cons(G, e, L, UL);
  orc_prim_to_cons(G, e, R, UR);
  orc_flux(G, e, L, dir, FL);
  orc_flux(G, e, R, dir, FR);
  orc_speeds(G, e, L, dir, &lmL, &lpL);
  orc_speeds(G, e, R, dir, &lmR, &lpR);
  const double sg = G->sqrtgam, smg = G->sqrtmg;
  if (solver == ORC_RIEMANN_HLL) {
    const double cm = fmin(0.0, fmin(lmL, lmR));
    const double cp = fmax(0.0, fmax(lpL, lpR));
    for (int v = 0; v < 9; ++v) {
      const double gl = smg * FL[v], gr = smg * FR[v];
      if (cp - cm > 0.0)
        flux[v] = (cp * gl - cm * gr + cp * cm * (sg * UR[v] - sg * UL[v])) / (cp - cm);
      else
        flux[v] = 0.5 * (gl + gr);
    }
  } else {
    const double c = fmax(fmax(fabs(lmL), fabs(lpL)), fmax(fabs(lmR), fabs(lpR)));
    for (int v = 0; v < 9; ++v)
      flux[v] = 0.5 * (smg * FL[v] + smg * FR[v]) - 0.5 * c * (sg * UR[v] - sg * UL[v]);
  }
}

/* T^{mu nu} = (rho + u + p + b^2) u^mu u^nu + (p + b^2/2) g^{mu nu} - b^mu b^nu */
void orc_tmunu(const orc_geom *G, const orc_eos *e, const orc_prim *P, double T[4][4])
{
  orc_aux A;
  orc_aux_from_prim(G, e, P, &A);
  const double wt = A.w + A.b2, pt = A.p + 0.5 * A.b2;
  for (int m = 0; m < 4; ++m)
    for (int n = 0; n < 4; ++n)
      T[m][n] = wt * A.ucon[m] * A.ucon[n] + pt * G->gi[m][n] - A.bcon[m] * A.bcon[n];
}
