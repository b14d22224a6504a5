/*
 * Flat point-wise entry points of the oracle, for the pin tests.
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 * Primitive vectors are packed as (rho, ut1, ut2, ut3, u, B1, B2, B3).
 */
#include <math.h>
#include <string.h>
#include "orc.h"

static void unpack(const double p[8], orc_prim *q)
{
  q->rho = p[0];
  for (int i = 0; i < 3; ++i) q->ut[i] = p[1 + i];
  q->u = p[4];
  for (int i = 0; i < 3; ++i) q->B[i] = p[5 + i];
  q->ye = 0.0;
}

/* An ideal-gas EOS object for the point entries that take gamma alone. */
static orc_eos ideal(double gam)
{
  orc_eos e;
  memset(&e, 0, sizeof e);
  e.gamma = gam;
  return e;
}

/* out: g[16], gi[16], alpha, beta[3], gam[9], gami[9], sqrtgam, sqrtmg (56) */
void orc_pt_geom(const orc_metric *m, const double x[3], double *out)
{
  orc_geom G;
  orc_geom_at(m, x, &G);
  int o = 0;
  for (int a = 0; a < 4; ++a) for (int b = 0; b < 4; ++b) out[o++] = G.g[a][b];
  for (int a = 0; a < 4; ++a) for (int b = 0; b < 4; ++b) out[o++] = G.gi[a][b];
  out[o++] = G.alpha;
  for (int i = 0; i < 3; ++i) out[o++] = G.beta[i];
  for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) out[o++] = G.gam[a][b];
  for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) out[o++] = G.gami[a][b];
  out[o++] = G.sqrtgam;
  out[o++] = G.sqrtmg;
}

void orc_pt_derivs(const orc_metric *m, const double x[3], double *dg, double *Gam,
                   double *dla)
{
  double a[4][4][4], b[4][4][4], c[4];
  orc_metric_derivs(m, x, a, b, c);
  memcpy(dg, a, sizeof a);
  memcpy(Gam, b, sizeof b);
  memcpy(dla, c, sizeof c);
}

void orc_pt_p2c(const orc_metric *m, const double x[3], double gam, const double p[8],
                double U[8])
{
  orc_geom G;
  orc_prim q;
  orc_geom_at(m, x, &G);
  unpack(p, &q);
  const orc_eos e = ideal(gam);
  double U9[9];
  orc_prim_to_cons(&G, &e, &q, U9);
  memcpy(U, U9, 8 * sizeof(double));
}

void orc_pt_flux(const orc_metric *m, const double x[3], double gam, const double p[8],
                 int dir, double F[8])
{
  orc_geom G;
  orc_prim q;
  orc_geom_at(m, x, &G);
  unpack(p, &q);
  const orc_eos e = ideal(gam);
  double F9[9];
  orc_flux(&G, &e, &q, dir, F9);
  memcpy(F, F9, 8 * sizeof(double));
}

void orc_pt_speeds(const orc_metric *m, const double x[3], double gam, const double p[8],
                   int dir, double out[2])
{
  orc_geom G;
  orc_prim q;
  orc_geom_at(m, x, &G);
  unpack(p, &q);
  const orc_eos e = ideal(gam);
  orc_speeds(&G, &e, &q, dir, &out[0], &out[1]);
}

void orc_pt_riemann(const orc_metric *m, const double x[3], double gam, int solver,
                    const double pl[8], const double pr[8], int dir, double flux[8])
{
  orc_geom G;
  orc_prim L, R;
  orc_geom_at(m, x, &G);
  unpack(pl, &L);
  unpack(pr, &R);
  const orc_eos e = ideal(gam);
  double f9[9];
  orc_riemann(&G, &e, solver, &L, &R, dir, f9);
  memcpy(flux, f9, 8 * sizeof(double));
}

void orc_pt_tmunu(const orc_metric *m, const double x[3], double gam, const double p[8],
                  double T[16])
{
  orc_geom G;
  orc_prim q;
  double t[4][4];
  orc_geom_at(m, x, &G);
  unpack(p, &q);
  const orc_eos e = ideal(gam);
  orc_tmunu(&G, &e, &q, t);
  memcpy(T, t, sizeof t);
}

int orc_pt_c2p(const orc_metric *m, const double x[3], double gam, const double Ud[5],
               const double B[3], double pout[8], double *mu)
{
  orc_geom G;
  orc_prim q;
  orc_geom_at(m, x, &G);
  const orc_eos e = ideal(gam);
  double U6[6] = {Ud[0], Ud[1], Ud[2], Ud[3], Ud[4], 0.0};
  int r = orc_c2p_point(&e, &G, U6, B, &q, mu);
  if (r == 0) {
    pout[0] = q.rho;
    for (int i = 0; i < 3; ++i) pout[1 + i] = q.ut[i];
    pout[4] = q.u;
    for (int i = 0; i < 3; ++i) pout[5 + i] = q.B[i];
  }
  return r;
}

/* n points of one metric location x: prims[n][8] -> U[n][8] (undensitized). */
void orc_p2c_batch(const orc_metric *m, const double x[3], double gam, long n,
                   const double *prims, double *U)
{
  orc_geom G;
  orc_geom_at(m, x, &G);
  const orc_eos e = ideal(gam);
  for (long k = 0; k < n; ++k) {
    orc_prim q;
    double U9[9];
    unpack(prims + 8 * k, &q);
    orc_prim_to_cons(&G, &e, &q, U9);
    memcpy(U + 8 * k, U9, 8 * sizeof(double));
  }
}

/* ---- general EOS (eos points at an orc_eos with its table, if any) ----
 * Primitive vectors of 9: (rho, ut1, ut2, ut3, u, B1, B2, B3, Y_e);
 * conserved / flux vectors of 9 (the last is D Y_e and its flux). */
static void unpack9(const double p[9], orc_prim *q)
{
  unpack(p, q);
  q->ye = p[8];
}

void orc_pt_thermo(const orc_eos *e, long n, const double *rho, const double *u,
                   const double *ye, double *p, double *gp)
{
  for (long k = 0; k < n; ++k) orc_thermo(e, rho[k], u[k], ye[k], &p[k], &gp[k]);
}

void orc_pt_table(const orc_table *t, long n, const double *rho, const double *eps,
                  const double *ye, double *lnp, double *g1)
{
  for (long k = 0; k < n; ++k) orc_table_eval(t, rho[k], eps[k], ye[k], &lnp[k], &g1[k]);
}

void orc_pt_p2c_eos(const orc_metric *m, const double x[3], const orc_eos *e,
                    const double p[9], double U[9])
{
  orc_geom G;
  orc_prim q;
  orc_geom_at(m, x, &G);
  unpack9(p, &q);
  orc_prim_to_cons(&G, e, &q, U);
}

void orc_pt_riemann_eos(const orc_metric *m, const double x[3], const orc_eos *e, int solver,
                        const double pl[9], const double pr[9], int dir, double flux[9])
{
  orc_geom G;
  orc_prim L, R;
  orc_geom_at(m, x, &G);
  unpack9(pl, &L);
  unpack9(pr, &R);
  orc_riemann(&G, e, solver, &L, &R, dir, flux);
}

void orc_pt_speeds_eos(const orc_metric *m, const double x[3], const orc_eos *e,
                       const double p[9], int dir, double out[2])
{
  orc_geom G;
  orc_prim q;
  orc_geom_at(m, x, &G);
  unpack9(p, &q);
  orc_speeds(&G, e, &q, dir, &out[0], &out[1]);
}

/* Ud = undensitized (D, S_1, S_2, S_3, tau, D Y_e) -> pout[9]. */
int orc_pt_c2p_eos(const orc_metric *m, const double x[3], const orc_eos *e, const double Ud[6],
                   const double B[3], double pout[9], double *mu)
{
  orc_geom G;
  orc_prim q;
  orc_geom_at(m, x, &G);
  int r = orc_c2p_point(e, &G, Ud, B, &q, mu);
  if (r == 0) {
    pout[0] = q.rho;
    for (int i = 0; i < 3; ++i) pout[1 + i] = q.ut[i];
    pout[4] = q.u;
    for (int i = 0; i < 3; ++i) pout[5 + i] = q.B[i];
    pout[8] = q.ye;
  }
  return r;
}

double orc_pt_master_tab(const orc_table *t, double D, double ye, double q, double r2, double b2,
                         double rb, double mu)
{
  return orc_c2p_master_tab(t, D, ye, q, r2, b2, rb, mu, NULL, NULL);
}

double orc_pt_master(double gam, double q, double r2, double b2, double rb, double mu)
{
  return orc_c2p_master(gam, q, r2, b2, rb, mu);
}

void orc_pt_recon(int method, int fv, const double f[5], double out[2])
{
  orc_recon1(method, fv, f, &out[0], &out[1]);
}

void orc_pt_weno(int fv, const double f[5], double w[3], double *sigma_side)
{
  orc_weno_weights(fv, f, w);
  *sigma_side = orc_weno_sigma_side(fv, w);
}

void orc_pt_beta(const double f[5], double b[3]) { orc_weno_beta(f, b); }

void orc_pt_coord(const orc_grid *g, const orc_metric *m, int loc, int i, int j, int k,
                  double x[3])
{
  orc_coord(g, m, loc, i, j, k, x);
}
