/*
 * Oracle equation of state: ideal gas or a table, and the master function of
 * the inversion for a general EOS.  TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * Table (Sec. 2.2 tabulated EOS, Sec. 3.2 table bounds): nodes uniform in
 * x = ln rho, y = ln eps, z = Y_e.  Each coordinate is clamped into
 * [lo, hi]; with h = (hi - lo)/(n - 1), t = (x - lo)/h, cell i = floor(t)
 * (at most n - 2) and weight w = t - i, the value is the trilinear blend of
 * the 8 surrounding nodes.  The table stores ln p (so p = exp of the blend)
 * and Gamma_1 (blended directly).
 */
#include <math.h>
#include "orc.h"

static void axis(const orc_table *t, int d, double x, int *i, double *w)
{
  if (x < t->lo[d]) x = t->lo[d];
  if (x > t->hi[d]) x = t->hi[d];
  const double h = (t->hi[d] - t->lo[d]) / (double)(t->n[d] - 1);
  const double s = (x - t->lo[d]) / h;
  int k = (int)floor(s);
  if (k > t->n[d] - 2) k = t->n[d] - 2;
  if (k < 0) k = 0;
  *i = k;
  *w = s - (double)k;
}

void orc_table_eval(const orc_table *t, double rho, double eps, double ye, double *lnp,
                    double *g1)
{
  int i[3];
  double w[3];
  axis(t, 0, log(rho), &i[0], &w[0]);
  axis(t, 1, log(eps), &i[1], &w[1]);
  axis(t, 2, ye, &i[2], &w[2]);
  double a = 0.0, b = 0.0;
  for (int c = 0; c < 2; ++c)
    for (int bb = 0; bb < 2; ++bb)
      for (int aa = 0; aa < 2; ++aa) {
        const double wt = (aa ? w[0] : 1.0 - w[0]) * (bb ? w[1] : 1.0 - w[1]) *
                          (c ? w[2] : 1.0 - w[2]);
        const long node = (long)(i[0] + aa) +
                          (long)t->n[0] * ((long)(i[1] + bb) + (long)t->n[1] * (long)(i[2] + c));
        a += wt * t->data[2 * node];
        b += wt * t->data[2 * node + 1];
      }
  *lnp = a;
  *g1 = b;
}

/* p and Gamma_1 p of (rho, u = rho eps, Y_e). */
void orc_thermo(const orc_eos *e, double rho, double u, double ye, double *p, double *gp)
{
  if (!e->tab) {
    *p = (e->gamma - 1.0) * u;
    *gp = e->gamma * *p;
    return;
  }
  double lnp, g1;
  orc_table_eval(e->tab, rho, u / rho, ye, &lnp, &g1);
  *p = exp(lnp);
  *gp = g1 * *p;
}

/*
 * Master function of the inversion for a general EOS (the method of Kastaun,
 * Kalinani & Ciolfi 2021 that Sec. 3.1 cites), unknown mu = 1/(h W):
 *   x = 1/(1 + mu b^2),  rbar^2, qbar as for the ideal gas (c2p.c),
 *   v^2 = min(mu^2 rbar^2, r^2/(1 + r^2))     (h >= 1 for this table),
 *   W = (1 - v^2)^(-1/2),  rho = D/W and eps = W (qbar - mu rbar^2) + v^2 W^2/(1 + W),
 *   both clamped into the table's range (Sec. 3.2),
 *   a = p(rho, eps, Y_e) / (rho (1 + eps)),
 *   nu = max((1 + a)(1 + eps)/W, (1 + a)(1 + qbar - mu rbar^2)),
 *   f(mu) = mu - 1/(nu + mu rbar^2).
 * Without clamping the two entries of the max agree (with h = (1 + a)(1 + eps)
 * this is the ideal-gas function of c2p.c).  rho_out / eps_out: the clamped
 * rho and eps at mu.
 */
double orc_c2p_master_tab(const orc_table *t, double D, double ye, double q, double r2,
                          double b2, double rb, double mu, double *rho_out, double *eps_out)
{
  const double x = 1.0 / (1.0 + mu * b2);
  const double rbar2 = r2 * x * x + mu * x * (1.0 + x) * rb * rb;
  const double qbar = q - 0.5 * b2 - 0.5 * mu * mu * x * x * (b2 * r2 - rb * rb);
  double v2 = mu * mu * rbar2;
  const double v2max = r2 / (1.0 + r2);
  if (v2 > v2max) v2 = v2max;
  const double W = 1.0 / sqrt(1.0 - v2);
  double rho = D / W;
  const double rmin = exp(t->lo[0]), rmax = exp(t->hi[0]);
  if (rho < rmin) rho = rmin;
  if (rho > rmax) rho = rmax;
  double eps = W * (qbar - mu * rbar2) + v2 * W * W / (1.0 + W);
  const double emin = exp(t->lo[1]), emax = exp(t->hi[1]);
  if (eps < emin) eps = emin;
  if (eps > emax) eps = emax;
  double lnp, g1;
  orc_table_eval(t, rho, eps, ye, &lnp, &g1);
  const double a = exp(lnp) / (rho * (1.0 + eps));
  const double nuA = (1.0 + a) * (1.0 + eps) / W;
  const double nuB = (1.0 + a) * (1.0 + qbar - mu * rbar2);
  const double nu = nuA > nuB ? nuA : nuB;
  if (rho_out) *rho_out = rho;
  if (eps_out) *eps_out = eps;
  return mu - 1.0 / (nu + mu * rbar2);
}
