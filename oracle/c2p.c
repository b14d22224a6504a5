/*
 * Oracle conserved-to-primitive inversion (Phoebus Sec. 3.1: the one-dimensional
 * master-function approach of Kastaun, Kalinani & Ciolfi 2021).
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * With q = tau/D, r_i = S_i/D, b^i = B^i/sqrt(D), the unknown is mu = 1/(hW),
 * x = 1/(1 + mu b^2) and
 *   rbar^2 = r^2 x^2 + mu x (1 + x) (r.b)^2
 *   qbar   = q - b^2/2 - mu^2 x^2 (b^2 r^2 - (r.b)^2)/2
 *   v^2    = min(mu^2 rbar^2, r^2/(1 + r^2))          (ideal gas: h >= 1)
 *   W      = (1 - v^2)^(-1/2),  rho = D/W
 *   eps    = max(W (qbar - mu rbar^2) + v^2 W^2/(1 + W), 0)
 *   h      = 1 + gamma eps                              (ideal gas)
 *   f(mu)  = mu - 1/(h/W + mu rbar^2).
 * These follow from the conserved-vector definitions of Sec. 2.1.  The root is
 * the unique zero in (0, 1]; the oracle finds it by plain bisection (the
 * defining property of the root), not by the Newton iteration of the HIP path.
 * With a tabulated EOS the same bisection runs on the general master
 * function of eos.c; the passive scalar is Y_e = (D Y_e)/D, clamped into the
 * table's range (Sec. 3.2) when a table is used.
 */
#include <math.h>
#include <stddef.h>
#include "orc.h"

double orc_c2p_master(double gam, double q, double r2, double b2, double rb, double mu)
{
  const double x = 1.0 / (1.0 + mu * b2);
  const double rbar2 = r2 * x * x + mu * x * (1.0 + x) * rb * rb;
  const double qbar = q - 0.5 * b2 - 0.5 * mu * mu * x * x * (b2 * r2 - rb * rb);
  double v2 = mu * mu * rbar2;
  const double v2max = r2 / (1.0 + r2);
  if (v2 > v2max) v2 = v2max;
  const double W = 1.0 / sqrt(1.0 - v2);
  double eps = W * (qbar - mu * rbar2) + v2 * W * W / (1.0 + W);
  if (eps < 0.0) eps = 0.0;
  const double h = 1.0 + gam * eps;
  return mu - 1.0 / (h / W + mu * rbar2);
}

/*
 * Ud = undensitized (D, S_1, S_2, S_3, tau, D Y_e) (the last entry is read only
 * with a scalar); B = undensitized B^i.
 * Returns 0 on success, 1 for an invalid state, 2 if the bracket fails, 3 if
 * the root's primitives are not finite.
 */
int orc_c2p_point(const orc_eos *e, const orc_geom *G, const double Ud[6], const double B[3],
                  orc_prim *P, double *mu_out)
{
  const double D = Ud[0];
  const double gam = e->gamma;
  const orc_table *t = e->tab;
  const int nv = 5 + e->nscalar;
  for (int v = 0; v < nv; ++v)
    if (!isfinite(Ud[v])) return 1;
  if (!(D > 0.0)) return 1;
  double ye = e->nscalar ? Ud[5] / D : 0.0;
  if (t) {
    if (ye < t->lo[2]) ye = t->lo[2];
    if (ye > t->hi[2]) ye = t->hi[2];
  }
  double Su[3], Bl[3];
  for (int i = 0; i < 3; ++i) {
    Su[i] = 0.0; Bl[i] = 0.0;
    for (int j = 0; j < 3; ++j) {
      Su[i] += G->gami[i][j] * Ud[1 + j];
      Bl[i] += G->gam[i][j] * B[j];
    }
  }
  double S2 = 0.0, BB = 0.0, SB = 0.0;
  for (int i = 0; i < 3; ++i) {
    S2 += Ud[1 + i] * Su[i];
    BB += Bl[i] * B[i];
    SB += Ud[1 + i] * B[i];
  }
  const double q = Ud[4] / D;
  const double r2 = S2 / (D * D);
  const double b2 = BB / D;
  const double rb = SB / (D * sqrt(D));

#define MASTER(m) (t ? orc_c2p_master_tab(t, D, ye, q, r2, b2, rb, (m), NULL, NULL) \
                   : orc_c2p_master(gam, q, r2, b2, rb, (m)))
  double lo = 0.0, hi = 1.0;
  double flo = MASTER(lo);
  double fhi = MASTER(hi);
  if (!(flo < 0.0)) return 2;
  if (fhi < 0.0) return 2;
  double mu = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    mu = 0.5 * (lo + hi);
    if (mu <= lo || mu >= hi) break;      /* bracket is two adjacent doubles */
    const double f = MASTER(mu);
    if (f == 0.0) { lo = hi = mu; break; }
    if (f < 0.0) lo = mu; else hi = mu;
  }
  mu = 0.5 * (lo + hi);

  const double x = 1.0 / (1.0 + mu * b2);
  const double rbar2 = r2 * x * x + mu * x * (1.0 + x) * rb * rb;
  const double qbar = q - 0.5 * b2 - 0.5 * mu * mu * x * x * (b2 * r2 - rb * rb);
  double v2 = mu * mu * rbar2;
  const double v2max = r2 / (1.0 + r2);
  if (v2 > v2max) v2 = v2max;
  const double W = 1.0 / sqrt(1.0 - v2);
  double eps = W * (qbar - mu * rbar2) + v2 * W * W / (1.0 + W);
  if (eps < 0.0) eps = 0.0;
  if (t) {          /* eps clamped into the table as in the master function */
    const double emin = exp(t->lo[1]), emax = exp(t->hi[1]);
    if (eps < emin) eps = emin;
    if (eps > emax) eps = emax;
  }
#undef MASTER
  P->rho = D / W;
  P->u = P->rho * eps;
  P->ye = ye;
  /* v^i = mu x (r^i + mu (r.b) b^i) with r^i = S^i/D, b^i = B^i/sqrt(D) */
  const double sD = sqrt(D);
  for (int i = 0; i < 3; ++i) {
    const double vi = mu * x * (Su[i] / D + mu * rb * B[i] / sD);
    P->ut[i] = W * vi;
    P->B[i] = B[i];
  }
  if (mu_out) *mu_out = mu;
  /* a root whose primitives are not finite (v^2 bound rounded to 1, so that
     W overflows) is no inversion: the state is reported as failed */
  if (!(P->rho > 0.0) || !isfinite(P->rho) || !isfinite(P->u)) return 3;
  for (int i = 0; i < 3; ++i)
    if (!isfinite(P->ut[i])) return 3;
  return 0;
}
