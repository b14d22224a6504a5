/*
 * Oracle reconstruction (Phoebus Sec. 3.1 list of reconstructions and
 * App. B, the WENO5-Z-AOAH scheme).  TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * Every routine takes the five values f[0..4] = f_{j-2} .. f_{j+2} around
 * cell j and returns the left-face (j-1/2) and right-face (j+1/2) values.
 *
 * WENO5-Z-AOAH (App. B):
 *   candidates on stencils {j-2..j}, {j-1..j+1}, {j..j+2} (the formula for
 *   P^(3)_k, which indexes them left, centred, right), Jiang-Shu smoothness
 *   indicators, Z weights w_k ~ gamma_k [1 + (tau_Z/(beta_k+eps))^p] with
 *   tau_Z = |beta_0 - beta_2|, p = 2, eps = 1e-40; the j-1/2 face by the mirror
 *   x -> -x; blending sigma P5 + (1 - sigma) PLM-MC with sigma the harmonic
 *   mean of the two per-face weight measures, clamped to [0, 1].
 *   Default candidates are the Lagrange interpolants of point values (the
 *   appendix's wording); weno_fv = 1 selects the cell-average variant.
 */
#include <math.h>
#include "orc.h"

static const double WENO_EPS = 1e-40;

static double sgn(double x) { return (x > 0.0) ? 1.0 : ((x < 0.0) ? -1.0 : 0.0); }

/* monotonized-central limited slope */
static double mc_slope(double dm, double dp)
{
  if (dm * dp <= 0.0) return 0.0;
  double a = fmin(2.0 * fabs(dm), 2.0 * fabs(dp));
  a = fmin(a, 0.5 * fabs(dm + dp));
  return sgn(dm) * a;
}

static double minmod_slope(double dm, double dp)
{
  if (dm * dp <= 0.0) return 0.0;
  return sgn(dm) * fmin(fabs(dm), fabs(dp));
}

static void linear_weights(int fv, double g[3])
{
  if (fv) { g[0] = 0.1; g[1] = 0.6; g[2] = 0.3; }
  else    { g[0] = 1.0 / 16.0; g[1] = 10.0 / 16.0; g[2] = 5.0 / 16.0; }
}

/* candidate values p_k at x_{j+1/2} */
static void candidates(int fv, const double f[5], double p[3])
{
  if (fv) {
    p[0] = (2.0 * f[0] - 7.0 * f[1] + 11.0 * f[2]) / 6.0;
    p[1] = (-f[1] + 5.0 * f[2] + 2.0 * f[3]) / 6.0;
    p[2] = (2.0 * f[2] + 5.0 * f[3] - f[4]) / 6.0;
  } else {
    p[0] = (3.0 * f[0] - 10.0 * f[1] + 15.0 * f[2]) / 8.0;
    p[1] = (-f[1] + 6.0 * f[2] + 3.0 * f[3]) / 8.0;
    p[2] = (3.0 * f[2] + 6.0 * f[3] - f[4]) / 8.0;
  }
}

void orc_weno_beta(const double f[5], double b[3])
{
  const double c = 13.0 / 12.0;
  double t;
  t = f[0] - 2.0 * f[1] + f[2]; b[0] = c * t * t;
  t = f[0] - 4.0 * f[1] + 3.0 * f[2]; b[0] += 0.25 * t * t;
  t = f[1] - 2.0 * f[2] + f[3]; b[1] = c * t * t;
  t = f[1] - f[3]; b[1] += 0.25 * t * t;
  t = f[2] - 2.0 * f[3] + f[4]; b[2] = c * t * t;
  t = 3.0 * f[2] - 4.0 * f[3] + f[4]; b[2] += 0.25 * t * t;
}

void orc_weno_weights(int fv, const double f[5], double w[3])
{
  double g[3], b[3];
  linear_weights(fv, g);
  orc_weno_beta(f, b);
  const double tau = fabs(b[0] - b[2]);
  double s = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double r = tau / (b[k] + WENO_EPS);
    w[k] = g[k] * (1.0 + r * r);
    s += w[k];
  }
  for (int k = 0; k < 3; ++k) w[k] /= s;
}

/* harmonic mean of w_k / gamma_k (App. B, per-face sigma) */
double orc_weno_sigma_side(int fv, const double w[3])
{
  double g[3];
  linear_weights(fv, g);
  return 3.0 * w[0] * w[1] * w[2]
       / (g[2] * w[0] * w[1] + g[1] * w[0] * w[2] + g[0] * w[1] * w[2]);
}

static double weno_face(int fv, const double f[5], double *sigma_side)
{
  double w[3], p[3];
  orc_weno_weights(fv, f, w);
  candidates(fv, f, p);
  *sigma_side = orc_weno_sigma_side(fv, w);
  return w[0] * p[0] + w[1] * p[1] + w[2] * p[2];
}

void orc_recon1(int method, int fv, const double f[5], double *fl, double *fr)
{
  if (method == ORC_RECON_CONST) {
    *fl = f[2]; *fr = f[2];
    return;
  }
  if (method == ORC_RECON_PLM_MINMOD) {
    const double s = minmod_slope(f[2] - f[1], f[3] - f[2]);
    *fl = f[2] - 0.5 * s; *fr = f[2] + 0.5 * s;
    return;
  }
  const double s = mc_slope(f[2] - f[1], f[3] - f[2]);
  const double pl = f[2] - 0.5 * s, pr = f[2] + 0.5 * s;
  if (method == ORC_RECON_PLM_MC) {
    *fl = pl; *fr = pr;
    return;
  }
  /* WENO5-Z-AOAH */
  const double fm[5] = {f[4], f[3], f[2], f[1], f[0]};   /* x -> -x */
  double sp, sm;
  const double p5r = weno_face(fv, f, &sp);
  const double p5l = weno_face(fv, fm, &sm);
  double sigma = 2.0 * sp * sm / (sp + sm);
  if (!(sigma > 0.0)) sigma = 0.0;
  if (sigma > 1.0) sigma = 1.0;
  *fr = sigma * p5r + (1.0 - sigma) * pr;
  *fl = sigma * p5l + (1.0 - sigma) * pl;
}
