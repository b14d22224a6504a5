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

/*
 * MP5, the monotonicity-preserving fifth-order scheme of Suresh & Huynh
 * (J. Comput. Phys. 136, 1997), which the paper lists among its
 * reconstructions without further detail.  Face j+1/2 from f[0..4]:
 *   the unlimited fifth-order value (Lagrange interpolation of the point
 *   values, or the cell-average reconstruction when fv = 1);
 *   f_MP = f_j + minmod(f_{j+1} - f_j, alpha (f_j - f_{j-1})), alpha = 4;
 *   if (f5 - f_j)(f5 - f_MP) <= 0 the value is kept; otherwise it is moved
 *   to the nearest point of [f_min, f_max] built from the curvatures
 *   d_i = f_{i-1} - 2 f_i + f_{i+1} and their M4 minmod combinations
 *   (upper limit f_UL, average f_AV, median f_MD, large-curvature f_LC).
 */
static double minmod2(double a, double b)
{
  if (a * b <= 0.0) return 0.0;
  return sgn(a) * fmin(fabs(a), fabs(b));
}

static double minmod4(double a, double b, double c, double d)
{
  const double s = sgn(a);
  if (sgn(b) != s || sgn(c) != s || sgn(d) != s) return 0.0;
  return s * fmin(fmin(fabs(a), fabs(b)), fmin(fabs(c), fabs(d)));
}

static double mp5_face(int fv, const double f[5])
{
  const double alpha = 4.0;
  const double fm2 = f[0], fm1 = f[1], f0 = f[2], fp1 = f[3], fp2 = f[4];
  const double f5 = fv ? (2.0 * fm2 - 13.0 * fm1 + 47.0 * f0 + 27.0 * fp1 - 3.0 * fp2) / 60.0
                       : (3.0 * fm2 - 20.0 * fm1 + 90.0 * f0 + 60.0 * fp1 - 5.0 * fp2) / 128.0;
  const double fmp = f0 + minmod2(fp1 - f0, alpha * (f0 - fm1));
  if ((f5 - f0) * (f5 - fmp) <= 0.0) return f5;
  const double dm = fm2 - 2.0 * fm1 + f0, d0 = fm1 - 2.0 * f0 + fp1, dp = f0 - 2.0 * fp1 + fp2;
  const double dM4p = minmod4(4.0 * d0 - dp, 4.0 * dp - d0, d0, dp);
  const double dM4m = minmod4(4.0 * d0 - dm, 4.0 * dm - d0, d0, dm);
  const double fUL = f0 + alpha * (f0 - fm1);
  const double fAV = 0.5 * (f0 + fp1);
  const double fMD = fAV - 0.5 * dM4p;
  const double fLC = f0 + 0.5 * (f0 - fm1) + (4.0 / 3.0) * dM4m;
  const double fmin_ = fmax(fmin(fmin(f0, fp1), fMD), fmin(fmin(f0, fUL), fLC));
  const double fmax_ = fmin(fmax(fmax(f0, fp1), fMD), fmax(fmax(f0, fUL), fLC));
  /* median(f5, fmin, fmax) */
  return f5 + minmod2(fmin_ - f5, fmax_ - f5);
}

void orc_recon1(int method, int fv, const double f[5], double *fl, double *fr)
{
  if (method == ORC_RECON_MP5) {
    const double fm[5] = {f[4], f[3], f[2], f[1], f[0]};   /* x -> -x */
    *fr = mp5_face(fv, f);
    *fl = mp5_face(fv, fm);
    return;
  }
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
