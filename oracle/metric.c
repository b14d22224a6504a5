/*
 * Oracle geometry (Phoebus Sec. 2.3: analytic metrics behind one coordinate
 * interface).  TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * The metric is written once, in complex arithmetic; values are taken at real
 * points and every derivative (d_mu g_{ab}, d_mu ln alpha) by complex-step
 * differentiation, which is exact to rounding for analytic functions.  The
 * Christoffel symbols then follow from their definition.
 */
#include <math.h>
#include <string.h>
#include "orc.h"

/* Kerr-Schild line element in (t, r, theta, phi), then dr = r dx1. */
void orc_gcov_c(const orc_metric *m, const double complex X[4], double complex g[4][4])
{
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) g[a][b] = 0.0;
  if (m->kind == ORC_MINKOWSKI) {
    g[0][0] = -1.0; g[1][1] = 1.0; g[2][2] = 1.0; g[3][3] = 1.0;
    return;
  }
  const double a = m->a, M = m->M;
  double complex r = cexp(X[1]);
  double complex s = csin(X[2]), c = ccos(X[2]);
  double complex s2 = s * s;
  double complex Sig = r * r + a * a * c * c;
  double complex z = 2.0 * M * r / Sig;
  double complex k[4][4];
  for (int p = 0; p < 4; ++p)
    for (int q = 0; q < 4; ++q) k[p][q] = 0.0;
  k[0][0] = -(1.0 - z);
  k[0][1] = z;
  k[0][3] = -z * a * s2;
  k[1][1] = 1.0 + z;
  k[1][3] = -a * (1.0 + z) * s2;
  k[2][2] = Sig;
  k[3][3] = s2 * (Sig + a * a * (1.0 + z) * s2);
  k[1][0] = k[0][1]; k[3][0] = k[0][3]; k[3][1] = k[1][3];
  double complex J[4] = {1.0, r, 1.0, 1.0};  /* d(t,r,th,ph)/d(t,x1,x2,x3) */
  for (int p = 0; p < 4; ++p)
    for (int q = 0; q < 4; ++q) g[p][q] = J[p] * J[q] * k[p][q];
}

int orc_invert4(const double a_in[4][4], double ai[4][4])
{
  double a[4][8];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      a[i][j] = a_in[i][j];
      a[i][j + 4] = (i == j) ? 1.0 : 0.0;
    }
  for (int col = 0; col < 4; ++col) {
    int piv = col;
    for (int r = col + 1; r < 4; ++r)
      if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
    if (a[piv][col] == 0.0) return -1;
    if (piv != col)
      for (int j = 0; j < 8; ++j) {
        double t = a[col][j]; a[col][j] = a[piv][j]; a[piv][j] = t;
      }
    double d = a[col][col];
    for (int j = 0; j < 8; ++j) a[col][j] /= d;
    for (int r = 0; r < 4; ++r) {
      if (r == col) continue;
      double f = a[r][col];
      if (f == 0.0) continue;
      for (int j = 0; j < 8; ++j) a[r][j] -= f * a[col][j];
    }
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) ai[i][j] = a[i][j + 4];
  return 0;
}

static double complex det3c(double complex m[3][3])
{
  return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
       - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
       + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

static double complex det4c(double complex m[4][4])
{
  double complex d = 0.0;
  for (int c = 0; c < 4; ++c) {
    double complex sub[3][3];
    for (int i = 1; i < 4; ++i) {
      int cc = 0;
      for (int j = 0; j < 4; ++j) {
        if (j == c) continue;
        sub[i - 1][cc++] = m[i][j];
      }
    }
    double complex t = m[0][c] * det3c(sub);
    d += (c % 2 == 0) ? t : -t;
  }
  return d;
}

void orc_geom_at(const orc_metric *m, const double x[3], orc_geom *G)
{
  double complex X[4] = {0.0, x[0], x[1], x[2]};
  double complex gc[4][4];
  orc_gcov_c(m, X, gc);
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) G->g[a][b] = creal(gc[a][b]);
  orc_invert4(G->g, G->gi);
  G->alpha = 1.0 / sqrt(-G->gi[0][0]);
  const double a2 = G->alpha * G->alpha;
  for (int i = 0; i < 3; ++i) G->beta[i] = a2 * G->gi[0][i + 1];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      G->gam[i][j] = G->g[i + 1][j + 1];
      G->gami[i][j] = G->gi[i + 1][j + 1] + G->beta[i] * G->beta[j] / a2;
    }
  const double (*q)[3] = G->gam;
  double det = q[0][0] * (q[1][1] * q[2][2] - q[1][2] * q[2][1])
             - q[0][1] * (q[1][0] * q[2][2] - q[1][2] * q[2][0])
             + q[0][2] * (q[1][0] * q[2][1] - q[1][1] * q[2][0]);
  G->sqrtgam = sqrt(det);
  G->sqrtmg = G->alpha * G->sqrtgam;
}

/*
 * dg[mu][a][b] = d_mu g_{ab};  Gam[l][a][b] = Gamma^l_{ab};
 * dlnalpha[mu] = d_mu ln(alpha) with alpha^2 = -det(g)/det(gamma).
 */
void orc_metric_derivs(const orc_metric *m, const double x[3],
                       double dg[4][4][4], double Gam[4][4][4], double dlnalpha[4])
{
  const double h = 1e-30;
  orc_geom G;
  orc_geom_at(m, x, &G);
  for (int mu = 0; mu < 4; ++mu) {
    double complex X[4] = {0.0, x[0], x[1], x[2]};
    X[mu] += I * h;
    double complex gc[4][4], sp[3][3];
    orc_gcov_c(m, X, gc);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) dg[mu][a][b] = cimag(gc[a][b]) / h;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) sp[i][j] = gc[i + 1][j + 1];
    double complex lna = 0.5 * clog(-det4c(gc) / det3c(sp));
    dlnalpha[mu] = cimag(lna) / h;
  }
  for (int l = 0; l < 4; ++l)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        double s = 0.0;
        for (int sg = 0; sg < 4; ++sg)
          s += G.gi[l][sg] * (dg[a][sg][b] + dg[b][sg][a] - dg[sg][a][b]);
        Gam[l][a][b] = 0.5 * s;
      }
}

/*
 * Code coordinates of a cell centre or lower face.  On a polar x2 boundary the
 * ghost rows take the theta of their mirror row, so metric values there are
 * those of the reflected interior point (the metric is even in theta about
 * either pole).
 */
void orc_coord(const orc_grid *g, const orc_metric *m, int loc, int i, int j, int k, double x[3])
{
  int idx[3] = {i, j, k};
  (void)m;
  for (int d = 0; d < 3; ++d) {
    int face = (loc == d + 1);
    int id = idx[d];
    if (d == 1) {
      int lo = g->ng, hi = g->ng + g->n[1];
      int plo = (g->bc[2] == ORC_BC_POLAR), phi = (g->bc[3] == ORC_BC_POLAR);
      if (face) {
        if (plo && id < lo) id = 2 * lo - id;
        if (phi && id > hi) id = 2 * hi - id;
      } else {
        if (plo && id < lo) id = 2 * lo - 1 - id;
        if (phi && id >= hi) id = 2 * hi - 1 - id;
      }
    }
    x[d] = g->xmin[d] + ((double)(id - g->ng) + (face ? 0.0 : 0.5)) * g->dx[d];
  }
}

double orc_radius(const orc_metric *m, const double x[3])
{
  return (m->kind == ORC_KS_LOGSPH) ? exp(x[0]) : 1.0;
}
