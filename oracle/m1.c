/*
 * Oracle gray M1 moments: closure and the implicit (backward-Euler) update of
 * the collision sources (Phoebus Sec. 2.4, moments).  TEST INFRASTRUCTURE
 * ONLY (see orc.h).
 *
 * Per species, the Eulerian moments E, F_i (F^i = gamma^ij F_j, F^0 = 0) and
 * the pressure P^ij (P^{0 mu} = 0) make the radiation stress tensor
 *   T^{mu nu} = E n^mu n^nu + F^mu n^nu + n^mu F^nu + P^{mu nu}.
 * Closure: flux factor f = |F|/E (clamped to [0, 1]), chi = (1 - 2f + 4f^2)/3
 * (maximum-entropy Fermi-Dirac closure at maximum packing),
 *   P = (3 chi - 1)/2 P_thin + 3 (1 - chi)/2 P_thick,
 *   P_thin^ij = E F^i F^j / (F_k F^k),
 *   P_thick^ij = the spatial projection of the tensor that is isotropic in the
 *   fluid frame, (4/3) J u u + (1/3) J g + H u + u H (H.u = 0), whose E and
 *   F_i equal the given ones (a linear 4x4 problem for J and H^i, solved here
 *   numerically).
 * Fluid-frame energy and flux of T: J = u_mu u_nu T^{mu nu},
 *   H_mu = -(g_{mu a} + u_mu u_a) u_b T^{ab}.
 * Four-force (absorption, emission, elastic scattering):
 *   G^nu = kappa_J u^nu (J_eq - J) - kappa_H H^nu.
 * Implicit update of one cell (opacities and J_eq held fixed):
 *   E - E* = dt alpha^2 G^0,   F_i - F_i* = dt alpha g_{i nu} G^nu,
 * the sources of the energy and momentum equations of Sec. 2.4.  The oracle
 * finds the root of that residual by Newton's method with a central-
 * difference Jacobian (the root is the definition; the HIP path uses another
 * iteration).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "orc.h"

/* u^mu, u_mu, n^mu, n_mu of the fluid with u-tilde^i = ut[i]. */
static void frames(const orc_geom *G, const double ut[3], double u[4], double ul[4],
                   double n[4], double nl[4], double *W)
{
  double ut2 = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) ut2 += G->gam[i][j] * ut[i] * ut[j];
  *W = sqrt(1.0 + ut2);
  u[0] = *W / G->alpha;
  for (int i = 0; i < 3; ++i) u[1 + i] = ut[i] - *W * G->beta[i] / G->alpha;
  for (int a = 0; a < 4; ++a) {
    ul[a] = 0.0;
    for (int b = 0; b < 4; ++b) ul[a] += G->g[a][b] * u[b];
  }
  n[0] = 1.0 / G->alpha;
  for (int i = 0; i < 3; ++i) n[1 + i] = -G->beta[i] / G->alpha;
  nl[0] = -G->alpha;
  nl[1] = nl[2] = nl[3] = 0.0;
}

/* Lab moments (E, F_i) of a 4x4 contravariant tensor T. */
static void lab_moments(const orc_geom *G, const double nl[4], const double T[4][4],
                        double *E, double F[3])
{
  double e = 0.0;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) e += nl[a] * nl[b] * T[a][b];
  *E = e;
  /* F_i = -n_mu gamma_{i nu} T^{mu nu}, gamma_{i nu} = g_{i nu} (n_i = 0) */
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) s += nl[a] * G->g[1 + i][b] * T[a][b];
    F[i] = -s;
  }
}

/* Fluid-frame-isotropic tensor of (J, H^1..3), H^0 from H.u = 0. */
static void thick_tensor(const orc_geom *G, const double u[4], const double ul[4], double J,
                         const double Hs[3], double T[4][4])
{
  double H[4];
  for (int i = 0; i < 3; ++i) H[1 + i] = Hs[i];
  H[0] = -(Hs[0] * ul[1] + Hs[1] * ul[2] + Hs[2] * ul[3]) / ul[0];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      T[a][b] = (4.0 / 3.0) * J * u[a] * u[b] + (1.0 / 3.0) * J * G->gi[a][b] + H[a] * u[b] +
                u[a] * H[b];
}

/* Gaussian elimination with partial pivoting; returns 0 on success. */
static int solve4(double A[4][4], double b[4], double x[4])
{
  int p[4] = {0, 1, 2, 3};
  for (int c = 0; c < 4; ++c) {
    int best = c;
    for (int r = c + 1; r < 4; ++r)
      if (fabs(A[p[r]][c]) > fabs(A[p[best]][c])) best = r;
    const int t = p[c]; p[c] = p[best]; p[best] = t;
    if (A[p[c]][c] == 0.0) return 1;
    for (int r = c + 1; r < 4; ++r) {
      const double m = A[p[r]][c] / A[p[c]][c];
      for (int k = c; k < 4; ++k) A[p[r]][k] -= m * A[p[c]][k];
      b[p[r]] -= m * b[p[c]];
    }
  }
  for (int c = 3; c >= 0; --c) {
    double s = b[p[c]];
    for (int k = c + 1; k < 4; ++k) s -= A[p[c]][k] * x[k];
    x[c] = s / A[p[c]][c];
  }
  return 0;
}

double orc_m1_chi(double f) { return (1.0 - 2.0 * f + 4.0 * f * f) / 3.0; }

/* Closure: P^ij (contravariant) of the moments (E, F_i) in the fluid ut. */
void orc_m1_closure(const orc_geom *G, const double ut[3], double E, const double Fl[3],
                    double P[3][3])
{
  double u[4], ul[4], n[4], nl[4], W;
  frames(G, ut, u, ul, n, nl, &W);
  double Fu[3], F2 = 0.0;
  for (int i = 0; i < 3; ++i) {
    Fu[i] = 0.0;
    for (int j = 0; j < 3; ++j) Fu[i] += G->gami[i][j] * Fl[j];
    F2 += Fu[i] * Fl[i];
  }
  double f = E > 0.0 ? sqrt(F2) / E : 0.0;
  if (f > 1.0) f = 1.0;
  const double chi = orc_m1_chi(f);
  const double a = 0.5 * (3.0 * chi - 1.0), b = 1.5 * (1.0 - chi);
  /* thick part: (J, H^i) reproducing (E, F_i); the map is linear, so its
     matrix columns are the moments of the unit tensors */
  double A[4][4], rhs[4] = {E, Fl[0], Fl[1], Fl[2]}, y[4];
  for (int c = 0; c < 4; ++c) {
    double J = c == 0 ? 1.0 : 0.0, Hs[3] = {c == 1, c == 2, c == 3}, T[4][4], e, Fc[3];
    thick_tensor(G, u, ul, J, Hs, T);
    lab_moments(G, nl, T, &e, Fc);
    A[0][c] = e;
    for (int i = 0; i < 3; ++i) A[1 + i][c] = Fc[i];
  }
  double Pt[3][3] = {{0}};
  if (solve4(A, rhs, y) == 0) {
    double T[4][4];
    thick_tensor(G, u, ul, y[0], y + 1, T);
    /* gamma^i_mu = delta^i_mu + n^i n_mu */
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int a2 = 0; a2 < 4; ++a2)
          for (int b2 = 0; b2 < 4; ++b2) {
            const double pi = (a2 == 1 + i ? 1.0 : 0.0) + n[1 + i] * nl[a2];
            const double pj = (b2 == 1 + j ? 1.0 : 0.0) + n[1 + j] * nl[b2];
            s += pi * pj * T[a2][b2];
          }
        Pt[i][j] = s;
      }
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const double thin = F2 > 0.0 ? E * Fu[i] * Fu[j] / F2 : 0.0;
      P[i][j] = a * thin + b * Pt[i][j];
    }
}

/* J, H_mu (covariant) and the sources (S_E, S_F_i) of the moments X =
   (E, F_1, F_2, F_3) with opacities op = (kappa_J, kappa_H, J_eq). */
void orc_m1_sources(const orc_geom *G, const double ut[3], const double X[4],
                    const double op[3], double *J_out, double S[4])
{
  double u[4], ul[4], n[4], nl[4], W;
  frames(G, ut, u, ul, n, nl, &W);
  double P[3][3];
  orc_m1_closure(G, ut, X[0], X + 1, P);
  double Fu[4] = {0, 0, 0, 0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Fu[1 + i] += G->gami[i][j] * X[1 + j];
  double T[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      double p = (a > 0 && b > 0) ? P[a - 1][b - 1] : 0.0;
      T[a][b] = X[0] * n[a] * n[b] + Fu[a] * n[b] + n[a] * Fu[b] + p;
    }
  double J = 0.0;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) J += ul[a] * ul[b] * T[a][b];
  double uT[4];                                   /* u_b T^{a b} */
  for (int a = 0; a < 4; ++a) {
    uT[a] = 0.0;
    for (int b = 0; b < 4; ++b) uT[a] += ul[b] * T[a][b];
  }
  double Hl[4];
  for (int m = 0; m < 4; ++m) {
    double s = 0.0;
    for (int a = 0; a < 4; ++a) s += (G->g[m][a] + ul[m] * ul[a]) * uT[a];
    Hl[m] = -s;
  }
  double Hu[4];
  for (int a = 0; a < 4; ++a) {
    Hu[a] = 0.0;
    for (int b = 0; b < 4; ++b) Hu[a] += G->gi[a][b] * Hl[b];
  }
  double Gu[4];
  for (int a = 0; a < 4; ++a) Gu[a] = op[0] * u[a] * (op[2] - J) - op[1] * Hu[a];
  S[0] = G->alpha * G->alpha * Gu[0];
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
    for (int b = 0; b < 4; ++b) s += G->g[1 + i][b] * Gu[b];
    S[1 + i] = G->alpha * s;
  }
  if (J_out) *J_out = J;
}

/* Backward-Euler update of one species in one cell: X solves
   X - Xs - dt S(X) = 0 (undensitized E, F_i).  Returns the number of Newton
   iterations (negative if it did not converge). */
int orc_m1_implicit(const orc_geom *G, const double ut[3], const double Xs[4],
                    const double op[3], double dt, double X[4])
{
  for (int k = 0; k < 4; ++k) X[k] = Xs[k];
  double scale = fabs(Xs[0]);
  for (int k = 1; k < 4; ++k) scale += fabs(Xs[k]);
  scale += fabs(dt * op[2]) + 1e-300;
  for (int it = 1; it <= 60; ++it) {
    double S[4], R[4];
    orc_m1_sources(G, ut, X, op, NULL, S);
    double rn = 0.0;
    for (int k = 0; k < 4; ++k) {
      R[k] = X[k] - Xs[k] - dt * S[k];
      rn += fabs(R[k]);
    }
    double A[4][4];
    for (int c = 0; c < 4; ++c) {
      double h = 1e-6 * (fabs(X[c]) + 1e-3 * scale);
      double Xp[4], Xm[4], Sp[4], Sm[4];
      for (int k = 0; k < 4; ++k) { Xp[k] = X[k]; Xm[k] = X[k]; }
      Xp[c] += h;
      Xm[c] -= h;
      orc_m1_sources(G, ut, Xp, op, NULL, Sp);
      orc_m1_sources(G, ut, Xm, op, NULL, Sm);
      for (int k = 0; k < 4; ++k)
        A[k][c] = (c == k ? 1.0 : 0.0) - dt * (Sp[k] - Sm[k]) / (2.0 * h);
    }
    double b[4] = {-R[0], -R[1], -R[2], -R[3]}, d[4];
    if (solve4(A, b, d)) return -it;
    double dn = 0.0, xn = 0.0;
    for (int k = 0; k < 4; ++k) {
      X[k] += d[k];
      dn += fabs(d[k]);
      xn += fabs(X[k]);
    }
    (void)rn;
    /* the step against the larger of the input and the solution (which can
       exceed the input by orders of magnitude where the emission dominates):
       the next step is far below rounding */
    if (dn <= 1e-14 * (scale + xn)) return it;
  }
  return -60;
}

/*
 * Every interior cell of a block: R [nsp][4][ncell] = sqrt(gamma) (E, F_i)
 * per species (updated in place), kap [nsp][3][ncell] = (kappa_J, kappa_H,
 * J_eq), the fluid from P (u-tilde^i = P[1..3]).  iters (optional) gets the
 * largest Newton count over the species of each cell (negative: no
 * convergence).  Returns the number of cells that did not converge.
 */
int orc_m1_update_grid(const orc_grid *g, const orc_metric *m, int nsp, const double *P,
                       double *R, const double *kap, double dt, int *iters, int nthreads)
{
  const int s1 = g->n[0] + 2 * g->ng, s2 = g->n[1] + 2 * g->ng, s3 = g->n[2] + 2 * g->ng;
  const size_t nc = (size_t)s1 * s2 * s3;
  int bad = 0;
  #pragma omp parallel for schedule(dynamic) num_threads(nthreads) reduction(+:bad)
  for (int k = g->ng; k < g->ng + g->n[2]; ++k)
    for (int j = g->ng; j < g->ng + g->n[1]; ++j)
      for (int i = g->ng; i < g->ng + g->n[0]; ++i) {
        const size_t c = (size_t)i + (size_t)s1 * ((size_t)j + (size_t)s2 * k);
        double x[3];
        orc_geom G;
        orc_coord(g, m, ORC_LOC_CENTER, i, j, k, x);
        orc_geom_at(m, x, &G);
        const double ut[3] = {P[nc + c], P[2 * nc + c], P[3 * nc + c]};
        int worst = 0, fail = 0;
        for (int s = 0; s < nsp; ++s) {
          double Xs[4], X[4], op[3];
          for (int v = 0; v < 4; ++v) Xs[v] = R[((size_t)s * 4 + v) * nc + c] / G.sqrtgam;
          for (int q = 0; q < 3; ++q) op[q] = kap[((size_t)s * 3 + q) * nc + c];
          const int it = orc_m1_implicit(&G, ut, Xs, op, dt, X);
          if (it < 0) fail = 1;
          if (abs(it) > worst) worst = abs(it);
          for (int v = 0; v < 4; ++v) R[((size_t)s * 4 + v) * nc + c] = G.sqrtgam * X[v];
        }
        if (iters) iters[c] = fail ? -worst : worst;
        bad += fail;
      }
  return bad;
}
