/*
 * FP64 CPU oracle for one Runge-Kutta stage of the Valencia ideal-GRMHD
 * finite-volume update (Phoebus paper, Sec. 2.1 and Sec. 3.1, App. B).
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, plain reference the HIP
 * path is checked against.  It shares no code with the HIP library: no
 * headers, helpers or tables.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.
 *
 * Conventions
 *   - Units G = c = M_bh = 1; Heaviside-Lorentz magnetic field (the flux and
 *     stress tensor carry p + b^2/2, Sec. 2.1 eqs. for F^i and T^{mu nu}).
 *   - Coordinates: Minkowski-Cartesian (t,x,y,z) or Kerr-Schild with
 *     x1 = ln r, x2 = theta, x3 = phi.
 *   - One block: n[d] interior cells plus ng ghosts per side; cell (i,j,k)
 *     has linear index i + s1*(j + s2*k), s_d = n[d] + 2 ng.
 *   - P[5][ncell]  : rho, W v^1, W v^2, W v^3 (contravariant), u = rho eps.
 *   - Bf[3][ncell] : sqrt(gamma) B^d on the lower d-face of each cell.
 *   - U[5][ncell]  : sqrt(gamma) (D, S_1, S_2, S_3, tau), S_j covariant.
 *   - With a passive scalar (nscalar = 1, the electron fraction Y_e of
 *     Sec. 2.1's advected quantities): P[5] = Y_e and U[5] = sqrt(gamma) D Y_e;
 *     its face flux is stored in the slot 5 + d of the direction-d flux
 *     block (the slot of the normal field component, whose induction flux
 *     vanishes identically).
 */
#ifndef ORC_H
#define ORC_H

#include <complex.h>
#include <stdint.h>

enum { ORC_MINKOWSKI = 0, ORC_KS_LOGSPH = 1 };
enum { ORC_BC_PERIODIC = 0, ORC_BC_OUTFLOW = 1, ORC_BC_POLAR = 2, ORC_BC_FIXED = 3 };
enum { ORC_RECON_CONST = 0, ORC_RECON_PLM_MC = 1, ORC_RECON_WENO5Z_AOAH = 2,
       ORC_RECON_PLM_MINMOD = 3, ORC_RECON_MP5 = 4 };
enum { ORC_RIEMANN_HLL = 0, ORC_RIEMANN_LLF = 1 };
enum { ORC_LOC_CENTER = 0, ORC_LOC_FACE1 = 1, ORC_LOC_FACE2 = 2, ORC_LOC_FACE3 = 3 };

/* c2p flag bits */
enum { ORC_FLAG_RHO_FLOOR = 1, ORC_FLAG_U_FLOOR = 2, ORC_FLAG_W_CAP = 4,
       ORC_FLAG_C2P_FAIL = 8, ORC_FLAG_YE_CLAMP = 32 };

typedef struct { int kind; double M, a; } orc_metric;

/*
 * Tabulated EOS (Sec. 2.2: tabulated equations of state with bounds on their
 * state variables, Sec. 3.2): nodes uniform in (ln rho, ln eps, Y_e), each
 * holding (ln p, Gamma_1) with Gamma_1 = (d ln p / d ln rho) at constant
 * entropy, so that rho h c_s^2 = Gamma_1 p.  Between nodes both are trilinear
 * in the three coordinates; outside the table the coordinates are clamped.
 */
typedef struct {
  const double *data;            /* [n[2]][n[1]][n[0]][2]                  */
  int n[3];                      /* nodes along ln rho, ln eps, Y_e (>= 2) */
  double lo[3], hi[3];           /* first and last node of each axis       */
} orc_table;

typedef struct {
  double gamma;                  /* ideal-gas adiabatic index            */
  double rho_flr0, rho_flr_pow;  /* rho_floor = rho_flr0 * r^-pow        */
  double u_flr0, u_flr_pow;      /* u_floor   = u_flr0   * r^-pow        */
  double W_max;                  /* Lorentz-factor ceiling               */
  int nscalar;                   /* 1: the Y_e passive scalar is evolved */
  const orc_table *tab;          /* NULL: ideal gas; else the table (needs nscalar = 1) */
} orc_eos;

typedef struct {
  int n[3], ng;
  double xmin[3], dx[3];
  int bc[6];                     /* x1 lo, x1 hi, x2 lo, x2 hi, x3 lo, x3 hi */
  int recon, riemann;
  int weno_fv;                   /* 0 = point-value interpolation, 1 = cell-average */
} orc_grid;

/* 3+1 quantities at a point (real). */
typedef struct {
  double g[4][4], gi[4][4];      /* g_{mu nu}, g^{mu nu}                  */
  double alpha, beta[3];         /* lapse, contravariant shift            */
  double gam[3][3], gami[3][3];  /* gamma_ij, gamma^ij                    */
  double sqrtgam, sqrtmg;        /* sqrt(gamma), sqrt(-g)                 */
} orc_geom;

/* metric.c */
void orc_gcov_c(const orc_metric *m, const double complex X[4], double complex g[4][4]);
void orc_geom_at(const orc_metric *m, const double x[3], orc_geom *G);
void orc_metric_derivs(const orc_metric *m, const double x[3],
                       double dg[4][4][4], double Gam[4][4][4], double dlnalpha[4]);
int  orc_invert4(const double a[4][4], double ai[4][4]);
void orc_coord(const orc_grid *g, const orc_metric *m, int loc, int i, int j, int k, double x[3]);
double orc_radius(const orc_metric *m, const double x[3]);

/* physics.c */
typedef struct {
  double rho, ut[3], u, B[3];    /* primitives; B^i undensitized           */
  double ye;                     /* passive scalar (0 when not evolved)   */
} orc_prim;
typedef struct {
  double W, v[3], vl[3], ucon[4], bcon[4], bcov[4], b2, p, w;  /* w = rho h */
  double gp;                     /* Gamma_1 p = rho h c_s^2               */
} orc_aux;
/* Vectors of 9: (D, S_1, S_2, S_3, tau, B^1, B^2, B^3, D Y_e) and fluxes. */
void orc_aux_from_prim(const orc_geom *G, const orc_eos *e, const orc_prim *P, orc_aux *A);
void orc_prim_to_cons(const orc_geom *G, const orc_eos *e, const orc_prim *P, double U[9]);
void orc_flux(const orc_geom *G, const orc_eos *e, const orc_prim *P, int dir, double F[9]);
void orc_speeds(const orc_geom *G, const orc_eos *e, const orc_prim *P, int dir,
                double *lm, double *lp);
void orc_riemann(const orc_geom *G, const orc_eos *e, int solver, const orc_prim *L,
                 const orc_prim *R, int dir, double flux[9]);
void orc_tmunu(const orc_geom *G, const orc_eos *e, const orc_prim *P, double T[4][4]);

/* eos.c */
void orc_table_eval(const orc_table *t, double rho, double eps, double ye, double *lnp,
                    double *g1);
void orc_thermo(const orc_eos *e, double rho, double u, double ye, double *p, double *gp);
double orc_c2p_master_tab(const orc_table *t, double D, double ye, double q, double r2,
                          double b2, double rb, double mu, double *rho_out, double *eps_out);

/* m1.c (gray M1 moments of one species: X = (E, F_1, F_2, F_3), op = (kappa_J,
   kappa_H, J_eq)) */
double orc_m1_chi(double f);
void orc_m1_closure(const orc_geom *G, const double ut[3], double E, const double Fl[3],
                    double P[3][3]);
void orc_m1_sources(const orc_geom *G, const double ut[3], const double X[4],
                    const double op[3], double *J_out, double S[4]);
int orc_m1_implicit(const orc_geom *G, const double ut[3], const double Xs[4],
                    const double op[3], double dt, double X[4]);

/* recon.c */
void orc_recon1(int method, int weno_fv, const double f[5], double *fl, double *fr);
void orc_weno_weights(int weno_fv, const double f[5], double w[3]);
double orc_weno_sigma_side(int weno_fv, const double w[3]);
void orc_weno_beta(const double f[5], double b[3]);

/* c2p.c */
int orc_c2p_point(const orc_eos *e, const orc_geom *G, const double Ud[6], const double B[3],
                  orc_prim *P, double *mu_out);
double orc_c2p_master(double gam, double q, double r2, double b2, double rb, double mu);

#endif
