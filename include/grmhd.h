/*
 * grmhd.h - C ABI of the MI355X (gfx950) GRMHD stage library, libgrmhd.so.
 *
 * One Runge-Kutta stage of the Valencia-formulation ideal GRMHD finite-volume
 * update (Phoebus paper, Sec. 2.1 conservation law with the conserved vector,
 * flux vector and source vector given there; Sec. 3.1 second-order finite
 * volumes, constrained transport, LLF/HLL Riemann solvers, the reconstruction
 * list and the master-function inversion; Sec. 3.2 floors; App. B
 * WENO5-Z-AOAH) over a pack of meshblocks on one GPU.
 *
 * Memory and ownership
 *   - All state arrays are device memory owned by the caller.  The library
 *     never allocates device memory: scratch lives in a caller-provided
 *     workspace of grmhd_pack_workspace_bytes() bytes (256-byte aligned).
 *   - A pack owns host metadata only and is bound to one HIP stream; every
 *     call below is asynchronous on that stream unless stated otherwise.
 *   - Arrays are structure-of-arrays, FP64: variable v of cell c of block b is
 *     at  base[v * ncell_total + offset[b] + c],  c = i + s1 (j + s2 k),
 *     s_d = n_d + 2 ng, offsets from grmhd_layout().
 *       P  [5]: rho, W v^1, W v^2, W v^3 (contravariant), u = rho eps
 *       Bf [3]: sqrt(gamma) B^d on the lower d-face of each cell
 *       U  [5]: sqrt(gamma) (D, S_1, S_2, S_3, tau), S_j covariant
 *       U0 [5], Bf0 [3]: Runge-Kutta base copies of U and Bf.
 *     With the passive scalar (desc.nscalar = 1) P, U and U0 have 6 planes:
 *       P[5] = Y_e and U[5] = sqrt(gamma) D Y_e (Sec. 2.1 advected scalars,
 *       X = Y_e, no source term).
 *   - Coordinates: Minkowski-Cartesian, or Kerr-Schild with x1 = ln r,
 *     x2 = theta, x3 = phi (units G = c = M = 1, Heaviside-Lorentz B).
 *
 * Errors: every int-returning call gives 0 on success or a negative code;
 * grmhd_last_error() returns the message.  No exception or abort crosses the
 * ABI.  Con2prim failures are not errors: they are flagged per cell.
 */
#ifndef GRMHD_H
#define GRMHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GRMHD_ABI_VERSION 3

enum { GRMHD_OK = 0, GRMHD_E_INVALID = -1, GRMHD_E_SHAPE = -2, GRMHD_E_HIP = -3,
       GRMHD_E_UNSUPPORTED = -4 };
enum { GRMHD_METRIC_MINKOWSKI = 0, GRMHD_METRIC_KS_LOGSPH = 1 };
enum { GRMHD_BC_PERIODIC = 0, GRMHD_BC_OUTFLOW = 1, GRMHD_BC_POLAR = 2, GRMHD_BC_FIXED = 3 };
enum { GRMHD_RECON_CONST = 0, GRMHD_RECON_PLM_MC = 1, GRMHD_RECON_WENO5Z_AOAH = 2,
       GRMHD_RECON_PLM_MINMOD = 3, GRMHD_RECON_MP5 = 4 };
enum { GRMHD_RIEMANN_HLL = 0, GRMHD_RIEMANN_LLF = 1 };
enum { GRMHD_PREC_FP64 = 0, GRMHD_PREC_MIXED = 1 };
enum { GRMHD_GUESS_COLD = 0, GRMHD_GUESS_PREV = 1, GRMHD_GUESS_MLP = 2 };
/* per-cell con2prim flag bits */
enum { GRMHD_FLAG_RHO_FLOOR = 1, GRMHD_FLAG_U_FLOOR = 2, GRMHD_FLAG_W_CAP = 4,
       GRMHD_FLAG_C2P_FAIL = 8, GRMHD_FLAG_GUESS_FALLBACK = 16, GRMHD_FLAG_YE_CLAMP = 32 };

typedef struct grmhd_pack grmhd_pack;

/* Analytic metric (Sec. 2.3): kind, black-hole mass M and spin a (KS only). */
typedef struct { int kind; double M, a; } grmhd_metric;

/*
 * Tabulated EOS (Sec. 2.2 tabulated equations of state; Sec. 3.2 their
 * bounds).  Nodes uniform in the coordinates (ln rho, ln eps, Y_e): axis d
 * has n[d] >= 2 nodes from lo[d] to hi[d].  data is DEVICE memory owned by
 * the caller, n[0] * n[1] * n[2] pairs of doubles (ln p, Gamma_1), node
 * (i, j, k) at pair i + n[0] (j + n[1] k), with Gamma_1 = d ln p / d ln rho
 * at constant entropy (rho h c_s^2 = Gamma_1 p).  Between nodes both entries
 * are trilinear in the coordinates; a state outside the table is looked up
 * at its clamped coordinates.  It must stay valid and unchanged while calls
 * that use it are in flight (a captured step graph keeps the pointer).
 */
typedef struct {
  const double *data;
  int n[3];
  double lo[3], hi[3];
} grmhd_eos_table;

/*
 * EOS (Sec. 2.2) and floors (Sec. 3.2):
 *   table == NULL: ideal gas p = (gamma - 1) u;
 *   table != NULL: the tabulated EOS above (the pack needs nscalar = 1, Y_e
 *     being its third coordinate), and gamma is unused;
 *   rho >= rho_flr0 r^-rho_flr_pow;  u >= u_flr0 r^-u_flr_pow
 *   (r = 1 in Minkowski);  W <= W_max; with a table also rho, u / rho and Y_e
 *   within the table's range (flags RHO_FLOOR, U_FLOOR, YE_CLAMP).
 * c2p_tol: relative Newton tolerance on mu = 1/(hW); c2p_max_iter: cap.
 */
typedef struct {
  double gamma, rho_flr0, rho_flr_pow, u_flr0, u_flr_pow, W_max, c2p_tol;
  int c2p_max_iter;
  const grmhd_eos_table *table;
} grmhd_eos;

/*
 * Pack descriptor.  nblocks blocks, block b has nx[3b..3b+2] interior cells,
 * refinement level level[b] (0 or 1; NULL = all 0) and logical location
 * lloc[3b..3b+2] = global index (in cells of its level) of its first interior
 * cell.  The whole domain spans [xmin, xmax] with root_nx cells at level 0
 * (root_nx << 1 at level 1); the blocks must tile it exactly once, level-1
 * blocks with even sizes and offsets.  Ghost zones between levels are filled
 * by restriction (cell means of 8 children, face means of 4 child faces) and
 * prolongation (parent plus monotonized-central limited slopes; faces constant
 * across a coarse face and linear along its normal); a face between cells of
 * different levels belongs to the finer side.  Each stage replaces the coarse
 * hydro fluxes and edge EMFs on level boundaries by the means of the fine
 * ones, so the totals are conserved and the field through an interface is
 * one (paper Sec. 1 and 3 use Parthenon's block-structured refinement).  bc[6] = boundary kind at (x1 lo, x1 hi, x2 lo, x2 hi, x3 lo,
 * x3 hi).  ng must be 4.
 * recon: GRMHD_RECON_* (Sec. 3.1 list: constant, linear with minmod or MC,
 *        mp5 of Suresh & Huynh 1997, WENO5-Z-AOAH of App. B).
 * weno_fv: 0 = the fifth-order candidates interpolate point values (App. B
 *          wording), 1 = cell-average reconstruction (WENO5 and MP5 alike).
 * nscalar: 0, or 1 for the Y_e passive scalar (Sec. 2.1): P, U and U0 gain the
 *          plane 5, reconstructed and fluxed like the hydro variables (its
 *          conserved form D Y_e, its flux Y_e times the mass flux).  Needs
 *          precision FP64 and a single-level pack (GRMHD_E_UNSUPPORTED
 *          otherwise); the flux tiles then use shape 0 except with
 *          WENO5-Z-AOAH point values and LLF.
 */
typedef struct {
  int nblocks, ng;
  int recon, riemann, precision, weno_fv;
  const int *nx, *level, *lloc;
  int root_nx[3];
  double xmin[3], xmax[3];
  int bc[6];
  int nscalar;
} grmhd_pack_desc;

/* Device pointers bound to a pack (caller-owned, see layout above). */
typedef struct { void *P, *Bf, *U, *U0, *Bf0; } grmhd_state_ptrs;

/*
 * Reduction results (O(1) scalars).
 *   dt: cfl / max over interior cells of sum_d max|lambda_d| / dx_d
 *       (directions with a single cell are skipped);
 *   divb_rel: max |sum_d delta_d Bf_d / dx_d| / (max |Bf| / min dx);
 *   totals[5]: sum over interior of U_v dx1 dx2 dx3;
 *   c2p_fail, floor_hits: flagged cells of the last con2prim;
 *   c2p_fail_total: failed inversions summed over every con2prim since the
 *   pack was created (a device counter that both inversions of every step
 *   add to; the difference of two reads counts the calls in between);
 *   c2p_iter_mean / c2p_iter_wavemax_mean: Newton iterations per cell and the
 *   mean over 64-cell wavefronts of the per-wavefront maximum;
 *   total_scalar: sum over interior of U_5 dx1 dx2 dx3 (0 without a scalar).
 */
typedef struct {
  double dt, divb_rel, divb_max, totals[5];
  long long c2p_fail, floor_hits;
  double c2p_iter_mean, c2p_iter_wavemax_mean;
  long long guess_fallback;   /* cells whose learned guess was rejected */
  double total_scalar;
  long long c2p_fail_total;
} grmhd_reduction_out;

int grmhd_abi_version(void);

/* Layout: fills offsets[nblocks] (cells) and *ncell_total (cells per variable
 * plane, every block offset a multiple of 32 cells = 256 bytes). */
int grmhd_layout(const grmhd_pack_desc *desc, long long *offsets, long long *ncell_total);

/* Workspace bytes a pack with this descriptor needs (0 on invalid desc). */
size_t grmhd_pack_workspace_bytes(const grmhd_pack_desc *desc);

/*
 * Validate desc, build block tables, ghost maps and tile lists, upload them
 * into the workspace (async on hip_stream).  ws must stay valid and unused by
 * anything else until grmhd_pack_destroy.  Errors: E_INVALID / E_SHAPE /
 * E_UNSUPPORTED for a bad descriptor, E_HIP for a failed HIP call.
 */
int grmhd_pack_create(const grmhd_pack_desc *desc, const grmhd_state_ptrs *state,
                      void *workspace, size_t ws_bytes, void *hip_stream, grmhd_pack **out);

/* Frees host metadata only (after synchronising the stream). */
int grmhd_pack_destroy(grmhd_pack *pack);

/* Replace the bound state pointers (same shapes). */
int grmhd_bind_state(grmhd_pack *pack, const grmhd_state_ptrs *state);

/*
 * Fill the ghost zones of P and Bf (boundary kinds and same-level block
 * copies), then the cell-centred field used by the next stage.
 */
int grmhd_fill_ghosts(grmhd_pack *pack, const grmhd_metric *metric);

/*
 * One Runge-Kutta stage (Sec. 2.1, Sec. 3.1):  with L = -div F + sqrt(-g) S
 * evaluated on the current P and Bf,
 *     U  <- c0 U0  + c1 U  + c_dt dt L
 *     Bf <- c0 Bf0 + c1 Bf + c_dt dt (CT update from edge-averaged EMFs).
 * rk_coeffs = {c0, c1, c_dt}.  When c1 == 0 the current U and Bf are the
 * base: they are first saved into U0 and Bf0 (so SSPRK2 is {1,0,1} then
 * {1/2,1/2,1/2}).  dt <= 0 means: use the device-resident dt written by the
 * last reduction fold (grmhd_reductions, or a grmhd_step with cfl > 0; no
 * host round trip); before any fold of this pack such a call returns
 * GRMHD_E_INVALID.  Requires grmhd_fill_ghosts since the last change of P
 * or Bf.
 */
int grmhd_stage(grmhd_pack *pack, const grmhd_metric *metric, const grmhd_eos *eos,
                double dt, const double rk_coeffs[3]);

/*
 * Con2prim + floors on interior cells: P <- P(U, Bf) by safeguarded Newton on
 * the master function f(mu) = mu - 1/(h/W + mu rbar^2) (the unknown mu =
 * 1/(hW); with a table, the general-EOS form of Kastaun et al. 2021 with
 * rho, eps clamped into the table and nu = max of its two expressions),
 * starting from guess (COLD: mu = 1/sqrt(1 + r^2); PREV: from the
 * current P; MLP: the learned initial guess bound by grmhd_mlp_bind, used
 * where the W it implies through the master function agrees with the
 * network's own W output to 50 %, else COLD and flag GUESS_FALLBACK).
 * The inversion fails (flag C2P_FAIL) for D <= 0 or a non-finite U, when
 * f(1) < 0 (no root in (0, 1]), when Newton has not met |dmu| <= c2p_tol mu
 * within c2p_max_iter iterations, and when the root's primitives are not
 * finite.  A failed inversion keeps the previous P.  Where a floor or the failure
 * acts, the hydro part of U is rewritten from the final P (Sec. 3.1
 * inversion, Sec. 3.2 floors).
 */
int grmhd_con2prim(grmhd_pack *pack, const grmhd_metric *metric, const grmhd_eos *eos,
                   int guess);

/* Initialise U from P and Bf on interior cells (same map as the inversion's inverse). */
int grmhd_prim_to_cons(grmhd_pack *pack, const grmhd_metric *metric, const grmhd_eos *eos);

/*
 * Reductions (see grmhd_reduction_out).  The dt is always stored device-side
 * for the next grmhd_stage(dt <= 0).  out == NULL: asynchronous; otherwise the
 * call synchronises the stream and fills *out.
 */
int grmhd_reductions(grmhd_pack *pack, const grmhd_metric *metric, const grmhd_eos *eos,
                     double cfl, grmhd_reduction_out *out);

/*
 * One SSPRK2 step: stage {1,0,1}, con2prim(guess), ghosts, stage {1/2,1/2,1/2},
 * con2prim(guess), ghosts, then (cfl > 0) reductions leaving the next dt on the
 * device.  dt <= 0 uses the device-resident dt.  Asynchronous.  The base of
 * the step is not copied: the first stage writes its state into U0 and Bf0
 * (which then hold that state after the call), the first inversion and ghost
 * fill and the second stage work on them, and the second stage combines U / Bf
 * with them into U / Bf.  P, U and Bf come out bitwise equal to the sequence
 * of the calls above (which copy the base), with one write of U and Bf per
 * cell less.  A pack with the fused stage (grmhd_set_fused) keeps the copying
 * form.
 */
int grmhd_step(grmhd_pack *pack, const grmhd_metric *metric, const grmhd_eos *eos, double dt,
               int guess, double cfl);

/*
 * The same step captured once into a HIP graph (dt from the device, no host
 * round trip) and replayed nsteps times on the pack's stream.  The graph is
 * re-captured when metric, eos, guess or cfl change; it binds the current
 * state pointers (re-capture after grmhd_bind_state by changing nothing is not
 * needed: bind_state drops the graph).
 */
int grmhd_step_graph(grmhd_pack *pack, const grmhd_metric *metric, const grmhd_eos *eos,
                     int guess, double cfl, int nsteps);

/*
 * Face-tile shapes of the flux kernels: shape s has TD faces along the flux
 * direction and 256/TD columns (TD = 16, 32, 8, 64, 4 for s = 0..4).  Shapes
 * 1..4 exist for the WENO5-Z-AOAH point-value reconstruction (with the
 * passive scalar: with LLF); every other combination runs shape 0.  grmhd_autotune times each shape's tile kernel
 * per direction (reps launches after one untimed launch, HIP events on the
 * pack's stream; the kernels only read the state and write the flux scratch),
 * keeps the fastest in chosen[3] and ms_table[3 * 5] (ms per launch, -1 when
 * not available) and applies it.  Synchronises the stream.
 */
#define GRMHD_NSHAPE 5
int grmhd_set_tiling(grmhd_pack *pack, const int shape[3]);
/* workgroups > 0: launch the flux-tile kernels as a persistent grid of that
 * many workgroups striding over the tile work-list; 0: one workgroup per tile.
 * With FP64 face states and no scalar the persistent tiles stream each
 * workgroup's next stencil window from global memory straight into LDS while
 * the current tile's Riemann solves run (the same fluxes to rounding). */
int grmhd_set_persistent(grmhd_pack *pack, int workgroups);
int grmhd_get_tiling(const grmhd_pack *pack, int shape[3]);
/*
 * Fused stage (optional, off by default; single-level packs without the
 * scalar): the flux tiles of x1 and x2 leave their part of the hydro flux divergence in
 * the workspace and those of x3 add theirs, the sources (Sec. 2.1) and the
 * Runge-Kutta combination, so no hydro face flux reaches device memory and
 * the boundary-plane launch is not needed (tiles along D overlap by one face);
 * the update kernel then does constrained transport only.  The face-flux
 * scratch then holds only the induction fluxes.  enable = 0 is the default
 * unfused path (every face flux stored, grmhd_debug_ptrs' flux array
 * complete).  GRMHD_E_UNSUPPORTED for two-level packs and packs with the
 * scalar, which always run unfused.
 */
int grmhd_set_fused(grmhd_pack *pack, int enable);
/*
 * Concurrency (on by default): the x2 and x3 flux tiles and the boundary
 * planes of a stage run on three auxiliary streams of the pack (default
 * priority, forked from and joined back into the pack's stream, so a captured
 * step graph holds them as parallel branches) beside the x1 tiles; they write
 * disjoint face fluxes.  With kernel timing (grmhd_profile), while autotuning,
 * in the fused stage, or with enable = 0 every launch stays on the pack's
 * stream.
 */
int grmhd_set_concurrency(grmhd_pack *pack, int enable);
int grmhd_autotune(grmhd_pack *pack, const grmhd_metric *metric, const grmhd_eos *eos, int reps,
                   int chosen[3], double *ms_table);

/* Device pointers to the per-cell int8 flags and uint8 Newton iteration
 * counts of the last con2prim (inside the workspace; same cell layout as P). */
int grmhd_debug_ptrs(grmhd_pack *pack, void **flags, void **iters, void **flux);

/*
 * Kernel timing.  grmhd_profile(pack, 1) starts recording a HIP event pair on
 * the pack's stream around every launch of a kernel family; grmhd_profile_read
 * synchronises the stream and returns, per family, the summed milliseconds and
 * the number of launches since the last read (arrays of GRMHD_PROF_NFAM).
 * Families: flux tiles along x1 / x2 / x3, boundary face planes, update,
 * con2prim (the learned guess's inference included: it runs inside the
 * inversion kernel, so the MLP family stays empty), ghost gather,
 * cell-centred field, reductions.
 */
enum { GRMHD_PROF_FLUX_X1 = 0, GRMHD_PROF_FLUX_X2 = 1, GRMHD_PROF_FLUX_X3 = 2,
       GRMHD_PROF_FLUX_PLANE = 3, GRMHD_PROF_UPDATE = 4, GRMHD_PROF_C2P = 5,
       GRMHD_PROF_GHOST = 6, GRMHD_PROF_BCC = 7, GRMHD_PROF_REDUCE = 8,
       GRMHD_PROF_MLP = 9, GRMHD_PROF_M1 = 10, GRMHD_PROF_NFAM = 11 };
int grmhd_profile(grmhd_pack *pack, int enable);
int grmhd_profile_read(grmhd_pack *pack, double *ms, long long *count);

/*
 * Learned initial guess of the inversion (growth on top of the paper's
 * method; the Newton solve still decides the result).  Network 5 -> 64 -> 64 -> 64 -> 2
 * with SiLU, GRMHD_MLP_NPARAM FP32 parameters laid out as W1[64][5] b1[64]
 * W2[64][64] b2[64] W3[64][64] b3[64] W4[2][64] b4[2] (W[out][in]).
 * Features of a cell's undensitized conserved state: log10 D, log(1+S^2/D^2),
 * log(1+tau/D), log(1+B^2/D), log(1+(S.B)^2/D^3), standardised by feat_mean /
 * feat_std; outputs y0 = log W, y1 = log(hW), guess mu0 = exp(-y1).
 * All pointers are device pointers; calls are asynchronous on the stream.
 */
#define GRMHD_MLP_NPARAM 8834
/* Copy the FP32 parameters into the pack as BF16 matrix-core operands. */
int grmhd_mlp_bind(grmhd_pack *pack, const float *params, const float *feat_mean,
                   const float *feat_std);
/* Scratch bytes the training / gradient / inference calls need for a batch. */
size_t grmhd_mlp_scratch_bytes(int batch);
/* FP32 loss (mean over the batch of the summed squared error) and its
 * gradient w.r.t. params (same layout).  X: [batch][5] standardised
 * features, Y: [batch][2] targets. */
int grmhd_mlp_grad(const float *params, const float *X, const float *Y, int batch, float *grad,
                   float *loss, void *scratch, size_t scratch_bytes, void *hip_stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, step number t >= 1) on the
 * FP32 master parameters; adam_m / adam_v: moment buffers (GRMHD_MLP_NPARAM). */
int grmhd_mlp_train_step(float *params, float *adam_m, float *adam_v, const float *X,
                         const float *Y, int batch, float lr, int t, float *loss, void *scratch,
                         size_t scratch_bytes, void *hip_stream);
/*
 * The training step above without a caller scratch, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight training or
 * serving loops, harnesses that forbid hipMalloc): the same kernels run on a
 * scratch the library holds in device memory of its own, a static array of
 * grmhd_mlp_scratch_bytes(GRMHD_MLP_NOALLOC_MAX_BATCH) bytes (about 9.5 MB)
 * per GPU, kept until the process ends.  The call allocates nothing; its
 * first call on a device looks up that device's copy.  batch must be at most
 * GRMHD_MLP_NOALLOC_MAX_BATCH (GRMHD_E_SHAPE otherwise, nothing launched);
 * hip_stream must belong to the current device (GRMHD_E_INVALID otherwise).
 * Every call on one GPU shares that GPU's scratch: calls that overlap on one
 * GPU (other streams, other threads) race and must be serialised by the
 * caller.  Nothing in the scratch needs to start at zero.
 */
#define GRMHD_MLP_NOALLOC_MAX_BATCH 4096
int grmhd_mlp_train_step_noalloc(float *params, float *adam_m, float *adam_v, const float *X,
                                 const float *Y, int batch, float lr, int t, float *loss,
                                 void *hip_stream);
/* BF16 matrix-core inference on raw features X [n][5] -> Y [n][2]. */
int grmhd_mlp_infer(const float *params, const float *feat_mean, const float *feat_std,
                    const float *X, float *Y, int n, void *scratch, size_t scratch_bytes,
                    void *hip_stream);

/*
 * Gray M1 moments (Sec. 2.4): the implicit (backward-Euler) update of the
 * collision sources of every interior cell, for nspecies neutrino species
 * (1..8; the paper evolves three).  Per species and cell the Eulerian
 * moments X = (E, F_1, F_2, F_3) solve
 *   X - X* = dt S(X),  S_E = alpha^2 G^0,  S_Fi = alpha g_{i nu} G^nu,
 *   G^nu = kappa_J u^nu (J_eq - J) - kappa_H H^nu,
 * with J, H the fluid-frame energy and flux of the M1 stress tensor and the
 * closure P^ij = (3 chi - 1)/2 P_thin + 3 (1 - chi)/2 P_thick, chi = (1 - 2f +
 * 4f^2)/3 (maximum-entropy Fermi-Dirac at maximum packing), f = |F|/E; the
 * opacities and J_eq are held fixed.  Newton's method with the exact
 * Jacobian, |dX| <= tol (|X*| + |X|) (tol <= 0: 1e-13), at most max_iter
 * (1..254) iterations.  The fluid velocity comes from the bound P.
 *   R      device, [nspecies][4][ncell_total]: sqrt(gamma) (E, F_1, F_2, F_3)
 *          (F_i covariant); X* on entry, the update on return (in place).
 *   kappa  device, [nspecies][3][ncell_total]: kappa_J, kappa_H, J_eq.
 *   couple 1: the fluid's U[4] (tau) and U[1..3] (S_i) take the opposite of
 *          the exchanged energy and momentum (run grmhd_con2prim after).
 *   iters  device uint8 [ncell_total] or NULL: the largest Newton count over
 *          the species (255: a species did not converge; its moments are the
 *          last iterate).
 * Asynchronous on the pack's stream.
 */
int grmhd_m1_source(grmhd_pack *pack, const grmhd_metric *metric, double dt, int nspecies,
                    void *R, const void *kappa, int couple, double tol, int max_iter,
                    void *iters);

/*
 * Refinement of the two-level block mesh (the paper evolves on Parthenon's
 * adaptive block mesh, Sec. 1 and 3; the operators are not given there).
 *
 * grmhd_tag: per block, the largest refinement indicator of P[var] over its
 * interior cells, max over the directions of |q(i+1) - q(i-1)| / (2 |q(i)|)
 * (directions with one cell skipped); needs filled ghosts.  block_max: host
 * array of nblocks.  Synchronises the stream.
 *
 * grmhd_regrid_layout: the next layout from the current descriptor and host
 * tags (+1 refine, -1 derefine, 0 keep): a level-0 block with tag +1 and even
 * sizes becomes its 8 level-1 children (the same size in level-1 cells); 8
 * level-1 blocks of one cubic size m at base + {0, m}^3 (base a multiple of
 * 2m) that are all tagged -1 become one level-0 block of size m; any other
 * level-1 block tagged -1 becomes the level-0 block over its region (half its
 * size, when that is at least ng); every other block is kept, in order
 * (children and merged blocks take the place of their first source block).  Host only.  *nb_out gets the new count; the
 * arrays (cap blocks) get nx[3 nb], lloc[3 nb], level[nb]; GRMHD_E_SHAPE when
 * cap is too small.
 *
 * grmhd_remap: the state of src (P, U, Bf, with its ghosts filled) onto the
 * layout of dst (same root grid and boundaries, no scalar): identical blocks
 * are copied whole; otherwise per cell copy or restriction (mean of 8) of P
 * and U, or prolongation (P by parent + MC-limited slopes toward the octant,
 * a non-positive rho or u keeping the parent value; U = U(P, B) of each child
 * plus the parent's U minus the mean over its 8 children, which keeps the
 * totals), per face copy, mean of 4 fine faces, or for new fine faces: the
 * existing fine neighbour's face across a coarse face, else the coarse
 * value, and inside each coarse cell the least-squares correction of the
 * linear interpolation that makes its 8 children divergence-free.  metric
 * and eos serve U(P, B).  Then run grmhd_fill_ghosts, grmhd_con2prim and
 * grmhd_fill_ghosts on dst.  scratch: device memory (256-byte aligned) of
 * grmhd_remap_scratch_bytes(dst, src) bytes; src must not be written while
 * the call runs (it synchronises dst's stream before returning).  dst and
 * src are two packs with their own state arrays (GRMHD_E_INVALID when they
 * share P, U or Bf).
 */
int grmhd_tag(grmhd_pack *pack, int var, double *block_max);
int grmhd_regrid_layout(const grmhd_pack_desc *desc, const int *tags, int cap, int *nb_out,
                        int *nx_out, int *lloc_out, int *level_out);
size_t grmhd_remap_scratch_bytes(const grmhd_pack *dst, const grmhd_pack *src);
int grmhd_remap(grmhd_pack *dst, const grmhd_pack *src, const grmhd_metric *metric,
                const grmhd_eos *eos, void *scratch, size_t scratch_bytes);

const char *grmhd_last_error(const grmhd_pack *pack);

#ifdef __cplusplus
}
#endif
#endif
