"""Seeded synthetic inputs shared by the HIP path, the tests and the benchmark.

This module holds problem descriptions and initial conditions only: grid
extents, boundary kinds, EOS and floor parameters, and primitive fields built
from analytic solutions (linear waves, shock tubes, Michel inflow, the
Fishbone-Moncrief torus) or seeded random draws.  It contains none of the
finite-volume stage: no reconstruction, Riemann flux, constrained transport,
source term or conserved-to-primitive inversion.  The torus and Michel
generators evaluate the Kerr / Schwarzschild metric themselves only to lay
down the initial fluid (their own short formulas); neither the oracle nor the
HIP library calls into this module's arithmetic.

Array conventions (both paths): cell-centred primitives ``P[5, s3, s2, s1]`` =
(rho, W v^1, W v^2, W v^3, u = rho eps) with contravariant velocities, and
face-centred densitized field ``Bf[3, s3, s2, s1]`` = sqrt(gamma) B^d on the
lower d-face of each cell; s_d = n_d + 2 ng.
"""
from dataclasses import dataclass, field

import numpy as np

# boundary kinds, reconstructions, Riemann solvers, metrics (ABI values)
BC_PERIODIC, BC_OUTFLOW, BC_POLAR, BC_FIXED = 0, 1, 2, 3
RECON_CONST, RECON_PLM_MC, RECON_WENO5Z, RECON_PLM_MINMOD, RECON_MP5 = 0, 1, 2, 3, 4
RIEMANN_HLL, RIEMANN_LLF = 0, 1
MINKOWSKI, KS_LOGSPH = 0, 1


@dataclass
class EosTable:
    """Tabulated EOS on nodes uniform in (ln rho, ln eps, Y_e): data[k, j, i] =
    (ln p, Gamma_1) at ln rho = lo[0] + i h0, ln eps = lo[1] + j h1,
    Y_e = lo[2] + k h2 (h_d = (hi[d] - lo[d]) / (n_d - 1)).  Gamma_1 is the
    adiabatic index d ln p / d ln rho at constant entropy (rho h c_s^2 =
    Gamma_1 p).  The tables here are synthetic: sampled from closed forms."""
    data: np.ndarray
    lo: tuple
    hi: tuple
    name: str = ""

    @property
    def n(self):
        return (self.data.shape[2], self.data.shape[1], self.data.shape[0])

    def nodes(self, d):
        return np.linspace(self.lo[d], self.hi[d], self.n[d])


TABLE_LO = (np.log(1e-14), np.log(1e-8), 0.05)
TABLE_HI = (np.log(1e3), np.log(1e3), 0.55)


IDEAL_LO = (np.log(1e-30), np.log(1e-30), 0.05)
IDEAL_HI = (np.log(1e10), np.log(1e10), 0.55)


def ideal_table(gamma, n=(64, 64, 6), lo=IDEAL_LO, hi=IDEAL_HI):
    """The ideal gas p = (gamma - 1) rho eps sampled on the table grid:
    ln p = ln(gamma - 1) + ln rho + ln eps, Gamma_1 = gamma (independent of
    Y_e).  Trilinear interpolation reproduces it exactly up to rounding; the
    default range is wide enough that no state of the test problems is
    clamped, so the table path must reproduce the ideal-gas path."""
    x = np.linspace(lo[0], hi[0], n[0])
    y = np.linspace(lo[1], hi[1], n[1])
    data = np.zeros((n[2], n[1], n[0], 2))
    data[..., 0] = np.log(gamma - 1.0) + x[None, None, :] + y[None, :, None]
    data[..., 1] = gamma
    return EosTable(data, tuple(lo), tuple(hi), name=f"ideal gamma={gamma:.6g}")


def synthetic_eos(rho, eps, ye, e0=0.2):
    """Closed-form EOS behind the synthetic table: an adiabatic index that
    falls from 5/3 to 4/3 once the specific energy exceeds a degeneracy-like
    scale e_c = e0 (rho Y_e)^(1/3):
        g = p / (rho eps) = 1/3 + (1/3) e_c / (e_c + eps).
    With k = e_c eps / (3 (e_c + eps)^2):  d ln p/d ln rho|eps = 1 + k/(3 g),
    d ln p/d ln eps|rho = 1 - k/g, and
        Gamma_1 = d ln p/d ln rho|eps + (p/(rho eps)) d ln p/d ln eps|rho
                = 1 + g - k (1 - 1/(3 g)).
    Returns (p, Gamma_1)."""
    ec = e0 * np.cbrt(rho * ye)
    g = (1.0 + ec / (ec + eps)) / 3.0
    k = ec * eps / (3.0 * (ec + eps) ** 2)
    return rho * eps * g, 1.0 + g - k * (1.0 - 1.0 / (3.0 * g))


def synthetic_table(n=(96, 96, 11), lo=TABLE_LO, hi=TABLE_HI, e0=0.2):
    """synthetic_eos sampled on the table grid (a stand-in for a nuclear
    table such as SFHo: p depends on all three of rho, eps and Y_e)."""
    x = np.linspace(lo[0], hi[0], n[0])
    y = np.linspace(lo[1], hi[1], n[1])
    z = np.linspace(lo[2], hi[2], n[2])
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    p, g1 = synthetic_eos(np.exp(X), np.exp(Y), Z, e0)
    data = np.stack([np.log(p), g1], axis=-1)
    return EosTable(np.ascontiguousarray(data), tuple(lo), tuple(hi), name=f"synthetic e0={e0}")


def with_ye(prob, ye, table=None):
    """The problem with the Y_e passive scalar: P gains the plane P[5] = ye
    (an array broadcast to the grid, or a function of the primitives
    ye(P) -> array), and the EOS becomes `table` when one is given."""
    P = prob.P
    yv = ye(P) if callable(ye) else ye
    prob.P = np.concatenate([P, np.broadcast_to(yv, P.shape[1:])[None]], axis=0).copy()
    prob.nscalar = 1
    prob.table = table
    return prob


def smooth_ye(prob, seed=11, base=0.3, amp=0.15):
    """Seeded smooth Y_e field of a periodic box: base + amp * (a few Fourier
    modes, scaled into [-1, 1])."""
    rng = np.random.default_rng(seed)
    x = [prob.centers(d) for d in range(3)]
    Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
    f = np.zeros(X.shape)
    for _ in range(3):
        kv = rng.integers(-2, 3, size=3)
        f += rng.uniform(0.5, 1.0) * np.cos(2 * np.pi * (kv[0] * X + kv[1] * Y + kv[2] * Z)
                                           + rng.uniform(0, 2 * np.pi))
    return base + amp * f / np.abs(f).max()


def torus_ye(P, rho_max=1.0):
    """Y_e of the torus: 0.5 in the atmosphere falling to 0.1 at the density
    maximum (a neutron-rich disc)."""
    return 0.5 - 0.4 * np.clip(P[0] / rho_max, 0.0, 1.0)


@dataclass
class Problem:
    n: tuple
    xmin: tuple
    xmax: tuple
    bc: tuple
    metric_kind: int = MINKOWSKI
    M: float = 1.0
    a: float = 0.0
    gamma: float = 4.0 / 3.0
    rho_flr0: float = 1e-20
    rho_flr_pow: float = 0.0
    u_flr0: float = 1e-22
    u_flr_pow: float = 0.0
    W_max: float = 50.0
    recon: int = RECON_PLM_MC
    riemann: int = RIEMANN_HLL
    weno_fv: int = 0
    cfl: float = 0.4
    ng: int = 4
    P: np.ndarray = None
    Bf: np.ndarray = None
    meta: dict = field(default_factory=dict)
    nscalar: int = 0              # 1: P[5] = Y_e, evolved as a passive scalar
    table: "EosTable" = None      # tabulated EOS (needs nscalar = 1); None = ideal gas

    @property
    def dx(self):
        return tuple((self.xmax[d] - self.xmin[d]) / self.n[d] for d in range(3))

    @property
    def shape(self):
        return tuple(self.n[2 - d] + 2 * self.ng for d in range(3))   # (s3, s2, s1)

    @property
    def ncell(self):
        s = self.shape
        return s[0] * s[1] * s[2]

    def centers(self, d):
        """Cell-centre coordinate along d for every index (ghosts included)."""
        idx = np.arange(self.n[d] + 2 * self.ng)
        return self.xmin[d] + (idx - self.ng + 0.5) * self.dx[d]

    def faces(self, d):
        idx = np.arange(self.n[d] + 2 * self.ng)
        return self.xmin[d] + (idx - self.ng) * self.dx[d]

    def interior(self):
        g = self.ng
        return (slice(g, g + self.n[2]), slice(g, g + self.n[1]), slice(g, g + self.n[0]))


def splitmix64(x):
    """SplitMix64 output for uint64 array x (Steele, Lea & Flood 2014)."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed, idx):
    """Uniform [0,1) doubles from SplitMix64(seed xor index), 53-bit mantissa."""
    z = splitmix64(np.uint64(seed) ^ np.asarray(idx, dtype=np.uint64))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


# ---------------------------------------------------------------------------
# Uniform state and random perturbations (unit tests)
# ---------------------------------------------------------------------------

def uniform_box(n, rho=1.0, ut=(0.0, 0.0, 0.0), u=1.0, B=(0.0, 0.0, 0.0), **kw):
    prob = Problem(n=tuple(n), xmin=(0.0, 0.0, 0.0), xmax=(1.0, 1.0, 1.0),
                   bc=(BC_PERIODIC,) * 6, **kw)
    P = np.zeros((5,) + prob.shape)
    P[0] = rho
    for d in range(3):
        P[1 + d] = ut[d]
    P[4] = u
    Bf = np.zeros((3,) + prob.shape)
    for d in range(3):
        Bf[d] = B[d]
    prob.P, prob.Bf = P, Bf
    return prob


def random_smooth_box(n, seed=0, amp=0.05, B0=(0.3, 0.2, 0.1), **kw):
    """Periodic box with a few seeded Fourier modes in every primitive and a
    divergence-free face field from a periodic vector potential."""
    prob = uniform_box(n, rho=1.0, u=1.0, **kw)
    rng = np.random.default_rng(seed)
    x = [prob.centers(d) for d in range(3)]
    xf = [prob.faces(d) for d in range(3)]
    Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
    P = prob.P
    for q, base in enumerate([1.0, 0.0, 0.0, 0.0, 1.0]):
        f = np.full(X.shape, base)
        for _ in range(3):
            kv = rng.integers(-2, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            f = f + amp * rng.uniform(0.5, 1.0) * np.cos(
                2 * np.pi * (kv[0] * X + kv[1] * Y + kv[2] * Z) + ph)
        P[q] = f
    # A_d at d-edges; B = curl A
    modes = [(rng.integers(-2, 3, size=3), rng.uniform(0, 2 * np.pi), rng.uniform(-1, 1, 3))
             for _ in range(3)]

    def A(comp, Xe, Ye, Ze):
        out = np.zeros(Xe.shape)
        for kv, ph, c in modes:
            out += amp * c[comp] * np.sin(2 * np.pi * (kv[0] * Xe + kv[1] * Ye + kv[2] * Ze) + ph)
        return out
    prob.Bf = _curl_faces(prob, A, B0)
    return prob


def _curl_faces(prob, A, B0, sqrtg_face=None):
    """Face field B^d = B0_d + (curl A)_d with A_c sampled at c-edges (Stokes
    on each face, so the discrete divergence vanishes to rounding)."""
    xc = [prob.centers(d) for d in range(3)]
    xf = [prob.faces(d) for d in range(3)]
    dx = prob.dx
    Bf = np.zeros((3,) + prob.shape)

    def grid(a, b, c):
        Z, Y, X = np.meshgrid(c, b, a, indexing="ij")
        return X, Y, Z

    def up(a, d):
        return a + dx[d]
    # B1 on x1-faces (x1 face, x2 centre, x3 centre)
    X, Y, Z = grid(xf[0], xc[1], xc[2])
    Bf[0] = B0[0] + (A(2, X, Y + 0.5 * dx[1], Z) - A(2, X, Y - 0.5 * dx[1], Z)) / dx[1] \
        - (A(1, X, Y, Z + 0.5 * dx[2]) - A(1, X, Y, Z - 0.5 * dx[2])) / dx[2]
    X, Y, Z = grid(xc[0], xf[1], xc[2])
    Bf[1] = B0[1] + (A(0, X, Y, Z + 0.5 * dx[2]) - A(0, X, Y, Z - 0.5 * dx[2])) / dx[2] \
        - (A(2, X + 0.5 * dx[0], Y, Z) - A(2, X - 0.5 * dx[0], Y, Z)) / dx[0]
    X, Y, Z = grid(xc[0], xc[1], xf[2])
    Bf[2] = B0[2] + (A(1, X + 0.5 * dx[0], Y, Z) - A(1, X - 0.5 * dx[0], Y, Z)) / dx[0] \
        - (A(0, X, Y + 0.5 * dx[1], Z) - A(0, X, Y - 0.5 * dx[1], Z)) / dx[1]
    return Bf


# ---------------------------------------------------------------------------
# Linear magnetosonic wave in a periodic box (Minkowski)
# ---------------------------------------------------------------------------

def sr_wave_eigen(rho, p, gamma, B, nhat, mode="fast"):
    """Right-going plane-wave eigenmode of linearised special-relativistic
    ideal MHD about a static uniform state.

    With enthalpy density w = rho + p gamma/(gamma-1), the velocity amplitude
    solves  K dv = V^2 M dv  with
        M = (w + B^2) I - B B^T
        K = (gamma p + B^2) n n^T - (n.B)(n B^T + B n^T) + (n.B)^2 I,
    obtained from linearising the conserved momentum (w + B^2) v - (B.v) B and
    its flux with dp = gamma p (n.dv)/V, drho = rho (n.dv)/V and
    dB = -[(n.B) dv - (n.dv) B]/V.  Returns (V, R) with R the primitive
    eigenvector (rho, ut1, ut2, ut3, u, B1, B2, B3) scaled to unit 2-norm.
    """
    import scipy.linalg
    n = np.asarray(nhat, float) / np.linalg.norm(nhat)
    B = np.asarray(B, float)
    w = rho + gamma * p / (gamma - 1.0)
    nB = n @ B
    M = (w + B @ B) * np.eye(3) - np.outer(B, B)
    K = (gamma * p + B @ B) * np.outer(n, n) - nB * (np.outer(n, B) + np.outer(B, n)) \
        + nB * nB * np.eye(3)
    vals, vecs = scipy.linalg.eigh(K, M)
    idx = {"slow": 0, "alfven": 1, "fast": 2}[mode]
    V = np.sqrt(vals[idx])
    dv = vecs[:, idx]
    if n @ dv < 0 and mode != "alfven":
        dv = -dv
    drho = rho * (n @ dv) / V
    dp = gamma * p * (n @ dv) / V
    dB = -(nB * dv - (n @ dv) * B) / V
    R = np.concatenate([[drho], dv, [dp / (gamma - 1.0)], dB])
    return V, R / np.linalg.norm(R)


def linear_wave(n=(32, 32, 32), k=(1, 1, 1), amp=1e-6, rho=1.0, p=1.0, gamma=4.0 / 3.0,
                B=(1.0, np.sqrt(2.0), 0.5), mode="fast", recon=RECON_PLM_MC,
                riemann=RIEMANN_HLL, cfl=0.4):
    """Periodic unit box carrying one right-going eigenmode along integer k."""
    box_len = [1.0, 1.0, 1.0]
    for d in range(3):
        if k[d] == 0 and n[d] == 1:
            box_len[d] = 1.0
    prob = Problem(n=tuple(n), xmin=(0.0, 0.0, 0.0), xmax=tuple(box_len),
                   bc=(BC_PERIODIC,) * 6, gamma=gamma, recon=recon, riemann=riemann, cfl=cfl)
    kvec = 2.0 * np.pi * np.asarray(k, float)
    nhat = kvec / np.linalg.norm(kvec)
    V, R = sr_wave_eigen(rho, p, gamma, B, nhat, mode)
    x = [prob.centers(d) for d in range(3)]
    Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
    phase = np.cos(kvec[0] * X + kvec[1] * Y + kvec[2] * Z)
    P = np.zeros((5,) + prob.shape)
    base = [rho, 0.0, 0.0, 0.0, p / (gamma - 1.0)]
    for q in range(5):
        P[q] = base[q] + amp * R[q] * phase
    dB = amp * R[5:8]
    kk = kvec @ kvec
    avec = np.cross(dB, kvec) / kk    # A = (dB x k)/|k|^2 sin(k.x)  ->  curl A = dB cos(k.x)

    def A(comp, Xe, Ye, Ze):
        return avec[comp] * np.sin(kvec[0] * Xe + kvec[1] * Ye + kvec[2] * Ze)
    prob.Bf = _curl_faces(prob, A, B)
    prob.P = P
    prob.meta = {"speed": V, "eigvec": R, "k": kvec, "amp": amp,
                 "period": (2.0 * np.pi / np.sqrt(kk)) / V}
    return prob


# ---------------------------------------------------------------------------
# Shock tube (Minkowski, B = 0, along x1)
# ---------------------------------------------------------------------------

def shock_tube(n1=400, left=(10.0, 0.0, 13.33), right=(1.0, 0.0, 1e-6), gamma=5.0 / 3.0,
               x0=0.5, recon=RECON_PLM_MC, riemann=RIEMANN_HLL, cfl=0.4):
    """States (rho, v^x, p).  Outflow along x1, one cell in x2 and x3."""
    prob = Problem(n=(n1, 1, 1), xmin=(0.0, 0.0, 0.0), xmax=(1.0, 1.0, 1.0),
                   bc=(BC_OUTFLOW, BC_OUTFLOW, BC_PERIODIC, BC_PERIODIC, BC_PERIODIC,
                       BC_PERIODIC), gamma=gamma, recon=recon, riemann=riemann, cfl=cfl)
    x = prob.centers(0)
    P = np.zeros((5,) + prob.shape)
    for st, mask in ((left, x < x0), (right, x >= x0)):
        rho, v, p = st
        W = 1.0 / np.sqrt(1.0 - v * v)
        P[0][..., mask] = rho
        P[1][..., mask] = W * v
        P[4][..., mask] = p / (gamma - 1.0)
    prob.P = P
    prob.Bf = np.zeros((3,) + prob.shape)
    prob.meta = {"left": left, "right": right, "x0": x0}
    return prob


# ---------------------------------------------------------------------------
# Michel (Bondi) inflow on Schwarzschild in Kerr-Schild coordinates
# ---------------------------------------------------------------------------

def michel_solution(r, rc=8.0, gamma=4.0 / 3.0, M=1.0):
    """Transonic polytropic radial inflow (Michel 1972) with sonic radius rc.

    T = p/rho, n = 1/(gamma-1), rho = T^n (K = 1).  Conserved along the flow:
    C1 = T^n u^r r^2 and C2 = (1 + (n+1)T)^2 (1 - 2M/r + (u^r)^2).  At the sonic
    point (u^r)^2 = M/(2 rc) and the sound speed^2 V^2 = u^2/(1 - 3u^2) fixes T.
    Returns (rho, u^r, T) arrays.
    """
    nn = 1.0 / (gamma - 1.0)
    uc2 = M / (2.0 * rc)
    Vc2 = uc2 / (1.0 - 3.0 * uc2)
    Tc = nn * Vc2 / ((nn + 1.0) * (1.0 - nn * Vc2))
    C1 = Tc ** nn * np.sqrt(uc2) * rc * rc
    C2 = (1.0 + (nn + 1.0) * Tc) ** 2 * (1.0 - 2.0 * M / rc + uc2)
    import scipy.optimize as so

    def f(T, rr):
        ur = C1 / (rr * rr * T ** nn)
        return (1.0 + (nn + 1.0) * T) ** 2 * (1.0 - 2.0 * M / rr + ur * ur) - C2

    rr = np.atleast_1d(np.asarray(r, float))
    T = np.zeros_like(rr)
    for i, x in enumerate(rr):
        if abs(x - rc) < 1e-12:
            T[i] = Tc
            continue
        # f has one minimum in T; the two roots straddle it.
        tm = so.minimize_scalar(lambda t: f(t, x), bounds=(1e-12, 10.0), method="bounded",
                                options={"xatol": 1e-14}).x
        if x > rc:       # subsonic branch: the larger-T root
            lo, hi = tm, tm
            while f(hi, x) < 0:
                hi *= 2.0
            T[i] = so.brentq(lambda t: f(t, x), tm, hi, xtol=1e-15, rtol=1e-15)
        else:            # supersonic branch: the smaller-T root
            lo = tm
            while f(lo, x) < 0:
                lo *= 0.5
            T[i] = so.brentq(lambda t: f(t, x), lo, tm, xtol=1e-15, rtol=1e-15)
    rho = T ** nn
    ur = -C1 / (rr * rr * T ** nn)
    return rho, ur, T


def _ks_lapse_shift_r(r, th, a=0.0, M=1.0):
    sig = r * r + a * a * np.cos(th) ** 2
    z = 2.0 * M * r / sig
    return 1.0 / np.sqrt(1.0 + z), z / (1.0 + z), z


def bondi(n1=64, rin=2.5, rout=20.0, rc=8.0, gamma=4.0 / 3.0, dtheta=0.1,
          recon=RECON_PLM_MC, riemann=RIEMANN_HLL, cfl=0.4):
    """Radial Michel inflow, a = 0, one cell in theta (equator) and phi; the
    x1 ghosts hold the exact solution (fixed boundary)."""
    prob = Problem(n=(n1, 1, 1), xmin=(np.log(rin), 0.5 * np.pi - 0.5 * dtheta, 0.0),
                   xmax=(np.log(rout), 0.5 * np.pi + 0.5 * dtheta, 2.0 * np.pi),
                   bc=(BC_FIXED, BC_FIXED, BC_OUTFLOW, BC_OUTFLOW, BC_PERIODIC, BC_PERIODIC),
                   metric_kind=KS_LOGSPH, M=1.0, a=0.0, gamma=gamma, recon=recon,
                   riemann=riemann, cfl=cfl)
    r = np.exp(prob.centers(0))
    rho, ur, T = michel_solution(r, rc, gamma)
    alpha, betar, z = _ks_lapse_shift_r(r, 0.5 * np.pi)
    # KS: g_tt = -(1-z), g_tr = z, g_rr = 1+z ; solve for u^t (future root)
    A = -(1.0 - z)
    Bq = 2.0 * z * ur
    C = (1.0 + z) * ur * ur + 1.0
    ut = (-Bq - np.sqrt(Bq * Bq - 4.0 * A * C)) / (2.0 * A)
    # u-tilde^r = u^r + u^t beta^r ; x1 = ln r  ->  divide by r
    utr = (ur + ut * betar) / r
    P = np.zeros((5,) + prob.shape)
    P[0] = rho[None, None, :]
    P[1] = utr[None, None, :]
    P[4] = (rho * T / (gamma - 1.0))[None, None, :]
    prob.P = P
    prob.Bf = np.zeros((3,) + prob.shape)
    prob.meta = {"rc": rc}
    return prob


# ---------------------------------------------------------------------------
# Fishbone-Moncrief torus around a Kerr black hole (Kerr-Schild, x1 = ln r)
# ---------------------------------------------------------------------------

def _bl_tphi(r, th, a, M=1.0):
    """Boyer-Lindquist (t, phi) block of g_{mu nu} and its determinant."""
    s2 = np.sin(th) ** 2
    sig = r * r + a * a * np.cos(th) ** 2
    delta = r * r - 2.0 * M * r + a * a
    Acal = (r * r + a * a) ** 2 - delta * a * a * s2
    gtt = -(1.0 - 2.0 * M * r / sig)
    gtp = -2.0 * M * a * r * s2 / sig
    gpp = Acal * s2 / sig
    return gtt, gtp, gpp


def fm_ell(rmax, a, M=1.0):
    """ell = u^t u_phi of the prograde equatorial circular geodesic at rmax
    (Bardeen, Press & Teukolsky 1972), the Fishbone-Moncrief constant that puts
    the pressure maximum at rmax."""
    sM = np.sqrt(M)
    den = rmax ** 0.75 * np.sqrt(rmax ** 1.5 - 3.0 * M * np.sqrt(rmax) + 2.0 * a * sM)
    ut = (rmax ** 1.5 + a * sM) / den
    uphi = sM * (rmax * rmax - 2.0 * a * sM * np.sqrt(rmax) + a * a) / den
    return ut * uphi


def fm_lnh(r, th, a, ell, M=1.0):
    """ln h + const for the constant-(u^t u_phi) torus.

    Circular flow u = u^t (1, 0, 0, Omega) with u^t u_phi = ell and u.u = -1
    gives u_phi^2 = Z, Z^2 + g_phiphi Z + D ell^2 = 0 (D = det of the (t,phi)
    block), and the Euler equation reduces to d ln h = ell d(u_t/u_phi) - d ln u_phi.
    Returns (ln h + const, u_t, u_phi)."""
    gtt, gtp, gpp = _bl_tphi(r, th, a, M)
    D = gtt * gpp - gtp * gtp
    Z = 0.5 * (-gpp + np.sqrt(gpp * gpp - 4.0 * D * ell * ell))
    uphi = np.sqrt(Z)
    gitt, gitp = gpp / D, -gtp / D
    ut_low = (ell - gitp * Z) / (gitt * uphi)
    return ell * ut_low / uphi - np.log(uphi), ut_low, uphi


def torus(n=(128, 128, 128), a=0.9375, rin=6.0, rmax=12.0, gamma=13.0 / 9.0, rmin=1.2,
          rout=40.0, seed=1, noise=4e-2, beta=100.0, rho_flr0=1e-6, rho_flr_pow=1.5,
          u_flr0=1e-8, u_flr_pow=2.5, recon=RECON_WENO5Z, riemann=RIEMANN_LLF, cfl=0.4,
          W_max=50.0):
    """Fishbone-Moncrief torus (rho_max = 1) with a seeded pressure noise and a
    poloidal loop field A_phi = max(rho/rho_max - 0.2, 0) scaled so that
    max p / max(b^2/2) = beta, on Kerr-Schild coordinates x1 = ln r, x2 = theta,
    x3 = phi.  Outside the torus the gas sits at the floor values with zero
    Eulerian velocity."""
    M = 1.0
    prob = Problem(n=tuple(n), xmin=(np.log(rmin), 0.0, 0.0),
                   xmax=(np.log(rout), np.pi, 2.0 * np.pi),
                   bc=(BC_OUTFLOW, BC_OUTFLOW, BC_POLAR, BC_POLAR, BC_PERIODIC, BC_PERIODIC),
                   metric_kind=KS_LOGSPH, M=M, a=a, gamma=gamma, rho_flr0=rho_flr0,
                   rho_flr_pow=rho_flr_pow, u_flr0=u_flr0, u_flr_pow=u_flr_pow, W_max=W_max,
                   recon=recon, riemann=riemann, cfl=cfl)
    ell = fm_ell(rmax, a, M)
    lnh_in = fm_lnh(rin, 0.5 * np.pi, a, ell, M)[0]
    lnh_max = fm_lnh(rmax, 0.5 * np.pi, a, ell, M)[0] - lnh_in
    hmax = np.exp(lnh_max)
    K = (hmax - 1.0) * (gamma - 1.0) / gamma     # rho(rmax) = 1

    def rho_of(r, th):
        with np.errstate(invalid="ignore", divide="ignore"):
            lnh, ut_low, uphi = fm_lnh(r, th, a, ell, M)
            lnh = lnh - lnh_in
            inside = (lnh > 0.0) & (r >= rin) & np.isfinite(lnh)
            h = np.where(inside, np.exp(np.where(inside, lnh, 0.0)), 1.0)
            rho = np.where(inside,
                           ((h - 1.0) * (gamma - 1.0) / (K * gamma)) ** (1.0 / (gamma - 1.0)),
                           0.0)
        return rho, inside, ut_low, uphi

    s1, s2 = prob.n[0] + 2 * prob.ng, prob.n[1] + 2 * prob.ng
    r1 = np.exp(prob.centers(0))
    th1 = prob.centers(1)
    # ghost rows beyond the poles take their mirror theta (the field there is
    # overwritten by the boundary fill anyway; this keeps the numbers finite)
    thc = np.clip(th1, 1e-12, np.pi - 1e-12)
    R2, TH2 = np.meshgrid(r1, thc, indexing="xy")        # shape (s2, s1)
    rho, inside, ut_low, uphi = rho_of(R2, TH2)
    p = np.where(inside, K * rho ** gamma, 0.0)

    # four-velocity of the torus (BL and KS share u^t, u^phi when u^r = 0)
    gtt, gtp, gpp = _bl_tphi(R2, TH2, a, M)
    D = gtt * gpp - gtp * gtp
    gitt, gitp, gipp = gpp / D, -gtp / D, gtt / D
    with np.errstate(invalid="ignore"):
        ucon_t = gitt * ut_low + gitp * uphi
        ucon_p = gitp * ut_low + gipp * uphi
    alpha, betar, z = _ks_lapse_shift_r(R2, TH2, a, M)
    # u-tilde^i = u^i + u^t beta^i ; beta^1 = beta^r / r in x1 = ln r ; beta^phi = 0
    ut1 = np.where(inside, ucon_t * betar / R2, 0.0)
    ut3 = np.where(inside, ucon_p, 0.0)

    rflr = rho_flr0 * R2 ** (-rho_flr_pow)
    uflr = u_flr0 * R2 ** (-u_flr_pow)
    rho_f = np.maximum(rho, rflr)
    u_f = np.maximum(p / (gamma - 1.0), uflr)

    shp = prob.shape
    P = np.zeros((5,) + shp)
    P[0] = rho_f[None]
    P[1] = ut1[None]
    P[3] = ut3[None]
    # seeded pressure noise inside the torus, keyed by the global cell index
    cell = np.arange(prob.ncell, dtype=np.uint64).reshape(shp)
    xi = uniform01(seed, cell)
    pert = 1.0 + noise * (xi - 0.5)
    P[4] = np.where(inside[None], u_f[None] * pert, u_f[None])

    # vector potential at (x1-face, x2-face) edges, axisymmetric
    rf = np.exp(prob.faces(0))
    thf = np.clip(prob.faces(1), 0.0, np.pi)
    RF, THF = np.meshgrid(rf, thf, indexing="xy")
    rhoe, _, _, _ = rho_of(RF, np.clip(THF, 1e-12, np.pi - 1e-12))
    Aphi = np.maximum(rhoe - 0.2, 0.0)
    Aphi[np.abs(THF) < 1e-14] = 0.0
    Aphi[np.abs(THF - np.pi) < 1e-14] = 0.0
    dx1, dx2 = prob.dx[0], prob.dx[1]
    Bf = np.zeros((3,) + shp)
    # B1 (x1 faces) = d_2 A_3 ; B2 (x2 faces) = -d_1 A_3   (densitized)
    b1 = np.zeros((s2, s1))
    b1[:-1, :] = (Aphi[1:, :] - Aphi[:-1, :]) / dx2
    b2 = np.zeros((s2, s1))
    b2[:, :-1] = -(Aphi[:, 1:] - Aphi[:, :-1]) / dx1
    Bf[0] = b1[None]
    Bf[1] = b2[None]

    # normalise: max p / max(b^2/2) = beta, with b^2 from the cell-centre field
    sqrtgam = _ks_sqrtgam(R2, TH2, a, M)
    Bc1 = 0.5 * (b1[:, :] + np.roll(b1, -1, axis=1)) / sqrtgam
    Bc2 = 0.5 * (b2[:, :] + np.roll(b2, -1, axis=0)) / sqrtgam
    b2fluid = _ks_b2(R2, TH2, a, M, ut1, np.zeros_like(ut1), ut3, Bc1, Bc2)
    g = prob.ng
    sl = (slice(g, g + prob.n[1]), slice(g, g + prob.n[0]))
    pmax = np.max(p[sl])
    bmax = np.max(b2fluid[sl])
    scale = np.sqrt(2.0 * pmax / (beta * bmax)) if bmax > 0 else 0.0
    Bf *= scale
    prob.P, prob.Bf = P, Bf
    prob.meta = {"ell": ell, "K": K, "pmax": pmax, "field_scale": scale, "seed": seed}
    return prob


def _ks_gamma_ij(r, th, a, M):
    """Spatial KS metric in (x1 = ln r, theta, phi): nonzero g11, g13, g22, g33."""
    s2 = np.sin(th) ** 2
    sig = r * r + a * a * np.cos(th) ** 2
    z = 2.0 * M * r / sig
    g11 = r * r * (1.0 + z)
    g13 = -a * (1.0 + z) * s2 * r
    g22 = sig
    g33 = s2 * (sig + a * a * (1.0 + z) * s2)
    return g11, g13, g22, g33


def _ks_sqrtgam(r, th, a, M):
    g11, g13, g22, g33 = _ks_gamma_ij(r, th, a, M)
    return np.sqrt(g22 * (g11 * g33 - g13 * g13))


def _ks_b2(r, th, a, M, u1, u2, u3, B1, B2):
    """Fluid-frame b^2 for the IC normalisation (B^3 = 0)."""
    g11, g13, g22, g33 = _ks_gamma_ij(r, th, a, M)
    alpha, betar, z = _ks_lapse_shift_r(r, th, a, M)
    W = np.sqrt(1.0 + g11 * u1 * u1 + 2.0 * g13 * u1 * u3 + g22 * u2 * u2 + g33 * u3 * u3)
    v1, v2, v3 = u1 / W, u2 / W, u3 / W
    vl1 = g11 * v1 + g13 * v3
    vl2 = g22 * v2
    Bv = B1 * vl1 + B2 * vl2
    BB = g11 * B1 * B1 + g22 * B2 * B2
    b0 = W * Bv / alpha
    return (BB + alpha * alpha * b0 * b0) / (W * W)


# ---------------------------------------------------------------------------
# Random primitive states for inversion tests and the learned-guess data set
# ---------------------------------------------------------------------------

def random_prims(count, seed=3, rho=(1e-8, 1.0), p_over_rho=(1e-6, 10.0), W=(1.0, 50.0),
                 sigma=(1e-4, 100.0), gamma=13.0 / 9.0):
    """Minkowski primitive samples: log-uniform rho, p/rho, W, sigma = b^2/rho;
    isotropic directions of v and B; |B| chosen so that b^2 = sigma rho.
    Returns dict of arrays rho, ut[3], u, B[3] (contravariant, flat metric)."""
    rng = np.random.default_rng(seed)

    def logu(lo, hi, size):
        return np.exp(rng.uniform(np.log(lo), np.log(hi), size))

    def iso(size):
        v = rng.normal(size=(size, 3))
        return v / np.linalg.norm(v, axis=1, keepdims=True)
    r = logu(*rho, count)
    pr = logu(*p_over_rho, count)
    Wl = logu(max(W[0], 1.0 + 1e-12), W[1], count) if W[0] > 1.0 else \
        1.0 + logu(1e-6, W[1] - 1.0, count)
    sg = logu(*sigma, count)
    vhat = iso(count)
    bhat = iso(count)
    vmag = np.sqrt(1.0 - 1.0 / (Wl * Wl))
    v = vhat * vmag[:, None]
    b2 = sg * r
    Bmag = np.sqrt(b2 / (1.0 / (Wl * Wl) + (np.sum(bhat * v, axis=1)) ** 2))
    B = bhat * Bmag[:, None]
    ut = v * Wl[:, None]
    u = pr * r / (gamma - 1.0)
    return {"rho": r, "ut": ut, "u": u, "B": B, "W": Wl, "gamma": gamma}


# ---------------------------------------------------------------------------
# Uneven meshblock layouts (batching)
# ---------------------------------------------------------------------------

def octree_layout(n, base=64, smallest=16, p_split=(0.45, 0.35), dense=None, p_dense=(0.9, 0.6),
                  seed=7):
    """Seeded octree cover of a root grid n[3] by cubic blocks of base, base/2,
    ... down to `smallest` cells.  A block of size s splits into 8 children
    with probability p_split[k] (k = level of s below base), or p_dense[k] when
    dense(lo, size) says it holds dense gas.  Returns (nx, lloc) flat lists."""
    rng = np.random.default_rng(seed)
    nx, lloc = [], []

    def visit(lo, s, k):
        if s > smallest:
            p = p_split[k] if k < len(p_split) else 0.0
            if dense is not None and dense(lo, s):
                p = p_dense[k] if k < len(p_dense) else 0.0
            if rng.uniform() < p:
                h = s // 2
                for dz in (0, h):
                    for dy in (0, h):
                        for dx in (0, h):
                            visit((lo[0] + dx, lo[1] + dy, lo[2] + dz), h, k + 1)
                return
        nx.extend([s, s, s])
        lloc.extend(list(lo))

    for z in range(0, n[2], base):
        for y in range(0, n[1], base):
            for x in range(0, n[0], base):
                visit((x, y, z), base, 0)
    return nx, lloc


def torus_dense_fn(prob, thresh=1e-2):
    """dense(lo, size): does the block's cube hold rho > thresh * rho_max?"""
    g = prob.ng
    rho = prob.P[0][g:-g, g:-g, g:-g]          # (z, y, x)
    big = rho > thresh * rho.max()

    def dense(lo, s):
        return bool(big[lo[2]:lo[2] + s, lo[1]:lo[1] + s, lo[0]:lo[0] + s].any())
    return dense


def batch_layout(prob, target=640, base=64, seed=7):
    """Octree layout of the torus with about `target` blocks: the split
    probabilities are scaled (deterministically, from the seed) until the
    block count is the closest to the target."""
    dense = torus_dense_fn(prob)
    best = None
    for scale in np.linspace(0.2, 2.0, 181):
        ps = tuple(min(1.0, scale * p) for p in (0.45, 0.35))
        pd = tuple(min(1.0, scale * p) for p in (0.9, 0.6))
        nx, lloc = octree_layout(prob.n, base, 16, ps, dense, pd, seed)
        nb = len(nx) // 3
        if best is None or abs(nb - target) < abs(best[0] - target):
            best = (nb, nx, lloc)
    return best[1], best[2]


# ---------------------------------------------------------------------------
# Two-level block meshes
# ---------------------------------------------------------------------------

def two_level_layout(root_n, node, dense, p_coarse=(0.5,), p_fine=(0.5, 0.35), smallest=16,
                     seed=7):
    """Seeded two-level block layout.  The level-0 root grid root_n[3] is cut
    into node^3 regions; a region where dense(lo, node) holds is refined into a
    (2 node)^3 region of level-1 cells, the others stay at level 0.  Each region
    is then split by the seeded octree (p_coarse / p_fine: split probability
    per octree depth) down to `smallest` cells.  Returns flat lists
    (level, nx, lloc), lloc in cells of the block's own level."""
    rng = np.random.default_rng(seed)
    level, nx, lloc = [], [], []

    def visit(lev, lo, s, k, probs):
        if s > smallest and k < len(probs) and rng.uniform() < probs[k]:
            h = s // 2
            for dz in (0, h):
                for dy in (0, h):
                    for dx in (0, h):
                        visit(lev, (lo[0] + dx, lo[1] + dy, lo[2] + dz), h, k + 1, probs)
            return
        level.append(lev)
        nx.extend([s, s, s])
        lloc.extend(list(lo))

    for d in range(3):
        if root_n[d] % node:
            raise ValueError("root grid must be a multiple of the region size")
    for z in range(0, root_n[2], node):
        for y in range(0, root_n[1], node):
            for x in range(0, root_n[0], node):
                if dense((x, y, z), node):
                    visit(1, (2 * x, 2 * y, 2 * z), 2 * node, 0, p_fine)
                else:
                    visit(0, (x, y, z), node, 0, p_coarse)
    return level, nx, lloc


def fine_dense_fn(prob_fine, thresh=1e-2):
    """dense(lo, size) on level-0 regions: does the region hold a level-1
    cell of prob_fine with rho > thresh * rho_max?"""
    g = prob_fine.ng
    rho = prob_fine.P[0][g:-g, g:-g, g:-g]
    big = rho > thresh * rho.max()

    def dense(lo, s):
        return bool(big[2 * lo[2]:2 * (lo[2] + s), 2 * lo[1]:2 * (lo[1] + s),
                        2 * lo[0]:2 * (lo[0] + s)].any())
    return dense


def amr_layout(prob_fine, target=640, node=32, smallest=16, seed=7, thresh=1e-2):
    """Two-level layout of a problem given at the level-1 resolution (level 0 =
    half of it): regions holding rho > thresh rho_max are refined; the octree
    split probabilities are scaled (deterministically) until the block count
    is the closest to `target`."""
    root_n = tuple(n // 2 for n in prob_fine.n)
    dense = fine_dense_fn(prob_fine, thresh)
    best = None
    for scale in np.linspace(0.1, 2.0, 96):
        pc = (min(1.0, 0.5 * scale),)
        pf = (min(1.0, 0.8 * scale), min(1.0, 0.45 * scale))
        lay = two_level_layout(root_n, node, dense, pc, pf, smallest, seed)
        nb = len(lay[0])
        if best is None or abs(nb - target) < abs(len(best[0]) - target):
            best = lay
    return best


def coarse_problem(prob_fine):
    """Level-0 description of a problem given at the level-1 resolution (same
    domain and physics, half the cells, no state arrays)."""
    import copy
    root = copy.copy(prob_fine)
    root.n = tuple(n // 2 for n in prob_fine.n)
    root.P = None
    root.Bf = None
    root.meta = dict(prob_fine.meta)
    return root


def mesh_blocks(prob_fine, level, nx, lloc):
    """Per-block padded initial arrays (P [5, s3, s2, s1], Bf [3, ...]) of a
    two-level layout: level-1 blocks copy prob_fine's interior; level-0 blocks
    hold its restriction (cell means of the 8 children; face means of the 4
    child faces, so the coarse field is divergence-free whenever the fine one
    is).  Ghost zones are left zero."""
    g = prob_fine.ng
    Pf, Bff = prob_fine.P, prob_fine.Bf
    nx = np.asarray(nx).reshape(-1, 3)
    lloc = np.asarray(lloc).reshape(-1, 3)
    Ps, Bs = [], []
    for b in range(len(level)):
        n = nx[b]
        s = n + 2 * g
        P = np.zeros((5, s[2], s[1], s[0]))
        Bf = np.zeros((3, s[2], s[1], s[0]))
        lo = lloc[b]
        if level[b] == 1:
            P[:, g:g + n[2], g:g + n[1], g:g + n[0]] = \
                Pf[:, g + lo[2]:g + lo[2] + n[2], g + lo[1]:g + lo[1] + n[1], g + lo[0]:g + lo[0] + n[0]]
            for c in range(3):
                e = [n[d] + (1 if d == c else 0) for d in range(3)]
                Bf[c, g:g + e[2], g:g + e[1], g:g + e[0]] = \
                    Bff[c, g + lo[2]:g + lo[2] + e[2], g + lo[1]:g + lo[1] + e[1],
                        g + lo[0]:g + lo[0] + e[0]]
        else:
            f0 = 2 * lo
            blk = Pf[:, g + f0[2]:g + f0[2] + 2 * n[2], g + f0[1]:g + f0[1] + 2 * n[1],
                     g + f0[0]:g + f0[0] + 2 * n[0]]
            acc = np.zeros((5, n[2], n[1], n[0]))
            for dz in (0, 1):
                for dy in (0, 1):
                    for dx in (0, 1):
                        acc += blk[:, dz::2, dy::2, dx::2]
            P[:, g:g + n[2], g:g + n[1], g:g + n[0]] = 0.125 * acc
            for c in range(3):
                e = [n[d] + (1 if d == c else 0) for d in range(3)]
                # child faces: normal index 2 F, transverse 2 t + {0, 1}
                ext = [2 * n[d] if d != c else 2 * n[d] + 1 for d in range(3)]
                fb = Bff[c, g + f0[2]:g + f0[2] + ext[2], g + f0[1]:g + f0[1] + ext[1],
                         g + f0[0]:g + f0[0] + ext[0]]
                sl = [None, None, None]
                acc = 0.0
                for t1 in (0, 1):
                    for t2 in (0, 1):
                        off = [0, 0, 0]
                        off[(c + 1) % 3] = t1
                        off[(c + 2) % 3] = t2
                        for d in range(3):
                            sl[d] = slice(off[d], ext[d], 2)
                        acc = acc + fb[sl[2], sl[1], sl[0]]
                Bf[c, g:g + e[2], g:g + e[1], g:g + e[0]] = 0.25 * acc
        Ps.append(P)
        Bs.append(Bf)
    return Ps, Bs


# ---------------------------------------------------------------------------
# Gray M1 radiation fields and opacities (synthetic)
# ---------------------------------------------------------------------------

M1_SPECIES = ("nu_e", "nu_e_bar", "nu_x")


def m1_fields(prob, seed=21, e0=(1e-3, 7e-4, 4e-4), fmax=0.9, a_abs=(10.0, 30.0, 100.0),
              a_scat=(5.0, 5.0, 20.0), c_eq=(0.3, 0.2, 0.1)):
    """Seeded radiation moments and opacities of three species on a problem's
    grid (ghosts included).  Returns (R, kap):
      R[s] = sqrt(gamma) (E, F_1, F_2, F_3) with E = e0_s (1 + 0.5 xi) and a
      flux F_i = f E nhat_i of flux factor f = fmax xi' (|F| measured with
      gamma^ij), nhat a seeded direction per cell;
      kap[s] = (kappa_J, kappa_H, J_eq) = (a_abs_s rho, (a_abs_s + a_scat_s) rho,
      c_eq_s u): constant opacities per unit density (absorption plus elastic
      scattering for kappa_H) and an equilibrium energy density proportional
      to the gas energy.
    The geometry (gamma_ij, sqrt(gamma)) comes from `geometry(prob)`."""
    P = prob.P
    shp = P.shape[1:]
    gam, gami, sg = geometry(prob)
    nsp = len(e0)
    R = np.zeros((nsp, 4) + shp)
    kap = np.zeros((nsp, 3) + shp)
    cell = np.arange(int(np.prod(shp)), dtype=np.uint64).reshape(shp)
    for s in range(nsp):
        xi = uniform01(seed + 101 * s, cell)
        xf = uniform01(seed + 101 * s + 1, cell)
        th = np.arccos(1.0 - 2.0 * uniform01(seed + 101 * s + 2, cell))
        ph = 2.0 * np.pi * uniform01(seed + 101 * s + 3, cell)
        dirc = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
        E = e0[s] * (1.0 + 0.5 * xi)
        norm = np.sqrt(np.einsum("i...,ij...,j...->...", dirc, gami, dirc))
        F = (fmax * xf * E / norm)[None] * dirc
        R[s, 0] = sg * E
        R[s, 1:] = sg[None] * F
        kap[s, 0] = a_abs[s] * P[0]
        kap[s, 1] = (a_abs[s] + a_scat[s]) * P[0]
        kap[s, 2] = c_eq[s] * P[4]
    return R, kap


def geometry(prob):
    """gamma_ij, gamma^ij [3, 3, s3, s2, s1] and sqrt(gamma) at cell centres
    (Minkowski or Kerr-Schild in x1 = ln r), for laying down input fields."""
    shp = prob.shape
    gam = np.zeros((3, 3) + shp)
    if prob.metric_kind == MINKOWSKI:
        for i in range(3):
            gam[i, i] = 1.0
    else:
        r = np.exp(prob.centers(0))[None, None, :]
        th = prob.centers(1)[None, :, None]
        g11, g13, g22, g33 = _ks_gamma_ij(r, th, prob.a, prob.M)
        gam[0, 0] = g11 + 0 * gam[0, 0]
        gam[0, 2] = gam[2, 0] = g13 + 0 * gam[0, 0]
        gam[1, 1] = g22 + 0 * gam[0, 0]
        gam[2, 2] = g33 + 0 * gam[0, 0]
    g = np.moveaxis(gam, (0, 1), (-2, -1))
    gi = np.moveaxis(np.linalg.inv(g), (-2, -1), (0, 1))
    sg = np.sqrt(np.abs(np.linalg.det(g)))
    return gam, gi, sg
