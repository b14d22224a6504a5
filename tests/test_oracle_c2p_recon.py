"""Pins of the oracle's inversion (Sec. 3.1, Kastaun-type master function) and
reconstructions (Sec. 3.1 list; App. B WENO5-Z-AOAH)."""
import numpy as np
import pytest

import oracle
from paper_2410_09146_amd import inputs as I

MINK = oracle.Metric(0, 1.0, 0.0)
KS = oracle.Metric(1, 1.0, 0.9375)


def _roundtrip(metric, x, g, p8):
    U = oracle.p2c(metric, x, g, p8)
    r, out, mu = oracle.c2p(metric, x, g, U[:5], U[5:8])
    return r, out, U


def test_roundtrip_sampled_minkowski():
    """prim -> cons -> prim on the learned-guess sampling ranges (rho, p/rho,
    W in [1,50], b^2/rho in [1e-4,100]).  rho, u-tilde within
    max(1e-12, 2e-14 W^2): the root mu = 1/(hW) is found to ~1e-14 (rounding
    noise of f), and W = (1 - mu^2 rbar^2)^-1/2 amplifies that by ~W^2.
    u is gated where kappa = (tau + D)/p <= 1e3 (cold fast flows lose p to
    cancellation, error ~ kappa eps_mach)."""
    s = I.random_prims(2000, seed=11)
    g = s["gamma"]
    bad = 0
    for n in range(2000):
        p8 = np.concatenate([[s["rho"][n]], s["ut"][n], [s["u"][n]], s["B"][n]])
        r, out, U = _roundtrip(MINK, np.zeros(3), g, p8)
        assert r == 0
        tol = max(1e-12, 2e-14 * s["W"][n] ** 2)
        assert out[0] == pytest.approx(p8[0], rel=tol)
        assert np.allclose(out[1:4], p8[1:4], rtol=tol, atol=tol * np.abs(p8[1:4]).max())
        kappa = (U[4] + U[0]) / ((g - 1) * p8[4])
        if kappa <= 1e3:
            assert out[4] == pytest.approx(p8[4], rel=1e-12)
        else:
            # error grows ~ kappa * eps_mach, reported not gated
            bad += abs(out[4] / p8[4] - 1) > 1e-12
    assert bad < 2000


def test_roundtrip_kerr_schild():
    rng = np.random.default_rng(12)
    g = 13.0 / 9.0
    for _ in range(300):
        x = np.array([np.log(rng.uniform(1.3, 40)), rng.uniform(0.05, 3.09), rng.uniform(0, 6)])
        G = oracle.geom(KS, x)
        v = rng.normal(size=3)
        v *= rng.uniform(0, 0.95) / np.sqrt(v @ G["gam"] @ v)
        W = 1 / np.sqrt(1 - v @ G["gam"] @ v)
        B = rng.normal(size=3) / np.sqrt(np.diag(G["gam"])) * rng.uniform(0, 1)
        p8 = np.concatenate([[rng.uniform(1e-3, 1)], W * v, [rng.uniform(1e-3, 1)], B])
        r, out, U = _roundtrip(KS, x, g, p8)
        assert r == 0
        assert out[0] == pytest.approx(p8[0], rel=1e-12)
        assert np.allclose(out[1:4], p8[1:4], rtol=1e-11, atol=1e-12 * np.abs(p8[1:4]).max())
        assert out[4] == pytest.approx(p8[4], rel=1e-10)


def test_master_function_unique_root_brute_force():
    """A dense scan of f(mu) on (0, 1] shows exactly one sign change, and the
    bisection root lies in that scan interval."""
    s = I.random_prims(40, seed=13)
    g = s["gamma"]
    mus = np.linspace(1e-6, 1.0, 10001)
    for n in range(40):
        p8 = np.concatenate([[s["rho"][n]], s["ut"][n], [s["u"][n]], s["B"][n]])
        U = oracle.p2c(MINK, np.zeros(3), g, p8)
        D, S, tau, B = U[0], U[1:4], U[4], U[5:8]
        q, r2, b2, rb = tau / D, S @ S / D ** 2, B @ B / D, S @ B / D ** 1.5
        f = np.array([oracle.master(g, q, r2, b2, rb, m) for m in mus])
        changes = np.nonzero(np.diff(np.sign(f)))[0]
        assert len(changes) == 1
        _, out, mu = oracle.c2p(MINK, np.zeros(3), g, U[:5], B)
        assert mus[changes[0]] <= mu <= mus[changes[0] + 1]
        # the root is mu = 1/(h W) of the original state
        W = np.sqrt(1 + p8[1:4] @ p8[1:4])
        h = 1 + g * p8[4] / p8[0]
        assert mu == pytest.approx(1 / (h * W), rel=1e-13)


def test_invalid_state_flagged():
    r, _, _ = oracle.c2p(MINK, np.zeros(3), 4 / 3, [-1.0, 0, 0, 0, 1.0], [0, 0, 0])
    assert r == 1
    r, _, _ = oracle.c2p(MINK, np.zeros(3), 4 / 3, [1.0, np.nan, 0, 0, 1.0], [0, 0, 0])
    assert r == 1


# ------------------------------------------------------------- reconstruction

CONST, MC, WENO, MINMOD, MP5 = 0, 1, 2, 3, 4


@pytest.mark.parametrize("method", [CONST, MC, WENO, MINMOD, MP5])
def test_constant_exact(method):
    fl, fr = oracle.recon(method, [2.5] * 5)
    assert fl == 2.5 and fr == 2.5


@pytest.mark.parametrize("method", [MC, WENO, MINMOD, MP5])
def test_linear_exact(method):
    f = 0.3 + 0.7 * np.arange(-2, 3)
    fl, fr = oracle.recon(method, f)
    assert fl == pytest.approx(0.3 - 0.35, abs=1e-15)
    assert fr == pytest.approx(0.3 + 0.35, abs=1e-15)


def test_weno_quadratic_exact_both_readings():
    """Quadratic data: all beta_k equal, w = gamma, sigma = 1, and the face
    value is exact (point values for the interpolation reading, cell averages
    for the finite-volume reading)."""
    q = lambda x: 1.0 - 0.4 * x + 0.9 * x * x
    xs = np.arange(-2, 3).astype(float)
    fl, fr = oracle.recon(WENO, q(xs), fv=0)
    assert fl == pytest.approx(q(-0.5), abs=1e-14)
    assert fr == pytest.approx(q(0.5), abs=1e-14)
    avg = lambda x: q(x) + 0.9 / 12.0          # exact cell average of a quadratic
    fl, fr = oracle.recon(WENO, avg(xs), fv=1)
    assert fl == pytest.approx(q(-0.5), abs=1e-14)
    assert fr == pytest.approx(q(0.5), abs=1e-14)
    w, s = oracle.weno(q(xs))
    assert np.allclose(w, [1 / 16, 10 / 16, 5 / 16], atol=1e-15)
    assert s == pytest.approx(1.0, abs=1e-15)


def test_weno_beta_brute_force():
    """beta_k = sum_l dx^(2l-1) int_cell (d^l P_k/dx^l)^2 for the quadratic
    through stencil k, integrated numerically."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        f = rng.normal(size=5)
        b = oracle.weno_beta(f)
        for k in range(3):
            xs = np.arange(-2 + k, 1 + k).astype(float)
            c = np.polyfit(xs, f[k:k + 3], 2)
            d1, d2 = np.polyder(c, 1), np.polyder(c, 2)
            gx, gw = np.polynomial.legendre.leggauss(6)
            gx = 0.5 * gx
            gw = 0.5 * gw
            ref = np.sum(gw * np.polyval(d1, gx) ** 2) + np.sum(gw * np.polyval(d2, gx) ** 2)
            assert b[k] == pytest.approx(ref, rel=1e-12, abs=1e-14)


def test_mirror_symmetry():
    rng = np.random.default_rng(8)
    for method in (MC, WENO, MINMOD, MP5):
        for _ in range(50):
            f = rng.normal(size=5)
            fl, fr = oracle.recon(method, f)
            gl, gr = oracle.recon(method, f[::-1])
            assert fl == pytest.approx(gr, rel=1e-14, abs=1e-15)
            assert fr == pytest.approx(gl, rel=1e-14, abs=1e-15)


def test_mc_zero_slope_at_extremum():
    fl, fr = oracle.recon(MC, [0.0, 1.0, 2.0, 1.5, 0.0])
    assert fl == 2.0 and fr == 2.0


def test_sigma_in_unit_interval_and_clamped():
    rng = np.random.default_rng(9)
    for _ in range(500):
        f = rng.normal(size=5) * rng.uniform(0, 10)
        w, sp = oracle.weno(f)
        assert sp > 0
    # reading: sigma_side can exceed 1 (harmonic mean of w/gamma); blended value
    # stays a convex combination of P5 and PLM after the clamp
    f = np.array([0.0, 0.0, 0.0, 1.0, 1.0])
    fl, fr = oracle.recon(WENO, f)
    assert min(f) - 1e-12 <= fr <= max(f) + 1e-12


def test_weno_fifth_order_smooth():
    errs = []
    for N in (16, 32, 64):
        h = 1.0 / N
        x = (np.arange(N) + 0.5) * h
        fun = lambda y: np.sin(2 * np.pi * y + 0.3)
        e = 0.0
        for j in range(N):
            st = fun(x[j] + h * np.arange(-2, 3))
            fl, fr = oracle.recon(WENO, st)
            e = max(e, abs(fr - fun(x[j] + 0.5 * h)), abs(fl - fun(x[j] - 0.5 * h)))
        errs.append(e)
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 4.5), (errs, orders)


# ---------------------------------------------------------------- MP5

def test_mp5_quartic_exact_both_readings():
    """Smooth monotone quartic: the limiter stays inactive and the face value
    is the exact fifth-order one (point-value interpolation, or cell averages
    with fv = 1)."""
    c = [1.0, 0.5, 0.05, 0.01, 0.002]
    q = lambda x: sum(ck * x ** k for k, ck in enumerate(c))
    xs = np.arange(-2, 3).astype(float)
    fl, fr = oracle.recon(MP5, q(xs), fv=0)
    assert fr == pytest.approx(q(0.5), abs=1e-14)
    assert fl == pytest.approx(q(-0.5), abs=1e-14)

    def avg(x):          # exact cell average of the quartic over [x-1/2, x+1/2]
        P = np.polynomial.Polynomial(c).integ()
        return P(x + 0.5) - P(x - 0.5)
    fl, fr = oracle.recon(MP5, avg(xs), fv=1)
    assert fr == pytest.approx(q(0.5), abs=1e-14)
    assert fl == pytest.approx(q(-0.5), abs=1e-14)


def test_mp5_monotone_data_no_new_extrema():
    """On monotone data every face value lies between its two neighbouring
    cell values (the monotonicity-preserving property)."""
    rng = np.random.default_rng(12)
    for _ in range(2000):
        inc = rng.exponential(size=5) * (rng.uniform(size=5) < 0.7)
        f = np.cumsum(inc) * rng.choice([-1.0, 1.0])
        for fv in (0, 1):
            fl, fr = oracle.recon(MP5, f, fv=fv)
            assert min(f[2], f[3]) - 1e-13 <= fr <= max(f[2], f[3]) + 1e-13
            assert min(f[1], f[2]) - 1e-13 <= fl <= max(f[1], f[2]) + 1e-13


def test_mp5_step_and_extremum():
    fl, fr = oracle.recon(MP5, [0.0, 0.0, 0.0, 1.0, 1.0])
    assert 0.0 <= fr <= 1.0 and fl == 0.0
    # a sharp isolated peak is not amplified
    fl, fr = oracle.recon(MP5, [0.0, 0.0, 1.0, 0.0, 0.0])
    assert 0.0 <= fl <= 1.0 and 0.0 <= fr <= 1.0


def test_mp5_fifth_order_smooth():
    errs = []
    for N in (32, 64, 128, 256):
        h = 1.0 / N
        x = (np.arange(N) + 0.5) * h
        fun = lambda y: np.sin(2 * np.pi * y + 0.3)
        e = 0.0
        for j in range(N):
            st = fun(x[j] + h * np.arange(-2, 3))
            fl, fr = oracle.recon(MP5, st)
            e = max(e, abs(fr - fun(x[j] + 0.5 * h)), abs(fl - fun(x[j] - 0.5 * h)))
        errs.append(e)
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders[-1] > 4.5, (errs, orders)
