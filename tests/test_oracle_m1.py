"""Pins of the oracle's gray M1 closure and implicit collision update
(Phoebus Sec. 2.4, moments: MEFD closure at maximum packing, backward-Euler
sources with fixed opacities)."""
import os

import numpy as np
import pytest

import oracle
from paper_2410_09146_amd import inputs as I

NT = min(8, os.cpu_count() or 1)
MINK = oracle.Metric(0, 1.0, 0.0)
KS = oracle.Metric(1, 1.0, 0.9375)


def _point(rng, metric, vmax=0.8):
    if metric.kind == 0:
        x = np.zeros(3)
    else:
        x = np.array([np.log(rng.uniform(1.5, 30)), rng.uniform(0.2, 2.9), rng.uniform(0, 6)])
    G = oracle.geom(metric, x)
    v = rng.normal(size=3)
    v *= rng.uniform(0, vmax) / np.sqrt(v @ G["gam"] @ v)
    W = 1 / np.sqrt(1 - v @ G["gam"] @ v)
    return x, G, W * v


def _moments(rng, G, E=None, f=None):
    E = rng.uniform(0.1, 2.0) if E is None else E
    f = rng.uniform(0, 0.95) if f is None else f
    d = rng.normal(size=3)
    d /= np.sqrt(d @ G["gami"] @ d)
    return E, f * E * d


def _tensor(G, E, F, P):
    """T^{mu nu} = E n n + F n + n F + P from the Eulerian moments."""
    n = np.concatenate([[1 / G["alpha"]], -G["beta"] / G["alpha"]])
    Fu = np.concatenate([[0.0], G["gami"] @ F])
    T = E * np.outer(n, n) + np.outer(Fu, n) + np.outer(n, Fu)
    T[1:, 1:] += P
    return T


def _fluid(G, ut):
    W = np.sqrt(1 + ut @ G["gam"] @ ut)
    u = np.concatenate([[W / G["alpha"]], ut - W * G["beta"] / G["alpha"]])
    return u, G["g"] @ u


def test_chi_values():
    assert oracle.m1_chi(0.0) == pytest.approx(1 / 3)
    assert oracle.m1_chi(1.0) == pytest.approx(1.0)
    assert oracle.m1_chi(0.5) == pytest.approx(1 / 3)
    assert oracle.m1_chi(0.25) == pytest.approx((1 - 0.5 + 0.25) / 3)


def test_closure_free_streaming_limit():
    """f = 1: the pressure is the free-streaming E F^i F^j / F^2 in any fluid."""
    rng = np.random.default_rng(1)
    for metric in (MINK, KS):
        for _ in range(50):
            x, G, ut = _point(rng, metric)
            E, F = _moments(rng, G, f=1.0)
            P = oracle.m1_closure(metric, x, ut, E, F)
            Fu = G["gami"] @ F
            assert np.allclose(P, E * np.outer(Fu, Fu) / (Fu @ F), rtol=1e-11, atol=1e-13 * E)


def test_closure_thick_part_is_isotropic_in_the_fluid_frame():
    """Below f = 1 the closure is a blend; its optically thick part, rebuilt
    into the full tensor with the given E and F, is isotropic in the fluid
    frame: h T h = (J/3) h with J = u u T (Kerr-Schild points, moving fluid)."""
    rng = np.random.default_rng(2)
    for metric in (MINK, KS):
        for _ in range(100):
            x, G, ut = _point(rng, metric)
            E, F = _moments(rng, G)
            f = np.sqrt(F @ G["gami"] @ F) / E
            chi = oracle.m1_chi(f)
            a, b = 0.5 * (3 * chi - 1), 1.5 * (1 - chi)
            Fu = G["gami"] @ F
            thin = E * np.outer(Fu, Fu) / (Fu @ F)
            Pthick = (oracle.m1_closure(metric, x, ut, E, F) - a * thin) / b
            T = _tensor(G, E, F, Pthick)
            u, ul = _fluid(G, ut)
            J = ul @ T @ ul
            h = G["g"] + np.outer(ul, ul)
            K = h @ T @ h
            assert np.allclose(K, J / 3 * h, rtol=0, atol=1e-11 * E)


def test_closure_of_zero_flux_in_static_fluid():
    rng = np.random.default_rng(3)
    x, G, _ = _point(rng, KS)
    P = oracle.m1_closure(KS, x, np.zeros(3), 0.7, np.zeros(3))
    assert np.allclose(P, 0.7 / 3 * G["gami"], rtol=1e-12)


def test_static_fluid_closed_form():
    """Fluid at rest in the Eulerian frame (u = n): J = E and H_i = F_i, so
    E = (E* + dt alpha kJ Jeq)/(1 + dt alpha kJ), F_i = F_i*/(1 + dt alpha kH)."""
    rng = np.random.default_rng(4)
    for metric in (MINK, KS):
        for _ in range(50):
            x, G, _ = _point(rng, metric)
            E, F = _moments(rng, G)
            op = np.array([rng.uniform(0, 50), rng.uniform(0, 80), rng.uniform(0.1, 3)])
            dt = rng.uniform(1e-3, 1.0)
            it, X = oracle.m1_implicit(metric, x, np.zeros(3), np.concatenate([[E], F]), op, dt)
            a = G["alpha"]
            assert it > 0
            assert X[0] == pytest.approx((E + dt * a * op[0] * op[2]) / (1 + dt * a * op[0]), rel=1e-12)
            assert np.allclose(X[1:], F / (1 + dt * a * op[1]), rtol=1e-11, atol=1e-14 * E)


def test_zero_opacity_leaves_moments():
    rng = np.random.default_rng(5)
    x, G, ut = _point(rng, KS)
    E, F = _moments(rng, G)
    Xs = np.concatenate([[E], F])
    it, X = oracle.m1_implicit(KS, x, ut, Xs, np.array([0.0, 0.0, 1.0]), 0.3)
    assert np.array_equal(X, Xs)


def test_root_residual():
    """The update satisfies X - X* = dt S(X) to rounding (moving fluid,
    Minkowski and Kerr-Schild points, moderate and strong coupling)."""
    rng = np.random.default_rng(6)
    for metric in (MINK, KS):
        for _ in range(60):
            x, G, ut = _point(rng, metric)
            E, F = _moments(rng, G)
            Xs = np.concatenate([[E], F])
            op = np.array([rng.uniform(0, 30), rng.uniform(0, 60), rng.uniform(0.1, 3)])
            dt = rng.uniform(1e-3, 0.5)
            it, X = oracle.m1_implicit(metric, x, ut, Xs, op, dt)
            assert it > 0
            J, S = oracle.m1_sources(metric, x, ut, X, op)
            scale = np.abs(Xs).sum() + np.abs(X).sum() + dt * op[2]
            assert np.abs(X - Xs - dt * S).max() <= 1e-13 * scale


def test_stiff_limit_reaches_equilibrium():
    """dt kappa -> infinity: the fluid-frame energy goes to J_eq and the
    fluid-frame flux to zero (G = 0 at the root)."""
    rng = np.random.default_rng(7)
    for _ in range(40):
        x, G, ut = _point(rng, KS, vmax=0.6)
        E, F = _moments(rng, G)
        Jeq = rng.uniform(0.2, 2.0)
        op = np.array([1e9, 1.3e9, Jeq])
        it, X = oracle.m1_implicit(KS, x, ut, np.concatenate([[E], F]), op, 1.0)
        assert it > 0
        P = oracle.m1_closure(KS, x, ut, X[0], X[1:])
        T = _tensor(G, X[0], X[1:], P)
        u, ul = _fluid(G, ut)
        J = ul @ T @ ul
        H = -(G["g"] + np.outer(ul, ul)) @ (T @ ul)
        assert J == pytest.approx(Jeq, rel=1e-7)
        assert np.abs(H).max() <= 1e-7 * Jeq


def test_grid_update_matches_point_update():
    prob = I.torus(n=(12, 12, 4))
    R, kap = I.m1_fields(prob)
    blk = oracle.Block(prob)
    R1 = R.copy()
    it, bad = blk.m1_update(prob.P, R1, kap, 0.01, nthreads=NT)
    assert bad == 0
    g = prob.ng
    k, j, i = g + 2, g + 5, g + 7
    x = blk.coord(0, i, j, k)
    G = oracle.geom(blk.metric, x)
    for s in range(3):
        Xs = R[s, :, k, j, i] / G["sqrtgam"]
        _, X = oracle.m1_implicit(blk.metric, x, prob.P[1:4, k, j, i], Xs, kap[s, :, k, j, i], 0.01)
        assert np.allclose(R1[s, :, k, j, i], G["sqrtgam"] * X, rtol=1e-14, atol=0)
    # ghosts untouched
    assert np.array_equal(R1[:, :, 0], R[:, :, 0])
