"""Exact solution of the 1-D special-relativistic hydrodynamics Riemann problem
(ideal gas, no tangential velocity), after Marti & Mueller (1994).

Rarefactions: the Riemann invariants
    atanh(v) +/- (1/sqrt(G-1)) ln[(sqrt(G-1) + c)/(sqrt(G-1) - c)]
are constant along the isentrope p = K rho^G.
Shocks: the Taub adiabat [h^2] = (h_b/rho_b + h_a/rho_a)(p_b - p_a) fixes h_b,
the invariant mass flux j^2 = (p_b - p_a)/(h_a/rho_a - h_b/rho_b), the shock
speed V_s and the post-shock velocity follow from the jump conditions.
The star pressure solves v*_L(p) = v*_R(p).  Used only as a test pin.
"""
import numpy as np
import scipy.optimize as so


def enthalpy(rho, p, g):
    return 1.0 + g / (g - 1.0) * p / rho


def sound_speed(rho, p, g):
    return np.sqrt(g * p / (rho * enthalpy(rho, p, g)))


def _riem_term(c, g):
    s = np.sqrt(g - 1.0)
    return np.log((s + c) / (s - c)) / s


def rarefaction(p, state, g, side):
    """Velocity and density behind a rarefaction from `state` at pressure p.
    side = -1: left-facing wave (state on the left), +1: right-facing."""
    rho_a, v_a, p_a = state
    rho = rho_a * (p / p_a) ** (1.0 / g)
    c_a = sound_speed(rho_a, p_a, g)
    c = sound_speed(rho, p, g)
    if side < 0:
        v = np.tanh(np.arctanh(v_a) + _riem_term(c_a, g) - _riem_term(c, g))
    else:
        v = np.tanh(np.arctanh(v_a) - _riem_term(c_a, g) + _riem_term(c, g))
    return v, rho


def shock(p, state, g, side):
    """Post-shock (v, rho, V_s) for a shock of strength p > p_a."""
    rho_a, v_a, p_a = state
    h_a = enthalpy(rho_a, p_a, g)
    W_a = 1.0 / np.sqrt(1.0 - v_a * v_a)
    dp = p_a - p
    # Taub adiabat for the ideal gas, quadratic in h_b
    A = 1.0 + (g - 1.0) * dp / (g * p)
    B = -(g - 1.0) * dp / (g * p)
    C = h_a * dp / rho_a - h_a * h_a
    h_b = (-B + np.sqrt(B * B - 4.0 * A * C)) / (2.0 * A)
    rho_b = g * p / ((g - 1.0) * (h_b - 1.0))
    j2 = (p - p_a) / (h_a / rho_a - h_b / rho_b)
    j = np.sqrt(j2)
    D2 = rho_a * rho_a * W_a * W_a
    Vs = (D2 * v_a + side * j * np.sqrt(j2 + D2 * (1.0 - v_a * v_a))) / (D2 + j2)
    Ws = 1.0 / np.sqrt(1.0 - Vs * Vs)
    jj = side * j
    v_b = (h_a * W_a * v_a + Ws * (p - p_a) / jj) / \
        (h_a * W_a + (p - p_a) * (Ws * v_a / jj + 1.0 / (rho_a * W_a)))
    return v_b, rho_b, Vs


def wave(p, state, g, side):
    if p > state[2]:
        v, rho, _ = shock(p, state, g, side)
    else:
        v, rho = rarefaction(p, state, g, side)
    return v, rho


class ExactRiemann:
    def __init__(self, left, right, g):
        self.L, self.R, self.g = tuple(map(float, left)), tuple(map(float, right)), g
        f = lambda p: wave(p, self.L, g, -1)[0] - wave(p, self.R, g, +1)[0]
        lo = 1e-12 * min(self.L[2], self.R[2])
        hi = 10.0 * max(self.L[2], self.R[2])
        while f(hi) > 0:
            hi *= 4.0
        self.pstar = so.brentq(f, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
        self.vstar, self.rhoL = wave(self.pstar, self.L, g, -1)
        _, self.rhoR = wave(self.pstar, self.R, g, +1)

    def _fan(self, xi, state, side):
        """State inside a rarefaction fan at similarity coordinate xi."""
        g = self.g
        rho_a, v_a, p_a = state

        def speed(p):
            v, rho = rarefaction(p, state, g, side)
            c = sound_speed(rho, p, g)
            return (v + side * c) / (1.0 + side * v * c) - xi
        p = so.brentq(speed, self.pstar, p_a, xtol=1e-15, rtol=1e-15, maxiter=500)
        v, rho = rarefaction(p, state, g, side)
        return rho, v, p

    def sample(self, xi):
        """(rho, v, p) at xi = (x - x0)/t."""
        g = self.g
        out = np.zeros((len(xi), 3))
        for n, x in enumerate(xi):
            if x < self.vstar:
                st, side, rs = self.L, -1, self.rhoL
            else:
                st, side, rs = self.R, +1, self.rhoR
            rho_a, v_a, p_a = st
            c_a = sound_speed(rho_a, p_a, g)
            star = (rs, self.vstar, self.pstar)
            if self.pstar > p_a:
                Vs = shock(self.pstar, st, g, side)[2]
                ahead = (x < Vs) if side < 0 else (x > Vs)
                out[n] = st if ahead else star
            else:
                head = (v_a + side * c_a) / (1.0 + side * v_a * c_a)
                c_s = sound_speed(rs, self.pstar, g)
                tail = (self.vstar + side * c_s) / (1.0 + side * self.vstar * c_s)
                if (side < 0 and x <= head) or (side > 0 and x >= head):
                    out[n] = st
                elif (side < 0 and x >= tail) or (side > 0 and x <= tail):
                    out[n] = star
                else:
                    out[n] = self._fan(x, st, side)
        return out


def jump_residuals(a, b, Vs, g):
    """Rankine-Hugoniot residuals [F - Vs U] for mass, momentum, energy."""
    def flux_state(rho, v, p):
        W = 1.0 / np.sqrt(1.0 - v * v)
        h = enthalpy(rho, p, g)
        D, S, E = rho * W, rho * h * W * W * v, rho * h * W * W - p
        return np.array([D * v - Vs * D, S * v + p - Vs * S, S - Vs * E])
    fa, fb = flux_state(*a), flux_state(*b)
    scale = np.abs(fa).max() + np.abs(fb).max()
    return (fa - fb) / scale
