"""Pins of the oracle's floors, CFL time step and physical-boundary ghost
rules against hand-computed values, and proof that each pin catches a
planted one-line mistake in the oracle (the mistake is planted in a copy of
the oracle's C sources, built and loaded on the CPU only).

* Floors (Sec. 3.2; the u floor and the W ceiling are readings of it): a
  cell below both floors at a known radius comes back with exactly
  rho = 1e-6 r^-1.5 and u = 1e-8 r^-2.5 and flags RHO_FLOOR | U_FLOOR; a cell
  at W = 80 comes back at W = 50 with its velocity direction kept and flag
  W_CAP; in every case U is rewritten as prim -> cons of the final P.  A
  state the inversion cannot invert keeps the previous primitives (floored)
  with flag C2P_FAIL and the same U rewrite.
* CFL (the paper gives no formula; the reading is dt = C / max over cells of
  sum over active directions of max|lambda_d| / dx_d): the uniform
  magnetised box of the 32^3 linear-wave configuration has the fast speed
  c = sqrt(5)/3 exactly in every direction, so dt = 0.4 / (32 sqrt 5); with
  one inactive direction the sum has two terms; a boosted 1-D hydro state
  has lambda = (v +- c_s)/(1 +- v c_s).
* Ghost rules (the paper states none; the reading is periodic wrap, outflow
  copy with the inflowing velocity zeroed, polar mirror with u-tilde^2 and
  the x2 face field negated): every ghost cell and face of a tiny 2-deep
  grid against a table of sources written out by hand.
"""
import ctypes
import math
import os
import shutil

import numpy as np
import pytest

import oracle
from paper_2410_09146_amd import inputs as I

FLAG_RHO, FLAG_U, FLAG_W, FLAG_FAIL = 1, 2, 4, 8


# ------------------------------------------------------------------- floors

def _ks_gamma(r, th, a, M=1.0):
    """Spatial Kerr-Schild metric in (x1 = ln r, theta, phi), written out from
    the line element: gamma_rr = 1 + z, gamma_rphi = -a (1 + z) sin^2,
    gamma_thth = Sigma, gamma_phph = sin^2 (Sigma + a^2 (1 + z) sin^2), z =
    2 M r / Sigma, then dr = r dx1."""
    s2 = math.sin(th) ** 2
    sig = r * r + a * a * math.cos(th) ** 2
    z = 2.0 * M * r / sig
    g = np.zeros((3, 3))
    g[0, 0] = r * r * (1.0 + z)
    g[0, 2] = g[2, 0] = -r * a * (1.0 + z) * s2
    g[1, 1] = sig
    g[2, 2] = s2 * (sig + a * a * (1.0 + z) * s2)
    return g


def _floor_problem():
    n = (6, 4, 2)
    prob = I.Problem(n=n, xmin=(math.log(2.0), 0.4, 0.0), xmax=(math.log(20.0), 2.6, 2.0 * math.pi),
                     bc=(I.BC_OUTFLOW, I.BC_OUTFLOW, I.BC_OUTFLOW, I.BC_OUTFLOW, I.BC_PERIODIC,
                         I.BC_PERIODIC),
                     metric_kind=I.KS_LOGSPH, M=1.0, a=0.9375, gamma=13.0 / 9.0, rho_flr0=1e-6,
                     rho_flr_pow=1.5, u_flr0=1e-8, u_flr_pow=2.5, W_max=50.0)
    P = np.zeros((5,) + prob.shape)
    P[0], P[4] = 1.0, 0.1
    P[1], P[2], P[3] = 0.02, -0.01, 0.03
    Bf = np.zeros((3,) + prob.shape)
    Bf[0] = 0.05      # sqrt(gamma) B^1 on x1 faces: a non-zero field in every cell
    prob.P, prob.Bf = P, Bf
    return prob


def _center(prob, i, j):
    g = prob.ng
    x1 = prob.xmin[0] + ((i - g) + 0.5) * prob.dx[0]
    th = prob.xmin[1] + ((j - g) + 0.5) * prob.dx[1]
    return math.exp(x1), th


def floor_case():
    """Run the oracle inversion on three hand-built cells; return what the
    pins compare (raises AssertionError on a mismatch)."""
    prob = _floor_problem()
    g = prob.ng
    blk = oracle.Block(prob)
    P, Bf = prob.P.copy(), prob.Bf.copy()
    cA, cB, cC = (g, g + 2, g + 1), (g + 1, g + 3, g + 4), (g + 1, g + 1, g + 2)   # (k, j, i)
    rA, _ = _center(prob, cA[2], cA[1])
    rC, _ = _center(prob, cC[2], cC[1])
    rho_flr = lambda r: 1e-6 * r ** -1.5
    u_flr = lambda r: 1e-8 * r ** -2.5
    # A: below both floors
    P[(0,) + cA] = 1e-3 * rho_flr(rA)
    P[(4,) + cA] = 1e-3 * u_flr(rA)
    # C: u below its floor only
    P[(0,) + cC] = 1e-3
    P[(4,) + cC] = 1e-4 * u_flr(rC)
    # B: W = 80 along a fixed contravariant direction
    rB, thB = _center(prob, cB[2], cB[1])
    gam = _ks_gamma(rB, thB, prob.a)
    dirn = np.array([0.3, -0.05, 0.02])
    ut = dirn * math.sqrt((80.0 ** 2 - 1.0) / (dirn @ gam @ dirn))
    for d in range(3):
        P[(1 + d,) + cB] = ut[d]
    U = blk.prim_to_cons(P, Bf)
    Pin = P.copy()
    flag, nfail = blk.con2prim(U, Bf, P)
    assert nfail == 0
    assert flag[cA] == FLAG_RHO | FLAG_U, flag[cA]
    assert P[(0,) + cA] == rho_flr(rA) and P[(4,) + cA] == u_flr(rA), (P[(0,) + cA], rho_flr(rA))
    assert flag[cC] == FLAG_U, flag[cC]
    assert P[(4,) + cC] == u_flr(rC)
    assert abs(P[(0,) + cC] / 1e-3 - 1.0) < 1e-9
    assert flag[cB] == FLAG_W, flag[cB]
    utB = np.array([P[(1 + d,) + cB] for d in range(3)])
    W = math.sqrt(1.0 + utB @ gam @ utB)
    assert abs(W / 50.0 - 1.0) < 1e-14, W
    np.testing.assert_allclose(utB / np.linalg.norm(utB), dirn / np.linalg.norm(dirn), rtol=0,
                               atol=1e-12)
    assert abs(P[(0,) + cB] - 1.0) < 1e-9 and abs(P[(4,) + cB] / 0.1 - 1.0) < 1e-8
    # untouched cells keep their state; every floored cell has U = U(P)
    Uf = blk.prim_to_cons(P, Bf)
    for c in (cA, cB, cC):
        np.testing.assert_allclose(U[(slice(None),) + c], Uf[(slice(None),) + c], rtol=1e-14,
                                   atol=0)
    intr = prob.interior()
    mask = np.zeros(prob.shape, bool)
    mask[intr] = True
    for c in (cA, cB, cC):
        mask[c] = False
    assert np.all(flag[mask] == 0)
    np.testing.assert_allclose(P[:, mask], Pin[:, mask], rtol=1e-9, atol=1e-13)
    return True


def test_floors_and_w_cap_hand_values():
    assert floor_case()


def fallback_case():
    """A cell whose conserved state is not finite keeps its previous
    primitives (then floored) with flag C2P_FAIL, and its U is rewritten."""
    prob = _floor_problem()
    g = prob.ng
    blk = oracle.Block(prob)
    P, Bf = prob.P.copy(), prob.Bf.copy()
    c = (g + 1, g + 2, g + 3)
    r, _ = _center(prob, c[2], c[1])
    P[(0,) + c] = 1e-9          # previous state: below the density floor
    U = blk.prim_to_cons(P, Bf)
    U[(4,) + c] = np.nan
    Pin = P.copy()
    flag, nfail = blk.con2prim(U, Bf, P)
    assert nfail == 1
    assert flag[c] == FLAG_FAIL | FLAG_RHO, flag[c]
    assert P[(0,) + c] == 1e-6 * r ** -1.5
    for q in range(1, 5):
        assert P[(q,) + c] == Pin[(q,) + c]
    Uf = blk.prim_to_cons(P, Bf)
    np.testing.assert_allclose(U[(slice(None),) + c], Uf[(slice(None),) + c], rtol=1e-14, atol=0)
    return True


def test_failed_inversion_keeps_previous_primitives():
    assert fallback_case()


def test_energy_below_cold_limit_inverts_to_cold_state():
    """With B = 0 and tau below the cold kinetic energy D (W - 1) of the given
    momentum (S = 3 D, tau = D: S^2 > (tau + D)^2), the clamps of the master
    function (v^2 <= r^2 / (1 + r^2), eps >= 0) make the root the cold state
    of that momentum: u-tilde = S / D, rho = D / sqrt(1 + S^2 / D^2), u = 0."""
    met = oracle.metric_struct(I.MINKOWSKI)
    for D, S in ((1.0, 3.0), (2.0, 10.0), (0.5, 40.0)):
        r, out, _ = oracle.c2p(met, [0.5, 0.5, 0.5], 4.0 / 3.0, [D, S, 0.0, 0.0, D], [0.0, 0.0, 0.0])
        assert r == 0
        tol = 1e-14 + 1e-15 * (1.0 + (S / D) ** 2)     # the root's rounding grows as W^2
        assert abs(out[1] / (S / D) - 1.0) < tol, out
        assert abs(out[0] / (D / math.sqrt(1.0 + (S / D) ** 2)) - 1.0) < tol, out
        assert out[4] == 0.0


# ---------------------------------------------------------------------- CFL

def cfl_case():
    """dt of three states whose characteristic speeds have closed forms."""
    # uniform magnetised box of the linear-wave configuration: rho = p = 1,
    # gamma = 4/3 (rho h = 5, c_s^2 = 4/15), B^2 = 3.25 (c_A^2 = 13/33), so the
    # fast speed c^2 = c_s^2 + c_A^2 - c_s^2 c_A^2 = 5/9 in every direction
    box = I.linear_wave((32, 32, 32), amp=0.0)
    blk = oracle.Block(box)
    P, Bf = box.P.copy(), box.Bf.copy()
    blk.fill_ghosts(P, Bf)
    U = blk.prim_to_cons(P, Bf)
    dt = blk.reductions(P, Bf, U, 0.4)["dt"]
    want = 0.4 / (32.0 * math.sqrt(5.0))
    assert abs(dt / want - 1.0) < 1e-14, (dt, want)
    # the same state with x3 a single cell: two terms in the sum
    slab = I.linear_wave((32, 32, 1), k=(1, 1, 0), amp=0.0)
    blk = oracle.Block(slab)
    P, Bf = slab.P.copy(), slab.Bf.copy()
    blk.fill_ghosts(P, Bf)
    U = blk.prim_to_cons(P, Bf)
    dt = blk.reductions(P, Bf, U, 0.4)["dt"]
    want = 0.4 / (2.0 * 32.0 * math.sqrt(5.0) / 3.0)
    assert abs(dt / want - 1.0) < 1e-14, (dt, want)
    # boosted hydro along x1 (1-D): lambda = (v +- c_s) / (1 +- v c_s)
    v, gam = 0.6, 5.0 / 3.0
    W = 1.0 / math.sqrt(1.0 - v * v)
    line = I.uniform_box((32, 1, 1), rho=1.0, ut=(W * v, 0.0, 0.0), u=1.5, gamma=gam)
    blk = oracle.Block(line)
    P, Bf = line.P.copy(), line.Bf.copy()
    blk.fill_ghosts(P, Bf)
    U = blk.prim_to_cons(P, Bf)
    dt = blk.reductions(P, Bf, U, 0.4)["dt"]
    p = (gam - 1.0) * 1.5
    cs = math.sqrt(gam * p / (1.0 + 1.5 + p))
    lam = max(abs((v + cs) / (1.0 + v * cs)), abs((v - cs) / (1.0 - v * cs)))
    want = 0.4 * (1.0 / 32.0) / lam
    assert abs(dt / want - 1.0) < 1e-13, (dt, want)
    return True


def test_cfl_dt_closed_forms():
    assert cfl_case()


# ------------------------------------------------------------------- ghosts

# Sources written out by hand for n = (3, 4, 2), ng = 2.  Cell-centred values
# along each axis, then the face-normal component along its own axis.
#   x1 outflow, interior cells 2..4, faces 2..5
#   x2 polar mirror, interior cells 2..5 (faces 2 and 6 on the axis)
#   x3 periodic, interior cells 2..3, faces 2..4
CELL_SRC = ({0: 2, 1: 2, 5: 4, 6: 4},
            {0: 3, 1: 2, 6: 5, 7: 4},
            {0: 2, 1: 3, 4: 2, 5: 3})
FACE_SRC = ({0: 2, 1: 2, 6: 5},
            {0: 4, 1: 3, 7: 5},
            {0: 2, 1: 3, 5: 3})


def ghost_case():
    n = (3, 4, 2)
    prob = I.Problem(n=n, xmin=(0.0, 0.0, 0.0), xmax=(1.0, 1.0, 1.0),
                     bc=(I.BC_OUTFLOW, I.BC_OUTFLOW, I.BC_POLAR, I.BC_POLAR, I.BC_PERIODIC,
                         I.BC_PERIODIC), ng=2)
    rng = np.random.default_rng(17)
    P = rng.uniform(-1.0, 1.0, (5,) + prob.shape)
    P[0] = np.abs(P[0]) + 0.5
    P[4] = np.abs(P[4]) + 0.5
    Bf = rng.uniform(-1.0, 1.0, (3,) + prob.shape)
    P0, B0 = P.copy(), Bf.copy()
    oracle.Block(prob).fill_ghosts(P, Bf)
    s3, s2, s1 = prob.shape
    nchk = 0
    for k in range(s3):
        for j in range(s2):
            for i in range(s1):
                gh = (i in CELL_SRC[0], j in CELL_SRC[1], k in CELL_SRC[2])
                src = (CELL_SRC[2].get(k, k), CELL_SRC[1].get(j, j), CELL_SRC[0].get(i, i))
                v = P0[(slice(None),) + src].copy()
                if gh[0]:
                    if i < 2 and v[1] > 0.0:
                        v[1] = 0.0          # no inflow through the lower x1 boundary
                    if i > 4 and v[1] < 0.0:
                        v[1] = 0.0          # nor through the upper one
                if gh[1]:
                    v[2] = -v[2]            # across the axis u-tilde^2 changes sign
                want = v if any(gh) else P0[:, k, j, i]
                assert np.array_equal(P[:, k, j, i], want), ("P", k, j, i, P[:, k, j, i], want)
                nchk += any(gh)
                for c in range(3):
                    tabs = [CELL_SRC[0], CELL_SRC[1], CELL_SRC[2]]
                    tabs[c] = FACE_SRC[c]
                    idx = (i, j, k)
                    gf = [idx[d] in tabs[d] for d in range(3)]
                    fsrc = (tabs[2].get(k, k), tabs[1].get(j, j), tabs[0].get(i, i))
                    w = B0[(c,) + fsrc]
                    if c == 1 and gf[1]:
                        w = -w              # the normal field reverses across the axis
                    want = w if any(gf) else B0[c, k, j, i]
                    assert Bf[c, k, j, i] == want, ("Bf", c, k, j, i, Bf[c, k, j, i], want)
    assert nchk == s1 * s2 * s3 - 3 * 4 * 2
    return True


def test_ghost_rules_hand_table():
    assert ghost_case()


# ------------------------------------------- planted mistakes must be caught

MUTATIONS = {
    # floors: the W rescale without its square root
    "w_cap_no_sqrt": ("stage.c", "const double s = sqrt((e->W_max * e->W_max - 1.0) / ut2);",
                      "const double s = (e->W_max * e->W_max - 1.0) / ut2;", floor_case),
    # floors: density floor with the wrong sign of the exponent
    "rho_floor_exponent": ("stage.c", "double rho_flr = e->rho_flr0 * pow(r, -e->rho_flr_pow);",
                           "double rho_flr = e->rho_flr0 * pow(r, e->rho_flr_pow);", floor_case),
    # floors: the u floor with the density's exponent
    "u_floor_exponent": ("stage.c", "double u_flr = e->u_flr0 * pow(r, -e->u_flr_pow);",
                         "double u_flr = e->u_flr0 * pow(r, -e->rho_flr_pow);", floor_case),
    # floors: U not rewritten after a floor acts
    "no_u_rewrite": ("stage.c", "        if (fl) {\n          double Uc[9];",
                     "        if (0) {\n          double Uc[9];", floor_case),
    # fallback: the failed cell takes the (non-finite) inversion result
    "fallback_not_kept": ("stage.c", "          load_prim(g, e, P, Bcc, c, &q);\n          fl |= ORC_FLAG_C2P_FAIL;",
                          "          fl |= ORC_FLAG_C2P_FAIL;", fallback_case),
    # CFL: maximum over directions instead of the sum
    "cfl_max_not_sum": ("stage.c", "s += fmax(fabs(lm), fabs(lp)) / g->dx[d];",
                        "s = fmax(s, fmax(fabs(lm), fabs(lp)) / g->dx[d]);", cfl_case),
    # CFL: single-cell directions counted
    "cfl_inactive_dir": ("stage.c", "if (g->n[d] <= 1) continue;\n          double lm, lp;",
                         "if (g->n[d] < 1) continue;\n          double lm, lp;", cfl_case),
    # CFL: the slower characteristic instead of the faster
    "cfl_min_speed": ("stage.c", "s += fmax(fabs(lm), fabs(lp)) / g->dx[d];",
                      "s += fmin(fabs(lm), fabs(lp)) / g->dx[d];", cfl_case),
    # ghosts: polar mirror of cells off by one (mirrors about a cell centre)
    "polar_cell_index": ("stage.c", "else        *src = low ? 2 * lo - 1 - idx : 2 * (ng + n) - 1 - idx;",
                         "else        *src = low ? 2 * lo - idx : 2 * (ng + n) - 1 - idx;", ghost_case),
    # ghosts: outflow clamp with the wrong sign
    "outflow_sign": ("stage.c", "if (side[d] < 0 && v[1 + d] > 0.0) v[1 + d] = 0.0;",
                     "if (side[d] < 0 && v[1 + d] < 0.0) v[1 + d] = 0.0;", ghost_case),
    # ghosts: periodic wrap shifted by one cell
    "periodic_shift": ("stage.c", "*src = ng + (((idx - ng) % n) + n) % n;",
                       "*src = ng + (((idx - ng + 1) % n) + n) % n;", ghost_case),
    # ghosts: the x2 face field not negated across the axis
    "polar_face_flip": ("stage.c", "if (flip[c]) v = -v;   /* normal component reverses across the pole */",
                        "if (0) v = -v;", ghost_case),
}


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    return tmp_path_factory.mktemp("oracle_mutants")


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pin_catches_planted_mistake(name, mutant_dir):
    fname, old, new, case = MUTATIONS[name]
    here = os.path.dirname(oracle.__file__)
    d = mutant_dir / name
    d.mkdir()
    for f in os.listdir(here):
        if f.endswith((".c", ".h")):
            shutil.copy(os.path.join(here, f), d / f)
    src = (d / fname).read_text()
    assert src.count(old) == 1, f"mutation site of {name} not unique in {fname}"
    (d / fname).write_text(src.replace(old, new))
    lib = oracle.build(force=True, src_dir=str(d), out=str(d / "liboracle_mut.so"))
    saved = oracle._lib
    try:
        oracle._lib = oracle.load(lib)
        with pytest.raises(AssertionError):
            case()
    finally:
        oracle._lib = saved
    assert case()     # the unmodified oracle passes the same pin
