"""GPU parity on the failure and limiter branches of the inversion and the
floors (Sec. 3.1 inversion, Sec. 3.2 floors), on the Kerr-Schild torus after
one stage:

* states no inversion can take (D <= 0, a non-finite U), states the oracle
  decides on (tau < 0, S^2 > (tau + D)^2), and states that invert above the
  Lorentz-factor cap, injected into single cells;
* Newton stopped by its iteration cap;
* a learned guess that is rejected (the cold guess takes over);
* a ghost field of garbage under constrained transport.

Flags must equal the oracle's bit for bit, P and U agree to 1e-11 of each
variable's max norm (the cells around the injected ones included), and the
cumulative failure counter counts exactly the flagged cells.
"""
import numpy as np
import pytest

import oracle
from paper_2410_09146_amd import inputs as I
from parity_util import interior, oracle_state, rel_err, say, upload_all

pytestmark = pytest.mark.gpu

TOL = 1e-11
FAIL = 8


@pytest.fixture(scope="module")
def G():
    import torch
    assert torch.cuda.is_available(), "GPU parity tests need an MI355X"
    from paper_2410_09146_amd import grmhd
    grmhd.lib()
    return grmhd


def _post_stage(prob):
    """Oracle state after one stage {1, 0, 1}: previous P, new face field, new U."""
    blk, P, Bf, U = oracle_state(prob)
    dt = blk.reductions(P, Bf, U, prob.cfl)["dt"]
    U1, B1 = blk.stage(P, Bf, U, Bf, U, dt, (1.0, 0.0, 1.0), nthreads=8)
    return blk, P, B1, U1


def _dense_cells(prob, P, count, seed):
    """count interior cells of the torus body (rho > 0.05), at least 3 cells
    apart in every index, in a seeded order: (k, j, i) of the padded arrays."""
    g = prob.ng
    it = prob.interior()
    k, j, i = np.nonzero(P[0][it] > 0.05)
    order = np.random.default_rng(seed).permutation(len(i))
    out = []
    for q in order:
        c = (k[q] + g, j[q] + g, i[q] + g)
        if all(max(abs(c[0] - o[0]), abs(c[1] - o[1]), abs(c[2] - o[2])) >= 3 for o in out):
            out.append(c)
        if len(out) == count:
            break
    assert len(out) == count
    return out


def _w_state(prob, blk, P, B1, cells, W):
    """U of the cells' own primitives with the velocity turned radial at
    Lorentz factor W (u^1 = sqrt((W^2 - 1) / gamma_11))."""
    P2 = P.copy()
    for (k, j, i) in cells:
        r, th = np.exp(prob.centers(0)[i]), prob.centers(1)[j]
        g11 = I._ks_gamma_ij(r, th, prob.a, prob.M)[0]
        P2[1, k, j, i] = np.sqrt((W * W - 1.0) / g11)
        P2[2, k, j, i] = 0.0
        P2[3, k, j, i] = 0.0
    return blk.prim_to_cons(P2, B1)


def _inject(prob, blk, P, B1, U1):
    """U1 with single-cell injections; returns (U, {kind: cells})."""
    U = U1.copy()
    cells = _dense_cells(prob, P, 18, seed=5)
    kinds = {"D<=0": cells[0:3], "NaN": cells[3:5], "inf": cells[5:6], "tau<0": cells[6:9],
             "S^2>(tau+D)^2": cells[9:12], "W>W_max": cells[12:18]}
    for c in kinds["D<=0"]:
        U[(0,) + c] = -abs(U[(0,) + c])
    U[(2,) + kinds["NaN"][0]] = np.nan
    U[(4,) + kinds["NaN"][1]] = np.nan
    U[(4,) + kinds["inf"][0]] = np.inf
    for c in kinds["tau<0"]:
        U[(4,) + c] = -0.5 * U[(0,) + c]
    for c in kinds["S^2>(tau+D)^2"]:
        # |S| scaled to three times tau + D (sqrt(gamma) cancels in the ratio)
        S = U[(slice(1, 4),) + c]
        r, th = np.exp(prob.centers(0)[c[2]]), prob.centers(1)[c[1]]
        g11, g13, g22, g33 = I._ks_gamma_ij(r, th, prob.a, prob.M)
        det = g22 * (g11 * g33 - g13 * g13)
        # |S|^2 = gamma^ij S_i S_j with the inverse of the (x1, x3) block
        S2 = (g33 * S[0] ** 2 - 2 * g13 * S[0] * S[2] + g11 * S[2] ** 2) * g22 / det + S[1] ** 2 / g22
        U[(slice(1, 4),) + c] = S * (3.0 * (U[(4,) + c] + U[(0,) + c]) / np.sqrt(S2))
    Uw = _w_state(prob, blk, P, B1, kinds["W>W_max"][:3], 60.0)
    Uw2 = _w_state(prob, blk, P, B1, kinds["W>W_max"][3:], 80.0)
    for c in kinds["W>W_max"][:3]:
        U[(slice(None),) + c] = Uw[(slice(None),) + c]
    for c in kinds["W>W_max"][3:]:
        U[(slice(None),) + c] = Uw2[(slice(None),) + c]
    return U, kinds


def _u_spread(prob, blk, U, B1, c, draws=32):
    """Spread of the oracle's u at cell c when the cell's conserved state is
    perturbed by one unit in the last place (random signs, seeded): the
    resolution to which FP64 fixes u there.  Above the Lorentz-factor cap
    ((tau + D)/p ~ 1e6) the inversion cancels W-sized terms down to eps."""
    met = oracle.metric_struct(prob.metric_kind, prob.M, prob.a)
    k, j, i = c
    x = np.array([prob.centers(0)[i], prob.centers(1)[j], prob.centers(2)[k]])
    Ud = U[(slice(0, 5),) + c] / oracle.geom(met, x)["sqrtgam"]
    B = blk.cell_B(B1)[(slice(None),) + c]
    rng = np.random.default_rng(1)
    us = []
    for _ in range(draws):
        r, out, _ = oracle.c2p(met, x, prob.gamma, Ud * (1 + 2.0 ** -52 * rng.choice([-1, 1], 5)), B)
        assert r == 0
        us.append(out[4])
    return max(us) - min(us)


def _gpu_c2p(G, prob, P, B1, U, guess, max_iter=40, mlp=None):
    import torch
    pack = G.Pack(prob, c2p_max_iter=max_iter)
    upload_all(pack, P, B1, U)
    if mlp is not None:
        pack.mlp_bind(*mlp)
    f0 = pack.reductions()["c2p_fail_total"]
    pack.con2prim(guess)
    flags, iters = pack.debug_arrays()
    Pg, Ug = pack.download("P"), pack.download("U")
    red = pack.reductions()
    torch.cuda.synchronize()
    return Pg, Ug, flags, iters, red["c2p_fail_total"] - f0, red


def test_injected_failure_and_cap_branches(G):
    prob = I.torus(n=(32, 32, 16))
    blk, P, B1, U1 = _post_stage(prob)
    U, kinds = _inject(prob, blk, P, B1, U1)
    Po, Uo = P.copy(), U.copy()
    flag_o, nfail_o = blk.con2prim(Uo, B1, Po, nthreads=8)
    it = prob.interior()
    # the oracle's own reading of the injected cells
    for kind, cells in kinds.items():
        say("oracle flags", kind, [int(flag_o[c]) for c in cells])
    for c in kinds["D<=0"] + kinds["NaN"] + kinds["inf"]:
        assert flag_o[c] & FAIL
    for c in kinds["W>W_max"]:
        assert flag_o[c] & 4 and not flag_o[c] & FAIL
    umax = np.abs(Po[4][it]).max()
    spread = {c: _u_spread(prob, blk, U, B1, c) for c in kinds["W>W_max"]}
    for guess in (G.GUESS_PREV, G.GUESS_COLD):
        Pg, Ug, flags, iters, nfail, _ = _gpu_c2p(G, prob, P, B1, U, guess)
        # u of the capped cells is judged against the resolution FP64 gives it
        # there (the oracle's own one-ulp spread), every other value at 1e-11
        du = {c: abs(Pg[(4,) + c] - Po[(4,) + c]) for c in kinds["W>W_max"]}
        say("W-capped cells: |du| / umax", [f"{du[c] / umax:.1e}" for c in du],
            "one-ulp spread / umax", [f"{spread[c] / umax:.1e}" for c in du])
        for c in du:
            assert du[c] <= max(2.0 * spread[c], TOL * umax), (c, du[c], spread[c])
        Pm = Pg.copy()
        for c in du:
            Pm[(4,) + c] = Po[(4,) + c]
        eP = rel_err(Pm, Po, prob)
        eU = rel_err(Ug, Uo, prob)
        nf = int(((flags[it] & FAIL) != 0).sum())
        say("injected cells, guess", guess, "eP", eP.max(), "eU", eU.max(), "failed", nf,
            "oracle", int(nfail_o), "counter", nfail, "W-capped", int(((flags[it] & 4) != 0).sum()))
        assert np.array_equal(flags[it], flag_o[it])
        assert np.all(np.isfinite(Pg[(slice(None),) + it])) and np.all(np.isfinite(Ug[(slice(None),) + it]))
        assert np.all(eP <= TOL), eP
        assert np.all(eU <= TOL), eU
        assert nfail == nf == int(nfail_o)
        # a failed cell keeps its previous primitives (floored)
        for c in kinds["D<=0"] + kinds["NaN"] + kinds["inf"]:
            assert np.array_equal(Pg[(slice(None),) + c], Po[(slice(None),) + c])


@pytest.mark.parametrize("guess,max_iter", [("cold", 3), ("prev", 2)])
def test_iteration_cap_fails_like_an_invalid_state(G, guess, max_iter):
    """Newton stopped by the cap: the GPU flags the cell as failed, keeps its
    previous P (floored) and rewrites U, which is the oracle's failure path on
    that cell (reached there by a non-finite U); every other cell converged
    within the cap and matches the oracle's root."""
    prob = I.torus(n=(32, 32, 16))
    blk, P, B1, U1 = _post_stage(prob)
    # The atmosphere's initial primitives equal the floors to the last bit, as
    # numpy evaluated r^-1.5; kept as they are by a failed inversion, they
    # would put the floor test on values one ulp either side of each side's
    # own r^-1.5.  Lifted by 1e-9 they sit clear of both.
    P = P.copy()
    P[0] *= 1.0 + 1e-9
    P[4] *= 1.0 + 1e-9
    gk = G.GUESS_COLD if guess == "cold" else G.GUESS_PREV
    Pg, Ug, flags, iters, nfail, _ = _gpu_c2p(G, prob, P, B1, U1, gk, max_iter=max_iter)
    it = prob.interior()
    capped = (flags & FAIL) != 0
    ncap = int(capped[it].sum())
    Uo, Po = U1.copy(), P.copy()
    Uo[:, capped] = np.nan
    flag_o, nfail_o = blk.con2prim(Uo, B1, Po, nthreads=8)
    eP = rel_err(Pg, Po, prob)
    eU = rel_err(Ug, Uo, prob)
    say("iteration cap", max_iter, guess, "capped cells", ncap, "of", int(np.prod(prob.n)),
        "eP", eP.max(), "eU", eU.max())
    assert 0 < ncap < int(np.prod(prob.n))
    assert np.all(iters[it][capped[it]] == max_iter + 1)
    assert np.array_equal(flags[it], flag_o[it])
    assert nfail == ncap == int(nfail_o)
    assert np.all(eP <= TOL), eP
    assert np.all(eU <= TOL), eU


@pytest.mark.parametrize("net", ["mu_not_positive", "W_inconsistent"])
def test_rejected_learned_guess_falls_back_to_cold(G, net):
    """A network whose guess fails the checks (mu0 = exp(-y1) not positive,
    or a W output far from the W that mu0 implies) is rejected in every cell:
    flag 16, and the Newton solve runs from the cold guess, so iterations and
    root are those of the cold-guess inversion."""
    import torch
    prob = I.torus(n=(32, 32, 16))
    blk, P, B1, U1 = _post_stage(prob)
    params = np.zeros(G.MLP_NPARAM, dtype=np.float32)
    params[-2:] = (0.0, 1e30) if net == "mu_not_positive" else (10.0, 0.5)
    dev = "cuda:0"
    mlp = (torch.tensor(params, device=dev), torch.zeros(5, dtype=torch.float32, device=dev),
           torch.ones(5, dtype=torch.float32, device=dev))
    Pm, Um, fm, im, nfm, rm = _gpu_c2p(G, prob, P, B1, U1, G.GUESS_MLP, mlp=mlp)
    Pc, Uc, fc, ic, nfc, rc = _gpu_c2p(G, prob, P, B1, U1, G.GUESS_COLD)
    Po, Uo = P.copy(), U1.copy()
    flag_o, _ = blk.con2prim(Uo, B1, Po, nthreads=8)
    it = prob.interior()
    ncell = int(np.prod(prob.n))
    dP = rel_err(Pm, Pc, prob)
    say("rejected guess", net, "fallbacks", rm["guess_fallback"], "of", ncell, "max rel dP vs cold",
        dP.max(), "bitwise", bool(np.array_equal(Pm, Pc)), "eP vs oracle", rel_err(Pm, Po, prob).max())
    assert rm["guess_fallback"] == ncell
    assert np.all(fm[it] & 16)
    assert np.array_equal(fm[it] & ~np.int8(16), fc[it])
    assert np.array_equal(fm[it] & ~np.int8(16), flag_o[it])
    assert np.array_equal(im[it], ic[it])
    assert np.all(dP <= 1e-14)
    assert np.all(rel_err(Pm, Po, prob) <= TOL) and np.all(rel_err(Um, Uo, prob) <= TOL)


def _div(prob, Bf):
    g = prob.ng
    n1, n2, n3 = prob.n
    it = prob.interior()
    d = np.zeros((n3, n2, n1))
    d += (Bf[0][g:g + n3, g:g + n2, g + 1:g + n1 + 1] - Bf[0][it]) / prob.dx[0]
    d += (Bf[1][g:g + n3, g + 1:g + n2 + 1, g:g + n1] - Bf[1][it]) / prob.dx[1]
    d += (Bf[2][g + 1:g + n3 + 1, g:g + n2, g:g + n1] - Bf[2][it]) / prob.dx[2]
    return d


def test_ghost_field_garbage_keeps_interior_divergence(G):
    """Constrained transport on the GPU: with the ghost faces of the field
    overwritten by garbage after the ghost fill, a stage changes the discrete
    divergence of no interior cell beyond rounding (every face update is a
    curl of edge EMFs, whatever their values)."""
    import torch
    prob = I.torus(n=(32, 32, 16))
    blk, P, Bf, U = oracle_state(prob)
    pack = G.Pack(prob)
    upload_all(pack, P, Bf, U)
    pack.fill_ghosts()
    pack._out()
    torch.cuda.synchronize()
    g = prob.ng
    s = prob.shape
    cnt = s[0] * s[1] * s[2]
    Bg = pack.Bf[:, :cnt].cpu().numpy().reshape((3,) + s)
    ghost = np.ones((3,) + s, dtype=bool)
    for v in range(3):
        ext = [prob.n[d] + (1 if d == v else 0) for d in range(3)]
        ghost[v, g:g + ext[2], g:g + ext[1], g:g + ext[0]] = False
    rng = np.random.default_rng(9)
    scale = np.abs(Bg).max()
    Bg[ghost] = scale * rng.uniform(-1.0, 1.0, int(ghost.sum()))
    pack.Bf[:, :cnt].copy_(torch.from_numpy(Bg.reshape(3, -1)))
    torch.cuda.synchronize()
    d0 = _div(prob, Bg)
    dt = blk.reductions(P, Bf, U, prob.cfl)["dt"]
    pack.stage(dt, (1.0, 0.0, 1.0))
    B1 = pack.download("Bf")
    d1 = _div(prob, B1)
    f0 = interior(prob, 0)
    bscale = np.abs(B1[0][f0]).max() / min(prob.dx)
    change = np.abs(d1 - d0).max() / bscale
    moved = np.abs(B1[0][f0] - Bg[0][f0]).max() / scale
    say("ghost garbage: interior div change", change, "field moved by", moved)
    assert np.all(np.isfinite(B1[(slice(None),) + prob.interior()]))
    assert moved > 1e-6
    assert change <= 1e-13
