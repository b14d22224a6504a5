"""GPU parity of the tabulated EOS and the Y_e passive scalar (Phoebus Sec. 2.1
advected scalars, Sec. 2.2 tabulated EOS, Sec. 3.1 general-EOS inversion,
Sec. 3.2 table bounds): every kernel family against the oracle on identical
inputs, at the per-stage bar of the ideal-gas path (1e-11 per variable)."""
import numpy as np
import pytest

import oracle
from paper_2410_09146_amd import inputs as I
from parity_util import oracle_state, rel_err, say, upload_all

pytestmark = pytest.mark.gpu

TOL = 1e-11


@pytest.fixture(scope="module")
def grmhd():
    import torch
    assert torch.cuda.is_available(), "GPU parity tests need an MI355X"
    from paper_2410_09146_amd import grmhd as G
    G.lib()
    return G


def _box(recon, riemann, table="synthetic", n=(20, 18, 16), seed=2):
    prob = I.random_smooth_box(n, seed=seed, amp=0.1, recon=recon, riemann=riemann)
    tab = {"synthetic": I.synthetic_table(), "ideal": I.ideal_table(prob.gamma), None: None}[table]
    return I.with_ye(prob, I.smooth_ye(prob), tab)


def _torus(table="synthetic", n=(32, 32, 16), **kw):
    prob = I.torus(n=n, **kw)
    tab = {"synthetic": I.synthetic_table(), "ideal": I.ideal_table(prob.gamma)}[table]
    return I.with_ye(prob, I.torus_ye, tab)


def _cases():
    return {
        "box_plm_hll": lambda: _box(I.RECON_PLM_MC, I.RIEMANN_HLL),
        "box_weno_llf": lambda: _box(I.RECON_WENO5Z, I.RIEMANN_LLF),
        "box_mp5_ideal_scalar": lambda: _box(I.RECON_MP5, I.RIEMANN_LLF, table=None),
        "torus": lambda: _torus(),
        "torus_ideal_table": lambda: _torus("ideal"),
    }


def _pack_layout(pack, arr):
    out = np.zeros((arr.shape[0], pack.nct))
    cnt = arr.shape[1] * arr.shape[2] * arr.shape[3]
    out[:, :cnt] = arr.reshape(arr.shape[0], -1)
    return out


@pytest.mark.parametrize("case", list(_cases().keys()))
def test_prim_to_cons(grmhd, case):
    prob = _cases()[case]()
    blk, P, Bf, U = oracle_state(prob)
    pack = grmhd.Pack(prob)
    pack.upload(P, Bf)
    pack.prim_to_cons()
    e = rel_err(pack.download("U"), U, prob)
    say("p2c", case, e)
    assert U.shape[0] == 6 and np.all(e <= 1e-13)


@pytest.mark.parametrize("case", list(_cases().keys()))
def test_stage_fluxes_and_update(grmhd, case):
    """One stage of each kind from identical inputs: every face flux slot
    (the normal-field slot carries the scalar's flux), U (6 planes) and Bf."""
    import torch
    prob = _cases()[case]()
    blk, P, Bf, U = oracle_state(prob)
    dt = blk.reductions(P, Bf, U, prob.cfl)["dt"]
    pack = grmhd.Pack(prob)
    for rk in [(1.0, 0.0, 1.0), (0.5, 0.5, 0.5)]:
        U0 = U * (1 + 1e-3) if rk[1] else U
        Bf0 = Bf * (1 - 1e-3) if rk[1] else Bf
        Uo, Bo, Fo = blk.stage(P, Bf, U0, Bf0, U, dt, rk, nthreads=8, want_flux=True)
        upload_all(pack, P, Bf, U)
        if rk[1]:
            pack.U0.copy_(torch.from_numpy(_pack_layout(pack, U0)))
            pack.Bf0.copy_(torch.from_numpy(_pack_layout(pack, Bf0)))
        pack.fill_ghosts()
        pack.stage(dt, rk)
        Fg = pack.flux_array()
        g = prob.ng
        worst = 0.0
        for d in range(3):
            lo = [g - 1] * 3
            hi = [g + prob.n[k] + 1 for k in range(3)]
            lo[d] = g
            sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
            den = max(np.abs(Fo[d][(slice(None),) + sl]).max(), 1e-300)
            for v in range(8):
                err = np.abs(Fg[d, v][sl] - Fo[d, v][sl]).max() / den
                worst = max(worst, err)
                assert err <= TOL, (case, d, v, err)
            # the scalar flux slot against its own scale
            dens = max(np.abs(Fo[d, 5 + d][sl]).max(), 1e-300)
            assert np.abs(Fg[d, 5 + d][sl] - Fo[d, 5 + d][sl]).max() / dens <= TOL
        eU = rel_err(pack.download("U"), Uo, prob)
        eB = rel_err(pack.download("Bf"), Bo, prob, face=True)
        say("stage", case, rk, "flux", worst, "eU", eU.max(), "eU scalar", eU[5], "eB", eB.max())
        assert np.all(eU <= TOL), eU
        assert np.all(eB <= TOL), eB


@pytest.mark.parametrize("case", list(_cases().keys()))
def test_con2prim_parity(grmhd, case):
    """Inversion + floors after a stage: flags identical (incl. Y_e clamps),
    P (with Y_e) and the rewritten U to 1e-11, for both initial guesses."""
    prob = _cases()[case]()
    blk, P, Bf, U = oracle_state(prob)
    dt = blk.reductions(P, Bf, U, prob.cfl)["dt"]
    U1, B1 = blk.stage(P, Bf, U, Bf, U, dt, (1.0, 0.0, 1.0), nthreads=8)
    Po, Uo = P.copy(), U1.copy()
    flag_o, nfail = blk.con2prim(Uo, B1, Po, nthreads=8)
    pack = grmhd.Pack(prob)
    for guess in (grmhd.GUESS_PREV, grmhd.GUESS_COLD):
        upload_all(pack, P, B1, U1)
        pack.con2prim(guess)
        eP = rel_err(pack.download("P"), Po, prob)
        eU = rel_err(pack.download("U"), Uo, prob)
        flags, iters = pack.debug_arrays()
        it = prob.interior()
        say("c2p", case, "guess", guess, "eP", eP.max(), "eU", eU.max(), "fail", nfail,
            "flagged", int((flag_o[it] != 0).sum()), "iters mean", float(iters[it].mean()),
            "max", int(iters[it].max()))
        assert np.array_equal(flags[it], flag_o[it])
        assert np.all(eP <= TOL), eP
        assert np.all(eU <= TOL), eU


def test_table_bounds_on_gpu(grmhd):
    """States partly outside a narrow table: the GPU floors and clamps the
    same cells as the oracle (flags 1, 2 and 32) to the same values."""
    tab = I.synthetic_table(lo=(np.log(0.08), np.log(1e-2), 0.2),
                            hi=(np.log(10.0), np.log(10.0), 0.4))
    prob = I.random_smooth_box((16, 16, 16), seed=5, amp=0.3)
    prob.P[0] *= 0.1
    prob = I.with_ye(prob, I.smooth_ye(prob, amp=0.25), tab)
    blk, P, Bf, U = oracle_state(prob)
    U1, B1 = blk.stage(P, Bf, U, Bf, U, 1e-3, (1.0, 0.0, 1.0), nthreads=8)
    Po, Uo = P.copy(), U1.copy()
    flag_o, nfail = blk.con2prim(Uo, B1, Po, nthreads=8)
    pack = grmhd.Pack(prob)
    upload_all(pack, P, B1, U1)
    pack.con2prim(grmhd.GUESS_PREV)
    flags, _ = pack.debug_arrays()
    it = prob.interior()
    eP = rel_err(pack.download("P"), Po, prob)
    eU = rel_err(pack.download("U"), Uo, prob)
    say("table bounds: flagged", int((flag_o[it] != 0).sum()), "ye clamps",
        int(((flag_o[it] & 32) != 0).sum()), "eP", eP.max(), "eU", eU.max())
    assert np.any(flag_o[it] & 1) and np.any(flag_o[it] & 32)
    assert np.array_equal(flags[it], flag_o[it])
    assert np.all(eP <= TOL) and np.all(eU <= TOL)


@pytest.mark.parametrize("case", list(_cases().keys()))
def test_reductions_parity(grmhd, case):
    prob = _cases()[case]()
    blk, P, Bf, U = oracle_state(prob)
    ro = blk.reductions(P, Bf, U, prob.cfl)
    pack = grmhd.Pack(prob)
    upload_all(pack, P, Bf, U)
    rg = pack.reductions()
    say("reductions", case, rg["dt"], ro["dt"], rg["total_scalar"], ro["total_scalar"])
    assert rg["dt"] == pytest.approx(ro["dt"], rel=1e-13)
    assert np.allclose(rg["totals"], ro["totals"], rtol=1e-13, atol=1e-13 * np.abs(ro["totals"]).max())
    assert rg["total_scalar"] == pytest.approx(ro["total_scalar"], rel=1e-13)


@pytest.mark.parametrize("case", ["box_weno_llf", "torus", "torus_ideal_table"])
def test_steps_from_identical_state(grmhd, case):
    prob = _cases()[case]()
    sim = oracle.Sim(prob, 8)
    pack = grmhd.Pack(prob)
    for s in range(2):
        dt = sim.dt()
        upload_all(pack, sim.P, sim.Bf, sim.U)
        pack.fill_ghosts()
        pack.step(dt)
        sim.step(dt)
        eP = rel_err(pack.download("P"), sim.P, prob)
        eU = rel_err(pack.download("U"), sim.U, prob)
        eB = rel_err(pack.download("Bf"), sim.Bf, prob, face=True)
        say("step", case, s, "eP", eP.max(), "eU", eU.max(), "eB", eB.max())
        assert np.all(eP <= TOL) and np.all(eU <= TOL) and np.all(eB <= TOL)


def test_ideal_table_reproduces_ideal_path(grmhd):
    """The torus with the ideal-gas table and a Y_e scalar takes the same
    steps as the plain ideal-gas torus on the GPU: per step, from identical
    hydro states, the two agree to the parity bar (free-running, the torus
    amplifies rounding-level differences in its atmosphere)."""
    import torch
    p0 = I.torus(n=(32, 32, 16))
    p1 = _torus("ideal")
    k0, k1 = grmhd.Pack(p0), grmhd.Pack(p1)
    k0.init()
    k1.init()
    for s in range(2):
        k1._out()
        k0._out()
        torch.cuda.synchronize()
        k1.P[:5].copy_(k0.P)
        k1.U[:5].copy_(k0.U)
        k1.Bf.copy_(k0.Bf)
        torch.cuda.synchronize()
        k1.fill_ghosts()          # the cell-centred field of the copied face field
        r0, r1 = k0.reductions(), k1.reductions()
        assert r1["dt"] == pytest.approx(r0["dt"], rel=1e-13)
        k0.step(r0["dt"])
        k1.step(r0["dt"])
        eP = rel_err(k1.download("P")[:5], k0.download("P"), p0)
        eB = rel_err(k1.download("Bf"), k0.download("Bf"), p0, face=True)
        say("ideal table vs ideal gas, step", s, "eP", eP.max(), "eB", eB.max())
        assert np.all(eP <= TOL) and np.all(eB <= TOL)


def test_graph_step_equals_eager_with_table(grmhd):
    import torch
    prob = _torus()
    res = []
    for graph in (False, True):
        pack = grmhd.Pack(prob)
        pack.init()
        pack.reductions(sync=False)
        for _ in range(3):
            if graph:
                pack.step_graph(1)
            else:
                pack.step_c(None, cfl=prob.cfl)
        torch.cuda.synchronize()
        res.append((pack.download("P"), pack.reductions()))
        del pack
    say("graph vs eager (table):", np.abs(res[0][0] - res[1][0]).max(), res[1][1]["c2p_fail"])
    assert np.array_equal(res[0][0], res[1][0])
    assert res[1][1]["c2p_fail"] == 0


def test_torus128_table_step_matches_oracle(grmhd):
    """The 128^3 torus with the synthetic table and Y_e: one graph-replayed
    GPU step against one oracle step on the whole grid."""
    import os
    import torch
    prob = _torus(n=(128, 128, 128))
    sim = oracle.Sim(prob, min(16, os.cpu_count() or 1))
    dt = sim.dt()
    pack = grmhd.Pack(prob)
    upload_all(pack, sim.P, sim.Bf, sim.U)
    pack.fill_ghosts()
    r0 = pack.reductions()
    assert r0["dt"] == pytest.approx(dt, rel=1e-12)
    pack.step_graph(1)
    torch.cuda.synchronize()
    sim.step(dt)
    eP = rel_err(pack.download("P"), sim.P, prob)
    eU = rel_err(pack.download("U"), sim.U, prob)
    eB = rel_err(pack.download("Bf"), sim.Bf, prob, face=True)
    say("128^3 table torus step: eP", eP, "eU", eU.max(), "eB", eB.max())
    assert np.all(eP <= TOL) and np.all(eU <= TOL) and np.all(eB <= TOL)


@pytest.mark.parametrize("scalar", [False, True])
def test_every_tile_shape_matches_oracle(grmhd, scalar):
    """Each of the five flux-tile shapes, forced in turn (16x16, 32x8, 8x32,
    64x4, 4x64 faces), gives the oracle's first stage on the torus with
    WENO5-Z-AOAH + LLF: the ideal-gas path, and the synthetic table with the
    Y_e scalar.  The sizes (40 x 36 x 20) leave a ragged tile on every axis."""
    n = (40, 36, 20)
    prob = _torus(n=n) if scalar else I.torus(n=n)
    blk, P, Bf, U = oracle_state(prob)
    dt = blk.reductions(P, Bf, U, prob.cfl)["dt"]
    rk = (1.0, 0.0, 1.0)
    Uo, Bo = blk.stage(P, Bf, U, Bf, U, dt, rk, nthreads=8)
    pack = grmhd.Pack(prob)
    for sh in range(5):
        pack.set_tiling([sh, sh, sh])
        upload_all(pack, P, Bf, U)
        pack.fill_ghosts()
        pack.stage(dt, rk)
        eU = rel_err(pack.download("U"), Uo, prob)
        eB = rel_err(pack.download("Bf"), Bo, prob, face=True)
        say("shape", sh, "scalar", scalar, "eU", eU.max(), "eB", eB.max())
        assert np.all(eU <= TOL) and np.all(eB <= TOL), (sh, eU, eB)
