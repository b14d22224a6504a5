"""Two-level block meshes on the GPU against the oracle's mesh: the ghost fill
(same-level copies, restriction, MC-limited prolongation, boundaries at each
level) and whole SSPRK2 steps, per block."""
import numpy as np
import pytest

import oracle
from paper_2410_09146_amd import inputs as I
from parity_util import say, totals_drift

pytestmark = pytest.mark.gpu


def _rel(a, b):
    """Per-variable max-norm error over whole padded blocks, normalised by the
    oracle's max norm over all blocks."""
    nv = a[0].shape[0]
    out = np.zeros(nv)
    for v in range(nv):
        den = max(np.abs(x[v]).max() for x in b)
        num = max(np.abs(x[v] - y[v]).max() for x, y in zip(a, b))
        out[v] = num / den if den > 0 else num
    return out


def _interior_rel(a, b, nx, ng, face=False):
    nv = a[0].shape[0]
    out = np.zeros(nv)
    for v in range(nv):
        num = den = 0.0
        for x, y, n in zip(a, b, nx):
            e = [n[d] + (1 if face and d == v else 0) for d in range(3)]
            sl = (v, slice(ng, ng + e[2]), slice(ng, ng + e[1]), slice(ng, ng + e[0]))
            num = max(num, float(np.abs(x[sl] - y[sl]).max()))
            den = max(den, float(np.abs(y[sl]).max()))
        out[v] = num / den if den > 0 else num
    return out


def _small_torus():
    fine = I.torus(n=(64, 64, 32))
    lay = I.amr_layout(fine, target=60, node=8, smallest=8)
    return fine, I.coarse_problem(fine), lay


def test_two_level_ghost_fill_matches_oracle():
    from paper_2410_09146_amd import grmhd as G
    fine, root, (lev, nx, ll) = _small_torus()
    Ps, Bs = I.mesh_blocks(fine, lev, nx, ll)
    mesh = oracle.Mesh(root, lev, nx, ll, Ps, Bs)
    pack = G.Pack(root, layout=(nx, ll, lev))
    pack.upload_blocks(Ps, Bs)
    pack.fill_ghosts()
    Pg, Bg = pack.download_blocks("P"), pack.download_blocks("Bf")
    eP, eB = _rel(Pg, mesh.P), _rel(Bg, mesh.Bf)
    say("two-level ghost fill:", len(lev), "blocks,", sum(lev), "at level 1; eP", eP, "eB", eB)
    assert 0 < sum(lev) < len(lev)
    assert np.all(eP <= 1e-14) and np.all(eB <= 1e-14)


@pytest.mark.parametrize("case", ["torus", "box"])
def test_two_level_steps_match_oracle(case):
    from paper_2410_09146_amd import grmhd as G
    if case == "torus":
        fine, root, (lev, nx, ll) = _small_torus()
        nsteps = 2
    else:
        fine = I.random_smooth_box((32, 32, 32), seed=6, amp=0.1)
        root = I.coarse_problem(fine)
        ref = {(0, 0, 0), (1, 1, 0), (1, 0, 1)}
        lev, nx, ll = I.two_level_layout(root.n, 8, lambda lo, s: tuple(x // 8 for x in lo) in ref,
                                         p_coarse=(0.5,), p_fine=(0.6,), smallest=8, seed=2)
        nsteps = 3
    Ps, Bs = I.mesh_blocks(fine, lev, nx, ll)
    mesh = oracle.Mesh(root, lev, nx, ll, Ps, Bs, nthreads=8)
    pack = G.Pack(root, layout=(nx, ll, lev))
    pack.init_blocks(Ps, Bs)
    nxa = np.array(nx).reshape(-1, 3)
    g = root.ng
    for s in range(nsteps):
        dt = mesh.dt()
        r = pack.reductions()
        assert r["dt"] == pytest.approx(dt, rel=1e-12)
        mesh.step(dt)
        pack.step(dt)
        Pg, Bg, Ug = pack.download_blocks("P"), pack.download_blocks("Bf"), pack.download_blocks("U")
        eP = _interior_rel(Pg, mesh.P, nxa, g)
        eB = _interior_rel(Bg, mesh.Bf, nxa, g, face=True)
        eU = _interior_rel(Ug, mesh.U, nxa, g)
        gP = _rel(Pg, mesh.P)
        say(case, "two-level step", s, "eP", eP.max(), "eU", eU.max(), "eB", eB.max(),
            "eP incl. ghosts", gP.max())
        assert np.all(eP <= 1e-11) and np.all(eU <= 1e-11) and np.all(eB <= 1e-11)
        assert np.all(gP <= 1e-11)
    red = pack.reductions()
    ro = mesh.reductions()
    say(case, "divb_rel gpu", red["divb_rel"], "oracle", ro["divb_rel"])
    assert red["divb_rel"] < 1e-12
    assert np.allclose(red["totals"], ro["totals"], rtol=1e-11, atol=1e-14 * np.abs(ro["totals"]).max())


def test_two_level_640_blocks_256_effective():
    """The torus at 256^3 effective resolution: level 0 = 128^3, level 1
    where rho > 1e-2 rho_max, about 640 uneven blocks (16^3 / 32^3 / 64^3),
    autotuned tiles, persistent flux grid, graph-replayed step against the
    oracle's mesh step, every block compared."""
    import torch
    from paper_2410_09146_amd import grmhd as G
    fine = I.torus(n=(256, 256, 256))
    lev, nx, ll = I.amr_layout(fine, target=640, node=32, smallest=16)
    root = I.coarse_problem(fine)
    Ps, Bs = I.mesh_blocks(fine, lev, nx, ll)
    del fine
    nxa = np.array(nx).reshape(-1, 3)
    ncell = int((nxa[:, 0] * nxa[:, 1] * nxa[:, 2]).sum())
    say("two-level layout:", len(lev), "blocks,", int(sum(lev)), "at level 1,", ncell, "cells; sizes",
        sorted(set(nxa[:, 0].tolist())))
    assert 560 <= len(lev) <= 720
    pack = G.Pack(root, layout=(nx, ll, lev))
    pack.init_blocks(Ps, Bs)
    pack.reductions(sync=False)
    pack.autotune(reps=1)
    pack.set_persistent(2048)
    mesh = oracle.Mesh(root, lev, nx, ll, Ps, Bs, nthreads=16)
    del Ps, Bs
    dt = mesh.dt()
    pack.step_graph(1)
    red = pack.reductions()
    torch.cuda.synchronize()
    mesh.step(dt)
    g = root.ng
    eP = _interior_rel(pack.download_blocks("P"), mesh.P, nxa, g)
    eB = _interior_rel(pack.download_blocks("Bf"), mesh.Bf, nxa, g, face=True)
    say("640-block two-level step: eP", eP.max(), "eB", eB.max(), "divb", red["divb_rel"],
        "c2p fail", red["c2p_fail"])
    assert np.all(eP <= 1e-11) and np.all(eB <= 1e-11)
    # every inversion since the pack was created (both of the step)
    assert red["divb_rel"] < 1e-12 and red["c2p_fail_total"] == 0


def test_two_level_box_conserves_on_gpu():
    """Periodic two-level box on the GPU: with the level-boundary flux and EMF
    corrections the conserved totals change only by rounding over five steps,
    and divergence stays at rounding."""
    from paper_2410_09146_amd import grmhd as G
    fine = I.random_smooth_box((32, 32, 32), seed=6, amp=0.1)
    root = I.coarse_problem(fine)
    ref = {(0, 0, 0), (1, 1, 0), (1, 0, 1)}
    lev, nx, ll = I.two_level_layout(root.n, 8, lambda lo, s: tuple(x // 8 for x in lo) in ref,
                                     p_coarse=(0.5,), p_fine=(0.6,), smallest=8, seed=2)
    Ps, Bs = I.mesh_blocks(fine, lev, nx, ll)
    pack = G.Pack(root, layout=(nx, ll, lev))
    pack.init_blocks(Ps, Bs)
    r0 = pack.reductions()
    pack.reductions(sync=False)
    for _ in range(5):
        pack.step_c(None, cfl=root.cfl)
    r1 = pack.reductions()
    drift = totals_drift(r1, r0)
    say("two-level box on GPU: relative change of each total over 5 steps", drift,
        "divb", r1["divb_rel"], "c2p fail", r1["c2p_fail_total"])
    assert np.all(drift < 1e-13) and r1["divb_rel"] < 1e-13 and r1["c2p_fail_total"] == 0
