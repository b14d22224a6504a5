"""Mesh refinement on the GPU against the oracle (two-level block mesh):
tagging, the next layout, the remap (conservative, divergence-free), and a
refine / derefine cycle inside a run."""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import amr
from paper_2410_09146_amd import inputs as I
from parity_util import say, totals_drift

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    assert torch.cuda.is_available(), "GPU parity tests need an MI355X"
    from paper_2410_09146_amd import grmhd
    grmhd.lib()
    return grmhd


def _box(refined, seed=6, amp=0.1, n=16, node=8, p_fine=(0.0,)):
    fine = I.random_smooth_box((2 * n,) * 3, seed=seed, amp=amp)
    root = I.coarse_problem(fine)
    lev, nx, ll = I.two_level_layout(root.n, node, lambda lo, s: tuple(x // node for x in lo) in refined,
                                     p_coarse=(0.0,), p_fine=p_fine, smallest=node // 2, seed=2)
    Ps, Bs = I.mesh_blocks(fine, lev, nx, ll)
    return root, lev, nx, ll, Ps, Bs


def _pack_from_mesh(G, mesh):
    """A pack holding exactly the oracle mesh's P, Bf (ghosts included) and U."""
    import torch
    pack = G.Pack(mesh.root, layout=(mesh.nx.ravel().tolist(), mesh.lloc.ravel().tolist(),
                                     mesh.level.tolist()))
    pack.upload_blocks(mesh.P, mesh.Bf)
    for b in range(pack.nb):
        pack._block_views(pack.U, b).copy_(torch.from_numpy(np.ascontiguousarray(mesh.U[b])))
    pack.fill_ghosts()
    torch.cuda.synchronize()
    return pack


def _raw_remap(G, dst, src):
    import torch
    src._out()
    dst._out()
    torch.cuda.synchronize()
    L = G.lib()
    nb = L.grmhd_remap_scratch_bytes(dst.h, src.h)
    assert nb > 0, L.grmhd_last_error(None)
    s = torch.empty(nb + 256, dtype=torch.uint8, device=dst.device)
    ptr = (s.data_ptr() + 255) // 256 * 256
    G._check(L.grmhd_remap(dst.h, src.h, ctypes.byref(dst.metric), ctypes.byref(dst.eos),
                           ctypes.c_void_p(ptr), ctypes.c_size_t(nb)), dst.h)
    torch.cuda.synchronize()


def _own(arrs, nx, g=4, face=False):
    out = []
    for a, n in zip(arrs, np.reshape(nx, (-1, 3))):
        if face:
            out.append([a[d, g:g + n[2] + (d == 2), g:g + n[1] + (d == 1), g:g + n[0] + (d == 0)]
                        for d in range(3)])
        else:
            out.append(a[:, g:g + n[2], g:g + n[1], g:g + n[0]])
    return out


def test_tag_and_layout_match_oracle(G):
    root, lev, nx, ll, Ps, Bs = _box({(0, 0, 0), (1, 1, 0)}, p_fine=(0.6,))
    mesh = oracle.Mesh(root, lev, nx, ll, Ps, Bs, nthreads=4)
    pack = _pack_from_mesh(G, mesh)
    tg = pack.tag(0)
    to = amr.tag_blocks(mesh, 0)
    say("tag: blocks", len(lev), "max rel diff", np.abs(tg - to).max() / to.max())
    assert np.allclose(tg, to, rtol=1e-13, atol=0)
    rng = np.random.default_rng(3)
    for trial in range(6):
        tags = rng.integers(-1, 2, size=len(lev)).tolist()
        if trial == 0:
            tags = [-1 if l == 1 else 1 for l in lev]
        got = G.regrid_layout(pack, tags)
        want = amr.regrid_layout(lev, nx, ll, tags)
        assert [list(x) for x in got] == [list(x) for x in want]


@pytest.mark.parametrize("mode", ["refine", "derefine", "mixed", "none"])
def test_remap_matches_oracle(G, mode):
    root, lev, nx, ll, Ps, Bs = _box({(0, 0, 0), (1, 0, 0), (0, 1, 1)}, p_fine=(0.5,))
    mesh = oracle.Mesh(root, lev, nx, ll, Ps, Bs, nthreads=4)
    coarse = [b for b, l in enumerate(lev) if l == 0]
    if mode == "refine":
        tags = [1 if b in coarse[:3] else 0 for b in range(len(lev))]
    elif mode == "derefine":
        tags = [-1 if l == 1 else 0 for l in lev]
    elif mode == "mixed":
        tags = [1 if b == coarse[1] else (-1 if l == 1 else 0) for b, l in enumerate(lev)]
    else:                      # no tag: the same layout, every cell and face copied
        tags = [0] * len(lev)
    nx2, ll2, lv2 = amr.regrid_layout(lev, nx, ll, tags)
    Po, Uo, Bo = amr.remap(mesh, lv2, nx2, ll2)
    src = _pack_from_mesh(G, mesh)
    dst = G.Pack(root, layout=(nx2, ll2, lv2))
    _raw_remap(G, dst, src)
    Pg, Ug, Bg = dst.download_blocks("P"), dst.download_blocks("U"), dst.download_blocks("Bf")
    wc = wf = 0.0
    for name, a, b in (("P", _own(Pg, nx2), _own(Po, nx2)), ("U", _own(Ug, nx2), _own(Uo, nx2))):
        for x, y in zip(a, b):
            den = np.abs(y).max(axis=(1, 2, 3), keepdims=True)
            wc = max(wc, float((np.abs(x - y) / den).max()))
    for x, y in zip(_own(Bg, nx2, face=True), _own(Bo, nx2, face=True)):
        for d in range(3):
            den = max(np.abs(y[d]).max(), 1e-300)
            wf = max(wf, float(np.abs(x[d] - y[d]).max() / den))
    say("remap", mode, len(lev), "->", len(lv2), "blocks; worst relative difference: cells", wc,
        "faces", wf)
    if mode == "none":         # every block is kept whole
        assert wc == 0.0 and wf == 0.0
    else:
        assert wc <= 1e-13 and wf <= 1e-13


def test_regrid_cycle_matches_oracle(G):
    """Two steps, tag by the density indicator, regrid (refine the most
    structured coarse blocks, derefine the smoothest fine groups), remap, two
    more steps: GPU and oracle per block to 1e-11; the remap keeps the totals
    and the divergence at rounding on the GPU."""
    import torch
    root, lev, nx, ll, Ps, Bs = _box({(0, 0, 0), (1, 0, 0)}, p_fine=(0.0,))
    mesh = oracle.Mesh(root, lev, nx, ll, Ps, Bs, nthreads=8)
    pack = G.Pack(root, layout=(nx, ll, lev))
    pack.init_blocks(Ps, Bs)
    for s in range(2):
        dt = mesh.dt()
        mesh.step(dt)
        pack.step(dt)
    tg, to = pack.tag(0), amr.tag_blocks(mesh, 0)
    assert np.allclose(tg, to, rtol=1e-11)
    order = np.argsort(to)
    tags = [0] * len(lev)
    for b in order[::-1]:
        if lev[b] == 0:
            tags[b] = 1
            break
    for b in range(len(lev)):
        if lev[b] == 1:
            tags[b] = -1
    nx2, ll2, lv2 = G.regrid_layout(pack, tags)
    assert (nx2, ll2, lv2) == tuple(amr.regrid_layout(lev, nx, ll, tags))
    r0 = pack.reductions()
    new = G.Pack(root, layout=(nx2, ll2, lv2))
    new.remap_from(pack)
    r1 = new.reductions()
    mesh2 = amr.remapped_mesh(mesh, lv2, nx2, ll2, nthreads=8)
    say("regrid:", len(lev), "->", len(lv2), "blocks; totals drift",
        np.abs(r1["totals"] - r0["totals"]).max() / np.abs(r0["totals"]).max(),
        "divb", r1["divb_rel"], "c2p fail", r1["c2p_fail"], "floors", r1["floor_hits"])
    assert r1["divb_rel"] < 1e-12
    assert r1["floor_hits"] == 0 and r1["c2p_fail_total"] == 0
    assert np.all(totals_drift(r1, r0) <= 1e-13)
    for s in range(2):
        dt = mesh2.dt()
        mesh2.step(dt)
        new.step(dt)
        g = root.ng
        nxa = np.reshape(nx2, (-1, 3))
        Pg, Bg = new.download_blocks("P"), new.download_blocks("Bf")
        eP = max(float(np.abs(x - y).max() / np.abs(y).max()) for x, y in
                 zip(_own(Pg, nx2), _own(mesh2.P, nx2)))
        eB = max(float(np.abs(x[d] - y[d]).max() / max(np.abs(y[d]).max(), 1e-300))
                 for x, y in zip(_own(Bg, nx2, face=True), _own(mesh2.Bf, nx2, face=True))
                 for d in range(3))
        say("after regrid step", s, "eP", eP, "eB", eB)
        assert eP <= 1e-11 and eB <= 1e-11
    torch.cuda.synchronize()


def test_remap_rejects_one_pack_as_both_sides(G):
    """dst and src must be two packs: the same pack on both sides is refused
    on the host, before any launch."""
    import torch
    root, lev, nx, ll, Ps, Bs = _box({(0, 0, 0)})
    pack = G.Pack(root, layout=(nx, ll, lev))
    pack.init_blocks(Ps, Bs)
    torch.cuda.synchronize()
    L = G.lib()
    s = torch.empty(1 << 20, dtype=torch.uint8, device=pack.device)
    ptr = (s.data_ptr() + 255) // 256 * 256
    rc = L.grmhd_remap(pack.h, pack.h, ctypes.byref(pack.metric), ctypes.byref(pack.eos),
                       ctypes.c_void_p(ptr), ctypes.c_size_t(1 << 19))
    assert rc == -1
    assert b"two packs" in L.grmhd_last_error(pack.h)
