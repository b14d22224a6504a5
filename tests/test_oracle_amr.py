"""Pins of the oracle's mesh refinement (two-level block mesh: tagging, the
next layout, the conservative and divergence-free remap).  The paper
evolves on Parthenon's adaptive block mesh (Sec. 1, Sec. 3) and does not
give the operators; the ones pinned here are a reading of that mesh."""
import numpy as np
import pytest

import oracle
from oracle import amr
from paper_2410_09146_amd import inputs as I


def _box_mesh(refined, seed=6, amp=0.1, n=16, node=8):
    fine = I.random_smooth_box((2 * n,) * 3, seed=seed, amp=amp)
    root = I.coarse_problem(fine)
    lev, nx, ll = I.two_level_layout(root.n, node, lambda lo, s: tuple(x // node for x in lo) in refined,
                                     p_coarse=(0.0,), p_fine=(0.0,), smallest=node, seed=2)
    Ps, Bs = I.mesh_blocks(fine, lev, nx, ll)
    return oracle.Mesh(root, lev, nx, ll, Ps, Bs, nthreads=4)


def _totals(mesh_or_layout, U, dx):
    lev, nx = mesh_or_layout
    g = 4
    tot = np.zeros(U[0].shape[0])
    for b, (l, n) in enumerate(zip(lev, np.asarray(nx).reshape(-1, 3))):
        vol = np.prod([dx[d] / (1 << l) for d in range(3)])
        tot += U[b][:, g:g + n[2], g:g + n[1], g:g + n[0]].sum(axis=(1, 2, 3)) * vol
    return tot


def _div(lev, nx, B, dx):
    g = 4
    worst = 0.0
    for b, (l, n) in enumerate(zip(lev, np.asarray(nx).reshape(-1, 3))):
        h = [dx[d] / (1 << l) for d in range(3)]
        Bx, By, Bz = B[b]
        it = (slice(g, g + n[2]), slice(g, g + n[1]), slice(g, g + n[0]))
        div = (Bx[g:g + n[2], g:g + n[1], g + 1:g + n[0] + 1] - Bx[it]) / h[0] \
            + (By[g:g + n[2], g + 1:g + n[1] + 1, g:g + n[0]] - By[it]) / h[1] \
            + (Bz[g + 1:g + n[2] + 1, g:g + n[1], g:g + n[0]] - Bz[it]) / h[2]
        worst = max(worst, np.abs(div).max())
    return worst


def test_regrid_layout_refine_then_derefine_is_identity():
    """Refining tagged level-0 blocks and then derefining all level-1 blocks
    gives the original single-level layout back (as a set of blocks)."""
    mesh = _box_mesh(set())
    lev, nx, ll = mesh.level.tolist(), mesh.nx.ravel().tolist(), mesh.lloc.ravel().tolist()
    tags = [1 if b % 3 == 0 else 0 for b in range(len(lev))]
    nx2, ll2, lv2 = amr.regrid_layout(lev, nx, ll, tags)
    assert len(lv2) == len(lev) + 7 * sum(1 for t in tags if t > 0)
    assert sum(np.prod(n) << (3 * (1 - l)) for n, l in zip(np.reshape(nx2, (-1, 3)), lv2)) == \
        8 * np.prod(mesh.root.n)
    nx3, ll3, lv3 = amr.regrid_layout(lv2, nx2, ll2, [-1] * len(lv2))
    blocks = lambda lv, n_, l_: sorted(zip(lv, map(tuple, np.reshape(n_, (-1, 3))),
                                           map(tuple, np.reshape(l_, (-1, 3)))))
    assert blocks(lv3, nx3, ll3) == blocks(lev, nx, ll)
    # a partial group is not merged: its tagged members become level-0
    # blocks over their own regions (half size), the untagged one stays
    tags3 = [-1] * len(lv2)
    first_fine = lv2.index(1)
    tags3[first_fine] = 0
    nx4, ll4, lv4 = amr.regrid_layout(lv2, nx2, ll2, tags3)
    assert lv4.count(1) == 1
    halves = [tuple(n) for n, l in zip(np.reshape(nx4, (-1, 3)), lv4) if l == 0 and n[0] == 4]
    assert len(halves) == 7
    assert sum(np.prod(n) << (3 * (1 - l)) for n, l in zip(np.reshape(nx4, (-1, 3)), lv4)) == \
        8 * np.prod(mesh.root.n)


def test_remap_identity_layout_copies():
    """A layout equal to the current one copies every block's cells and
    faces, also the coarse faces on level boundaries (a block's own value,
    not the mean of the fine faces across it)."""
    mesh = _box_mesh({(0, 0, 0)})
    P, U, B = amr.remap(mesh, mesh.level, mesh.nx, mesh.lloc)
    g = 4
    for b in range(mesh.nb):
        n = mesh.nx[b]
        it = (slice(None), slice(g, g + n[2]), slice(g, g + n[1]), slice(g, g + n[0]))
        assert np.array_equal(P[b][it], mesh.P[b][it])
        assert np.array_equal(U[b][it], mesh.U[b][it])
        for d in range(3):
            f = (d, slice(g, g + n[2] + (d == 2)), slice(g, g + n[1] + (d == 1)),
                 slice(g, g + n[0] + (d == 0)))
            assert np.array_equal(B[b][f], mesh.Bf[b][f])


@pytest.mark.parametrize("mode", ["refine", "derefine"])
def test_remap_conserves_and_stays_divergence_free(mode):
    """Totals of U are kept (restriction and mean-preserving prolongation),
    and every cell of the new layout is divergence-free to rounding, also
    where new fine blocks border existing fine blocks."""
    mesh = _box_mesh({(0, 0, 0), (1, 0, 0)})
    lev, nx, ll = mesh.level.tolist(), mesh.nx.ravel().tolist(), mesh.lloc.ravel().tolist()
    if mode == "refine":
        # the level-0 block next to the refined region, and one further away
        tags = [0] * len(lev)
        coarse = [b for b, l in enumerate(lev) if l == 0]
        tags[coarse[0]] = tags[coarse[3]] = 1
    else:
        tags = [-1 if l == 1 else 0 for l in lev]
    nx2, ll2, lv2 = amr.regrid_layout(lev, nx, ll, tags)
    assert lv2 != lev
    P, U, B = amr.remap(mesh, lv2, nx2, ll2)
    dx = mesh.root.dx
    t0 = _totals((lev, nx), mesh.U, dx)
    t1 = _totals((lv2, nx2), U, dx)
    assert np.allclose(t1, t0, rtol=1e-13, atol=1e-13 * np.abs(t0).max())
    d0 = _div(lev, nx, mesh.Bf, dx)
    d1 = _div(lv2, nx2, B, dx)
    bmax = max(np.abs(x).max() for x in mesh.Bf)
    assert d0 <= 1e-12 * bmax / min(dx) and d1 <= 1e-12 * bmax / min(dx), (d0, d1)


def test_refine_then_derefine_returns_the_state():
    """Restricting a prolonged state gives it back: the mean of the 8
    children of each cell is the parent, the mean of the 4 fine faces of each
    coarse face is the coarse face."""
    mesh = _box_mesh(set())
    lev, nx, ll = mesh.level.tolist(), mesh.nx.ravel().tolist(), mesh.lloc.ravel().tolist()
    tags = [1] * len(lev)
    nx2, ll2, lv2 = amr.regrid_layout(lev, nx, ll, tags)
    P, U, B = amr.remap(mesh, lv2, nx2, ll2)
    fine = oracle.Mesh(mesh.root, lv2, nx2, ll2, P, B, nthreads=4)
    fine.U = U
    back = amr.regrid_layout(lv2, nx2, ll2, [-1] * len(lv2))
    P3, U3, B3 = amr.remap(fine, *[back[2], back[0], back[1]])
    # the merged layout is the original one up to block order
    key = lambda lv, ll_: {tuple(x): i for i, x in enumerate(np.reshape(ll_, (-1, 3)))}
    k0, k3 = key(lev, ll), key(back[2], back[1])
    g = 4
    for loc, b0 in k0.items():
        b3 = k3[loc]
        n = mesh.nx[b0]
        it = (slice(None), slice(g, g + n[2]), slice(g, g + n[1]), slice(g, g + n[0]))
        assert np.allclose(U3[b3][it], mesh.U[b0][it], rtol=1e-14, atol=1e-15)
        for d in range(3):
            e = [n[k] + (1 if k == d else 0) for k in range(3)]
            f = (d, slice(g, g + e[2]), slice(g, g + e[1]), slice(g, g + e[0]))
            assert np.allclose(B3[b3][f], mesh.Bf[b0][f], rtol=1e-13, atol=1e-14)


def test_prolongation_of_linear_data_is_exact():
    """Linear P: the MC slopes are the exact gradient, so the children take
    the linear function at their centres; the children's U keep the parent's
    U on average."""
    mesh = _box_mesh(set())
    g = 4
    h = mesh.root.dx
    for b in range(mesh.nb):
        n = mesh.nx[b]
        s = n + 2 * g
        Z, Y, X = np.meshgrid(*[(np.arange(s[2 - d]) - g + mesh.lloc[b][2 - d] + 0.5) * h[2 - d]
                                for d in range(3)], indexing="ij")
        for q in range(5):
            mesh.P[b][q] = 1.0 + 0.03 * X - 0.02 * Y + 0.01 * Z + (0.0 if q in (0, 4) else -0.9)
        mesh.U[b] = mesh.blocks[b].prim_to_cons(mesh.P[b], mesh.Bf[b])
    lev, nx, ll = mesh.level.tolist(), mesh.nx.ravel().tolist(), mesh.lloc.ravel().tolist()
    nx2, ll2, lv2 = amr.regrid_layout(lev, nx, ll, [1] + [0] * (len(lev) - 1))
    P, U, B = amr.remap(mesh, lv2, nx2, ll2)
    n0 = mesh.nx[0]
    for b, (l, n, L) in enumerate(zip(lv2, np.reshape(nx2, (-1, 3)), np.reshape(ll2, (-1, 3)))):
        if l != 1:
            continue
        hf = [x / 2 for x in h]
        Z, Y, X = np.meshgrid(*[(np.arange(n[2 - d]) + L[2 - d] + 0.5) * hf[2 - d] for d in range(3)],
                              indexing="ij")
        it = (slice(g, g + n[2]), slice(g, g + n[1]), slice(g, g + n[0]))
        for q in range(5):
            lin = 1.0 + 0.03 * X - 0.02 * Y + 0.01 * Z + (0.0 if q in (0, 4) else -0.9)
            assert np.allclose(P[b][q][it], lin, rtol=1e-13, atol=1e-14)
        for k in range(0, n[2], 2):
            for j in range(0, n[1], 2):
                for i in range(0, n[0], 2):
                    pc = [(L[0] + i) // 2, (L[1] + j) // 2, (L[2] + k) // 2]
                    kids = U[b][:, g + k:g + k + 2, g + j:g + j + 2, g + i:g + i + 2].mean(axis=(1, 2, 3))
                    par = mesh.U[0][:, g + pc[2], g + pc[1], g + pc[0]]
                    assert np.allclose(kids, par, rtol=1e-13, atol=1e-15)


def test_tag_indicator():
    mesh = _box_mesh(set())
    t = amr.tag_blocks(mesh, 0)
    assert t.shape == (mesh.nb,) and np.all(t > 0)
    # a uniform density has indicator 0
    for b in range(mesh.nb):
        mesh.P[b][0][:] = 1.3
    assert np.all(amr.tag_blocks(mesh, 0) == 0.0)
