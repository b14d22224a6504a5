"""Pins of the oracle's two-level block mesh (ghost zones by prolongation,
restriction and same-level copies; one global dt).

The inter-level operators are pinned by what they must reproduce exactly:
linear primitives and normal-linear face fields (restriction of a linear
function is its value at the coarse centre; the monotonized-central
prolongation of linear data is the linear function), divergence-free face
ghosts, agreement with the single-block ghost fill when all blocks share a
level, and an exactly preserved uniform state."""
import numpy as np
import pytest

import oracle
from paper_2410_09146_amd import inputs as I

FIXED = 3


def _box(n, bc):
    prob = I.uniform_box(n, rho=1.0, u=1.0)
    prob.bc = tuple(bc)
    return prob


def _centre_layout(root_n, node, refine, smallest, seed=5):
    """Regions (level-0 index triples) in `refine` become level 1."""
    def dense(lo, s):
        return tuple(x // node for x in lo) in refine
    return I.two_level_layout(root_n, node, dense, p_coarse=(0.5,), p_fine=(0.6,),
                              smallest=smallest, seed=seed)


def _coords(root, lev, lo, n, ng, loc, face=None):
    """Global coordinates of every cell (or face along `face`) of a block,
    as (X, Y, Z) arrays shaped (s3, s2, s1), and the global indices."""
    out, gidx = [], []
    for d in range(3):
        dxl = root.dx[d] / (1 << lev)
        idx = np.arange(n[d] + 2 * ng) - ng + lo[d]
        off = 0.0 if face == d else 0.5
        out.append(root.xmin[d] + (idx + off) * dxl)
        gidx.append(idx)
    Z, Y, X = np.meshgrid(out[2], out[1], out[0], indexing="ij")
    GZ, GY, GX = np.meshgrid(gidx[2], gidx[1], gidx[0], indexing="ij")
    return (X, Y, Z), (GX, GY, GZ)


def test_linear_data_reproduced_across_levels():
    """Linear primitives and normal-linear densitized faces: every ghost
    inside the domain equals the linear function at its own position."""
    root = _box((32, 32, 32), (FIXED,) * 6)
    lev, nx, ll = _centre_layout(root.n, 8, {(1, 1, 1), (2, 1, 1)}, smallest=8)
    assert 1 in lev and 0 in lev
    nx = np.array(nx).reshape(-1, 3)
    ll = np.array(ll).reshape(-1, 3)
    rng = np.random.default_rng(11)
    coef = rng.uniform(-0.3, 0.3, (5, 4))
    coef[:, 0] = [2.0, 0.1, -0.2, 0.3, 3.0]
    bco = rng.uniform(-0.5, 0.5, (3, 2))
    g = root.ng

    def pfun(q, X, Y, Z):
        return coef[q, 0] + coef[q, 1] * X + coef[q, 2] * Y + coef[q, 3] * Z

    Ps, Bs, exp_P, exp_B, masks = [], [], [], [], []
    for b in range(len(lev)):
        n = nx[b]
        (X, Y, Z), (GX, GY, GZ) = _coords(root, lev[b], ll[b], n, g, None)
        N = [root.n[d] << lev[b] for d in range(3)]
        inside = (GX >= 0) & (GX < N[0]) & (GY >= 0) & (GY < N[1]) & (GZ >= 0) & (GZ < N[2])
        P = np.stack([pfun(q, X, Y, Z) for q in range(5)])
        Bf = np.zeros_like(P[:3])
        for c in range(3):
            (Xf, Yf, Zf), _ = _coords(root, lev[b], ll[b], n, g, None, face=c)
            xc = (Xf, Yf, Zf)[c]
            Bf[c] = bco[c, 0] + bco[c, 1] * xc
        exp_P.append(P.copy())
        exp_B.append(Bf.copy())
        P[:, :g] = 0; P[:, -g:] = 0; P[:, :, :g] = 0; P[:, :, -g:] = 0
        P[:, :, :, :g] = 0; P[:, :, :, -g:] = 0
        Bf2 = np.zeros_like(Bf)
        for c in range(3):
            e = [n[d] + (1 if d == c else 0) for d in range(3)]
            Bf2[c, g:g + e[2], g:g + e[1], g:g + e[0]] = Bf[c, g:g + e[2], g:g + e[1], g:g + e[0]]
        Ps.append(P)
        Bs.append(Bf2)
        masks.append(inside)
    mesh = oracle.Mesh(root, lev, nx, ll, Ps, Bs)
    worst_p = worst_b = 0.0
    for b in range(len(lev)):
        m = masks[b]
        worst_p = max(worst_p, float(np.abs(mesh.P[b] - exp_P[b])[:, m].max()))
        for c in range(3):
            n = nx[b]
            _, (GX, GY, GZ) = _coords(root, lev[b], ll[b], n, g, None, face=c)
            N = [root.n[d] << lev[b] for d in range(3)]
            G = (GX, GY, GZ)
            fm = np.ones(m.shape, bool)
            for d in range(3):
                top = N[d] if d == c else N[d] - 1
                fm &= (G[d] >= 0) & (G[d] <= top)
            worst_b = max(worst_b, float(np.abs(mesh.Bf[b][c] - exp_B[b][c])[fm].max()))
    assert worst_p < 1e-13, worst_p
    assert worst_b < 1e-13, worst_b


def _owner_level(root, lev, nx, ll):
    """Level of the block owning each level-0 cell."""
    own = np.full(root.n[::-1], -1)
    for b in range(len(lev)):
        lo = ll[b] >> lev[b]
        hi = (ll[b] + nx[b]) >> lev[b]
        own[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = lev[b]
    assert (own >= 0).all()
    return own


def test_ghost_faces_divergence_free():
    """A divergence-free two-level field (level 1 = discrete curl, level 0 =
    its restriction): prolonged fine ghost cells and restricted coarse ghost
    cells carry zero divergence."""
    fine = I.random_smooth_box((32, 32, 32), seed=4, amp=0.2)
    root = I.coarse_problem(fine)
    lev, nx, ll = _centre_layout(root.n, 8, {(0, 0, 0), (1, 0, 1), (1, 1, 1)}, smallest=8)
    Ps, Bs = I.mesh_blocks(fine, lev, nx, ll)
    mesh = oracle.Mesh(root, lev, nx, ll, Ps, Bs)
    nx = np.array(nx).reshape(-1, 3)
    ll = np.array(ll).reshape(-1, 3)
    own = _owner_level(root, np.array(lev), nx, ll)
    g = root.ng
    bmax = max(np.abs(B).max() for B in mesh.Bf)
    checked, worst = 0, 0.0
    for b in range(len(lev)):
        L = lev[b]
        n = nx[b]
        dx = [root.dx[d] / (1 << L) for d in range(3)]
        B = mesh.Bf[b]
        div = ((B[0, :-1, :-1, 1:] - B[0, :-1, :-1, :-1]) / dx[0] +
               (B[1, :-1, 1:, :-1] - B[1, :-1, :-1, :-1]) / dx[1] +
               (B[2, 1:, :-1, :-1] - B[2, :-1, :-1, :-1]) / dx[2])
        s = n + 2 * g
        for k in range(s[2] - 1):
            for j in range(s[1] - 1):
                for i in range(s[0] - 1):
                    loc = (i, j, k)
                    if all(g <= loc[d] < g + n[d] for d in range(3)):
                        continue
                    G = [ll[b][d] + loc[d] - g for d in range(3)]   # periodic box
                    N = [root.n[d] << L for d in range(3)]
                    ok = True
                    for c in range(3):          # a face of the block's own: not a ghost
                        for up in (0, 1):
                            f = [loc[e] + (up if e == c else 0) for e in range(3)]
                            if all(g <= f[e] <= g + n[e] - (0 if e == c else 1) for e in range(3)):
                                ok = False
                    for c in range(3):          # level owning each face of the cell
                        for up in (0, 1):
                            # the two cells beside the face (periodic box): the
                            # finer one owns it, else the one above
                            F = [G[e] + (up if e == c else 0) for e in range(3)]
                            above = [F[e] % N[e] for e in range(3)]
                            below = list(above)
                            below[c] = (F[c] - 1) % N[c]
                            la = own[above[2] >> L, above[1] >> L, above[0] >> L]
                            lb = own[below[2] >> L, below[1] >> L, below[0] >> L]
                            if max(la, lb) == L:
                                ok = False      # a same-level copy: not an inter-level value
                    if not ok:
                        continue
                    checked += 1
                    worst = max(worst, abs(div[k, j, i]))
    assert checked > 500
    assert worst < 1e-12 * bmax / min(root.dx) * 2, (worst, checked)


@pytest.mark.parametrize("level", [0, 1])
def test_same_level_mesh_equals_single_block_fill(level):
    """All blocks on one level: the mesh fill must equal the single-block
    ghost fill of the whole grid (torus boundaries: outflow, polar, periodic)."""
    n = (32, 32, 16)
    prob = I.torus(n=n)
    blk = oracle.Block(prob)
    Pg, Bg = prob.P.copy(), prob.Bf.copy()
    blk.fill_ghosts(Pg, Bg)
    nxb, llb = I.octree_layout(n, base=16, smallest=8, p_split=(0.5,), seed=3)
    lev = [level] * (len(nxb) // 3)
    root = I.coarse_problem(prob) if level == 1 else prob
    g = prob.ng
    nxa = np.array(nxb).reshape(-1, 3)
    lla = np.array(llb).reshape(-1, 3)
    Ps, Bs = [], []
    for b in range(len(lev)):
        sl = tuple(slice(lla[b][2 - d], lla[b][2 - d] + nxa[b][2 - d] + 2 * g) for d in range(3))
        P = prob.P[(slice(None),) + sl].copy()
        Bf = prob.Bf[(slice(None),) + sl].copy()
        P[:, :g] = -7.0
        Bf[:, :g] = -7.0
        Ps.append(P)
        Bs.append(Bf)
    mesh = oracle.Mesh(root, lev, nxb, llb, Ps, Bs)
    for b in range(len(lev)):
        sl = tuple(slice(lla[b][2 - d], lla[b][2 - d] + nxa[b][2 - d] + 2 * g) for d in range(3))
        assert np.array_equal(mesh.P[b], Pg[(slice(None),) + sl])
        for c in range(3):
            assert np.array_equal(mesh.Bf[b][c], Bg[(c,) + sl])


def test_two_level_uniform_state_preserved_exactly():
    fine = I.uniform_box((32, 32, 32), rho=1.3, ut=(0.2, -0.1, 0.05), u=0.7, B=(0.3, 0.2, -0.1))
    root = I.coarse_problem(fine)
    lev, nx, ll = _centre_layout(root.n, 8, {(0, 0, 0), (1, 1, 0)}, smallest=8)
    Ps, Bs = I.mesh_blocks(fine, lev, nx, ll)
    mesh = oracle.Mesh(root, lev, nx, ll, Ps, Bs, nthreads=4)
    U_ref = [u.copy() for u in mesh.U]
    mesh.step()
    g = root.ng
    nx = np.array(nx).reshape(-1, 3)
    for b in range(len(lev)):
        n = nx[b]
        it = (slice(None), slice(g, g + n[2]), slice(g, g + n[1]), slice(g, g + n[0]))
        assert np.abs(mesh.P[b][it] - fine.P[(slice(None),) + (slice(g, g + n[2]),
                                                               slice(g, g + n[1]),
                                                               slice(g, g + n[0]))]).max() < 1e-14
        assert np.abs(mesh.U[b][it] - U_ref[b][it]).max() < 1e-14


def test_mesh_reductions_match_single_level():
    """Reductions of a same-level mesh equal the single-block ones."""
    prob = I.random_smooth_box((16, 16, 16), seed=2)
    blk = oracle.Block(prob)
    P, Bf = prob.P.copy(), prob.Bf.copy()
    blk.fill_ghosts(P, Bf)
    U = blk.prim_to_cons(P, Bf)
    ref = blk.reductions(P, Bf, U, prob.cfl)
    nxb, llb = I.octree_layout(prob.n, base=8, smallest=8, p_split=(0.0,), seed=1)
    g = prob.ng
    nxa = np.array(nxb).reshape(-1, 3)
    lla = np.array(llb).reshape(-1, 3)
    Ps, Bs = [], []
    for b in range(len(nxa)):
        sl = tuple(slice(lla[b][2 - d], lla[b][2 - d] + nxa[b][2 - d] + 2 * g) for d in range(3))
        Ps.append(P[(slice(None),) + sl].copy())
        Bs.append(Bf[(slice(None),) + sl].copy())
    mesh = oracle.Mesh(prob, [0] * len(nxa), nxb, llb, Ps, Bs)
    red = mesh.reductions()
    assert red["dt"] == pytest.approx(ref["dt"], rel=1e-15)
    assert red["divb_max"] == pytest.approx(ref["divb_max"], rel=1e-12, abs=1e-14)
    assert np.allclose(red["totals"], ref["totals"], rtol=1e-13, atol=1e-15)


def _box_two_level(correct):
    fine = I.random_smooth_box((32, 32, 32), seed=6, amp=0.1)
    root = I.coarse_problem(fine)
    ref = {(0, 0, 0), (1, 1, 0), (1, 0, 1)}
    lev, nx, ll = I.two_level_layout(root.n, 8, lambda lo, s: tuple(x // 8 for x in lo) in ref,
                                     p_coarse=(0.5,), p_fine=(0.6,), smallest=8, seed=2)
    Ps, Bs = I.mesh_blocks(fine, lev, nx, ll)
    return root, lev, oracle.Mesh(root, lev, nx, ll, Ps, Bs, nthreads=4, correct=correct)


def test_level_coupling_conserves():
    """Periodic two-level box: with the coarse fluxes at level boundaries
    replaced by the mean of the fine ones, the totals of sqrt(gamma) U are
    conserved to rounding over three steps; without, they are not."""
    out = {}
    for corr in (False, True):
        root, lev, mesh = _box_two_level(corr)
        t0 = mesh.reductions()["totals"]
        for _ in range(3):
            mesh.step()
        t1 = mesh.reductions()["totals"]
        out[corr] = np.abs(t1 - t0).max() / np.abs(t0).max()
    assert out[True] < 1e-14, out
    assert out[False] > 1e-8, out


def test_level_boundary_faces_stay_restrictions():
    """With the coarse EMFs on level boundaries replaced by the mean of the
    fine EMFs, every coarse face on a level boundary stays the mean of its 4
    fine faces (the composite field keeps one divergence-free flux through
    the interface)."""
    root, lev, mesh = _box_two_level(True)
    for _ in range(3):
        mesh.step()
    g = root.ng
    nx, ll = mesh.nx, mesh.lloc
    N0 = root.n
    own = np.full(N0[::-1], -1)
    for b in range(mesh.nb):
        lo = ll[b] >> lev[b]
        hi = (ll[b] + nx[b]) >> lev[b]
        own[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = b
    worst, count = 0.0, 0
    scale = max(np.abs(B).max() for B in mesh.Bf)
    for c in range(mesh.nb):
        if lev[c] != 0:
            continue
        for d in range(3):
            t1, t2 = (d + 1) % 3, (d + 2) % 3
            for side in (0, 1):
                other = (ll[c][d] + nx[c][d]) % N0[d] if side else (ll[c][d] - 1) % N0[d]
                for u2 in range(nx[c][t2]):
                    for u1 in range(nx[c][t1]):
                        C0 = [0, 0, 0]
                        C0[d], C0[t1], C0[t2] = other, ll[c][t1] + u1, ll[c][t2] + u2
                        f = own[C0[2], C0[1], C0[0]]
                        if lev[f] != 1:
                            continue
                        Lc = [0, 0, 0]
                        Lc[d], Lc[t1], Lc[t2] = g + (nx[c][d] if side else 0), g + u1, g + u2
                        vc = mesh.Bf[c][d][Lc[2], Lc[1], Lc[0]]
                        X = [0, 0, 0]
                        X[d] = 2 * other if side else 2 * (other + 1)
                        vals = []
                        for a in (0, 1):
                            for bb in (0, 1):
                                X[t1], X[t2] = 2 * C0[t1] + a, 2 * C0[t2] + bb
                                Lf = [X[k] - ll[f][k] + g for k in range(3)]
                                vals.append(mesh.Bf[f][d][Lf[2], Lf[1], Lf[0]])
                        worst = max(worst, abs(vc - np.mean(vals)) / scale)
                        count += 1
    assert count > 100
    assert worst < 1e-13, worst
