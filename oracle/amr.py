"""Oracle of the two-level mesh refinement: tagging, the next layout, and the
remap of a state onto it.  TEST INFRASTRUCTURE ONLY (see orc.h).

Plain numpy over per-block padded arrays (nvar, s3, s2, s1) as oracle.Mesh
holds them.  The operators (not given in the paper, which relies on
Parthenon's refinement):
  * indicator of a block: max over its interior cells and the directions
    with more than one cell of |q(i+1) - q(i-1)| / (2 |q(i)|);
  * next layout: a tagged (+1) level-0 block with even sizes -> its 8 level-1
    children; 8 level-1 siblings (one cubic size m at base + {0, m}^3, base a
    multiple of 2m) all tagged -1 -> one level-0 block of size m; any other
    level-1 block tagged -1 -> the level-0 block over the same region (half
    its size, if that is at least the ghost depth); other blocks kept, in
    order, children and merged blocks at the place of their first source;
  * remap per cell: copy from the block of the same level, mean of the 8
    children, or, for new fine cells, P by parent + monotonized-central
    slopes toward the octant (from its ghosts; the parent where rho or u
    would not stay positive) and U = U(P, B) of each child with the new face
    field plus the parent's U minus the mean of its 8 children (the totals
    are kept);
  * remap per face: copy, mean of the 4 fine faces, or (new fine faces) the
    face of an existing fine cell across a coarse face, else the coarse
    value; the 12 faces inside a coarse cell: the linear interpolation
    between the outer faces plus the minimum-norm correction that zeroes the
    divergence of the 8 children (numpy's least-squares solution).
"""
import numpy as np


def mc(dm, dp):
    if dm * dp <= 0.0:
        return 0.0
    s = min(2.0 * abs(dm), 2.0 * abs(dp), 0.5 * abs(dm + dp))
    return s if dm > 0.0 else -s


def tag_blocks(mesh, var=0):
    g = mesh.root.ng
    out = []
    for b in range(mesh.nb):
        q = mesh.P[b][var]
        n = mesh.nx[b]
        c = q[g:g + n[2], g:g + n[1], g:g + n[0]]
        best = 0.0
        for d in range(3):
            if mesh.root.n[d] <= 1:
                continue
            ax = 2 - d
            up = np.roll(q, -1, axis=ax)[g:g + n[2], g:g + n[1], g:g + n[0]]
            dn = np.roll(q, 1, axis=ax)[g:g + n[2], g:g + n[1], g:g + n[0]]
            best = max(best, float((np.abs(up - dn) / (2.0 * np.abs(c) + 1e-300)).max()))
        out.append(best)
    return np.array(out)


def regrid_layout(level, nx, lloc, tags, ng=4):
    level = [int(v) for v in level]
    nx = np.asarray(nx, dtype=int).reshape(-1, 3)
    lloc = np.asarray(lloc, dtype=int).reshape(-1, 3)
    nb = len(level)
    groups = {}
    for b in range(nb):
        if level[b] != 1 or len(set(nx[b].tolist())) != 1:
            continue
        m = int(nx[b, 0])
        base = tuple(int(v) - int(v) % (2 * m) for v in lloc[b])
        groups.setdefault((m,) + base, []).append(b)
    merged = {}
    for key, members in groups.items():
        if len(members) == 8 and all(tags[b] < 0 for b in members):
            lead = min(members)
            for b in members:
                merged[b] = lead
    out_nx, out_ll, out_lv = [], [], []
    for b in range(nb):
        n, ll = nx[b], lloc[b]
        if level[b] == 0 and tags[b] > 0 and not (n % 2).any():
            for z in range(2):
                for y in range(2):
                    for x in range(2):
                        out_nx += n.tolist()
                        out_ll += [2 * ll[0] + x * n[0], 2 * ll[1] + y * n[1], 2 * ll[2] + z * n[2]]
                        out_lv.append(1)
        elif b in merged:
            if merged[b] == b:
                m = int(n[0])
                out_nx += [m, m, m]
                out_ll += [(int(v) - int(v) % (2 * m)) // 2 for v in ll]
                out_lv.append(0)
        elif level[b] == 1 and tags[b] < 0 and (n // 2 >= ng).all():
            out_nx += (n // 2).tolist()
            out_ll += (ll // 2).tolist()
            out_lv.append(0)
        else:
            out_nx += n.tolist()
            out_ll += ll.tolist()
            out_lv.append(level[b])
    return out_nx, out_ll, out_lv


class _Lookup:
    """Which block of a layout holds global cell c of level l."""

    def __init__(self, root_n, level, nx, lloc):
        self.root_n = root_n
        self.maps = {}
        for l in (0, 1):
            self.maps[l] = -np.ones(tuple(root_n[2 - d] << l for d in range(3)), dtype=np.int64)
        for b, (lv, n, ll) in enumerate(zip(level, nx, lloc)):
            for l in (0, 1):
                if l == lv:
                    lo, hi = ll, ll + n
                elif l == 0:             # a fine block seen at level 0
                    lo, hi = ll // 2, (ll + n) // 2
                else:                    # a coarse block seen at level 1
                    lo, hi = 2 * ll, 2 * (ll + n)
                self.maps[l][lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = b

    def at(self, l, c):
        N = [self.root_n[d] << l for d in range(3)]
        if any(c[d] < 0 or c[d] >= N[d] for d in range(3)):
            return -1
        return int(self.maps[l][c[2], c[1], c[0]])


def remap(src, level, nx, lloc):
    """Per-block padded (P, U, Bf) of the layout (level, nx, lloc) from the
    oracle mesh src (ghosts filled); ghost zones of the result are zero."""
    root = src.root
    g = root.ng
    level = [int(v) for v in level]
    nx = np.asarray(nx, dtype=int).reshape(-1, 3)
    lloc = np.asarray(lloc, dtype=int).reshape(-1, 3)
    look = _Lookup(root.n, src.level, src.nx, src.lloc)
    slev, sll = src.level, src.lloc
    per = [root.bc[2 * d] == 0 for d in range(3)]

    def loc(b, c, lsrc):
        """Local (k, j, i) of level-lsrc cell c in source block b."""
        return tuple(int(c[2 - d] - sll[b][2 - d] + g) for d in range(3))

    def sface(bs, comp, cu, cl, up):
        """Face value in source block bs: lower face of cu or upper face of cl."""
        if up:
            return src.Bf[bs][(comp,) + loc(bs, cu, 0)]
        k, j, i = loc(bs, cl, 0)
        ijk = [i, j, k]
        ijk[comp] += 1
        return src.Bf[bs][comp, ijk[2], ijk[1], ijk[0]]

    Ps, Us, Bs = [], [], []
    parents = []           # (dst block, k, j, i of child (0,0,0), parent U)
    fine_dx = None
    for b in range(len(level)):
        if level[b] == 1:
            fine_dx = [root.dx[d] / 2 for d in range(3)]
            break
    for b, (l, n, L) in enumerate(zip(level, nx, lloc)):
        shp = tuple(int(n[2 - d]) + 2 * g for d in range(3))
        P = np.zeros((5,) + shp)
        U = np.zeros((5,) + shp)
        B = np.zeros((3,) + shp)
        # a block present in both layouts (same level, position and size)
        # keeps its own state: cells and every face, the faces it shares with
        # a finer neighbour included
        kept = [bs for bs in range(len(slev)) if slev[bs] == l and
                tuple(sll[bs]) == tuple(L) and tuple(src.nx[bs]) == tuple(n)]
        if kept:
            bs = kept[0]
            it = (slice(None), slice(g, g + n[2]), slice(g, g + n[1]), slice(g, g + n[0]))
            P[it] = src.P[bs][it]
            U[it] = src.U[bs][it]
            for d in range(3):
                f = (d, slice(g, g + n[2] + (d == 2)), slice(g, g + n[1] + (d == 1)),
                     slice(g, g + n[0] + (d == 0)))
                B[f] = src.Bf[bs][f]
            Ps.append(P)
            Us.append(U)
            Bs.append(B)
            continue
        for k in range(n[2]):
            for j in range(n[1]):
                for i in range(n[0]):
                    c = (L[0] + i, L[1] + j, L[2] + k)
                    t = (slice(None), g + k, g + j, g + i)
                    bs = look.at(l, c)
                    if slev[bs] == l:
                        P[t] = src.P[bs][(slice(None),) + loc(bs, c, l)]
                        U[t] = src.U[bs][(slice(None),) + loc(bs, c, l)]
                    elif l == 0:
                        c2 = [2 * v for v in c]
                        kk, jj, ii = loc(bs, c2, 1)
                        P[t] = src.P[bs][:, kk:kk + 2, jj:jj + 2, ii:ii + 2].mean(axis=(1, 2, 3))
                        U[t] = src.U[bs][:, kk:kk + 2, jj:jj + 2, ii:ii + 2].mean(axis=(1, 2, 3))
                    else:
                        pc = [v // 2 for v in c]
                        kk, jj, ii = loc(bs, pc, 0)
                        octv = [c[d] & 1 for d in range(3)]
                        for q in range(5):
                            arr = src.P[bs][q]
                            c0 = arr[kk, jj, ii]
                            nb_ = {0: (arr[kk, jj, ii - 1], arr[kk, jj, ii + 1]),
                                   1: (arr[kk, jj - 1, ii], arr[kk, jj + 1, ii]),
                                   2: (arr[kk - 1, jj, ii], arr[kk + 1, jj, ii])}
                            sl = [mc(c0 - nb_[d][0], nb_[d][1] - c0) for d in range(3)]
                            v = c0 + 0.25 * sum(sl[d] if octv[d] else -sl[d] for d in range(3))
                            if q in (0, 4) and (not (v > 0.0) or not np.isfinite(v)):
                                v = c0
                            P[(q, g + k, g + j, g + i)] = v
                        if not any(octv):
                            parents.append((b, k, j, i, src.U[bs][:, kk, jj, ii].copy()))
        # faces
        N = [root.n[d] << l for d in range(3)]
        for d in range(3):
            for k in range(n[2] + (d == 2)):
                for j in range(n[1] + (d == 1)):
                    for i in range(n[0] + (d == 0)):
                        cu = [L[0] + i, L[1] + j, L[2] + k]
                        cl = list(cu)
                        cl[d] -= 1
                        upin = cu[d] < N[d]
                        cs = cu if upin else cl
                        bs = look.at(l, cs)
                        t = (d, g + k, g + j, g + i)
                        if slev[bs] == l:
                            B[t] = sface(bs, d, cu, cl, upin)
                        elif l == 0:
                            fu = [2 * v for v in cu]
                            flo = [2 * v for v in cl]
                            flo[d] += 1
                            tr = [e for e in range(3) if e != d]
                            acc = 0.0
                            for a1 in range(2):
                                for a2 in range(2):
                                    u2, l2 = list(fu), list(flo)
                                    u2[tr[0]] += a1; l2[tr[0]] += a1
                                    u2[tr[1]] += a2; l2[tr[1]] += a2
                                    acc += sface(bs, d, u2, l2, upin)
                            B[t] = 0.25 * acc
                        else:
                            if cu[d] % 2:
                                continue
                            co = list(cl if upin else cu)
                            ok = True
                            if co[d] < 0 or co[d] >= N[d]:
                                if per[d]:
                                    co[d] %= N[d]
                                else:
                                    ok = False
                            bo = look.at(1, co) if ok else -1
                            if bo >= 0 and slev[bo] == 1:
                                B[t] = sface(bo, d, co, co, not upin) if not upin else \
                                    sface(bo, d, None, co, False)
                            else:
                                pu = [v // 2 for v in cu]
                                pl = [v // 2 for v in cl]
                                B[t] = sface(bs, d, pu, pl, upin)
        # faces inside refined parents
        if l == 1:
            Dm = np.zeros((8, 12))
            idx = [1.0 / fine_dx[e] for e in range(3)]
            for c_ in range(2):
                for b_ in range(2):
                    for a_ in range(2):
                        r = a_ + 2 * b_ + 4 * c_
                        Dm[r, b_ + 2 * c_] = -idx[0] if a_ else idx[0]
                        Dm[r, 4 + a_ + 2 * c_] = -idx[1] if b_ else idx[1]
                        Dm[r, 8 + a_ + 2 * b_] = -idx[2] if c_ else idx[2]
            for k in range(0, n[2], 2):
                for j in range(0, n[1], 2):
                    for i in range(0, n[0], 2):
                        c = (L[0] + i, L[1] + j, L[2] + k)
                        if slev[look.at(1, c)] != 0:
                            continue
                        K0, J0, I0 = g + k, g + j, g + i
                        Bx = lambda a, bb, cc: B[0, K0 + cc, J0 + bb, I0 + a]
                        By = lambda a, bb, cc: B[1, K0 + cc, J0 + bb, I0 + a]
                        Bz = lambda a, bb, cc: B[2, K0 + cc, J0 + bb, I0 + a]
                        x0 = np.zeros(12)
                        for c_ in range(2):
                            for b_ in range(2):
                                x0[b_ + 2 * c_] = 0.5 * (Bx(0, b_, c_) + Bx(2, b_, c_))
                        for c_ in range(2):
                            for a_ in range(2):
                                x0[4 + a_ + 2 * c_] = 0.5 * (By(a_, 0, c_) + By(a_, 2, c_))
                        for b_ in range(2):
                            for a_ in range(2):
                                x0[8 + a_ + 2 * b_] = 0.5 * (Bz(a_, b_, 0) + Bz(a_, b_, 2))
                        rhs = np.zeros(8)
                        for c_ in range(2):
                            for b_ in range(2):
                                for a_ in range(2):
                                    xl = x0[b_ + 2 * c_] if a_ else Bx(0, b_, c_)
                                    xh = Bx(2, b_, c_) if a_ else x0[b_ + 2 * c_]
                                    yl = x0[4 + a_ + 2 * c_] if b_ else By(a_, 0, c_)
                                    yh = By(a_, 2, c_) if b_ else x0[4 + a_ + 2 * c_]
                                    zl = x0[8 + a_ + 2 * b_] if c_ else Bz(a_, b_, 0)
                                    zh = Bz(a_, b_, 2) if c_ else x0[8 + a_ + 2 * b_]
                                    rhs[a_ + 2 * b_ + 4 * c_] = -((xh - xl) * idx[0] + (yh - yl) * idx[1]
                                                                  + (zh - zl) * idx[2])
                        x = x0 + np.linalg.lstsq(Dm, rhs, rcond=None)[0]
                        for c_ in range(2):
                            for b_ in range(2):
                                B[0, K0 + c_, J0 + b_, I0 + 1] = x[b_ + 2 * c_]
                        for c_ in range(2):
                            for a_ in range(2):
                                B[1, K0 + c_, J0 + 1, I0 + a_] = x[4 + a_ + 2 * c_]
                        for b_ in range(2):
                            for a_ in range(2):
                                B[2, K0 + 1, J0 + b_, I0 + a_] = x[8 + a_ + 2 * b_]
        Ps.append(P)
        Us.append(U)
        Bs.append(B)
    if parents:
        # refined cells: U(P, B) of each child plus the parent's excess over
        # the children's mean
        import oracle as _o
        tmp = _o.Mesh(root, level, nx.ravel(), lloc.ravel(), Ps, Bs, correct=False)
        for b, k, j, i, up in parents:
            sl = (slice(None), slice(g + k, g + k + 2), slice(g + j, g + j + 2), slice(g + i, g + i + 2))
            kids = tmp.U[b][sl]
            Us[b][sl] = kids + (up - kids.mean(axis=(1, 2, 3)))[:, None, None, None]
    return Ps, Us, Bs


def remapped_mesh(src, level, nx, lloc, nthreads=1):
    """An oracle Mesh on the layout (level, nx, lloc) holding src's state:
    remap, fill ghosts, invert (U -> P with floors), fill ghosts."""
    import oracle as _o
    P, U, B = remap(src, level, nx, lloc)
    m = _o.Mesh(src.root, level, nx, lloc, P, B, nthreads=nthreads, correct=src.correct)
    m.U = U
    for b, blk in enumerate(m.blocks):
        blk.con2prim(m.U[b], m.Bf[b], m.P[b], nthreads)
    m.fill_ghosts()
    m.t = src.t
    return m
