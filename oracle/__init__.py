"""FP64 CPU oracle for the GRMHD stage (Phoebus paper, Sec. 2.1, Sec. 3.1, App. B).

TEST INFRASTRUCTURE ONLY.  The plain C implementation under this directory is
what the HIP library is checked against; it shares no code with it.  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may load
it.  Nothing in the product path imports this package.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = ["metric.c", "physics.c", "eos.c", "recon.c", "c2p.c", "stage.c", "api.c", "mesh.c",
           "m1.c"]
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-std=c11", "-Wall"]


def build(force=True, src_dir=_HERE, out=LIB_PATH):
    """Compile liboracle.so with gcc (no fast-math, no FMA contraction).
    src_dir / out: another copy of the sources and its library (the pin tests
    build deliberately broken copies to show that each pin catches them)."""
    if not force and os.path.exists(out):
        return out
    cmd = ["gcc"] + CFLAGS + ["-I", _HERE, "-o", out + ".tmp"] + \
        [os.path.join(src_dir, s) for s in SOURCES] + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("ng", ctypes.c_int),
                ("xmin", ctypes.c_double * 3), ("dx", ctypes.c_double * 3),
                ("bc", ctypes.c_int * 6), ("recon", ctypes.c_int),
                ("riemann", ctypes.c_int), ("weno_fv", ctypes.c_int)]


class Metric(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("M", ctypes.c_double), ("a", ctypes.c_double)]


class Table(ctypes.Structure):
    _fields_ = [("data", ctypes.POINTER(ctypes.c_double)), ("n", ctypes.c_int * 3),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3)]


class Eos(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("rho_flr0", ctypes.c_double),
                ("rho_flr_pow", ctypes.c_double), ("u_flr0", ctypes.c_double),
                ("u_flr_pow", ctypes.c_double), ("W_max", ctypes.c_double),
                ("nscalar", ctypes.c_int), ("tab", ctypes.POINTER(Table))]


def table_struct(tab):
    """ctypes view of an inputs.EosTable (keeps a reference to its data)."""
    data = np.ascontiguousarray(tab.data, dtype=np.float64)
    t = Table()
    t.data = data.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    for d in range(3):
        t.n[d] = data.shape[2 - d]
        t.lo[d] = tab.lo[d]
        t.hi[d] = tab.hi[d]
    t._keep = data
    return t


def eos_struct(prob):
    """orc_eos of a problem: ideal gas, or its table (with the Y_e scalar)."""
    e = Eos(prob.gamma, prob.rho_flr0, prob.rho_flr_pow, prob.u_flr0, prob.u_flr_pow,
            prob.W_max, int(getattr(prob, "nscalar", 0)), None)
    tab = getattr(prob, "table", None)
    if tab is not None:
        t = table_struct(tab)
        e.tab = ctypes.pointer(t)
        e._keep = t
    return e


_lib = None


def load(path):
    """A ctypes handle of an oracle library with the return types set."""
    L = ctypes.CDLL(path)
    L.orc_pt_master.restype = ctypes.c_double
    L.orc_pt_master_tab.restype = ctypes.c_double
    L.orc_m1_chi.restype = ctypes.c_double
    L.orc_m1_chi.argtypes = [ctypes.c_double]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = load(LIB_PATH)
    return _lib


_P = ctypes.POINTER(ctypes.c_double)


def _ptr(a):
    if a.dtype == np.float64 and a.ndim == 1 and not a.flags["C_CONTIGUOUS"] and a.size <= 16:
        a = np.ascontiguousarray(a)       # small point vectors (views) are copied
    if not (a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]):
        raise TypeError("oracle arrays must be C-contiguous float64")
    return a.ctypes.data_as(_P)


def metric_struct(kind, M=1.0, a=0.0):
    return Metric(kind, M, a)


# ----------------------------------------------------------------- point API

def geom(metric, x):
    out = np.zeros(56)
    lib().orc_pt_geom(ctypes.byref(metric), _ptr(np.asarray(x, float)), _ptr(out))
    return {"g": out[0:16].reshape(4, 4), "gi": out[16:32].reshape(4, 4),
            "alpha": out[32], "beta": out[33:36], "gam": out[36:45].reshape(3, 3),
            "gami": out[45:54].reshape(3, 3), "sqrtgam": out[54], "sqrtmg": out[55]}


def derivs(metric, x):
    dg = np.zeros((4, 4, 4)); Gam = np.zeros((4, 4, 4)); dla = np.zeros(4)
    lib().orc_pt_derivs(ctypes.byref(metric), _ptr(np.asarray(x, float)), _ptr(dg),
                        _ptr(Gam), _ptr(dla))
    return dg, Gam, dla


def p2c(metric, x, gam, prim):
    U = np.zeros(8)
    lib().orc_pt_p2c(ctypes.byref(metric), _ptr(np.asarray(x, float)), ctypes.c_double(gam),
                     _ptr(np.asarray(prim, float)), _ptr(U))
    return U


def flux(metric, x, gam, prim, d):
    F = np.zeros(8)
    lib().orc_pt_flux(ctypes.byref(metric), _ptr(np.asarray(x, float)), ctypes.c_double(gam),
                      _ptr(np.asarray(prim, float)), ctypes.c_int(d), _ptr(F))
    return F


def speeds(metric, x, gam, prim, d):
    out = np.zeros(2)
    lib().orc_pt_speeds(ctypes.byref(metric), _ptr(np.asarray(x, float)),
                        ctypes.c_double(gam), _ptr(np.asarray(prim, float)), ctypes.c_int(d),
                        _ptr(out))
    return out[0], out[1]


def riemann(metric, x, gam, solver, pl, pr, d):
    F = np.zeros(8)
    lib().orc_pt_riemann(ctypes.byref(metric), _ptr(np.asarray(x, float)),
                         ctypes.c_double(gam), ctypes.c_int(solver),
                         _ptr(np.asarray(pl, float)), _ptr(np.asarray(pr, float)),
                         ctypes.c_int(d), _ptr(F))
    return F


def tmunu(metric, x, gam, prim):
    T = np.zeros(16)
    lib().orc_pt_tmunu(ctypes.byref(metric), _ptr(np.asarray(x, float)), ctypes.c_double(gam),
                       _ptr(np.asarray(prim, float)), _ptr(T))
    return T.reshape(4, 4)


def c2p(metric, x, gam, Ud, B):
    out = np.zeros(8)
    mu = ctypes.c_double(0.0)
    r = lib().orc_pt_c2p(ctypes.byref(metric), _ptr(np.asarray(x, float)), ctypes.c_double(gam),
                         _ptr(np.asarray(Ud, float)), _ptr(np.asarray(B, float)), _ptr(out),
                         ctypes.byref(mu))
    return r, out, mu.value


def p2c_batch(metric, x, gam, prims):
    """prims [n, 8] -> undensitized U [n, 8] at one point x."""
    prims = np.ascontiguousarray(prims, dtype=float)
    U = np.zeros_like(prims)
    lib().orc_p2c_batch(ctypes.byref(metric), _ptr(np.asarray(x, float)), ctypes.c_double(gam),
                        ctypes.c_long(prims.shape[0]), _ptr(prims), _ptr(U))
    return U


def master(gam, q, r2, b2, rb, mu):
    return lib().orc_pt_master(ctypes.c_double(gam), ctypes.c_double(q), ctypes.c_double(r2),
                               ctypes.c_double(b2), ctypes.c_double(rb), ctypes.c_double(mu))


def recon(method, f, fv=0):
    out = np.zeros(2)
    lib().orc_pt_recon(ctypes.c_int(method), ctypes.c_int(fv), _ptr(np.ascontiguousarray(f, dtype=float)),
                       _ptr(out))
    return out[0], out[1]


def weno(f, fv=0):
    w = np.zeros(3)
    s = ctypes.c_double(0.0)
    lib().orc_pt_weno(ctypes.c_int(fv), _ptr(np.ascontiguousarray(f, dtype=float)), _ptr(w), ctypes.byref(s))
    return w, s.value


# --------------------------------------------------- general EOS point API
# eos: an Eos structure (eos_struct); primitive vectors of 9 end with Y_e,
# conserved and flux vectors of 9 end with D Y_e and its flux.

def table_eval(tab_struct, rho, eps, ye):
    rho, eps, ye = (np.ascontiguousarray(np.broadcast_to(a, np.broadcast(rho, eps, ye).shape),
                                         dtype=float).ravel() for a in (rho, eps, ye))
    lnp, g1 = np.zeros_like(rho), np.zeros_like(rho)
    lib().orc_pt_table(ctypes.byref(tab_struct), ctypes.c_long(rho.size), _ptr(rho), _ptr(eps),
                       _ptr(ye), _ptr(lnp), _ptr(g1))
    return lnp, g1


def thermo(eos, rho, u, ye):
    rho, u, ye = (np.ascontiguousarray(np.broadcast_to(a, np.broadcast(rho, u, ye).shape),
                                       dtype=float).ravel() for a in (rho, u, ye))
    p, gp = np.zeros_like(rho), np.zeros_like(rho)
    lib().orc_pt_thermo(ctypes.byref(eos), ctypes.c_long(rho.size), _ptr(rho), _ptr(u), _ptr(ye),
                        _ptr(p), _ptr(gp))
    return p, gp


def p2c_eos(metric, x, eos, prim9):
    U = np.zeros(9)
    lib().orc_pt_p2c_eos(ctypes.byref(metric), _ptr(np.asarray(x, float)), ctypes.byref(eos),
                         _ptr(np.ascontiguousarray(prim9, dtype=float)), _ptr(U))
    return U


def riemann_eos(metric, x, eos, solver, pl, pr, d):
    F = np.zeros(9)
    lib().orc_pt_riemann_eos(ctypes.byref(metric), _ptr(np.asarray(x, float)), ctypes.byref(eos),
                             ctypes.c_int(solver), _ptr(np.ascontiguousarray(pl, dtype=float)),
                             _ptr(np.ascontiguousarray(pr, dtype=float)), ctypes.c_int(d), _ptr(F))
    return F


def speeds_eos(metric, x, eos, prim9, d):
    out = np.zeros(2)
    lib().orc_pt_speeds_eos(ctypes.byref(metric), _ptr(np.asarray(x, float)), ctypes.byref(eos),
                            _ptr(np.ascontiguousarray(prim9, dtype=float)), ctypes.c_int(d),
                            _ptr(out))
    return out[0], out[1]


def c2p_eos(metric, x, eos, Ud6, B):
    out = np.zeros(9)
    mu = ctypes.c_double(0.0)
    r = lib().orc_pt_c2p_eos(ctypes.byref(metric), _ptr(np.asarray(x, float)), ctypes.byref(eos),
                             _ptr(np.ascontiguousarray(Ud6, dtype=float)),
                             _ptr(np.asarray(B, float)), _ptr(out), ctypes.byref(mu))
    return r, out, mu.value


def master_tab(tab_struct, D, ye, q, r2, b2, rb, mu):
    return lib().orc_pt_master_tab(ctypes.byref(tab_struct), *(ctypes.c_double(v) for v in
                                                                (D, ye, q, r2, b2, rb, mu)))


# ------------------------------------------------------------ gray M1 moments
# X = (E, F_1, F_2, F_3) undensitized Eulerian moments of one species, ut the
# fluid's u-tilde^i, op = (kappa_J, kappa_H, J_eq).

def _geom_struct(metric, x):
    class _G(ctypes.Structure):
        _fields_ = [("g", ctypes.c_double * 16), ("gi", ctypes.c_double * 16),
                    ("alpha", ctypes.c_double), ("beta", ctypes.c_double * 3),
                    ("gam", ctypes.c_double * 9), ("gami", ctypes.c_double * 9),
                    ("sqrtgam", ctypes.c_double), ("sqrtmg", ctypes.c_double)]
    G = _G()
    lib().orc_geom_at(ctypes.byref(metric), _ptr(np.asarray(x, float)), ctypes.byref(G))
    return G


def m1_chi(f):
    return lib().orc_m1_chi(float(f))


def m1_closure(metric, x, ut, E, F):
    G = _geom_struct(metric, x)
    P = np.zeros((3, 3))
    lib().orc_m1_closure(ctypes.byref(G), _ptr(np.asarray(ut, float)), ctypes.c_double(E),
                         _ptr(np.asarray(F, float)), _ptr(P))
    return P


def m1_sources(metric, x, ut, X, op):
    G = _geom_struct(metric, x)
    S = np.zeros(4)
    J = ctypes.c_double(0.0)
    lib().orc_m1_sources(ctypes.byref(G), _ptr(np.asarray(ut, float)),
                         _ptr(np.asarray(X, float)), _ptr(np.asarray(op, float)),
                         ctypes.byref(J), _ptr(S))
    return J.value, S


def m1_implicit(metric, x, ut, Xs, op, dt):
    G = _geom_struct(metric, x)
    X = np.zeros(4)
    it = lib().orc_m1_implicit(ctypes.byref(G), _ptr(np.asarray(ut, float)),
                               _ptr(np.asarray(Xs, float)), _ptr(np.asarray(op, float)),
                               ctypes.c_double(dt), _ptr(X))
    return it, X


# ----------------------------------------------------------------- block API

class Block:
    """One meshblock of a problem description, evaluated by the oracle."""

    def __init__(self, prob):
        self.prob = prob
        g = Grid()
        for d in range(3):
            g.n[d] = prob.n[d]
            g.xmin[d] = prob.xmin[d]
            g.dx[d] = prob.dx[d]
        g.ng = prob.ng
        for s in range(6):
            g.bc[s] = prob.bc[s]
        g.recon = prob.recon
        g.riemann = prob.riemann
        g.weno_fv = prob.weno_fv
        self.grid = g
        self.metric = Metric(prob.metric_kind, prob.M, prob.a)
        self.eos = eos_struct(prob)
        self.nv = 5 + int(getattr(prob, "nscalar", 0))
        self.shape = prob.shape

    def coord(self, loc, i, j, k):
        x = np.zeros(3)
        lib().orc_pt_coord(ctypes.byref(self.grid), ctypes.byref(self.metric), loc, i, j, k,
                           _ptr(x))
        return x

    def fill_ghosts(self, P, Bf):
        lib().orc_fill_ghosts_n(ctypes.byref(self.grid), ctypes.byref(self.metric),
                                ctypes.c_int(self.nv), _ptr(P), _ptr(Bf))

    def cell_B(self, Bf):
        Bcc = np.zeros((3,) + self.shape)
        lib().orc_cell_B(ctypes.byref(self.grid), ctypes.byref(self.metric), _ptr(Bf),
                         _ptr(Bcc))
        return Bcc

    def prim_to_cons(self, P, Bf, U=None):
        if U is None:
            U = np.zeros((self.nv,) + self.shape)
        lib().orc_prim_to_cons_grid(ctypes.byref(self.grid), ctypes.byref(self.metric),
                                    ctypes.byref(self.eos), _ptr(P), _ptr(Bf), _ptr(U))
        return U

    def stage(self, P, Bf, U0, Bf0, U, dt, rk, nthreads=1, want_flux=False):
        Uout = np.zeros_like(U)
        Bfout = np.zeros_like(Bf)
        F = np.zeros((3, 8) + self.shape) if want_flux else None
        rkc = (ctypes.c_double * 3)(*rk)
        r = lib().orc_stage(ctypes.byref(self.grid), ctypes.byref(self.metric),
                            ctypes.byref(self.eos), _ptr(P), _ptr(Bf), _ptr(U0), _ptr(Bf0),
                            _ptr(U), ctypes.c_double(dt), rkc, _ptr(Uout), _ptr(Bfout),
                            _ptr(F) if want_flux else None, ctypes.c_int(nthreads))
        if r != 0:
            raise RuntimeError("orc_stage failed")
        return (Uout, Bfout, F) if want_flux else (Uout, Bfout)

    def con2prim(self, U, Bf, P, nthreads=1):
        flag = np.zeros(self.shape, dtype=np.int8)
        nfail = lib().orc_con2prim(ctypes.byref(self.grid), ctypes.byref(self.metric),
                                   ctypes.byref(self.eos), _ptr(U), _ptr(Bf), _ptr(P),
                                   flag.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                                   ctypes.c_int(nthreads))
        return flag, nfail

    def m1_update(self, P, R, kap, dt, nthreads=1):
        """Implicit gray-M1 collision update of R [nsp, 4, s3, s2, s1] (in place)."""
        nsp = R.shape[0]
        it = np.zeros(self.shape, dtype=np.int32)
        bad = lib().orc_m1_update_grid(ctypes.byref(self.grid), ctypes.byref(self.metric),
                                       ctypes.c_int(nsp), _ptr(P), _ptr(R), _ptr(kap),
                                       ctypes.c_double(dt),
                                       it.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                       ctypes.c_int(nthreads))
        return it, bad

    def reductions(self, P, Bf, U, cfl):
        out = np.zeros(9)
        lib().orc_reductions(ctypes.byref(self.grid), ctypes.byref(self.metric),
                             ctypes.byref(self.eos), _ptr(P), _ptr(Bf), _ptr(U),
                             ctypes.c_double(cfl), _ptr(out))
        return {"dt": out[0], "divb_rel": out[1], "divb_max": out[2], "totals": out[3:8].copy(),
                "total_scalar": out[8]}


class Sim:
    """SSPRK2 driver over the oracle's stage (Shu-Osher form)."""

    def __init__(self, prob, nthreads=1):
        self.blk = Block(prob)
        self.nthreads = nthreads
        self.P = prob.P.copy()
        self.Bf = prob.Bf.copy()
        self.blk.fill_ghosts(self.P, self.Bf)
        self.U = self.blk.prim_to_cons(self.P, self.Bf)
        self.cfl = prob.cfl
        self.t = 0.0

    def dt(self):
        return self.blk.reductions(self.P, self.Bf, self.U, self.cfl)["dt"]

    def stage(self, dt, rk, U0, Bf0):
        U, Bf = self.blk.stage(self.P, self.Bf, U0, Bf0, self.U, dt, rk, self.nthreads)
        self.U, self.Bf = U, Bf
        flag, nfail = self.blk.con2prim(self.U, self.Bf, self.P, self.nthreads)
        self.blk.fill_ghosts(self.P, self.Bf)
        self.flag = flag
        return flag, nfail

    def step(self, dt=None):
        if dt is None:
            dt = self.dt()
        U0, Bf0 = self.U.copy(), self.Bf.copy()
        self.stage(dt, (1.0, 0.0, 1.0), U0, Bf0)
        self.stage(dt, (0.5, 0.5, 0.5), U0, Bf0)
        self.t += dt
        return dt


class _MeshDesc(ctypes.Structure):
    _fields_ = [("nb", ctypes.c_int), ("ng", ctypes.c_int), ("root_nx", ctypes.c_int * 3),
                ("bc", ctypes.c_int * 6), ("level", ctypes.POINTER(ctypes.c_int)),
                ("nx", ctypes.POINTER(ctypes.c_int)), ("lloc", ctypes.POINTER(ctypes.c_int))]


BC_FIXED = 3


class Mesh:
    """A two-level block mesh evaluated block by block with the oracle's stage,
    its ghost zones filled by orc_mesh_fill_ghosts (prolongation, restriction
    and same-level copies; see mesh.c for the reading).

    root: the level-0 problem description (domain, boundaries, physics);
    level[nb], nx[nb,3], lloc[nb,3] (level units); P_blocks / Bf_blocks:
    per-block padded arrays (nvar, s3, s2, s1) with the interiors set.
    One global dt, no flux or EMF correction at level boundaries."""

    def __init__(self, root, level, nx, lloc, P_blocks, Bf_blocks, nthreads=1, correct=True):
        if getattr(root, "nscalar", 0):
            raise NotImplementedError("two-level meshes carry no passive scalar")
        self.root = root
        self.level = np.asarray(level, dtype=np.int32)
        self.nx = np.asarray(nx, dtype=np.int32).reshape(-1, 3)
        self.lloc = np.asarray(lloc, dtype=np.int32).reshape(-1, 3)
        self.nb = len(self.level)
        self.nthreads = nthreads
        self.correct = correct
        self.cfl = root.cfl
        self.blocks = []
        for b in range(self.nb):
            blk = Block(root)
            l = int(self.level[b])
            g = blk.grid
            for d in range(3):
                dxl = root.dx[d] / (1 << l)
                g.n[d] = int(self.nx[b, d])
                g.dx[d] = dxl
                g.xmin[d] = root.xmin[d] + int(self.lloc[b, d]) * dxl
                nl = root.n[d] << l
                g.bc[2 * d] = root.bc[2 * d] if self.lloc[b, d] == 0 else BC_FIXED
                g.bc[2 * d + 1] = root.bc[2 * d + 1] if self.lloc[b, d] + self.nx[b, d] == nl \
                    else BC_FIXED
            blk.shape = tuple(int(self.nx[b, 2 - d]) + 2 * root.ng for d in range(3))
            self.blocks.append(blk)
        self.P = [np.ascontiguousarray(p, dtype=np.float64).copy() for p in P_blocks]
        self.Bf = [np.ascontiguousarray(p, dtype=np.float64).copy() for p in Bf_blocks]
        self.fill_ghosts()
        self.U = [blk.prim_to_cons(P, Bf) for blk, P, Bf in zip(self.blocks, self.P, self.Bf)]
        self.t = 0.0

    def _desc(self):
        d = _MeshDesc()
        d.nb, d.ng = self.nb, self.root.ng
        for k in range(3):
            d.root_nx[k] = self.root.n[k]
        for s in range(6):
            d.bc[s] = self.root.bc[s]
        self._keep = (np.ascontiguousarray(self.level, dtype=np.int32),
                      np.ascontiguousarray(self.nx.ravel(), dtype=np.int32),
                      np.ascontiguousarray(self.lloc.ravel(), dtype=np.int32))
        ip = ctypes.POINTER(ctypes.c_int)
        d.level, d.nx, d.lloc = (a.ctypes.data_as(ip) for a in self._keep)
        return d

    def fill_ghosts(self, P=None, Bf=None):
        P = self.P if P is None else P
        Bf = self.Bf if Bf is None else Bf
        d = _MeshDesc()
        d.nb, d.ng = self.nb, self.root.ng
        for k in range(3):
            d.root_nx[k] = self.root.n[k]
        for s in range(6):
            d.bc[s] = self.root.bc[s]
        lev = np.ascontiguousarray(self.level, dtype=np.int32)
        nx = np.ascontiguousarray(self.nx.ravel(), dtype=np.int32)
        ll = np.ascontiguousarray(self.lloc.ravel(), dtype=np.int32)
        ip = ctypes.POINTER(ctypes.c_int)
        d.level, d.nx, d.lloc = lev.ctypes.data_as(ip), nx.ctypes.data_as(ip), ll.ctypes.data_as(ip)
        pp = (_P * self.nb)(*[_ptr(a) for a in P])
        bp = (_P * self.nb)(*[_ptr(a) for a in Bf])
        if lib().orc_mesh_fill_ghosts(ctypes.byref(d), pp, bp) != 0:
            raise RuntimeError("blocks do not tile the domain")

    def reductions(self):
        outs = [blk.reductions(P, Bf, U, self.cfl)
                for blk, P, Bf, U in zip(self.blocks, self.P, self.Bf, self.U)]
        g = self.root.ng
        bmax = 0.0
        for b in range(self.nb):
            n = self.nx[b]
            for c in range(3):
                ext = [n[d] + (1 if d == c else 0) for d in range(3)]
                a = self.Bf[b][c, g:g + ext[2], g:g + ext[1], g:g + ext[0]]
                bmax = max(bmax, float(np.abs(a).max()))
        lmax = int(self.level.max())
        dxmin = min(self.root.dx[d] / (1 << lmax) for d in range(3) if self.root.n[d] > 1)
        dmax = max(o["divb_max"] for o in outs)
        tot = np.zeros(5)
        for o in outs:
            tot += o["totals"]
        return {"dt": min(o["dt"] for o in outs), "divb_max": dmax,
                "divb_rel": dmax / (bmax / dxmin) if bmax > 0 else dmax, "totals": tot}

    def dt(self):
        return self.reductions()["dt"]

    def stage(self, dt, rk, U0, Bf0):
        """Fluxes and EMFs of every block, their correction at level
        boundaries (orc_mesh_correct), then each block's update."""
        L = lib()
        F = [np.zeros((3, 8) + blk.shape) for blk in self.blocks]
        E = [np.zeros((3,) + blk.shape) for blk in self.blocks]
        for b, blk in enumerate(self.blocks):
            if L.orc_fluxes_emfs(ctypes.byref(blk.grid), ctypes.byref(blk.metric),
                                 ctypes.byref(blk.eos), _ptr(self.P[b]), _ptr(self.Bf[b]),
                                 _ptr(F[b]), _ptr(E[b]), ctypes.c_int(self.nthreads)) != 0:
                raise RuntimeError("orc_fluxes_emfs failed")
        if self.correct:
            d = self._desc()
            fp = (_P * self.nb)(*[_ptr(a) for a in F])
            ep = (_P * self.nb)(*[_ptr(a) for a in E])
            self.corrected = L.orc_mesh_correct(ctypes.byref(d), fp, ep)
        rkc = (ctypes.c_double * 3)(*rk)
        for b, blk in enumerate(self.blocks):
            Uo, Bo = np.zeros_like(self.U[b]), np.zeros_like(self.Bf[b])
            if L.orc_stage_from(ctypes.byref(blk.grid), ctypes.byref(blk.metric),
                                ctypes.byref(blk.eos), _ptr(self.P[b]), _ptr(self.Bf[b]),
                                _ptr(U0[b]), _ptr(Bf0[b]), _ptr(self.U[b]), ctypes.c_double(dt),
                                rkc, _ptr(F[b]), _ptr(E[b]), _ptr(Uo), _ptr(Bo),
                                ctypes.c_int(self.nthreads)) != 0:
                raise RuntimeError("orc_stage_from failed")
            self.U[b], self.Bf[b] = Uo, Bo
        nfail = 0
        for b, blk in enumerate(self.blocks):
            nfail += blk.con2prim(self.U[b], self.Bf[b], self.P[b], self.nthreads)[1]
        self.fill_ghosts()
        return nfail

    def step(self, dt=None):
        if dt is None:
            dt = self.dt()
        U0 = [u.copy() for u in self.U]
        Bf0 = [b.copy() for b in self.Bf]
        self.stage(dt, (1.0, 0.0, 1.0), U0, Bf0)
        self.stage(dt, (0.5, 0.5, 0.5), U0, Bf0)
        self.t += dt
        return dt


def weno_beta(f):
    b = np.zeros(3)
    lib().orc_pt_beta(_ptr(np.ascontiguousarray(f, dtype=float)), _ptr(b))
    return b
