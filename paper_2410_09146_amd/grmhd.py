"""Python binding of libgrmhd.so (include/grmhd.h): argument marshalling only.

Device memory comes from PyTorch (state tensors and the workspace); every step
of the method runs in the library's HIP kernels.  The binding fails loudly if
the library is missing or no GPU is present: there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrmhd.so")

OK = 0
METRIC_MINKOWSKI, METRIC_KS = 0, 1
GUESS_COLD, GUESS_PREV, GUESS_MLP = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1

_cint_p = ctypes.POINTER(ctypes.c_int)


class PackDesc(ctypes.Structure):
    _fields_ = [("nblocks", ctypes.c_int), ("ng", ctypes.c_int), ("recon", ctypes.c_int),
                ("riemann", ctypes.c_int), ("precision", ctypes.c_int), ("weno_fv", ctypes.c_int),
                ("nx", _cint_p), ("level", _cint_p), ("lloc", _cint_p),
                ("root_nx", ctypes.c_int * 3), ("xmin", ctypes.c_double * 3),
                ("xmax", ctypes.c_double * 3), ("bc", ctypes.c_int * 6), ("nscalar", ctypes.c_int)]


class StatePtrs(ctypes.Structure):
    _fields_ = [("P", ctypes.c_void_p), ("Bf", ctypes.c_void_p), ("U", ctypes.c_void_p),
                ("U0", ctypes.c_void_p), ("Bf0", ctypes.c_void_p)]


class Metric(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("M", ctypes.c_double), ("a", ctypes.c_double)]


class EosTable(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("n", ctypes.c_int * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3)]


class Eos(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("rho_flr0", ctypes.c_double),
                ("rho_flr_pow", ctypes.c_double), ("u_flr0", ctypes.c_double),
                ("u_flr_pow", ctypes.c_double), ("W_max", ctypes.c_double),
                ("c2p_tol", ctypes.c_double), ("c2p_max_iter", ctypes.c_int),
                ("table", ctypes.POINTER(EosTable))]


class ReductionOut(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("divb_rel", ctypes.c_double),
                ("divb_max", ctypes.c_double), ("totals", ctypes.c_double * 5),
                ("c2p_fail", ctypes.c_longlong), ("floor_hits", ctypes.c_longlong),
                ("c2p_iter_mean", ctypes.c_double), ("c2p_iter_wavemax_mean", ctypes.c_double),
                ("guess_fallback", ctypes.c_longlong), ("total_scalar", ctypes.c_double),
                ("c2p_fail_total", ctypes.c_longlong)]


EXPORTS = ["grmhd_abi_version", "grmhd_layout", "grmhd_pack_workspace_bytes",
           "grmhd_pack_create", "grmhd_pack_destroy", "grmhd_bind_state", "grmhd_fill_ghosts",
           "grmhd_stage", "grmhd_con2prim", "grmhd_prim_to_cons", "grmhd_reductions",
           "grmhd_debug_ptrs", "grmhd_profile", "grmhd_profile_read", "grmhd_mlp_bind",
           "grmhd_mlp_scratch_bytes", "grmhd_mlp_grad", "grmhd_mlp_train_step",
           "grmhd_mlp_train_step_noalloc",
           "grmhd_mlp_infer", "grmhd_step", "grmhd_step_graph", "grmhd_set_tiling",
           "grmhd_get_tiling", "grmhd_autotune", "grmhd_set_persistent", "grmhd_set_fused",
           "grmhd_set_concurrency",
           "grmhd_m1_source",
           "grmhd_tag", "grmhd_regrid_layout", "grmhd_remap_scratch_bytes", "grmhd_remap",
           "grmhd_last_error"]
NSHAPE = 5

PROF_FAMILIES = ["flux_x1", "flux_x2", "flux_x3", "flux_plane", "update", "con2prim",
                 "ghost", "bcc", "reduce", "mlp", "m1"]
MLP_NPARAM = 8834
MLP_NOALLOC_MAX_BATCH = 4096

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not built; run paper_2410_09146_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        L.grmhd_pack_workspace_bytes.restype = ctypes.c_size_t
        L.grmhd_last_error.restype = ctypes.c_char_p
        L.grmhd_last_error.argtypes = [ctypes.c_void_p]
        L.grmhd_pack_create.argtypes = [ctypes.POINTER(PackDesc), ctypes.POINTER(StatePtrs),
                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_void_p)]
        for f in ("grmhd_pack_destroy",):
            getattr(L, f).argtypes = [ctypes.c_void_p]
        L.grmhd_fill_ghosts.argtypes = [ctypes.c_void_p, ctypes.POINTER(Metric)]
        L.grmhd_stage.argtypes = [ctypes.c_void_p, ctypes.POINTER(Metric), ctypes.POINTER(Eos),
                                  ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
        L.grmhd_con2prim.argtypes = [ctypes.c_void_p, ctypes.POINTER(Metric), ctypes.POINTER(Eos),
                                     ctypes.c_int]
        L.grmhd_prim_to_cons.argtypes = [ctypes.c_void_p, ctypes.POINTER(Metric),
                                         ctypes.POINTER(Eos)]
        L.grmhd_reductions.argtypes = [ctypes.c_void_p, ctypes.POINTER(Metric),
                                       ctypes.POINTER(Eos), ctypes.c_double,
                                       ctypes.POINTER(ReductionOut)]
        L.grmhd_bind_state.argtypes = [ctypes.c_void_p, ctypes.POINTER(StatePtrs)]
        L.grmhd_debug_ptrs.argtypes = [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_void_p)] * 3
        L.grmhd_profile.argtypes = [ctypes.c_void_p, ctypes.c_int]
        vp = ctypes.c_void_p
        L.grmhd_step.argtypes = [vp, ctypes.POINTER(Metric), ctypes.POINTER(Eos), ctypes.c_double,
                                 ctypes.c_int, ctypes.c_double]
        L.grmhd_autotune.argtypes = [vp, ctypes.POINTER(Metric), ctypes.POINTER(Eos), ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
        L.grmhd_set_tiling.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
        L.grmhd_set_persistent.argtypes = [vp, ctypes.c_int]
        L.grmhd_set_fused.argtypes = [vp, ctypes.c_int]
        L.grmhd_set_concurrency.argtypes = [vp, ctypes.c_int]
        L.grmhd_get_tiling.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
        L.grmhd_step_graph.argtypes = [vp, ctypes.POINTER(Metric), ctypes.POINTER(Eos),
                                       ctypes.c_int, ctypes.c_double, ctypes.c_int]
        L.grmhd_mlp_bind.argtypes = [vp, vp, vp, vp]
        L.grmhd_mlp_scratch_bytes.argtypes = [ctypes.c_int]
        L.grmhd_mlp_scratch_bytes.restype = ctypes.c_size_t
        L.grmhd_mlp_grad.argtypes = [vp, vp, vp, ctypes.c_int, vp, vp, vp, ctypes.c_size_t, vp]
        L.grmhd_mlp_train_step.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int, ctypes.c_float,
                                           ctypes.c_int, vp, vp, ctypes.c_size_t, vp]
        L.grmhd_mlp_train_step_noalloc.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int,
                                                   ctypes.c_float, ctypes.c_int, vp, vp]
        L.grmhd_mlp_infer.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int, vp, ctypes.c_size_t, vp]
        L.grmhd_profile_read.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_longlong)]
        L.grmhd_m1_source.argtypes = [vp, ctypes.POINTER(Metric), ctypes.c_double, ctypes.c_int,
                                      vp, vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, vp]
        L.grmhd_tag.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        ip = ctypes.POINTER(ctypes.c_int)
        L.grmhd_regrid_layout.argtypes = [ctypes.POINTER(PackDesc), ip, ctypes.c_int, ip, ip, ip, ip]
        L.grmhd_remap_scratch_bytes.argtypes = [vp, vp]
        L.grmhd_remap_scratch_bytes.restype = ctypes.c_size_t
        L.grmhd_remap.argtypes = [vp, vp, ctypes.POINTER(Metric), ctypes.POINTER(Eos), vp,
                                  ctypes.c_size_t]
        _lib = L
    return _lib


class GrmhdError(RuntimeError):
    pass


def _check(rc, pack=None):
    if rc != OK:
        msg = lib().grmhd_last_error(pack).decode()
        raise GrmhdError(f"grmhd error {rc}: {msg}")


def regrid_layout(pack, tags):
    """Next (nx, lloc, level) from a pack's layout and per-block tags (+1
    refine, -1 derefine, 0 keep), by grmhd_regrid_layout."""
    tags = np.asarray(tags, dtype=np.int32)
    cap = 8 * pack.nb + 8
    ip = ctypes.c_int
    nb = ip()
    nx, ll, lv = (ip * (3 * cap))(), (ip * (3 * cap))(), (ip * cap)()
    t = (ip * pack.nb)(*tags.tolist())
    _check(lib().grmhd_regrid_layout(ctypes.byref(pack.desc), t, cap, ctypes.byref(nb), nx, ll, lv))
    n = nb.value
    return list(nx[:3 * n]), list(ll[:3 * n]), list(lv[:n])


def block_split(n, nblk):
    """Uniform split of a root grid n[3] into nblk[3] equal blocks."""
    nx, lloc = [], []
    for bk in range(nblk[2]):
        for bj in range(nblk[1]):
            for bi in range(nblk[0]):
                sz = [n[d] // nblk[d] for d in range(3)]
                nx += sz
                lloc += [bi * sz[0], bj * sz[1], bk * sz[2]]
    return nx, lloc


class Pack:
    """A pack of meshblocks covering a problem's domain.

    prob: a problem description (paper_2410_09146_amd.inputs.Problem); for a
          two-level layout it describes level 0.
    nblk: blocks per direction (uniform split), or
    layout: (nx, lloc) flat lists of one level, or (nx, lloc, level) with
            levels 0 / 1 and lloc in cells of the block's own level.
    """

    def __init__(self, prob, nblk=(1, 1, 1), device="cuda:0", precision=PREC_FP64,
                 c2p_tol=1e-14, c2p_max_iter=40, layout=None):
        import torch
        if not torch.cuda.is_available():
            raise GrmhdError("no GPU available: the HIP path has no CPU fallback")
        self.torch = torch
        self.prob = prob
        self.device = torch.device(device)
        self.ng = prob.ng
        level = None
        if layout is not None:
            nx, lloc = list(layout[0]), list(layout[1])
            if len(layout) > 2:
                level = [int(v) for v in layout[2]]
        else:
            for d in range(3):
                if prob.n[d] % nblk[d]:
                    raise GrmhdError("block split must divide the grid")
            nx, lloc = block_split(prob.n, nblk)
        self.nb = len(nx) // 3
        self._nx = (ctypes.c_int * len(nx))(*nx)
        self._lloc = (ctypes.c_int * len(lloc))(*lloc)
        if level is None:
            level = [0] * self.nb
        self.level = np.array(level, dtype=np.int32)
        self._level = (ctypes.c_int * self.nb)(*level)
        self.nx = np.array(nx).reshape(-1, 3)
        self.lloc = np.array(lloc).reshape(-1, 3)
        d = PackDesc()
        d.nblocks = self.nb
        d.ng = prob.ng
        d.recon, d.riemann, d.precision, d.weno_fv = prob.recon, prob.riemann, precision, prob.weno_fv
        d.nx, d.level, d.lloc = self._nx, self._level, self._lloc
        for k in range(3):
            d.root_nx[k] = prob.n[k]
            d.xmin[k] = prob.xmin[k]
            d.xmax[k] = prob.xmax[k]
        for s in range(6):
            d.bc[s] = prob.bc[s]
        self.nscalar = int(getattr(prob, "nscalar", 0))
        d.nscalar = self.nscalar
        self.npv = 5 + self.nscalar
        self.desc = d
        L = lib()
        offs = (ctypes.c_longlong * self.nb)()
        nct = ctypes.c_longlong()
        _check(L.grmhd_layout(ctypes.byref(d), offs, ctypes.byref(nct)))
        self.offsets = np.array(offs[:], dtype=np.int64)
        self.nct = nct.value
        wsb = L.grmhd_pack_workspace_bytes(ctypes.byref(d))
        if wsb == 0:
            _check(-1)
        f64 = dict(dtype=torch.float64, device=self.device)
        self.P = torch.zeros((self.npv, self.nct), **f64)
        self.Bf = torch.zeros((3, self.nct), **f64)
        self.U = torch.zeros((self.npv, self.nct), **f64)
        self.U0 = torch.zeros((self.npv, self.nct), **f64)
        self.Bf0 = torch.zeros((3, self.nct), **f64)
        self.ws = torch.zeros(wsb + 256, dtype=torch.uint8, device=self.device)
        ws_ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.ws_bytes = wsb
        st = StatePtrs(self.P.data_ptr(), self.Bf.data_ptr(), self.U.data_ptr(),
                       self.U0.data_ptr(), self.Bf0.data_ptr())
        # a stream of the pack's own (default priority): graph capture is not
        # permitted on the legacy default stream
        self.stream = torch.cuda.Stream(device=self.device)
        h = ctypes.c_void_p()
        _check(L.grmhd_pack_create(ctypes.byref(d), ctypes.byref(st), ctypes.c_void_p(ws_ptr),
                                   ctypes.c_size_t(wsb), ctypes.c_void_p(self.stream.cuda_stream),
                                   ctypes.byref(h)))
        self.h = h
        self.metric = Metric(prob.metric_kind, prob.M, prob.a)
        self.eos = Eos(prob.gamma, prob.rho_flr0, prob.rho_flr_pow, prob.u_flr0, prob.u_flr_pow,
                       prob.W_max, c2p_tol, c2p_max_iter, None)
        if getattr(prob, "table", None) is not None:
            self.set_table(prob.table)
        self.cfl = prob.cfl
        self.t = 0.0

    def set_table(self, tab):
        """Bind a tabulated EOS (inputs.EosTable): its nodes are copied to the
        device once; None restores the ideal gas."""
        if tab is None:
            self.eos.table = None
            self._tab = None
            return
        t = self.torch
        data = t.from_numpy(np.ascontiguousarray(tab.data, dtype=np.float64)).to(self.device)
        et = EosTable()
        et.data = data.data_ptr()
        n = tab.n
        for d in range(3):
            et.n[d] = int(n[d])
            et.lo[d] = float(tab.lo[d])
            et.hi[d] = float(tab.hi[d])
        self._tab = (data, et)
        self.eos.table = ctypes.pointer(et)

    def __del__(self):
        if getattr(self, "h", None):
            try:
                lib().grmhd_pack_destroy(self.h)
            except Exception:
                pass
            self.h = None

    # ---------------------------------------------------------- data movement
    def _block_views(self, arr, b):
        n = self.nx[b]
        s = n + 2 * self.ng
        o = self.offsets[b]
        cnt = int(s[0] * s[1] * s[2])
        return arr[:, o:o + cnt].reshape(arr.shape[0], s[2], s[1], s[0])

    def upload_blocks(self, Ps, Bfs):
        """Copy per-block padded numpy arrays (nvar, s3, s2, s1) into the pack."""
        torch = self.torch
        self._out()
        for b in range(self.nb):
            self._block_views(self.P, b).copy_(torch.from_numpy(np.ascontiguousarray(Ps[b])))
            self._block_views(self.Bf, b).copy_(torch.from_numpy(np.ascontiguousarray(Bfs[b])))

    def download_blocks(self, which="P"):
        """Per-block padded numpy arrays (ghosts included) of one state array."""
        arr = {"P": self.P, "Bf": self.Bf, "U": self.U, "U0": self.U0, "Bf0": self.Bf0}[which]
        self._out()
        self.torch.cuda.synchronize(self.device)
        host = arr.cpu().numpy()
        out = []
        for b in range(self.nb):
            s = self.nx[b] + 2 * self.ng
            o = self.offsets[b]
            out.append(host[:, o:o + s[0] * s[1] * s[2]].reshape(host.shape[0], s[2], s[1], s[0]).copy())
        return out

    def init_blocks(self, Ps, Bfs):
        """Upload per-block initial arrays, fill ghosts, build U."""
        self.upload_blocks(Ps, Bfs)
        self.fill_ghosts()
        self.prim_to_cons()

    def upload(self, P, Bf):
        """Copy global padded numpy arrays (nvar, s3, s2, s1) into the blocks."""
        if self.level.any():
            raise GrmhdError("a two-level pack takes per-block arrays (upload_blocks)")
        torch = self.torch
        self._out()
        for b in range(self.nb):
            lo = self.lloc[b]
            n = self.nx[b]
            sl = tuple(slice(lo[2 - d], lo[2 - d] + n[2 - d] + 2 * self.ng) for d in range(3))
            self._block_views(self.P, b).copy_(torch.from_numpy(np.ascontiguousarray(P[(slice(None),) + sl])))
            self._block_views(self.Bf, b).copy_(torch.from_numpy(np.ascontiguousarray(Bf[(slice(None),) + sl])))

    def download(self, which="P"):
        """Assemble a global padded numpy array from the blocks' interiors
        (and, for face arrays, the upper boundary faces)."""
        if self.level.any():
            raise GrmhdError("a two-level pack has no global array (download_blocks)")
        arr = {"P": self.P, "Bf": self.Bf, "U": self.U, "U0": self.U0, "Bf0": self.Bf0}[which]
        self._out()
        self.torch.cuda.synchronize(self.device)
        host = arr.cpu().numpy()
        nv = host.shape[0]
        g = self.ng
        shape = tuple(self.prob.n[2 - d] + 2 * g for d in range(3))
        out = np.zeros((nv,) + shape)
        face = which in ("Bf", "Bf0")
        for b in range(self.nb):
            n = self.nx[b]
            lo = self.lloc[b]
            s = n + 2 * g
            o = self.offsets[b]
            blk = host[:, o:o + s[0] * s[1] * s[2]].reshape(nv, s[2], s[1], s[0])
            for v in range(nv):
                ext = [n[d] + (1 if face and d == v else 0) for d in range(3)]
                src = blk[v, g:g + ext[2], g:g + ext[1], g:g + ext[0]]
                out[v, lo[2] + g:lo[2] + g + ext[2], lo[1] + g:lo[1] + g + ext[1],
                    lo[0] + g:lo[0] + g + ext[0]] = src
        return out

    def debug_arrays(self):
        """(flags, iters) of the last inversion as global padded numpy arrays."""
        f, it, fl = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        _check(lib().grmhd_debug_ptrs(self.h, ctypes.byref(f), ctypes.byref(it), ctypes.byref(fl)))
        base = self.ws.data_ptr()
        self._out()
        off_f = f.value - base
        off_i = it.value - base
        self.torch.cuda.synchronize(self.device)
        flags = self.ws[off_f:off_f + self.nct].cpu().numpy().view(np.int8)
        iters = self.ws[off_i:off_i + self.nct].cpu().numpy()
        out = []
        for arr in (flags, iters):
            g = self.ng
            shape = tuple(self.prob.n[2 - d] + 2 * g for d in range(3))
            glob = np.zeros(shape, dtype=arr.dtype)
            for b in range(self.nb):
                n, lo, o = self.nx[b], self.lloc[b], self.offsets[b]
                s = n + 2 * g
                blk = arr[o:o + s[0] * s[1] * s[2]].reshape(s[2], s[1], s[0])
                glob[lo[2] + g:lo[2] + g + n[2], lo[1] + g:lo[1] + g + n[1],
                     lo[0] + g:lo[0] + g + n[0]] = blk[g:g + n[2], g:g + n[1], g:g + n[0]]
            out.append(glob)
        return out

    def flux_array(self):
        """Face fluxes [3, 8, s3, s2, s1] of a single-block pack (debug)."""
        assert self.nb == 1
        fl = ctypes.c_void_p()
        _check(lib().grmhd_debug_ptrs(self.h, None, None, ctypes.byref(fl)))
        off = fl.value - self.ws.data_ptr()
        self._out()
        self.torch.cuda.synchronize(self.device)
        raw = self.ws[off:off + 24 * self.nct * 8].cpu().numpy().view(np.float64)
        s = self.nx[0] + 2 * self.ng
        cnt = s[0] * s[1] * s[2]
        return raw.reshape(3, 8, self.nct)[:, :, :cnt].reshape(3, 8, s[2], s[1], s[0])

    def _in(self):
        """Order the pack's stream after work queued on torch's current stream."""
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))

    def _out(self):
        """Order torch's current stream after the pack's work."""
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)

    # ------------------------------------------------------------------ calls
    def fill_ghosts(self):
        self._in()
        _check(lib().grmhd_fill_ghosts(self.h, ctypes.byref(self.metric)), self.h)

    def prim_to_cons(self):
        self._in()
        _check(lib().grmhd_prim_to_cons(self.h, ctypes.byref(self.metric), ctypes.byref(self.eos)),
               self.h)

    def stage(self, dt, rk):
        self._in()
        rkc = (ctypes.c_double * 3)(*rk)
        _check(lib().grmhd_stage(self.h, ctypes.byref(self.metric), ctypes.byref(self.eos),
                                 ctypes.c_double(dt), rkc), self.h)

    def con2prim(self, guess=GUESS_PREV):
        self._in()
        _check(lib().grmhd_con2prim(self.h, ctypes.byref(self.metric), ctypes.byref(self.eos),
                                    ctypes.c_int(guess)), self.h)

    def reductions(self, cfl=None, sync=True):
        self._in()
        out = ReductionOut()
        _check(lib().grmhd_reductions(self.h, ctypes.byref(self.metric), ctypes.byref(self.eos),
                                      ctypes.c_double(self.cfl if cfl is None else cfl),
                                      ctypes.byref(out) if sync else None), self.h)
        if not sync:
            return None
        return {"dt": out.dt, "divb_rel": out.divb_rel, "divb_max": out.divb_max,
                "totals": np.array(out.totals[:]), "c2p_fail": out.c2p_fail,
                "floor_hits": out.floor_hits, "c2p_iter_mean": out.c2p_iter_mean,
                "c2p_iter_wavemax_mean": out.c2p_iter_wavemax_mean,
                "guess_fallback": out.guess_fallback, "total_scalar": out.total_scalar,
                "c2p_fail_total": out.c2p_fail_total}

    def m1_source(self, R, kap, dt, couple=False, tol=1e-13, max_iter=40, iters=None):
        """Implicit gray-M1 collision update (grmhd_m1_source).  R: float64
        device tensor [nsp, 4, nct] (in place); kap: [nsp, 3, nct]; iters:
        optional uint8 device tensor [nct]."""
        for t in (R, kap):
            if t.dtype != self.torch.float64 or not t.is_contiguous() or t.device != self.device:
                raise GrmhdError("M1 arrays must be contiguous float64 on the pack's device")
        if R.shape[0] != kap.shape[0] or R.shape[1:] != (4, self.nct) or kap.shape[1:] != (3, self.nct):
            raise GrmhdError("M1 arrays must be [nsp, 4, nct] and [nsp, 3, nct]")
        if iters is not None and (iters.dtype != self.torch.uint8 or iters.numel() < self.nct):
            raise GrmhdError("iters must be a uint8 tensor of nct entries")
        self._m1_keep = (R, kap, iters)
        self._in()
        _check(lib().grmhd_m1_source(self.h, ctypes.byref(self.metric), ctypes.c_double(dt),
                                     int(R.shape[0]), R.data_ptr(), kap.data_ptr(), int(couple),
                                     ctypes.c_double(tol), int(max_iter),
                                     iters.data_ptr() if iters is not None else None), self.h)

    def to_pack_layout(self, arr):
        """Global padded numpy array [..., s3, s2, s1] of a single-level pack ->
        host array [..., nct] in the pack's block layout (interiors and
        ghosts of each block copied from the global array)."""
        lead = arr.shape[:-3]
        out = np.zeros(lead + (self.nct,))
        for b in range(self.nb):
            lo, n = self.lloc[b], self.nx[b]
            g = self.ng
            s = n + 2 * g
            sl = tuple(slice(lo[2 - d], lo[2 - d] + s[2 - d]) for d in range(3))
            blk = arr[(Ellipsis,) + sl]
            o = self.offsets[b]
            out[..., o:o + s[0] * s[1] * s[2]] = blk.reshape(lead + (-1,))
        return out

    def from_pack_layout(self, host, shape):
        """Inverse of to_pack_layout for the block interiors: [..., nct] ->
        global padded [..., s3, s2, s1] (ghosts of the global array zero)."""
        lead = host.shape[:-1]
        out = np.zeros(lead + tuple(shape))
        g = self.ng
        for b in range(self.nb):
            lo, n = self.lloc[b], self.nx[b]
            s = n + 2 * g
            o = self.offsets[b]
            blk = host[..., o:o + s[0] * s[1] * s[2]].reshape(lead + (s[2], s[1], s[0]))
            out[(Ellipsis,) + tuple(slice(lo[2 - d] + g, lo[2 - d] + g + n[2 - d]) for d in range(3))] = \
                blk[(Ellipsis, slice(g, g + n[2]), slice(g, g + n[1]), slice(g, g + n[0]))]
        return out

    def tag(self, var=0):
        """Per-block refinement indicator of P[var] (grmhd_tag)."""
        self._in()
        out = (ctypes.c_double * self.nb)()
        _check(lib().grmhd_tag(self.h, int(var), out), self.h)
        return np.array(out[:])

    def layout(self):
        """(nx, lloc, level) flat lists of this pack."""
        return (self.nx.ravel().tolist(), self.lloc.ravel().tolist(), self.level.tolist())

    def remap_from(self, src, guess=GUESS_PREV):
        """Take src's state onto this pack's layout (grmhd_remap), then fill
        ghosts, invert and fill ghosts again."""
        torch = self.torch
        src._out()
        self._out()
        torch.cuda.synchronize(self.device)
        L = lib()
        nbytes = L.grmhd_remap_scratch_bytes(self.h, src.h)
        if nbytes == 0:
            _check(-2, None)
        scratch = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (scratch.data_ptr() + 255) // 256 * 256
        _check(L.grmhd_remap(self.h, src.h, ctypes.byref(self.metric), ctypes.byref(self.eos),
                             ctypes.c_void_p(ptr), ctypes.c_size_t(nbytes)), self.h)
        del scratch
        self.fill_ghosts()
        self.con2prim(guess)
        self.fill_ghosts()

    def mlp_bind(self, params, mean, std):
        """params: float32 device tensor [MLP_NPARAM]; mean/std: float32 device [5]."""
        self._mlp_keep = (params, mean, std)
        self._in()
        _check(lib().grmhd_mlp_bind(self.h, params.data_ptr(), mean.data_ptr(), std.data_ptr()),
               self.h)

    def profile(self, enable=True):
        _check(lib().grmhd_profile(self.h, int(enable)), self.h)

    def profile_read(self):
        n = len(PROF_FAMILIES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_longlong * n)()
        _check(lib().grmhd_profile_read(self.h, ms, cnt), self.h)
        return {f: (ms[i], cnt[i]) for i, f in enumerate(PROF_FAMILIES)}

    def init(self, P=None, Bf=None):
        """Upload the problem's initial state, fill ghosts, build U."""
        self.upload(self.prob.P if P is None else P, self.prob.Bf if Bf is None else Bf)
        self.fill_ghosts()
        self.prim_to_cons()

    def autotune(self, reps=3):
        """Time every face-tile shape per direction; keep and return the fastest."""
        self._in()
        ch = (ctypes.c_int * 3)()
        tab = (ctypes.c_double * (3 * NSHAPE))()
        _check(lib().grmhd_autotune(self.h, ctypes.byref(self.metric), ctypes.byref(self.eos),
                                    reps, ch, tab), self.h)
        return list(ch), np.array(tab[:]).reshape(3, NSHAPE)

    def set_persistent(self, workgroups):
        _check(lib().grmhd_set_persistent(self.h, int(workgroups)), self.h)

    def set_fused(self, enable):
        """Fused stage on or off (the default; grmhd_set_fused)."""
        _check(lib().grmhd_set_fused(self.h, int(enable)), self.h)

    def set_concurrency(self, enable):
        """Flux directions on streams of their own (default) or all on the
        pack's stream (grmhd_set_concurrency)."""
        _check(lib().grmhd_set_concurrency(self.h, int(enable)), self.h)

    def set_tiling(self, shape):
        _check(lib().grmhd_set_tiling(self.h, (ctypes.c_int * 3)(*shape)), self.h)

    def step_c(self, dt=None, guess=GUESS_PREV, cfl=None):
        """One SSPRK2 step through grmhd_step (+ reductions when cfl given)."""
        self._in()
        _check(lib().grmhd_step(self.h, ctypes.byref(self.metric), ctypes.byref(self.eos),
                                ctypes.c_double(-1.0 if dt is None else dt), guess,
                                ctypes.c_double(0.0 if cfl is None else cfl)), self.h)

    def step_graph(self, nsteps, guess=GUESS_PREV, cfl=None):
        """nsteps replays of the HIP-graph-captured step (dt on the device)."""
        self._in()
        _check(lib().grmhd_step_graph(self.h, ctypes.byref(self.metric), ctypes.byref(self.eos),
                                      guess, ctypes.c_double(self.cfl if cfl is None else cfl),
                                      nsteps), self.h)

    def step(self, dt=None, guess=GUESS_PREV):
        """One SSPRK2 step (Shu-Osher) through the public calls: stage {1,0,1},
        con2prim, ghosts, stage {1/2,1/2,1/2}, con2prim, ghosts (the first
        stage saves the base into U0 / Bf0).  dt = None: device-resident dt
        from reductions(sync=False) (no host round trip)."""
        h = dt if dt is not None else -1.0
        self.stage(h, (1.0, 0.0, 1.0))
        self.con2prim(guess)
        self.fill_ghosts()
        self.stage(h, (0.5, 0.5, 0.5))
        self.con2prim(guess)
        self.fill_ghosts()
