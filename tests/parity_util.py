"""Shared helpers of the GPU parity tests (HIP path through the C ABI versus
the oracle on identical inputs)."""
import sys

import numpy as np

import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def interior(prob, face_axis=None):
    g = prob.ng
    ext = [prob.n[d] + (1 if face_axis == d else 0) for d in range(3)]
    return (slice(g, g + ext[2]), slice(g, g + ext[1]), slice(g, g + ext[0]))


def rel_err(a, b, prob, face=False):
    """Per-variable max-norm error normalised by the oracle's max norm."""
    out = []
    for v in range(a.shape[0]):
        sl = interior(prob, v if face else None)
        x, y = a[v][sl], b[v][sl]
        den = np.abs(y).max()
        num = np.abs(x - y).max()
        out.append(num / den if den > 0 else num)
    return np.array(out)


def totals_drift(r1, r0, floor=1e-2):
    """Per-total relative change of the conserved totals between two
    reductions, each normalised by its own magnitude (at least floor times
    the largest total, so that a total near zero is judged on a scale of its
    own kind rather than the energy's)."""
    t0, t1 = np.asarray(r0["totals"]), np.asarray(r1["totals"])
    den = np.maximum(np.abs(t0), floor * np.abs(t0).max())
    return np.abs(t1 - t0) / den


def oracle_state(prob, nthreads=8):
    """Initial (P, Bf, U) from the oracle (ghosts filled)."""
    blk = oracle.Block(prob)
    P, Bf = prob.P.copy(), prob.Bf.copy()
    blk.fill_ghosts(P, Bf)
    U = blk.prim_to_cons(P, Bf)
    return blk, P, Bf, U


def upload_all(pack, P, Bf, U=None):
    """Load identical global arrays into the pack (U via its own per-block copy)."""
    import torch
    pack.upload(P, Bf)
    pack._out()
    if U is not None:
        for b in range(pack.nb):
            lo, n = pack.lloc[b], pack.nx[b]
            g = pack.ng
            sl = tuple(slice(lo[2 - d], lo[2 - d] + n[2 - d] + 2 * g) for d in range(3))
            pack._block_views(pack.U, b).copy_(torch.from_numpy(np.ascontiguousarray(U[(slice(None),) + sl])))
    torch.cuda.synchronize()
