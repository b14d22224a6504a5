"""Batching: uneven meshblocks (octree mix of block sizes) in one launch per
kernel family, persistent flux grid, autotuned tile shapes, graph replay.
Same-level decompositions change nothing but the data layout, so every run is
compared with the single-block run of the same grid."""
import numpy as np
import pytest

from paper_2410_09146_amd import inputs as I
from parity_util import rel_err, say

pytestmark = pytest.mark.gpu


def _run(G, prob, layout, nsteps, graph=False, persist=0, tune=False):
    pack = G.Pack(prob, layout=layout)
    pack.init()
    pack.reductions(sync=False)
    if tune:
        pack.autotune(reps=1)
    if persist:
        pack.set_persistent(persist)
    if graph:
        pack.step_graph(nsteps)
    else:
        for _ in range(nsteps):
            pack.step_c(None, cfl=prob.cfl)
    out = (pack.download("P"), pack.download("Bf"), pack.reductions())
    return pack, out


def test_uneven_blocks_match_single_block():
    from paper_2410_09146_amd import grmhd as G
    prob = I.torus(n=(64, 64, 32))
    nx, lloc = I.octree_layout(prob.n, base=32, smallest=8, p_split=(0.5, 0.5), seed=3)
    nb = len(nx) // 3
    sizes = sorted(set(nx[0::3]))
    _, (P1, B1, r1) = _run(G, prob, None, 3)
    _, (Pn, Bn, rn) = _run(G, prob, (nx, lloc), 3, graph=True, persist=1024, tune=True)
    eP, eB = rel_err(Pn, P1, prob), rel_err(Bn, B1, prob, face=True)
    say("uneven", nb, "blocks of", sizes, "eP", eP.max(), "eB", eB.max(), "dt", r1["dt"], rn["dt"])
    assert nb > 20 and len(sizes) >= 2
    assert np.all(eP <= 1e-13) and np.all(eB <= 1e-13)
    assert rn["dt"] == pytest.approx(r1["dt"], rel=1e-13)


def test_batch_256_octree_pack():
    """256^3 torus on ~700 uneven blocks (16^3 / 32^3 / 64^3): two graph-replayed
    steps equal two eager single-block steps."""
    import torch
    from paper_2410_09146_amd import grmhd as G
    prob = I.torus(n=(256, 256, 256))
    nx, lloc = I.batch_layout(prob, 640)
    nb = len(nx) // 3
    pk, (Pn, Bn, rn) = _run(G, prob, (nx, lloc), 2, graph=True, persist=2048, tune=True)
    del pk
    torch.cuda.empty_cache()
    pk, (P1, B1, r1) = _run(G, prob, None, 2)
    del pk
    torch.cuda.empty_cache()
    eP, eB = rel_err(Pn, P1, prob), rel_err(Bn, B1, prob, face=True)
    say("256^3 batch:", nb, "blocks; eP", eP.max(), "eB", eB.max(), "divb", rn["divb_rel"])
    assert 500 <= nb <= 800
    assert np.all(eP <= 1e-13) and np.all(eB <= 1e-13)
    assert rn["divb_rel"] < 1e-12 and rn["c2p_fail_total"] == 0
