"""GPU parity of the gray M1 implicit collision update (Phoebus Sec. 2.4,
moments): the HIP Newton solve with its exact Jacobian against the oracle's
Newton solve on the same cells, three species, Minkowski and Kerr-Schild."""
import numpy as np
import pytest

import oracle
from paper_2410_09146_amd import inputs as I
from parity_util import say

pytestmark = pytest.mark.gpu

TOL = 1e-11


@pytest.fixture(scope="module")
def grmhd():
    import torch
    assert torch.cuda.is_available(), "GPU parity tests need an MI355X"
    from paper_2410_09146_amd import grmhd as G
    G.lib()
    return G


def _run(G, prob, dt, couple=False, scale_kappa=1.0):
    import torch
    R, kap = I.m1_fields(prob)
    kap[:, :2] *= scale_kappa
    pack = G.Pack(prob)
    pack.upload(prob.P, prob.Bf)
    pack.fill_ghosts()
    pack.prim_to_cons()
    dev = pack.device
    Rd = torch.from_numpy(pack.to_pack_layout(R).reshape(3, 4, -1)).to(dev).contiguous()
    Kd = torch.from_numpy(pack.to_pack_layout(kap).reshape(3, 3, -1)).to(dev).contiguous()
    it = torch.zeros(pack.nct, dtype=torch.uint8, device=dev)
    U0 = pack.download("U")
    pack.m1_source(Rd, Kd, dt, couple=couple, iters=it)
    pack._out()
    torch.cuda.synchronize()
    Rg = pack.from_pack_layout(Rd.cpu().numpy(), prob.shape)
    itg = pack.from_pack_layout(it.cpu().numpy().astype(np.float64), prob.shape)
    return R, kap, Rg, itg, U0, pack


def _compare(prob, Rg, Ro):
    it = (slice(None), slice(None)) + prob.interior()
    out = np.zeros((Ro.shape[0], 4))
    for s in range(Ro.shape[0]):
        for v in range(4):
            a, b = Rg[s, v][prob.interior()], Ro[s, v][prob.interior()]
            den = np.abs(b).max()
            out[s, v] = np.abs(a - b).max() / den if den > 0 else np.abs(a - b).max()
    return out


@pytest.mark.parametrize("case,dt,kscale", [("torus", 0.01, 1.0), ("torus", 1.0, 1.0),
                                            ("torus_stiff", 0.01, 1e4), ("box", 0.05, 1.0)])
def test_m1_source_matches_oracle(grmhd, case, dt, kscale):
    prob = I.torus(n=(32, 32, 16)) if case.startswith("torus") else \
        I.random_smooth_box((20, 18, 16), seed=3, amp=0.2)
    if case == "box":
        prob.P[1:4] *= 4.0          # |v| up to ~0.6
    R, kap, Rg, itg, U0, pack = _run(grmhd, prob, dt, scale_kappa=kscale)   # kap is scaled
    Ro = R.copy()
    blk = oracle.Block(prob)
    ito, bad = blk.m1_update(prob.P, Ro, kap, dt, nthreads=8)
    e = _compare(prob, Rg, Ro)
    interior = itg[prob.interior()]
    say("m1", case, "dt", dt, "kappa x", kscale, "err per species/component", e.max(axis=1),
        "newton its gpu mean", interior.mean(), "max", interior.max(),
        "oracle max", np.abs(ito[prob.interior()]).max())
    assert bad == 0
    assert interior.max() < 255
    assert np.all(e <= TOL), e


def test_m1_zero_opacity_is_identity(grmhd):
    prob = I.torus(n=(24, 24, 8))
    R, kap, Rg, itg, U0, pack = _run(grmhd, prob, 0.5, scale_kappa=0.0)
    it = (slice(None), slice(None)) + prob.interior()
    assert np.array_equal(Rg[it], R[it])


def test_m1_coupling_conserves_energy_momentum(grmhd):
    """With coupling the fluid's tau and S_i absorb exactly what the
    radiation gains: tau + sum_s E_s and S_i + sum_s F_i,s are unchanged per
    cell (densitized, to rounding)."""
    prob = I.torus(n=(24, 24, 8))
    R, kap, Rg, itg, U0, pack = _run(grmhd, prob, 0.2, couple=True)
    U1 = pack.download("U")
    itr = prob.interior()
    dE = (Rg[:, 0] - R[:, 0]).sum(axis=0)[itr]
    dtau = (U1[4] - U0[4])[itr]
    scale = np.abs(U0[4][itr]).max() + np.abs(R[:, 0]).sum(axis=0)[itr].max()
    say("coupling: max |d tau + d E| / scale", np.abs(dtau + dE).max() / scale)
    assert np.abs(dtau + dE).max() <= 1e-14 * scale
    for i in range(3):
        dF = (Rg[:, 1 + i] - R[:, 1 + i]).sum(axis=0)[itr]
        dS = (U1[1 + i] - U0[1 + i])[itr]
        sc = np.abs(U0[1 + i][itr]).max() + np.abs(R[:, 1 + i]).sum(axis=0)[itr].max()
        assert np.abs(dS + dF).max() <= 1e-14 * sc
    assert np.abs(dE).max() > 0


def test_m1_torus128_sampled(grmhd):
    """The 128^3 torus with three species at the benchmark's dt: every cell
    of a few sampled planes against the oracle's point solve."""
    import torch
    prob = I.torus(n=(128, 128, 128))
    dt = 0.006
    R, kap, Rg, itg, U0, pack = _run(grmhd, prob, dt)
    blk = oracle.Block(prob)
    g = prob.ng
    worst = 0.0
    for k in (g, g + 37, g + 127):
        for j in range(g, g + 128, 9):
            for i in range(g, g + 128, 7):
                x = blk.coord(0, i, j, k)
                G = oracle.geom(blk.metric, x)
                ut = prob.P[1:4, k, j, i]
                for s in range(3):
                    Xs = R[s, :, k, j, i] / G["sqrtgam"]
                    it, X = oracle.m1_implicit(blk.metric, x, ut, Xs, kap[s, :, k, j, i], dt)
                    assert it > 0
                    ref = G["sqrtgam"] * X
                    err = np.abs(Rg[s, :, k, j, i] - ref).max() / (np.abs(ref).max() + 1e-300)
                    worst = max(worst, err)
    say("128^3 sampled cells: worst relative error", worst, "newton its max",
        itg[prob.interior()].max())
    assert worst <= TOL
