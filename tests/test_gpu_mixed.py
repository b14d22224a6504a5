"""Mixed precision (FP32 staging, reconstruction, Riemann solve; FP64
densitization, U, face field, RK accumulation and inversion) against FP64."""
import numpy as np
import pytest

import oracle
from paper_2410_09146_amd import inputs as I
from parity_util import rel_err, say, upload_all

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    assert torch.cuda.is_available()
    from paper_2410_09146_amd import grmhd
    grmhd.lib()
    return grmhd


def test_mixed_step_close_to_oracle(G):
    """One SSPRK2 step from the oracle's state: FP32-level agreement."""
    prob = I.torus(n=(32, 32, 16))
    sim = oracle.Sim(prob, 8)
    pack = G.Pack(prob, precision=G.PREC_MIXED)
    for s in range(2):
        dt = sim.dt()
        upload_all(pack, sim.P, sim.Bf, sim.U)
        pack.fill_ghosts()
        pack.step(dt)
        sim.step(dt)
        eP = rel_err(pack.download("P"), sim.P, prob)
        eB = rel_err(pack.download("Bf"), sim.Bf, prob, face=True)
        say("mixed step", s, "eP", eP, "eB", eB)
        # FP32 face states: rho and u agree to ~1e-8, the small velocity
        # components (own-norm) and the field to ~1e-4
        assert eP[0] < 1e-6 and eP[4] < 1e-5
        assert np.all(eP < 5e-4) and np.all(eB < 5e-4)
        assert eP.max() > 1e-12   # the FP32 path really ran


def test_fp64_192_27blocks_step_matches_oracle(G):
    """The production shape of the mixed-precision configuration in FP64 (the
    run its 100-step L1 is measured against): the 192^3 torus in 27 blocks of
    64^3, one SSPRK2 step against the oracle's single-block step from the same
    state, per variable 1e-11 of its max norm, and no failed inversion."""
    import torch
    prob = I.torus(n=(192, 192, 192))
    sim = oracle.Sim(prob, 16)
    pack = G.Pack(prob, nblk=(3, 3, 3))
    dt = sim.dt()
    upload_all(pack, sim.P, sim.Bf, sim.U)
    pack.fill_ghosts()
    f0 = pack.reductions()["c2p_fail_total"]
    pack.step(dt)
    sim.step(dt)
    eP = rel_err(pack.download("P"), sim.P, prob)
    eU = rel_err(pack.download("U"), sim.U, prob)
    eB = rel_err(pack.download("Bf"), sim.Bf, prob, face=True)
    red = pack.reductions()
    say("fp64 192^3 x 27 blocks, one step vs oracle: eP", eP.max(), "eU", eU.max(), "eB", eB.max(),
        "dt", dt, "c2p fail", red["c2p_fail_total"] - f0)
    del pack
    torch.cuda.empty_cache()
    assert np.all(eP <= 1e-11) and np.all(eU <= 1e-11) and np.all(eB <= 1e-11)
    assert red["c2p_fail_total"] == f0


def l1_rel(a, b, dV):
    return np.sum(np.abs(a - b) * dV) / np.sum(np.abs(b) * dV)


def test_mixed_192_27blocks_100_steps(G):
    """Torus at 192^3 in 27 blocks of 64^3, 100 steps: per-variable relative
    L1 of rho, u, B against the FP64 path (at this very shape equal to the
    oracle per step to 1e-11, test above) and the div B maximum.  Gate:
    L1(rho) <= 1e-5."""
    import torch
    prob = I.torus(n=(192, 192, 192))
    runs = {}
    for prec in (G.PREC_FP64, G.PREC_MIXED):
        pack = G.Pack(prob, nblk=(3, 3, 3), precision=prec)
        pack.init()
        pack.reductions(sync=False)
        for _ in range(100):
            pack.step(None)
            pack.reductions(sync=False)
        red = pack.reductions()
        runs[prec] = (pack.download("P"), pack.download("Bf"), red)
        del pack
        torch.cuda.empty_cache()
    (P64, B64, r64), (P32, B32, r32) = runs[G.PREC_FP64], runs[G.PREC_MIXED]
    g = prob.ng
    it = (slice(g, -g),) * 3
    r = np.exp(prob.centers(0))[g:-g]
    th = prob.centers(1)[g:-g]
    dV = (r[None, None, :] ** 3 * np.sin(th)[None, :, None])   # ~ sqrt(-g) in (ln r, theta, phi)
    out = {"rho": l1_rel(P32[0][it], P64[0][it], dV), "u": l1_rel(P32[4][it], P64[4][it], dV)}
    for d in range(3):
        out[f"B{d + 1}"] = l1_rel(B32[d][it], B64[d][it], dV) if np.abs(B64[d][it]).max() > 0 else 0.0
    say("mixed 192^3 x 27 blocks, 100 steps: L1", {k: f"{v:.2e}" for k, v in out.items()},
        "divb_rel fp64", r64["divb_rel"], "mixed", r32["divb_rel"],
        "c2p fail", r64["c2p_fail_total"], r32["c2p_fail_total"])
    assert out["rho"] <= 1e-5
    assert r32["divb_rel"] < 1e-10
