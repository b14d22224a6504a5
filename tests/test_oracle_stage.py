"""Stage-level pins of the oracle: exact invariants of the scheme and
convergence to analytic solutions (Phoebus Sec. 3.1 scheme, Sec. 4.1.1 linear
waves; an SR shock tube with exact solution; stationary Michel inflow)."""
import os

import numpy as np
import pytest

import oracle
from paper_2410_09146_amd import inputs as I
from srhd_exact import ExactRiemann

NT = min(8, os.cpu_count() or 1)


def test_uniform_state_preserved_exactly():
    prob = I.uniform_box((8, 8, 8), rho=1.3, ut=(0.2, -0.1, 0.3), u=0.8, B=(0.4, 0.1, -0.2),
                         recon=I.RECON_WENO5Z, riemann=I.RIEMANN_LLF)
    sim = oracle.Sim(prob, NT)
    U0, B0 = sim.U.copy(), sim.Bf.copy()
    for _ in range(3):
        sim.step()
    it = (slice(None),) + prob.interior()
    assert np.array_equal(sim.U[it], U0[it])
    assert np.array_equal(sim.Bf[it], B0[it])


@pytest.mark.parametrize("recon,riemann", [(I.RECON_PLM_MC, I.RIEMANN_HLL),
                                           (I.RECON_WENO5Z, I.RIEMANN_LLF)])
def test_periodic_conservation_and_divb(recon, riemann):
    """Periodic Minkowski box: sum of sqrt(gamma) U is conserved to rounding and
    the discrete div of the face field stays at rounding (CT antisymmetry)."""
    prob = I.random_smooth_box((12, 10, 8), seed=4, amp=0.08, recon=recon, riemann=riemann)
    sim = oracle.Sim(prob, NT)
    red0 = sim.blk.reductions(sim.P, sim.Bf, sim.U, 0.4)
    for _ in range(10):
        sim.step()
        red = sim.blk.reductions(sim.P, sim.Bf, sim.U, 0.4)
        scale = np.abs(red0["totals"]).max()
        assert np.all(np.abs(red["totals"] - red0["totals"]) <= 1e-13 * scale)
        assert red["divb_rel"] <= 1e-13


def test_divb_insensitive_to_ghost_garbage():
    """The interior discrete divergence of the CT update does not depend on
    any EMF value, so garbage in the ghost field leaves it at rounding."""
    prob = I.random_smooth_box((8, 8, 8), seed=5)
    blk = oracle.Block(prob)
    P, Bf = prob.P.copy(), prob.Bf.copy()
    blk.fill_ghosts(P, Bf)
    U = blk.prim_to_cons(P, Bf)
    rng = np.random.default_rng(0)
    g = prob.ng
    Bbad = Bf.copy()
    Bbad[:, :, :, :g] += rng.normal(size=Bbad[:, :, :, :g].shape)
    Uo, Bo = blk.stage(P, Bbad, U, Bbad, U, 0.01, (1.0, 0.0, 1.0))
    div0 = blk.reductions(P, Bbad, U, 0.4)["divb_max"]
    div1 = blk.reductions(P, Bo, Uo, 0.4)["divb_max"]
    assert abs(div1 - div0) < 1e-11


def _wave_l1(N, mode="fast"):
    prob = I.linear_wave((N, N, 1), k=(1, 1, 0), amp=1e-6, mode=mode)
    sim = oracle.Sim(prob, NT)
    T = prob.meta["period"]
    while sim.t < T - 1e-14:
        dt = min(sim.dt(), T - sim.t)
        sim.step(dt)
    it = (slice(None),) + prob.interior()
    err = np.abs(sim.P[it] - prob.P[it]).sum(axis=(1, 2, 3)) / (prob.meta["amp"] * N * N)
    return err


def test_linear_fast_wave_second_order():
    """Fast magnetosonic eigenmode, one period: amplitude-scaled L1 error of
    every primitive converges at about second order (Sec. 4.1.1)."""
    e = [_wave_l1(N) for N in (16, 32, 64)]
    e = np.array(e)
    tot = e[:, [0, 1, 2, 4]].sum(axis=1)
    orders = np.log2(tot[:-1] / tot[1:])
    assert np.all(orders > 1.7), (tot, orders)
    assert tot[-1] < 0.05


@pytest.mark.parametrize("case", ["sod", "strong", "sod_mp5"])
def test_shock_tube_vs_exact(case):
    """B = 0 shock tube against the exact SR Riemann solution: L1(rho)
    converges at about first order (discontinuities)."""
    recon = I.RECON_MP5 if case.endswith("mp5") else I.RECON_PLM_MC
    if case.startswith("sod"):
        L, R, g, tend = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 5.0 / 3.0, 0.4
    else:
        L, R, g, tend = (10.0, 0.0, 13.33), (1.0, 0.0, 0.01333), 5.0 / 3.0, 0.35
    ex = ExactRiemann(L, R, g)
    errs = []
    for N in (100, 200, 400):
        prob = I.shock_tube(N, L, R, g, recon=recon)
        sim = oracle.Sim(prob, NT)
        while sim.t < tend - 1e-14:
            sim.step(min(sim.dt(), tend - sim.t))
        x = prob.centers(0)[prob.ng:prob.ng + N]
        rho = sim.P[0, prob.ng, prob.ng, prob.ng:prob.ng + N]
        rho_ex = ex.sample((x - 0.5) / tend)[:, 0]
        errs.append(np.mean(np.abs(rho - rho_ex)))
    errs = np.array(errs)
    orders = np.log2(errs[:-1] / errs[1:])
    assert np.all(orders > 0.6), (errs, orders)
    assert errs[-1] < (0.01 if case.startswith("sod") else 0.05)


def test_michel_inflow_held_to_truncation_error():
    """Stationary transonic inflow on Schwarzschild (KS): after a fixed time
    the deviation from the exact solution shrinks at about second order."""
    errs = []
    for N in (32, 64, 128):
        prob = I.bondi(N)
        sim = oracle.Sim(prob, NT)
        tend = 5.0
        while sim.t < tend - 1e-14:
            sim.step(min(sim.dt(), tend - sim.t))
        g = prob.ng
        rho = sim.P[0, g, g, g:g + N]
        rho0 = prob.P[0, g, g, g:g + N]
        errs.append(np.mean(np.abs(rho - rho0) / rho0))
    errs = np.array(errs)
    orders = np.log2(errs[:-1] / errs[1:])
    assert np.all(orders > 1.5), (errs, orders)
