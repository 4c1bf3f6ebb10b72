"""The paper's validation of its reactive boundary condition ("Validation of
Numerical Model"): a 2-D laminar channel between parallel plates, 150 x 50
nodes, body-force-driven Poiseuille flow, Peclet number about 253, reactant
injected at the inlet and removed at the bottom plate with reaction and
sticking probability 1.  The wall-normal concentration gradient at the
reactive plate is compared with Leveque's solution,

    d[R]/dy (x) = (4 Pe L_y / x)^(1/3) / (9^(1/3) Gamma(4/3)),

in units of the entering concentration over L_y, with Pe = U_max L_y / D
(wall shear 4 U_max / L_y).  The paper reports a mean absolute error of
about 4 %.

The channel runs on the paper's own D2Q9 (FP64) and on one z-plane of the
3-D lattice (z periodic; with p = p_S = 1 nothing is re-emitted, so the two
evolve the same): fluid rows
y = 1..50, a catalytic row y = 0 and an inert row y = 51.  The gradient
follows from the absorbed flux, d[R]/dy = J / D with D = c_s^2 (tau_R - 1/2),
J the reactant absorbed per wall node and step (the conversion map's growth
with p = p_S = 1).  The reservoir inlet holds rest-equilibrium populations
w_i c_in, which at a cell Peclet number of 5 let only part of c_in into the
flow; the gradient is therefore normalised by the flow-weighted mean
concentration entering at x = 0 (measured: 0.79 c_in).  The INFLOW
boundary injects with the flow (the equilibrium of c_in at the carrier
velocity of the inlet plane); there the gradient is measured against c_in
itself, with no normalisation.
"""

import math

import numpy as np
import pytest

from paper_1607_02874_amd import inputs, lbm

pytestmark = pytest.mark.gpu

LY, LX, PE, UMAX, TAU_C = 50, 150, 253.0, 0.1, 0.8


def channel():
    vox = np.zeros((1, LY + 2, LX), np.uint8)
    vox[0, 0, :] = inputs.CATALYTIC  # reactive bottom plate
    vox[0, LY + 1, :] = inputs.INERT  # inert top plate
    return vox


D3, D2 = lbm.LATTICE_D3Q19, lbm.LATTICE_D2Q9


@pytest.mark.parametrize("storage,species_x,lattice", [
    (0, lbm.XBC_RESERVOIR, D3), (3, lbm.XBC_RESERVOIR, D3), (0, lbm.XBC_INFLOW, D3), (3, lbm.XBC_INFLOW, D3),
    (3, lbm.XBC_RESERVOIR, D2), (3, lbm.XBC_INFLOW, D2)])
def test_leveque_reactive_channel(storage, species_x, lattice):
    nu = (TAU_C - 0.5) / 3.0
    # discrete Poiseuille with halfway bounce-back: U_max = F (h^2 / (2 nu) - 1 / (8 nu) + 6 nu), h = L_y / 2
    force = UMAX / (LY**2 / (8.0 * nu) - 1.0 / (8.0 * nu) + 6.0 * nu)
    diff = UMAX * LY / PE
    tau_r = 0.5 + 3.0 * diff
    vox = channel()
    with lbm.Sim(vox, da=1e-9, tau=(TAU_C, tau_r), pore_size=1.0, force=(force, 0.0, 0.0), p_stick=1.0,
                 c_inlet=1.0, storage=storage, species_x=species_x, lattice=lattice) as s:
        assert s.info()["p"] == 1.0  # instantaneous reaction
        s.step(99000)  # viscous time L_y^2 / nu = 25,000 steps; the boundary layer settles within that
        before = s.conversion_map()
        s.step(1000)
        flux = (s.conversion_map() - before)[0, 0, :] / 1000.0
        _, u, conc = s.fields()
    ux, c = u[0, 0, 1:LY + 1, :], conc[0, 1:LY + 1, :]
    umax = ux[:, LX // 2].max()
    assert abs(umax - UMAX) < 1e-3 * UMAX, umax
    pe = umax * LY / diff
    entering = float((ux[:, 0] * c[:, 0]).sum() / ux[:, 0].sum())
    inflow = species_x == lbm.XBC_INFLOW
    x = np.arange(LX) + 0.5
    grad = flux * LY / diff / (1.0 if inflow else entering)
    leveque = (4.0 * pe * LY / x) ** (1.0 / 3.0) / (9.0 ** (1.0 / 3.0) * math.gamma(4.0 / 3.0))
    sel = (x > 5) & (x < LX - 10)
    mae = float(np.mean(np.abs(grad[sel] - leveque[sel])) / np.mean(leveque[sel]))
    raw = float(np.mean(np.abs(flux * LY / diff - leveque)[sel]) / np.mean(leveque[sel]))
    print(f"Leveque channel lattice {lattice} storage {storage} species_x {species_x}: Pe {pe:.1f}, entering concentration "
          f"{entering:.4f} c_in, MAE {mae:.4f} (against c_in: {raw:.4f})", flush=True)
    if inflow:
        assert 0.95 < entering <= 1.0 + 1e-6, entering
    else:
        assert 0.7 < entering < 0.9, entering
    # measured: 3.77 % with INFLOW (against c_in), 5.00 % with RESERVOIR (normalised by the entering
    # concentration), the same on both lattices; the paper reports about 4 %
    assert mae < (0.045 if inflow else 0.055), mae


def reactor_eta(w, p, steps=60000, window=20000, lattice=D3):
    """The paper's 2-D reactor (Table 1; the p and w/h sweep of "Results &
    Discussion") on one z-plane: efficiency of Eq. (eff) as product leaving
    through the outlet over the reactant inlet flow c_in sum_y u_x(0, y),
    over the last `window` steps, and the mean inlet speed."""
    vox = inputs.disk_ingot(w, seed=w)
    gas = vox[0, :, 0] == inputs.FLUID
    c_in = 0.2
    with lbm.Sim(vox, da=math.sqrt(1.0 / 3.0) / (p * 3.0), tau=(4.0, 4.0), pore_size=3.0, force=(4e-5, 0.0, 0.0),
                 rho0=0.8, c_inlet=c_in, p_stick=0.95, species_x=lbm.XBC_INFLOW, product=True,
                 p_stick_product=0.0, lattice=lattice, storage=3 if lattice == D2 else 0) as s:
        s.step(steps - window)
        t0, q0 = s.totals(), float(s.fields()[1][0, 0, gas, 0].sum())
        s.step(window)
        t1, q1 = s.totals(), float(s.fields()[1][0, 0, gas, 0].sum())
    q = 0.5 * (q0 + q1)
    return (t1["product_out_outlet"] - t0["product_out_outlet"]) / (window * c_in * q), q / int(gas.sum())


@pytest.mark.parametrize("lattice", [D3, D2])
def test_reactor2d_efficiency_trends(lattice):
    """The paper's qualitative findings on its 2-D reactor: the efficiency
    grows with the reaction probability, and the ingot thickness matters
    little next to its perimeter (a five times thicker ingot, five times the
    area, changes eta by far less than five times; eta stays finite as
    w/h -> 0).  The absolute level is not compared: the gas here is periodic
    and force-driven instead of the paper's velocity inlet, and the paper
    gives p_S^R as 0.95 (Table 1) and as about 0.5 (text)."""
    res = {(w, p): reactor_eta(w, p, lattice=lattice) for w in (6, 30) for p in (0.35, 0.65)}
    for (w, p), (eta, u) in res.items():
        print(f"lattice {lattice} w {w} p {p}: eta {eta:.4f}, inlet mean speed {u:.4f}", flush=True)
        assert 0.05 < u < 0.1  # the paper's inlet speed is 0.08
        assert eta > 0.0
    for w in (6, 30):
        assert res[(w, 0.65)][0] > 1.3 * res[(w, 0.35)][0]
    for p in (0.35, 0.65):
        ratio = res[(30, p)][0] / res[(6, p)][0]
        assert 0.5 < ratio < 2.0, ratio


def test_reactor2d_setup_matches_oracle():
    """The exact 2-D reactor configuration behind the efficiency figures
    (disk-carved ingot w = 10, tau 4, INFLOW at 0.2, product lattice,
    p = 0.45), 600 steps, the FP64 build against the oracle.  The carrier and
    reactant fields agree to 1e-12 relative.  The product is made only from
    the In(k) sums, which the library adds in fixed point with absolute
    resolution 2^-S (S = 47 - ceil(log2 c_in) = 49 here, each term rounded to
    half of that); while the product is still minute a relative comparison
    measures that resolution, so it is held to the absolute bound
    steps * 18 terms * 2^-(S + 1)."""
    import oracle

    vox = inputs.disk_ingot(10, seed=10)
    p, steps, c_in = 0.45, 600, 0.2
    kw = dict(tau=(4.0, 4.0), force=(4e-5, 0.0, 0.0), rho0=0.8, c_inlet=c_in, p_stick=0.95)
    o = oracle.Oracle(vox, p=p, species_x=oracle.XINFLOW, product=True, p_stick_product=0.0, **kw)
    o.step(steps)
    ref_rho, ref_u, ref_c = o.fields()
    ref_cp, ref_tp, _ = o.product()
    with lbm.Sim(vox, da=math.sqrt(1.0 / 3.0) / (p * 3.0), pore_size=3.0, species_x=lbm.XBC_INFLOW, product=True,
                 p_stick_product=0.0, storage=3, **kw) as s:
        s.step(steps)
        rho, u, c = s.fields()
        cp, _, _ = s.product_fields()
        t = s.totals()
    gas = vox == inputs.FLUID

    def rel(a, b):
        d, r = ((a - b)[:, gas], b[:, gas]) if a.ndim == 4 else ((a - b)[gas], b[gas])
        return np.linalg.norm(d) / np.linalg.norm(r)

    for a, b in ((rho, ref_rho), (u, ref_u), (c, ref_c)):
        assert rel(a, b) < 1e-12
    shift = 47 - math.ceil(math.log2(c_in))
    bound = steps * 18 * 2.0 ** -(shift + 1)
    assert np.abs(cp - ref_cp).max() < bound
    assert np.abs(ref_cp).max() > 1e3 * bound  # the product is well resolved by then
    assert abs(t["mass_product"] - ref_tp["mass_product"]) < bound * int(gas.sum())
