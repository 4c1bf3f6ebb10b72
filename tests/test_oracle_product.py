"""Pins of the oracle's product lattice P (Appendix, second line of the
sputtering equations; the conversion efficiency and the product flux profile
of "Results & Discussion").

Each check ties P to something other than the oracle's own P code:
- superposition: with p = 1 and p_S^P = 0 the catalytic wall re-emits all that
  reaches it as R or P, so R + P evolves as a single species at a
  non-sticking wall (a plain two-lattice run with p_S^R = 0);
- mapping: with p = 0 nothing is produced, and an initial product evolves as
  a reactant with sticking probability p_S^P, no inlet supply and no
  conversion (a plain two-lattice run);
- linearity: the reactant does not depend on p, and P's only source is
  p p_S^R In_R, so P scales exactly with p (PASSIVE);
- bookkeeping: each step M_P changes by what was converted, minus what stuck
  (p_S^P In_P), minus what left through either x-face;
- Phi_P: in a solid-free periodic box the total carrier momentum grows by
  exactly F per node and step, which fixes Phi_P for a product proportional
  to the carrier.
"""

import numpy as np
import pytest

from paper_1607_02874_amd import inputs

SPUTTERS = ["UNIFORM", "WEIGHTED", "BOUNCEBACK", "STOCHASTIC"]


@pytest.fixture(scope="module")
def porous32():
    return inputs.PLAIN_32.voxels()


def _sum_fields(a):
    return a.get_state()[1] + a.get_state_product()


@pytest.mark.parametrize("sputter", SPUTTERS)
@pytest.mark.parametrize("xbc", ["XRESERVOIR", "XINFLOW", "XPERIODIC"])
def test_product_superposition_full_reaction(orc, porous32, sputter, xbc):
    """p = 1, p_S^P = 0: f_R + f_P of the three-lattice run equals f_R of a
    two-lattice run whose wall does not stick (p_S^R = 0), node by node."""
    kw = dict(tau=(0.8, 0.7), c_inlet=1.0, c0=0.2, force=inputs.body_force(4.0, 0.8),
              sputter=getattr(orc, sputter), species_x=getattr(orc, xbc))
    a = orc.Oracle(porous32, p=1.0, p_stick=0.7, product=True, p_stick_product=0.0, **kw)
    b = orc.Oracle(porous32, p=0.3, p_stick=0.0, **kw)
    for steps in (1, 40):
        a.step(steps)
        b.step(steps)
        fa = _sum_fields(a)
        fb = b.get_state()[1]
        assert np.abs(fa - fb).max() < 1e-13
    ta, tb = a.totals(), b.totals()
    _, pa, _ = a.product()
    assert ta["mass_species"] + pa["mass_product"] == pytest.approx(tb["mass_species"], rel=1e-12)
    assert ta["lost"] == 0.0 and pa["lost_product"] == 0.0
    # everything that reached the wall as R came back as P
    assert ta["converted"] > 0.0
    assert ta["influx"] == pytest.approx(tb["influx"], rel=1e-12, abs=1e-14)
    assert ta["outflux"] + pa["product_out_inlet"] + pa["product_out_outlet"] == pytest.approx(
        tb["outflux"], rel=1e-11, abs=1e-13)


@pytest.mark.parametrize("sputter", SPUTTERS)
def test_product_without_reaction_is_a_sticking_reactant(orc, porous32, sputter):
    """p = 0: P receives nothing from R, and a product initially in the gas
    behaves as a reactant with p_S^R = p_S^P, c_inlet = 0 and no conversion."""
    kw = dict(tau=(0.8, 0.7), force=inputs.body_force(4.0, 0.8), sputter=getattr(orc, sputter),
              species_x=orc.XRESERVOIR)
    a = orc.Oracle(porous32, p=0.0, p_stick=0.9, c_inlet=1.0, c0=0.1, product=True,
                   p_stick_product=0.35, **kw)
    b = orc.Oracle(porous32, p=0.0, p_stick=0.35, c_inlet=0.0, c0=0.6, **kw)
    a.set_state_product(b.get_state()[1])  # the same initial equilibrium, c = 0.6
    a.step(60)
    b.step(60)
    assert np.abs(a.get_state_product() - b.get_state()[1]).max() < 1e-14
    conc, tp, stuck = a.product()
    tb = b.totals()
    assert np.abs(conc - b.fields()[2]).max() < 1e-14
    assert tp["lost_product"] == pytest.approx(tb["lost"], rel=1e-12)
    assert tp["product_out_inlet"] + tp["product_out_outlet"] == pytest.approx(tb["outflux"], rel=1e-12)
    # the stuck map is p_S^P times the arrivals; b's lost is (1 - 0) p_S sum In
    assert stuck.sum() == pytest.approx(tb["lost"], rel=1e-12)
    assert (stuck[porous32 != inputs.CATALYTIC] == 0).all()


@pytest.mark.parametrize("sputter", SPUTTERS)
def test_product_scales_with_reaction_probability(orc, porous32, sputter):
    """PASSIVE: the reactant is independent of p, so the product field is
    exactly proportional to p (sources p p_S^R In_R, no product at t = 0)."""
    kw = dict(tau=(0.8, 0.7), p_stick=0.8, c_inlet=1.0, force=inputs.body_force(4.0, 0.8),
              sputter=getattr(orc, sputter), product=True, p_stick_product=0.3)
    a = orc.Oracle(porous32, p=1.0, **kw)
    b = orc.Oracle(porous32, p=0.25, **kw)
    a.step(50)
    b.step(50)
    pa, pb = a.get_state_product(), b.get_state_product()
    assert np.abs(pa).max() > 1e-4
    assert np.abs(0.25 * pa - pb).max() < 1e-15
    assert np.array_equal(a.get_state()[1], b.get_state()[1])
    ta, tb = a.product()[1], b.product()[1]
    for k in ta:
        assert tb[k] == pytest.approx(0.25 * ta[k], rel=1e-11, abs=1e-16)


@pytest.mark.parametrize("sputter", SPUTTERS)
@pytest.mark.parametrize("xbc", ["XRESERVOIR", "XINFLOW", "XPERIODIC"])
@pytest.mark.parametrize("coupling", ["PASSIVE", "BARYCENTRIC"])
def test_product_bookkeeping_per_step(orc, porous32, sputter, xbc, coupling):
    """M_P(t+1) - M_P(t) = converted - p_S^P In_P - out(inlet) - out(outlet)
    each step; no product is injected."""
    o = orc.Oracle(porous32, tau=(0.8, 0.7), p=0.6, p_stick=0.8, c_inlet=1.0, c0=0.3,
                   force=inputs.body_force(4.0, 0.8), sputter=getattr(orc, sputter),
                   species_x=getattr(orc, xbc), coupling=getattr(orc, coupling), product=True,
                   p_stick_product=0.3)
    prev_t, prev_p = o.totals(), o.product()[1]
    assert prev_p["mass_product"] == 0.0
    for _ in range(40):
        o.step(1)
        t, tp = o.totals(), o.product()[1]
        lhs = tp["mass_product"] - prev_p["mass_product"]
        rhs = ((t["converted"] - prev_t["converted"]) - (tp["lost_product"] - prev_p["lost_product"])
               - (tp["product_out_inlet"] - prev_p["product_out_inlet"])
               - (tp["product_out_outlet"] - prev_p["product_out_outlet"]))
        assert abs(lhs - rhs) < 1e-13 * max(t["mass_species"], 1.0)
        prev_t, prev_p = t, tp
    assert tp["mass_product"] > 0.0 and tp["lost_product"] > 0.0
    if xbc == "XPERIODIC":
        assert tp["product_out_inlet"] == 0.0 and tp["product_out_outlet"] == 0.0


@pytest.mark.parametrize("coupling", ["PASSIVE", "BARYCENTRIC"])
def test_product_flux_profile_momentum_closed_form(orc, coupling):
    """Solid-free periodic box driven by F: the carrier's total momentum after
    t steps is exactly N F t (Guo forcing; nothing removes momentum), uniform
    over the box.  With f_P = kappa f_C and no reactant, rho_P u_x summed over
    a cross-section of A nodes is kappa A F (t + 1/2) for PASSIVE and
    kappa A F t + kappa / (1 + kappa) A F / 2 for BARYCENTRIC."""
    nz, ny, nx = 4, 5, 6
    vox = np.zeros((nz, ny, nx), dtype=np.uint8)
    F = 3e-4
    o = orc.Oracle(vox, tau=(0.9, 0.7), p=0.5, p_stick=0.5, c0=0.0, rho0=1.1, force=(F, 0.0, 0.0),
                   species_x=orc.XPERIODIC, coupling=getattr(orc, coupling), product=True)
    assert np.array_equal(o.product_flux(), np.zeros(nx))
    t = 7
    o.step(t)
    kappa = 0.3
    o.set_state_product(kappa * o.get_state()[0])
    A = ny * nz
    want = kappa * A * F * (t + 0.5) if coupling == "PASSIVE" else kappa * A * F * t + kappa / (1 + kappa) * A * F / 2
    assert np.abs(o.product_flux() - want).max() < 1e-15


def test_product_lattice_off_reports_zeros(orc, porous32):
    o = orc.Oracle(porous32, p=0.5, p_stick=0.9, force=inputs.body_force(4.0, 0.8))
    o.step(5)
    conc, tp, stuck = o.product()
    assert not conc.any() and not stuck.any() and all(v == 0.0 for v in tp.values())
    assert not o.product_flux().any()
