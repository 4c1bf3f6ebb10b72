"""Pins of the oracle's diffuse gas wall (Maxwell accommodation, fraction
sigma diffuse, the rest bounced back; lattice Boltzmann form of Ansumali and
Karlin 2002).

- sigma = 0 is halfway bounce-back, bit for bit;
- one step with distinct populations and no collision: every population
  pulled from a solid source is (1 - sigma) f*_opp + sigma w_i M / W with M the
  mass the node sent into the wall, computed here independently;
- mass is conserved exactly in a closed box at any sigma;
- more diffuse reflection means more slip: the flow rate of a forced channel
  grows with sigma (full accommodation of tangential momentum is less drag
  than its reversal).
"""

import numpy as np
import pytest

from paper_1607_02874_amd import inputs


def test_zero_diffuse_fraction_is_bounce_back(orc):
    vox = inputs.PLAIN_32.voxels()
    kw = dict(tau=(0.8, 0.7), p=0.3, p_stick=0.9, force=inputs.body_force(4.0, 0.8))
    a = orc.Oracle(vox, wall_diffuse=0.0, **kw)
    b = orc.Oracle(vox, **kw)
    a.step(30)
    b.step(30)
    for x, y in zip(a.get_state(), b.get_state()):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("sigma", [0.3, 1.0])
def test_wall_rule_on_distinct_populations(orc, sigma):
    rng = np.random.default_rng(9)
    shape = (5, 6, 7)
    vox = np.where(rng.random(shape) < 0.3, inputs.INERT, inputs.FLUID).astype(np.uint8)
    vox[rng.random(shape) < 0.1] = inputs.CATALYTIC
    nz, ny, nx = shape
    c, w, opp = orc.d3q19()
    o = orc.Oracle(vox, tau=(1e15, 0.7), p=0.0, p_stick=0.0, species_x=orc.XPERIODIC, wall_diffuse=sigma)
    fC, _ = o.get_state()
    gas = vox.reshape(-1) == inputs.FLUID
    fC = np.where(gas[:, None], rng.random(fC.shape) + 1.0, 0.0)
    o.set_state(fC=fC)
    o.step(1)
    fC1, _ = o.get_state()
    checked = 0
    for z, y, x in zip(*np.nonzero(vox == inputs.FLUID)):
        n = (z * ny + y) * nx + x
        solid = []
        for i in range(19):
            s = ((z - c[i][2]) % nz, (y - c[i][1]) % ny, (x - c[i][0]) % nx)
            if vox[s] != inputs.FLUID:
                solid.append(i)
        if not solid:
            continue
        M = sum(fC[n, opp[i]] for i in solid)
        W = sum(w[i] for i in solid)
        for i in solid:
            want = (1 - sigma) * fC[n, opp[i]] + sigma * w[i] * M / W
            assert fC1[n, i] == pytest.approx(want, rel=1e-12)
            checked += 1
    assert checked > 100


@pytest.mark.parametrize("sigma", [0.5, 1.0])
def test_diffuse_wall_conserves_mass(orc, sigma):
    vox = inputs.PLAIN_32.voxels()
    o = orc.Oracle(vox, tau=(0.8, 0.7), p=0.3, p_stick=0.0, c0=0.4, force=inputs.body_force(4.0, 0.8),
                   species_x=orc.XPERIODIC, wall_diffuse=sigma)
    t0 = o.totals()
    o.step(100)
    t1 = o.totals()
    assert abs(t1["mass_gas"] / t0["mass_gas"] - 1) < 1e-13
    assert abs(t1["mass_species"] / t0["mass_species"] - 1) < 1e-12


def test_diffuse_wall_slips(orc):
    """Forced plane channel (one inert wall row, y periodic), tau 1.5
    (rarefied, Kn ~ c_s (tau - 1/2) / H): the steady flow rate grows with the
    diffuse fraction."""
    vox = inputs.channel(12, nx=1, nz=1)
    flow = []
    for sigma in (0.0, 0.5, 1.0):
        o = orc.Oracle(vox, tau=(1.5, 0.7), p=0.0, p_stick=0.0, force=(1e-5, 0.0, 0.0), species_x=orc.XPERIODIC,
                       wall_diffuse=sigma)
        o.step(3000)
        flow.append(float(o.fields()[1][0].sum()))
    assert flow[0] < flow[1] < flow[2], flow
