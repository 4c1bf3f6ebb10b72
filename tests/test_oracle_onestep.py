"""One-step pins of two parts of the oracle that the closed forms and the
bookkeeping invariants cannot see.

With tau = 1e15 the collision leaves every population as it is (to 1e-15),
so one step of the oracle is pure streaming plus the sputtering boundary,
and its output can be recomputed here, link by link, from distinct random
populations:

- WEIGHTED sputtering (reading of the random matrix S as a diffuse,
  w_i-weighted re-emission; first line of the sputtering equations): the
  reactant a gas node pulls from catalytic node k along c_i is
  (1 - p_S^R) In(k) w_i / sum_{m in A'(k)} w_m, with
  In(k) = sum_{j in A(k)} f_j(k - c_j).  The slab and D1Q3 pins only see sums
  over each c_x group, and mass conservation only the total; these per-link
  values would change if WEIGHTED spread In(k) uniformly.
- The RESERVOIR outlet ghost (zero-gradient outlet plane at x = nx): a node
  at x = nx - 1 pulling along c_i with c_ix = -1 takes f*_i of the gas node
  (nx - 1, y - c_iy, z - c_iz), the source row of a pull across the plane,
  or its own reversed population where that node is solid.  A ghost that
  copied the node's own row (nx - 1, y, z) would give different values.
"""

import numpy as np
import pytest

from paper_1607_02874_amd import inputs


def _distinct_state(o, vox, rng):
    fC, fR = o.get_state()
    gas = vox.reshape(-1) == inputs.FLUID
    fC = np.where(gas[:, None], 1.0 + rng.random(fC.shape), 0.0)
    fR = np.where(gas[:, None], 0.5 + rng.random(fR.shape), 0.0)
    o.set_state(fC, fR)
    return fC, fR


@pytest.mark.parametrize("p_stick", [0.4, 0.0])
def test_weighted_sputter_share_per_link(orc, p_stick):
    rng = np.random.default_rng(31)
    shape = (6, 7, 9)
    nz, ny, nx = shape
    vox = np.where(rng.random(shape) < 0.35, inputs.CATALYTIC, inputs.FLUID).astype(np.uint8)
    vox[rng.random(shape) < 0.05] = inputs.INERT
    c, w, opp = orc.d3q19()
    o = orc.Oracle(vox, tau=(1e15, 1e15), p=0.3, p_stick=p_stick, species_x=orc.XPERIODIC,
                   sputter=orc.WEIGHTED)
    _, fR = _distinct_state(o, vox, rng)
    o.step(1)
    _, fR1 = o.get_state()
    o.close()

    def idx(z, y, x):
        return ((z % nz) * ny + (y % ny)) * nx + (x % nx)

    checked = differs = 0
    for z, y, x in zip(*np.nonzero(vox == inputs.CATALYTIC)):
        act = [j for j in range(1, 19) if vox.flat[idx(z - c[j][2], y - c[j][1], x - c[j][0])] == inputs.FLUID]
        if not act:
            continue
        inflow = sum(fR[idx(z - c[j][2], y - c[j][1], x - c[j][0]), j] for j in act)
        exits = [opp[j] for j in act]
        wsum = sum(w[i] for i in exits)
        for i in exits:
            n = idx(z + c[i][2], y + c[i][1], x + c[i][0])  # the gas node that pulls along c_i from k
            want = (1.0 - p_stick) * inflow * w[i] / wsum
            uniform = (1.0 - p_stick) * inflow / len(exits)
            assert fR1[n, i] == pytest.approx(want, rel=1e-12, abs=1e-15), (z, y, x, i)
            checked += 1
            differs += abs(want - uniform) > 1e-6 * inflow
    assert checked > 200
    if p_stick < 1.0:
        assert differs > 100  # a uniform spread would fail on these links


def test_outlet_ghost_copies_the_source_row(orc):
    rng = np.random.default_rng(32)
    shape = (7, 8, 10)
    nz, ny, nx = shape
    vox = np.where(rng.random(shape) < 0.25, inputs.CATALYTIC, inputs.FLUID).astype(np.uint8)
    vox[:, :, 0] = inputs.FLUID
    # the outlet plane keeps some solid, so the bounce-back branch is seen too
    c, w, opp = orc.d3q19()
    o = orc.Oracle(vox, tau=(1e15, 1e15), p=0.3, p_stick=0.7, species_x=orc.XRESERVOIR)
    _, fR = _distinct_state(o, vox, rng)
    o.step(1)
    _, fR1 = o.get_state()
    o.close()
    x = nx - 1
    checked = reflected = differs = 0
    for z in range(nz):
        for y in range(ny):
            n = (z * ny + y) * nx + x
            if vox[z, y, x] != inputs.FLUID:
                continue
            for i in range(1, 19):
                if c[i][0] != -1:
                    continue
                sy, sz = (y - c[i][1]) % ny, (z - c[i][2]) % nz
                m = (sz * ny + sy) * nx + x
                if vox[sz, sy, x] == inputs.FLUID:
                    want = fR[m, i]
                else:
                    want = fR[n, opp[i]]
                    reflected += 1
                assert fR1[n, i] == pytest.approx(want, rel=1e-13), (z, y, i)
                checked += 1
                differs += (c[i][1] != 0 or c[i][2] != 0) and abs(want - fR[n, i]) > 1e-6
    assert checked > 100 and reflected > 5
    assert differs > 50  # a ghost copying the node's own row would fail here
