"""Pins of the oracle's lattice, equilibrium, forcing, relaxation and the
parameter maps, against what the paper and the mathematics fix.

Paper: Appendix "Numerical Method" (Eq. LBE, the equilibrium, the moment and
weight-constraint equations), "Dimensionless Numbers" (Eq. knudsen,
Eq. Da_def) and Table 1.
"""

import itertools
import json
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")


def test_d3q19_velocity_set(orc):
    c, w, opp = orc.d3q19()
    expected = {(0, 0, 0)}
    for a in range(3):
        for s in (1, -1):
            e = [0, 0, 0]
            e[a] = s
            expected.add(tuple(e))
    for a, b in itertools.combinations(range(3), 2):
        for sa, sb in itertools.product((1, -1), repeat=2):
            e = [0, 0, 0]
            e[a], e[b] = sa, sb
            expected.add(tuple(e))
    assert {tuple(v) for v in c.tolist()} == expected
    assert len(expected) == 19
    for i in range(19):
        assert opp[opp[i]] == i
        assert (c[opp[i]] == -c[i]).all()
        norm2 = int((c[i] ** 2).sum())
        assert w[i] == pytest.approx({0: 1 / 3, 1: 1 / 18, 2: 1 / 36}[norm2], abs=0)


def test_weight_constraints(orc):
    """sum w = 1, sum w c = 0, sum w c c = cs^2 I (Appendix), plus the fourth-
    order isotropy D3Q19 needs for the Navier-Stokes limit."""
    c, w, _ = orc.d3q19()
    c = c.astype(float)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs(w @ c).max() < 1e-16
    second = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.abs(second - np.eye(3) / 3.0).max() < 1e-15
    fourth = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.abs(fourth - iso).max() < 1e-15


def test_d2q9_weights_printed_meet_the_same_constraints():
    """The paper's own D2Q9 weights satisfy the constraints the D3Q19 set is
    held to (guards the reading that D3Q19 is the 3-D counterpart)."""
    g = json.load(open(GOLDEN))["d2q9_weights"]
    vel = [(0, 0)] + [(1, 0), (-1, 0), (0, 1), (0, -1)] + [(1, 1), (-1, -1), (1, -1), (-1, 1)]
    w = np.array([g["rest"]] + [g["axis"]] * 4 + [g["diagonal"]] * 4)
    c = np.array(vel, dtype=float)
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(np.einsum("i,ia,ib->ab", w, c, c) - np.eye(2) / 3).max() < 1e-15


@pytest.mark.parametrize("rho,u", [(1.0, (0.0, 0.0, 0.0)), (0.8, (0.05, -0.02, 0.01)),
                                   (1.3, (-0.1, 0.07, 0.03)), (0.2, (0.0, 0.0, 0.09))])
def test_equilibrium_moments(orc, rho, u):
    """Moments of the second-order equilibrium: rho, rho u and
    rho cs^2 I + rho u u, exactly (up to rounding)."""
    c, _, _ = orc.d3q19()
    c = c.astype(float)
    u = np.array(u)
    feq = orc.equilibrium(rho, u)
    assert abs(feq.sum() - rho) < 1e-15
    assert np.abs(feq @ c - rho * u).max() < 1e-15
    pi = np.einsum("i,ia,ib->ab", feq, c, c)
    assert np.abs(pi - (rho / 3 * np.eye(3) + rho * np.outer(u, u))).max() < 1e-15


@pytest.mark.parametrize("tau", [0.55, 0.8, 1.7])
def test_guo_forcing_moments(orc, tau):
    """Guo's source: zero mass, momentum (1 - 1/(2 tau)) F, second moment
    (1 - 1/(2 tau)) (u F + F u)."""
    c, _, _ = orc.d3q19()
    c = c.astype(float)
    u = np.array([0.03, -0.01, 0.02])
    F = np.array([2e-3, 5e-4, -1e-3])
    S = orc.guo_source(tau, u, F)
    k = 1 - 1 / (2 * tau)
    assert abs(S.sum()) < 1e-18
    assert np.abs(S @ c - k * F).max() < 1e-18
    second = np.einsum("i,ia,ib->ab", S, c, c)
    assert np.abs(second - k * (np.outer(u, F) + np.outer(F, u))).max() < 1e-18


@pytest.mark.parametrize("tau", [0.7, 1.0, 1.9])
def test_bgk_relaxation_of_uniform_state(orc, tau):
    """In a uniform periodic box streaming is the identity, so the BGK step
    (Eq. LBE) makes the non-equilibrium part decay exactly as (1 - 1/tau)^t."""
    c, _, _ = orc.d3q19()
    c = c.astype(float)
    nz = ny = nx = 2
    vox = np.zeros((nz, ny, nx), np.uint8)
    rng = np.random.default_rng(7)
    # perturbation with zero mass and momentum: project out 1, c_x, c_y, c_z
    basis = np.column_stack([np.ones(19), c])
    d = rng.normal(size=19) * 1e-3
    d -= basis @ np.linalg.lstsq(basis, d, rcond=None)[0]
    rho, u = 1.1, np.array([0.02, -0.01, 0.015])
    feq = orc.equilibrium(rho, u)
    f0 = np.tile(feq + d, (8, 1))
    o = orc.Oracle(vox, tau=(tau, tau), p=0.0, p_stick=0.0, species_x=orc.XPERIODIC)
    o.set_state(fC=f0, fR=0.5 * f0)
    for t in range(1, 6):
        o.step(1)
        fC, fR = o.get_state()
        expect = feq + (1 - 1 / tau) ** t * d
        assert np.abs(fC - expect).max() < 1e-15
        assert np.abs(fR - 0.5 * expect).max() < 1e-15


def test_knudsen_map_matches_paper_example(orc):
    """Eq. (knudsen): tau ~ 4, delta ~ 3 gives Kn ~ 0.6 (the exact value is
    0.674; the paper rounds)."""
    g = json.load(open(GOLDEN))["knudsen_example"]
    kn = orc.kn_from_tau(g["tau"], g["delta"])
    assert kn == pytest.approx(3.5 / math.sqrt(3) / 3, rel=1e-15)
    assert abs(kn - g["kn_printed"]) < g["kn_tolerance"]
    assert orc.tau_from_kn(kn, g["delta"]) == pytest.approx(g["tau"], rel=1e-15)


def test_damkohler_map_matches_table1(orc):
    """Eq. (Da_def) with tau_ch = 1/p and tau_tr = delta / cs (Table 1:
    tau_tr = 3 sqrt 3 at delta = 3, p = 0.45 gives Da ~ 0.4)."""
    g = json.load(open(GOLDEN))["damkohler_example"]
    da = orc.da_from_p(g["p"], g["delta"])
    assert abs(da - g["da_printed"]) < g["da_tolerance"]
    tau_tr = g["delta"] / math.sqrt(1 / 3)
    assert tau_tr == pytest.approx(3 * math.sqrt(3), rel=1e-15)
    assert da == pytest.approx((1 / g["p"]) / tau_tr, rel=1e-15)
    p, clamped = orc.p_from_da(da, g["delta"])
    assert p == pytest.approx(g["p"], rel=1e-14) and not clamped
    # Da -> 0 is fast chemistry: the probability saturates at 1
    p, clamped = orc.p_from_da(1e-3, 3.0)
    assert p == 1.0 and clamped
    # Da -> infinity is infinitely slow chemistry: p = 0
    p, clamped = orc.p_from_da(float("inf"), 3.0)
    assert p == 0.0 and not clamped
