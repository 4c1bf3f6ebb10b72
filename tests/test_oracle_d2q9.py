"""Pins of the oracle built for the paper's own lattice, D2Q9 (Appendix
"Numerical Method", Fig. A1): the same source as the D3Q19 oracle with the
velocity set switched at compile time, run on one plane.

- the velocity set and weights are the paper's (golden fixture, as printed);
  the weights meet sum w = 1, sum w c = 0, sum w c c = cs^2 I and D2Q9's
  fourth-order isotropy;
- a catalytic node has at most 8 active links, counted by brute force;
- body-force channel: the exact discrete solution (parabola plus the
  bounce-back constant that vanishes at tau = 1/2 + sqrt(3)/4) and, with a
  diffuse wall, the closed form with sigma (shared by D2Q9 and D3Q19: the
  x-momentum shares 1/6, 1/6, 2/3 of the up, down and level groups are the
  same);
- reactive slab closed form (a y-uniform D2Q9 run reduces to D1Q3 with
  weights 1/6, 2/3, 1/6) and the D1Q3 run reproduced step by step;
- a closed periodic box with p_S = 0 keeps both lattices' masses, and the
  per-step bookkeeping of the species balances with the product lattice on.
"""

import itertools
import json
import os

import numpy as np
import pytest

import oracle
from paper_1607_02874_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")


def D2(vox, **kw):
    return oracle.Oracle(vox, lattice="D2Q9", **kw)


def test_velocity_set_and_printed_weights():
    c, w, opp = oracle.d3q19("D2Q9")
    g = json.load(open(GOLDEN))["d2q9_weights"]
    expected = {(0, 0, 0)} | {(a, b, 0) for a, b in itertools.product((-1, 0, 1), repeat=2)}
    assert {tuple(v) for v in c.tolist()} == expected and len(c) == 9
    for i in range(9):
        assert opp[opp[i]] == i and (c[opp[i]] == -c[i]).all()
        norm2 = int((c[i] ** 2).sum())
        assert w[i] == pytest.approx({0: g["rest"], 1: g["axis"], 2: g["diagonal"]}[norm2], rel=1e-15)
    cf = c[:, :2].astype(float)
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(w @ cf).max() < 1e-16
    assert np.abs(np.einsum("i,ia,ib->ab", w, cf, cf) - np.eye(2) / 3).max() < 1e-15
    d = np.eye(2)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.abs(np.einsum("i,ia,ib,ic,id->abcd", w, cf, cf, cf, cf) - iso).max() < 1e-15


def test_d2q9_needs_one_plane():
    with pytest.raises(ValueError):
        D2(np.zeros((2, 4, 4), np.uint8))


def test_active_links_at_most_eight_brute_force():
    vox = inputs.porous_slab(30, 24, 1, 0.55, 2.0, 5)
    vox[0, 3, 0] = inputs.CATALYTIC   # at the inlet plane: sources at x = -1 are outside
    vox[0, 10, 1] = inputs.CATALYTIC  # isolated in the gas buffer: all 8 neighbours are gas
    o = D2(vox, species_x=oracle.XRESERVOIR)
    b = o.link_counts()[0]
    c, _, _ = oracle.d3q19("D2Q9")
    ny, nx = vox.shape[1:]
    brute = np.zeros_like(b)
    for y in range(ny):
        for x in range(nx):
            if vox[0, y, x] != inputs.CATALYTIC:
                continue
            for i in range(1, 9):
                sx, sy = x - c[i, 0], (y - c[i, 1]) % ny
                if 0 <= sx < nx and vox[0, sy, sx] == inputs.FLUID:
                    brute[y, x] += 1
    assert np.array_equal(b, brute)
    assert b.max() <= 8 and b[10, 1] == 8 and b[3, 0] == 5


def closed_channel(N, tau, sigma, F):
    nu = (tau - 0.5) / 3
    K = F / nu
    M0 = K * ((N - 1) ** 2 / 8 + N * (1 + sigma * (tau - 1)) / (2 * (2 - sigma)) + (8 * tau ** 2 - 8 * tau - 1) / 12)
    return M0 - (K / 2) * (np.arange(N) - (N - 1) / 2) ** 2


@pytest.mark.parametrize("N,tau,sigma", [(16, 0.8, 0.0), (12, 0.5 + np.sqrt(3) / 4, 0.0), (10, 1.3, 0.6),
                                         (8, 1.1, 1.0)])
def test_channel_exact_solution(N, tau, sigma):
    F = 1e-6
    o = D2(inputs.channel(N), tau=(tau, tau), force=(F, 0, 0), p=0.0, p_stick=0.0, species_x=oracle.XPERIODIC,
           wall_diffuse=sigma)
    o.step(int(60 * N * N / ((tau - 0.5) / 3)) + 500)
    rho, u, _ = o.fields()
    m = (rho * u[0])[0, :N, 0]
    ref = closed_channel(N, tau, sigma, F)
    assert np.abs(m - ref).max() < 1e-9 * np.abs(ref).max()
    assert np.abs(u[1]).max() < 1e-10 * np.abs(u[0]).max()  # round-off only


@pytest.mark.parametrize("sputter", ["UNIFORM", "WEIGHTED"])
@pytest.mark.parametrize("p_stick,tau", [(0.6, 0.7), (0.3, 1.4)])
def test_reactive_slab_closed_form(sputter, p_stick, tau):
    n, cin, p = 12, 0.8, 0.45
    o = D2(inputs.reactive_slab(n, ny=3, nz=1), tau=(0.8, tau), p=p, p_stick=p_stick, c_inlet=cin,
           sputter=getattr(oracle, sputter), species_x=oracle.XRESERVOIR)
    D = (tau - 0.5) / 3
    o.step(int(60 * n * n / D) + 2000)
    _, _, c = o.fields()
    x = np.arange(n)
    exact = cin * (1 - p_stick * (x + tau) / (n * p_stick + 2 * tau - 1))
    for y in range(3):
        assert np.abs(c[0, y, :n] - exact).max() < 1e-10
    t0 = o.totals()
    o.step(1)
    t1 = o.totals()
    J = (tau - 0.5) * p_stick * cin / (3 * (n * p_stick + 2 * tau - 1))
    assert t1["converted"] - t0["converted"] == pytest.approx(3 * p * J, rel=1e-9)


def test_y_uniform_run_reduces_to_d1q3():
    n, steps, tau, ps, cin = 7, 40, 0.9, 0.35, 1.0
    w = {1: 1 / 6, 0: 2 / 3, -1: 1 / 6}
    f = {d: [0.0] * n for d in (1, 0, -1)}
    ref = []
    for _ in range(steps):
        rho = [f[1][x] + f[0][x] + f[-1][x] for x in range(n)]
        post = {d: [f[d][x] - (f[d][x] - w[d] * rho[x]) / tau for x in range(n)] for d in f}
        arrived = post[1][n - 1]
        new = {d: [0.0] * n for d in f}
        for x in range(n):
            new[0][x] = post[0][x]
            new[1][x] = post[1][x - 1] if x > 0 else w[1] * cin
            new[-1][x] = post[-1][x + 1] if x + 1 < n else (1 - ps) * arrived
        f = new
        ref.append((list(f[1]), list(f[0]), list(f[-1])))
    c, _, _ = oracle.d3q19("D2Q9")
    cx = c[:, 0]
    o = D2(inputs.reactive_slab(n, ny=4, nz=1), tau=(0.8, tau), p=0.5, p_stick=ps, c_inlet=cin,
           sputter=oracle.UNIFORM, species_x=oracle.XRESERVOIR)
    for t in range(steps):
        o.step(1)
        _, fR = o.get_state()
        fR = fR.reshape(4, n + 1, 9)
        for y in range(4):
            g = fR[y, :n]
            for k, sel in enumerate((cx == 1, cx == 0, cx == -1)):
                assert np.abs(g[:, sel].sum(1) - ref[t][k]).max() < 1e-15


@pytest.mark.parametrize("sputter", ["UNIFORM", "WEIGHTED", "BOUNCEBACK"])
def test_closed_box_conserves_mass(sputter):
    vox = inputs.porous_slab(40, 32, 1, 0.6, 3.0, 9, x_lo=0, x_hi=40)
    o = D2(vox, tau=(0.8, 0.7), p=0.3, p_stick=0.0, c0=0.5, force=(2e-5, 0, 0), sputter=getattr(oracle, sputter),
           species_x=oracle.XPERIODIC)
    t0 = o.totals()
    o.step(200)
    t1 = o.totals()
    assert abs(t1["mass_gas"] / t0["mass_gas"] - 1) < 1e-13
    assert abs(t1["mass_species"] / t0["mass_species"] - 1) < 1e-12


def test_species_and_product_bookkeeping_per_step():
    """Reactant and product with an inflow inlet: per step, the change of
    (R + P) mass equals influx - outflux (both species) - the stuck and lost
    parts, to round-off."""
    vox = inputs.disk_ingot(6, h=40, length=60, width=80, seed=3)
    o = D2(vox, tau=(1.0, 1.0), p=0.45, p_stick=0.95, c_inlet=0.2, rho0=0.8, force=(4e-5, 0, 0),
           species_x=oracle.XINFLOW, product=True, p_stick_product=0.2)
    o.step(50)
    for _ in range(5):
        t0, (_, tp0, _) = o.totals(), o.product()
        o.step(1)
        t1, (_, tp1, _) = o.totals(), o.product()
        dm = (t1["mass_species"] + tp1["mass_product"]) - (t0["mass_species"] + tp0["mass_product"])
        flux = (t1["influx"] - t0["influx"]) - (t1["outflux"] - t0["outflux"])
        flux -= (tp1["product_out_inlet"] - tp0["product_out_inlet"]) + (tp1["product_out_outlet"] - tp0["product_out_outlet"])
        sink = (t1["lost"] - t0["lost"]) + (tp1["lost_product"] - tp0["lost_product"])
        assert dm == pytest.approx(flux - sink, abs=1e-12 * t1["mass_species"])
