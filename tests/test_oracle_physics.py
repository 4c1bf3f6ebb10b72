"""Pins of the oracle's whole step against closed forms, invariants, special
cases and brute force.

Paper: Appendix "Numerical Method" (Eq. LBE; the sputtering boundary
condition, eqnarray f_R_in / f_P_in, and the remark that it conserves
R + P mass only when the sticking probabilities vanish) and "Validation of
Numerical Model" (body-force-driven channel).
"""

import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1607_02874_amd import inputs


def _group_sums(f, cx):
    return f[:, cx == 1].sum(1), f[:, cx == 0].sum(1), f[:, cx == -1].sum(1)


# ----------------------------------------------------------- Poiseuille --

@pytest.mark.parametrize("n,tau", [(32, 0.8), (16, 0.5 + np.sqrt(3) / 4), (20, 1.3)])
def test_poiseuille_discrete_closed_form(orc, n, tau):
    """Body-force channel with halfway bounce-back walls.  The steady lattice
    solution is exactly rho u(y) = F/(2 nu) (h^2 - z^2) + F (6 nu - 1/(8 nu)),
    z = y - (n-1)/2, h = n/2, nu = (tau - 1/2)/3 (a parabola plus a constant
    slip that vanishes at tau = 1/2 + sqrt(3)/4)."""
    F = 1e-5
    o = orc.Oracle(inputs.channel(n), tau=(tau, tau), force=(F, 0, 0), p=0.0, p_stick=0.0,
                   species_x=orc.XPERIODIC)
    nu = (tau - 0.5) / 3
    steps = int(40.0 * n * n / (nu * np.pi ** 2)) + 1000
    o.step(steps)
    rho, u, _ = o.fields()
    ru = (rho * u[0])[0, :n, 0]
    z = np.arange(n) - (n - 1) / 2
    h = n / 2
    exact = F / (2 * nu) * (h * h - z * z) + F * (6 * nu - 1 / (8 * nu))
    assert np.abs(ru - exact).max() < 1e-10 * np.abs(exact).max()
    assert np.abs(u[1:]).max() < 1e-11 * np.abs(u[0]).max()
    if n == 32 and tau == 0.8:
        analytic = F / (2 * nu) * (h * h - z * z)
        err = np.linalg.norm(ru - analytic) / np.linalg.norm(analytic)
        assert err < 1e-3
        assert err == pytest.approx(6.954e-4, rel=1e-3)


# ------------------------------------------------------- reactive slab --

@pytest.mark.parametrize("sputter", ["UNIFORM", "WEIGHTED"])
@pytest.mark.parametrize("p_stick,tau", [(0.6, 0.7), (1.0, 1.0), (0.3, 1.4)])
def test_reactive_slab_closed_form(orc, sputter, p_stick, tau):
    """Species between a reservoir (x = -1, c_in) and a catalytic plane at
    x = n that removes the fraction p_S of what arrives.  Steady state:
    c(x) = c_in [1 - p_S (x + tau) / (n p_S + 2 tau - 1)], wall flux
    J = (tau - 1/2) p_S c_in / (3 (n p_S + 2 tau - 1)), converted p J per
    column and step, and J = -D dc/dx with D = (tau - 1/2)/3 exactly."""
    n, cin, p = 12, 0.8, 0.45
    o = orc.Oracle(inputs.reactive_slab(n, ny=2, nz=2), tau=(0.8, tau), p=p, p_stick=p_stick,
                   c_inlet=cin, sputter=getattr(orc, sputter), species_x=orc.XRESERVOIR)
    D = (tau - 0.5) / 3
    o.step(int(60 * n * n / D) + 2000)
    _, u, c = o.fields()
    x = np.arange(n)
    exact = cin * (1 - p_stick * (x + tau) / (n * p_stick + 2 * tau - 1))
    for yz in [(0, 0), (1, 1), (0, 1)]:
        assert np.abs(c[yz[0], yz[1], :n] - exact).max() < 1e-10
    assert np.abs(u).max() == 0.0
    t0 = o.totals()
    o.step(1)
    t1 = o.totals()
    J = (tau - 0.5) * p_stick * cin / (3 * (n * p_stick + 2 * tau - 1))
    columns = 4
    assert t1["converted"] - t0["converted"] == pytest.approx(columns * p * J, rel=1e-9)
    assert t1["lost"] - t0["lost"] == pytest.approx(columns * (1 - p) * J, rel=1e-9)
    grad = c[0, 0, 1] - c[0, 0, 0]
    assert J == pytest.approx(-D * grad, rel=1e-9)


def _d1q3_slab(n, steps, tau, p_stick, cin):
    """Brute-force D1Q3 (weights 2/3, 1/6, 1/6) of the same slab: what the
    3-D lattice must reduce to when nothing varies in y and z."""
    w = {1: 1 / 6, 0: 2 / 3, -1: 1 / 6}
    f = {d: [0.0] * n for d in (1, 0, -1)}
    hist = []
    for _ in range(steps):
        rho = [f[1][x] + f[0][x] + f[-1][x] for x in range(n)]
        post = {d: [f[d][x] - (f[d][x] - w[d] * rho[x]) / tau for x in range(n)] for d in f}
        arrived = post[1][n - 1]
        new = {d: [0.0] * n for d in f}
        for x in range(n):
            new[0][x] = post[0][x]
            new[1][x] = post[1][x - 1] if x > 0 else w[1] * cin
            new[-1][x] = post[-1][x + 1] if x + 1 < n else (1 - p_stick) * arrived
        f = new
        hist.append((list(f[1]), list(f[0]), list(f[-1])))
    return hist


@pytest.mark.parametrize("sputter", ["UNIFORM", "WEIGHTED", "BOUNCEBACK"])
def test_yz_uniform_run_reduces_to_d1q3(orc, sputter):
    """A y/z-uniform D3Q19 run equals the D1Q3 run step by step, transient
    included (group sums over c_x; pins streaming, inlet ghost and the
    one-step timing of the sputter re-emission)."""
    n, steps, tau, ps, cin = 7, 40, 0.9, 0.35, 1.0
    ref = _d1q3_slab(n, steps, tau, ps, cin)
    c, _, _ = orc.d3q19()
    cx = c[:, 0]
    o = orc.Oracle(inputs.reactive_slab(n, ny=3, nz=2), tau=(0.8, tau), p=0.5, p_stick=ps,
                   c_inlet=cin, sputter=getattr(orc, sputter), species_x=orc.XRESERVOIR)
    nx = n + 1
    for t in range(steps):
        o.step(1)
        _, fR = o.get_state()
        fR = fR.reshape(2, 3, nx, 19)
        for z in range(2):
            for y in range(3):
                plus, rest, minus = _group_sums(fR[z, y, :n], cx)
                assert np.abs(plus - ref[t][0]).max() < 1e-15
                assert np.abs(rest - ref[t][1]).max() < 1e-15
                assert np.abs(minus - ref[t][2]).max() < 1e-15


# -------------------------------------------------------- invariants --

@pytest.fixture(scope="module")
def porous32():
    return inputs.PLAIN_32.voxels()


@pytest.mark.parametrize("sputter", ["UNIFORM", "WEIGHTED", "BOUNCEBACK", "STOCHASTIC"])
def test_closed_box_conserves_mass(orc, porous32, sputter):
    """Periodic box, porous catalytic solid, p_S^R = 0: the sputtering
    condition conserves what it re-emits, so both lattices keep their mass
    (relative drift < 1e-12 over 200 steps)."""
    o = orc.Oracle(porous32, tau=(0.8, 0.7), p=0.3, p_stick=0.0, c0=0.5,
                   force=inputs.body_force(4.0, 0.8), sputter=getattr(orc, sputter),
                   species_x=orc.XPERIODIC)
    t0 = o.totals()
    o.step(200)
    t1 = o.totals()
    assert abs(t1["mass_gas"] / t0["mass_gas"] - 1) < 1e-12
    assert abs(t1["mass_species"] / t0["mass_species"] - 1) < 1e-12
    assert t1["converted"] == 0.0 and t1["lost"] == 0.0


@pytest.mark.parametrize("sputter", ["UNIFORM", "WEIGHTED", "BOUNCEBACK", "STOCHASTIC"])
@pytest.mark.parametrize("coupling", ["PASSIVE", "BARYCENTRIC"])
def test_species_bookkeeping_per_step(orc, porous32, sputter, coupling):
    """M_R(t+1) - M_R(t) = influx - outflux - p_S^R sum_k In(k) each step, and
    the removed mass splits p : (1 - p) into converted and lost (the
    non-conservation noted after the sputtering equations)."""
    p, ps = 0.1443, 0.95
    o = orc.Oracle(porous32, tau=(0.8, 0.7), p=p, p_stick=ps, force=inputs.body_force(4.0, 0.8),
                   sputter=getattr(orc, sputter), coupling=getattr(orc, coupling))
    prev = o.totals()
    for _ in range(60):
        o.step(1)
        t = o.totals()
        removed = (t["converted"] - prev["converted"]) + (t["lost"] - prev["lost"])
        lhs = t["mass_species"] - prev["mass_species"]
        rhs = (t["influx"] - prev["influx"]) - (t["outflux"] - prev["outflux"]) - removed
        assert abs(lhs - rhs) < 1e-12 * max(t["mass_species"], 1.0)
        assert abs(t["mass_gas"] / prev["mass_gas"] - 1) < 1e-13
        prev = t
    assert t["converted"] == pytest.approx(p / (1 - p) * t["lost"], rel=1e-12)
    conv = o.conversion_map()
    assert conv.sum() == pytest.approx(t["converted"], rel=1e-12)
    assert (conv[porous32 != inputs.CATALYTIC] == 0).all()


# ----------------------------------------------------- special cases --

def test_zero_sticking_bounceback_is_plain_bounceback(orc, porous32):
    """p_S^R = 0 with reversal re-emission is halfway bounce-back, bit for bit."""
    kw = dict(tau=(0.8, 0.7), p=0.5, p_stick=0.0, force=inputs.body_force(4.0, 0.8))
    a = orc.Oracle(porous32, sputter=orc.BOUNCEBACK, **kw)
    inert = np.where(porous32 == inputs.CATALYTIC, inputs.INERT, porous32).astype(np.uint8)
    b = orc.Oracle(inert, sputter=orc.UNIFORM, **kw)
    a.step(50)
    b.step(50)
    for fa, fb in zip(a.fields(), b.fields()):
        assert np.array_equal(fa, fb)
    assert a.totals()["mass_species"] == b.totals()["mass_species"]


def test_zero_reaction_probability_converts_nothing(orc, porous32):
    o = orc.Oracle(porous32, tau=(0.8, 0.7), p=0.0, p_stick=0.95, force=inputs.body_force(4.0, 0.8))
    o.step(40)
    t = o.totals()
    assert t["converted"] == 0.0 and t["lost"] > 0.0
    assert not o.conversion_map().any()


def test_inflow_inlet_reduces_to_reservoir_when_the_carrier_rests(orc, porous32):
    """With no force the carrier stays exactly at rest, so the moving inlet
    ghost (the equilibrium of c_in at the carrier velocity) is the rest
    equilibrium w_i c_in: INFLOW and RESERVOIR give the same bits."""
    kw = dict(tau=(0.8, 0.7), p=0.2, p_stick=0.9, c_inlet=1.0, c0=0.3, force=(0.0, 0.0, 0.0))
    a = orc.Oracle(porous32, species_x=orc.XINFLOW, **kw)
    b = orc.Oracle(porous32, species_x=orc.XRESERVOIR, **kw)
    a.step(30)
    b.step(30)
    for fa, fb in zip(a.get_state(), b.get_state()):
        assert np.array_equal(fa, fb)
    assert a.totals() == b.totals()
    a.close()
    b.close()


def test_inflow_inlet_moves_with_the_carrier(orc):
    """In an open channel with flow, the inlet plane pulls exactly the
    equilibrium of c_in at its own carrier velocity (a direct check of the
    ghost values), and the species bookkeeping holds step by step with the
    influx counting what the ghost supplied."""
    ny, nx = 12, 20
    vox = np.zeros((1, ny, nx), np.uint8)
    vox[0, 0, :] = inputs.CATALYTIC
    vox[0, ny - 1, :] = inputs.INERT
    F = (2e-4, 0.0, 0.0)
    o = orc.Oracle(vox, tau=(0.8, 0.6), p=1.0, p_stick=1.0, c_inlet=1.0, force=F, species_x=orc.XINFLOW)
    o.step(400)
    prev = o.totals()
    o.step(1)
    t = o.totals()
    fC, fR = o.get_state()
    c, w, _ = orc.d3q19()
    f = fC.reshape(1, ny, nx, 19)[0, 1:ny - 1, 0]      # gas nodes of the inlet plane
    g = fR.reshape(1, ny, nx, 19)[0, 1:ny - 1, 0]
    rho = f.sum(1)
    u = (f @ c + 0.5 * np.array(F)) / rho[:, None]
    assert u[:, 0].max() > 1e-3
    cu = u @ c.T
    feq = w * (1.0 + 3.0 * cu + 4.5 * cu**2 - 1.5 * (u**2).sum(1)[:, None])
    inlet = c[:, 0] == 1
    assert np.abs(g[:, inlet] - feq[:, inlet]).max() < 1e-15
    absorbed = (t["converted"] + t["lost"]) - (prev["converted"] + prev["lost"])
    lhs = t["mass_species"] - prev["mass_species"]
    rhs = (t["influx"] - prev["influx"]) - (t["outflux"] - prev["outflux"]) - absorbed
    assert abs(lhs - rhs) < 1e-12 * t["mass_species"]
    assert t["influx"] - prev["influx"] == pytest.approx(g[:, inlet].sum(), rel=1e-13)
    o.close()


@pytest.mark.parametrize("coupling", ["PASSIVE", "BARYCENTRIC"])
def test_reactant_field_depends_on_sticking_not_reaction(orc, porous32, coupling):
    """In the reactant sputtering equation only (1 - p_S^R) multiplies the
    re-emitted reactant; p enters the product equation alone.  So runs that
    differ only in p hold the same state bit for bit, and their conversion
    maps differ by the factor p."""
    kw = dict(tau=(0.8, 0.7), p_stick=0.95, c0=0.4, force=inputs.body_force(4.0, 0.8),
              coupling=getattr(orc, coupling))
    runs = []
    for p in (0.05, 0.7):
        o = orc.Oracle(porous32, p=p, **kw)
        o.step(40)
        runs.append((p, o.get_state(), o.conversion_map(), o.totals()))
        o.close()
    (pa, (ca, ra), ma, ta), (pb, (cb, rb), mb, tb) = runs
    assert np.array_equal(ca, cb) and np.array_equal(ra, rb)
    assert ta["mass_species"] == tb["mass_species"]
    assert ma.any()
    assert np.allclose(ma / pa, mb / pb, rtol=1e-14, atol=0.0)
    absorbed_a = ta["converted"] + ta["lost"]
    assert absorbed_a == pytest.approx(tb["converted"] + tb["lost"], rel=1e-14)
    # a change of p_S^R does change the field
    o = orc.Oracle(porous32, p=pa, **dict(kw, p_stick=0.5))
    o.step(40)
    assert not np.array_equal(o.get_state()[1], ra)
    o.close()


def test_full_sticking_and_reaction_absorbs_everything(orc):
    """p_S^R = p = 1: nothing is re-emitted, all arrivals are converted."""
    n = 9
    o = orc.Oracle(inputs.reactive_slab(n), tau=(0.8, 0.8), p=1.0, p_stick=1.0, c_inlet=1.0)
    o.step(30)
    _, fR = o.get_state()
    c, _, _ = orc.d3q19()
    # populations coming back from the wall (c_x = -1 at x = n-1) are zero
    assert np.abs(fR.reshape(n + 1, 19)[n - 1, c[:, 0] == -1]).max() == 0.0
    t = o.totals()
    assert t["lost"] == 0.0 and t["converted"] > 0.0


def test_barycentric_tends_to_passive_in_dilute_limit(orc):
    """The common velocity of the moment equations reduces to the carrier
    velocity as c_in / rho_C -> 0: identical at c_in = 0, and the difference
    is linear in c_in (the reservoir feeds the mixture x-momentum c_in/6 per
    inlet node and step, which the barycentric velocity shares with the gas)."""
    vox = inputs.porous_slab(16, 12, 12, 0.7, 3.0, 5)
    diffs = []
    for cin in (1e-2, 1e-4, 0.0):
        kw = dict(tau=(0.8, 0.7), p=0.3, p_stick=0.9, c_inlet=cin, force=(2e-4, 0, 0))
        a = orc.Oracle(vox, coupling=orc.PASSIVE, **kw)
        b = orc.Oracle(vox, coupling=orc.BARYCENTRIC, **kw)
        a.step(60)
        b.step(60)
        diffs.append(np.abs(a.fields()[1] - b.fields()[1]).max())
    assert diffs[2] == 0.0
    assert diffs[0] / diffs[1] == pytest.approx(100.0, rel=0.05)


# ------------------------------------------------- geometry bookkeeping --

def test_active_link_counts_brute_force(orc):
    """b(k) per catalytic node (number of gas neighbours it receives from),
    and L_K = sum_k b(k) = #(gas node, direction) whose pull source is
    catalytic, counted from the gas side."""
    vox = inputs.porous_slab(14, 9, 7, 0.6, 2.0, 3)
    vox[2, 3, 0] = inputs.CATALYTIC            # solid touching the inlet plane
    vox[4, 4, 13] = inputs.INERT
    c, _, _ = orc.d3q19()
    nz, ny, nx = vox.shape
    o = orc.Oracle(vox, species_x=orc.XRESERVOIR)
    b = o.link_counts()
    brute = np.zeros_like(b)
    from_gas = 0
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                for i in range(1, 19):
                    sx, sy, sz = x - c[i, 0], (y - c[i, 1]) % ny, (z - c[i, 2]) % nz
                    if not 0 <= sx < nx:
                        continue
                    if vox[z, y, x] == inputs.CATALYTIC and vox[sz, sy, sx] == inputs.FLUID:
                        brute[z, y, x] += 1
                    if vox[z, y, x] == inputs.FLUID and vox[sz, sy, sx] == inputs.CATALYTIC:
                        from_gas += 1
    assert np.array_equal(b, brute)
    assert int(b.sum(dtype=np.int64)) == from_gas


def test_results_independent_of_thread_count(orc, tmp_path):
    code = (
        "import sys, hashlib; sys.path.insert(0, %r)\n"
        "import oracle\n"
        "from paper_1607_02874_amd import inputs\n"
        "w = inputs.PLAIN_32\n"
        "o = oracle.Oracle(w.voxels(), tau=w.tau, p=0.14, force=w.force())\n"
        "o.step(20)\n"
        "h = hashlib.sha256()\n"
        "[h.update(a.tobytes()) for a in o.fields()]\n"
        "h.update(o.conversion_map().tobytes())\n"
        "print(h.hexdigest())\n" % os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    out = []
    for nt in ("1", "5"):
        env = dict(os.environ, OMP_NUM_THREADS=nt)
        out.append(subprocess.run([sys.executable, "-c", code], env=env, check=True,
                                  capture_output=True, text=True).stdout.strip())
    assert out[0] == out[1]


@pytest.mark.parametrize("tau", [0.8, 1.3])
def test_steady_bulk_diffusion_is_exact_fick_law(orc, tau):
    """Steady 1-D diffusion of the reactant towards a fully absorbing wall
    (no flow): the flux carried across a link in one step, the mean of the
    pre- and post-collision first moments, (1 - 1/(2 tau)) j, equals
    -D dc/dx with D = c_s^2 (tau - 1/2) and a centred difference, exactly
    (the Appendix's diffusion of the species across the carrier, BGK with
    equal-velocity equilibrium)."""
    n = 20
    vox = inputs.reactive_slab(n, ny=2, nz=2)
    p, clamped = orc.p_from_da(1e-6, 1.0)
    assert clamped and p == 1.0
    o = orc.Oracle(vox, tau=(0.9, tau), p=p, p_stick=1.0, c_inlet=1.0, force=(0.0, 0.0, 0.0))
    o.step(30000)
    _, fR = o.get_state()
    o.close()
    c, _, _ = orc.d3q19()
    f = fR.reshape(2, 2, n + 1, 19)
    rho = f.sum(axis=3)
    j = (f * c[:, 0]).sum(axis=3)
    D = (tau - 0.5) / 3.0
    flux = (1.0 - 0.5 / tau) * j[..., 2:n - 2]
    grad = (rho[..., 3:n - 1] - rho[..., 1:n - 3]) / 2.0
    assert np.abs(flux + D * grad).max() < 1e-12 * np.abs(flux).max()
    # steady: the same flux through every plane, and a linear profile
    assert np.ptp(flux) < 1e-12 * np.abs(flux).max()
    assert np.abs(np.diff(rho[..., 1:n - 1], 2)).max() < 1e-12
