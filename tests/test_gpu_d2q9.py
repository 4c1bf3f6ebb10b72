"""Parity of the D2Q9 path (lbm_bc.lattice = LBM_LATTICE_D2Q9: the paper's
own lattice on one plane, FP64) with the oracle built for D2Q9, through the
C ABI: fields, conversion map, product fields and totals within 1e-12
(L2-relative over the gas or catalytic nodes; totals relative), over every
option the path offers, ragged plane sizes, and a catalytic voxel with all
8 links active."""

import numpy as np
import pytest

import oracle
from paper_1607_02874_amd import inputs, lbm

from parity import l2rel

pytestmark = pytest.mark.gpu

F64 = 3
SPUT = {"UNIFORM": (oracle.UNIFORM, lbm.SPUTTER_UNIFORM), "WEIGHTED": (oracle.WEIGHTED, lbm.SPUTTER_WEIGHTED),
        "BOUNCEBACK": (oracle.BOUNCEBACK, lbm.SPUTTER_BOUNCEBACK)}
XBC = {"PERIODIC": (oracle.XPERIODIC, lbm.XBC_PERIODIC), "RESERVOIR": (oracle.XRESERVOIR, lbm.XBC_RESERVOIR),
       "INFLOW": (oracle.XINFLOW, lbm.XBC_INFLOW)}
CPL = {"PASSIVE": (oracle.PASSIVE, lbm.COUPLE_PASSIVE), "BARYCENTRIC": (oracle.BARYCENTRIC, lbm.COUPLE_BARYCENTRIC)}


def plane(nx, ny, phi=0.6, ell=3.0, seed=21):
    vox = inputs.porous_slab(nx, ny, 1, phi, ell, seed)
    vox[0, ny // 2, 1] = inputs.CATALYTIC  # isolated in the inlet buffer: 8 active links
    return vox


def run_pair(vox, steps, sputter="UNIFORM", species_x="RESERVOIR", coupling="PASSIVE", product=False, sigma=0.0,
             tau=(0.9, 0.8), da=0.4, p_stick=0.7, p_stick_product=0.3, force=(3e-5, 1e-5, 0.0), c0=0.1):
    p, _ = oracle.p_from_da(da, 3.0)
    o = oracle.Oracle(vox, tau=tau, p=p, p_stick=p_stick, c_inlet=1.0, c0=c0, force=force,
                      sputter=SPUT[sputter][0], coupling=CPL[coupling][0], species_x=XBC[species_x][0],
                      product=product, p_stick_product=p_stick_product, wall_diffuse=sigma, lattice="D2Q9")
    print(f"D2Q9 {vox.shape} {steps} steps {sputter} {species_x} {coupling} product {product} sigma {sigma}",
          flush=True)
    o.step(steps)
    rho, u, conc = o.fields()
    ref = dict(rho=rho, u=u, conc=conc, conv=o.conversion_map(), totals=o.totals(), links=o.link_counts())
    if product:
        cp, tp, st = o.product()
        ref.update(cp=cp, tp=tp, stuck=st, phi=o.product_flux())
    o.close()
    with lbm.Sim(vox, da=da, tau=tau, pore_size=3.0, p_stick=p_stick, c_inlet=1.0, c0=c0, force=force,
                 sputter=SPUT[sputter][1], coupling=CPL[coupling][1], species_x=XBC[species_x][1], product=product,
                 p_stick_product=p_stick_product, wall_diffuse=sigma, storage=F64,
                 lattice=lbm.LATTICE_D2Q9) as s:
        assert s.info()["p"] == pytest.approx(p, rel=1e-15)
        s.step(steps)
        rho, u, conc = s.fields()
        got = dict(rho=rho, u=u, conc=conc, conv=s.conversion_map(), totals=s.totals(), links=s.active_links())
        if product:
            cp, st, phi = s.product_fields()
            got.update(cp=cp, tp=got["totals"], stuck=st, phi=phi)
    return got, ref


def check(got, ref, vox, bar=1e-12):
    gas, cat = vox == inputs.FLUID, vox == inputs.CATALYTIC
    assert np.array_equal(got["links"], ref["links"])
    e = {k: l2rel(got[k], ref[k], gas) for k in ("rho", "u", "conc")}
    e["conv"] = l2rel(got["conv"], ref["conv"], cat)
    if "cp" in ref:
        e["cp"] = l2rel(got["cp"], ref["cp"], gas)
        e["stuck"] = l2rel(got["stuck"], ref["stuck"], cat) if ref["stuck"].any() else 0.0
        e["phi"] = float(np.abs(got["phi"] - ref["phi"]).max() / max(np.abs(ref["phi"]).max(), 1e-300))
    scale = abs(ref["totals"]["mass_gas"])
    for k, v in ref["totals"].items():
        e["t_" + k] = abs(got["totals"][k] - v) / max(abs(v), 1e-9 * scale)
    if "tp" in ref:
        for k, v in ref["tp"].items():
            e["tp_" + k] = abs(got["tp"][k] - v) / max(abs(v), 1e-9 * scale)
    print({k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    for k, v in e.items():
        assert v < bar, (k, v)


@pytest.mark.parametrize("sputter,species_x,coupling", [
    ("UNIFORM", "RESERVOIR", "PASSIVE"), ("WEIGHTED", "PERIODIC", "BARYCENTRIC"),
    ("BOUNCEBACK", "INFLOW", "PASSIVE"), ("UNIFORM", "INFLOW", "BARYCENTRIC")])
def test_d2q9_matches_oracle(sputter, species_x, coupling):
    vox = plane(70, 48)
    check(*run_pair(vox, 150, sputter, species_x, coupling), vox)


@pytest.mark.parametrize("sputter,species_x", [("UNIFORM", "INFLOW"), ("WEIGHTED", "RESERVOIR"),
                                               ("BOUNCEBACK", "PERIODIC")])
def test_d2q9_product_lattice_matches_oracle(sputter, species_x):
    vox = inputs.disk_ingot(6, h=40, length=64, width=90, seed=4)
    check(*run_pair(vox, 200, sputter, species_x, product=True), vox)


@pytest.mark.parametrize("shape", [(37, 29), (257, 3), (5, 130)])
def test_d2q9_ragged_planes(shape):
    nx, ny = shape
    vox = inputs.porous_slab(nx, ny, 1, 0.55, 2.0, 31, x_lo=1, x_hi=max(2, nx - 1))
    check(*run_pair(vox, 80, "UNIFORM", "RESERVOIR"), vox)


@pytest.mark.parametrize("sigma", [0.5, 1.0])
def test_d2q9_diffuse_wall(sigma):
    vox = plane(60, 40, seed=22)
    check(*run_pair(vox, 120, "UNIFORM", "RESERVOIR", sigma=sigma, tau=(1.3, 0.9)), vox)


def test_d2q9_kn_wall_has_maxwell_slip():
    """The Kn-derived wall on the D2Q9 channel: the slip length is Maxwell's."""
    N, kn, F = 8, 0.05, 1e-6
    vox = inputs.channel(N, nx=1, nz=1)
    with lbm.Sim(vox, da=1.0, kn=kn, tau=(0.0, 0.7), pore_size=float(N), force=(F, 0.0, 0.0), p_stick=0.0,
                 species_x=lbm.XBC_PERIODIC, storage=F64, wall_accommodation=1.0, lattice=lbm.LATTICE_D2Q9) as s:
        nu = (s.info()["tau_gas"] - 0.5) / 3.0
        s.step(int(60 * N * N / nu) + 200)
        rho, u, _ = s.fields()
    m = (rho * u[0])[0, :N, 0]
    c2, c1, c0 = np.polyfit(np.arange(N, dtype=np.float64), m, 2)
    slip = (c2 * 0.25 - 0.5 * c1 + c0) / (-c2 + c1)
    assert slip == pytest.approx(kn * N, rel=1e-8)


def test_d2q9_unsupported_calls():
    vox = plane(20, 16)
    with lbm.Sim(vox, da=1.0, tau=(0.8, 0.7), pore_size=3.0, storage=F64, lattice=lbm.LATTICE_D2Q9) as s:
        for call in (lambda: s.set_tunable(lbm.TUNE_SWEEP, 1), lambda: s.set_timing(1), lambda: s.autotune(1),
                     lambda: s.populations(), lambda: s.fields_noalloc()):
            with pytest.raises(lbm.LbmError) as e:
                call()
            assert e.value.status == lbm.LBM_EUNSUPPORTED
        s.step(3)
        assert s.totals()["step"] == 3
    for kw in (dict(storage=0), dict(storage=F64, sputter=lbm.SPUTTER_STOCHASTIC)):
        with pytest.raises(lbm.LbmError) as e:
            lbm.Sim(vox, da=1.0, tau=(0.8, 0.7), pore_size=3.0, lattice=lbm.LATTICE_D2Q9, **kw)
        assert e.value.status == lbm.LBM_EUNSUPPORTED
    with pytest.raises(lbm.LbmError):
        lbm.Sim(np.zeros((2, 8, 8), np.uint8), da=1.0, tau=(0.8, 0.7), storage=F64, lattice=lbm.LATTICE_D2Q9)
