"""Parity of the HIP path (called through the C ABI) with the FP64 oracle.

Bars: the FP64 build of the kernels agrees with the oracle to 1e-12 (same
arithmetic, different summation order); the FP32 path to 1e-5 L2-relative
on density, velocity and concentration over the gas nodes (the stated target
for FP32); geometry bookkeeping (link counts, node counts) bit-exact.
"""

import numpy as np
import pytest

import oracle
from paper_1607_02874_amd import inputs

from parity import NEAREST, STOCHASTIC, case, errors, make_sim, mean_ux, run_gpu, run_oracle, totals_rel

pytestmark = pytest.mark.gpu

F32, F16, BF16, F64 = 0, 1, 2, 3

PLAIN = inputs.PLAIN_32


def plain_case(steps=PLAIN.steps, **kw):
    args = dict(da=PLAIN.da, tau=PLAIN.tau, pore_size=PLAIN.pore_size, force=PLAIN.force(),
                p_stick=PLAIN.p_stick, c_inlet=PLAIN.c_inlet)
    args.update(kw)
    return case(PLAIN.voxels(), steps, **args)


@pytest.fixture(scope="module")
def plain_ref():
    c = plain_case()
    return c, run_oracle(c)


def _report(name, e, t=None):
    print(name, {k: (f"{v:.3e}" if isinstance(v, float) else v) for k, v in e.items()},
          "" if t is None else {k: f"{v:.2e}" for k, v in t.items()}, flush=True)


def test_plain_fp64_build_matches_oracle(plain_ref):
    c, ref = plain_ref
    gpu = run_gpu(c, F64)
    e, t = errors(gpu, ref, c["vox"]), totals_rel(gpu, ref)
    _report("fp64", e, t)
    for k in ("rho", "u", "conc", "conv"):
        assert e[k] < 1e-12, (k, e[k])
        assert e[k + "_max"] < 1e-11, (k, e[k + "_max"])
    assert e["rho_solid_zero"] and e["conc_solid_zero"]
    for k, v in t.items():
        assert v < 1e-11, (k, v)
    assert gpu["totals"]["step"] == c["steps"]


def test_plain_fp32_matches_oracle(plain_ref):
    c, ref = plain_ref
    gpu = run_gpu(c, F32)
    e, t = errors(gpu, ref, c["vox"]), totals_rel(gpu, ref)
    _report("fp32", e, t)
    for k in ("rho", "u", "conc", "conv"):
        assert e[k] < 1e-5, (k, e[k])
        assert e[k + "_max"] < 1e-5, (k, e[k + "_max"])
    for k, v in t.items():
        assert v < 1e-5, (k, v)


# BF16 keeps 8 significant bits: at 32^3 after 200 steps it misses the 1e-3
# target on one field with either rounding (measured).
BF16_PLAIN_MISS = {
    NEAREST: "BF16, nearest: conc 1.32e-3 (rho 8.9e-6, u 8.6e-4) after 200 steps",
    STOCHASTIC: "BF16, stochastic rounding: u 1.23e-3 (rho 1.3e-5, conc 9.0e-4) after 200 steps",
}


@pytest.mark.parametrize("storage,rounding", [
    (F16, NEAREST), (F16, STOCHASTIC),
    pytest.param(BF16, NEAREST, marks=pytest.mark.xfail(reason=BF16_PLAIN_MISS[NEAREST], strict=False)),
    pytest.param(BF16, STOCHASTIC, marks=pytest.mark.xfail(reason=BF16_PLAIN_MISS[STOCHASTIC], strict=False)),
])
def test_plain_16bit_storage_error(plain_ref, storage, rounding):
    """16-bit deviation storage with FP32 arithmetic against the FP64
    oracle: the 1e-3 target (L2-relative) on density, velocity and
    concentration after the 200 steps of the plain case."""
    c, ref = plain_ref
    gpu = run_gpu(dict(c, rounding=rounding), storage)
    e = errors(gpu, ref, c["vox"])
    _report(f"{ {F16: 'f16', BF16: 'bf16'}[storage]} rounding {rounding}", e)
    for k in ("rho", "u", "conc"):
        assert e[k] < 1e-3, (k, e[k])


# The carrier's 16-bit storage with a reference flow (store_ux): the stored
# deviations lose the part linear in the mean x-velocity, which dominates
# them in the directions along the flow, so their rounding errors shrink.
# The reference velocity is the FP32 path's own mean over the gas nodes, as
# a user would take it from an FP32 run.
# Measured: BF16 with stochastic rounding u 7.9e-4 (from 1.23e-3), conc
# 9.1e-4.  With rounding to nearest the reactant lattice, which the shift
# leaves alone, still misses.
@pytest.mark.parametrize("storage,rounding", [
    (F16, NEAREST), (F16, STOCHASTIC),
    pytest.param(BF16, NEAREST, marks=pytest.mark.xfail(
        reason="BF16, nearest: conc 1.28e-3 (the reactant is not shifted; u 6.5e-4)", strict=False)),
    (BF16, STOCHASTIC)])
def test_plain_16bit_storage_with_reference_flow(plain_ref, storage, rounding):
    c, ref = plain_ref
    ux = mean_ux(run_gpu(c, F32), c["vox"])
    assert 0.0 < ux < 0.05
    gpu = run_gpu(dict(c, rounding=rounding, store_ux=ux), storage)
    e = errors(gpu, ref, c["vox"])
    _report(f"{ {F16: 'f16', BF16: 'bf16'}[storage]} rounding {rounding}, store_ux {ux:.4g}", e)
    for k in ("rho", "u", "conc"):
        assert e[k] < 1e-3, (k, e[k])


@pytest.mark.parametrize("sputter,coupling,species_x", [
    ("UNIFORM", "PASSIVE", "RESERVOIR"),
    ("BOUNCEBACK", "BARYCENTRIC", "INFLOW"),
    ("WEIGHTED", "PASSIVE", "PERIODIC"),
])
def test_reference_flow_fp64_matches_oracle(sputter, coupling, species_x):
    """The carrier in its shifted form (a reference flow far from the flow's
    own) gives the oracle's fields to FP64 rounding: the shift is exact
    algebra, through bounce-back, both couplings and the moving inlet."""
    c = plain_case(steps=60, sputter=sputter, coupling=coupling, species_x=species_x, c0=0.2, p_stick=0.6)
    ref = run_oracle(c)
    gpu = run_gpu(dict(c, store_ux=0.05), F64)
    e, t = errors(gpu, ref, c["vox"]), totals_rel(gpu, ref)
    _report(f"reference flow 0.05, fp64, {sputter}-{coupling}-{species_x}", e, t)
    for k in ("rho", "u", "conc", "conv"):
        assert e[k] < 1e-12, (k, e[k])
    for k, v in t.items():
        assert v < 1e-11, (k, v)


def test_reference_flow_is_ignored_by_fp32():
    c = plain_case(steps=30)
    a, b = run_gpu(c, F32), run_gpu(dict(c, store_ux=0.05), F32)
    for k in ("rho", "u", "conc", "conv"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("storage", [F64, F16])
def test_reference_flow_compact_and_chunk_sweeps_agree(storage):
    from paper_1607_02874_amd import lbm

    c = dict(plain_case(steps=23, sputter="BOUNCEBACK", species_x="PERIODIC", c0=0.2), store_ux=0.02)
    out = []
    for variant in (1, 0):
        s = make_sim(c, storage)
        s.set_tunable(lbm.TUNE_SWEEP, variant)
        s.step(c["steps"])
        out.append((s.fields(), s.conversion_map()))
        s.close()
    (fa, ca), (fb, cb) = out
    assert all(np.array_equal(a, b) for a, b in zip(fa, fb))
    assert np.array_equal(ca, cb)


def test_reference_flow_checkpoint(tmp_path):
    """A 16-bit run with a reference flow resumes bit for bit from its
    checkpoint; a context with another reference flow refuses it (its
    stored deviations mean other populations)."""
    from paper_1607_02874_amd import lbm

    c = dict(plain_case(steps=30), store_ux=0.01)
    whole = make_sim(c, F16)
    whole.step(30)
    want = whole.fields()
    whole.close()
    first = make_sim(c, F16)
    first.step(12)
    first.save(tmp_path / "ck.bin")
    first.close()
    second = make_sim(c, F16)
    second.load(tmp_path / "ck.bin")
    second.step(18)
    got = second.fields()
    second.close()
    for a, b in zip(want, got):
        assert np.array_equal(a, b)
    other = make_sim(dict(c, store_ux=0.0), F16)
    with pytest.raises(lbm.LbmError) as e:
        other.load(tmp_path / "ck.bin")
    assert e.value.status == lbm.LBM_EINVAL
    other.close()


def test_geometry_bookkeeping_is_exact(plain_ref):
    c, ref = plain_ref
    s = make_sim(c, F32)
    info = s.info()
    links = s.active_links()
    s.close()
    vox = c["vox"]
    assert np.array_equal(links, ref["links"])
    assert info["n_fluid"] == int((vox == 0).sum())
    assert info["n_interface"] == int((ref["links"] > 0).sum())
    assert info["n_catalytic_links"] == int(ref["links"].sum(dtype=np.int64))
    assert info["p"] == pytest.approx(ref["p"], rel=1e-15, abs=0)
    assert info["kn"] == pytest.approx(oracle.kn_from_tau(c["tau"][0], c["pore_size"]), rel=1e-14)


@pytest.mark.parametrize("sputter,coupling,species_x", [
    ("WEIGHTED", "PASSIVE", "RESERVOIR"),
    ("BOUNCEBACK", "PASSIVE", "RESERVOIR"),
    ("UNIFORM", "BARYCENTRIC", "RESERVOIR"),
    ("UNIFORM", "PASSIVE", "PERIODIC"),
    ("WEIGHTED", "BARYCENTRIC", "PERIODIC"),
    ("UNIFORM", "PASSIVE", "INFLOW"),
    ("BOUNCEBACK", "BARYCENTRIC", "INFLOW"),
])
def test_modes_fp64_match_oracle(sputter, coupling, species_x):
    c = plain_case(steps=60, sputter=sputter, coupling=coupling, species_x=species_x, c0=0.2, p_stick=0.6)
    ref = run_oracle(c)
    gpu = run_gpu(c, F64)
    e, t = errors(gpu, ref, c["vox"]), totals_rel(gpu, ref)
    _report(f"{sputter}-{coupling}-{species_x}", e, t)
    for k in ("rho", "u", "conc", "conv"):
        assert e[k] < 1e-12, (k, e[k])
    for k, v in t.items():
        assert v < 1e-11, (k, v)


RAGGED = [
    ("nx1", (3, 4, 1)),
    ("nx63", (5, 6, 63)),
    ("nx64", (3, 5, 64)),
    ("nx65", (4, 3, 65)),
    ("nx130", (3, 4, 130)),
    ("tall", (9, 2, 7)),
]


@pytest.mark.parametrize("name,shape", RAGGED)
def test_ragged_shapes_fp64_and_fp32(name, shape):
    """Chunk edges, partial chunks and x-wrap: sizes that do not fill a
    64-wide chunk, span several chunks with a ragged tail, or are 1 wide."""
    nz, ny, nx = shape
    rng = np.random.default_rng(sum(shape))
    vox = np.where(rng.random(shape) < 0.3, 2, 0).astype(np.uint8)
    vox[rng.random(shape) < 0.1] = 1
    if nx > 2:
        vox[:, :, 0] = 0
    for species_x in ("RESERVOIR", "PERIODIC", "INFLOW"):
        c = case(vox, 25, da=0.3, tau=(0.9, 0.75), pore_size=2.0, force=(1e-4, 2e-5, -1e-5), c0=0.1,
                 p_stick=0.7, species_x=species_x)
        ref = run_oracle(c)
        g64 = run_gpu(c, F64)
        e = errors(g64, ref, vox)
        _report(f"{name}-{species_x}-f64", e)
        for k in ("rho", "u", "conc", "conv"):
            assert e[k] < 1e-12, (k, e[k])
            assert e[k + "_max"] < 1e-11, (k, e[k + "_max"])
        assert np.array_equal(g64["links"], ref["links"])
        g32 = run_gpu(c, F32)
        e = errors(g32, ref, vox)
        for k in ("rho", "u", "conc", "conv"):
            assert e[k] < 1e-5, (k, e[k])


def test_degenerate_geometries():
    """All solid (nothing to update), all gas (no interface), and a single
    gas voxel surrounded by catalyst."""
    solid = np.full((4, 4, 8), 2, np.uint8)
    c = case(solid, 5)
    g = run_gpu(c, F32)
    assert g["info"]["n_fluid"] == 0 and g["info"]["n_interface"] == 0
    assert g["totals"]["mass_gas"] == 0.0 and not g["rho"].any()
    gas = np.zeros((4, 5, 70), np.uint8)
    c = case(gas, 20, force=(1e-4, 0, 0), c0=0.3)
    ref, g = run_oracle(c), run_gpu(c, F64)
    e = errors(g, ref, gas)
    for k in ("rho", "u", "conc"):
        assert e[k] < 1e-12
    one = np.full((3, 3, 3), 2, np.uint8)
    one[1, 1, 1] = 0
    c = case(one, 10, c0=0.5, p_stick=0.3, species_x="PERIODIC")
    ref, g = run_oracle(c), run_gpu(c, F64)
    e = errors(g, ref, one)
    for k in ("rho", "conc", "conv"):
        assert e[k] < 1e-12, (k, e[k])


def test_step_zero_fields_and_totals():
    c = plain_case(steps=0, c0=0.25)
    ref, g = run_oracle(c), run_gpu(c, F64)
    e = errors(g, ref, c["vox"])
    for k in ("rho", "u", "conc"):
        assert e[k] < 1e-14, (k, e[k])
    assert g["totals"]["mass_gas"] == pytest.approx(ref["totals"]["mass_gas"], rel=1e-14)


@pytest.mark.parametrize("storage", [F64, F32])
def test_poiseuille_closed_form_on_gpu(storage):
    """Discrete Poiseuille profile rho u(y) = F/(2 nu) (h^2 - z^2) + F (6 nu -
    1/(8 nu)) reached by the kernels themselves."""
    n, tau, F = 32, 0.8, 1e-5
    vox = inputs.channel(n, nx=3, nz=2)
    c = case(vox, 30000, da=float("inf"), tau=(tau, tau), force=(F, 0, 0), p_stick=0.0, species_x="PERIODIC")
    g = run_gpu(c, storage)
    nu = (tau - 0.5) / 3
    z = np.arange(n) - (n - 1) / 2
    exact = F / (2 * nu) * ((n / 2) ** 2 - z * z) + F * (6 * nu - 1 / (8 * nu))
    ru = (g["rho"] * g["u"][0])[:, :n, :]
    err = np.abs(ru - exact[None, :, None]).max() / np.abs(exact).max()
    print("poiseuille", storage, err)
    # FP32 bound, from the rounding of the steady state: every step the FP32
    # collision makes the same rounding errors at a node, which act on the
    # flow as a fixed body force q per node.  |q| <= k u_r sum_i w_i |c_ix|
    # max |h_i| with u_r = 2^-24, k = 3 roundings per stored value,
    # sum w |c_x| = 1/3 and max |h_i| ~ 3 u_max = 0.039, so |q| <= 2.3e-9; the
    # channel answers a uniform force q with a Poiseuille profile q h^2/(2 nu),
    # so the relative error is at most |q| / F = 2.3e-4.  Measured 4.0e-5 (the
    # roundings partly cancel); the bound 5e-5 sits between.
    assert err < (1e-10 if storage == F64 else 5e-5)


@pytest.mark.parametrize("storage", [F64, F32])
@pytest.mark.parametrize("sputter", ["UNIFORM", "WEIGHTED"])
def test_reactive_slab_closed_form_on_gpu(storage, sputter):
    n, tau, ps, cin = 12, 0.7, 0.6, 1.0
    c = case(inputs.reactive_slab(n, ny=2, nz=3), 40000, da=0.5, tau=(0.8, tau), p_stick=ps, c_inlet=cin,
             sputter=sputter)
    g = run_gpu(c, storage)
    x = np.arange(n)
    exact = cin * (1 - ps * (x + tau) / (n * ps + 2 * tau - 1))
    err = np.abs(g["conc"][:, :, :n] - exact).max()
    print("slab", storage, sputter, err)
    # FP32 bound as for the channel: a fixed mass source per node |q| <= k u_r
    # max |h| = 1.8e-7 (c ~ 1, k = 3) in a diffusion problem of length n with
    # D = (tau - 1/2)/3 gives |dc| <= q n^2 / (2 D) = 1.9e-4; measured 1.0e-5
    # (UNIFORM) and 8.2e-6 (WEIGHTED).
    assert err < (1e-10 if storage == F64 else 5e-5)


@pytest.mark.parametrize("storage", [F32, F16])
def test_reaction_probability_only_scales_conversion(storage):
    """Only (1 - p_S^R) multiplies the re-emitted reactant, so two runs that
    differ only in Da (hence p) hold bit-identical fields, and their
    conversion maps differ by the factor p."""
    runs = [run_gpu(plain_case(steps=50, da=da, c0=0.4), storage) for da in (10.0, 0.1)]
    (a, b) = runs
    for k in ("rho", "u", "conc"):
        assert np.array_equal(a[k], b[k]), k
    pa, pb = a["info"]["p"], b["info"]["p"]
    assert pa < 0.05 and pb > 0.5
    assert a["conv"].any()
    assert np.allclose(a["conv"] / pa, b["conv"] / pb, rtol=1e-14, atol=0.0)
    ta, tb = a["totals"], b["totals"]
    assert ta["mass_species"] == tb["mass_species"]
    assert ta["converted"] + ta["lost"] == pytest.approx(tb["converted"] + tb["lost"], rel=1e-13)


def test_totals_do_not_depend_on_how_steps_are_split():
    """The reductions of a step run in the launches of the next two steps of
    the same lbm_step call, and a call closes its own: the totals after 7
    steps are the same in one call or in three."""
    c = plain_case(steps=7)
    a, b = make_sim(c, F32), make_sim(c, F32)
    a.step(7)
    for n in (3, 1, 3):
        b.step(n)
    assert a.totals() == b.totals()
    assert all(np.array_equal(x, y) for x, y in zip(a.fields(), b.fields()))
    a.close()
    b.close()


def test_timing_levels():
    from paper_1607_02874_amd import lbm

    s = make_sim(plain_case(steps=5), F32)
    s.set_timing(2)  # the sweep only
    s.step(5)
    kt = s.kernel_times()
    assert kt["n_sweep"] == 5 and kt["ms_sweep"] > 0
    assert kt["n_interface"] == kt["n_reduce"] == 0 and kt["ms_interface"] == kt["ms_reduce"] == 0.0
    s.set_timing(1)  # every launch; the closing reductions once per call
    s.step(3)
    s.step(2)
    kt = s.kernel_times()
    assert kt["n_sweep"] == kt["n_interface"] == 5 and kt["n_reduce"] == 2
    with pytest.raises(lbm.LbmError) as e:
        s.set_timing(3)
    assert e.value.status == lbm.LBM_EINVAL
    s.close()


def test_runs_are_bit_identical():
    c = plain_case(steps=50)
    a, b = run_gpu(c, F32), run_gpu(c, F32)
    for k in ("rho", "u", "conc", "conv"):
        assert np.array_equal(a[k], b[k])
    assert a["totals"] == b["totals"]


def test_checkpoint_resume_is_bit_identical(tmp_path):
    c = plain_case(steps=40)
    whole = make_sim(c, F32)
    whole.step(40)
    want = whole.fields(), whole.conversion_map(), whole.totals()
    whole.close()
    first = make_sim(c, F32)
    first.step(15)
    first.save(tmp_path / "ck.bin")
    first.close()
    second = make_sim(c, F32)
    second.load(tmp_path / "ck.bin")
    second.step(25)
    got = second.fields(), second.conversion_map(), second.totals()
    second.close()
    for a, b in zip(want[0], got[0]):
        assert np.array_equal(a, b)
    assert np.array_equal(want[1], got[1])
    assert want[2] == got[2]


def test_checkpoint_rejects_other_geometry(tmp_path):
    from paper_1607_02874_amd import lbm

    c = plain_case(steps=3)
    s = make_sim(c, F32)
    s.step(3)
    s.save(tmp_path / "a.bin")
    s.close()
    other = plain_case(steps=3)
    other["vox"] = other["vox"].copy()
    other["vox"][5, 5, 10] = 0 if other["vox"][5, 5, 10] else 2
    t = make_sim(other, F32)
    with pytest.raises(lbm.LbmError) as e:
        t.load(tmp_path / "a.bin")
    assert e.value.status == lbm.LBM_EINVAL
    t.close()


def test_nonfinite_watchdog():
    """A violently unstable run (tau near 1/2, large force) overflows; the
    FP64 totals see it and the API reports LBM_ENONFINITE."""
    from paper_1607_02874_amd import lbm

    vox = inputs.porous_slab(16, 8, 8, 0.7, 2.0, 3)
    c = case(vox, 1, tau=(0.5001, 0.5001), force=(0.9, 0.5, 0.0), pore_size=2.0)
    s = make_sim(c, F32)
    with pytest.raises(lbm.LbmError) as e:
        for _ in range(400):
            s.step(10)
            s.synchronize()
    assert e.value.status == lbm.LBM_ENONFINITE
    t = lbm.lbm_totals_t()
    assert lbm.library().lbm_totals(s.handle, t) == lbm.LBM_ENONFINITE and t.nonfinite == 1
    s.close()


def test_fields_device_matches_host_fields():
    import torch

    c = plain_case(steps=20)
    s = make_sim(c, F32)
    s.step(20)
    rho, u, conc = s.fields()
    n = rho.size
    d_rho = torch.empty(n, device="cuda", dtype=torch.float32)
    d_u = torch.empty(3 * n, device="cuda", dtype=torch.float32)
    d_c = torch.empty(n, device="cuda", dtype=torch.float32)
    s.fields_device(d_rho, d_u, d_c)
    torch.cuda.synchronize()
    assert np.array_equal(d_rho.cpu().numpy(), rho.ravel().astype(np.float32))
    assert np.array_equal(d_u.cpu().numpy(), u.ravel().astype(np.float32))
    assert np.array_equal(d_c.cpu().numpy(), conc.ravel().astype(np.float32))
    s.close()


SHAPES_SWEEP = {
    "plain32": lambda: PLAIN.voxels(),
    "nx1": lambda: np.zeros((7, 9, 1), np.uint8),
    "nx65_tall": lambda: inputs.porous_slab(65, 40, 6, 0.6, 3.0, 21),
    "nx130": lambda: inputs.porous_slab(130, 11, 9, 0.65, 3.0, 22),
    "nx63": lambda: inputs.porous_slab(63, 14, 12, 0.55, 2.5, 23),
}


@pytest.mark.parametrize("shape", sorted(SHAPES_SWEEP))
@pytest.mark.parametrize("sputter,coupling,species_x", [("UNIFORM", "PASSIVE", "RESERVOIR"),
                                                        ("WEIGHTED", "BARYCENTRIC", "PERIODIC"),
                                                        ("BOUNCEBACK", "PASSIVE", "PERIODIC"),
                                                        ("UNIFORM", "BARYCENTRIC", "RESERVOIR"),
                                                        ("WEIGHTED", "PASSIVE", "INFLOW")])
def test_compact_and_chunk_sweeps_agree(shape, sputter, coupling, species_x):
    """The node-compact sweep (default) and the 64-voxel-chunk sweep compute
    the same populations: fields and conversion map bit-identical, totals to
    the rounding of their differently grouped partial sums."""
    from paper_1607_02874_amd import lbm

    vox = SHAPES_SWEEP[shape]()
    c = case(vox, 23, da=0.5, tau=(0.8, 0.7), pore_size=3.0, force=(2e-5, 1e-6, 0.0), p_stick=0.8, c0=0.2,
             sputter=sputter, coupling=coupling, species_x=species_x)
    out = []
    for variant in (1, 0):
        s = make_sim(c, F32)
        assert s.get_tunable(lbm.TUNE_SWEEP) == 1
        s.set_tunable(lbm.TUNE_SWEEP, variant)
        s.step(c["steps"])
        out.append((s.fields(), s.conversion_map(), s.totals()))
        s.close()
    (fa, ca, ta), (fb, cb, tb) = out
    assert all(np.array_equal(a, b) for a, b in zip(fa, fb)), shape
    assert np.array_equal(ca, cb)
    for k in ("mass_gas", "mass_species", "converted", "lost", "influx", "outflux"):
        assert abs(ta[k] - tb[k]) <= 1e-12 * max(abs(tb[k]), abs(tb["mass_gas"])), (k, ta[k], tb[k])


def test_autotune_leaves_state_unchanged():
    """Autotuning mid-run picks a launch shape without touching the state:
    the run continues exactly as a run that used the chosen shape throughout
    (fields and conversion map bit-identical, totals to partial-sum rounding)."""
    from paper_1607_02874_amd import lbm

    c = plain_case(steps=10, sputter="UNIFORM")
    a = make_sim(c, F32)
    a.step(10)
    ms = a.autotune(reps=2)
    assert ms > 0
    variant, ytile = a.get_tunable(lbm.TUNE_SWEEP), a.get_tunable(lbm.TUNE_YTILE)
    emission = a.get_tunable(lbm.TUNE_EMISSION)
    a.step(10)
    b = make_sim(c, F32)
    b.set_tunable(lbm.TUNE_SWEEP, variant)
    b.set_tunable(lbm.TUNE_YTILE, ytile)
    b.set_tunable(lbm.TUNE_EMISSION, emission)
    b.step(20)
    fa, fb = a.fields(), b.fields()
    assert all(np.array_equal(x, y) for x, y in zip(fa, fb))
    assert np.array_equal(a.conversion_map(), b.conversion_map())
    ta, tb = a.totals(), b.totals()
    assert ta["step"] == tb["step"] == 20
    for k in ("mass_gas", "mass_species", "converted", "lost", "influx", "outflux"):
        assert abs(ta[k] - tb[k]) <= 1e-12 * max(abs(tb[k]), abs(tb["mass_gas"])), k
    a.close()
    b.close()


@pytest.mark.parametrize("storage,sputter,species_x", [(F32, "UNIFORM", "RESERVOIR"), (F32, "WEIGHTED", "INFLOW"),
                                                       (F64, "UNIFORM", "PERIODIC"), (F64, "WEIGHTED", "RESERVOIR")])
def test_emission_read_modes_are_bit_identical(storage, sputter, species_x):
    """LBM_TUNE_EMISSION: the compact sweep's emission reads gathered through
    LDS (1, a context's default) and read once per direction (0) give the same
    state bit for bit.  The 32^3 sample's wavefronts take the gather; the
    random geometry (30 % catalytic voxels, about 300 sources per wavefront)
    takes the direct fallback; the last wavefront of each has idle lanes."""
    from paper_1607_02874_amd import lbm

    rng = np.random.default_rng(5)
    ragged = np.where(rng.random((5, 6, 70)) < 0.3, 2, 0).astype(np.uint8)
    ragged[:, :, 0] = 0
    for vox in (PLAIN.voxels(), ragged):
        c = case(vox, 15, da=0.5, tau=(0.8, 0.7), pore_size=3.0, force=(2e-5, 1e-6, 0.0), p_stick=0.8, c0=0.2,
                 sputter=sputter, species_x=species_x)
        runs = []
        for mode in (1, 0):
            print(f"emission mode {mode} storage {storage} {sputter} {species_x} {vox.shape}", flush=True)
            s = make_sim(c, storage)
            assert s.get_tunable(lbm.TUNE_EMISSION) == 1
            s.set_tunable(lbm.TUNE_EMISSION, mode)
            assert s.get_tunable(lbm.TUNE_EMISSION) == mode
            s.step(15)
            runs.append((s.fields(), s.conversion_map(), s.totals()))
            if mode == 0:
                with pytest.raises(lbm.LbmError) as e:
                    s.set_tunable(lbm.TUNE_EMISSION, 2)
                assert e.value.status == lbm.LBM_EINVAL
            s.close()
        (fa, ca, ta), (fb, cb, tb) = runs
        assert all(np.array_equal(x, y) for x, y in zip(fa, fb))
        assert np.array_equal(ca, cb)
        assert ta == tb


@pytest.mark.parametrize("c_inlet,c0", [(1000.0, 200.0), (1e-6, 0.0), (0.0, 0.0)])
def test_fixed_point_in_sums_across_concentration_scales(c_inlet, c0):
    """The In(k) sums are fixed point with a scale taken from the
    concentration scale: the FP64 build still meets 1e-12 against the oracle
    for large, tiny and zero concentrations."""
    c = plain_case(steps=60, c_inlet=c_inlet, c0=c0)
    ref = run_oracle(c)
    gpu = run_gpu(c, F64)
    e = errors(gpu, ref, c["vox"])
    _report(f"fixed point c_in={c_inlet}", e)
    if c_inlet == 0.0 and c0 == 0.0:
        assert np.abs(gpu["conc"]).max() == 0.0 and np.abs(gpu["conv"]).max() == 0.0
        return
    for k in ("rho", "u", "conc", "conv"):
        assert e[k] < 1e-12, (k, e[k])
