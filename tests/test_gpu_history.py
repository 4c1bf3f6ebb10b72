"""Parity over the stated histories of the benchmark workloads, on crops the
FP64 oracle can run in under a minute.

- 256^3 single-sample workload: the 64^3 crop (voxels [0, 64)^3 of the
  256^3 sample, outlet planes 60-63 gas) over 2000 steps at Da = 1, FP32
  against the oracle within 1e-5 per field, in the L2-relative and the
  max-abs form.  Da = 0.1 and 10 change only p, and p enters only the
  conversion (the reactant re-emission is (1 - p_S) In(k), independent of p;
  pinned in the oracle by test_reactant_field_depends_on_sticking_not_reaction):
  their GPU runs hold the Da = 1 fields bit for bit and the conversion map
  scaled by the ratio of p.
- 512^3 precision workload: a 128^3 crop of its geometry (outlet planes
  124-127 gas), 300 steps against the oracle (FP32 1e-5, 16-bit 1e-3), and
  1000 steps (the workload's stated history) against the FP64 build of the
  kernels (itself within 1e-12 of the oracle on every small case).
"""

import numpy as np
import pytest

import oracle
from paper_1607_02874_amd import inputs, lbm

from parity import errors, mean_ux

pytestmark = pytest.mark.gpu

F32, F16, BF16, F64 = 0, 1, 2, 3
NEAREST, STOCHASTIC = 0, 1


def _run_oracle(vox, w, da, steps):
    p, _ = oracle.p_from_da(da, w.pore_size)
    print(f"oracle {vox.shape} {steps} steps on {oracle.threads()} threads", flush=True)
    o = oracle.Oracle(vox, tau=w.tau, p=p, p_stick=w.p_stick, c_inlet=w.c_inlet, force=w.force())
    o.step(steps)
    rho, u, conc = o.fields()
    out = dict(rho=rho, u=u, conc=conc, conv=o.conversion_map())
    o.close()
    return out


def _run_gpu(vox, w, da, steps, storage=F32, rounding=NEAREST, store_ux=0.0):
    with lbm.Sim(vox, da=da, tau=w.tau, pore_size=w.pore_size, force=w.force(), p_stick=w.p_stick,
                 c_inlet=w.c_inlet, storage=storage, rounding=rounding, store_ux=store_ux) as s:
        s.step(steps)
        rho, u, conc = s.fields()
        return dict(rho=rho, u=u, conc=conc, conv=s.conversion_map(), p=s.info()["p"])


def _report(label, e):
    print(label, {k: f"{v:.2e}" for k, v in e.items() if isinstance(v, float)}, flush=True)


@pytest.fixture(scope="module")
def crop64():
    w = inputs.SINGLE_256
    vox = inputs.crop(w.voxels(), 64, 64, 64)
    return w, vox, _run_oracle(vox, w, w.da, w.steps)


def test_single_workload_crop_2000_steps_fp32(crop64):
    w, vox, ref = crop64
    assert w.steps == 2000
    gpu = _run_gpu(vox, w, w.da, w.steps)
    e = errors(gpu, ref, vox)
    _report("64^3 crop, 2000 steps, FP32", e)
    assert ref["conv"].sum() > 0
    for k in ("rho", "u", "conc", "conv"):
        assert e[k] < 1e-5, (k, e[k])
        assert e[k + "_max"] < 1e-5, (k + "_max", e[k + "_max"])


def test_single_workload_crop_other_damkohler_numbers(crop64):
    w, vox, ref = crop64
    base = _run_gpu(vox, w, w.da, w.steps)
    for da in (0.1, 10.0):
        g = _run_gpu(vox, w, da, w.steps)
        for k in ("rho", "u", "conc"):
            assert np.array_equal(g[k], base[k]), (da, k)
        assert np.allclose(g["conv"] / g["p"], base["conv"] / base["p"], rtol=1e-13, atol=0.0), da
        # and hence against the oracle at Da = 1, scaled by p
        e = errors(dict(g, conv=g["conv"] * base["p"] / g["p"]), ref, vox)
        assert e["conv"] < 1e-5 and e["conv_max"] < 1e-5, (da, e["conv"], e["conv_max"])


# BF16 (8 significant bits) misses the 1e-3 target on the velocity with
# either rounding; measured on this crop.
BF16_MISS = {
    NEAREST: "BF16, nearest: conc 2.3e-3, conv 2.4e-3 after 300 steps; u 8.7e-3, conc 1.2e-2 after 1000",
    STOCHASTIC: "BF16, stochastic rounding: u 1.22e-3 after 300 steps, u 1.23e-3 after 1000",
}


def _p(storage, rounding):
    marks = [pytest.mark.xfail(reason=BF16_MISS[rounding], strict=False)] if storage == BF16 else []
    return pytest.param(storage, rounding, marks=marks, id=f"s{storage}-r{rounding}")


@pytest.fixture(scope="module")
def crop128():
    w = inputs.PRECISION_512
    print("512^3 geometry", flush=True)
    vox = inputs.crop(w.voxels(), 128, 128, 128)
    ref300 = _run_oracle(vox, w, w.da, 300)
    print("FP64 build, 1000 steps", flush=True)
    ref1000 = _run_gpu(vox, w, w.da, w.steps, F64)
    return w, vox, ref300, ref1000


@pytest.mark.parametrize("storage,rounding", [_p(F32, NEAREST), _p(F16, STOCHASTIC), _p(F16, NEAREST),
                                              _p(BF16, STOCHASTIC), _p(BF16, NEAREST)])
def test_precision_workload_crop(crop128, storage, rounding):
    w, vox, ref300, ref1000 = crop128
    assert w.steps == 1000
    bar = 1e-5 if storage == F32 else 1e-3
    for steps, ref, label in ((300, ref300, "oracle"), (w.steps, ref1000, "FP64 build")):
        e = errors(_run_gpu(vox, w, w.da, steps, storage, rounding), ref, vox)
        _report(f"128^3 crop of the 512^3 geometry, {steps} steps vs {label}, storage {storage} r{rounding}", e)
        for k in ("rho", "u", "conc", "conv"):
            assert e[k] < bar, (steps, k, e[k])


# The same crop with the carrier's 16-bit storage shifted by a reference flow
# (store_ux: the FP32 path's mean x-velocity at the end of the run), after
# 300 steps against the oracle and after the workload's 1000 steps against
# the FP64 build.  Here the mean flow is slow (0.0029 at 300 steps) and still
# developing, and the shift gains little for BF16 (measured).
SHIFT_MISS = {
    (BF16, STOCHASTIC, 300): "BF16, stochastic rounding, reference flow: u 1.07e-3 after 300 steps (1.22e-3 unshifted)",
    (BF16, NEAREST, 300): "BF16, nearest, reference flow: u 4.4e-3, conc 2.4e-3 after 300 steps",
    (BF16, NEAREST, 1000): "BF16, nearest, reference flow: rounding to nearest accumulates over the history",
}


def _ps(storage, rounding, steps):
    miss = SHIFT_MISS.get((storage, rounding, steps))
    marks = [pytest.mark.xfail(reason=miss, strict=False)] if miss else []
    return pytest.param(storage, rounding, steps, marks=marks, id=f"s{storage}-r{rounding}-{steps}")


@pytest.mark.parametrize("storage,rounding,steps", [_ps(st, r, n) for n in (300, 1000)
                                                    for st, r in ((F16, NEAREST), (BF16, STOCHASTIC), (BF16, NEAREST))])
def test_precision_workload_crop_with_reference_flow(crop128, storage, rounding, steps):
    w, vox, ref300, ref1000 = crop128
    assert w.steps == 1000
    ref, label = (ref300, "oracle") if steps == 300 else (ref1000, "FP64 build")
    ux = mean_ux(_run_gpu(vox, w, w.da, steps), vox)
    assert 0.0 < ux < 0.05
    e = errors(_run_gpu(vox, w, w.da, steps, storage, rounding, ux), ref, vox)
    _report(f"128^3 crop, {steps} steps vs {label}, storage {storage} r{rounding}, store_ux {ux:.4g}", e)
    for k in ("rho", "u", "conc", "conv"):
        assert e[k] < 1e-3, (steps, k, e[k])
