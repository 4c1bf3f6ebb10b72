"""Batched stepping (lbm_batch_*): every sample of a batch must evolve exactly
as the same sample alone.  The batched kernels run the single-sample code and
partial-sum layout per sample, so fields, conversion map and totals are
compared bit for bit; one sample is also checked against the FP64 oracle.
Graph replays are compared with eager stepping after every replay."""

import numpy as np
import pytest

from paper_1607_02874_amd import inputs, lbm

from parity import case, errors, run_oracle

pytestmark = pytest.mark.gpu

F32, F16, BF16, F64 = 0, 1, 2, 3


def mixed_samples(storage=F32, sputter=lbm.SPUTTER_UNIFORM, coupling=lbm.COUPLE_PASSIVE,
                  species_x=lbm.XBC_RESERVOIR):
    """Five samples of different shapes (ragged nx across 64-voxel chunks),
    porosities, relaxation times, Da, forces and sticking probabilities; one
    has no catalytic voxel at all."""
    specs = [
        (40, 20, 12, 0.65, 3.0, 11, (0.8, 0.7), 1.0, 0.95),
        (70, 18, 10, 0.60, 4.0, 12, (0.9, 0.9), 0.3, 0.5),
        (130, 12, 9, 0.70, 3.0, 13, (0.6, 0.75), 20.0, 0.95),
        (33, 33, 7, 0.55, 2.5, 14, (1.1, 0.65), 0.05, 0.8),
        (64, 10, 10, 1.00, 3.0, 15, (0.7, 0.7), 1.0, 0.95),
    ]
    out = []
    for nx, ny, nz, phi, ell, seed, tau, da, ps in specs:
        vox = inputs.porous_slab(nx, ny, nz, phi, ell, seed) if phi < 1.0 else np.zeros((nz, ny, nx), np.uint8)
        out.append(dict(vox=vox, da=da, tau=tau, pore_size=ell, force=inputs.body_force(ell, tau[0]), p_stick=ps,
                        c_inlet=1.0, storage=storage, sputter=sputter, coupling=coupling, species_x=species_x))
    return out


def single(smp, steps):
    kw = {k: v for k, v in smp.items() if k not in ("vox", "da", "tau", "pore_size")}
    with lbm.Sim(smp["vox"], da=smp["da"], tau=smp["tau"], pore_size=smp["pore_size"], **kw) as s:
        s.step(steps)
        return s.fields(), s.conversion_map(), s.totals()


def assert_same(batch, i, ref):
    (rho, u, c), conv, tot = ref
    brho, bu, bc = batch.fields(i)
    assert np.array_equal(brho, rho) and np.array_equal(bu, u) and np.array_equal(bc, c), i
    assert np.array_equal(batch.conversion_map(i), conv), i
    assert batch.totals(i) == tot, (i, batch.totals(i), tot)


@pytest.mark.parametrize("storage,sputter", [(F32, lbm.SPUTTER_UNIFORM), (F32, lbm.SPUTTER_WEIGHTED),
                                             (F32, lbm.SPUTTER_BOUNCEBACK), (F16, lbm.SPUTTER_UNIFORM),
                                             (F64, lbm.SPUTTER_UNIFORM)])
def test_batch_bit_identical_to_single_samples(storage, sputter):
    samples = mixed_samples(storage=storage, sputter=sputter)
    steps = 23
    print(f"batch storage={storage} sputter={sputter}", flush=True)
    with lbm.Batch(samples) as b:
        b.step(10)
        b.step(steps - 10)
        for i, smp in enumerate(samples):
            assert_same(b, i, single(smp, steps))
            assert b.totals(i)["step"] == steps


def test_batch_reference_flow_per_sample():
    """16-bit samples with different reference flows (lbm_bc.store_ux) in
    one batch step exactly as they do alone."""
    samples = mixed_samples(storage=BF16)
    for smp, ux in zip(samples, (0.0, 0.01, 0.02, -0.005, 0.004)):
        smp["store_ux"] = ux
    with lbm.Batch(samples) as b:
        b.step(17)
        for i, smp in enumerate(samples):
            assert_same(b, i, single(smp, 17))


def test_batch_emission_modes_agree_and_graphs_follow():
    """LBM_TUNE_EMISSION on a batch (default 0, direct reads): with the
    emission gather the batch gives the same bits, and a change after graphs
    were captured discards them, so the replays use the new launch."""
    samples = mixed_samples()
    with lbm.Batch(samples) as a, lbm.Batch(samples, graph=True) as b:
        assert a.get_tunable(lbm.TUNE_EMISSION) == 0
        b.step(4)  # captures the step graphs with direct reads
        b.set_tunable(lbm.TUNE_EMISSION, 1)
        assert b.get_tunable(lbm.TUNE_EMISSION) == 1
        with pytest.raises(lbm.LbmError) as e:
            b.set_tunable(lbm.TUNE_EMISSION, -1)
        assert e.value.status == lbm.LBM_EINVAL
        b.step(8)
        a.step(12)
        for i in range(len(samples)):
            assert_same(b, i, (a.fields(i), a.conversion_map(i), a.totals(i)))


def test_batch_barycentric_periodic_matches_single():
    samples = mixed_samples(coupling=lbm.COUPLE_BARYCENTRIC, species_x=lbm.XBC_PERIODIC)
    for s in samples:
        s["c0"] = 0.3
    with lbm.Batch(samples) as b:
        b.step(17)
        for i, smp in enumerate(samples):
            assert_same(b, i, single(smp, 17))


@pytest.mark.parametrize("variant", [1, 0])
def test_batch_inflow_matches_single(variant):
    """The moving-inlet boundary (INFLOW) in a batch, both sweep variants:
    every sample bit-identical to the same sample alone."""
    samples = mixed_samples(species_x=lbm.XBC_INFLOW)
    with lbm.Batch(samples) as b:
        b.set_tunable(lbm.TUNE_SWEEP, variant)
        b.set_tunable(lbm.TUNE_YTILE, 4)
        b.step(13)
        for i, smp in enumerate(samples):
            kw = {k: v for k, v in smp.items() if k not in ("vox", "da", "tau", "pore_size")}
            with lbm.Sim(smp["vox"], da=smp["da"], tau=smp["tau"], pore_size=smp["pore_size"], **kw) as s:
                s.set_tunable(lbm.TUNE_SWEEP, variant)
                s.set_tunable(lbm.TUNE_YTILE, min(4, smp["vox"].shape[1]))
                s.step(13)
                assert_same(b, i, (s.fields(), s.conversion_map(), s.totals()))


def test_batch_graph_replays_match_eager():
    samples = mixed_samples()
    with lbm.Batch(samples) as eager, lbm.Batch(samples, graph=True) as graphed:
        for rep in range(4):
            n = 2 if rep < 3 else 3  # three two-step replays, then a replay plus one eager step
            print(f"graph replay {rep} ({n} steps)", flush=True)
            graphed.step(n)
            eager.step(n)
            graphed.synchronize()
            eager.synchronize()
            for i in range(len(samples)):
                assert graphed.totals(i) == eager.totals(i), (rep, i)
                ge, ee = graphed.fields(i), eager.fields(i)
                assert all(np.array_equal(a, b) for a, b in zip(ge, ee)), (rep, i)
                assert np.array_equal(graphed.conversion_map(i), eager.conversion_map(i)), (rep, i)


def test_batch_sweep_timing_counts_every_sweep_and_leaves_results_unchanged():
    """lbm_batch_set_timing(2) brackets each batched sweep with events: the
    kernel times count every timed step (graphs are bypassed while it is on),
    the results equal untimed graphed stepping, and disabling it resumes the
    graph path."""
    samples = mixed_samples()[:3]
    with lbm.Batch(samples, graph=True) as timed, lbm.Batch(samples, graph=True) as plain:
        timed.set_timing(True)
        timed.step(5)
        plain.step(5)
        kt = timed.kernel_times()
        assert kt["n_sweep"] == 5 and kt["ms_sweep"] > 0.0, kt
        timed.set_timing(False)
        timed.step(4)
        plain.step(4)
        assert timed.kernel_times()["n_sweep"] == 5  # no events after disabling
        timed.synchronize()
        plain.synchronize()
        for i in range(len(samples)):
            assert timed.totals(i) == plain.totals(i), i
            assert all(np.array_equal(a, b) for a, b in zip(timed.fields(i), plain.fields(i))), i
        with pytest.raises(lbm.LbmError):  # per-launch timing of every kernel is not offered for batches
            lbm._bcheck(lbm._LIB.lbm_batch_set_timing(timed._h, 1), timed._h)


def test_batch_long_graph_replays_match_eager():
    """Runs of 64 steps and more replay the captured 64-step loop (then pairs
    and one eager step for the rest); after every replay, with eager work and
    synchronisations in between, the graphed batch equals eager stepping."""
    samples = mixed_samples()[:3]
    with lbm.Batch(samples) as eager, lbm.Batch(samples, graph=True) as graphed:
        for rep, n in enumerate((64, 64 + 2 + 1, 128, 64)):
            print(f"long graph replay {rep} ({n} steps)", flush=True)
            graphed.step(n)
            eager.step(n)
            graphed.synchronize()
            eager.synchronize()
            for i in range(len(samples)):
                assert graphed.totals(i) == eager.totals(i), (rep, i)
                ge, ee = graphed.fields(i), eager.fields(i)
                assert all(np.array_equal(a, b) for a, b in zip(ge, ee)), (rep, i)
                assert np.array_equal(graphed.conversion_map(i), eager.conversion_map(i)), (rep, i)


def test_batch64_smallest_samples_match_oracle():
    """The 64-sample batch workload (sides U{48..128}, porosity U[0.5, 0.75],
    tau U[0.55, 1.2], Da log-uniform in [0.01, 100]) stepped as one batch for
    its 1000 steps (graph replays); the 8 smallest samples, at full size,
    against the FP64 oracle within the FP32 target 1e-5."""
    from parity import run_oracle as _run_oracle

    ws = inputs.batch_samples(64, 2000)
    samples = [dict(vox=w.voxels(), da=w.da, tau=w.tau, pore_size=w.pore_size, force=w.force(), p_stick=w.p_stick,
                    c_inlet=w.c_inlet) for w in ws]
    steps = ws[0].steps
    assert steps == 1000
    smallest = sorted(range(len(ws)), key=lambda i: (ws[i].nx, i))[:8]
    print("batch64: stepping", steps, "steps; checking samples", smallest, flush=True)
    with lbm.Batch(samples, graph=True) as b:
        b.step(steps)
        b.synchronize()
        got = {i: (b.fields(i), b.conversion_map(i)) for i in smallest}
    for i in smallest:
        smp = samples[i]
        c = case(smp["vox"], steps, da=smp["da"], tau=smp["tau"], pore_size=smp["pore_size"],
                 p_stick=smp["p_stick"], force=smp["force"])
        ref = _run_oracle(c)
        (rho, u, conc), conv = got[i]
        e = errors(dict(rho=rho, u=u, conc=conc, conv=conv), ref, c["vox"])
        print(f"batch sample {i} side {ws[i].nx} tau {ws[i].tau[0]:.3f} Da {ws[i].da:.3g} vs oracle",
              {k: f"{v:.2e}" for k, v in e.items() if isinstance(v, float)}, flush=True)
        for k in ("rho", "u", "conc", "conv"):
            assert e[k] < 1e-5, (i, k, e[k])


def test_batch_sample_matches_oracle():
    samples = mixed_samples()
    smp = samples[0]
    steps = 40
    c = case(smp["vox"], steps, da=smp["da"], tau=smp["tau"], pore_size=smp["pore_size"], p_stick=smp["p_stick"],
             force=smp["force"])
    ref = run_oracle(c)
    with lbm.Batch(samples) as b:
        b.step(steps)
        rho, u, conc = b.fields(0)
        gpu = dict(rho=rho, u=u, conc=conc, conv=b.conversion_map(0))
    e = errors(gpu, ref, c["vox"])
    print("batch sample 0 vs oracle", {k: f"{v:.2e}" for k, v in e.items() if isinstance(v, float)}, flush=True)
    for k in ("rho", "u", "conc", "conv"):
        assert e[k] < 1e-5, (k, e[k])


def test_batch_info_and_index_errors():
    samples = mixed_samples()
    with lbm.Batch(samples) as b:
        for i, smp in enumerate(samples):
            inf = b.info(i)
            assert inf["n_nodes"] == smp["vox"].size
            assert inf["n_fluid"] == int((smp["vox"] == 0).sum())
            assert inf["tau_gas"] == smp["tau"][0]
        assert b.info(4)["n_interface"] == 0
        L = lbm.library()
        for bad in (-1, len(samples)):
            assert L.lbm_batch_fields(b._h, bad, None, None, None) == lbm.LBM_EINVAL
            assert L.lbm_batch_conversion_map(b._h, bad, None) == lbm.LBM_EINVAL
        assert b"out of range" in L.lbm_batch_last_error(b._h)
        with pytest.raises(lbm.LbmError):
            b.step(-1)


def test_batch_chunk_sweep_variant_matches_single():
    samples = mixed_samples()
    with lbm.Batch(samples) as b:
        assert b.get_tunable(lbm.TUNE_SWEEP) == 1
        b.set_tunable(lbm.TUNE_SWEEP, 0)
        b.set_tunable(lbm.TUNE_YTILE, 4)
        b.step(11)
        for i, smp in enumerate(samples):
            kw = {k: v for k, v in smp.items() if k not in ("vox", "da", "tau", "pore_size")}
            with lbm.Sim(smp["vox"], da=smp["da"], tau=smp["tau"], pore_size=smp["pore_size"], **kw) as s:
                s.set_tunable(lbm.TUNE_SWEEP, 0)
                s.set_tunable(lbm.TUNE_YTILE, min(4, smp["vox"].shape[1]))
                s.step(11)
                assert_same(b, i, (s.fields(), s.conversion_map(), s.totals()))


def test_batch_autotune_leaves_state_unchanged():
    samples = mixed_samples()
    with lbm.Batch(samples) as a, lbm.Batch(samples) as b:
        a.step(9)
        assert a.autotune(reps=2) > 0
        b.set_tunable(lbm.TUNE_SWEEP, a.get_tunable(lbm.TUNE_SWEEP))
        b.set_tunable(lbm.TUNE_YTILE, a.get_tunable(lbm.TUNE_YTILE))
        b.set_tunable(lbm.TUNE_EMISSION, a.get_tunable(lbm.TUNE_EMISSION))
        a.step(8)
        b.step(17)
        for i in range(len(samples)):
            fa, fb = a.fields(i), b.fields(i)
            assert all(np.array_equal(x, y) for x, y in zip(fa, fb)), i
            assert np.array_equal(a.conversion_map(i), b.conversion_map(i)), i
