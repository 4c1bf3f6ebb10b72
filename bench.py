"""Benchmark of the reactive two-lattice LBM hot path on one MI355X.

Workload: 256^3 porous membrane (Gaussian random field, porosity 0.60,
correlation length 8, seed 1001) with 4-voxel gas buffers in x, periodic y/z;
D3Q19 carrier (tau 0.8, body force) + D3Q19 reactant (tau 0.7, reservoir
inlet c = 1), sputtering boundary at every gas-catalyst link (UNIFORM,
p_S^R = 0.95, Da = 1 with delta = 8), FP32 storage and arithmetic.

One step = one interface gather + boundary-flux tally + fused stream-collide
sweep of both lattices + FP64 reduction.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--storage f32|f16|bf16|f64]
    python bench.py --workload batch [--steps K]   (64-sample batch vs sequential)
    python bench.py --workload precision [--steps K]   (512^3, FP32/FP16/BF16 vs the FP64 build)
    python bench.py --workload membrane [--steps K]    (1024x512x512 layer, Da 10 and 0.1, FP32 and FP16)
    python bench.py --workload shard [--steps K]       (one 128x512x512 x-slab of the membrane)
    python bench.py --workload product [--steps K]     (256^3 with the product lattice P)
    python bench.py --workload reactor2d               (the paper's 2-D reactor: efficiency vs p and w/h)
    python bench.py --workload stochastic [--steps K]  (256^3 with the random sputtering matrix)
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
STORAGES = {"f32": 0, "f16": 1, "bf16": 2, "f64": 3}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(info, s, product=False, stochastic=False):
    """Bytes the method must move per step (per launch for each kernel).

    Sweep: every population of both lattices written once (38 s per gas node)
    and read once (38 s), except the L_K reactant populations whose source is
    a catalytic node, which come from the emission array (s bytes per
    interface node); plus the 8-byte In(k) sum per interface node and the
    32-byte chunk record per 64 voxels.  Interface: per interface node, In(k)
    read and clear (16), mask and scale (4 + 8), the FP64 accumulator
    read-modify-write (16) and the emission write (s).

    With the product lattice the sweep also reads and writes every product
    population once (38 s per gas node, less the L_K that come from E_P),
    reads E_P and adds In_P (s + 8 per interface node); the interface also
    reads and clears In_P (16), updates Acc_P (16) and writes E_P (s)."""
    nf, n, nk, lk = info["n_fluid"], info["n_nodes"], info["n_interface"], info["n_catalytic_links"]
    sweep = (76 * nf - lk) * s + (8 + s) * nk + n // 2
    iface = nk * (16 + 4 + 8 + 16 + s)
    if product:
        sweep += (38 * nf - lk) * s + (8 + s) * nk
        iface += nk * (16 + 16 + s)
    if stochastic:
        # one In sum and one emission value per exit slot (L_K of them)
        # instead of one per interface node
        sweep += (lk - nk) * (8 + s)
        iface = nk * (4 + 16) + lk * (16 + s)
    return {"sweep": sweep, "interface": iface, "step": sweep + iface}


def measured_traffic(kernel, workload, storage_name, sweep, ytile, emission):
    """Calibrated HBM bytes per launch from the PMC records in
    profiles/traffic.json, or None when no record matches this kernel,
    workload, storage and launch shape (sweep variant, y-tile, emission read
    mode), or the kernel source has changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            recs = json.load(f).get(kernel, [])
        for rec in recs:
            if (rec["workload"], rec["storage"], rec["sweep"], rec["ytile"], rec.get("emission")) != (
                    workload, storage_name, sweep, ytile, emission):
                continue
            with open(os.path.join(ROOT, rec["source"]), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
                    return None
            return int(rec["fetch_kib_per_dispatch"] * 1024 * rec["fetch_scale"]
                       + rec["write_kib_per_dispatch"] * 1024 * rec["write_scale"])
    except (OSError, KeyError, ValueError):
        return None
    return None


def emission_mode(tunable, storage, applies=True):
    """The compact sweep's emission reads as run: "gather" where the
    LBM_TUNE_EMISSION value asks for it and the gather applies (FP32 or FP64
    storage, UNIFORM or WEIGHTED sputtering, no product lattice), else
    "direct"."""
    from paper_1607_02874_amd import lbm

    return "gather" if applies and tunable == 1 and storage in (lbm.STORE_F32, lbm.STORE_F64) else "direct"


def cpu_info():
    """CPU model and core counts of this host."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(vox256, w, steps, multi_steps=100, single_steps=12, runs=3):
    """The FP64 oracle on the 64^3 crop of the same geometry: one run of
    `steps` on all threads for the error check, then the median of `runs`
    timed runs on all threads and on one thread."""
    import statistics

    import oracle

    crop = __import__("paper_1607_02874_amd.inputs", fromlist=["crop"]).crop(vox256, 64, 64, 64)
    p, _ = oracle.p_from_da(w.da, w.pore_size)

    def make():
        return oracle.Oracle(crop, tau=w.tau, p=p, p_stick=w.p_stick, c_inlet=w.c_inlet, force=w.force())

    all_threads = oracle.threads()
    o = make()
    t0 = time.perf_counter()
    o.step(steps)
    dt_ref = time.perf_counter() - t0
    ref = o.fields() + (o.conversion_map(),)
    o.close()

    def timed(threads, n):
        oracle.set_threads(threads)
        o = make()
        o.step(1)
        t = time.perf_counter()
        o.step(n)
        dt = time.perf_counter() - t
        o.close()
        return crop.size * n / dt / 1e6

    multi = [timed(all_threads, multi_steps) for _ in range(runs)]
    single = [timed(1, single_steps) for _ in range(runs)]
    oracle.set_threads(all_threads)
    return crop, ref, {"value": round(statistics.median(multi), 3), "unit": "MLUPS", "cores": all_threads,
                       "kind": "oracle", "single_thread": round(statistics.median(single), 3),
                       "runs": runs, **cpu_info(),
                       "sample": f"64^3 crop of the 256^3 sample (outlet planes 60-63 gas), FP64 C oracle, OpenMP "
                                 f"over z-planes: median of {runs} runs of {multi_steps} steps on {all_threads} "
                                 f"threads and of {runs} runs of {single_steps} steps on 1 thread; the error "
                                 f"check's {steps} steps took {dt_ref:.1f} s on {all_threads} threads"}


def cpu_baseline_batch(ws, n_samples=8, steps=20, runs=3):
    """The FP64 oracle on the n_samples smallest samples of the batch (their
    own tau, Da and geometry), all threads: median of `runs` runs of `steps`
    steps over those samples, in MLUPS of the samples' nodes."""
    import statistics

    import oracle

    small = sorted(ws, key=lambda w: w.nx * w.ny * w.nz)[:n_samples]
    voxs = [w.voxels() for w in small]
    nodes = sum(v.size for v in voxs)

    def run():
        t = 0.0
        for w, v in zip(small, voxs):
            p, _ = oracle.p_from_da(w.da, w.pore_size)
            o = oracle.Oracle(v, tau=w.tau, p=p, p_stick=w.p_stick, c_inlet=w.c_inlet, force=w.force())
            o.step(1)
            t0 = time.perf_counter()
            o.step(steps)
            t += time.perf_counter() - t0
            o.close()
        return nodes * steps / t / 1e6

    vals = [run() for _ in range(runs)]
    sides = ", ".join(str(w.nx) for w in small)
    return {"value": round(statistics.median(vals), 3), "unit": "MLUPS", "cores": oracle.threads(), "kind": "oracle",
            "runs": runs, **cpu_info(),
            "sample": f"the {n_samples} smallest samples of the same 64-sample batch (cubes of side {sides}; "
                      f"{nodes} nodes), FP64 C oracle, OpenMP over z-planes: median of {runs} runs of {steps} "
                      f"steps of each"}


def _median_event_ms(launch, stream, reps):
    """Median over `reps` launches of their time between HIP events recorded
    on `stream` (the stream the launch uses), after two untimed launches."""
    import statistics

    import torch

    launch()
    launch()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        launch()
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return statistics.median(times)


PULL_SIDE = 256  # the pull-streaming reference runs on a dense periodic 256^3 lattice


def copy_ceiling(pair_bytes=None, gib=2, reps=5):
    """HBM copy rate of this GPU with the library's streaming copy (one
    16-byte element per thread, non-temporal): median of `reps` copies of
    `gib` GiB, timed with HIP events on the current stream.  With
    `pair_bytes` (a population pair: 4, 8 or 16 bytes), also the rate of
    lbm_stream_pull: one D3Q19 pull-streaming pass, no collision, over a dense
    periodic 256^3 lattice in the sweep's blocked layout (the sweep's
    population traffic in its own access pattern)."""
    import torch

    from paper_1607_02874_amd import lbm

    n = gib << 30
    a = torch.zeros(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    lib = lbm.library()

    def copy():
        st = lib.lbm_stream_copy(b.data_ptr(), a.data_ptr(), n, stream.cuda_stream)
        if st != lbm.LBM_OK:
            raise RuntimeError(f"lbm_stream_copy failed with status {st}")

    ms = _median_event_ms(copy, stream, reps)
    del a, b
    out = {"copy_GBps": round(2 * n / (ms * 1e-3) / 1e9, 1), "copy_bytes": 2 * n, "kernel": "k_stream_copy",
           "method": f"median of {reps} device copies of {gib} GiB"}
    if pair_bytes:
        side = PULL_SIDE
        nodes = side ** 3
        nbuf = (nodes + 63) // 64 * 64 * 19 * pair_bytes
        a = torch.zeros(nbuf, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)

        def pull():
            st = lib.lbm_stream_pull(b.data_ptr(), a.data_ptr(), side, side, side, pair_bytes, stream.cuda_stream)
            if st != lbm.LBM_OK:
                raise RuntimeError(f"lbm_stream_pull failed with status {st}")

        ms = _median_event_ms(pull, stream, reps)
        del a, b
        moved = 2 * 19 * pair_bytes * nodes
        out.update({"pull_GBps": round(moved / (ms * 1e-3) / 1e9, 1), "pull_bytes": moved, "pull_us": round(ms * 1e3, 2),
                    "pull_kernel": "k_stream_pull",
                    "pull_method": f"median of {reps} D3Q19 pull-streaming passes (no collision) over a dense "
                                   f"periodic {side}^3 lattice in the blocked layout, {pair_bytes}-byte pairs"})
    return out


def ceiling_fracs(ceiling, achieved):
    """The achieved rate as fractions of the copy (and pull-streaming) rates."""
    f = {"frac_of_copy": round(achieved / ceiling["copy_GBps"], 4)}
    if "pull_GBps" in ceiling:
        f["frac_of_pull"] = round(achieved / ceiling["pull_GBps"], 4)
    return f


def crop_errors(crop, ref, w, steps, storage):
    from paper_1607_02874_amd import lbm

    with lbm.Sim(crop, da=w.da, tau=w.tau, pore_size=w.pore_size, force=w.force(), p_stick=w.p_stick,
                 c_inlet=w.c_inlet, storage=storage) as s:
        s.step(steps)
        got = s.fields() + (s.conversion_map(),)
    gas = crop == 0
    out = {}
    for name, a, b in zip(("rho", "u", "conc", "conv"), got, ref):
        if name == "u":
            d, r = (a - b)[:, gas], b[:, gas]
        elif name == "conv":
            d, r = a - b, b
        else:
            d, r = (a - b)[gas], b[gas]
        out[name] = float(np.linalg.norm(d) / np.linalg.norm(r))
        out[name + "_maxabs_rel"] = float(np.abs(d).max() / np.abs(r).max())
    return out


def run_batch(args):
    """The mixed-size batch: 64 cubes (side U{48..128}, porosity U[0.5, 0.75],
    correlation length 6, tau U[0.55, 1.2] for both lattices, Da log-uniform in
    [0.01, 100], seeds 2000 + s), all stepped together by lbm_batch_step, and
    the same 64 samples stepped one after another as single contexts."""
    import torch

    from paper_1607_02874_amd import inputs, lbm

    storage = STORAGES[args.storage]
    t0 = time.perf_counter()
    ws = inputs.batch_samples(64, 2000)
    samples = [dict(vox=w.voxels(), da=w.da, tau=w.tau, pore_size=w.pore_size, force=w.force(),
                    p_stick=w.p_stick, c_inlet=w.c_inlet, storage=storage) for w in ws]
    n_nodes = sum(s["vox"].size for s in samples)
    n_fluid = sum(int((s["vox"] == 0).sum()) for s in samples)
    log(f"batch geometry: 64 samples, {n_nodes} nodes, {n_fluid} gas ({time.perf_counter() - t0:.1f} s)")

    def timed(step_fn, sync_fn, steps):
        step_fn(args.warmup)
        sync_fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        step_fn(steps)
        sync_fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t

    batch = lbm.Batch(samples, graph=not args.no_graph)
    if args.sweep is not None:
        batch.set_tunable(lbm.TUNE_SWEEP, args.sweep)
    if args.ytile:
        batch.set_tunable(lbm.TUNE_YTILE, args.ytile)
    if args.emission is not None:
        batch.set_tunable(lbm.TUNE_EMISSION, args.emission)
    if not args.no_autotune and args.ytile is None and args.sweep is None and args.emission is None:
        ms = batch.autotune(3)
        log(f"autotune: sweep {batch.get_tunable(lbm.TUNE_SWEEP)} ytile {batch.get_tunable(lbm.TUNE_YTILE)} "
            f"({ms * 1e3:.1f} us)")
    sweep_variant = batch.get_tunable(lbm.TUNE_SWEEP)
    ytile_batch = batch.get_tunable(lbm.TUNE_YTILE)
    emission = emission_mode(batch.get_tunable(lbm.TUNE_EMISSION), storage)
    infos = [batch.info(i) for i in range(len(samples))]
    log(f"batched: timing {args.steps} steps")
    t_batch = timed(batch.step, batch.synchronize, args.steps)
    # the batched sweep's launch duration: captured graphs cannot hold timing
    # events, so a second pass of eager steps brackets every sweep with HIP
    # events on the batch stream
    t_steps = min(args.steps, 200)
    batch.set_timing(True)
    batch.step(t_steps)
    kt = batch.kernel_times()
    batch.set_timing(False)
    t_sweep = kt["ms_sweep"] / max(kt["n_sweep"], 1) * 1e-3
    batch.close()
    ceiling = copy_ceiling(2 * lbm.STORAGE_BYTES[storage])
    log(f"copy ceiling {ceiling}")
    sims = [] if args.no_sequential else [
        lbm.Sim(s["vox"], da=s["da"], tau=s["tau"], pore_size=s["pore_size"], force=s["force"],
                p_stick=s["p_stick"], c_inlet=s["c_inlet"], storage=storage) for s in samples]
    for sim in sims:  # the sequential runs autotune each sample on its own
        if args.no_autotune or args.ytile is not None or args.sweep is not None:
            sim.set_tunable(lbm.TUNE_SWEEP, sweep_variant)
            if args.ytile:
                sim.set_tunable(lbm.TUNE_YTILE, min(args.ytile, sim.shape[1]))
        else:
            sim.autotune(3)

    def seq_step(k):
        for sim in sims:
            sim.step(k)

    def seq_sync():
        for sim in sims:
            sim.synchronize()

    t_seq = None
    if sims:
        log(f"sequential: timing {args.steps} steps of each sample")
        t_seq = timed(seq_step, seq_sync, args.steps)
    for sim in sims:
        sim.close()

    s_bytes = lbm.STORAGE_BYTES[storage]
    step_bytes = sum(algorithmic_bytes(i, s_bytes)["step"] for i in infos)
    sweep_bytes = sum(algorithmic_bytes(i, s_bytes)["sweep"] for i in infos)
    ms_step = t_batch / args.steps * 1e3
    mlups = n_nodes * args.steps / t_batch / 1e6
    achieved = sweep_bytes / t_sweep / 1e9
    storage_name = {v: k for k, v in STORAGES.items()}[storage]
    traffic = measured_traffic("k_sweep_batch_c", "batch64", storage_name,
                               "node-compact" if sweep_variant == 1 else "64-voxel chunks", ytile_batch, emission)
    cpu = None
    if args.cpu_steps > 0:
        log("oracle on the 8 smallest samples of the batch")
        cpu = cpu_baseline_batch(ws)
    line = {
        "metric": "MLUPS (flow+species) and % of HBM roofline at stated error vs FP64 oracle",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {0: "f32", 1: "f16-storage/f32", 2: "bf16-storage/f32", 3: "f64"}[storage],
        "data": "synthetic (seeded Gaussian-random-field porous geometries)",
        "config": {"workload": "batch64: 64 porous cubes, side U{48..128}, porosity U[0.5,0.75], correlation "
                               "length 6, tau U[0.55,1.2], Da logU[0.01,100], seeds 2000+s",
                   "n_nodes": n_nodes, "n_fluid": n_fluid, "graph": not args.no_graph,
                   "sweep": "node-compact" if sweep_variant == 1 else "64-voxel chunks", "ytile": ytile_batch,
                   "emission": emission,
                   "sequential_mlups": round(n_nodes * args.steps / t_seq / 1e6, 1) if t_seq else None,
                   "sequential_ms_per_step": round(t_seq / args.steps * 1e3, 4) if t_seq else None,
                   "speedup_vs_sequential": round(t_seq / t_batch, 3) if t_seq else None,
                   "step_bytes": step_bytes, "step_GBps": round(step_bytes / (ms_step * 1e-3) / 1e9, 1)},
        "roofline": {"bound": "hbm", "kernel": "k_sweep_batch_c",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "bytes_per_launch": sweep_bytes, "avg_launch_us": round(t_sweep * 1e6, 2),
                     "timing": f"HIP events around each batched sweep of {kt['n_sweep']} eager steps after "
                               f"the timed graph replays",
                     "ceiling": {**ceiling, **ceiling_fracs(ceiling, achieved)}},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def run_precision(args):
    """512^3 porous sample (porosity 0.70, correlation length 12, seed 1002):
    the same run with FP32, FP16 and BF16 storage (FP32 arithmetic) and the
    FP64 build, and FP16 with stochastic rounding and BF16 with stochastic
    rounding and the carrier's reference flow (the FP32 run's mean
    x-velocity); per run the throughput, the speedup over FP32 and the
    L2-relative field errors against the FP64 build after the same steps."""
    import torch

    from paper_1607_02874_amd import inputs, lbm

    w = inputs.PRECISION_512
    t0 = time.perf_counter()
    vox = w.voxels()
    gas = vox == 0
    log(f"geometry {w.nx}x{w.ny}x{w.nz} porosity {inputs.porosity(vox):.4f} ({time.perf_counter() - t0:.1f} s)")
    results, fields = {}, {}
    # name: storage, rounding of 16-bit stores, reference flow (the FP32 run's
    # mean x-velocity over the gas nodes)
    runs = {"f64": ("f64", 0, False), "f32": ("f32", 0, False), "f16": ("f16", 0, False), "bf16": ("bf16", 0, False),
            "f16-sr": ("f16", 1, False), "bf16-sr-ref": ("bf16", 1, True)}
    u_ref = 0.0
    for name, (sname, rounding, shifted) in runs.items():
        storage = STORAGES[sname]
        sim = lbm.Sim(vox, da=w.da, tau=w.tau, pore_size=w.pore_size, force=w.force(), p_stick=w.p_stick,
                      c_inlet=w.c_inlet, storage=storage, rounding=rounding, store_ux=u_ref if shifted else 0.0)
        info = sim.info()
        if not args.no_autotune:
            sim.autotune(3)
        sim.step(args.warmup)
        sim.synchronize()
        sim.set_timing(2)  # events around the sweeps only
        torch.cuda.synchronize()
        t = time.perf_counter()
        sim.step(args.steps)
        sim.synchronize()
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        kt = sim.kernel_times()
        sim_tunables = {"variant": sim.get_tunable(lbm.TUNE_SWEEP), "ytile": sim.get_tunable(lbm.TUNE_YTILE)}
        rho, u, c = sim.fields()
        conv = sim.conversion_map()
        sim.close()
        ab = algorithmic_bytes(info, lbm.STORAGE_BYTES[storage])
        t_sweep = kt["ms_sweep"] / kt["n_sweep"] * 1e-3
        if name == "f32":
            u_ref = float(u[0][gas].mean())
        results[name] = {"mlups": round(vox.size * args.steps / el / 1e6, 1),
                         "rounding": "stochastic" if rounding else "nearest",
                         "store_ux": round(u_ref, 6) if shifted else 0.0,
                         "sweep": sim_tunables,
                         "ms_per_step": round(el / args.steps * 1e3, 4),
                         "sweep_us": round(t_sweep * 1e6, 2),
                         "sweep_GBps": round(ab["sweep"] / t_sweep / 1e9, 1)}
        if name == "f64":
            fields["f64"] = (rho[gas], u[:, gas], c[gas], conv)
        else:
            ref = fields["f64"]
            got = (rho[gas], u[:, gas], c[gas], conv)
            results[name]["error_vs_f64"] = {k: float(np.linalg.norm(a - b) / np.linalg.norm(b))
                                             for k, a, b in zip(("rho", "u", "conc", "conv"), got, ref)}
        del rho, u, c, conv
        log(f"{name}: {results[name]}")
    for name in ("f16", "bf16", "f16-sr", "bf16-sr-ref"):
        results[name]["speedup_vs_f32"] = round(results["f32"]["ms_per_step"] / results[name]["ms_per_step"], 3)
    best = "f16"
    line = {
        "metric": "MLUPS (flow+species) and % of HBM roofline at stated error vs FP64 oracle",
        "value": results[best]["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": results[best]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16-storage/f32",
        "data": "synthetic (seeded Gaussian-random-field porous geometry)",
        "config": {"workload": f"{w.name}: {w.nx}x{w.ny}x{w.nz} porous sample, porosity {w.phi}, correlation length "
                               f"{w.ell}, seed {w.seed}, tau {w.tau}, Da {w.da}",
                   "n_nodes": int(vox.size), "n_fluid": int(gas.sum()), "per_storage": results},
        "roofline": {"bound": "hbm", "kernel": "k_sweep (f16 storage)",
                     "achieved": results[best]["sweep_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(results[best]["sweep_GBps"] / HBM_PEAK_GBS, 4), "traffic": None},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def run_membrane(args):
    """1024x512x512 thin membrane (porous layer x in [384, 640), porosity 0.65,
    correlation length 10, seed 1004): Da = 10 (reaction-limited under the
    paper's convention) and Da = 0.1 (transport-limited), FP32 and FP16
    storage, reactant initially at c_in everywhere.  Per case the throughput
    and the conversion profile through the layer, reported as the ratio of
    what the front and the rear quarter of the layer converted."""
    import torch

    from paper_1607_02874_amd import inputs, lbm

    w = inputs.MEMBRANE_1024
    t0 = time.perf_counter()
    vox = w.voxels()
    log(f"geometry {w.nx}x{w.ny}x{w.nz} porosity {inputs.porosity(vox):.4f} ({time.perf_counter() - t0:.1f} s)")
    lo, hi = w.x_lo, w.x_hi
    q = (hi - lo) // 4
    results = {}
    storages = [args.storage] if args.storage != "f32" else ["f32", "f16"]
    for name in storages:
        for da in (10.0, 0.1):
            # reactant everywhere from the start (c0 = c_in): the inlet alone
            # would not reach a layer 384 nodes downstream within the run
            sim = lbm.Sim(vox, da=da, tau=w.tau, pore_size=w.pore_size, force=w.force(), p_stick=w.p_stick,
                          c_inlet=w.c_inlet, c0=w.c_inlet, storage=STORAGES[name])
            info = sim.info()
            if not args.no_autotune:
                sim.autotune(2)
            sim.step(args.warmup)
            sim.synchronize()
            sim.set_timing(2)  # events around the sweeps only
            torch.cuda.synchronize()
            t = time.perf_counter()
            sim.step(args.steps)
            sim.synchronize()
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            kt = sim.kernel_times()
            conv = sim.conversion_map()
            tot = sim.totals()
            prof = conv[:, :, lo:hi].sum(axis=(0, 1))
            ab = algorithmic_bytes(info, lbm.STORAGE_BYTES[STORAGES[name]])
            t_sweep = kt["ms_sweep"] / kt["n_sweep"] * 1e-3
            key = f"{name}_da{da:g}"
            results[key] = {"mlups": round(vox.size * args.steps / el / 1e6, 1),
                            "ms_per_step": round(el / args.steps * 1e3, 3),
                            "sweep_us": round(t_sweep * 1e6, 1),
                            "sweep_GBps": round(ab["sweep"] / t_sweep / 1e9, 1),
                            "p": round(info["p"], 6),
                            "sweep": "node-compact" if sim.get_tunable(lbm.TUNE_SWEEP) == 1 else "64-voxel chunks",
                            "ytile": sim.get_tunable(lbm.TUNE_YTILE),
                            "converted": tot["converted"], "lost": tot["lost"],
                            "front_rear_ratio": float(prof[:q].sum() / max(prof[-q:].sum(), 1e-300))}
            sim.close()
            del conv
            log(f"{key}: {results[key]}")
    first = f"{storages[0]}_da10"
    line = {
        "metric": "MLUPS (flow+species) and % of HBM roofline at stated error vs FP64 oracle",
        "value": results[first]["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": results[first]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f16": "f16-storage/f32", "bf16": "bf16-storage/f32", "f64": "f64"}[storages[0]],
        "data": "synthetic (seeded Gaussian-random-field porous layer)",
        "config": {"workload": f"{w.name}: {w.nx}x{w.ny}x{w.nz}, porous layer x in [{lo}, {hi}), porosity {w.phi}, "
                               f"correlation length {w.ell}, seed {w.seed}, tau {w.tau}; Da 10 and 0.1",
                   "n_nodes": int(vox.size), "cases": results},
        "roofline": {"bound": "hbm", "kernel": f"sweep ({first})", "achieved": results[first]["sweep_GBps"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(results[first]["sweep_GBps"] / HBM_PEAK_GBS, 4), "traffic": None},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def run_shard(args):
    """One rank's share of the 1024x512x512 membrane on 8 GPUs: the central
    128x512x512 x-slab of the porous layer (x in [448, 576) of the membrane
    geometry), stepped alone with periodic x for both lattices as an interior
    slab sees its neighbours.  Reports the sweep time next to the bytes the
    x-face halo exchange would move per step."""
    import torch

    from paper_1607_02874_amd import inputs, lbm

    w = inputs.MEMBRANE_1024
    t0 = time.perf_counter()
    vox = np.ascontiguousarray(w.voxels()[:, :, 448:576])
    log(f"shard 128x512x512 porosity {inputs.porosity(vox):.4f} ({time.perf_counter() - t0:.1f} s)")
    storage = STORAGES[args.storage]
    sim = lbm.Sim(vox, da=w.da, tau=w.tau, pore_size=w.pore_size, force=w.force(), p_stick=w.p_stick,
                  c_inlet=w.c_inlet, c0=w.c_inlet, species_x=lbm.XBC_PERIODIC, storage=storage)
    info = sim.info()
    if not args.no_autotune:
        sim.autotune(3)
    sim.step(args.warmup)
    sim.synchronize()
    sim.set_timing(2)  # events around the sweeps only
    torch.cuda.synchronize()
    t = time.perf_counter()
    sim.step(args.steps)
    sim.synchronize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    kt = sim.kernel_times()
    sweep_variant = sim.get_tunable(lbm.TUNE_SWEEP)
    ytile = sim.get_tunable(lbm.TUNE_YTILE)
    sim.close()
    s_bytes = lbm.STORAGE_BYTES[storage]
    ab = algorithmic_bytes(info, s_bytes)
    t_sweep = kt["ms_sweep"] / kt["n_sweep"] * 1e-3
    face_nodes = int((vox[:, :, 0] == 0).sum())
    halo = 2 * 5 * s_bytes * face_nodes  # per face and direction: 5 populations of each lattice
    line = {
        "metric": "MLUPS (flow+species) and % of HBM roofline at stated error vs FP64 oracle",
        "value": round(vox.size * args.steps / el / 1e6, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {0: "f32", 1: "f16-storage/f32", 2: "bf16-storage/f32", 3: "f64"}[storage],
        "data": "synthetic (seeded Gaussian-random-field porous layer)",
        "config": {"workload": "membrane shard: x in [448, 576) of the 1024x512x512 membrane (one of 8 x-slabs), "
                               "periodic x",
                   "n_nodes": int(vox.size), "n_fluid": info["n_fluid"],
                   "sweep": "node-compact" if sweep_variant == 1 else "64-voxel chunks", "ytile": ytile,
                   "sweep_us": round(t_sweep * 1e6, 1),
                   "halo_bytes_per_face_per_direction": halo,
                   "halo_us_at_153GBps": round(halo / 153e9 * 1e6, 1)},
        "roofline": {"bound": "hbm", "kernel": "k_sweep_c" if sweep_variant == 1 else "k_sweep",
                     "achieved": round(ab["sweep"] / t_sweep / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ab["sweep"] / t_sweep / 1e9 / HBM_PEAK_GBS, 4), "traffic": None},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def run_product(args):
    """The 256^3 porous sample with the product lattice P (three D3Q19
    lattices: carrier, reactant, product; p_S^P = 0 as in the paper), FP32
    unless --storage says otherwise.  Reports lattice updates per second (one
    update covers all three lattices), the sweep's share of the HBM roofline,
    the product totals and the conversion efficiency of Eq. (eff) over the
    timed window."""
    import torch

    from paper_1607_02874_amd import inputs, lbm

    w = inputs.SINGLE_256
    vox = w.voxels()
    storage = STORAGES[args.storage]
    sim = lbm.Sim(vox, da=w.da, tau=w.tau, pore_size=w.pore_size, force=w.force(), p_stick=w.p_stick,
                  c_inlet=w.c_inlet, storage=storage, product=True, p_stick_product=0.0)
    info = sim.info()
    if args.ytile:
        sim.set_tunable(lbm.TUNE_YTILE, args.ytile)
    if not args.no_autotune and args.ytile is None:
        sim.autotune(3)
    sim.step(args.warmup)
    sim.synchronize()
    t0 = sim.totals()
    sim.set_timing(2)  # events around the sweeps only
    torch.cuda.synchronize()
    t = time.perf_counter()
    sim.step(args.steps)
    sim.synchronize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    kt = sim.kernel_times()
    t1 = sim.totals()
    sweep_variant = sim.get_tunable(lbm.TUNE_SWEEP)
    ytile = sim.get_tunable(lbm.TUNE_YTILE)
    sim.close()
    ceiling = copy_ceiling()
    s_bytes = lbm.STORAGE_BYTES[storage]
    ab = algorithmic_bytes(info, s_bytes, product=True)
    t_sweep = kt["ms_sweep"] / kt["n_sweep"] * 1e-3
    d_in = t1["influx"] - t0["influx"]
    eta = (t1["product_out_outlet"] - t0["product_out_outlet"]) / d_in if d_in else None
    storage_name = {0: "f32", 1: "f16", 2: "bf16", 3: "f64"}[storage]
    line = {
        "metric": "MLUPS (flow+species) and % of HBM roofline at stated error vs FP64 oracle",
        "value": round(vox.size * args.steps / el / 1e6, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {0: "f32", 1: "f16-storage/f32", 2: "bf16-storage/f32", 3: "f64"}[storage],
        "data": "synthetic (seeded Gaussian-random-field porous sample)",
        "config": {"workload": f"{w.name} with the product lattice: {w.nx}x{w.ny}x{w.nz}, carrier, reactant and "
                               f"product D3Q19 lattices, p_S^P = 0",
                   "n_nodes": int(vox.size), "n_fluid": info["n_fluid"], "n_interface": info["n_interface"],
                   "sweep": "node-compact" if sweep_variant == 1 else "64-voxel chunks", "ytile": ytile,
                   "sweep_us": round(t_sweep * 1e6, 1),
                   "mass_product": t1["mass_product"], "converted": t1["converted"],
                   "conversion_efficiency_window": eta},
        "roofline": {"bound": "hbm", "kernel": "k_sweep_c",
                     "achieved": round(ab["sweep"] / t_sweep / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ab["sweep"] / t_sweep / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("k_sweep_c", w.name + "_product", storage_name, "node-compact",
                                                 ytile, "direct"),
                     "algorithmic_bytes": ab["sweep"],
                     "ceiling": {**ceiling, "frac_of_copy": round(ab["sweep"] / t_sweep / 1e9 / ceiling["copy_GBps"], 4)}},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def run_stochastic(args):
    """The 256^3 porous sample with the random sputtering matrix
    (STOCHASTIC: each arrival leaves along one exit drawn by Philox4x32-10),
    otherwise the default workload.  Reports lattice updates per second and
    the sweep's share of the HBM roofline."""
    import torch

    from paper_1607_02874_amd import inputs, lbm

    w = inputs.SINGLE_256
    vox = w.voxels()
    storage = STORAGES[args.storage]
    sim = lbm.Sim(vox, da=w.da, tau=w.tau, pore_size=w.pore_size, force=w.force(), p_stick=w.p_stick,
                  c_inlet=w.c_inlet, storage=storage, sputter=lbm.SPUTTER_STOCHASTIC, seed=2016)
    info = sim.info()
    if args.ytile:
        sim.set_tunable(lbm.TUNE_YTILE, args.ytile)
    if not args.no_autotune and args.ytile is None:
        sim.autotune(3)
    sim.step(args.warmup)
    sim.synchronize()
    sim.set_timing(2)
    torch.cuda.synchronize()
    t = time.perf_counter()
    sim.step(args.steps)
    sim.synchronize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    kt = sim.kernel_times()
    tot = sim.totals()
    sweep_variant = sim.get_tunable(lbm.TUNE_SWEEP)
    ytile = sim.get_tunable(lbm.TUNE_YTILE)
    sim.close()
    ceiling = copy_ceiling()
    s_bytes = lbm.STORAGE_BYTES[storage]
    ab = algorithmic_bytes(info, s_bytes, stochastic=True)
    t_sweep = kt["ms_sweep"] / kt["n_sweep"] * 1e-3
    line = {
        "metric": "MLUPS (flow+species) and % of HBM roofline at stated error vs FP64 oracle",
        "value": round(vox.size * args.steps / el / 1e6, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {0: "f32", 1: "f16-storage/f32", 2: "bf16-storage/f32", 3: "f64"}[storage],
        "data": "synthetic (seeded Gaussian-random-field porous sample)",
        "config": {"workload": f"{w.name} with STOCHASTIC sputtering (Philox4x32-10 draws, seed 2016)",
                   "n_nodes": int(vox.size), "n_fluid": info["n_fluid"], "n_interface": info["n_interface"],
                   "sweep": "node-compact" if sweep_variant == 1 else "64-voxel chunks", "ytile": ytile,
                   "sweep_us": round(t_sweep * 1e6, 1), "converted": tot["converted"]},
        "roofline": {"bound": "hbm", "kernel": "k_sweep_c" if sweep_variant == 1 else "k_sweep",
                     "achieved": round(ab["sweep"] / t_sweep / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ab["sweep"] / t_sweep / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("k_sweep_c" if sweep_variant == 1 else "k_sweep",
                                                 w.name + "_stochastic", {0: "f32", 1: "f16", 2: "bf16",
                                                                          3: "f64"}[storage],
                                                 "node-compact" if sweep_variant == 1 else "64-voxel chunks", ytile,
                                                 "direct"),
                     "algorithmic_bytes": ab["sweep"],
                     "ceiling": {**ceiling, "frac_of_copy": round(ab["sweep"] / t_sweep / 1e9 / ceiling["copy_GBps"], 4)}},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def run_reactor2d(args):
    """The paper's 2-D reactor ("Results & Discussion", Table 1, the p and
    w/h sweep of Fig. 6) on one z-plane of D3Q19, whose populations project
    exactly onto D2Q9's weights (4/9, 1/9, 1/36): L = 250 along the flow,
    H = 500 across, a horizontal ingot h = 200 wide and w = 6, 10, 20, 30
    thick carved to porosity 0.70 with 3-unit disks, tau 4 for every lattice,
    rho_C = 0.8, reactant injected with the flow at 0.2 (INFLOW), no product
    at the inlet, p_S^R = 0.95 (Table 1), p_S^P = 0, p = 0.35 ... 0.65.  The
    gas is periodic and driven by a body force; the mean inlet speed it
    reaches is reported (the paper imposes 0.08).  The conversion efficiency
    of Eq. (eff), product mass leaving through the outlet over reactant mass
    entering through the inlet, is taken over the last 20000 of 60000 steps
    with the reactant inflow c_in sum_y u_x(0, y) per step (the inlet flow;
    the ghost populations' gross influx, mostly diffusion that returns, is
    reported beside it)."""
    import torch

    from paper_1607_02874_amd import inputs, lbm

    steps, window = 60000, 20000
    tau, rho0, c_in = 4.0, 0.8, 0.2
    d2q9 = args.lattice == "d2q9"
    lattice = lbm.LATTICE_D2Q9 if d2q9 else lbm.LATTICE_D3Q19
    storage = STORAGES["f64"] if d2q9 else STORAGES[args.storage]  # the D2Q9 path is FP64
    force = 4.0e-5
    ps = (0.35, 0.45, 0.55, 0.65)
    ws = (6, 10, 20, 30)
    eta, eta_gross, u_mean = {}, {}, {}
    n_updates, t_total = 0, 0.0
    for w in ws:
        vox = inputs.disk_ingot(w, seed=w)
        for p in ps:
            da = np.sqrt(1.0 / 3.0) / (p * 3.0)  # p = cs / (Da delta), delta = 3
            with lbm.Sim(vox, da=da, tau=(tau, tau), pore_size=3.0, force=(force, 0.0, 0.0), rho0=rho0,
                         c_inlet=c_in, p_stick=0.95, species_x=lbm.XBC_INFLOW, product=True,
                         p_stick_product=0.0, storage=storage, lattice=lattice) as sim:
                torch.cuda.synchronize()
                t = time.perf_counter()
                gas = vox[0, :, 0] == inputs.FLUID
                sim.step(steps - window)
                t0 = sim.totals()
                q0 = float(sim.fields()[1][0, 0, gas, 0].sum())
                sim.step(window)
                t1 = sim.totals()
                q1 = float(sim.fields()[1][0, 0, gas, 0].sum())
                t_total += time.perf_counter() - t
                n_updates += vox.size * steps
                d_out = t1["product_out_outlet"] - t0["product_out_outlet"]
                key = f"p={p}"
                eta.setdefault(key, {})[f"w={w}"] = round(d_out / (window * c_in * 0.5 * (q0 + q1)), 4)
                eta_gross.setdefault(key, {})[f"w={w}"] = round(d_out / (t1["influx"] - t0["influx"]), 5)
                if p == ps[0]:
                    u_mean[f"w={w}"] = round(0.5 * (q0 + q1) / int(gas.sum()), 4)
            log(f"w {w} p {p}: eta {eta[f'p={p}'][f'w={w}']}")
    line = {
        "metric": "conversion efficiency eta (Eq. eff) of the paper's 2-D reactor vs p and w/h",
        "value": round(n_updates / t_total / 1e6, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 0,
        "ms_per_step": round(t_total / (len(ps) * len(ws) * steps) * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {0: "f32", 1: "f16-storage/f32", 2: "bf16-storage/f32", 3: "f64"}[storage],
        "data": "synthetic (seeded disk-carved porous ingot, the paper's recipe)",
        "config": {"workload": ("reactor2d: 250 x 500 on D2Q9 (the paper's lattice, b(k) <= 8)" if d2q9 else
                                "reactor2d: 250 x 500 x 1, D3Q19 on one plane (b(k) counts 3-D links)") +
                               ", ingot h = 200, porosity 0.70, tau 4, rho_C 0.8, c_in 0.2 (INFLOW), p_S^R 0.95, "
                               "p_S^P 0, UNIFORM re-emission, 60000 steps, eta over the last 20000",
                   "lattice": args.lattice,
                   "body_force": force, "inlet_mean_u": u_mean, "eta": eta,
                   "eta_over_gross_ghost_influx": eta_gross,
                   "paper": "eta = 0.2 at p = 0.45, w = 10 (the experimental value the paper matches)"},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--storage", default="f32", choices=sorted(STORAGES))
    ap.add_argument("--da", type=float, default=None)
    ap.add_argument("--wall-diffuse", type=float, default=0.0,
                    help="diffuse fraction of the carrier's wall reflection (default 0: bounce-back)")
    ap.add_argument("--cpu-steps", type=int, default=300, help="oracle steps on the 64^3 crop (0 = skip)")
    ap.add_argument("--no-timing", action="store_true", help="do not record per-kernel HIP events")
    ap.add_argument("--copy-calib", action="store_true", help="also run a 4 GiB device copy (counter calibration)")
    ap.add_argument("--lattice", default="d3q19", choices=("d3q19", "d2q9"),
                    help="reactor2d workload: velocity set (d2q9 runs in FP64)")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batch workload: skip stepping the samples one after another (for profiling runs)")
    ap.add_argument("--ytile", type=int, default=None, help="sweep y-tile height (default: the library's)")
    ap.add_argument("--scan-ytile", default="", help="comma list of y-tile heights to time before the run")
    ap.add_argument("--sweep", type=int, default=None, choices=(0, 1),
                    help="sweep variant: 1 node-compact (library default), 0 one wave per 64-voxel chunk")
    ap.add_argument("--emission", type=int, default=None, choices=(0, 1),
                    help="emission reads of the compact sweep: 1 gathered through LDS (a context's default), "
                         "0 direct (a batch's default); single and batch workloads")
    ap.add_argument("--workload", default="single", choices=("single", "batch", "precision", "membrane", "shard", "product", "reactor2d", "stochastic"),
                    help="single: the 256^3 sample; batch: the 64-sample mixed batch; precision: 512^3 "
                         "with FP32/FP16/BF16 storage against the FP64 build; membrane: 1024x512x512 layer; "
                         "shard: one 128x512x512 x-slab of the membrane")
    ap.add_argument("--no-graph", action="store_true", help="batch: launch directly instead of graph replays")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default launch shape instead of autotuning it before timing")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: the library runs on one GPU only (asked for {max(args.gpus, world)}); "
              "sharding across GPUs (x-slabs with a population halo) is designed but not implemented",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1607_02874_amd import inputs, lbm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "precision":
        run_precision(args)
        return
    if args.workload == "membrane":
        run_membrane(args)
        return
    if args.workload == "product":
        return run_product(args)
    if args.workload == "reactor2d":
        return run_reactor2d(args)
    if args.workload == "stochastic":
        return run_stochastic(args)
    if args.workload == "shard":
        run_shard(args)
        return
    w = inputs.SINGLE_256
    if args.da is not None:
        w.da = args.da
    storage = STORAGES[args.storage]
    s_bytes = lbm.STORAGE_BYTES[storage]

    t0 = time.perf_counter()
    vox = w.voxels()
    log(f"geometry {w.nx}x{w.ny}x{w.nz} porosity {inputs.porosity(vox):.4f} ({time.perf_counter() - t0:.1f} s)")
    t0 = time.perf_counter()
    sim = lbm.Sim(vox, da=w.da, tau=w.tau, pore_size=w.pore_size, force=w.force(), p_stick=w.p_stick,
                  c_inlet=w.c_inlet, storage=storage, wall_diffuse=args.wall_diffuse)
    info = sim.info()
    log(f"create {time.perf_counter() - t0:.1f} s, info {info}")

    if args.sweep is not None:
        sim.set_tunable(lbm.TUNE_SWEEP, args.sweep)
    if args.scan_ytile:
        for yt in [int(v) for v in args.scan_ytile.split(",")]:
            sim.set_tunable(lbm.TUNE_YTILE, yt)
            sim.step(20)
            sim.synchronize()
            sim.set_timing(2)  # events around the sweeps only
            sim.step(100)
            kt = sim.kernel_times()
            sim.set_timing(False)
            log(f"ytile {yt}: sweep {kt['ms_sweep'] / kt['n_sweep'] * 1e3:.1f} us")
    if args.ytile:
        sim.set_tunable(lbm.TUNE_YTILE, args.ytile)
    if args.emission is not None:
        sim.set_tunable(lbm.TUNE_EMISSION, args.emission)
    tuned = None
    if not args.no_autotune and args.ytile is None and args.sweep is None and args.emission is None:
        tuned = sim.autotune(10)
        log(f"autotune: sweep {sim.get_tunable(lbm.TUNE_SWEEP)} ytile {sim.get_tunable(lbm.TUNE_YTILE)} "
            f"emission {sim.get_tunable(lbm.TUNE_EMISSION)} ({tuned * 1e3:.1f} us)")
    sweep_variant = sim.get_tunable(lbm.TUNE_SWEEP)
    emission = emission_mode(sim.get_tunable(lbm.TUNE_EMISSION), storage)
    sim.step(args.warmup)
    sim.synchronize()
    torch.cuda.synchronize()
    # HIP events around every sweep of the timed region (the sweep's launch
    # time for the roofline); events between the other launches would cost
    # step time
    if not args.no_timing:
        sim.set_timing(2)
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = sim.kernel_times() if not args.no_timing else None
    tot = sim.totals()
    if kt is not None:
        # the other launches, timed after the measurement (every launch evented)
        sim.set_timing(1)
        sim.step(min(200, args.steps))
        kt_all = sim.kernel_times()
        sim.set_timing(0)
        for k in ("interface", "reduce"):
            kt["ms_" + k], kt["n_" + k] = kt_all["ms_" + k], kt_all["n_" + k]
    ytile = sim.get_tunable(lbm.TUNE_YTILE)
    sim.close()
    log(f"elapsed {elapsed:.3f} s, totals {tot}")

    ceiling = copy_ceiling(2 * lbm.STORAGE_BYTES[storage])
    log(f"copy ceiling {ceiling}")
    if args.copy_calib:
        a = torch.empty(1 << 30, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    n = info["n_nodes"]
    ms_step = elapsed / args.steps * 1e3
    mlups = n * args.steps / elapsed / 1e6
    ab = algorithmic_bytes(info, s_bytes)
    roofline = None
    if kt and kt["n_sweep"]:
        t_sweep = kt["ms_sweep"] / kt["n_sweep"] * 1e-3
        achieved = ab["sweep"] / t_sweep / 1e9
        kname = "k_sweep_c" if sweep_variant == 1 else "k_sweep"
        roofline = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(kname, w.name, args.storage,
                                                "node-compact" if sweep_variant == 1 else "64-voxel chunks", ytile,
                                                emission),
                    "bytes_per_launch": ab["sweep"], "avg_launch_us": round(t_sweep * 1e6, 2),
                    "ceiling": {**ceiling, **ceiling_fracs(ceiling, achieved)}}
    kernels = None
    if kt:
        kernels = {k: round(kt["ms_" + k] / max(kt["n_" + k], 1) * 1e3, 2) for k in ("sweep", "interface", "reduce")}

    cpu, errs = None, None
    if args.cpu_steps > 0 and args.wall_diffuse:
        log("the oracle crop check runs the default workload only; skipped with --wall-diffuse")
    if args.cpu_steps > 0 and not args.wall_diffuse:
        log(f"oracle {args.cpu_steps} steps on the 64^3 crop")
        crop, ref, cpu = cpu_baseline(vox, w, args.cpu_steps)
        errs = crop_errors(crop, ref, w, args.cpu_steps, storage)
        log(f"cpu baseline {cpu}, errors {errs}")

    line = {
        "metric": "MLUPS (flow+species) and % of HBM roofline at stated error vs FP64 oracle",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {0: "f32", 1: "f16-storage/f32", 2: "bf16-storage/f32", 3: "f64"}[storage],
        "data": "synthetic (seeded Gaussian-random-field porous geometry)",
        "config": {"workload": f"{w.name}: {w.nx}x{w.ny}x{w.nz} porous membrane, porosity {w.phi}, "
                               f"correlation length {w.ell}, seed {w.seed}, tau {w.tau}, Da {w.da}, "
                               f"p_S {w.p_stick}, UNIFORM sputter, PASSIVE coupling, reservoir x-BC"
                               + (f", diffuse wall fraction {args.wall_diffuse}" if args.wall_diffuse else ""),
                   "n_nodes": n, "n_fluid": info["n_fluid"], "n_interface": info["n_interface"],
                   "n_catalytic_links": info["n_catalytic_links"], "mflups": round(mlups * info["n_fluid"] / n, 1),
                   "step_bytes": ab["step"], "step_GBps": round(ab["step"] / (ms_step * 1e-3) / 1e9, 1),
                   "kernel_us": kernels, "ytile": ytile, "autotuned": tuned is not None,
                   "sweep": "node-compact" if sweep_variant == 1 else "64-voxel chunks", "emission": emission},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "error_vs_oracle": None if errs is None else {
            "crop": "64^3", "steps": args.cpu_steps, "metric": "L2-relative over gas nodes", **errs},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
