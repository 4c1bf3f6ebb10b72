"""Shared helpers of the GPU parity tests: run the HIP library and the FP64
oracle on the same seeded input and compare what they output."""

import numpy as np

import oracle
from paper_1607_02874_amd import inputs

SPUTTER = {"UNIFORM": 0, "WEIGHTED": 1, "BOUNCEBACK": 2}
COUPLING = {"PASSIVE": 0, "BARYCENTRIC": 1}
XBC = {"PERIODIC": 0, "RESERVOIR": 1, "INFLOW": 2}


NEAREST, STOCHASTIC = 0, 1  # rounding of 16-bit stores


def case(vox, steps, da=1.0, tau=(0.8, 0.7), pore_size=4.0, p_stick=0.95, c_inlet=1.0, c0=0.0, rho0=1.0,
         force=(0.0, 0.0, 0.0), sputter="UNIFORM", coupling="PASSIVE", species_x="RESERVOIR", rounding=NEAREST):
    return dict(vox=np.ascontiguousarray(vox, np.uint8), steps=steps, da=da, tau=tau, pore_size=pore_size,
                p_stick=p_stick, c_inlet=c_inlet, c0=c0, rho0=rho0, force=tuple(force), sputter=sputter,
                coupling=coupling, species_x=species_x, rounding=rounding)


def run_oracle(c):
    p, _ = oracle.p_from_da(c["da"], c["pore_size"])
    o = oracle.Oracle(c["vox"], tau=c["tau"], p=p, p_stick=c["p_stick"], c_inlet=c["c_inlet"], rho0=c["rho0"],
                      c0=c["c0"], force=c["force"], sputter=SPUTTER[c["sputter"]],
                      coupling=COUPLING[c["coupling"]], species_x=XBC[c["species_x"]])
    o.step(c["steps"])
    rho, u, conc = o.fields()
    out = dict(rho=rho, u=u, conc=conc, conv=o.conversion_map(), totals=o.totals(), links=o.link_counts(), p=p)
    o.close()
    return out


def make_sim(c, storage):
    from paper_1607_02874_amd import lbm

    return lbm.Sim(c["vox"], da=c["da"], tau=c["tau"], pore_size=c["pore_size"], p_stick=c["p_stick"],
                   c_inlet=c["c_inlet"], c0=c["c0"], rho0=c["rho0"], force=c["force"],
                   sputter=SPUTTER[c["sputter"]], coupling=COUPLING[c["coupling"]],
                   species_x=XBC[c["species_x"]], storage=storage, rounding=c.get("rounding", NEAREST),
                   store_ux=c.get("store_ux", 0.0))


def run_gpu(c, storage):
    s = make_sim(c, storage)
    s.step(c["steps"])
    rho, u, conc = s.fields()
    out = dict(rho=rho, u=u, conc=conc, conv=s.conversion_map(), totals=s.totals(), links=s.active_links(),
               info=s.info())
    s.close()
    return out


def l2rel(a, b, mask):
    """||a - b|| / ||b|| over the gas nodes (vector fields: over all components)."""
    if a.ndim == mask.ndim + 1:
        d = (a - b)[:, mask]
        r = b[:, mask]
    else:
        d = (a - b)[mask]
        r = b[mask]
    den = np.linalg.norm(r)
    num = np.linalg.norm(d)
    return num / den if den > 0 else num


def maxrel(a, b, mask):
    """max |a - b| / max |b| over the gas nodes (vector fields: all components)."""
    if a.ndim == mask.ndim + 1:
        d, r = (a - b)[:, mask], b[:, mask]
    else:
        d, r = (a - b)[mask], b[mask]
    den = np.abs(r).max() if r.size else 0.0
    num = np.abs(d).max() if d.size else 0.0
    return num / den if den > 0 else num


def errors(gpu, ref, vox):
    """L2-relative errors per field over the gas nodes (the conversion map
    over catalytic voxels), and the max-abs form under the "_max" keys."""
    gas = vox == inputs.FLUID
    cat = vox == inputs.CATALYTIC
    e = {k: l2rel(gpu[k], ref[k], gas) for k in ("rho", "u", "conc")}
    e["conv"] = l2rel(gpu["conv"], ref["conv"], cat) if cat.any() else 0.0
    for k in ("rho", "u", "conc"):
        e[k + "_max"] = maxrel(gpu[k], ref[k], gas)
    e["conv_max"] = maxrel(gpu["conv"], ref["conv"], cat) if cat.any() else 0.0
    for k in ("rho", "conc"):
        e[k + "_solid_zero"] = bool((gpu[k][~gas] == 0).all())
    return e


def mean_ux(gpu, vox):
    """Mean x-velocity over the gas nodes of a run's output."""
    return float(gpu["u"][0][vox == inputs.FLUID].mean())


def totals_rel(gpu, ref):
    out = {}
    for k in ("mass_gas", "mass_species", "converted", "lost", "influx", "outflux"):
        a, b = gpu["totals"][k], ref["totals"][k]
        scale = max(abs(b), abs(ref["totals"]["mass_gas"]) * 1e-9, 1e-300)
        out[k] = abs(a - b) / scale
    return out
