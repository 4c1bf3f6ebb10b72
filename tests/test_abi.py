"""The C-ABI library: it loads, exports every function include/lbm.h
declares, and rejects invalid arguments before touching a device (so these
run on a machine without a GPU)."""

import ctypes

import numpy as np
import pytest

from paper_1607_02874_amd import lbm


def test_every_declared_function_is_exported():
    names = lbm.header_functions()
    assert {"lbm_create", "lbm_create_on", "lbm_step", "lbm_fields", "lbm_conversion_map", "lbm_totals",
            "lbm_query", "lbm_destroy", "lbm_last_error"} <= set(names)
    for n in names:
        assert hasattr(lbm.library(), n), n


def test_struct_sizes_match_header_layout():
    assert ctypes.sizeof(lbm.lbm_geometry) == 32
    assert ctypes.sizeof(lbm.lbm_bc) == 16 + 5 * 8 + 24 + 8 + 8 + 8 + 8 + 8 + 8 + 8
    assert ctypes.sizeof(lbm.lbm_totals_t) == 8 + 6 * 8 + 8 + 4 * 8
    assert ctypes.sizeof(lbm.lbm_device) == 32


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """Sizes and field offsets of the binding's structs equal what a C
    compiler makes of include/lbm.h."""
    import os
    import subprocess

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    structs = {"lbm_geometry": lbm.lbm_geometry, "lbm_bc": lbm.lbm_bc, "lbm_totals_t": lbm.lbm_totals_t,
               "lbm_info": lbm.lbm_info, "lbm_kernel_times_t": lbm.lbm_kernel_times_t}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "lbm.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        name, field, value = line.split()
        got[(name, field)] = int(value)
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)


def _create(vox, **kw):
    args = dict(da=1.0, tau=(0.8, 0.7), pore_size=4.0)
    args.update(kw)
    return lbm.lbm_create(vox, **args)


@pytest.mark.parametrize("kw,msg", [
    (dict(tau=(0.5, 0.7)), "tau"),
    (dict(tau=(0.8, 0.3)), "tau"),
    (dict(da=0.0), "da"),
    (dict(da=-1.0), "da"),
    (dict(da=float("nan")), "da"),
    (dict(p_stick=1.5), "p_stick"),
    (dict(p_stick=-0.1), "p_stick"),
    (dict(pore_size=0.0), "pore_size"),
    (dict(rho0=0.0), "rho0"),
    (dict(c_inlet=-1.0), "c_inlet"),
    (dict(tau=(0.0, 0.0), kn=0.0), "kn"),
    (dict(kn=-0.5), "kn"),
    (dict(tau=(0.8, 0.7), kn=0.3), "disagree"),
    (dict(force=(float("inf"), 0, 0)), "force"),
    (dict(product=True, p_stick_product=1.5), "p_stick_product"),
    (dict(product=True, p_stick_product=-0.1), "p_stick_product"),
    (dict(wall_diffuse=1.5), "wall_diffuse"),
    (dict(wall_diffuse=-0.5), "wall_diffuse"),
    (dict(storage=1, store_ux=0.25), "store_ux"),
    (dict(storage=2, store_ux=float("nan")), "store_ux"),
])
def test_invalid_parameters_are_rejected(kw, msg):
    vox = np.zeros((4, 4, 8), np.uint8)
    with pytest.raises(lbm.LbmError) as e:
        _create(vox, **kw)
    assert e.value.status == lbm.LBM_EINVAL
    assert msg in str(e.value)


def test_invalid_voxel_and_mode_values():
    vox = np.zeros((4, 4, 8), np.uint8)
    vox[1, 2, 3] = 3
    with pytest.raises(lbm.LbmError) as e:
        _create(vox)
    assert e.value.status == lbm.LBM_EINVAL and "voxel" in str(e.value)
    vox[1, 2, 3] = 0
    for kw in (dict(sputter=7), dict(coupling=2), dict(species_x=5), dict(storage=9)):
        with pytest.raises(lbm.LbmError) as e:
            _create(vox, **kw)
        assert e.value.status == lbm.LBM_EUNSUPPORTED


def test_null_arguments():
    L = lbm.library()
    out = ctypes.c_void_p(1)
    st = L.lbm_create(None, 0.0, 1.0, None, None, ctypes.byref(out))
    assert st == lbm.LBM_EINVAL and out.value is None
    assert b"NULL" in L.lbm_last_error(None)
    assert L.lbm_step(None, 1) == lbm.LBM_EINVAL
    L.lbm_destroy(None)  # no-op


@pytest.mark.parametrize("args, msg", [
    ((None, 1024, 4, 4, 4, 8), b"NULL"),
    ((4096, 1024, 0, 4, 4, 8), b">= 1"),
    ((4096, 1024, 4, 70000, 4, 8), b"65535"),
    ((4096, 1024, 1024, 1024, 512, 8), b"2^27"),
    ((4096, 1024, 4, 4, 4, 12), b"pair_bytes"),
    ((4100, 1024, 4, 4, 4, 8), b"aligned"),
    ((4096, 4096 + 64, 4, 4, 4, 8), b"overlap"),
])
def test_stream_pull_rejects_invalid_arguments_before_device_work(args, msg):
    """The checks come before any HIP call, so they run without a GPU (the
    addresses are never dereferenced)."""
    L = lbm.library()
    dst, src, nx, ny, nz, pb = args
    assert L.lbm_stream_pull(dst, src, nx, ny, nz, pb, None) == lbm.LBM_EINVAL
    assert msg in L.lbm_last_error(None)


def _batch_args(n, storages=None, taus=None):
    geoms = (lbm.lbm_geometry * max(n, 1))()
    bcs = (lbm.lbm_bc * max(n, 1))()
    vox = np.zeros((4, 4, 8), np.uint8)
    for i in range(n):
        geoms[i] = lbm.lbm_geometry(8, 4, 4, 0, vox.ctypes.data, 4.0)
        bcs[i] = lbm._bc(storage=(storages[i] if storages else 0))
    da = (ctypes.c_double * max(n, 1))(*([1.0] * n))
    tau = (ctypes.c_double * (2 * max(n, 1)))()
    for i in range(n):
        tau[2 * i], tau[2 * i + 1] = (taus[i] if taus else (0.8, 0.7))
    return vox, geoms, da, tau, bcs


def test_batch_rejects_invalid_arguments_before_device_work():
    L = lbm.library()
    out = ctypes.c_void_p(1)
    vox, geoms, da, tau, bcs = _batch_args(3)
    assert L.lbm_batch_create(0, geoms, None, da, tau, bcs, None, ctypes.byref(out)) == lbm.LBM_EINVAL
    assert out.value is None and b"n >= 1" in L.lbm_batch_last_error(None)
    assert L.lbm_batch_create(3, geoms, None, None, tau, bcs, None, ctypes.byref(out)) == lbm.LBM_EINVAL
    # every sample must share storage, sputter, coupling and species_x
    vox, geoms, da, tau, bcs = _batch_args(3, storages=[0, 1, 0])
    assert L.lbm_batch_create(3, geoms, None, da, tau, bcs, None, ctypes.byref(out)) == lbm.LBM_EINVAL
    assert b"sample 1" in L.lbm_batch_last_error(None)
    # a sample's own parameters are checked by lbm_create; the message names it
    vox, geoms, da, tau, bcs = _batch_args(2, taus=[(0.4, 0.7), (0.8, 0.7)])
    assert L.lbm_batch_create(2, geoms, None, da, tau, bcs, None, ctypes.byref(out)) == lbm.LBM_EINVAL
    assert b"sample 0" in L.lbm_batch_last_error(None) and b"tau" in L.lbm_batch_last_error(None)
    assert L.lbm_batch_step(None, 1) == lbm.LBM_EINVAL
    assert L.lbm_batch_set_graph(None, 1) == lbm.LBM_EINVAL
    L.lbm_batch_destroy(None)  # no-op


def test_product_lattice_needs_passive_coupling():
    """The product lattice is advected by the carrier (PASSIVE); asking for it
    with BARYCENTRIC coupling is rejected before any device work."""
    vox = np.zeros((4, 4, 8), np.uint8)
    with pytest.raises(lbm.LbmError) as e:
        _create(vox, product=True, coupling=lbm.COUPLE_BARYCENTRIC)
    assert e.value.status == lbm.LBM_EUNSUPPORTED
    assert "PASSIVE" in str(e.value)


def test_inspect_counts_the_product_buffers():
    """The planned device bytes grow by the product lattice's buffers: two
    population buffers of 19 nfp elements, E_P, In_P, Acc_P and partials."""
    from paper_1607_02874_amd import inputs

    vox = inputs.PLAIN_32.voxels()
    a = lbm.inspect(vox, 1.0, tau=(0.8, 0.7), pore_size=4.0)
    b = lbm.inspect(vox, 1.0, tau=(0.8, 0.7), pore_size=4.0, product=True, p_stick_product=0.2)
    nfp = (a["n_fluid"] + 1 + 127) // 128 * 128
    grow = b["device_bytes"] - a["device_bytes"]
    assert grow >= (38 * nfp + a["n_interface"]) * 4 + 2 * a["n_interface"] * 8
    assert grow < (38 * nfp + a["n_interface"]) * 4 + 2 * a["n_interface"] * 8 + 64 * 1024


def test_stochastic_sputter_without_product_lattice():
    vox = np.zeros((4, 4, 8), np.uint8)
    with pytest.raises(lbm.LbmError) as e:
        _create(vox, product=True, sputter=lbm.SPUTTER_STOCHASTIC)
    assert e.value.status == lbm.LBM_EUNSUPPORTED


def test_inspect_counts_the_stochastic_slots():
    """STOCHASTIC keeps 18 In and emission slots per interface node."""
    from paper_1607_02874_amd import inputs

    vox = inputs.PLAIN_32.voxels()
    a = lbm.inspect(vox, 1.0, tau=(0.8, 0.7), pore_size=4.0)
    b = lbm.inspect(vox, 1.0, tau=(0.8, 0.7), pore_size=4.0, sputter=lbm.SPUTTER_STOCHASTIC)
    grow = b["device_bytes"] - a["device_bytes"]
    assert abs(grow - 17 * a["n_interface"] * (8 + 4)) < 1024
