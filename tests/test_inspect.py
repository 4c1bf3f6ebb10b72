"""The host-side preprocessing of the C ABI, through lbm_inspect (no GPU):
parameter maps against the oracle's, and node, interface and link counts
against the oracle's link counts and a brute-force recount."""

import numpy as np
import pytest

import oracle
from paper_1607_02874_amd import inputs, lbm


def brute_force_links(vox, periodic_x):
    """b(k) per voxel: for each catalytic voxel, the number of directions j
    whose source k - c_j is a gas voxel (y and z periodic; x periodic only when
    asked)."""
    c, _, _ = oracle.d3q19()
    nz, ny, nx = vox.shape
    b = np.zeros(vox.shape, np.int64)
    for z, y, x in zip(*np.nonzero(vox == inputs.CATALYTIC)):
        for j in range(1, 19):
            xs = x - c[j][0]
            if not 0 <= xs < nx:
                if not periodic_x:
                    continue
                xs %= nx
            if vox[(z - c[j][2]) % nz, (y - c[j][1]) % ny, xs] == inputs.FLUID:
                b[z, y, x] += 1
    return b


GEOMETRIES = {
    "plain32": lambda: inputs.PLAIN_32.voxels(),
    "ragged65": lambda: inputs.porous_slab(65, 12, 7, 0.6, 2.5, 5),
    "slab": lambda: inputs.reactive_slab(9, ny=3, nz=2),
    "mixed": lambda: np.where(inputs.porous_slab(40, 10, 9, 0.6, 3.0, 8) == inputs.CATALYTIC,
                              np.uint8(inputs.INERT), inputs.porous_slab(40, 10, 9, 0.6, 3.0, 8)).astype(np.uint8),
}


@pytest.mark.parametrize("name", sorted(GEOMETRIES))
@pytest.mark.parametrize("species_x", [lbm.XBC_RESERVOIR, lbm.XBC_PERIODIC])
def test_counts_match_oracle_and_brute_force(name, species_x):
    vox = GEOMETRIES[name]()
    if name == "mixed":  # inert and catalytic solid side by side
        vox = vox.copy()
        vox[:, ::2, 20:30][vox[:, ::2, 20:30] == inputs.INERT] = inputs.CATALYTIC
    info = lbm.inspect(vox, da=1.0, tau=(0.8, 0.7), pore_size=4.0, species_x=species_x)
    o = oracle.Oracle(vox, species_x=species_x)
    b_or = o.link_counts().astype(np.int64)
    o.close()
    b_bf = brute_force_links(vox, species_x == lbm.XBC_PERIODIC)
    assert np.array_equal(b_or, b_bf)
    assert info["n_nodes"] == vox.size
    assert info["n_fluid"] == int((vox == inputs.FLUID).sum())
    assert info["n_interface"] == int((b_bf > 0).sum())
    assert info["n_catalytic_links"] == int(b_bf.sum())


def test_parameter_maps_match_oracle():
    vox = inputs.PLAIN_32.voxels()
    for delta in (3.0, 8.0):
        for da in (0.05, 0.4, 1.0, 10.0, float("inf")):
            info = lbm.inspect(vox, da=da, tau=(0.8, 0.7), pore_size=delta)
            p, clamped = oracle.p_from_da(da, delta)
            assert info["p"] == pytest.approx(p, rel=1e-15, abs=0.0)
            assert bool(info["p_clamped"]) == bool(clamped)
        for kn in (0.05, 0.674, 2.0):
            info = lbm.inspect(vox, da=1.0, kn=kn, pore_size=delta)
            assert info["tau_gas"] == pytest.approx(oracle.tau_from_kn(kn, delta), rel=1e-15)
            assert info["tau_species"] == info["tau_gas"]  # equal for all species unless given
            assert info["kn"] == pytest.approx(kn, rel=1e-12)
        info = lbm.inspect(vox, da=1.0, tau=(0.9, 0.0), pore_size=delta)
        assert info["kn"] == pytest.approx(oracle.kn_from_tau(0.9, delta), rel=1e-15)


def test_inspect_applies_create_argument_checks():
    vox = np.zeros((4, 4, 8), np.uint8)
    for kw in (dict(da=0.0), dict(tau=(0.4, 0.7)), dict(p_stick=2.0), dict(kn=0.3, tau=(0.8, 0.7))):
        args = dict(da=1.0, tau=(0.8, 0.7), pore_size=4.0)
        args.update(kw)
        with pytest.raises(lbm.LbmError) as e:
            lbm.inspect(vox, **args)
        assert e.value.status == lbm.LBM_EINVAL
    vox[0, 0, 0] = 7
    with pytest.raises(lbm.LbmError) as e:
        lbm.inspect(vox, da=1.0, tau=(0.8, 0.7))
    assert e.value.status == lbm.LBM_EINVAL and "voxel" in str(e.value)


def test_planned_device_bytes_scale_with_storage():
    vox = inputs.PLAIN_32.voxels()
    by = {st: lbm.inspect(vox, da=1.0, tau=(0.8, 0.7), storage=st)["device_bytes"]
          for st in (lbm.STORE_F16, lbm.STORE_F32, lbm.STORE_F64)}
    nf = int((vox == inputs.FLUID).sum())
    # the population buffers dominate: 76 arrays of >= n_fluid elements
    assert by[lbm.STORE_F32] - by[lbm.STORE_F16] >= 76 * nf * 2
    assert by[lbm.STORE_F64] - by[lbm.STORE_F32] >= 76 * nf * 4


def test_inspect_d2q9_counts_match_the_oracle():
    """lbm_inspect of a D2Q9 plane (host only): gas nodes, interface nodes and
    links as the D2Q9 oracle counts them (b(k) <= 8), and the device bytes of
    the plane's arrays."""
    import oracle

    vox = inputs.disk_ingot(10, h=60, length=80, width=120, seed=2)
    for xbc, obc in ((lbm.XBC_INFLOW, oracle.XINFLOW), (lbm.XBC_PERIODIC, oracle.XPERIODIC)):
        for product in (False, True):
            info = lbm.inspect(vox, 1.0, tau=(4.0, 4.0), pore_size=3.0, species_x=xbc, storage=3, product=product,
                               lattice=lbm.LATTICE_D2Q9)
            b = oracle.Oracle(vox, species_x=obc, lattice="D2Q9").link_counts()
            assert info["n_nodes"] == vox.size
            assert info["n_fluid"] == int((vox == inputs.FLUID).sum())
            assert info["n_interface"] == int((b > 0).sum())
            assert info["n_catalytic_links"] == int(b.sum(dtype=np.int64))
            assert b.max() <= 8
            lat = 3 if product else 2
            assert info["device_bytes"] >= lat * 3 * 9 * vox.size * 8
