"""The seeded input generator: exact porosity, determinism, gas buffers."""

import numpy as np
import pytest

from paper_1607_02874_amd import inputs


@pytest.mark.parametrize("shape,phi,ell", [((20, 16, 24), 0.65, 4.0), ((8, 8, 8), 0.5, 2.0),
                                           ((10, 12, 9), 0.75, 3.0)])
def test_grf_porosity_is_exact(shape, phi, ell):
    solid = inputs.grf_solid_mask(shape, phi, ell, 11)
    n = np.prod(shape)
    assert solid.sum() == int(round((1 - phi) * n))


def test_seeded_geometry_is_deterministic():
    a = inputs.PLAIN_32.voxels()
    b = inputs.PLAIN_32.voxels()
    assert inputs.sha256(a) == inputs.sha256(b)
    c = inputs.porous_slab(32, 32, 32, 0.65, 4.0, 1001)
    assert inputs.sha256(a) != inputs.sha256(c)


def test_buffers_are_gas_and_solid_is_catalytic():
    v = inputs.PLAIN_32.voxels()
    assert (v[:, :, :4] == inputs.FLUID).all() and (v[:, :, -4:] == inputs.FLUID).all()
    assert set(np.unique(v).tolist()) == {inputs.FLUID, inputs.CATALYTIC}
    block = v[:, :, 4:28]
    assert (block == inputs.FLUID).mean() == pytest.approx(0.65, abs=1e-4)


def test_field_correlation_length_controls_grain():
    """Longer correlation length gives fewer gas/solid faces per voxel."""
    def faces(ell):
        s = inputs.grf_solid_mask((32, 32, 32), 0.6, ell, 3)
        return sum((s != np.roll(s, 1, a)).mean() for a in range(3))
    assert faces(8.0) < faces(4.0) < faces(2.0)


def test_crop_forces_outlet_gas():
    v = inputs.porous_slab(40, 20, 20, 0.6, 3.0, 9)
    c = inputs.crop(v, 24, 16, 12)
    assert c.shape == (12, 16, 24)
    assert (c[:, :, -4:] == 0).all()
    assert np.array_equal(c[:, :, :20], v[:12, :16, :20])


@pytest.mark.parametrize("w", [6, 10, 20, 30])
def test_disk_ingot_follows_the_papers_recipe(w):
    """The 2-D reactor geometry: a (1, 500, 250) map, a catalytic ingot w
    along x and 200 across, centred, porosity 0.70 +- 0.005 inside it, one
    inert wall row, gas elsewhere; seeded, so deterministic."""
    vox = inputs.disk_ingot(w, seed=w)
    assert vox.shape == (1, 500, 250)
    x0, y0 = (250 - w) // 2, 150
    block = vox[0, y0:y0 + 200, x0:x0 + w]
    assert abs((block == inputs.FLUID).mean() - 0.70) <= 0.005 + 1e-12
    assert set(np.unique(block)) <= {inputs.FLUID, inputs.CATALYTIC}
    outside = vox[0].copy()
    outside[y0:y0 + 200, x0:x0 + w] = inputs.FLUID
    assert (outside[0] == inputs.INERT).all() and (outside[1:] == inputs.FLUID).all()
    assert np.array_equal(vox, inputs.disk_ingot(w, seed=w))
