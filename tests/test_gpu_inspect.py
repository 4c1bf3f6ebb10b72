"""lbm_inspect plans, on the host, the device memory lbm_create then
allocates: for every option the planned figure (each buffer rounded up to
256 B) is at most 256 B per buffer above what the context really holds."""

import pytest

from paper_1607_02874_amd import inputs, lbm

pytestmark = pytest.mark.gpu

CONFIGS = [
    dict(),
    dict(storage=lbm.STORE_F16),
    dict(product=True, p_stick_product=0.2),
    dict(sputter=lbm.SPUTTER_STOCHASTIC, seed=5),
    dict(wall_diffuse=0.5, species_x=lbm.XBC_INFLOW),
    dict(product=True, storage=lbm.STORE_F64),
]


@pytest.mark.parametrize("kw", CONFIGS)
def test_planned_device_bytes_match_the_context(kw):
    vox = inputs.PLAIN_32.voxels()
    args = dict(da=1.0, tau=(0.8, 0.7), pore_size=4.0)
    planned = lbm.inspect(vox, **args, **kw)["device_bytes"]
    with lbm.Sim(vox, **args, **kw) as s:
        held = s.info()["device_bytes"]
    assert 0 <= planned - held < 256 * 24, (kw, planned, held)
