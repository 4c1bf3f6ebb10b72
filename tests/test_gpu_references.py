"""The streaming references the sweep's bandwidth is reported against
(lbm_stream_copy, lbm_stream_pull): not part of the method, but their
results are checked so that the rates they give are those of the data
movement they claim.  The pull-streaming pass is checked element by element
against the D3Q19 permutation written out in numpy: ragged sizes (a partial
last block of 64 nodes, an x extent that is not a multiple of the 256-thread
block), every periodic wrap, and each pair size."""

import numpy as np
import pytest

from paper_1607_02874_amd import lbm

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _layout_index(n, i):
    """Element (node n, slot i) of the blocked layout."""
    return (n // 64) * 1216 + 64 * i + n % 64


def test_velocity_table_is_d3q19():
    c = np.asarray(lbm.D3Q19)
    assert c.shape == (19, 3) and len({tuple(v) for v in c}) == 19
    norms = (c * c).sum(axis=1)
    assert sorted(norms.tolist()) == [0] + [1] * 6 + [2] * 12


@pytest.mark.parametrize("nx, ny, nz", [(70, 9, 5), (300, 3, 2), (1, 1, 1), (64, 4, 4)])
@pytest.mark.parametrize("pair_bytes", [4, 8, 16])
def test_stream_pull_is_the_d3q19_permutation(nx, ny, nz, pair_bytes):
    lib = lbm.library()
    nodes = nx * ny * nz
    k = pair_bytes // 4  # 32-bit words per element
    n_elem = (nodes + 63) // 64 * 64 * 19
    rng = np.random.default_rng(nodes * 31 + pair_bytes)
    host = rng.integers(-2**31, 2**31 - 1, size=(n_elem, k), dtype=np.int64).astype(np.int32)
    src = torch.from_numpy(host.ravel()).to("cuda")
    dst = torch.zeros_like(src)
    stream = torch.cuda.current_stream()
    print(f"stream_pull {nx}x{ny}x{nz} pair_bytes={pair_bytes}", flush=True)
    assert lib.lbm_stream_pull(dst.data_ptr(), src.data_ptr(), nx, ny, nz, pair_bytes,
                               stream.cuda_stream) == lbm.LBM_OK
    torch.cuda.synchronize()
    got = dst.cpu().numpy().reshape(n_elem, k)

    want = np.zeros_like(host)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    n = (x + nx * (y + ny * z)).ravel()
    written = np.zeros(n_elem, bool)
    for i, (cx, cy, cz) in enumerate(lbm.D3Q19):
        m = ((x - cx) % nx + nx * ((y - cy) % ny + ny * ((z - cz) % nz))).ravel()
        want[_layout_index(n, i)] = host[_layout_index(m, i)]
        written[_layout_index(n, i)] = True
    assert np.array_equal(got, want)  # padding of the last block: never written, still zero
    assert written.sum() == 19 * nodes


def test_stream_copy_copies():
    lib = lbm.library()
    n = (1 << 20) + 48
    a = torch.randint(-2**31, 2**31 - 1, (n // 4,), dtype=torch.int32, device="cuda")
    b = torch.zeros_like(a)
    assert lib.lbm_stream_copy(b.data_ptr(), a.data_ptr(), n, torch.cuda.current_stream().cuda_stream) == lbm.LBM_OK
    torch.cuda.synchronize()
    assert torch.equal(a, b)
