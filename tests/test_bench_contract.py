"""Host-side parts of the benchmark's contract (no GPU needed)."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_options():
    """The product and STOCHASTIC figures add to the two-lattice one what
    their extra lattice or per-exit slots move."""
    sys.path.insert(0, ROOT)
    import bench

    info = dict(n_fluid=1000, n_nodes=1500, n_interface=100, n_catalytic_links=400)
    base = bench.algorithmic_bytes(info, 4)
    prod = bench.algorithmic_bytes(info, 4, product=True)
    stoch = bench.algorithmic_bytes(info, 4, stochastic=True)
    assert base["sweep"] == (76 * 1000 - 400) * 4 + 12 * 100 + 750
    assert prod["sweep"] - base["sweep"] == (38 * 1000 - 400) * 4 + 12 * 100
    assert stoch["sweep"] - base["sweep"] == (400 - 100) * 12
    assert stoch["interface"] == 20 * 100 + 20 * 400
