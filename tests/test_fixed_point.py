"""The kernels' fixed-point In(k) encoder and stochastic-rounding words,
compiled for the host from the same header the kernels include
(paper_1607_02874_amd/csrc/fixed_point.h) and checked on the CPU.

- term(x, 2^S) - MAGIC_BITS == round-to-nearest(x 2^S) up to |x 2^S| < 2^51,
  and the pattern is poisoned at and beyond 2^51 and for NaN / Inf;
- a sum of up to 18 terms (the most one interface node receives per step)
  that holds 1..18 poisoned terms is out of range for the reader, in both
  forms the kernels use (patterns minus b MAGIC_BITS, and terms stored
  minus MAGIC_BITS), whatever the in-range terms beside them;
- rounding words: nearest mode is 0x80000000 for every word; stochastic
  words have uniform top bits, differ between steps and seeds, and drive an
  emulation of the hardware's rounding rule (top bits of the word added to
  the discarded bits) to an unbiased mean.
"""

import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1607_02874_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdint>
#include <cmath>
#include "fixed_point.h"
using namespace lbmfx;
int main() {
    const double S = std::ldexp(1.0, 40);
    // encoder near the edge of its window
    const double ks[] = {0.0, 1.0, -1.0, 12345.25, -12345.75, 2251799813685247.0, -2251799813685247.0,
                         2251799813685248.0, -2251799813685248.0, 4503599627370496.0, 1e30, -1e30};
    for (double k : ks) {
        const unsigned long long t = term(k / S, S);
        const bool poisoned = t == POISON;
        const long long got = (long long)(t - MAGIC_BITS);
        std::printf("term %.17g %d %lld\n", k, poisoned ? 1 : 0, poisoned ? 0ll : got);
    }
    std::printf("nan %d\n", term(std::nan(""), S) == POISON ? 1 : 0);
    std::printf("inf %d\n", term(INFINITY, S) == POISON ? 1 : 0);
    // poisoned sums: m poisoned terms among b = 18, the others at both extremes
    int bad = 0;
    for (int m = 1; m <= 18; ++m)
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            unsigned long long pat = 0, sto = 0;
            for (int j = 0; j < 18; ++j) {
                const unsigned long long t = j < m ? POISON : term(sgn * 2251799813685247.0 / S, S);
                pat += t;
                sto += t - MAGIC_BITS;
            }
            if (sum_in_range((long long)(pat - 18ull * MAGIC_BITS))) ++bad;
            if (sum_in_range((long long)sto)) ++bad;
        }
    std::printf("poison_in_range %d\n", bad);
    // 16 terms at the edge of the window still read back in range
    unsigned long long pat = 0;
    for (int j = 0; j < 16; ++j) pat += term(2251799813685247.0 / S, S);
    std::printf("extreme_in_range %d\n", sum_in_range((long long)(pat - 16ull * MAGIC_BITS)) ? 1 : 0);
    // rounding words
    const RoundWords nr = round_words(false, 123u, 77u);
    int nearest_ok = 1;
    for (int t = 0; t < 64; ++t) nearest_ok &= nr.at(t) == ROUND_NEAREST_BITS;
    std::printf("nearest %d\n", nearest_ok);
    std::printf("keys %u %u %u %u\n", round_key(1, 0, 0), round_key(2, 0, 0), round_key(1, 5, 0), round_key(1, 0, 1));
    for (uint32_t n = 0; n < 4096; ++n) {
        const RoundWords w = round_words(true, round_key(7, 42, 0), n);
        for (int t = 0; t < 38; t += 37) std::printf("w %u\n", w.at(t));
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver_output(tmp_path_factory):
    d = tmp_path_factory.mktemp("fx")
    src = d / "fx.cpp"
    exe = d / "fx"
    src.write_text(DRIVER)
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-I", CSRC, str(src), "-o", str(exe)],
                   check=True)
    return subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines()


def _lines(out, tag):
    return [line.split()[1:] for line in out if line.split()[0] == tag]


def test_term_is_exact_inside_the_window_and_poisoned_outside(driver_output):
    rows = _lines(driver_output, "term")
    for k, poisoned, got in rows:
        k, poisoned, got = float(k), int(poisoned), int(got)
        if abs(k) < 2.0 ** 51:
            assert poisoned == 0 and got == round(k), (k, got)
        else:
            assert poisoned == 1, k
    assert _lines(driver_output, "nan") == [["1"]]
    assert _lines(driver_output, "inf") == [["1"]]


def test_poisoned_sums_are_out_of_range(driver_output):
    assert _lines(driver_output, "poison_in_range") == [["0"]]
    assert _lines(driver_output, "extreme_in_range") == [["1"]]


def test_rounding_words(driver_output):
    assert _lines(driver_output, "nearest") == [["1"]]
    keys = [int(v) for v in _lines(driver_output, "keys")[0]]
    assert len(set(keys)) == 4  # steps, seeds and salts give different keys
    words = np.array([int(v[0]) for v in _lines(driver_output, "w")], dtype=np.uint64)
    assert words.size == 8192
    for bits in (13, 16):  # FP16 and BF16 use the top 13 or 16 bits
        top = (words >> np.uint64(32 - bits)).astype(np.float64) / 2.0 ** bits
        # uniform on [0, 1): mean 1/2, variance 1/12, 16 equal-width bins
        assert abs(top.mean() - 0.5) < 0.015
        assert abs(top.var() - 1.0 / 12.0) < 0.004
        counts = np.histogram(top, bins=16, range=(0.0, 1.0))[0]
        chi2 = float(((counts - words.size / 16) ** 2 / (words.size / 16)).sum())
        assert chi2 < 40.0  # 15 degrees of freedom; p ~ 5e-4 at 40
        # emulated hardware rule: round the magnitude up when the discarded
        # fraction plus the top bits of the word carry past one unit
        for frac in (0.1, 0.37, 0.5, 0.93):
            up = (frac + top) >= 1.0
            assert abs(up.mean() - frac) < 0.02, (bits, frac, up.mean())
