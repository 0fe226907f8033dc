"""The FP64 Box-Muller transform of the HIP path (table-driven logarithm and
Taylor sine/cosine of normal64.h), built for the host and checked on the CPU:

* ln u1 and sin/cos(pi x) against 40-digit references (Python's decimal
  module: its ln, and the sine and cosine series after an exact reduction),
  over every word class that matters (u1 = 1, u1 = 2^-32, the neighbours of
  powers of two and of the table's grid points, quarter-turn boundaries of
  the angle) and a seeded random sample;
* the two normals against the oracle's transform (numpy log, cos and sin of
  2 pi u2) on 200000 random word pairs.
"""
import os
import shutil
import subprocess
from decimal import Decimal, getcontext

import numpy as np
import pytest

from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1212_6427_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PROGRAM = r'''
#include "normal64.h"
#include <cstdio>
#include <vector>
// reads n, then n (wa, wb) pairs; writes ln u1, sin(pi x), cos(pi x), z0, z1
int main() {
    double inv[icm::kLogTab], lnf[icm::kLogTab];
    for (int j = 0; j < icm::kLogTab; ++j) icm::log_table_entry(j, inv, lnf);
    unsigned long long n = 0;
    if (fread(&n, sizeof(n), 1, stdin) != 1) return 1;
    std::vector<uint32_t> w(2 * n);
    if (fread(w.data(), sizeof(uint32_t), 2 * n, stdin) != 2 * n) return 1;
    std::vector<double> out(5 * n);
    for (unsigned long long i = 0; i < n; ++i) {
        const uint32_t wa = w[2 * i], wb = w[2 * i + 1];
        const double u1 = ((double)wa + 1.0) * 2.3283064365386963e-10;
        const double x = (double)wb * 4.6566128730773926e-10;
        out[5 * i] = icm::log_unit(u1, inv, lnf);
        icm::sincospi_unit(x, &out[5 * i + 1], &out[5 * i + 2]);
        icm::box_muller64(wa, wb, inv, lnf, out[5 * i + 3], out[5 * i + 4]);
    }
    fwrite(out.data(), sizeof(double), out.size(), stdout);
    return 0;
}
'''


@pytest.fixture(scope="module")
def run(tmp_path_factory):
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("normal64")
    src = os.path.join(d, "normal64_host.hip")
    exe = os.path.join(d, "normal64_host")
    with open(src, "w") as fh:
        fh.write(PROGRAM)
    r = subprocess.run([HIPCC, "--cuda-host-only", "-O2", "-std=c++17", "-I" + CSRC, src, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr

    def go(wa, wb):
        wa = np.asarray(wa, dtype=np.uint32)
        wb = np.asarray(wb, dtype=np.uint32)
        pairs = np.stack([wa, wb], axis=1).ravel()
        inp = np.uint64(len(wa)).tobytes() + pairs.tobytes()
        p = subprocess.run([exe], input=inp, capture_output=True)
        assert p.returncode == 0
        return np.frombuffer(p.stdout, dtype=np.float64).reshape(-1, 5)
    return go


getcontext().prec = 45
PI = Decimal("3.141592653589793238462643383279502884197169399375105820974944592")


def dec_ln_u1(wa):
    return ((Decimal(int(wa)) + 1) / Decimal(2) ** 32).ln()


def dec_sincospi(wb):
    """sin(pi x), cos(pi x) for x = wb 2^-31, reduced exactly to pi t + q pi/2."""
    x2 = Decimal(int(wb)) / Decimal(2) ** 30          # 2x, exact
    q = int((x2 + Decimal("0.5")).to_integral_value(rounding="ROUND_FLOOR"))
    t = (x2 - q) / 2                                  # x - q/2, exact
    a = PI * t
    s, c, term_s, term_c, k = Decimal(0), Decimal(0), a, Decimal(1), 0
    while abs(term_s) > Decimal("1e-44") or abs(term_c) > Decimal("1e-44"):
        s += term_s
        c += term_c
        term_s = -term_s * a * a / ((2 * k + 2) * (2 * k + 3))
        term_c = -term_c * a * a / ((2 * k + 1) * (2 * k + 2))
        k += 1
    n = q % 4
    sa, ca = (c, s) if n % 2 else (s, c)
    return (-sa if n >= 2 else sa), (-ca if n in (1, 2) else ca)


def special_words():
    w = {0, 1, 2, 3, 2 ** 31 - 1, 2 ** 31, 2 ** 31 + 1, 2 ** 32 - 3, 2 ** 32 - 2, 2 ** 32 - 1}
    for e in range(1, 32):                           # neighbours of powers of two
        for d in (-1, 0, 1):
            if 0 <= 2 ** e + d - 1 < 2 ** 32:
                w.add(2 ** e + d - 1)
    # u1 where round(256 m) changes: u1 = (j + 1/2) / 256 in [3/4, 1) and
    # u1 = (j + 1/2) / 512 in [1/2, 3/4) (m = 2 u1 there)
    for j in range(192, 384, 5):
        for shift in (23, 22):
            for d in (-2, -1, 0, 1):
                v = (2 * j + 1) * 2 ** shift - 1 + d
                if 0 <= v < 2 ** 32:
                    w.add(v)
    for k in range(9):                               # eighth turns (x = k / 4): the reduction's edges
        for d in (-1, 0, 1):
            v = k * 2 ** 29 + d
            if 0 <= v < 2 ** 32:
                w.add(v)
    return np.array(sorted(w), dtype=np.uint64).astype(np.uint32)


def test_log_unit_matches_40_digits(run):
    rng = np.random.default_rng(11)
    wa = np.concatenate([special_words(), rng.integers(0, 2 ** 32, 1500, dtype=np.uint64).astype(np.uint32)])
    got = run(wa, np.zeros_like(wa))[:, 0]
    worst = 0.0
    for w, g in zip(wa, got):
        ref = dec_ln_u1(w)
        if ref == 0:
            assert g == 0.0
            continue
        rel = abs((Decimal(float(g)) - ref) / ref)
        worst = max(worst, float(rel))
    print("ln u1: worst relative error %.2e" % worst)
    assert worst < 4e-16


def test_sincospi_matches_40_digits(run):
    rng = np.random.default_rng(12)
    wb = np.concatenate([special_words(), rng.integers(0, 2 ** 32, 1500, dtype=np.uint64).astype(np.uint32)])
    got = run(np.zeros_like(wb), wb)
    worst = 0.0
    for w, s, c in zip(wb, got[:, 1], got[:, 2]):
        rs, rc = dec_sincospi(w)
        worst = max(worst, float(abs(Decimal(float(s)) - rs)), float(abs(Decimal(float(c)) - rc)))
        if w % (2 ** 30) == 0:   # quarter turns (x = k / 2) are exact
            assert (s, c) == (float(rs), float(rc)), (w, s, c)
    print("sin/cos: worst absolute error %.2e" % worst)
    assert worst < 3e-16


def test_normals_match_the_oracle_transform(run):
    rng = np.random.default_rng(13)
    n = 200000
    wa = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    wb = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    wa[:10] = [0, 1, 2 ** 31, 2 ** 32 - 2, 2 ** 32 - 1, 0, 2 ** 32 - 1, 5, 7, 9]
    wb[:10] = [0, 2 ** 30, 2 ** 31, 3 * 2 ** 30, 2 ** 32 - 1, 1, 2 ** 29, 2 ** 32 - 1, 0, 12345]
    got = run(wa, wb)
    z0, z1 = philox.box_muller(wa, wb)
    scale = np.maximum(1.0, np.hypot(z0, z1))
    err = np.max(np.maximum(np.abs(got[:, 3] - z0), np.abs(got[:, 4] - z1)) / scale)
    print("normals vs the oracle: worst %.2e" % err)
    # the oracle rounds 2 pi u2 before its cosine: up to ~1 ulp of the angle
    assert err < 2e-15
    # u1 = 1 gives radius 0 exactly
    assert got[4, 3] == 0.0 and got[4, 4] == 0.0
