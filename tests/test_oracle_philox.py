"""Pins of the oracle's Philox4x32-10 and its uniform / normal draws.

The float64 oracle and the binary32 mirror are both checked against rocRAND's
own Philox4x32-10 engine (an independent implementation shipped as readable
source with ROCm), compiled here for the host.
"""

import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import philox as ph
from oracle import seed as sd

HERE = os.path.dirname(os.path.abspath(__file__))


def _xcheck_binary(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("pxc") / "pxc")
    subprocess.check_call([hipcc, "--offload-host-only", "-O1", "-o", out,
                           os.path.join(HERE, "golden", "philox_xcheck.cpp")])
    return out


@pytest.fixture(scope="module")
def xcheck(tmp_path_factory):
    return _xcheck_binary(tmp_path_factory)


def test_philox_matches_rocrand_engine(xcheck, ra):
    rng = np.random.default_rng(1234)
    n = 20000
    words = rng.integers(0, 2 ** 32, size=(n, 6), dtype=np.uint64)
    # include the all-zero and all-ones corners
    words[0] = 0
    words[1] = 0xFFFFFFFF
    text = "\n".join(" ".join(f"{int(v):x}" for v in row) for row in words) + "\n"
    res = subprocess.run([xcheck], input=text, capture_output=True, text=True, check=True)
    ref = np.array([[int(t, 16) for t in line.split()] for line in res.stdout.strip().splitlines()],
                   dtype=np.uint64)
    got = np.stack(ph.philox4x32_10(*[words[:, k] for k in range(6)]), axis=1).astype(np.uint64)
    assert np.array_equal(got, ref)
    for k in range(0, n, 997):
        w = ra.philox(words[k, :4], words[k, 4:])
        assert np.array_equal(w.astype(np.uint64), ref[k])


def test_philox_bit_balance():
    w = np.stack(ph.draw(np.arange(1 << 16, dtype=np.uint64), 0, 7, 99)).reshape(-1)
    bits = ((w[:, None] >> np.arange(32, dtype=np.uint32)) & 1).mean(axis=0)
    # 2^18 words per bit position: std of the mean is 0.001
    assert np.all(np.abs(bits - 0.5) < 0.006)


def test_uniform24_exact_grid():
    w = np.array([0, 255, 256, 0xFFFFFFFF, 0x80000000], dtype=np.uint32)
    u = ph.uniform24(w)
    assert np.array_equal(u * 2 ** 24, np.floor(u * 2 ** 24))
    assert u[0] == 0.0 and u[1] == 0.0 and u[2] == 2.0 ** -24
    assert u[3] == 1.0 - 2.0 ** -24 and u[4] == 0.5
    uo = ph.uniform24_open0(w)
    assert uo.min() > 0 and uo[3] == 1.0


def test_counter_fields_are_independent():
    base = np.stack(ph.draw(np.arange(64, dtype=np.uint64), 0, 3, 11))
    for other in (ph.draw(np.arange(64, dtype=np.uint64), 1, 3, 11),
                  ph.draw(np.arange(64, dtype=np.uint64), 0, 4, 11),
                  ph.draw(np.arange(64, dtype=np.uint64), 0, 3, 12),
                  ph.draw(np.arange(64, dtype=np.uint64), 0, 3 + (1 << 32), 11)):
        assert not np.any(np.stack(other) == base)


def test_box_muller_moments():
    n = 200000
    i = np.arange(n, dtype=np.uint64)
    h = ph.draw(i, ph.STREAM_PHOTO, 5, 17)
    z = sd.box_muller_cos(h[1], h[2])
    assert abs(z.mean()) < 5 * 1 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 0.02
    from scipy import stats
    assert stats.kstest(z, "norm").pvalue > 1e-3
