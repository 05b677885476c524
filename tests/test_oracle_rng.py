"""Pins for the oracle's random streams (CPU only).

Philox4x32-10 is pinned to the published known-answer vectors and to
PyTorch's independent host implementation; the normal transform to its
distribution and its exact edge values; bf16 rounding to PyTorch's cast."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[:4], v[4:6], v[6:]))
    return rows


@pytest.mark.parametrize("ctr,key,want", _kat())
def test_philox_known_answers(ctr, key, want):
    assert list(oracle.philox(ctr, key)) == want


@pytest.fixture(scope="module")
def torch_philox(tmp_path_factory):
    import torch
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    exe = str(tmp_path_factory.mktemp("tp") / "torch_philox")
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", inc,
                    os.path.join(HERE, "helpers", "torch_philox.cpp"), "-o", exe], check=True)
    return exe


def test_philox_matches_torch_engine(torch_philox):
    rng = np.random.default_rng(123)
    cases = [list(rng.integers(0, 2 ** 32, 6, dtype=np.uint64)) for _ in range(200)]
    # counters as the simulation uses them: (k, trial, setting, stream)
    cases += [[k, t, s, st, 1, 0] for k in (0, 1, 999) for t in (0, 5, 2 ** 32 - 1)
              for s in (0, 63, 4095) for st in (0, 127, 0x40000000, 0xFFFFFFFF)]
    text = "".join("%x %x %x %x %x %x\n" % tuple(int(x) for x in c) for c in cases)
    out = subprocess.run([torch_philox], input=text, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for c, line in zip(cases, out):
        want = [int(x, 16) for x in line.split()]
        got = list(oracle.philox([int(x) for x in c[:4]], [int(x) for x in c[4:]]))
        assert got == want, (c, got, want)


def _words(n, seed=5):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2 ** 32, (n, 4), dtype=np.uint64).astype(np.uint32)


def test_normals64_distribution():
    w = _words(100_000)
    z = np.array([oracle.normals64(x) for x in w]).ravel()
    assert abs(z.mean()) < 4 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 4 * np.sqrt(2 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # the two outputs of one block are uncorrelated
    zz = np.array([oracle.normals64(x) for x in w[:50_000]])
    assert abs(np.corrcoef(zz[:, 0], zz[:, 1])[0, 1]) < 4 / np.sqrt(50_000)


def test_normals32_distribution():
    w = _words(100_000, seed=6)
    z = np.array([oracle.normals32(x) for x in w], np.float64).ravel()
    assert abs(z.mean()) < 4 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 4 * np.sqrt(2 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_normals_edge_words():
    # all-ones words give u = 1 exactly: log(1) = 0, so both normals are 0
    assert list(oracle.normals64([0xFFFFFFFF] * 4)) == [0.0, 0.0]
    assert list(oracle.normals32([0xFFFFFFFF] * 4)) == [0.0, 0.0]
    # all-zero words give the smallest uniform 2^-53 and the angle 2*pi*2^-53
    z = oracle.normals64([0, 0, 0, 0])
    rho = np.sqrt(-2 * np.log(2.0 ** -53))
    assert z[0] == pytest.approx(rho, rel=1e-15)
    assert abs(z[1]) < 1e-13
    # the FP32 path reads only the top 24 bits of words 1 and 3
    a = oracle.normals32([0x12345678, 0xABCDEF00, 0x0, 0x55555500])
    b = oracle.normals32([0x0, 0xABCDEFFF, 0xFFFFFFFF, 0x555555FF])
    assert list(a) == list(b)


def test_normals64_uses_53_bits_of_both_word_pairs():
    base = np.array([0x11111111, 0x22222222, 0x33333333, 0x44444444], np.uint32)
    z0 = oracle.normals64(base)
    for i, bit in ((0, 11), (2, 11), (1, 31), (3, 31)):
        w = base.copy()
        w[i] ^= np.uint32(1 << bit)
        assert not np.array_equal(oracle.normals64(w), z0)
    for i in (0, 2):  # the low 11 bits of words 0 and 2 are dropped
        w = base.copy()
        w[i] ^= np.uint32(1 << 10)
        assert np.array_equal(oracle.normals64(w), z0)


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(9)
    vals = np.concatenate([rng.normal(0, 1, 2000), rng.normal(0, 1e-3, 500),
                           [0.0, -0.0, 1.0, 1.00390625, 1.0078125, 1 + 3 * 2 ** -9,
                            3.4e38, -1e-40]])
    for v in vals:
        t = torch.tensor(v, dtype=torch.float64).float().to(torch.bfloat16)
        assert oracle.bf16_bits(v) == int(t.view(torch.int16).item()) & 0xFFFF, v
