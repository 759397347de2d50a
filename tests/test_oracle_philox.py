"""Pins of the oracle's Philox4x32-10 and Box-Muller (CPU)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            lhs, rhs = line.split(":")
            rows.append(([int(v, 16) for v in lhs.split()],
                         [int(v, 16) for v in rhs.split()]))
    return rows


def test_random123_kat():
    for (c0, c1, c2, c3, k0, k1), expect in _kat():
        got = philox.philox4x32_10(c0, c1, c2, c3, k0, k1)
        assert [int(g) for g in got] == expect


@pytest.fixture(scope="module")
def rocrand_words(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND host pin")
    exe = str(tmp_path_factory.mktemp("rr") / "rr")
    subprocess.check_call([hipcc, "-O1", "--offload-host-only", "-o", exe,
                           os.path.join(HERE, "pins", "rocrand_philox_words.cpp")])

    def run(seed, stream, ctrs):
        out = subprocess.check_output([exe, str(seed), str(stream)] +
                                      [str(int(c)) for c in ctrs]).decode()
        return np.array([[int(v, 16) for v in l.split()] for l in out.splitlines()],
                        dtype=np.uint64)
    return run


@pytest.mark.parametrize("seed,stream", [(1234, 0), (1234, 1), (0xDEADBEEFCAFEF00D, 0),
                                         (7, 3), (2 ** 64 - 1, 2 ** 32 - 1)])
def test_words_match_rocrand(rocrand_words, seed, stream):
    rng = np.random.default_rng(5)
    ctrs = np.concatenate([np.arange(8), rng.integers(0, 2 ** 62, 40),
                           [2 ** 32 - 1, 2 ** 32, 2 ** 33 + 5, 4_294_967_296 * 4095]])
    ref = rocrand_words(seed, stream, ctrs)
    got = philox.words(seed, stream, ctrs.astype(np.uint64))
    np.testing.assert_array_equal(got, ref)


def test_uniforms_exact_and_open():
    w = np.concatenate([np.array([0, 511, 512, 2 ** 32 - 1, 2 ** 31], dtype=np.uint64),
                        np.random.default_rng(1).integers(0, 2 ** 32, 10000).astype(np.uint64)])
    u = philox.uniform_from_word(w)
    # exactly representable in FP32 (24 significant bits)
    assert np.all(u.astype(np.float32).astype(np.float64) == u)
    assert u[0] == 2.0 ** -24 and u[1] == 2.0 ** -24
    assert u[2] == 3 * 2.0 ** -24
    assert u[3] == 1.0 - 2.0 ** -24
    assert np.all((u > 0) & (u < 1))


def test_box_muller_moments():
    lin = np.arange(2 * 400_000, dtype=np.uint64)
    z1, z2 = philox.normal_pair(99, 0, lin)
    z = np.concatenate([z1, z2])
    assert abs(z.mean()) < 5 * 1 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    # kurtosis of a normal is 3
    assert abs(np.mean(z ** 4) - 3) < 0.03
    assert abs(np.corrcoef(z1, z2)[0, 1]) < 5 / np.sqrt(z1.size)


def test_normal_pair_word_selection():
    # lin and lin^1 share one Philox call: words (0,1) and (2,3)
    w = philox.words(11, 0, np.array([5], dtype=np.uint64))[0]
    z_even = philox.normal_pair(11, 0, np.array([10], dtype=np.uint64))
    z_odd = philox.normal_pair(11, 0, np.array([11], dtype=np.uint64))
    u = philox.uniform_from_word(w)
    e1, e2 = philox.box_muller(u[0], u[1])
    o1, o2 = philox.box_muller(u[2], u[3])
    assert z_even[0][0] == e1 and z_even[1][0] == e2
    assert z_odd[0][0] == o1 and z_odd[1][0] == o2
