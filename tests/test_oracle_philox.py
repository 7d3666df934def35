"""Pins of the oracle's Philox4x32-10 and of its uniform conversions.

Philox is not part of the paper (it stores a PCG state per thread, Sec. 3.2.3);
the generator is pinned to its published known-answer vectors, to a second
implementation in Python integers, and to the rocRAND library's engine.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import philox_py

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    return rows


def test_known_answer_vectors(orc):
    for w in _kat():
        out = orc.philox(np.array(w[:4], np.uint32), np.array(w[4:6], np.uint32))[0]
        assert [int(x) for x in out] == w[6:]
        assert philox_py.philox4x32_10(w[:4], w[4:6]) == w[6:]


def test_c_matches_python_integers(orc):
    g = np.random.default_rng(1)
    ctr = g.integers(0, 2**32, size=(400, 4), dtype=np.uint64).astype(np.uint32)
    key = g.integers(0, 2**32, size=(400, 2), dtype=np.uint64).astype(np.uint32)
    out = orc.philox(ctr, key)
    for i in range(ctr.shape[0]):
        assert philox_py.philox4x32_10(ctr[i], key[i]) == [int(x) for x in out[i]]


def test_matches_rocrand_engine(orc, tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "rr"
    subprocess.run([hipcc, "-O1", "--offload-arch=gfx950", "-I/opt/rocm/include",
                    os.path.join(HERE, "golden", "rocrand_philox_ref.hip"), "-o", str(exe)],
                   check=True, capture_output=True)
    g = np.random.default_rng(2)
    ctr = g.integers(0, 2**32, size=(300, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:, 1] &= (1 << 30) - 1      # the library's seek API takes 4*c1:c0 in 64 bits
    key = g.integers(0, 2**32, size=(300, 2), dtype=np.uint64).astype(np.uint32)
    inp = "\n".join(" ".join("%08x" % v for v in list(c) + list(k)) for c, k in zip(ctr, key))
    res = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True)
    lib_out = np.array([[int(x, 16) for x in l.split()] for l in res.stdout.split("\n") if l],
                       np.uint32)
    np.testing.assert_array_equal(orc.philox(ctr, key), lib_out)


def test_uniform_conversion(orc):
    # extremes and symmetry: u(x) + u(~x) = 1 exactly, v = 2u - 1 exactly, v != 0
    assert orc.u01(0) == 2.0 ** -24
    assert orc.u01(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    g = np.random.default_rng(3)
    for x in list(g.integers(0, 2**32, size=2000)) + [0, 511, 512, 0x7FFFFFFF, 0x80000000]:
        x = int(x)
        u = orc.u01(x)
        assert u == philox_py.u01(x)
        assert 0.0 < u < 1.0
        assert u + orc.u01(~x & 0xFFFFFFFF) == 1.0
        v = orc.v11(x)
        assert v == 2.0 * u - 1.0 and v != 0.0 and -1.0 < v < 1.0
        # the low 9 bits never reach the uniform
        assert orc.u01(x ^ 0x1FF) == u
