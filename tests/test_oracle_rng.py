"""Pins of the oracle's random numbers (CPU).

Philox4x32-10 is checked against rocRAND's own implementation of the published
generator (its header-only device API compiled for the host and run), and the
uniform maps against their edge values.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    d = tempfile.mkdtemp(prefix="philox_ref_")
    exe = os.path.join(d, "ref")
    subprocess.run([hipcc, "-O1", os.path.join(HERE, "rocrand_philox_ref.cpp"), "-o", exe],
                   check=True, capture_output=True, timeout=300)

    def run(queries):
        inp = "".join("%d %d %d %d\n" % q for q in queries)
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True,
                             timeout=60).stdout.split("\n")
        return [[int(w, 16) for w in line.split()] for line in out if line.strip()]

    yield run
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(oracle, rocrand_ref):
    # rocRAND keys Philox with the 64-bit seed, puts the subsequence in counter
    # words 2-3 and the block offset in words 0-1.
    rng = np.random.default_rng(3)
    queries, expect = [], []
    for _ in range(24):
        seed = int(rng.integers(0, 2 ** 63))
        sub = int(rng.integers(0, 2 ** 40))
        off = int(rng.integers(0, 2 ** 20)) * 4
        queries.append((seed, sub, off, 3))
        for i in range(3):
            blk = off // 4 + i
            ctr = [blk & 0xFFFFFFFF, blk >> 32, sub & 0xFFFFFFFF, sub >> 32]
            key = [seed & 0xFFFFFFFF, seed >> 32]
            expect.append([int(v) for v in oracle.philox(ctr, key)])
    queries.append((0, 0, 0, 1))
    expect.append([int(v) for v in oracle.philox([0, 0, 0, 0], [0, 0])])
    got = rocrand_ref(queries)
    assert got == expect


def test_philox_counter_fields_are_independent(oracle):
    # Changing any one counter word or key word changes the block.
    base = oracle.philox([5, 6, 7, 8], [9, 10])
    for i in range(4):
        ctr = [5, 6, 7, 8]
        ctr[i] += 1
        assert not np.array_equal(oracle.philox(ctr, [9, 10]), base)
    for i in range(2):
        key = [9, 10]
        key[i] += 1
        assert not np.array_equal(oracle.philox([5, 6, 7, 8], key), base)


def test_uniform_map_edges(oracle):
    # all-zero words: u_open = 2^-53 (never 0, so -log is finite), u_sel = 0
    uo, us = oracle.uniforms([0, 0, 0, 0])
    assert uo == 2.0 ** -53 and us == 0.0
    # all-one words: u_open = 1 exactly, u_sel = 1 - 2^-53 < 1
    uo, us = oracle.uniforms([0xFFFFFFFF] * 4)
    assert uo == 1.0 and us == 1.0 - 2.0 ** -53
    # the low 11 bits of each 64-bit word are dropped; word 1 / word 3 are the high halves
    uo, us = oracle.uniforms([0x7FF, 0, 0x7FF, 0])
    assert uo == 2.0 ** -53 and us == 0.0
    uo, us = oracle.uniforms([0, 0x80000000, 0, 0x80000000])
    assert uo == 0.5 + 2.0 ** -53 and us == 0.5


def test_uniforms_are_uniform(oracle):
    # chi-square over 32 bins for both uniforms from consecutive counters
    n = 20000
    uo = np.empty(n)
    us = np.empty(n)
    for i in range(n):
        uo[i], us[i] = oracle.uniforms(oracle.philox([i, 1, 2, 3], [11, 12]))
    for u in (uo, us):
        h, _ = np.histogram(u, bins=32, range=(0, 1))
        e = n / 32
        chi2 = ((h - e) ** 2 / e).sum()
        assert chi2 < 70  # 31 dof: p ~ 1e-4
