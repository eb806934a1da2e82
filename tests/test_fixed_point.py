"""The exact 64.64 fixed-point ParRep clock of the device code, compiled for
the host (the clock T_s of Alg. 1, Sec. II A, kept exact so that the horizon
and the burn-in time are crossed at one event whatever the summation order).

* fx_from(d) = floor(d 2^64) for 0 <= d < 2^52, and 2^52 for larger values
  and +inf (the holding time of an absorbing state), checked against exact
  rational arithmetic;
* the replica sums saturate: 4096 absorbing replicas (4096 x 2^52 = 2^64)
  wrap the plain 64-bit high word to 0, which would hide the horizon from
  the parallel step; the saturating sum equals min(exact sum, 2^52);
* the workgroup reductions' three-part sums (high words, and the two halves
  of the low words, summed over up to 1024 lanes in any order) joined by
  fx_join3 equal the saturating sum, with and without saturation.
"""
import math
import os
import random
import shutil
import subprocess
from fractions import Fraction

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SAT = 1 << 52


@pytest.fixture(scope="module")
def fx(tmp_path_factory):
    cxx = shutil.which("g++")
    if not cxx:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("fx") / "fx_host")
    subprocess.run([cxx, "-O2", "-std=c++17", "-ffp-contract=off", "-o", exe,
                    os.path.join(HERE, "fx_host.cpp")], check=True)

    def run(ds):
        out = subprocess.run([exe], input="\n".join(float.hex(d) for d in ds) + "\n",
                             capture_output=True, text=True, check=True).stdout.splitlines()
        vals = [tuple(int(w, 16) for w in line.split()) for line in out[:-4]]
        plain = tuple(int(w, 16) for w in out[-4].split()[1:])
        sat = tuple(int(w, 16) for w in out[-3].split()[1:])
        run.join3 = tuple(int(w, 16) for w in out[-2].split()[1:])
        run.sat1024 = tuple(int(w, 16) for w in out[-1].split()[1:])
        return vals, plain, sat
    return run


def _exact(d):
    if not d < 2.0 ** 52:
        return SAT << 64
    if not d > 0.0:
        return 0
    return math.floor(Fraction(d) * (1 << 64))


def test_fx_from_exact(fx):
    rng = random.Random(3)
    ds = [0.0, 2.0 ** -64, 2.0 ** -65, 1.0, 0.1, 2.0 ** 52, 2.0 ** 52 - 1.0, 2.0 ** 51, math.inf,
          1e300, 5e-324, 2.0 ** 52 * (1 - 2.0 ** -53)]
    ds += [rng.expovariate(1.0) * 10 ** rng.randint(-12, 12) for _ in range(3000)]
    vals, _, _ = fx(ds)
    for d, (hi, lo) in zip(ds, vals):
        assert (hi << 64) | lo == _exact(d), d


@pytest.mark.parametrize("n_inf", [1, 4095, 4096, 8192, 65536])
def test_replica_sum_saturates(fx, n_inf):
    # n_inf absorbing replicas (tau = +inf) among finite holding times
    rng = random.Random(n_inf)
    ds = [rng.expovariate(300.0) for _ in range(500)] + [math.inf] * n_inf
    rng.shuffle(ds)
    _, plain, sat = fx(ds)
    exact = sum(_exact(d) for d in ds)
    assert (sat[0] << 64) | sat[1] == min(exact, SAT << 64)
    assert sat[0] == SAT  # at least the horizon bound 2^51 < 2^52: the horizon is seen
    # the plain sum is the exact one modulo 2^128 (its high word wraps at 4096 x 2^52)
    assert (plain[0] << 64) | plain[1] == exact % (1 << 128)
    if n_inf % 4096 == 0:
        assert plain[0] < 2 ** 51  # wrapped below any horizon: what the saturation prevents


def test_finite_sums_are_exact(fx):
    rng = random.Random(11)
    ds = [rng.expovariate(1.0) * 10 ** rng.randint(-6, 3) for _ in range(65536)]
    _, plain, sat = fx(ds)
    exact = sum(_exact(d) for d in ds)
    assert (plain[0] << 64) | plain[1] == exact
    assert sat == plain


@pytest.mark.parametrize("case", ["small", "carries", "saturated", "one_inf", "empty_lo"])
def test_three_part_join_equals_saturating_sum(fx, case):
    rng = random.Random(case)
    if case == "small":
        ds = [rng.expovariate(300.0) for _ in range(1024)]
    elif case == "carries":  # low words near 2^64: the halves' sums carry into the high word
        ds = [1.0 - 2.0 ** -40 * rng.random() for _ in range(1024)]
    elif case == "saturated":  # 1024 absorbing lanes: 1024 x 2^52 in the high words
        ds = [math.inf] * 1024
    elif case == "one_inf":
        ds = [rng.expovariate(1.0) for _ in range(1023)] + [math.inf]
        rng.shuffle(ds)
    else:  # integral times only (low words 0) and one just below saturation
        ds = [float(rng.randint(0, 1000)) for _ in range(1023)] + [2.0 ** 52 - 2.0 ** 20]
    fx(ds)
    exact = sum(_exact(d) for d in ds[:1024])
    assert (fx.join3[0] << 64) | fx.join3[1] == min(exact, SAT << 64)
    assert fx.join3 == fx.sat1024
