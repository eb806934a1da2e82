"""Accuracy of the device -log(u) routine (the waiting-time draw
tau = -log(u)/a0 of the Gillespie step, Sec. II A), compiled for the host.

The routine is table-driven and may differ from the C library's log in the
last bit; the parity tests allow for that.  Here it is checked against the
exact value (50-digit decimal arithmetic) on random and boundary inputs:
error below 0.8 ulp everywhere, exact -0.0 at u = 1; and the two-word entry
the kernels use gives the same bits.
"""
import math
import os
import random
import shutil
import struct
import subprocess
from decimal import Decimal, getcontext

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def neglog(tmp_path_factory):
    cxx = shutil.which("g++")
    if not cxx:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("neglog") / "neglog_host")
    subprocess.run([cxx, "-O2", "-std=c++20", "-ffp-contract=off", "-o", exe,
                    os.path.join(HERE, "neglog_host.cpp")], check=True)

    def run(ms, words=False):
        out = subprocess.run([exe], input="\n".join(map(str, ms)), capture_output=True,
                             text=True, check=True).stdout.split()
        vals = [float.fromhex(h) for h in out]
        return vals[1::2] if words else vals[0::2]
    return run


def _inputs():
    rng = random.Random(7)
    ms = [1, 2, 3, 2 ** 53, 2 ** 53 - 1, 2 ** 53 - 2, 2 ** 52, 2 ** 52 + 1, 2 ** 52 - 1]
    ms += [rng.randrange(1, 2 ** 53 + 1) for _ in range(6000)]
    ms += [2 ** 53 - rng.randrange(1, 2 ** 24) for _ in range(2000)]  # u -> 1
    # both sides of every table sub-interval boundary, in every binade
    for e in range(0, 54, 3):
        for i in range(129):
            z = (0x3FE6000000000000 + (i << 45))
            zf = struct.unpack("<d", z.to_bytes(8, "little"))[0]
            v = int(zf * 2 ** e)
            for dv in (-1, 0, 1):
                if 1 <= v + dv <= 2 ** 53:
                    ms.append(v + dv)
    return ms


def test_neglog_accuracy(neglog):
    getcontext().prec = 50
    ms = _inputs()
    got = neglog(ms)
    worst = 0.0
    for m, g in zip(ms, got):
        exact = -(Decimal(m) / Decimal(2 ** 53)).ln()
        if exact == 0:
            assert g == 0.0 and math.copysign(1.0, g) < 0, (m, g)
            continue
        err = float(abs((Decimal(g) - exact) / Decimal(math.ulp(float(exact)))))
        worst = max(worst, err)
        assert err < 0.8, (m, g, float(exact), err)
    assert worst > 0.0


def test_neglog_extremes(neglog):
    lo, one = neglog([1, 2 ** 53])
    assert lo == pytest.approx(53 * math.log(2.0), rel=2 ** -52)
    assert one == 0.0 and math.copysign(1.0, one) < 0


def test_two_word_entry_is_the_same_routine(neglog):
    """The kernels form m from Philox's two 32-bit words without a 64-bit
    integer (m = hi 2^21 + (lo >> 11) + 1); results equal bit for bit,
    signs of zero included."""
    ms = _inputs()
    a, b = neglog(ms), neglog(ms, words=True)
    for m, x, y in zip(ms, a, b):
        assert struct.pack("<d", x) == struct.pack("<d", y), (m, x, y)
