"""One ParRep instance spread over the workgroups of a cooperative launch
(the wide kernel), through the C ABI, against the CPU oracle on the same
Philox streams (Alg. 1, Sec. II A).  Integers must match exactly and floats
within 1e-12 relative, for any number of workgroups, replicas per lane and
chunk lengths: the split into replica ranges changes neither the
dephasing nor the key order of the credited parallel-step events."""
import sys

import numpy as np
import pytest

from paper_1705_06807_amd import workloads as W
from test_gpu_parity import assert_same

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_06807_amd import binding
    binding.lib()
    return binding


def _run(B, p, **kw):
    import torch
    out = B.parrep_solve_batch([p], cycle_log_cap=4096, **kw)[0]
    torch.cuda.synchronize()
    return out.to_host()


def _om(i, omega=5.0, R=600, T=60.0, t_cp=1.0, **kw):
    hi = int(8 * omega)
    p = W.c2_toggle(seed=41, instance_id=i, omega=omega, R=R, T=T, t_cp=t_cp)
    kw.setdefault("hist_hi", (hi, hi))
    return p.replace(**kw)


CASES = [
    # many cycles, exits and Fleming-Viot restarts; ragged last wave
    ("om5_R600", lambda i: _om(i)),
    ("om2_R300_exits", lambda i: _om(i, omega=2.0, R=300, T=30.0, t_cp=0.5)),
    ("om5_steps", lambda i: _om(i, R=700, T=40.0, decorr_mode=W.STEPS, decorr=50,
                                dephase_mode=W.STEPS, dephase=40)),
    ("om5_outside_box", lambda i: _om(i, hist_lo=(2, 0), hist_hi=(12, 9))),
    # the event budget stops the dephasing step (i = 0) or the parallel step (i = 1)
    ("c1_budget", lambda i: W.c1_schlogl(seed=42, instance_id=i, R=300, T=50.0).replace(
        max_events=(150000, 270000)[i])),
    ("om50_R1024", lambda i: W.c2_toggle(seed=43, instance_id=i, T=40.0)),
]

SPREADS = [
    # (workgroups, replicas per lane, (dephasing chunk, parallel chunk))
    (3, 1, (5, 3)),
    (4, 1, (0, 0)),
    (2, 4, (1, 1)),
    (6, 1, (64, 64)),
]


@pytest.mark.parametrize("spread", SPREADS, ids=["g%d_rpl%d_c%d_%d" % (g, r, c[0], c[1])
                                                 for g, r, c in SPREADS])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_wide_parity(B, oracle, case, spread):
    name, make = case
    G, rpl, chunks = spread
    for i in range(2):
        p = make(i)
        if G * 256 * rpl < p.R:
            G = -(-p.R // (256 * rpl))
        _flush("wide %s instance %d R=%d G=%d rpl=%d chunks=%s" % (name, i, p.R, G, rpl, chunks))
        o = oracle.run(p, cycle_log_cap=4096)
        g = _run(B, p, workgroups=G, replicas_per_lane=rpl, chunk_rounds=chunks)
        assert o.counters["n_cycle_log"] <= 4096
        assert_same(o, g, what="wide %s/%d G=%d" % (name, i, G))


def test_wide_absorbing_replicas(B, oracle):
    # every replica of the parallel step holds at an absorbing state (tau = +inf):
    # the exact round must still end the run at the horizon
    p = W.Problem(net=W.pure_death(), c=(1.0,), x0=(1,), region_w=(1,), region_theta=3,
                  R=8192, decorr_mode=W.STEPS, decorr=1, dephase_mode=W.STEPS, dephase=2,
                  T=50.0, t_burn=25.0, hist_lo=(0,), hist_hi=(10,), rer_eps=None,
                  max_events=64 * 8192)
    for G in (32, 40):
        _flush("wide absorbing G=%d" % G)
        o = oracle.run(p, cycle_log_cap=4096)
        g = _run(B, p, workgroups=G)
        assert_same(o, g, what="wide absorbing G=%d" % G)
        assert g.T_s == 50.0


LARGE = [
    ("om5_R20000", lambda i: W.c2_toggle(seed=11, instance_id=i, omega=5.0, R=20000, T=30.0,
                                         t_cp=1.0).replace(hist_hi=(40, 40))),
    ("c4_R65536_short", lambda i: W.c4_toggle(seed=31, instance_id=i, T=100.0, t_cp=0.5)),
]


@pytest.mark.parametrize("case", LARGE, ids=[c[0] for c in LARGE])
def test_large_replica_counts_both_kernels(B, oracle, case):
    # the default spreads R >= 8192 over R/256 workgroups; one workgroup of
    # 16 waves (64 replicas per lane) must give the same
    name, make = case
    p = make(0)
    o = oracle.run(p, cycle_log_cap=4096)
    assert o.counters["cycles"] >= 1
    for kw in ({}, {"workgroups": 1}, {"workgroups": -(-p.R // 1024), "replicas_per_lane": 4}):
        _flush("large %s %s" % (name, kw))
        g = _run(B, p, **kw)
        assert_same(o, g, what="%s %s" % (name, kw))


def test_wide_barrier_wait_is_bounded(B, oracle):
    """A wait at a grid barrier longer than barrier_wait_us makes the run give
    up: every workgroup leaves, the run reports PARREP_RUN_ABORTED (2), and
    the device and library stay usable (forced from the host with a 1 us
    limit, which workgroups arriving microseconds apart exceed)."""
    p = _om(0, R=20000, T=30.0)
    g = _run(B, p, workgroups=79, barrier_wait_us=1)
    assert g.counters["status"] == 2
    o = oracle.run(p, cycle_log_cap=4096)
    g2 = _run(B, p, workgroups=79)
    assert_same(o, g2, what="after an aborted run")


def test_wide_full_size_c4_properties(B):
    """The large single run at full size (toggle Omega = 150, R = 65536,
    T = 1e5) on 256 workgroups: properties that hold at any size, and the
    same integer outcome as on one workgroup of 16 waves."""
    p = W.c4_toggle(seed=0)
    _flush("full-size C4 spread")
    g = _run(B, p)
    assert g.counters["spill_overflow"] == 0 and g.counters["status"] == 0
    assert g.T_s == p.T
    assert g.hist.sum() + g.outside == pytest.approx(p.T, rel=1e-12)
    c = g.counters
    assert c["ev_dephase"] == c["s2_rounds"] * p.R
    assert c["ev_par_credited"] + c["ev_par_discarded"] == c["s3_rounds"] * p.R
    _flush("full-size C4 one workgroup")
    one = _run(B, p, workgroups=1)
    assert one.counters == g.counters
    assert np.array_equal(one.x_final, g.x_final) and np.array_equal(one.cycle_log, g.cycle_log)
    scale = np.abs(one.hist).max()
    assert np.abs(one.hist - g.hist).max() <= 1e-12 * scale
