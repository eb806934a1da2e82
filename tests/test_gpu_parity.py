"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same Philox streams.

Integers (states, counters, cycle records, exit indices) must match exactly.
Floats: the clock is an exact fixed-point sum on both sides, so T_s matches to
the last bit up to the ulp-level difference between the device and host
`log`; histograms, FIM, RER and window integrals differ only by summation
order and must agree within 1e-12 relative (FIM/RER/Y are computed on the
device from the window histogram, on the oracle per event; the two are equal
in exact arithmetic).
"""
import math
import os
import sys

import numpy as np
import pytest

from paper_1705_06807_amd import workloads as W

pytestmark = pytest.mark.gpu

RTOL = 1e-12
# tau = -log(u)/a0: the device log is within 0.8 ulp and its quotient (-log u
# times a Newton-refined 1/a0) within 1.5 more; the C library's log is within
# about 0.5 ulp and its IEEE quotient within 0.5 more: 3.5 ulp in all.
TAU_RTOL = 3.5 * 2.0 ** -52


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


def _gpu_run(B, p, **kw):
    import torch
    out = B.parrep_solve(p, cycle_log_cap=kw.get("cycle_log_cap", 4096))
    torch.cuda.synchronize()
    return out.to_host()


def assert_same(o, g, rtol=RTOL, what=""):
    gc = dict(g.counters)
    assert gc.pop("spill_overflow") == 0, (what, "spill table overflow")
    oc = dict(o.counters)
    oc.pop("reserved")
    assert gc == oc, (what, gc, oc)
    assert np.array_equal(g.x_final, o.x_final), (what, g.x_final, o.x_final)
    assert np.array_equal(g.cycle_log, o.cycle_log), what
    assert g.T_s == pytest.approx(o.T_s, rel=1e-15, abs=0), what
    for name in ("hist", "hist_w"):
        a, b = getattr(o, name), getattr(g, name)
        scale = max(np.abs(a).max(), 1e-300)
        err = np.abs(a - b).max() / scale
        assert err < rtol, (what, name, err)
        assert np.array_equal(a != 0, b != 0), (what, name, "support differs")
    for name in ("outside", "outside_w"):
        assert getattr(g, name) == pytest.approx(getattr(o, name), rel=rtol, abs=1e-300), what
    for name in ("fim", "rer", "y"):
        a, b = getattr(o, name), getattr(g, name)
        scale = max(np.abs(a).max(), 1e-300)
        assert np.abs(a - b).max() <= rtol * scale, (what, name, a, b)


def test_philox_blocks(B, oracle):
    rng = np.random.default_rng(0)
    ck = rng.integers(0, 2 ** 32, size=(4096, 6), dtype=np.uint64).astype(np.uint32)
    ck[:4] = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF] * 6, [1, 0, 0, 0, 0, 0], [0, 0, 5, 0, 0x1234, 0]]
    got = B.parrep_philox(ck)
    want = np.array([oracle.philox(c[:4], c[4:]) for c in ck])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("name", ["schlogl", "toggle", "toggle_beta", "genetic_switch"])
def test_ssa_events(B, oracle, name):
    rng = np.random.default_rng(1)
    if name == "schlogl":
        net, c = W.schlogl_classic(), W.SCHLOGL_CLASSIC_C
        states = rng.integers(0, 1200, size=(3000, 1))
        states[:4, 0] = [0, 1, 2, 3]
    elif name == "toggle":
        net, c = W.toggle(50.0), W.TOGGLE_C
        states = rng.integers(0, 450, size=(3000, 2))
        states[:3] = [[0, 0], [0, 9], [9, 0]]
    elif name == "genetic_switch":
        net, c = W.genetic_switch(), W.genetic_switch_c(2400.0)
        xi = rng.integers(0, 2, size=3000)
        states = np.stack([1 - xi, xi, rng.integers(0, 12, size=3000),
                           rng.integers(0, 4000, size=3000)], axis=1)
        states[:4, 2:] = [[0, 0], [0, 1], [1, 0], [0, 1000]]
    else:  # non-integral Hill exponents are outside the GPU path
        net, c = W.toggle(50.0), (3.0, 3.0, 2.5, 1.5)
        with pytest.raises(B.ParrepError, match="integers"):
            B.parrep_events(net, c, np.zeros((4, 2), dtype=np.int32),
                            np.zeros((4, 4), dtype=np.uint32))
        return
    blocks = rng.integers(0, 2 ** 32, size=(len(states), 4), dtype=np.uint64).astype(np.uint32)
    blocks[0] = [0xFFFFFFFF, 0xFFFFFFFF, 0, 0]
    a0, tau, J = B.parrep_events(net, c, states, blocks)
    for i in range(len(states)):
        lam, oa0, otau, oJ, _ = oracle.event(net, c, states[i], blocks[i])
        assert a0[i] == oa0, (i, a0[i], oa0)
        assert J[i] == oJ, i
        assert tau[i] == pytest.approx(otau, rel=TAU_RTOL, abs=0), i


C1_CASES = [
    ("c1", lambda i: W.c1_schlogl(seed=0, instance_id=i)),
    ("c1_R1", lambda i: W.c1_schlogl(seed=1, instance_id=i, R=1)),
    ("c1_R100_ragged", lambda i: W.c1_schlogl(seed=2, instance_id=i, R=100)),
    ("c1_steps", lambda i: W.c1_schlogl(seed=3, instance_id=i).replace(
        decorr_mode=W.STEPS, decorr=400, dephase_mode=W.STEPS, dephase=300)),
    ("c1_no_burn", lambda i: W.c1_schlogl(seed=4, instance_id=i).replace(t_burn=0.0)),
    ("c1_budget", lambda i: W.c1_schlogl(seed=5, instance_id=i).replace(max_events=20000 + 997 * i)),
    ("c1_narrow_hist", lambda i: W.c1_schlogl(seed=6, instance_id=i).replace(
        hist_lo=(60,), hist_hi=(110,))),
    # the paper's own setting (Sec. IV A): V = 25, W+ = {x <= 25.96}, n_c = n_p = 5000
    # transitions, R = 100, with the horizon cut from 1e5 to 5000 (about 10 exits)
    ("paper_schlogl_v25", lambda i: W.paper_schlogl_problem(seed=5, instance_id=i, T=5000.0)),
    # degenerate thresholds: no decorrelation and no dephasing (every cycle is S3 from X~)
    ("c1_zero_thresholds", lambda i: W.c1_schlogl(seed=7, instance_id=i).replace(
        decorr_mode=W.STEPS, decorr=0, dephase_mode=W.STEPS, dephase=0)),
]


@pytest.mark.parametrize("case", C1_CASES, ids=[c[0] for c in C1_CASES])
def test_schlogl_solve_parity(B, oracle, case):
    name, make = case
    for i in range(3):
        p = make(i)
        _flush("case %s instance %d R=%d" % (name, i, p.R))
        o = oracle.run(p, cycle_log_cap=4096)
        g = _gpu_run(B, p)
        assert_same(o, g, what="%s/%d" % (name, i))


def _toggle_small(i, **kw):
    # Omega = 5 switches every ~12 time units: with t_c = t_p = 1, many cycles,
    # exits and FV restarts
    p = W.c2_toggle(seed=11, instance_id=i, omega=5.0, R=kw.pop("R", 64), T=kw.pop("T", 300.0),
                    t_cp=1.0)
    kw.setdefault("hist_hi", (40, 40))
    return p.replace(**kw)


TOGGLE_CASES = [
    ("om5_R64", lambda i: _toggle_small(i)),
    ("om5_R1000", lambda i: _toggle_small(i, R=1000, T=60.0)),
    ("om5_R3000", lambda i: _toggle_small(i, R=3000, T=30.0)),
    ("om5_R5000_global_fv", lambda i: _toggle_small(i, R=5000, T=20.0)),
    ("om5_steps", lambda i: _toggle_small(i, decorr_mode=W.STEPS, decorr=50,
                                          dephase_mode=W.STEPS, dephase=40)),
    ("om5_outside_box", lambda i: _toggle_small(i, hist_lo=(2, 0), hist_hi=(12, 9))),
    ("om5_time_zero", lambda i: _toggle_small(i, decorr=0.0, dephase=0.0)),
    ("om50_R1024", lambda i: W.c2_toggle(seed=12, instance_id=i, T=20.0, t_cp=1.0)),
    ("om50_R1024_t20", lambda i: W.c2_toggle(seed=13, instance_id=i, T=120.0)),
]


@pytest.mark.parametrize("case", TOGGLE_CASES, ids=[c[0] for c in TOGGLE_CASES])
def test_toggle_solve_parity(B, oracle, case):
    name, make = case
    for i in range(2):
        p = make(i)
        _flush("case %s instance %d R=%d" % (name, i, p.R))
        o = oracle.run(p, cycle_log_cap=4096)
        g = _gpu_run(B, p)
        assert o.counters["n_cycle_log"] <= 4096
        assert_same(o, g, what="%s/%d" % (name, i))


def test_absorbing_state(B, oracle):
    p = W.Problem(net=W.pure_death(), c=(1.0,), x0=(5,), region_w=(1,), region_theta=3, R=4,
                  decorr_mode=W.STEPS, decorr=2, dephase_mode=W.STEPS, dephase=2, T=50.0,
                  t_burn=25.0, hist_lo=(0,), hist_hi=(10,), rer_eps=None)
    for i in range(8):
        q = p.replace(instance_id=i)
        assert_same(oracle.run(q, cycle_log_cap=4096), _gpu_run(B, q), what="absorbing")


@pytest.mark.parametrize("R", [4096, 8192, 65536])
def test_absorbing_replicas_reach_the_horizon(B, oracle, R):
    # Decorrelation ends on the jump into the absorbing state x = 0, so every
    # replica of the parallel step holds there with tau = +inf.  Each enters
    # the round's clock sum as 2^52; a multiple of 4096 of them must still
    # end the run at the horizon (the fixed-point replica sums saturate).
    # The event budget bounds the run had the horizon been missed.
    p = W.Problem(net=W.pure_death(), c=(1.0,), x0=(1,), region_w=(1,), region_theta=3, R=R,
                  decorr_mode=W.STEPS, decorr=1, dephase_mode=W.STEPS, dephase=2, T=50.0,
                  t_burn=25.0, hist_lo=(0,), hist_hi=(10,), rer_eps=None,
                  max_events=64 * R)
    for i in range(3):
        q = p.replace(instance_id=i)
        _flush("absorbing R=%d instance %d" % (R, i))
        o = oracle.run(q, cycle_log_cap=4096)
        assert o.counters["status"] == 0 and o.counters["end_phase"] == 3
        g = _gpu_run(B, q)
        assert_same(o, g, what="absorbing R=%d" % R)
        assert g.T_s == 50.0


@pytest.mark.parametrize("shape", [(1, 1), (4, 1), (16, 1), (1, 4), (4, 4), (16, 4), (1, 16),
                                   (4, 16), (16, 16), (64, 16)])
def test_launch_shapes_agree(B, oracle, shape):
    import torch
    probs = [_toggle_small(i, R=60, T=100.0) for i in range(3)]
    outs = B.parrep_solve_batch(probs, replicas_per_lane=shape[0], waves=shape[1],
                                cycle_log_cap=4096)
    torch.cuda.synchronize()
    for p, o in zip(probs, outs):
        assert_same(oracle.run(p, cycle_log_cap=4096), o.to_host(), what=str(shape))


@pytest.mark.parametrize("shape,R", [((4, 1), 256), ((4, 1), 255), ((16, 1), 1024),
                                     ((4, 4), 1024), ((4, 4), 1023), ((4, 16), 4096),
                                     ((4, 16), 4095)])
@pytest.mark.parametrize("steps", [False, True])
def test_full_slot_dephasing(B, oracle, shape, R, steps):
    """With 4 replicas per lane, dephasing rounds in which every slot of
    every thread holds a replica (R = 4 x 64 x waves) run without per-slot
    lane masks; one replica fewer takes the masked rounds, as do the other
    shapes (16 per lane).  All against the oracle, with the dephasing phase
    ended by time and by a round count."""
    import torch
    kw = dict(R=R, T=40.0)
    if steps:
        kw.update(dephase_mode=W.STEPS, dephase=12)
    probs = [_toggle_small(i, **kw) for i in range(2)]
    _flush("full-slot dephasing shape %s R=%d steps=%s" % (shape, R, steps))
    outs = B.parrep_solve_batch(probs, replicas_per_lane=shape[0], waves=shape[1],
                                cycle_log_cap=4096)
    torch.cuda.synchronize()
    for p, o in zip(probs, outs):
        assert_same(oracle.run(p, cycle_log_cap=4096), o.to_host(),
                    what="full-slot %s R=%d" % (shape, R))


@pytest.mark.parametrize("shape,R", [((4, 1), 256), ((4, 4), 1024)])
def test_full_slot_dephasing_budget(B, oracle, shape, R):
    """An event budget that runs out inside the dephasing phase, in the
    rounds without per-slot lane masks: the run stops there (end phase 9)
    exactly as the oracle's does."""
    import torch
    probs = [_toggle_small(i, R=R, T=40.0, max_events=(R * 30 + 517, R * 58 + 3)[i])
             for i in range(2)]
    _flush("full-slot dephasing budget shape %s R=%d" % (shape, R))
    outs = B.parrep_solve_batch(probs, replicas_per_lane=shape[0], waves=shape[1],
                                cycle_log_cap=4096)
    torch.cuda.synchronize()
    for p, o in zip(probs, outs):
        ref = oracle.run(p, cycle_log_cap=4096)
        assert ref.counters["end_phase"] == 9
        assert_same(ref, o.to_host(), what="full-slot budget %s R=%d" % (shape, R))


@pytest.mark.parametrize("shape,R", [((1, 4), 230), ((1, 16), 700)])
def test_chunked_dephasing_replays(B, oracle, shape, R):
    """STEPS-mode dephasing with one replica per lane over several waves runs
    in barrier-free chunks and rewinds every wave to the first round with an
    exit (replaying from the chunk start).  Omega = 5 with replicas in every
    wave (the last one ragged) exits in most rounds, so nearly every chunk
    replays; the result must still equal the round-by-round oracle."""
    import torch
    probs = [_toggle_small(i, R=R, T=40.0, decorr_mode=W.STEPS, decorr=50,
                           dephase_mode=W.STEPS, dephase=300) for i in range(3)]
    _flush("chunked dephasing shape %s R=%d" % (shape, R))
    outs = B.parrep_solve_batch(probs, replicas_per_lane=shape[0], waves=shape[1],
                                cycle_log_cap=4096)
    torch.cuda.synchronize()
    for p, o in zip(probs, outs):
        h = o.to_host()
        assert h.counters["fv_restarts"] > 0
        assert_same(oracle.run(p, cycle_log_cap=4096), h, what="chunked %s" % (shape,))


def test_mixed_batch_equals_oracle(B, oracle):
    import torch
    probs = W.c3_batch(seed=0, n_schlogl=6, n_toggle=6, r_lo=16, r_hi=700, T_schlogl=20.0,
                       T_toggle=4.0)
    outs = B.parrep_solve_batch(probs, cycle_log_cap=4096)
    torch.cuda.synchronize()
    for p, o in zip(probs, outs):
        _flush("batch instance %d %s R=%d" % (p.instance_id, p.net.name, p.R))
        assert_same(oracle.run(p, cycle_log_cap=4096), o.to_host(), what="batch")


def test_dephase_hook(B, oracle):
    # R = 1024 takes shape (4, 4) with every slot full; 1000 the masked rounds
    for R, tp in ((64, 1.0), (1000, 0.5), (1024, 0.5), (5000, 0.3)):
        p = W.c2_toggle(seed=3, omega=5.0, R=R).replace(dephase=tp)
        Yg, ng = B.parrep_dephase_only(p, (12, 3), cycle=7)
        Yo, no = oracle.dephase(p, (12, 3), cycle=7)
        assert ng == no and np.array_equal(Yg, Yo), R


@pytest.mark.parametrize("R", [1, 16, 256, 4096])
def test_time_mode_dephasing_stop_hook(B, oracle, R):
    # the chain of the oracle's dephasing stop-rule pin (constant a0, one set):
    # the device stops after the same round as the oracle, whose round count
    # follows the exact law P(N <= n) = P(Poisson(a0 t_p) <= n - 1)^R
    for i in range(40 if R < 4096 else 8):
        p = W.self_loop_problem(seed=R, instance_id=i, R=R)
        _flush("self-loop dephasing R=%d instance %d" % (R, i))
        Yg, ng = B.parrep_dephase_only(p, (0,), cycle=i % 7)
        Yo, no = oracle.dephase(p, (0,), cycle=i % 7)
        assert ng == no and np.array_equal(Yg, Yo), (R, i, ng, no)


@pytest.mark.parametrize("R", [1, 64])
def test_time_mode_decorrelation_stop_parity(B, oracle, R):
    # the chain of the oracle's decorrelation stop-rule pin: thousands of
    # cycles, each decorrelation ended by the time-in-set rule; the cycle
    # records (decorrelation events per cycle among them) must be equal
    for i in range(2):
        p = W.flip_chain_problem(seed=5, instance_id=i, R=R, T=2000.0)
        _flush("flip chain R=%d instance %d" % (R, i))
        o = oracle.run(p, cycle_log_cap=8192)
        assert 100 < o.counters["n_cycle_log"] <= 8192
        g = _gpu_run(B, p, cycle_log_cap=8192)
        assert_same(o, g, what="flip chain R=%d" % R)


def test_parallel_hook(B, oracle):
    rng = np.random.default_rng(5)
    for R in (1, 16, 300):
        for t in range(5):
            p = W.c2_toggle(seed=9, instance_id=t, omega=2.0, R=R)
            init = np.stack([rng.integers(3, 12, size=R), rng.integers(0, 3, size=R)], axis=1)
            g = B.parrep_parallel_only(p, init, cycle=3)
            o = oracle.parallel(p, init, cycle=3)
            assert g[:2] == o[:2] and np.array_equal(g[2], o[2]), (R, t)
            assert g[3] == pytest.approx(o[3], rel=1e-15)


def test_full_size_toggle_sampled(B, oracle):
    """Toggle Omega=50, R=1024, T=2e4 (the benchmark workload) run the way the
    benchmark runs it: a plan with 4 replicas per lane and 4 waves, executed
    with parrep_plan_run; one sampled instance against the oracle, and
    properties that hold for every instance."""
    import torch
    probs = [W.c2_toggle(seed=0, instance_id=i) for i in range(4)]
    _flush("full-size toggle batch of %d" % len(probs))
    plan = B.Plan(probs, replicas_per_lane=4, waves=4)
    plan.run()
    torch.cuda.synchronize()
    outs = plan.outputs
    hs = [o.to_host() for o in outs]
    for p, h in zip(probs, hs):
        assert h.T_s == p.T
        assert h.hist.sum() + h.outside == pytest.approx(p.T, rel=1e-12)
        assert h.hist_w.sum() + h.outside_w == pytest.approx(p.T - p.t_burn, rel=1e-12)
        assert h.counters["status"] == 0
    if os.environ.get("PARREP_SKIP_SLOW_ORACLE") != "1":
        _flush("oracle on instance 0 (about 30 s)")
        o = oracle.run(probs[0], cycle_log_cap=0)
        hs[0].cycle_log = None
        o.cycle_log = None
        assert_same(o, hs[0], what="full-size")
    plan.close()


def _gs(i, V=240.0, **kw):
    # the genetic switch of Sec. IV B at system size V; at V = 240 the wells
    # are left every ~10-50 time units, so short runs see many cycles
    f = V / 2400.0
    kw.setdefault("hist_hi", (1, 1, int(math.ceil(24 * f)) + 6, int(math.ceil(3000 * f))))
    p = W.genetic_switch_problem(seed=21, instance_id=i, V=V, R=kw.pop("R", 8),
                                 T=kw.pop("T", 2000.0), n_c=kw.pop("n_c", 500),
                                 n_p=kw.pop("n_p", 500))
    return p.replace(**kw)


GS_CASES = [
    ("v240_R8", lambda i: _gs(i)),
    ("v240_R100", lambda i: _gs(i, R=100, T=400.0)),
    ("v240_time", lambda i: _gs(i, decorr_mode=W.TIME, decorr=2.0, dephase_mode=W.TIME,
                                dephase=1.5)),
    ("v240_narrow_hist", lambda i: _gs(i, hist_lo=(0, 0, 1, 20), hist_hi=(1, 1, 3, 200))),
    ("v2400_R100", lambda i: _gs(i, V=2400.0, R=100, T=1500.0, n_c=2e4, n_p=2e4)),
    ("v2400_R100_short", lambda i: _gs(i, V=2400.0, R=100, T=5000.0, n_c=2e3, n_p=2e3)),
]


@pytest.mark.parametrize("case", GS_CASES, ids=[c[0] for c in GS_CASES])
def test_genetic_switch_solve_parity(B, oracle, case):
    name, make = case
    for i in range(2):
        p = make(i)
        _flush("case gs_%s instance %d R=%d" % (name, i, p.R))
        o = oracle.run(p, cycle_log_cap=4096)
        g = _gpu_run(B, p)
        assert o.counters["n_cycle_log"] <= 4096
        assert_same(o, g, what="gs_%s/%d" % (name, i))


LARGE_R_CASES = [
    # more than 16384 replicas: 64 replica slots per lane (rolled loops)
    ("om5_R20000", lambda i: _toggle_small(i, R=20000, T=30.0), 2),
    # the large single run at Omega = 150, R = 65536, cut short with t_c = t_p = 0.5
    ("c4_R65536_short", lambda i: W.c4_toggle(seed=31, instance_id=i, T=100.0, t_cp=0.5), 1),
]


@pytest.mark.parametrize("case", LARGE_R_CASES, ids=[c[0] for c in LARGE_R_CASES])
def test_large_replica_count_parity(B, oracle, case):
    name, make, n = case
    for i in range(n):
        p = make(i)
        _flush("case %s instance %d R=%d" % (name, i, p.R))
        o = oracle.run(p, cycle_log_cap=4096)
        g = _gpu_run(B, p)
        assert o.counters["cycles"] >= 1
        assert_same(o, g, what="%s/%d" % (name, i))


def test_full_size_c4_properties(B):
    """The large single run (toggle Omega = 150, R = 65536, T = 1e5) at full
    size: too long for the oracle, so properties that hold at any size."""
    import torch
    p = W.c4_toggle(seed=0)
    _flush("full-size C4, one instance")
    out = B.parrep_solve(p, cycle_log_cap=256)
    torch.cuda.synchronize()
    h = out.to_host()
    assert h.counters["spill_overflow"] == 0 and h.counters["status"] == 0
    assert h.T_s == p.T
    assert h.hist.sum() + h.outside == pytest.approx(p.T, rel=1e-12)
    assert h.hist_w.sum() + h.outside_w == pytest.approx(p.T - p.t_burn, rel=1e-12)
    c = h.counters
    # every S2 and S3 round moves all replicas; S3 credits R per round but the last
    assert c["ev_dephase"] == c["s2_rounds"] * p.R
    assert c["ev_par_credited"] + c["ev_par_discarded"] == c["s3_rounds"] * p.R
    assert np.all(h.fim.diagonal() > 0)


STAGED_CASES = [
    # one species: the whole box (1001 bins) fits the 1024-bin tile
    ("c1", lambda i: W.c1_schlogl(seed=51, instance_id=i)),
    ("paper_schlogl_v25", lambda i: W.paper_schlogl_problem(seed=52, instance_id=i, T=2000.0)),
    # two species: a tile of the 41 x 41 box, with exits and restarts
    ("om5_R1000", lambda i: _toggle_small(i, R=1000, T=60.0)),
    # the benchmark's box (401 x 401) and shape, horizon cut
    ("om50_R1024_t20", lambda i: W.c2_toggle(seed=53, instance_id=i, T=120.0)),
]


@pytest.mark.parametrize("flush", [0, 1, 7])
@pytest.mark.parametrize("case", STAGED_CASES, ids=[c[0] for c in STAGED_CASES])
def test_histogram_staging_parity(B, oracle, case, flush):
    """Parallel-step credits staged in an LDS tile of the histogram and
    flushed at the step's end and the burn-in time (flush 0), or also every
    1 or 7 rounds: the same outputs as the oracle (summation order aside)."""
    import torch
    name, make = case
    probs = [make(i) for i in range(2)]
    _flush("staged %s flush=%d" % (name, flush))
    outs = B.parrep_solve_batch(probs, cycle_log_cap=4096, histogram_staging=1,
                                flush_period=flush)
    torch.cuda.synchronize()
    for p, o in zip(probs, outs):
        assert_same(oracle.run(p, cycle_log_cap=4096), o.to_host(),
                    what="staged %s flush=%d" % (name, flush))
