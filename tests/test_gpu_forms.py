"""GPU tests of the batched and served forms: plans (hipGraph replays and
problem updates), the launch-shape autotuner, and the request server, each
checked against plain solves of the same problems (integers exactly, floats
to summation order) and, for a sample, against the CPU oracle."""
import sys

import numpy as np
import pytest

from paper_1705_06807_amd import workloads as W

from test_gpu_parity import RTOL, assert_same

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


def _mixed(seed=0, n=4):
    # Schloegl and toggle instances, uneven R: several launch-shape groups
    return W.c3_batch(seed=seed, n_schlogl=n, n_toggle=n, r_lo=16, r_hi=3000, T_schlogl=20.0,
                      T_toggle=3.0)


def _host(outs):
    import torch
    torch.cuda.synchronize()
    return [o.to_host() for o in outs]


def _same_float(a, b, rtol=RTOL):
    scale = max(np.abs(a).max(), 1e-300)
    return np.abs(a - b).max() <= rtol * scale


def assert_gpu_same(a, b, what=""):
    """Two GPU results of the same problem: integers equal, floats to order."""
    assert a.counters == b.counters, (what, a.counters, b.counters)
    assert np.array_equal(a.x_final, b.x_final), what
    assert a.T_s == b.T_s, what
    for name in ("hist", "hist_w", "fim", "rer", "y"):
        assert _same_float(getattr(a, name), getattr(b, name)), (what, name)


def test_plan_replays_match_eager(B, oracle):
    import torch
    probs = _mixed()
    _flush("plan over %d instances, R in %s" % (len(probs), sorted(p.R for p in probs)))
    eager = _host(B.parrep_solve_batch(probs, cycle_log_cap=0))
    plan = B.Plan(probs)
    for rep in range(3):
        plan.launch()
        torch.cuda.synchronize()
        # eager work between replays
        B.parrep_solve(W.c1_schlogl(seed=9, instance_id=rep, T=5.0), cycle_log_cap=0)
        torch.cuda.synchronize()
        got = [o.to_host() for o in plan.outputs]
        for i, (g, e) in enumerate(zip(got, eager)):
            assert_gpu_same(g, e, what="replay %d instance %d" % (rep, i))
    # one instance against the oracle
    o = oracle.run(probs[0], cycle_log_cap=0)
    got[0].cycle_log = None
    o.cycle_log = None
    assert_same(o, got[0], what="plan vs oracle")
    plan.close()


def test_plan_update(B):
    import torch
    probs = _mixed(seed=1, n=2)
    plan = B.Plan(probs)
    plan.launch()
    torch.cuda.synchronize()
    i = 1
    newp = probs[i].replace(seed=77, c=tuple(1.05 * v for v in probs[i].c))
    plan.update(i, newp)
    plan.launch()
    torch.cuda.synchronize()
    want = _host(B.parrep_solve_batch([newp], cycle_log_cap=0))[0]
    assert_gpu_same(plan.outputs[i].to_host(), want, what="updated")
    # the others are unchanged
    want0 = _host(B.parrep_solve_batch([probs[0]], cycle_log_cap=0))[0]
    assert_gpu_same(plan.outputs[0].to_host(), want0, what="untouched")
    with pytest.raises(B.ParrepError):
        plan.update(0, probs[0].replace(hist_hi=tuple(h + 1 for h in probs[0].hist_hi)))
    plan.close()


def test_autotune_then_parity(B, oracle):
    import torch
    p = W.c2_toggle(seed=4, omega=5.0, R=200, T=40.0, t_cp=1.0).replace(hist_hi=(40, 40))
    rpl, waves, staging, flush = B.parrep_autotune(p, instances=64, trial_events=50000)
    _flush("autotuned shape for R=200: rpl=%d waves=%d staging=%d flush=%d"
           % (rpl, waves, staging, flush))
    assert staging in (-1, 1) and flush >= 0
    assert rpl * waves * 64 >= 200
    probs = [p.replace(instance_id=i) for i in range(3)]
    outs = B.parrep_solve_batch(probs, cycle_log_cap=4096)
    torch.cuda.synchronize()
    for q, o in zip(probs, outs):
        assert_same(oracle.run(q, cycle_log_cap=4096), o.to_host(), what="autotuned")


def _pooled_alone(B, p, runs):
    outs = _host(B.parrep_solve_batch([p.replace(instance_id=p.instance_id + k)
                                       for k in range(runs)], cycle_log_cap=0))
    return outs


def test_server_results_alone_and_in_the_mix(B):
    reqs = [(W.c1_schlogl(seed=3, instance_id=10 * i, T=30.0), 3) for i in range(3)]
    reqs += [(W.c2_toggle(seed=5, instance_id=10 * i, omega=5.0, R=R, T=30.0, t_cp=1.0)
              .replace(hist_hi=(40, 40)), 2) for i, R in enumerate((64, 700, 3000))]
    srv = B.Server(n_streams=4)
    tickets = [srv.submit(p, min_runs=n, max_runs=n) for p, n in reqs]
    _flush("submitted %d requests" % len(tickets))
    results = [srv.poll(t) for t in tickets]
    srv.close()
    for (p, n), (pooled, info) in zip(reqs, results):
        alone = _pooled_alone(B, p, n)
        assert info["runs"] == n and info["status"] == 0
        assert info["events"] == sum(a.events for a in alone)
        for k in pooled.counters:
            vals = [a.counters[k] for a in alone]
            want = max(vals) if k == "status" else sum(vals)
            assert pooled.counters[k] == want, k
        assert pooled.T_s == pytest.approx(sum(a.T_s for a in alone), rel=1e-15)
        assert _same_float(pooled.hist, sum(a.hist for a in alone))
        assert _same_float(pooled.hist_w, sum(a.hist_w for a in alone))
        assert _same_float(pooled.fim, sum(a.fim for a in alone) / n)
        assert _same_float(pooled.y, sum(a.y for a in alone) / n)
        ys = np.array([a.y for a in alone])
        if n >= 2:
            iaf = ys.var(axis=0, ddof=1) / (p.T - p.t_burn)
            assert np.allclose(info["iaf"], iaf, rtol=1e-9)


def test_server_rse_target_and_cancel(B):
    srv = B.Server(n_streams=2)
    p = W.c1_schlogl(seed=8, instance_id=0, T=30.0)
    t = srv.submit(p, rse_target=0.05, min_runs=4, max_runs=40)
    pooled, info = srv.poll(t)
    _flush("rse request: runs=%d rse=%.4f" % (info["runs"], info["rse"]))
    assert 4 <= info["runs"] <= 40
    assert info["rse"] <= 0.05 or info["runs"] == 40
    long = W.c2_toggle(seed=1, omega=50.0, R=1024, T=2e4)
    t2 = srv.submit(long, min_runs=2, max_runs=2)
    srv.cancel(t2)
    with pytest.raises(B.ParrepError, match="cancelled"):
        srv.poll(t2)
    srv.close()


def _general_mix():
    # general kernels (4 species, 6 reactions: the genetic switch at V = 240)
    # beside narrow ones, and one instance with 64 replica slots per lane
    gs = [W.genetic_switch_problem(seed=12, instance_id=i, V=240.0, R=R, n_c=300, n_p=300,
                                   T=300.0).replace(hist_hi=(1, 1, 8, 700))
          for i, R in enumerate((8, 100, 900))]
    big = [W.c2_toggle(seed=13, instance_id=0, omega=5.0, R=20000, T=6.0, t_cp=1.0)
           .replace(hist_hi=(40, 40))]
    return gs + big + _mixed(seed=2, n=2)


def test_plan_with_general_kernels_and_large_r(B, oracle):
    import torch
    probs = _general_mix()
    _flush("plan over %d instances, R in %s" % (len(probs), sorted(p.R for p in probs)))
    eager = _host(B.parrep_solve_batch(probs, cycle_log_cap=0))
    plan = B.Plan(probs)
    for rep in range(2):
        plan.launch()
        torch.cuda.synchronize()
        B.parrep_solve(W.c1_schlogl(seed=9, instance_id=rep, T=5.0), cycle_log_cap=0)
        torch.cuda.synchronize()
        got = [o.to_host() for o in plan.outputs]
        for i, (g, e) in enumerate(zip(got, eager)):
            assert_gpu_same(g, e, what="replay %d instance %d" % (rep, i))
    for i in (0, 3):  # a genetic switch instance and the large-R one against the oracle
        o = oracle.run(probs[i], cycle_log_cap=0)
        got[i].cycle_log = None
        o.cycle_log = None
        assert_same(o, got[i], what="plan vs oracle %d" % i)
    plan.close()


def test_persistent_batch_equals_one_workgroup_per_instance(B, oracle):
    """The persistent form (resident workgroups taking the instances of their
    group from a counter) gives every instance the result it gets with a
    workgroup of its own: narrow and general kernels, several shape groups,
    as a batch and as a plan replayed twice; one instance against the
    oracle."""
    import torch
    probs = _general_mix()[:3] + _mixed(seed=3, n=3)
    _flush("persistent batch over %d instances, R in %s" % (len(probs), sorted(p.R for p in probs)))
    eager = _host(B.parrep_solve_batch(probs, cycle_log_cap=0))
    pers = _host(B.parrep_solve_batch(probs, cycle_log_cap=0, persistent=1))
    for i, (g, e) in enumerate(zip(pers, eager)):
        assert_gpu_same(g, e, what="persistent batch instance %d" % i)
    plan = B.Plan(probs, persistent=1)
    for rep in range(2):
        plan.launch()
        torch.cuda.synchronize()
        got = [o.to_host() for o in plan.outputs]
        for i, (g, e) in enumerate(zip(got, eager)):
            assert_gpu_same(g, e, what="persistent plan replay %d instance %d" % (rep, i))
    plan.close()
    o = oracle.run(probs[0], cycle_log_cap=0)
    pers[0].cycle_log = None
    o.cycle_log = None
    assert_same(o, pers[0], what="persistent vs oracle")


def test_persistent_batch_takes_more_instances_than_the_device_holds(B):
    """1500 instances in 16-wave workgroups, more than the device holds at
    once: each resident workgroup runs several instances in turn."""
    probs = [W.c1_schlogl(seed=21, instance_id=i, R=32, T=2.0) for i in range(1500)]
    _flush("persistent batch of %d instances, shape (1,16)" % len(probs))
    eager = _host(B.parrep_solve_batch(probs, replicas_per_lane=1, waves=16))
    pers = _host(B.parrep_solve_batch(probs, replicas_per_lane=1, waves=16, persistent=1))
    for i, (g, e) in enumerate(zip(pers, eager)):
        assert_gpu_same(g, e, what="instance %d" % i)
    assert all(h.T_s == 2.0 for h in pers)


def test_persistent_rejects_bad_value(B):
    with pytest.raises(B.ParrepError, match="persistent"):
        B.parrep_solve_batch([W.c1_schlogl(seed=0, instance_id=0, T=1.0)], persistent=2)


def test_server_with_general_kernels(B):
    reqs = [(p, 2) for p in _general_mix()[:4]]
    srv = B.Server(n_streams=4)
    tickets = [srv.submit(p, min_runs=n, max_runs=n) for p, n in reqs]
    _flush("submitted %d requests" % len(tickets))
    results = [srv.poll(t) for t in tickets]
    srv.close()
    for (p, n), (pooled, info) in zip(reqs, results):
        alone = _pooled_alone(B, p, n)
        assert info["runs"] == n and info["status"] == 0
        assert info["events"] == sum(a.events for a in alone)
        assert pooled.T_s == pytest.approx(sum(a.T_s for a in alone), rel=1e-15)
        assert _same_float(pooled.hist, sum(a.hist for a in alone))
        assert _same_float(pooled.fim, sum(a.fim for a in alone) / n)


def test_plan_run_matches_eager_and_times_the_instance_kernels(B):
    import torch
    probs = _mixed(seed=4)
    eager = _host(B.parrep_solve_batch(probs, cycle_log_cap=0))
    plan = B.Plan(probs)
    ev_b = torch.cuda.Event(enable_timing=True)
    ev_a = torch.cuda.Event(enable_timing=True)
    # torch creates the HIP events on first record; the library records them again
    ev_b.record()
    ev_a.record()
    for rep in range(2):
        plan.run(events=(ev_b, ev_a))
        torch.cuda.synchronize()
        assert ev_b.elapsed_time(ev_a) > 0.0
        got = [o.to_host() for o in plan.outputs]
        for i, (g, e) in enumerate(zip(got, eager)):
            assert_gpu_same(g, e, what="run %d instance %d" % (rep, i))
    plan.launch()  # graph replays and runs mix on one plan
    torch.cuda.synchronize()
    for i, (g, e) in enumerate(zip([o.to_host() for o in plan.outputs], eager)):
        assert_gpu_same(g, e, what="replay after runs, instance %d" % i)
    plan.close()
