"""Error paths of the C ABI on a device: invalid input is rejected with the
documented status before anything is enqueued, and the context, its
networks and a running server stay usable afterwards."""
import numpy as np
import pytest

from paper_1705_06807_amd import workloads as W

pytestmark = pytest.mark.gpu

EINVAL, ENOMEM, EUNSUPPORTED = -1, -2, -4


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_06807_amd import binding
    binding.lib()
    return binding


def _code(B, fn):
    with pytest.raises(B.ParrepError) as e:
        fn()
    return int(str(e.value).split("error ")[1].split(":")[0])


BAD_PROBLEMS = [
    ("R=0", lambda p: p.replace(R=0), EINVAL),
    ("R too large", lambda p: p.replace(R=65537), EINVAL),
    ("T<=0", lambda p: p.replace(T=0.0, t_burn=0.0), EINVAL),
    ("t_burn>=T", lambda p: p.replace(t_burn=p.T), EINVAL),
    ("negative c", lambda p: p.replace(c=(-1.0,) + tuple(p.c[1:])), EINVAL),
    ("nan threshold", lambda p: p.replace(dephase=float("nan")), EINVAL),
    ("box inverted", lambda p: p.replace(hist_lo=(5, 0), hist_hi=(4, 40)), EINVAL),
    ("Hill exponent 2.5", lambda p: p.replace(c=(3.0, 3.0, 2.5, 2.0)), EUNSUPPORTED),
]


@pytest.mark.parametrize("case", BAD_PROBLEMS, ids=[c[0] for c in BAD_PROBLEMS])
def test_invalid_problem_rejected(B, case):
    import torch
    name, make, want = case
    good = W.c2_toggle(seed=1, omega=5.0, R=64, T=20.0, t_cp=1.0).replace(hist_hi=(40, 40))
    bad = make(good)
    ctx = B.context()
    # outputs sized for the good problem; validation fails before any use
    outs = [B.Outputs(ctx, good, cycle_log_cap=0)]
    assert _code(B, lambda: B.parrep_solve_batch([bad], outputs=outs)) == want
    # the context still works
    g = B.parrep_solve(good, cycle_log_cap=0)
    torch.cuda.synchronize()
    assert g.to_host().T_s == good.T


def test_mixed_batch_with_one_bad_instance_enqueues_nothing(B):
    import torch
    good = W.c1_schlogl(seed=2, T=5.0)
    outs = [B.Outputs(B.context(), good, cycle_log_cap=0) for _ in range(3)]
    for o in outs:
        o.stats.fill_(-7.0)
    probs = [good, good.replace(instance_id=1, R=0), good.replace(instance_id=2)]
    assert _code(B, lambda: B.parrep_solve_batch(probs, outputs=outs)) == EINVAL
    torch.cuda.synchronize()
    assert all(float(o.stats[0]) == -7.0 for o in outs)  # nothing ran


def test_server_errors_leave_it_running(B):
    srv = B.Server(mem_budget=1 << 20, n_streams=2)  # 1 MiB: a toggle run does not fit
    big = W.c2_toggle(seed=3, omega=50.0, R=1024, T=10.0)
    assert _code(B, lambda: srv.submit(big)) == ENOMEM
    assert _code(B, lambda: srv.submit(big.replace(R=0))) == EINVAL
    assert _code(B, lambda: srv.cancel(987654321)) == EINVAL
    small = W.c1_schlogl(seed=3, T=5.0, R=8).replace(hist_hi=(200,))
    t = srv.submit(small, min_runs=2, max_runs=2)
    pooled, info = srv.poll(t)
    assert info["runs"] == 2 and info["status"] == 0
    assert pooled.T_s == pytest.approx(2 * small.T)
    srv.close()


def test_net_of_another_context_rejected(B):
    from paper_1705_06807_amd import binding
    other = binding.Context(0)
    p = W.c1_schlogl(seed=4, T=5.0)
    net_other = other.net(p.net)
    ctx = binding.context()
    ps = binding.problem_struct(p)
    out = binding.Outputs(ctx, p, cycle_log_cap=0)
    rs = out.struct()
    import ctypes as C
    rc = binding.lib().parrep_solve(ctx.h, net_other, C.byref(ps), C.byref(rs), None)
    assert rc == EINVAL
    assert "another context" in binding.lib().parrep_last_error().decode()


def test_empty_batch_rejected(B):
    assert _code(B, lambda: B.parrep_solve_batch([])) == EINVAL


def test_spill_overflow_is_reported(B):
    """Time at states outside the histogram box goes to a 2048-slot spill
    table per run; a run that visits more distinct outside states cannot
    keep their FIM, RER and window-integral terms, and says so: its status
    counter is PARREP_RUN_SPILL_OVERFLOW (3), and a served request that
    pools such a run fails with PARREP_EOVERFLOW (-7), its outputs written."""
    import torch
    # toggle at Omega = 150 visits ~10^4 distinct states in T = 300; a box
    # of one state leaves them all to the spill table
    p = W.c4_toggle(seed=1, R=64, T=300.0, t_cp=1.0).replace(hist_hi=(0, 0))
    g = B.parrep_solve(p, cycle_log_cap=0)
    torch.cuda.synchronize()
    h = g.to_host()
    assert h.T_s == p.T
    assert h.counters["spill_overflow"] > 0 and h.counters["status"] == 3
    # the totals are still whole: the box's one state (the start) plus the outside
    assert h.outside + h.hist.sum() == pytest.approx(p.T, rel=1e-12)
    ok = W.c4_toggle(seed=1, R=64, T=300.0, t_cp=1.0)
    g2 = B.parrep_solve(ok, cycle_log_cap=0)
    torch.cuda.synchronize()
    h2 = g2.to_host()
    assert h2.counters["spill_overflow"] == 0 and h2.counters["status"] == 0
    srv = B.Server(n_streams=1)
    t = srv.submit(p, min_runs=1, max_runs=1)
    assert _code(B, lambda: srv.poll(t)) == -7
    t = srv.submit(ok, min_runs=1, max_runs=1)
    _, info = srv.poll(t)
    assert info["status"] == 0
    srv.close()
