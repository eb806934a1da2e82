"""The allocation-free solve (parrep_solve_noalloc) through the C ABI: its
scratch lives in the library's fixed device array, and its outputs equal
parrep_solve's on the same problem (integers exactly, floats within 1e-12
relative).  Two calls in a row, the second with a smaller problem, so that
the second runs on the first's leftover scratch contents; then a problem
whose scratch exceeds the array is rejected without running."""
import ctypes as C

import numpy as np
import pytest

from paper_1705_06807_amd import workloads as W

pytestmark = pytest.mark.gpu

RTOL = 1e-12


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_06807_amd import binding
    binding.lib()
    return binding


def _same(a, b, what):
    ac, bc = dict(a.counters), dict(b.counters)
    assert ac == bc, (what, ac, bc)
    assert ac["spill_overflow"] == 0 and ac["status"] == 0, what
    assert np.array_equal(a.x_final, b.x_final), what
    assert np.array_equal(a.cycle_log, b.cycle_log), what
    assert a.T_s == b.T_s, what
    for name in ("hist", "hist_w", "fim", "rer", "y"):
        x, y = getattr(a, name), getattr(b, name)
        scale = max(np.abs(x).max(), 1e-300)
        assert np.abs(x - y).max() <= RTOL * scale, (what, name)
        if name.startswith("hist"):
            assert np.array_equal(x != 0, y != 0), (what, name)
    for name in ("outside", "outside_w"):
        assert getattr(a, name) == pytest.approx(getattr(b, name), rel=RTOL, abs=1e-300), what


def test_noalloc_equals_solve(B):
    import torch
    ctx = B.context()
    probs = [
        # larger first: 1024 replicas, a 2-D box, many cycles
        W.c2_toggle(seed=21, instance_id=3, omega=5.0, R=1024, T=200.0, t_cp=1.0).replace(
            hist_hi=(40, 40)),
        # then smaller: fewer replicas, a 1-D box
        W.c1_schlogl(seed=22, instance_id=4, R=32, T=100.0),
    ]
    for p in probs:
        print("noalloc %s R=%d" % (p.net.name, p.R), flush=True)
        ref = B.parrep_solve(p, ctx=ctx, cycle_log_cap=4096)
        out = B.Outputs(ctx, p, cycle_log_cap=4096)
        ctx.net(p.net)
        torch.cuda.synchronize()
        B.parrep_solve_noalloc(p, out, ctx=ctx)
        torch.cuda.synchronize()
        _same(out.to_host(), ref.to_host(), p.net.name)


def test_noalloc_rejects_scratch_beyond_the_array(B):
    import torch
    ctx = B.context()
    big = W.c4_toggle(seed=1, T=10.0)  # R = 65536: about 3 MB of scratch
    out = B.Outputs(ctx, big, cycle_log_cap=0)
    out.stats.fill_(-3.0)
    with pytest.raises(B.ParrepError, match="fixed array holds"):
        B.parrep_solve_noalloc(big, out, ctx=ctx)
    torch.cuda.synchronize()
    assert float(out.stats[0]) == -3.0  # nothing ran
    # and the entry point still works afterwards
    p = W.c1_schlogl(seed=23, R=8, T=20.0)
    ref = B.parrep_solve(p, ctx=ctx, cycle_log_cap=4096)
    o2 = B.Outputs(ctx, p, cycle_log_cap=4096)
    torch.cuda.synchronize()
    B.parrep_solve_noalloc(p, o2, ctx=ctx)
    torch.cuda.synchronize()
    _same(o2.to_host(), ref.to_host(), "after rejection")
