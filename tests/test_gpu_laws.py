"""GPU accuracy against exact laws: pooled stationary histograms of the HIP
path within total variation 0.01 of the closed-form birth-death law (Schloegl)
and of the truncated-generator stationary vector (toggle switch), and the
FIM of the benchmark workload against its exact value."""
import sys

import numpy as np
import pytest

import exact_laws as E
from paper_1705_06807_amd import workloads as W

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


def _pooled(B, probs):
    import torch
    outs = B.parrep_solve_batch(probs, cycle_log_cap=0)
    torch.cuda.synchronize()
    shape = tuple(hi - lo + 1 for lo, hi in zip(probs[0].hist_lo, probs[0].hist_hi))
    H = sum(o.hist.double() for o in outs).cpu().numpy().reshape(shape)
    Hw = sum(o.hist_window.double() for o in outs).cpu().numpy().reshape(shape)
    fim = sum(o.stats[3:3 + 16].double() for o in outs).cpu().numpy() / len(outs)
    outside = sum(float(o.stats[1]) for o in outs)
    return H, Hw, fim.reshape(4, 4) if len(fim) == 16 else fim, outside


def test_c1_low_well_tv(B):
    # C1 (T = 200 from x0 = 85) samples the x < 250 well: pooled over 256
    # trajectories the histogram is the stationary law conditioned on x < 250
    pi = E.schlogl_classic_pi(1000)
    low = np.zeros_like(pi)
    low[:250] = pi[:250] / pi[:250].sum()
    H, _, _, _ = _pooled(B, [W.c1_schlogl(seed=0, instance_id=i) for i in range(256)])
    tv = E.tv(H / H.sum(), low)
    _flush("C1 pooled TV vs conditioned law: %.4f" % tv)
    assert tv < 0.01


def test_toggle_omega5_tv(B):
    # weak metastability (switching every ~12 time units): few replicas and
    # t_c = t_p = 3, the regime where the oracle's own law test holds
    N = 60
    _, pi = E.toggle_pi(5.0, N)
    probs = [W.c2_toggle(seed=2, instance_id=i, omega=5.0, R=32, T=2e4, t_cp=3.0)
             .replace(hist_hi=(N, N)) for i in range(64)]
    H, _, _, outside = _pooled(B, probs)
    tv = E.tv(H / (H.sum() + outside), pi)
    _flush("toggle Omega=5 pooled TV vs exact: %.4f" % tv)
    assert tv < 0.02


def test_benchmark_workload_accuracy(B):
    """The benchmark workload (toggle Omega = 50, R = 1024, t_c = t_p = 20,
    T = 2e4) pooled over 1024 trajectories: histogram TV and FIM vs exact
    (the FIM's spread is the noise of the wells' occupation, ~0.7 %)."""
    N = 300
    L, pi = E.toggle_pi(50.0, N)
    U, V = L.states()
    fim_exact = np.einsum("s,sab->ab", pi.ravel(), E.toggle_fim_integrand(U, V, 50.0))
    probs = [W.c2_toggle(seed=0, instance_id=10000 + i) for i in range(1024)]
    _flush("benchmark workload, 1024 trajectories (about 4 s)")
    H, Hw, fim, outside = _pooled(B, probs)
    assert outside == 0.0
    p = np.zeros_like(pi)
    p[:, :] = H[:N + 1, :N + 1] / H.sum()
    tv = E.tv(p, pi)
    rel = np.abs(np.diag(fim) - np.diag(fim_exact)) / np.diag(fim_exact)
    _flush("Omega=50: TV %.4f, FIM diagonal rel. errors %s" % (tv, np.round(rel, 4)))
    assert tv < 0.01
    assert rel.max() < 0.03
