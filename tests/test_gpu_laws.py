"""GPU accuracy against exact laws: pooled stationary histograms of the HIP
path within total variation 0.01 of the closed-form birth-death law (Schloegl)
and of the truncated-generator stationary vector (toggle switch, genetic
switch), and FIMs against their exact values."""
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
    npar = probs[0].net.n_params
    fim = sum(o.stats[B.ST_FIM:B.ST_FIM + npar * npar].double() for o in outs).cpu().numpy()
    outside = sum(float(o.stats[B.ST_OUTSIDE]) for o in outs)
    return H, Hw, fim.reshape(npar, npar) / len(outs), outside


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
    # weak metastability (switching every ~12 time units), few replicas and
    # t_c = t_p = 3; pooled over 128 trajectories of T = 2e4 (the oracle's
    # own runs of the first 64 of them are at TV 0.0046)
    N = 60
    _, pi = E.toggle_pi(5.0, N)
    probs = [W.c2_toggle(seed=2, instance_id=i, omega=5.0, R=32, T=2e4, t_cp=3.0)
             .replace(hist_hi=(N, N)) for i in range(128)]
    H, _, _, outside = _pooled(B, probs)
    tv = E.tv(H / (H.sum() + outside), pi)
    _flush("toggle Omega=5 pooled TV vs exact: %.4f" % tv)
    assert tv < 0.01


def test_large_single_run_within_well_tv(B):
    """The large single run (toggle Omega = 150, R = 65536, t_c = t_p = 20,
    T = 1e5, one instance spread over 256 workgroups) never leaves the well
    it first falls into: its switching time is ~1e7.  Pooled over 64 runs
    (each reflected into the u > v well, the law being symmetric under
    u <-> v), the histogram is within TV 0.01 of the stationary law
    restricted to that well (a truncated-generator solve on a box 7 standard
    deviations around it)."""
    import torch
    box = (220, 620, 0, 150)
    law = E.toggle_well_law(150.0, *box)
    ctx = B.context()
    pooled = np.zeros((1201, 1201))
    total = 0.0
    for i in range(64):
        p = W.c4_toggle(seed=5, instance_id=i)
        out = B.parrep_solve_batch([p], ctx=ctx, cycle_log_cap=0)[0]
        torch.cuda.synchronize()
        h = out.to_host()
        assert h.counters["status"] == 0 and h.T_s == p.T
        H = h.hist
        if np.triu(H, 1).sum() > np.tril(H, -1).sum():  # mass at v > u: reflect
            H = H.T
        pooled += H
        total += h.T_s
    inbox = pooled[box[0]:box[1] + 1, box[2]:box[3] + 1] / total
    tv = 0.5 * (np.abs(inbox - law).sum() + (1.0 - inbox.sum()))
    _flush("Omega=150 large single run, 64 runs: TV within the well %.4f" % tv)
    assert tv < 0.01


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


def test_genetic_switch_small_volume_law(B):
    """Genetic switch (Sec. IV B) at V = 240, R = 8, n_c = n_p = 2000 steps,
    pooled over 1024 trajectories: window histogram marginals against the
    exact stationary law of the generator, and the FIM diagonal against
    E_pi of the exact FIM integrand.  The FIM entries of the switching
    parameters hang on the rarely visited upper well (10 % of the mass at
    this size): over 2e5 time units the oracle's ParRep estimate of them
    scatters by about 5 %, so the pooled window here is 5e6."""
    V, N1, N2 = 240.0, 8, 700
    c = W.genetic_switch_c(V)
    L, _, pi = E.genetic_switch_pi(c, N1, N2)
    xi, x1, x2 = L.states()
    pi_p = np.bincount(x2, weights=pi, minlength=N2 + 1)
    pi_sm = np.zeros((2, N1 + 1))
    np.add.at(pi_sm, (xi, x1), pi)
    fim_exact = np.einsum("s,sab->ab", pi, E.genetic_switch_fim_integrand(xi, x1, x2, c))
    probs = [W.genetic_switch_problem(seed=3, instance_id=i, V=V, R=8, n_c=2000, n_p=2000,
                                      T=1e4).replace(hist_hi=(1, 1, N1, N2))
             for i in range(1024)]
    _flush("genetic switch V=240, 1024 trajectories")
    _, Hw, fim, outside = _pooled(B, probs)
    assert outside < 1e-6 * Hw.sum()
    assert Hw[0, 0].sum() == 0.0 and Hw[1, 1].sum() == 0.0
    Hx = np.stack([Hw[1, 0], Hw[0, 1]])  # indexed by xi (active DNA)
    tv_p = E.tv(Hx.sum(axis=(0, 1)) / Hx.sum(), pi_p)
    tv_sm = E.tv(Hx.sum(axis=2) / Hx.sum(), pi_sm)
    rel = np.abs(np.diag(fim) - np.diag(fim_exact)) / np.diag(fim_exact)
    _flush("genetic switch: TV protein %.4f, TV (xi, mRNA) %.4f, FIM rel. errors %s"
           % (tv_p, tv_sm, np.round(rel, 4)))
    assert tv_p < 0.01 and tv_sm < 0.005
    assert rel.max() < 0.04
