"""Pins of the oracle's accumulators and estimators (CPU).

* time accounting: the ParRep clock ends exactly at T, the histogram holds
  all credited time, the window holds T - t_b;
* the path-space FIM integrand sum_j lam_j grad log lam_j grad log lam_j^T
  (Appendix A; the main text's lam grad lam grad lam^T is a misprint: the
  printed FIM_33 = 200 = bV/c_3 only follows from the log form):
  FIM_33 = B/c_3 exactly on every Schloegl trajectory; the linear identity
  FIM = sum_x hist_w(x) F(x) / (T - t_b) with F written independently;
  the toggle FIM against E_pi[F] from the truncated generator;
* the relative entropy rate (Appendix A): closed form for rates linear in
  c_k, and its Taylor link H ~ 1/2 delta^T FIM delta;
* the paper's printed Schloegl numbers (Tables II-III) reproduced by the
  exact tools, which pins the reading of the FIM formula and of the IAF.
"""
import math
import os

import numpy as np
import pytest

import exact_laws as E
from paper_1705_06807_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden():
    out = {}
    with open(os.path.join(GOLDEN, "paper_schlogl_v25.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v, hw = line.split()[:3]
            out[k] = (float(v), None if hw == "-" else float(hw))
    return out


@pytest.fixture(scope="module")
def c1_runs(oracle):
    return [oracle.run(W.c1_schlogl(seed=0, instance_id=i)) for i in range(3)]


def test_time_accounting(c1_runs):
    for r in c1_runs:
        assert r.T_s == 200.0
        assert r.hist.sum() + r.outside == pytest.approx(200.0, rel=1e-13)
        assert r.hist_w.sum() + r.outside_w == pytest.approx(100.0, rel=1e-13)
        assert np.all(r.hist_w <= r.hist * (1 + 1e-15) + 1e-300)
        c = r.counters
        assert c["status"] == 0 and c["end_phase"] in (1, 3)
        assert c["n_cycle_log"] == c["cycles"] + 1
        log = r.cycle_log
        assert np.array_equal(log[-1, 6:7], r.x_final)
        # cycle records add up to the counters
        assert log[:, 1].sum() == c["ev_decorr"]
        assert log[:, 2].sum() == c["s2_rounds"]
        assert log[:, 3].sum() == c["s3_rounds"]


def test_fim33_exact_on_every_trajectory(c1_runs):
    # lam_3 = c3 B does not depend on x: FIM_33 = lam_3 (1/c3)^2 = B / c3.
    for r in c1_runs:
        assert r.fim[2, 2] == pytest.approx(2e5 / 1e-3, rel=1e-13)


def test_schlogl_fim_linear_identity(c1_runs):
    c = np.array(W.SCHLOGL_CLASSIC_C)
    x = np.arange(1001)
    lam = E.schlogl_classic_rates(x)
    for r in c1_runs:
        assert r.outside_w == 0.0
        ref = np.array([np.dot(r.hist_w, lam[k]) / c[k] ** 2 for k in range(4)]) / 100.0
        np.testing.assert_allclose(np.diag(r.fim), ref, rtol=1e-12)
        off = r.fim - np.diag(np.diag(r.fim))
        assert np.all(off == 0.0)
        # Y_f = int_{t_b}^T x ds
        assert r.y[0] == pytest.approx(np.dot(r.hist_w, x), rel=1e-12)


def test_schlogl_rer_closed_form(c1_runs):
    # each lam_k is proportional to c_k, so perturbing c_k by (1+eps) gives
    # H_k = E[lam_k] (eps - log(1 + eps)), and H_k ~ 1/2 (eps c_k)^2 FIM_kk
    eps = 0.01
    c = np.array(W.SCHLOGL_CLASSIC_C)
    lam = E.schlogl_classic_rates(np.arange(1001))
    for r in c1_runs:
        ref = np.array([np.dot(r.hist_w, lam[k]) for k in range(4)]) / 100.0 * (eps - math.log1p(eps))
        np.testing.assert_allclose(r.rer, ref, rtol=1e-9)
        taylor = 0.5 * (eps * c) ** 2 * np.diag(r.fim)
        np.testing.assert_allclose(r.rer, taylor, rtol=2 * eps)


def test_toggle_fim_and_rer_identity(oracle):
    om = 5.0
    p = W.c2_toggle(seed=3, omega=om, R=8, T=2e3).replace(hist_hi=(60, 60), decorr=3.0,
                                                          dephase=3.0)
    r = oracle.run(p)
    assert r.outside_w == 0.0
    g = np.arange(61)
    U, V = np.meshgrid(g, g, indexing="ij")
    F = E.toggle_fim_integrand(U.ravel(), V.ravel(), om)
    win = p.T - p.t_burn
    ref = np.einsum("s,sab->ab", r.hist_w.ravel(), F) / win
    np.testing.assert_allclose(r.fim, ref, rtol=1e-10, atol=1e-14)
    # RER: perturb each of (a1, a2, beta, gamma) by 1%
    lam = E.toggle_rates(U.ravel(), V.ravel(), om)
    for k in range(4):
        cp = list(W.TOGGLE_C)
        cp[k] *= 1.01
        lp = E.toggle_rates(U.ravel(), V.ravel(), om, cp)
        with np.errstate(divide="ignore", invalid="ignore"):
            h = np.where(lam > 0, lam * np.log(lam / lp) - lam + lp, lp).sum(axis=0)
        ref_k = np.dot(r.hist_w.ravel(), h) / win
        assert r.rer[k] == pytest.approx(ref_k, rel=1e-8)


def test_toggle_fim_statistical(oracle):
    om, N = 5.0, 60
    exact = E.toggle_fim_exact(om, N)
    acc = 0
    for s in range(4):
        p = W.c2_toggle(seed=s, omega=om, R=8, T=2e4).replace(hist_hi=(N, N), decorr=3.0,
                                                              dephase=3.0)
        acc = acc + oracle.run(p).fim
    acc /= 4
    # symmetric network: FIM_11 = FIM_22, FIM_33 = FIM_44 in law
    np.testing.assert_allclose(acc, exact, rtol=0.03, atol=0.01 * np.abs(exact).max())


def test_c1_low_well_law(oracle):
    # T = 200 from x0 = 85 samples the x < 250 well only (mean switching time
    # ~2.4e4): pooled over seeds the histogram is the stationary law
    # conditioned on x < 250 within TV 0.01.
    pi = E.schlogl_classic_pi(1000)
    low = np.zeros_like(pi)
    low[:250] = pi[:250] / pi[:250].sum()
    H = 0
    for i in range(128):
        H = H + oracle.run(W.c1_schlogl(seed=0, instance_id=i)).hist
    assert E.tv(H / H.sum(), low) < 0.01


def test_absorbing_state_run(oracle):
    # X -> 0 at rate x from x0 = 5: absorbed at 0 (a0 = 0, infinite holding
    # time); the run ends in decorrelation with the remaining time at x = 0.
    p = W.Problem(net=W.pure_death(), c=(1.0,), x0=(5,), region_w=(1,), region_theta=100, R=4,
                  decorr_mode=W.STEPS, decorr=10, T=50.0, t_burn=25.0, hist_lo=(0,),
                  hist_hi=(10,), rer_eps=None)
    means = np.zeros(11)
    n = 400
    for i in range(n):
        r = oracle.run(p.replace(instance_id=i))
        assert r.T_s == 50.0 and r.x_final[0] == 0 and r.counters["end_phase"] == 1
        assert r.hist.sum() == pytest.approx(50.0, rel=1e-13)
        means += r.hist
    means /= n
    # mean holding time at k is 1/k (k = 1..5)
    for k in range(1, 6):
        assert means[k] == pytest.approx(1.0 / k, rel=5.0 / math.sqrt(n))


def test_event_budget(oracle):
    r = oracle.run(W.c1_schlogl().replace(max_events=5000))
    assert r.counters["status"] == 1 and r.counters["end_phase"] == 9
    assert r.events <= 5000 and r.T_s < 200.0


def test_no_replicas_needed_when_decorrelation_never_ends(oracle):
    r = oracle.run(W.c1_schlogl().replace(decorr_mode=W.STEPS, decorr=1e18))
    c = r.counters
    assert c["ev_dephase"] == 0 and c["ev_par_credited"] == 0 and c["end_phase"] == 1


def test_paper_tables_from_exact_laws():
    g = _golden()
    V = 25.0
    c = np.array(W.SCHLOGL_PAPER_C)
    x = np.arange(401)
    pi = E.schlogl_paper_pi(400, V=V)
    lam = E.schlogl_paper_rates(x, V=V)
    assert E.schlogl_rre_roots()[1] * V == pytest.approx(g["unstable_point_times_V"][0], abs=1e-4)
    fim = np.array([np.dot(pi, lam[k]) / c[k] ** 2 for k in range(4)])
    for k in (0, 3):  # inside the printed 95% half-widths
        v, hw = g["fim_%d%d" % (k + 1, k + 1)]
        assert abs(fim[k] - v) < 1.05 * hw
    assert fim[2] == pytest.approx(g["fim_33"][0], rel=1e-14)  # 200 = b V / c3 exactly
    # FIM_22: exact 1626 vs printed 1670 +- 5.66 (outside the half-width)
    assert 1600 < fim[1] < 1650
    iaf = E.birth_death_iaf(pi, lam[0] + lam[2], x.astype(float))
    assert iaf == pytest.approx(g["iaf_x"][0], rel=0.15)  # printed from N = 100 runs
    # Table III bounds are sqrt(IAF * FIM_kk) with the printed IAF and FIM_11,
    # FIM_33, FIM_44; the printed c2 bound matches the exact FIM_22, not the
    # printed one, so Table II's 1.67e3 reads as a misprint.
    for k in (0, 2, 3):
        b = math.sqrt(g["iaf_x"][0] * g["fim_%d%d" % (k + 1, k + 1)][0])
        assert b == pytest.approx(g["bound_c%d" % (k + 1)][0], rel=0.005)
    assert math.sqrt(g["iaf_x"][0] * fim[1]) == pytest.approx(g["bound_c2"][0], rel=0.005)
    assert math.sqrt(g["iaf_x"][0] * g["fim_22"][0]) > 1.01 * g["bound_c2"][0]
    # CME sensitivities: c1, c3, c4 match; c2 is printed with the wrong sign and value
    for k in (0, 2, 3):
        s = E.schlogl_paper_sensitivity(k, V=V)
        assert s == pytest.approx(g["cme_sens_c%d" % (k + 1)][0], rel=0.005)
    assert E.schlogl_paper_sensitivity(1, V=V) < 0
    # the bounds dominate the sensitivities
    for k in range(4):
        assert abs(E.schlogl_paper_sensitivity(k, V=V)) <= g["bound_c%d" % (k + 1)][0]


# ----------------------------------------------------------------------------
# Multi-run estimators (Sec. III): the oracle's or_estimate
# ----------------------------------------------------------------------------

def test_estimate_hand_example(oracle):
    """Three runs of a 2-parameter, 1-species problem, window 2, by hand:
    FIM_11 = 1, 2, 3 -> mean 2, sample variance 1, half-width 1.96/sqrt(3);
    Y = 10, 12, 14 -> mean 12, squared deviations 8, IAF = 8 / (2 * 2) = 2;
    bound_1 = sqrt(2 * 2) = 2, bound_2 = sqrt(2 * 8) = 4."""
    fim = np.array([[[1.0, 0.5], [0.5, 8.0]], [[2.0, 0.5], [0.5, 8.0]], [[3.0, 0.5], [0.5, 8.0]]])
    rer = np.array([[0.1, 0.2], [0.3, 0.2], [0.5, 0.2]])
    y = np.array([[10.0], [12.0], [14.0]])
    e = oracle.estimate(fim, rer, y, window=2.0)
    assert e["fim_mean"].tolist() == [[2.0, 0.5], [0.5, 8.0]]
    assert e["fim_hw"][0] == pytest.approx(1.96 / math.sqrt(3.0), rel=1e-15)
    assert e["fim_hw"][1] == 0.0
    assert e["rer_mean"] == pytest.approx([0.3, 0.2], rel=1e-15)
    assert e["y_mean"].tolist() == [12.0]
    assert e["iaf"].tolist() == [2.0]
    assert e["bound"].tolist() == [[2.0, 4.0]]


def test_estimate_reproduces_table3_from_table2(oracle):
    """Table III's bounds are sqrt(IAF FIM_kk) of Table II's FIM and the printed
    IAF 5.87e5 (Sec. IV A): two runs whose FIM diagonals average to Table II's
    values (FIM_22 taken exact, A20) and whose window integrals are spread so
    that the IAF is 5.87e5; the estimator's bounds match Table III to 0.5 %."""
    g = _golden()
    V = 25.0
    c = np.array(W.SCHLOGL_PAPER_C)
    x = np.arange(401)
    pi = E.schlogl_paper_pi(400, V=V)
    lam = E.schlogl_paper_rates(x, V=V)
    fim22 = float(np.dot(pi, lam[1]) / c[1] ** 2)
    diag = np.array([g["fim_11"][0], fim22, g["fim_33"][0], g["fim_44"][0]])
    fim = np.stack([np.diag(diag * 0.9), np.diag(diag * 1.1)])
    rer = np.zeros((2, 4))
    window = 1e5
    # two runs: sum of squared deviations = 2 d^2 = IAF * window * (n - 1)
    d = math.sqrt(g["iaf_x"][0] * window / 2.0)
    y = np.array([[7.2e6 - d], [7.2e6 + d]])
    e = oracle.estimate(fim, rer, y, window=window)
    assert e["iaf"][0] == pytest.approx(g["iaf_x"][0], rel=1e-12)
    assert e["fim_mean"].diagonal() == pytest.approx(diag, rel=1e-15)
    for k in range(4):
        assert e["bound"][0, k] == pytest.approx(g["bound_c%d" % (k + 1)][0], rel=0.005), k


def test_estimate_is_unbiased(oracle):
    """Runs with i.i.d. normal FIM entries (variance s2) and window integrals of
    variance v * window: averaged over 400 batches of 20 runs, the squared
    half-width times n / 1.96^2 estimates s2 and the IAF estimates v, both to
    within the sampling error of the average (about 1.6 %)."""
    rng = np.random.default_rng(3)
    n, reps, window, s2, v = 20, 400, 50.0, 4.0, 3.0
    hw2, iafs = [], []
    for _ in range(reps):
        fim = np.zeros((n, 1, 1))
        fim[:, 0, 0] = 10.0 + math.sqrt(s2) * rng.standard_normal(n)
        y = (100.0 + math.sqrt(v * window) * rng.standard_normal(n))[:, None]
        e = oracle.estimate(fim, np.zeros((n, 1)), y, window=window)
        hw2.append(e["fim_hw"][0] ** 2 * n / 1.96 ** 2)
        iafs.append(e["iaf"][0])
    assert np.mean(hw2) == pytest.approx(s2, rel=0.05)
    assert np.mean(iafs) == pytest.approx(v, rel=0.05)
