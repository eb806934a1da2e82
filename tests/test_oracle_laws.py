"""Statistical pins of the oracle against exact laws (CPU).

* plain SSA (decorrelation that never ends) against the exact stationary law;
* full ParRep (Alg. 1) against the exact stationary law, for several R
  (the accuracy does not depend on R, Sec. IV A);
* the parallel step from exact quasi-stationary samples: the exit index
  R(N*-1)+K is geometric with the embedded chain's rate, for every R
  (Sec. II A, properties 1 and 2), and the credited time has the serial mean;
* Fleming-Viot dephasing against the law of the embedded chain conditioned
  on survival.
"""
import math

import numpy as np
import pytest
from scipy import stats

import exact_laws as E
from paper_1705_06807_amd import workloads as W

N5 = 60  # truncation of the Omega = 5 toggle lattice (boundary mass < 1e-16)


@pytest.fixture(scope="module")
def toggle5_pi():
    _, pi = E.toggle_pi(5.0, N5)
    return pi


def _toggle5(seed, R, T, **kw):
    return W.c2_toggle(seed=seed, omega=5.0, R=R, T=T, t_cp=1.0).replace(hist_hi=(N5, N5), **kw)


def test_ssa_poisson_law(oracle):
    # 0 -> X at rate 5, X -> 0 at rate x: stationary law Poisson(5).
    net = W.birth_death()
    p = W.Problem(net=net, c=(5.0, 1.0), x0=(0,), region_w=(1,), region_theta=1000, R=4,
                  decorr_mode=W.STEPS, decorr=1e18, T=2e4, t_burn=1e4, hist_lo=(0,),
                  hist_hi=(40,), rer_eps=None, seed=1)
    r = oracle.run(p)
    assert r.counters["ev_dephase"] == 0 and r.counters["cycles"] == 0
    law = stats.poisson(5.0).pmf(np.arange(41))
    assert E.tv(r.hist / r.hist.sum(), law) < 0.015
    # and it is not, e.g., Poisson(4.9)
    assert E.tv(r.hist / r.hist.sum(), stats.poisson(4.9).pmf(np.arange(41))) > 0.005


def test_ssa_toggle_law(oracle, toggle5_pi):
    H = 0
    for s in range(4):
        r = oracle.run(_toggle5(s, 8, 2e4, decorr_mode=W.STEPS, decorr=1e18))
        H = H + r.hist
    assert E.tv(H / H.sum(), toggle5_pi) < 0.02


@pytest.mark.parametrize("R", [2, 8, 32])
def test_parrep_toggle_law_independent_of_R(oracle, toggle5_pi, R):
    H = 0
    cycles = 0
    for s in range(4):
        r = oracle.run(_toggle5(s, R, 2e4, decorr=3.0, dephase=3.0))
        H = H + r.hist
        cycles += r.counters["cycles"]
    assert cycles > 1000  # many metastable exits were simulated by the parallel step
    assert E.tv(H / H.sum(), toggle5_pi) < 0.02


def test_parrep_short_thresholds_are_biased(oracle, toggle5_pi):
    # ParRep is only asymptotically exact in the decorrelation/dephasing
    # thresholds (Sec. II B): with t_c = t_p = 1 and many replicas the
    # stationary estimate is visibly off.  The test guards the pins above
    # from being vacuous.
    H = 0
    for s in range(2):
        r = oracle.run(_toggle5(s, 64, 1e4, decorr=1.0, dephase=1.0))
        H = H + r.hist
    assert E.tv(H / H.sum(), toggle5_pi) > 0.05


def test_parrep_paper_schlogl_law(oracle):
    # The paper's Schloegl network (Table I) at V = 10, STEPS thresholds, the
    # separatrix at the unstable RRE point times V (Sec. IV A).
    V = 10.0
    theta = int(math.ceil(E.schlogl_rre_roots()[1] * V))
    pi = E.schlogl_paper_pi(400, V=V)
    H = 0
    cycles = 0
    for s in range(4):
        p = W.paper_schlogl_problem(seed=s, R=16, n_c=200, n_p=200, T=2e3, V=V).replace(
            hist_hi=(400,), region_theta=theta)
        r = oracle.run(p)
        H = H + r.hist
        cycles += r.counters["cycles"]
    assert cycles > 200
    assert E.tv(H / H.sum(), pi) < 0.03


@pytest.fixture(scope="module")
def toggle2_qsd():
    om, N = 2.0, 30
    L, Q = E.toggle_generator(om, N)
    U, V = L.states()
    in_W = (V - U) < 0  # the set u > v (region 0 of the half-space test v - u >= 0)
    PW, Wi = E.embedded_substochastic(L, Q, in_W)
    nu, rho = E.qsd_embedded(PW)
    a0 = E.toggle_rates(U, V, om).sum(axis=0)
    return dict(om=om, U=U, V=V, PW=PW, Wi=Wi, nu=nu, rho=rho, a0=a0)


@pytest.mark.parametrize("R", [1, 4, 16])
def test_exit_law_from_qsd(oracle, toggle2_qsd, R):
    q = toggle2_qsd
    rng = np.random.default_rng(100 + R)
    n = 3000
    idx = np.empty(n)
    cred = np.empty(n)
    for t in range(n):
        st = rng.choice(len(q["nu"]), size=R, p=q["nu"])
        init = np.stack([q["U"][q["Wi"][st]], q["V"][q["Wi"][st]]], axis=1)
        p = W.c2_toggle(seed=5, instance_id=t, omega=q["om"], R=R)
        ns, K, xs, c = oracle.parallel(p, init)
        assert ns >= 1 and 1 <= K <= R
        assert xs[0] <= xs[1]  # the exit state has left {u > v}
        idx[t] = R * (ns - 1) + K
        cred[t] = c
    p_exit = 1.0 - q["rho"]
    mean = 1.0 / p_exit
    sd = math.sqrt(q["rho"]) / p_exit
    assert abs(idx.mean() - mean) < 4 * sd / math.sqrt(n)
    # distribution: geometric in 10 equiprobable bins
    edges = np.unique(np.ceil(stats.geom(p_exit).ppf(np.linspace(0, 1, 11)[1:-1])).astype(int))
    h = np.histogram(idx, bins=np.concatenate([[0], edges, [np.inf]]))[0]
    cdf = stats.geom(p_exit).cdf(np.concatenate([edges, [np.inf]]))
    e = np.diff(np.concatenate([[0], cdf])) * n
    chi2 = ((h - e) ** 2 / e).sum()
    assert chi2 < stats.chi2(len(h) - 1).ppf(0.9999)
    # the credited time has the serial mean nu(1/a0) / (1 - rho)
    mt = float(np.dot(q["nu"], 1.0 / q["a0"][q["Wi"]])) / p_exit
    assert abs(cred.mean() - mt) < 4.5 * cred.std() / math.sqrt(n)


def test_exit_state_law_independent_of_R(oracle, toggle2_qsd):
    q = toggle2_qsd
    rng = np.random.default_rng(9)
    states = {}
    for R in (1, 16):
        xs_all = []
        for t in range(2000):
            st = rng.choice(len(q["nu"]), size=R, p=q["nu"])
            init = np.stack([q["U"][q["Wi"][st]], q["V"][q["Wi"][st]]], axis=1)
            p = W.c2_toggle(seed=6, instance_id=t, omega=q["om"], R=R)
            _, _, xs, _ = oracle.parallel(p, init)
            xs_all.append(tuple(xs))
        states[R] = xs_all
    keys = sorted(set(states[1]) | set(states[16]))
    tab = np.array([[states[R].count(k) for k in keys] for R in (1, 16)])
    tab = tab[:, tab.sum(axis=0) >= 10]
    _, pval, _, _ = stats.chi2_contingency(tab)
    assert pval > 1e-4


def test_fleming_viot_conditioned_law(oracle):
    om, N = 5.0, N5
    L, Q = E.toggle_generator(om, N)
    U, V = L.states()
    in_W = (V - U) < 0
    PW, Wi = E.embedded_substochastic(L, Q, in_W)
    start = (12, 3)
    s0 = int(np.flatnonzero((U[Wi] == start[0]) & (V[Wi] == start[1]))[0])
    n_p = 24
    exact = E.conditioned_law(PW, s0, n_p)
    wrong = E.conditioned_law(PW, s0, n_p - 1)  # other parity class
    R = 4096
    counts = np.zeros(len(Wi))
    lookup = {(int(U[w]), int(V[w])): i for i, w in enumerate(Wi)}
    for seed in range(3):
        p = W.c2_toggle(seed=seed, omega=om, R=R).replace(dephase_mode=W.STEPS, dephase=n_p)
        Y, rounds = oracle.dephase(p, start)
        assert rounds == n_p
        for u, v in Y:
            counts[lookup[(int(u), int(v))]] += 1
    emp = counts / counts.sum()
    assert E.tv(emp, exact) < 0.04
    assert E.tv(emp, wrong) > 0.9


def test_time_mode_dephasing_rounds(oracle):
    # time mode stops after the first round with min_r t^r >= t_p: more time
    # means more rounds, and a zero threshold means none
    p = W.c2_toggle(seed=0, omega=5.0, R=64)
    rounds = []
    for tp in (0.0, 0.5, 2.0):
        _, n = oracle.dephase(p.replace(dephase=tp), (12, 3))
        rounds.append(n)
    assert rounds[0] == 0 and 0 < rounds[1] < rounds[2]


def _self_repressor():
    # 0 -> X at c0 / (1 + (x / 5) ** c2), X -> 0 at c1 x: a birth-death chain
    # whose Hill exponent is a parameter, here not an integer
    return W.Network(
        name="self_repressor", n_species=1, n_params=3, param_names=("k", "gamma", "n"),
        reactions=(
            W.Reaction(0, 1.0, (W.Factor(W.HILL_REP, 0, K=5.0, hill_param=2),), (1,)),
            W.Reaction(1, 1.0, (W.Factor(W.FALLING, 0, order=1),), (-1,)),
        ))


def _repressor_pi(c, N):
    x = np.arange(N + 1, dtype=np.float64)
    return E.birth_death_pi(c[0] / (1.0 + (x / 5.0) ** c[2]), c[1] * x)


def test_ssa_law_non_integral_hill_exponent(oracle):
    """The GPU takes integral Hill exponents only; the oracle also evaluates
    non-integral ones.  Pinned by the product-form stationary law of the
    birth-death chain (Sec. I A's generator with one species): exponent 2.5
    matches, while exponents 2.3 and 2.7 (and the integers around 2.5) are
    rejected by the same statistic."""
    c = (40.0, 1.0, 2.5)
    p = W.Problem(net=_self_repressor(), c=c, x0=(0,), region_w=(1,), region_theta=1000, R=4,
                  decorr_mode=W.STEPS, decorr=1e18, T=1e5, t_burn=1e3, hist_lo=(0,),
                  hist_hi=(60,), rer_eps=None, seed=3)
    r = oracle.run(p)
    assert r.counters["cycles"] == 0 and r.outside == 0.0
    h = r.hist / r.hist.sum()
    assert E.tv(h, _repressor_pi(c, 60)) < 0.006
    for n in (2.0, 2.3, 2.7, 3.0):
        assert E.tv(h, _repressor_pi((c[0], c[1], n), 60)) > 0.035, n


def _chi2_ok(counts, probs, min_expected=5.0, q=1e-4):
    """Chi-square goodness of fit with adjacent cells merged until each
    expects at least min_expected; True when the fit is not rejected at
    level q."""
    n = counts.sum()
    cells_o, cells_e = [], []
    acc_o = acc_e = 0.0
    for o, p in zip(counts, probs):
        acc_o += o
        acc_e += p * n
        if acc_e >= min_expected:
            cells_o.append(acc_o)
            cells_e.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0 or acc_o > 0:
        cells_o[-1] += acc_o
        cells_e[-1] += acc_e
    o = np.array(cells_o)
    e = np.array(cells_e)
    chi2 = ((o - e) ** 2 / e).sum()
    return chi2 < stats.chi2(len(o) - 1).ppf(1.0 - q), chi2, len(o)


@pytest.mark.parametrize("R", [1, 16, 256])
def test_time_mode_dephasing_stop_law(oracle, R):
    """Dephasing in time mode stops after the first round at which every
    replica's own elapsed time has reached t_p (Alg. 1, dephasing step).
    With a constant total rate a0 and one set holding every state, no
    replica restarts, each replica's elapsed time after n rounds is a sum of
    n iid Exp(a0), and the round count N = max_r n_r follows
    P(N <= n) = P(Poisson(a0 t_p) <= n - 1)^R exactly.  Stopping on the
    largest elapsed time instead (N = min_r n_r), or one round early or
    late, is rejected at R = 16 and 256."""
    a0, t_p = 4.0, 2.5
    n_samp = 3000 if R < 256 else 1500
    rounds = np.empty(n_samp, dtype=np.int64)
    for i in range(n_samp):
        p = W.self_loop_problem(seed=R, instance_id=i, rate=a0, R=R, t_p=t_p)
        Y, n = oracle.dephase(p, (0,), cycle=i % 7)
        assert (Y == 0).all()
        rounds[i] = n
    n_max = int(rounds.max()) + 40
    cdf = E.dephase_rounds_cdf(a0, t_p, R, n_max)
    pmf = np.diff(np.concatenate([[0.0], cdf]))
    counts = np.bincount(rounds, minlength=n_max + 1)[:n_max + 1].astype(float)
    ok, chi2, cells = _chi2_ok(counts, pmf)
    assert ok, (chi2, cells)
    if R > 1:
        # the same statistic rejects the plausible misreadings
        cdf_min = 1.0 - (1.0 - E.dephase_rounds_cdf(a0, t_p, 1, n_max)) ** R
        for wrong in (cdf_min, np.concatenate([[0.0], cdf[:-1]]), np.concatenate([cdf[1:], [1.0]])):
            pw = np.clip(np.diff(np.concatenate([[0.0], wrong])), 1e-300, None)
            assert not _chi2_ok(counts, pw)[0]


def test_time_mode_decorrelation_stop_law(oracle):
    """Decorrelation in time mode ends at the first jump after which the
    process has spent t_c in its current set without interruption; leaving
    the set makes the new set current and restarts the time (Alg. 1,
    decorrelation step).  On the flip chain every jump leaves the set with
    probability p = c2/(c1+c2) and the holding times are iid Exp(c1+c2), so
    the number of decorrelation events per cycle has the renewal law of
    decorr_events_pmf.  Not restarting the time on leaving the set, or also
    counting the holding time of the jump that leaves it, gives other laws
    that the same statistic rejects."""
    c1, c2, t_c = 3.0, 1.0, 1.0
    a0, pf = c1 + c2, c2 / (c1 + c2)
    s1 = []
    for seed in range(3):
        r = oracle.run(W.flip_chain_problem(seed=seed, c1=c1, c2=c2, t_c=t_c, T=2e4),
                       cycle_log_cap=40000)
        log = r.cycle_log
        assert r.counters["n_cycle_log"] <= 40000 and len(log) > 3000
        s1.extend(int(v) for v in log[:-1, 1])  # the last cycle is cut by the horizon
    s1 = np.array(s1)
    k_max = int(s1.max()) + 60
    pmf = E.decorr_events_pmf(a0, pf, t_c, k_max)
    counts = np.bincount(s1, minlength=k_max + 1)[:k_max + 1].astype(float)
    ok, chi2, cells = _chi2_ok(counts, pmf)
    assert ok, (chi2, cells)
    # no restart: K = jumps until the in-set holding times alone reach t_c
    rng = np.random.default_rng(0)
    no_reset = []
    with_exit_time = []
    for _ in range(40000):
        e, k = 0.0, 0
        while not e >= t_c:
            tau = rng.exponential(1.0 / a0)
            k += 1
            if rng.random() >= pf:
                e += tau
        no_reset.append(k)
        e, k = 0.0, 0
        while not e >= t_c:
            tau = rng.exponential(1.0 / a0)
            k += 1
            e = tau if rng.random() < pf else e + tau
        with_exit_time.append(k)
    for wrong in (no_reset, with_exit_time):
        pw = np.bincount(np.array(wrong), minlength=k_max + 1)[:k_max + 1] / len(wrong)
        assert not _chi2_ok(counts, np.clip(pw, 1e-12, None))[0]
