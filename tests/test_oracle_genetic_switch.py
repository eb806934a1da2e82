"""Pins of the oracle on the genetic switch with positive feedback (Sec. IV B).

The oracle evaluates this network through its generic factored propensities
(a rate parameter times parameter factors times state factors; the switching
rates F and G of Eq. (10) are two-level Hill factors).  The pins come from
outside the oracle:

* the equilibria of the rescaled RRE, Eq. (12), that the paper prints: the
  oracle's own F and G (read off its propensities at integer protein counts)
  must bracket and, interpolated, reproduce them;
* Table V: the stationary path-space FIM diagonal.  The exact value is
  E_pi of the per-state FIM integrand, with pi the stationary law of the
  truncated generator (the test helpers write Table IV out again); the exact
  value lies within the paper's confidence intervals, and the average of the
  oracle's per-state FIM over the same law agrees with it to rounding;
* Table VI: the IAFs, as asymptotic variances from the Poisson equation of
  the exact generator (the paper's are estimates, within a few percent);
* the relative entropy rate is the second-order term of the FIM: for a small
  perturbation eps of c_k, RER_k = eps^2 c_k^2 FIM_kk / 2 (1 + O(eps)).  The
  oracle computes RER from propensities alone and the FIM from its analytic
  gradient, so this checks every gradient term of the new factor kinds;
* SSA and ParRep stationary laws at a smaller system size V = 240 against
  the exact stationary law of the generator.
"""
import math
import os

import numpy as np
import pytest

import exact_laws as E
from paper_1705_06807_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    out = {}
    with open(os.path.join(HERE, "golden", "paper_genetic_switch_v2400.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v, hw = line.split()[:3]
            out[k] = (float(v), None if hw == "-" else float(hw))
    return out


G = _golden()
C2400 = W.genetic_switch_c(2400.0)


def _oracle_state(xi, x1, x2):
    # species (DNA_in, DNA_act, mRNA, protein); xi = active DNA
    return (1 - int(xi), int(xi), int(x1), int(x2))


@pytest.fixture(scope="module")
def law2400():
    L, Q, pi = E.genetic_switch_pi(C2400, 14, 3300)
    return L, Q, pi


def test_parameters_are_the_papers():
    a, b, g, k0n, k0x, k1n, k1x, D = C2400
    assert a * b == pytest.approx(2400.0) and b == 22.5 and g == 50.0
    assert k0n == k1n == pytest.approx(24.0 / b) and k0x == k1x == pytest.approx(2400.0 / b)
    assert D == 1000.0


def test_oracle_switching_rates(oracle):
    """The activation and deactivation channels at the end points: F(0) =
    k0min, G(0) = k1max, F -> k0max and G -> k1min as x2 -> infinity, and
    F(D) = G(D) = (k_min + k_max)/2 at x2 = D."""
    net = W.genetic_switch()
    a, b, g, k0n, k0x, k1n, k1x, D = C2400
    lam0, *_ = oracle.event(net, C2400, _oracle_state(0, 0, 0), (1, 2, 3, 4))
    lam1, *_ = oracle.event(net, C2400, _oracle_state(1, 0, 0), (1, 2, 3, 4))
    assert lam0[4] == pytest.approx(k0n, rel=1e-15) and lam1[5] == pytest.approx(k1x, rel=1e-15)
    assert lam0[5] == 0.0 and lam1[4] == 0.0
    lamD0, *_ = oracle.event(net, C2400, _oracle_state(0, 0, 1000), (1, 2, 3, 4))
    lamD1, *_ = oracle.event(net, C2400, _oracle_state(1, 0, 1000), (1, 2, 3, 4))
    assert lamD0[4] == pytest.approx(0.5 * (k0n + k0x), rel=1e-14)
    assert lamD1[5] == pytest.approx(0.5 * (k1n + k1x), rel=1e-14)
    lamH0, *_ = oracle.event(net, C2400, _oracle_state(0, 0, 10 ** 7), (1, 2, 3, 4))
    assert lamH0[4] == pytest.approx(k0x, rel=1e-7)


def test_oracle_gives_the_papers_equilibria(oracle):
    """Fixed points of Eq. (12): x2 = a b p(x2), x1 = x2 / (gamma b), with
    p = F / (F + G).  F and G are taken from the oracle's activation and
    deactivation propensities at integer protein counts; the printed
    equilibria must lie between consecutive integers where x2 - a b p(x2)
    changes sign, and linear interpolation must reproduce them."""
    net = W.genetic_switch()
    a, b, g = C2400[:3]

    def resid(x2):
        F = oracle.event(net, C2400, _oracle_state(0, 0, x2), (1, 2, 3, 4))[0][4]
        Gd = oracle.event(net, C2400, _oracle_state(1, 0, x2), (1, 2, 3, 4))[0][5]
        return x2 - a * b * F / (F + Gd)

    xs = np.arange(0, 2500)
    r = np.array([resid(int(x)) for x in xs])
    roots = []
    for i in np.flatnonzero(np.sign(r[:-1]) != np.sign(r[1:])):
        roots.append(xs[i] + r[i] / (r[i] - r[i + 1]))
    assert len(roots) == 3
    for root, name in zip(roots, ("stable_low", "saddle", "stable_high")):
        want2 = G[name + "_x2"][0]
        assert math.floor(want2) <= root <= math.floor(want2) + 1
        assert root == pytest.approx(want2, abs=2e-3)
        assert root / (g * b) == pytest.approx(G[name + "_x1"][0], abs=6e-5)


def test_exact_fim_within_table5_intervals(law2400):
    L, Q, pi = law2400
    xi, x1, x2 = L.states()
    assert pi[x2 == L.N2].sum() < 1e-6 and pi[x1 == L.N1].sum() < 1e-7
    F = np.einsum("s,sab->ab", pi, E.genetic_switch_fim_integrand(xi, x1, x2, C2400))
    for k in range(8):
        v, hw = G["fim_%d%d" % (k + 1, k + 1)]
        assert abs(F[k, k] - v) < 1.5 * hw, (k, F[k, k], v, hw)


def test_exact_iaf_near_table6(law2400):
    L, Q, pi = law2400
    xi, x1, x2 = L.states()
    for f, key in ((xi, "iaf_active_dna"), (1 - xi, "iaf_inactive_dna"), (x1, "iaf_mrna"),
                   (x2, "iaf_protein")):
        got = E.ctmc_iaf(L, Q, pi, f.astype(np.float64))
        assert got == pytest.approx(G[key][0], rel=0.05), (key, got)


def test_oracle_fim_matches_exact_law_and_table5(oracle, law2400):
    """Average the oracle's per-state FIM over the exact stationary law (the
    states holding all but 1e-12 of the mass): equal to the test helpers' exact
    value to rounding, hence within the Table V intervals; the off-diagonal
    entries are checked too."""
    L, Q, pi = law2400
    xi, x1, x2 = L.states()
    order = np.argsort(pi)[::-1]
    keep = order[: int(np.searchsorted(np.cumsum(pi[order]), 1.0 - 1e-12)) + 1]
    net = W.genetic_switch()
    F = np.zeros((8, 8))
    for s in keep:
        fim, _ = oracle.fim_rer(net, C2400, _oracle_state(xi[s], x1[s], x2[s]))
        F += pi[s] * fim
    X = E.genetic_switch_fim_integrand(xi[keep], x1[keep], x2[keep], C2400)
    Fx = np.einsum("s,sab->ab", pi[keep], X)
    assert np.abs(F - Fx).max() <= 1e-12 * np.abs(Fx).max()
    assert np.allclose(F, Fx, rtol=1e-11, atol=0)
    for k in range(8):
        v, hw = G["fim_%d%d" % (k + 1, k + 1)]
        assert abs(F[k, k] - v) < 1.5 * hw


def test_oracle_rer_is_half_eps2_fim(oracle):
    net = W.genetic_switch()
    eps = 1e-5
    rng = np.random.default_rng(7)
    states = [(0, 0, 0), (1, 0, 0), (0, 0, 1), (1, 3, 1000), (0, 2, 511), (1, 1, 1839),
              (0, 0, 25)] + [(int(rng.integers(0, 2)), int(rng.integers(0, 6)),
                              int(rng.integers(0, 3000))) for _ in range(40)]
    for st in states:
        fim, rer = oracle.fim_rer(net, C2400, _oracle_state(*st), rer_eps=(eps,) * 8)
        want = 0.5 * eps ** 2 * np.asarray(C2400) ** 2 * np.diag(fim)
        for k in range(8):
            if want[k] == 0.0:
                assert rer[k] == 0.0, (st, k)
            else:
                assert rer[k] == pytest.approx(want[k], rel=5e-5), (st, k, rer[k], want[k])


V_SMALL, N1_SMALL, N2_SMALL = 240.0, 8, 700


@pytest.fixture(scope="module")
def law240():
    L, Q, pi = E.genetic_switch_pi(W.genetic_switch_c(V_SMALL), N1_SMALL, N2_SMALL)
    xi, x1, x2 = L.states()
    pi_p = np.bincount(x2, weights=pi, minlength=N2_SMALL + 1)
    pi_sm = np.zeros((2, N1_SMALL + 1))
    np.add.at(pi_sm, (xi, x1), pi)
    return pi_p, pi_sm


def _marginals(h):
    h = h.reshape(2, 2, N1_SMALL + 1, N2_SMALL + 1)
    # only (DNA_in, DNA_act) = (1, 0) and (0, 1) are reachable
    assert h[0, 0].sum() == 0.0 and h[1, 1].sum() == 0.0
    H = np.stack([h[1, 0], h[0, 1]])  # indexed by xi
    return H.sum(axis=(0, 1)) / H.sum(), H.sum(axis=2) / H.sum()


def _run_small(oracle, seeds, R, T, **kw):
    H = 0
    cycles = 0
    for s in seeds:
        p = W.genetic_switch_problem(seed=s, V=V_SMALL, R=R, T=T).replace(
            hist_hi=(1, 1, N1_SMALL, N2_SMALL), **kw)
        r = oracle.run(p)
        assert r.outside == 0.0
        H = H + r.hist
        cycles += r.counters["cycles"]
    return H, cycles


def test_ssa_law_small_volume(oracle, law240):
    pi_p, pi_sm = law240
    H, cycles = _run_small(oracle, (0, 1), 4, 5e4, decorr=1e18)
    assert cycles == 0
    mp, msm = _marginals(H)
    assert E.tv(mp, pi_p) < 0.01 and E.tv(msm, pi_sm) < 0.005


def test_parrep_law_small_volume(oracle, law240):
    pi_p, pi_sm = law240
    H, cycles = _run_small(oracle, (2, 3), 8, 5e4, decorr=500, dephase=500)
    assert cycles > 500
    mp, msm = _marginals(H)
    assert E.tv(mp, pi_p) < 0.012 and E.tv(msm, pi_sm) < 0.01


def test_parrep_short_thresholds_biased_small_volume(oracle, law240):
    # n_c = n_p = 20 steps leave the replicas far from the QSD: the estimate
    # is visibly off (keeps the two tests above from being vacuous)
    pi_p, _ = law240
    H, _ = _run_small(oracle, (4,), 16, 5e4, decorr=20, dephase=20)
    mp, _ = _marginals(H)
    assert E.tv(mp, pi_p) > 0.05
