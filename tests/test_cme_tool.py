"""Pins of the host CME sensitivity tool (paper_1705_06807_amd.cme).

Each check compares the tool with something fixed independently of it:
* Table III (Sec. IV A): the CME sensitivities of the Schloegl mean for c1,
  c3 and c4 on the box [0, 149] (the printed c2 entry disagrees with the
  closed form in sign and size, so it is not used);
* the birth-death closed form of the Schloegl stationary law, differentiated
  by central differences;
* two-species networks whose stationary mean has a closed form (species 0
  is an immigration-death process, so its law is Poisson; species 1 is born
  at a rate that depends on species 0 through a Hill factor and dies
  linearly, so E[x1] = E[birth rate] / death rate), one per factor kind,
  differentiated by central differences of the closed form;
* the toggle's stationary law and, by central differences of it, its
  sensitivities, from the tests' own truncated-generator solve, which shares
  no code with the tool.
"""
import math

import numpy as np
import pytest

from paper_1705_06807_amd import cme
from paper_1705_06807_amd import workloads as W

import exact_laws as X


def _mean_x0(Xs):
    return Xs[:, 0]


def _mean_x1(Xs):
    return Xs[:, 1]


def test_table3_schloegl_sensitivities():
    """Table III 'CME Approx.' row: 4.07E+02, 6.30E+02, -2.65E+02 for c1, c3, c4."""
    E, d = cme.expectation_sensitivity(W.schlogl_paper(25.0), W.SCHLOGL_PAPER_C,
                                       cme.Box([0], [149]), _mean_x0)
    printed = {0: 407.0, 2: 630.0, 3: -265.0}
    for k, v in printed.items():
        assert abs(d[k] - v) <= 0.005 * abs(v) + 0.5, (k, d[k], v)
    # the stationary mean the paper quotes the relative error against
    assert abs(E - 72.4495) < 1e-3


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_schloegl_against_closed_form(k):
    """All four derivatives on a box large enough that truncation is invisible."""
    _, d = cme.expectation_sensitivity(W.schlogl_paper(25.0), W.SCHLOGL_PAPER_C,
                                       cme.Box([0], [400]), _mean_x0)
    ref = X.schlogl_paper_sensitivity(k, N=400)
    assert abs(d[k] - ref) <= 1e-6 * abs(ref), (k, d[k], ref)


def test_pi_is_a_law_and_dpi_sums_to_zero():
    Xs, pi, dpi = cme.stationary_and_sensitivity(W.schlogl_paper(25.0), W.SCHLOGL_PAPER_C,
                                                 cme.Box([0], [149]))
    assert abs(pi.sum() - 1.0) < 1e-12
    assert pi.min() > -1e-15
    assert np.all(np.abs(dpi.sum(axis=1)) < 1e-9)
    assert Xs.shape == (150, 1)


# --- two-species closed forms ------------------------------------------------

def _poisson(k, n):
    return np.exp(-k + n * math.log(k) - np.array([math.lgamma(i + 1) for i in n]))


def _hill_rep_net(K):
    # params (k, a, h, g): 0 -> X0 at k, X0 -> 0 at x0, 0 -> X1 at a / (1 + (x0/K)^h), X1 -> 0 at g x1
    return W.Network(
        name="hill_rep_pair", n_species=2, n_params=4,
        reactions=(
            W.Reaction(0, 1.0, (), (1, 0)),
            W.Reaction(-1, 1.0, (W.Factor(W.FALLING, 0, order=1),), (-1, 0)),
            W.Reaction(1, 1.0, (W.Factor(W.HILL_REP, 0, K=K, hill_param=2),), (0, 1)),
            W.Reaction(3, 1.0, (W.Factor(W.FALLING, 1, order=1),), (0, -1)),
        ))


def _hill_rep_mean(c, K, nmax=80):
    k, a, h, g = c
    n = np.arange(nmax + 1, dtype=np.float64)
    phi = 1.0 / (1.0 + (n / K) ** h)
    return a / g * float(np.sum(_poisson(k, n) * phi))


def _hill_switch_net():
    # params (k, lo, hi, Kp, m, g): 0 -> X1 at m (lo + (hi - lo) q/(1+q)), q = (x0/Kp)^2
    sw = W.Factor(W.HILL_SWITCH, 0, order=2, hill_param=1, param2=2, param3=3)
    return W.Network(
        name="hill_switch_pair", n_species=2, n_params=6,
        reactions=(
            W.Reaction(0, 1.0, (), (1, 0)),
            W.Reaction(-1, 1.0, (W.Factor(W.FALLING, 0, order=1),), (-1, 0)),
            W.Reaction(-1, 1.0, (sw, W.Factor(W.PARAM, 0, hill_param=4)), (0, 1)),
            W.Reaction(5, 1.0, (W.Factor(W.FALLING, 1, order=1),), (0, -1)),
        ))


def _hill_switch_mean(c, nmax=80):
    k, lo, hi, Kp, m, g = c
    n = np.arange(nmax + 1, dtype=np.float64)
    q = (n / Kp) ** 2
    phi = lo + (hi - lo) * q / (1.0 + q)
    return m / g * float(np.sum(_poisson(k, n) * phi))


def _central(fun, c, k, h=1e-5):
    cp, cm = np.array(c, float), np.array(c, float)
    cp[k] *= 1 + h
    cm[k] *= 1 - h
    return (fun(cp) - fun(cm)) / (2 * h * c[k])


def test_hill_repression_factor():
    K = 3.0
    c = (4.0, 6.0, 2.0, 1.25)
    E, d = cme.expectation_sensitivity(_hill_rep_net(K), c, cme.Box([0, 0], [40, 45]), _mean_x1)
    fun = lambda cc: _hill_rep_mean(cc, K)
    assert abs(E - fun(c)) < 1e-9 * fun(c)
    for k in range(4):
        ref = _central(fun, c, k)
        assert abs(d[k] - ref) <= 1e-7 * max(1.0, abs(ref)), (k, d[k], ref)


def test_hill_switch_and_param_factors():
    c = (3.0, 1.0, 8.0, 2.5, 1.5, 2.0)
    E, d = cme.expectation_sensitivity(_hill_switch_net(), c, cme.Box([0, 0], [40, 45]), _mean_x1)
    assert abs(E - _hill_switch_mean(c)) < 1e-9 * E
    for k in range(6):
        ref = _central(_hill_switch_mean, c, k)
        assert abs(d[k] - ref) <= 1e-7 * max(1.0, abs(ref)), (k, d[k], ref)


def test_species_zero_marginal_is_poisson():
    """The x0 marginal of the pair networks is Poisson(k) and insensitive to the Hill parameters."""
    c = (4.0, 6.0, 2.0, 1.25)
    Xs, pi, dpi = cme.stationary_and_sensitivity(_hill_rep_net(3.0), c, cme.Box([0, 0], [40, 45]))
    marg = np.bincount(Xs[:, 0], weights=pi)
    n = np.arange(41, dtype=np.float64)
    assert np.max(np.abs(marg - _poisson(4.0, n))) < 1e-12
    for k in (1, 2, 3):
        assert np.max(np.abs(np.bincount(Xs[:, 0], weights=dpi[k]))) < 1e-10


# --- multi-species laws against the tests' own generator solves ---------------

def test_toggle_law_matches_generator_solve():
    omega, N = 4.0, 40
    c = (3.0, 3.0, 2.0, 2.0)
    _, pi_ref = X.toggle_pi(omega, N, c)
    _, pi, _ = cme.stationary_and_sensitivity(W.toggle(omega), c, cme.Box([0, 0], [N, N]))
    assert np.max(np.abs(pi.reshape(N + 1, N + 1) - pi_ref)) < 1e-12


def test_toggle_sensitivity_by_differences_of_generator_solve():
    omega, N = 4.0, 40
    c = (3.0, 3.0, 2.0, 2.0)
    _, d = cme.expectation_sensitivity(W.toggle(omega), c, cme.Box([0, 0], [N, N]), _mean_x0)
    U = np.arange(N + 1)[:, None] * np.ones((1, N + 1))

    def mean_u(cc):
        _, p = X.toggle_pi(omega, N, tuple(cc))
        return float(np.sum(p * U))

    for k in range(4):
        ref = _central(mean_u, c, k)
        assert abs(d[k] - ref) <= 1e-6 * max(1.0, abs(ref)), (k, d[k], ref)


def test_command_line(capsys):
    assert cme.main(["--model", "schlogl", "--box", "149"]) == 0
    out = capsys.readouterr().out.split("\n")
    assert out[0].startswith("E_pi[x0] = 72.44")
    assert "407.3" in out[1] and "630.2" in out[3] and "-264.6" in out[4]
