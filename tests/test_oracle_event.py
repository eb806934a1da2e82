"""Unit pins of the oracle's SSA event (CPU): propensities at edge states,
selection rule, waiting time and the absorbing state (Sec. I A, Alg. 1)."""
import math

import numpy as np
import pytest

import exact_laws as E
from paper_1705_06807_amd import workloads as W


def _block_for(us_target):
    """A Philox-shaped block whose u_sel is exactly us_target (a multiple of 2^-53)
    and whose u_open is 1/2."""
    w23 = int(round(us_target * 2 ** 53)) << 11
    w01 = ((2 ** 52) - 1) << 11  # (w01>>11)+1 = 2^52 -> u_open = 0.5
    return [w01 & 0xFFFFFFFF, w01 >> 32, w23 & 0xFFFFFFFF, w23 >> 32]


@pytest.mark.parametrize("x", [0, 1, 2, 3, 85, 250, 1000])
def test_schlogl_classic_propensities(oracle, x):
    net = W.schlogl_classic()
    lam, a0, tau, J, absorbing = oracle.event(net, W.SCHLOGL_CLASSIC_C, [x], _block_for(0.0))
    ref = E.schlogl_classic_rates([x])[:, 0]
    np.testing.assert_allclose(lam, ref, rtol=1e-15, atol=0)
    assert a0 == pytest.approx(ref.sum(), rel=1e-15)
    assert not absorbing


def test_schlogl_edge_values(oracle):
    net = W.schlogl_classic()
    c = W.SCHLOGL_CLASSIC_C
    lam, *_ = oracle.event(net, c, [0], _block_for(0.0))
    assert list(lam) == [0.0, 0.0, c[2] * 2e5, 0.0]
    lam, *_ = oracle.event(net, c, [2], _block_for(0.0))
    assert lam[0] == c[0] * 5e4 * 2.0 and lam[1] == 0.0 and lam[3] == c[3] * 2
    lam, *_ = oracle.event(net, c, [3], _block_for(0.0))
    assert lam[1] == c[1] * (1.0 / 6.0) * 6.0


@pytest.mark.parametrize("u,v", [(0, 0), (0, 7), (7, 0), (50, 50), (131, 19), (400, 3)])
def test_toggle_propensities(oracle, u, v):
    net = W.toggle(50.0)
    lam, a0, *_ = oracle.event(net, W.TOGGLE_C, [u, v], _block_for(0.0))
    ref = E.toggle_rates([u], [v], 50.0)[:, 0]
    np.testing.assert_allclose(lam, ref, rtol=2e-15, atol=0)


def test_toggle_zero_repressor_gives_full_rate(oracle):
    lam, *_ = oracle.event(W.toggle(50.0), W.TOGGLE_C, [0, 0], _block_for(0.0))
    assert lam[0] == 150.0 and lam[2] == 150.0 and lam[1] == 0.0 and lam[3] == 0.0


def test_selection_rule_and_zero_channels(oracle):
    # x = 0 in Schloegl: only channel 3 (B -> X) is positive; every u_sel picks it
    net = W.schlogl_classic()
    for us in (0.0, 0.25, 0.5, 1.0 - 2.0 ** -53):
        _, _, _, J, _ = oracle.event(net, W.SCHLOGL_CLASSIC_C, [0], _block_for(us))
        assert J == 2
    # at x = 85 the picks follow the cumulative sums: J = first j with u*a0 < S_j
    lam, a0, *_ = oracle.event(net, W.SCHLOGL_CLASSIC_C, [85], _block_for(0.0))
    S = np.cumsum(lam)
    for us in np.linspace(0, 1 - 2 ** -20, 97):
        us = math.floor(us * 2 ** 53) / 2 ** 53
        _, _, _, J, _ = oracle.event(net, W.SCHLOGL_CLASSIC_C, [85], _block_for(us))
        t = us * a0
        assert J == int(np.argmax(t < S))


def test_waiting_time(oracle):
    net = W.schlogl_classic()
    lam, a0, tau, J, _ = oracle.event(net, W.SCHLOGL_CLASSIC_C, [85], _block_for(0.0))
    assert tau == pytest.approx(math.log(2.0) / a0, rel=1e-15)
    # u_open = 1 gives a zero holding time
    _, _, tau1, _, _ = oracle.event(net, W.SCHLOGL_CLASSIC_C, [85], [0xFFFFFFFF] * 2 + [0, 0])
    assert tau1 == 0.0


def test_absorbing_state(oracle):
    lam, a0, tau, J, absorbing = oracle.event(W.pure_death(), [1.0], [0], _block_for(0.3))
    assert absorbing and a0 == 0.0 and math.isinf(tau) and J == -1


def test_exponential_holding_times(oracle):
    # tau = -log(u)/a0 with Philox uniforms is Exp(a0): mean and KS distance
    net = W.toggle(5.0)
    taus = []
    for i in range(20000):
        blk = oracle.philox([i, 0, 0, 1 << 28], [1, 2])
        _, a0, tau, _, _ = oracle.event(net, W.TOGGLE_C, [3, 4], blk)
        taus.append(tau * a0)
    taus = np.sort(taus)
    assert abs(taus.mean() - 1.0) < 4 * 1 / math.sqrt(len(taus))
    cdf = 1 - np.exp(-taus)
    ks = np.max(np.abs(cdf - (np.arange(1, len(taus) + 1) / len(taus))))
    assert ks < 1.63 / math.sqrt(len(taus))  # p ~ 0.01
