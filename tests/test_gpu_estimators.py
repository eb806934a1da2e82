"""The multi-run estimators of Sec. III on the device (parrep_estimate)
against the oracle's or_estimate on host copies of the same runs' outputs:
means, FIM half-widths, IAFs and bounds agree to 2 ulp (both sides sum in run
order with the same operations; the device's square root and division are
correctly rounded as the host's are, so most entries agree bit for bit)."""
import math

import numpy as np
import pytest

from paper_1705_06807_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_06807_amd import binding
    binding.lib()
    return binding


CASES = [
    ("paper_schlogl", lambda i: W.paper_schlogl_problem(seed=5, instance_id=i, T=2e4), 16),
    ("toggle", lambda i: W.c2_toggle(seed=6, instance_id=i, omega=5.0, R=64, T=400.0, t_cp=1.0)
     .replace(hist_hi=(40, 40)), 9),
    ("genetic_switch", lambda i: W.genetic_switch_problem(seed=7, instance_id=i, V=240.0, R=8,
                                                          n_c=500, n_p=500, T=2000.0)
     .replace(hist_hi=(1, 1, 8, 700)), 5),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_estimate_matches_oracle(B, oracle, case):
    import torch
    name, make, n = case
    probs = [make(i) for i in range(n)]
    outs = B.parrep_solve_batch(probs, cycle_log_cap=0)
    est = B.parrep_estimate(outs)
    torch.cuda.synchronize()
    hs = [o.to_host() for o in outs]
    p = probs[0]
    g = B.split_estimates(est, p.net.n_params, p.net.n_species)
    o = oracle.estimate(np.array([h.fim for h in hs]), np.array([h.rer for h in hs]),
                        np.array([h.y for h in hs]), window=p.T - p.t_burn)
    for key in ("fim_mean", "fim_hw", "rer_mean", "y_mean", "iaf", "bound"):
        np.testing.assert_allclose(g[key], o[key], rtol=4.5e-16, atol=0, err_msg=key)
    assert np.all(g["bound"] > 0) or name == "genetic_switch"
    rest = est.cpu().numpy()
    np_, ns = p.net.n_params, p.net.n_species
    assert np.all(rest[B.EST_FIM + np_ * np_:B.EST_FIM_HW] == 0.0)
    assert np.all(rest[B.EST_BOUND + ns * np_:] == 0.0)


EINVAL = -1


def _code(e):
    return int(str(e.value).split("error ")[1].split(":")[0])


def test_estimate_rejects_bad_arguments(B):
    import torch
    probs = [W.paper_schlogl_problem(seed=5, instance_id=i, T=200.0) for i in range(2)]
    outs = B.parrep_solve_batch(probs, cycle_log_cap=0)
    torch.cuda.synchronize()
    with pytest.raises(B.ParrepError) as e:
        B.parrep_estimate(outs[:1])
    assert _code(e) == EINVAL
    bad = probs[0].replace(t_burn=probs[0].T)  # zero window
    outs[0].problem = bad
    with pytest.raises(B.ParrepError) as e:
        B.parrep_estimate(outs)
    assert _code(e) == EINVAL
