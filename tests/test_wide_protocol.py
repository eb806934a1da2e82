"""The multi-workgroup protocol of one ParRep instance (a host model, see
wide_protocol.py) reproduces the oracle's serial Alg. 1 (Sec. II A) for
several group counts and chunk lengths: integers exactly (counters, cycle
records, final state), times up to summation order."""
import numpy as np
import pytest

from paper_1705_06807_amd import workloads as W
from wide_protocol import Model


def _check(oracle, p, G, S2, S3):
    o = oracle.run(p, cycle_log_cap=4096)
    m = Model(oracle, p, G=G, S2=S2, S3=S3).run()
    oc = dict(o.counters)
    oc.pop("reserved")
    assert m.counters == oc, (m.counters, oc)
    log = np.array([list(r) + [0] * (12 - len(r)) for r in m.cycle_log], dtype=np.int64)
    log[:, 6 + p.net.n_species:] = 0
    assert np.array_equal(log, o.cycle_log)
    assert tuple(m.x_final) == tuple(o.x_final)
    assert m.T_s == o.T_s
    scale = np.abs(o.hist).max()
    assert np.abs(m.hist - o.hist).max() <= 1e-12 * scale
    assert np.abs(m.hist_w - o.hist_w).max() <= 1e-12 * max(np.abs(o.hist_w).max(), 1e-300)
    assert m.outside == pytest.approx(o.outside, rel=1e-12, abs=1e-300)
    return m, o


CASES = [
    # toggle at Omega = 5: many exits, Fleming-Viot restarts, both boundaries
    ("om5_time", lambda i: W.c2_toggle(seed=31, instance_id=i, omega=5.0, R=24, T=40.0,
                                       t_cp=1.0).replace(hist_hi=(40, 40))),
    ("om5_steps", lambda i: W.c2_toggle(seed=32, instance_id=i, omega=5.0, R=20, T=40.0,
                                        t_cp=1.0).replace(
        hist_hi=(40, 40), decorr_mode=W.STEPS, decorr=20, dephase_mode=W.STEPS, dephase=15)),
    ("om2_many_exits", lambda i: W.c2_toggle(seed=33, instance_id=i, omega=2.0, R=16, T=30.0,
                                             t_cp=0.5).replace(hist_hi=(20, 20))),
    # the event budget runs out in the dephasing step (i = 0), the parallel step (i = 1)
    ("schlogl_budget", lambda i: W.c1_schlogl(seed=34, instance_id=i, R=12, T=50.0).replace(
        max_events=(5000, 9500)[i])),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("G,S2,S3", [(1, 5, 3), (3, 4, 2), (4, 1, 1), (5, 16, 7)])
def test_wide_protocol_matches_oracle(oracle, case, G, S2, S3):
    name, make = case
    for i in range(2):
        _check(oracle, make(i), G, S2, S3)
