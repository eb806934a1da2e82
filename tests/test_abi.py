"""Host-side checks of the C ABI (CPU, no GPU calls): the library loads and
exports every function the headers in include/ declare; the binding's structs
have the header's layout; the input generators produce valid problems."""
import ctypes
import glob
import os
import re

import pytest

from paper_1705_06807_amd import binding as B
from paper_1705_06807_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "parrep.h")


def declared_functions():
    src = "".join(open(h).read() for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(parrep_[a-z_0-9]+)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def so():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libparrep.so is not built; run paper_1705_06807_amd/build.py")
    return ctypes.CDLL(B.LIB_PATH)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("parrep_ctx_create", "parrep_ctx_destroy", "parrep_last_error", "parrep_net_create",
              "parrep_net_destroy", "parrep_solve", "parrep_solve_batch", "parrep_philox",
              "parrep_events", "parrep_dephase_only", "parrep_parallel_only",
              "parrep_problem_nbins", "parrep_plan_create", "parrep_plan_update",
              "parrep_plan_launch", "parrep_plan_run", "parrep_plan_destroy", "parrep_autotune",
              "parrep_server_create", "parrep_server_submit", "parrep_server_poll",
              "parrep_server_cancel", "parrep_server_destroy", "parrep_estimate"):
        assert n in names


def test_library_exports_every_declared_function(so):
    missing = [n for n in declared_functions() if not hasattr(so, n)]
    assert not missing, missing


def test_struct_layouts_match_header():
    # sizes implied by the header's field lists on x86-64
    assert ctypes.sizeof(B.Factor) == 6 * 4 + 8
    assert ctypes.sizeof(B.Reaction) == 8 + 8 + 16 + 2 * 32
    assert ctypes.sizeof(B.Result) == 6 * 8 + 8 + 8
    assert ctypes.sizeof(B.Launch) == 56
    assert B.Launch.persistent.offset == 48
    assert ctypes.sizeof(B.Request) == 8 + 4 + 4 + 8
    assert ctypes.sizeof(B.RequestInfo) == 4 + 4 + 8 + 8 + 8 + 4 * 8
    assert B.Problem.max_events.offset + 8 == ctypes.sizeof(B.Problem)


def test_header_constants_match_binding():
    src = open(HEADER).read()

    def const(name):
        return int(re.search(r"#define %s (\d+)" % name, src).group(1))

    assert const("PARREP_MAX_SPECIES") == B.MAX_S
    assert const("PARREP_MAX_REACTIONS") == B.MAX_M
    assert const("PARREP_MAX_FACTORS") == B.MAX_F
    assert const("PARREP_MAX_PARAMS") == B.MAX_P
    assert const("PARREP_NCOUNTERS") == B.NCOUNTERS
    assert const("PARREP_NSTATS") == B.NSTATS
    assert const("PARREP_MAX_REPLICAS") == B.MAX_REPLICAS
    for name, v in (("PARREP_ST_FIM", B.ST_FIM), ("PARREP_ST_RER", B.ST_RER),
                    ("PARREP_ST_Y", B.ST_Y)):
        assert int(re.search(r"%s = (\d+)" % name, src).group(1)) == v
    est = open(os.path.join(ROOT, "include", "parrep_estimate.h")).read()
    for name, v in (("PARREP_EST_FIM", B.EST_FIM), ("PARREP_EST_FIM_HW", B.EST_FIM_HW),
                    ("PARREP_EST_RER", B.EST_RER), ("PARREP_EST_Y", B.EST_Y),
                    ("PARREP_EST_IAF", B.EST_IAF), ("PARREP_EST_BOUND", B.EST_BOUND),
                    ("PARREP_EST_LEN", B.EST_LEN)):
        assert int(re.search(r"%s = (\d+)" % name, est).group(1)) == v


def test_validation_without_a_device(so):
    # network validation is host-only; a bad factor is rejected before any HIP call
    L = B.lib()
    ctx_like = ctypes.c_void_p(1)  # never dereferenced on the failing paths below
    rx = (B.Reaction * B.MAX_M)()
    rx[0].n_factors = 1
    rx[0].factor[0].kind = 7
    out = ctypes.c_void_p()
    rc = L.parrep_net_create(ctx_like, 1, 1, 1, rx, ctypes.byref(out))
    assert rc == -1 and b"bad factor" in L.parrep_last_error()
    rc = L.parrep_net_create(ctx_like, 5, 1, 1, rx, ctypes.byref(out))
    assert rc == -1


def test_problem_validation_and_nbins(so):
    L = B.lib()
    ctx_like = ctypes.c_void_p(1)
    out = ctypes.c_void_p()
    net = W.toggle(50.0)
    rx = (B.Reaction * B.MAX_M)()
    for j, r in enumerate(net.reactions):
        rx[j].rate_param, rx[j].kappa, rx[j].n_factors = r.rate_param, r.kappa, len(r.factors)
        for i, v in enumerate(r.stoich):
            rx[j].stoich[i] = v
        for k, f in enumerate(r.factors):
            rx[j].factor[k].kind, rx[j].factor[k].species = f.kind, f.species
            rx[j].factor[k].order, rx[j].factor[k].hill_param = f.order, f.hill_param
            rx[j].factor[k].K = f.K
    assert L.parrep_net_create(ctx_like, 2, 4, 4, rx, ctypes.byref(out)) == 0
    p = W.c2_toggle()
    ps = B.problem_struct(p)
    assert L.parrep_problem_nbins(out, ctypes.byref(ps)) == 401 * 401
    for bad in (dict(R=0), dict(R=B.MAX_REPLICAS + 1), dict(T=0.0), dict(t_burn=p.T),
                dict(hist_hi=(-1, 400)), dict(c=(3.0, -1.0, 2.0, 2.0))):
        ps = B.problem_struct(p.replace(**bad))
        assert L.parrep_problem_nbins(out, ctypes.byref(ps)) == -1, bad
    L.parrep_net_destroy(out)


def test_workload_generators_are_valid():
    batch = W.c3_batch(seed=0)
    assert len(batch) == 256
    assert all(64 <= p.R <= 4096 for p in batch)
    assert len({p.instance_id for p in batch}) == 256
    om = [p.net.reactions[0].kappa for p in batch if p.net.name == "toggle"]
    assert min(om) >= 25 and max(om) <= 100
    arrivals, reqs = W.c5_requests(seed=1, n=40)
    assert len(reqs) == 40 and all(256 <= p.R <= 16384 for p in reqs)
    assert all(b >= a for a, b in zip(arrivals[:-1], arrivals[1:]))


def test_counter_names_line_up_with_the_oracle(oracle):
    # the two sides name the same counters in the same order, except the last
    # slot: the library's spill-overflow count, the oracle's reserved word
    from oracle import oracle as O
    assert B.COUNTER_NAMES[:-1] == O.COUNTER_NAMES[:-1]
    assert B.COUNTER_NAMES[-1] == "spill_overflow" and O.COUNTER_NAMES[-1] == "reserved"
