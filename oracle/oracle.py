"""ctypes front end of the CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module.  It marshals :mod:`paper_1705_06807_amd.workloads` inputs into the
oracle's own C structs (``parrep_oracle.h``) and shares nothing with the GPU
library's binding.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from . import build as _build

MAX_S, MAX_R, MAX_F, MAX_P = 4, 8, 2, 8
NCOUNTERS = 12
CYCLE_REC = 12

COUNTER_NAMES = ("ev_decorr", "ev_dephase", "ev_par_credited", "ev_par_discarded", "cycles",
                 "s3_rounds", "s2_rounds", "status", "fv_restarts", "end_phase", "n_cycle_log",
                 "reserved")


class Factor(C.Structure):
    _fields_ = [("kind", C.c_int32), ("species", C.c_int32), ("order", C.c_int32),
                ("hill_param", C.c_int32), ("param2", C.c_int32), ("param3", C.c_int32),
                ("K", C.c_double)]


class Reaction(C.Structure):
    _fields_ = [("rate_param", C.c_int32), ("n_factors", C.c_int32), ("kappa", C.c_double),
                ("stoich", C.c_int32 * MAX_S), ("f", Factor * MAX_F)]


class Net(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_reactions", C.c_int32), ("n_params", C.c_int32),
                ("reserved", C.c_int32), ("rx", Reaction * MAX_R)]


class ProblemS(C.Structure):
    _fields_ = [("c", C.c_double * MAX_P), ("rer_eps", C.c_double * MAX_P),
                ("use_rer", C.c_int32), ("x0", C.c_int32 * MAX_S),
                ("region_w", C.c_int32 * MAX_S), ("region_theta", C.c_int64), ("R", C.c_int32),
                ("decorr_mode", C.c_int32), ("decorr", C.c_double), ("dephase_mode", C.c_int32),
                ("dephase", C.c_double), ("T", C.c_double), ("t_burn", C.c_double),
                ("hist_lo", C.c_int32 * MAX_S), ("hist_hi", C.c_int32 * MAX_S),
                ("seed", C.c_uint32), ("instance_id", C.c_uint32), ("max_events", C.c_int64)]


class ResultS(C.Structure):
    _fields_ = [("hist", C.POINTER(C.c_double)), ("hist_w", C.POINTER(C.c_double)),
                ("outside", C.c_double), ("outside_w", C.c_double), ("T_s", C.c_double),
                ("fim", C.c_double * (MAX_P * MAX_P)), ("rer", C.c_double * MAX_P),
                ("y", C.c_double * MAX_S), ("x_final", C.c_int32 * MAX_S),
                ("counters", C.c_int64 * NCOUNTERS), ("cycle_log", C.POINTER(C.c_int64)),
                ("cycle_log_cap", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build(force=True)
        L = C.CDLL(path)
        L.or_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        L.or_uniforms.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_double)]
        L.or_event.argtypes = [C.POINTER(Net), C.POINTER(C.c_double), C.POINTER(C.c_int32),
                               C.POINTER(C.c_uint32), C.POINTER(C.c_double),
                               C.POINTER(C.c_double), C.POINTER(C.c_double),
                               C.POINTER(C.c_int32)]
        L.or_event.restype = C.c_int
        L.or_fim_rer.argtypes = [C.POINTER(Net), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                 C.POINTER(C.c_double)]
        dp = C.POINTER(C.c_double)
        L.or_estimate.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, dp, C.c_double, dp, dp, dp,
                                  dp, dp, dp]
        L.or_estimate.restype = None
        L.or_run.argtypes = [C.POINTER(Net), C.POINTER(ProblemS), C.POINTER(ResultS)]
        L.or_run.restype = C.c_int
        L.or_dephase.argtypes = [C.POINTER(Net), C.POINTER(ProblemS), C.POINTER(C.c_int32),
                                 C.c_uint32, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.or_dephase.restype = C.c_int
        L.or_parallel.argtypes = [C.POINTER(Net), C.POINTER(ProblemS), C.POINTER(C.c_int32),
                                  C.c_uint32, C.c_int64, C.POINTER(C.c_int64),
                                  C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.or_parallel.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def make_net(net) -> Net:
    s = Net()
    s.n_species = net.n_species
    s.n_reactions = net.n_reactions
    s.n_params = net.n_params
    for j, r in enumerate(net.reactions):
        rx = s.rx[j]
        rx.rate_param = r.rate_param
        rx.kappa = r.kappa
        rx.n_factors = len(r.factors)
        for i, v in enumerate(r.stoich):
            rx.stoich[i] = v
        for k, f in enumerate(r.factors):
            rx.f[k].kind = f.kind
            rx.f[k].species = f.species
            rx.f[k].order = f.order
            rx.f[k].hill_param = f.hill_param
            rx.f[k].param2 = f.param2
            rx.f[k].param3 = f.param3
            rx.f[k].K = f.K
    return s


def make_problem(p) -> ProblemS:
    s = ProblemS()
    for i, v in enumerate(p.c):
        s.c[i] = v
    if p.rer_eps is not None:
        s.use_rer = 1
        for i, v in enumerate(p.rer_eps):
            s.rer_eps[i] = v
    for i, v in enumerate(p.x0):
        s.x0[i] = v
    for i, v in enumerate(p.region_w):
        s.region_w[i] = v
    s.region_theta = p.region_theta
    s.R = p.R
    s.decorr_mode, s.decorr = p.decorr_mode, p.decorr
    s.dephase_mode, s.dephase = p.dephase_mode, p.dephase
    s.T, s.t_burn = p.T, p.t_burn
    for i, (lo, hi) in enumerate(zip(p.hist_lo, p.hist_hi)):
        s.hist_lo[i], s.hist_hi[i] = lo, hi
    s.seed, s.instance_id = p.seed, p.instance_id
    s.max_events = p.max_events
    return s


def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def uniforms(blk):
    b = np.asarray(blk, dtype=np.uint32)
    out = np.zeros(2)
    lib().or_uniforms(_ptr(b, C.c_uint32), _ptr(out, C.c_double))
    return float(out[0]), float(out[1])


def event(net, c, x, blk):
    """One SSA event: returns (lam[m], a0, tau, J, absorbing)."""
    n = make_net(net)
    cc = np.zeros(MAX_P)
    cc[:len(c)] = c
    xx = np.zeros(MAX_S, dtype=np.int32)
    xx[:len(x)] = x
    b = np.asarray(blk, dtype=np.uint32)
    lam = np.zeros(MAX_R)
    a0 = C.c_double()
    tau = C.c_double()
    J = C.c_int32()
    rc = lib().or_event(C.byref(n), _ptr(cc, C.c_double), _ptr(xx, C.c_int32),
                        _ptr(b, C.c_uint32), _ptr(lam, C.c_double), C.byref(a0), C.byref(tau),
                        C.byref(J))
    return lam[:net.n_reactions].copy(), a0.value, tau.value, J.value, bool(rc)


def fim_rer(net, c, x, rer_eps=None):
    n = make_net(net)
    np_ = net.n_params
    cc = np.zeros(MAX_P)
    cc[:len(c)] = c
    ee = np.zeros(MAX_P)
    if rer_eps is not None:
        ee[:len(rer_eps)] = rer_eps
    xx = np.zeros(MAX_S, dtype=np.int32)
    xx[:len(x)] = x
    fim = np.zeros(MAX_P * MAX_P)
    rer = np.zeros(MAX_P)
    lib().or_fim_rer(C.byref(n), _ptr(cc, C.c_double), _ptr(ee, C.c_double),
                     1 if rer_eps is not None else 0, _ptr(xx, C.c_int32),
                     _ptr(fim, C.c_double), _ptr(rer, C.c_double))
    return fim[:np_ * np_].reshape(np_, np_).copy(), rer[:np_].copy()


def estimate(fim, rer, y, window):
    """Multi-run estimators (Sec. III) of n runs: fim (n, p, p), rer (n, p),
    y (n, s) window integrals.  Returns a dict of fim_mean (p, p), fim_hw (p),
    rer_mean (p), y_mean (s), iaf (s), bound (s, p)."""
    fim = np.ascontiguousarray(fim, dtype=np.float64)
    rer = np.ascontiguousarray(rer, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    n, p = rer.shape
    s = y.shape[1]
    assert fim.shape == (n, p, p) and y.shape[0] == n and n >= 2
    out = dict(fim_mean=np.zeros((p, p)), fim_hw=np.zeros(p), rer_mean=np.zeros(p),
               y_mean=np.zeros(s), iaf=np.zeros(s), bound=np.zeros((s, p)))
    d = C.c_double
    lib().or_estimate(n, p, s, _ptr(fim, d), _ptr(rer, d), _ptr(y, d), float(window),
                      _ptr(out["fim_mean"], d), _ptr(out["fim_hw"], d), _ptr(out["rer_mean"], d),
                      _ptr(out["y_mean"], d), _ptr(out["iaf"], d), _ptr(out["bound"], d))
    return out


class OracleResult:
    def __init__(self, p, hist, hist_w, r: ResultS, cycle_log):
        npar = p.net.n_params
        ns = p.net.n_species
        shape = tuple(hi - lo + 1 for lo, hi in zip(p.hist_lo, p.hist_hi))
        self.hist = hist.reshape(shape)
        self.hist_w = hist_w.reshape(shape)
        self.outside = r.outside
        self.outside_w = r.outside_w
        self.T_s = r.T_s
        self.fim = np.array(r.fim[:npar * npar]).reshape(npar, npar)
        self.rer = np.array(r.rer[:npar])
        self.y = np.array(r.y[:ns])
        self.x_final = np.array(r.x_final[:ns], dtype=np.int32)
        self.counters = {k: int(v) for k, v in zip(COUNTER_NAMES, r.counters)}
        n = min(self.counters["n_cycle_log"], cycle_log.shape[0]) if cycle_log is not None else 0
        self.cycle_log = cycle_log[:n].copy() if cycle_log is not None else None

    @property
    def events(self) -> int:
        c = self.counters
        return c["ev_decorr"] + c["ev_dephase"] + c["ev_par_credited"] + c["ev_par_discarded"]


def run(p, cycle_log_cap: int = 256) -> OracleResult:
    """Full ParRep run of problem p (Alg. 1 until the clock reaches T)."""
    n = make_net(p.net)
    ps = make_problem(p)
    nb = p.nbins()
    hist = np.zeros(nb)
    hist_w = np.zeros(nb)
    log = np.zeros((max(cycle_log_cap, 1), CYCLE_REC), dtype=np.int64)
    r = ResultS()
    r.hist = _ptr(hist, C.c_double)
    r.hist_w = _ptr(hist_w, C.c_double)
    r.cycle_log = _ptr(log, C.c_int64)
    r.cycle_log_cap = cycle_log_cap
    rc = lib().or_run(C.byref(n), C.byref(ps), C.byref(r))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return OracleResult(p, hist, hist_w, r, log)


def dephase(p, xt, cycle: int = 0):
    """Dephasing step alone from xt; returns (replica states R x n, rounds)."""
    n = make_net(p.net)
    ps = make_problem(p)
    xx = np.zeros(MAX_S, dtype=np.int32)
    xx[:len(xt)] = xt
    Y = np.zeros((p.R, p.net.n_species), dtype=np.int32)
    rounds = C.c_int64()
    rc = lib().or_dephase(C.byref(n), C.byref(ps), _ptr(xx, C.c_int32), cycle,
                          _ptr(Y, C.c_int32), C.byref(rounds))
    if rc != 0:
        raise ValueError("oracle dephase failed")
    return Y, rounds.value


def parallel(p, init: np.ndarray, cycle: int = 0, max_rounds: int = -1):
    """Parallel step alone from replica states init (R x n) with no horizon.
    Returns (N*, K, exit_state, credited_time); N* = -1 if max_rounds ran out."""
    n = make_net(p.net)
    ps = make_problem(p)
    init = np.ascontiguousarray(init, dtype=np.int32)
    assert init.shape == (p.R, p.net.n_species)
    nk = np.zeros(2, dtype=np.int64)
    xs = np.zeros(MAX_S, dtype=np.int32)
    cred = C.c_double()
    rc = lib().or_parallel(C.byref(n), C.byref(ps), _ptr(init, C.c_int32), cycle, max_rounds,
                           _ptr(nk, C.c_int64), _ptr(xs, C.c_int32), C.byref(cred))
    if rc != 0:
        return -1, 0, None, cred.value
    return int(nk[0]), int(nk[1]), xs[:p.net.n_species].copy(), cred.value
