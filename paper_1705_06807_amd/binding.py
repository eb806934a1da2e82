"""ctypes binding of libparrep (include/parrep.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels.  PyTorch is used
for device memory and streams: outputs are torch tensors on the context's
device, and calls are enqueued on torch's current stream.  If the library has
not been built, the first call raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from typing import List, Optional, Sequence

import numpy as np

from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libparrep.so")

MAX_S, MAX_M, MAX_F, MAX_P = 4, 8, 2, 8
MAX_REPLICAS = 65536
NCOUNTERS = 12
CYCLE_REC = 12
NSTATS = 80
ST_T, ST_OUTSIDE, ST_OUTSIDE_W, ST_FIM, ST_RER, ST_Y = 0, 1, 2, 3, 67, 75
COUNTER_NAMES = ("ev_decorr", "ev_dephase", "ev_par_credited", "ev_par_discarded", "cycles",
                 "s3_rounds", "s2_rounds", "status", "fv_restarts", "end_phase", "n_cycle_log",
                 "spill_overflow")


class ParrepError(RuntimeError):
    pass


class Factor(C.Structure):
    _fields_ = [("kind", C.c_int32), ("species", C.c_int32), ("order", C.c_int32),
                ("hill_param", C.c_int32), ("param2", C.c_int32), ("param3", C.c_int32),
                ("K", C.c_double)]


class Reaction(C.Structure):
    _fields_ = [("rate_param", C.c_int32), ("n_factors", C.c_int32), ("kappa", C.c_double),
                ("stoich", C.c_int32 * MAX_S), ("factor", Factor * MAX_F)]


class Problem(C.Structure):
    _fields_ = [("c", C.c_double * MAX_P), ("rer_eps", C.c_double * MAX_P),
                ("use_rer", C.c_int32), ("x0", C.c_int32 * MAX_S),
                ("region_w", C.c_int32 * MAX_S), ("region_theta", C.c_int64), ("R", C.c_int32),
                ("decorr_mode", C.c_int32), ("decorr", C.c_double),
                ("dephase_mode", C.c_int32), ("dephase", C.c_double), ("T", C.c_double),
                ("t_burn", C.c_double), ("hist_lo", C.c_int32 * MAX_S),
                ("hist_hi", C.c_int32 * MAX_S), ("seed", C.c_uint32),
                ("instance_id", C.c_uint32), ("max_events", C.c_int64)]


class Result(C.Structure):
    _fields_ = [("hist", C.c_void_p), ("hist_window", C.c_void_p), ("stats", C.c_void_p),
                ("x_final", C.c_void_p), ("counters", C.c_void_p), ("cycle_log", C.c_void_p),
                ("cycle_log_cap", C.c_int32), ("reserved", C.c_int32),
                ("phase_clock", C.c_void_p)]


class Launch(C.Structure):
    _fields_ = [("replicas_per_lane", C.c_int32), ("waves", C.c_int32),
                ("event_before", C.c_void_p), ("event_after", C.c_void_p),
                ("workgroups", C.c_int32), ("chunk_rounds", C.c_int32 * 2),
                ("barrier_wait_us", C.c_int32), ("histogram_staging", C.c_int32),
                ("flush_period", C.c_int32), ("persistent", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("rse_target", C.c_double), ("min_runs", C.c_int32), ("max_runs", C.c_int32),
                ("event_budget", C.c_int64)]


class RequestInfo(C.Structure):
    _fields_ = [("runs", C.c_int32), ("status", C.c_int32), ("rse", C.c_double),
                ("events", C.c_int64), ("latency_s", C.c_double), ("iaf", C.c_double * MAX_S)]


_lib = None
_lib_lock = threading.Lock()


def lib():
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ParrepError(
                    "libparrep.so is not built (%s); run paper_1705_06807_amd/build.py" % LIB_PATH)
            L = C.CDLL(LIB_PATH)
            vp = C.c_void_p
            L.parrep_last_error.restype = C.c_char_p
            L.parrep_wall_clock_hz.argtypes = [vp]
            L.parrep_wall_clock_hz.restype = C.c_double
            L.parrep_ctx_create.argtypes = [C.c_int, C.POINTER(vp)]
            L.parrep_ctx_destroy.argtypes = [vp]
            L.parrep_net_create.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32,
                                            C.POINTER(Reaction), C.POINTER(vp)]
            L.parrep_net_destroy.argtypes = [vp]
            L.parrep_problem_nbins.argtypes = [vp, C.POINTER(Problem)]
            L.parrep_problem_nbins.restype = C.c_int64
            L.parrep_solve.argtypes = [vp, vp, C.POINTER(Problem), C.POINTER(Result), vp]
            L.parrep_solve_noalloc.argtypes = [vp, vp, C.POINTER(Problem), C.POINTER(Result), vp]
            L.parrep_solve_batch.argtypes = [vp, C.c_int32, C.POINTER(vp), C.POINTER(Problem),
                                             C.POINTER(Result), C.POINTER(Launch), vp]
            L.parrep_philox.argtypes = [vp, C.c_int64, vp, vp, vp]
            L.parrep_estimate.argtypes = [vp, C.c_int32, C.POINTER(vp), C.c_int32, C.c_int32,
                                          C.c_double, vp, vp]
            L.parrep_events.argtypes = [vp, vp, C.POINTER(C.c_double), C.c_int64, vp, vp, vp, vp,
                                        vp, vp]
            L.parrep_dephase_only.argtypes = [vp, vp, C.POINTER(Problem), C.POINTER(C.c_int32),
                                              C.c_uint32, vp, vp, vp]
            L.parrep_parallel_only.argtypes = [vp, vp, C.POINTER(Problem), vp, C.c_uint32,
                                               C.c_int64, vp, vp, vp, vp]
            L.parrep_plan_create.argtypes = [vp, C.c_int32, C.POINTER(vp), C.POINTER(Problem),
                                             C.POINTER(Result), C.POINTER(Launch),
                                             C.POINTER(vp)]
            L.parrep_plan_update.argtypes = [vp, C.c_int32, C.POINTER(Problem), vp]
            L.parrep_plan_run.argtypes = [vp, vp, vp, vp]
            L.parrep_plan_launch.argtypes = [vp, vp]
            L.parrep_plan_destroy.argtypes = [vp]
            L.parrep_autotune.argtypes = [vp, vp, C.POINTER(Problem), C.c_int32, C.c_int64,
                                          C.POINTER(Result), C.POINTER(Launch)]
            L.parrep_server_create.argtypes = [vp, C.c_size_t, C.c_int32, C.POINTER(vp)]
            L.parrep_server_submit.argtypes = [vp, vp, C.POINTER(Problem), C.POINTER(Request),
                                               C.POINTER(C.c_uint64)]
            L.parrep_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(Result),
                                             C.POINTER(RequestInfo), C.c_int32]
            L.parrep_server_cancel.argtypes = [vp, C.c_uint64]
            L.parrep_server_destroy.argtypes = [vp]
            _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise ParrepError("libparrep error %d: %s" % (rc, lib().parrep_last_error().decode()))


def _torch():
    import torch
    return torch


def _stream_ptr(stream) -> Optional[int]:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Context:
    """A device context; owns the networks it creates."""

    def __init__(self, device: int = 0):
        self.device = device
        h = C.c_void_p()
        _check(lib().parrep_ctx_create(device, C.byref(h)))
        self.h = h
        self._nets = {}

    def __del__(self):
        try:
            for n in self._nets.values():
                lib().parrep_net_destroy(n)
            if getattr(self, "h", None):
                lib().parrep_ctx_destroy(self.h)
        except Exception:
            pass

    @property
    def torch_device(self):
        return _torch().device("cuda", self.device)

    def net(self, net: W.Network) -> C.c_void_p:
        h = self._nets.get(net)
        if h is not None:
            return h
        rx = (Reaction * MAX_M)()
        for j, r in enumerate(net.reactions):
            rx[j].rate_param = r.rate_param
            rx[j].kappa = r.kappa
            rx[j].n_factors = len(r.factors)
            for i, v in enumerate(r.stoich):
                rx[j].stoich[i] = v
            for k, f in enumerate(r.factors):
                rx[j].factor[k].kind = f.kind
                rx[j].factor[k].species = f.species
                rx[j].factor[k].order = f.order
                rx[j].factor[k].hill_param = f.hill_param
                rx[j].factor[k].param2 = f.param2
                rx[j].factor[k].param3 = f.param3
                rx[j].factor[k].K = f.K
        h = C.c_void_p()
        _check(lib().parrep_net_create(self.h, net.n_species, net.n_reactions, net.n_params, rx,
                                       C.byref(h)))
        self._nets[net] = h
        return h


def problem_struct(p: W.Problem) -> Problem:
    s = Problem()
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


class Outputs:
    """Device output buffers of one solve (torch tensors)."""

    def __init__(self, ctx: Context, p: W.Problem, cycle_log_cap: int = 256,
                 phase_clock: bool = False):
        torch = _torch()
        dev = ctx.torch_device
        self.problem = p
        nb = p.nbins()
        self.hist = torch.empty(nb, dtype=torch.float64, device=dev)
        self.hist_window = torch.empty(nb, dtype=torch.float64, device=dev)
        self.stats = torch.empty(NSTATS, dtype=torch.float64, device=dev)
        self.x_final = torch.empty(MAX_S, dtype=torch.int32, device=dev)
        self.counters = torch.empty(NCOUNTERS, dtype=torch.int64, device=dev)
        self.cycle_log_cap = cycle_log_cap
        self.cycle_log = torch.empty((max(cycle_log_cap, 1), CYCLE_REC), dtype=torch.int64,
                                     device=dev)
        self.phase_clock = (torch.zeros(4, dtype=torch.int64, device=dev) if phase_clock
                            else None)

    def struct(self) -> Result:
        r = Result()
        r.hist = self.hist.data_ptr()
        r.hist_window = self.hist_window.data_ptr()
        r.stats = self.stats.data_ptr()
        r.x_final = self.x_final.data_ptr()
        r.counters = self.counters.data_ptr()
        r.cycle_log = self.cycle_log.data_ptr() if self.cycle_log_cap > 0 else None
        r.cycle_log_cap = self.cycle_log_cap
        r.phase_clock = self.phase_clock.data_ptr() if self.phase_clock is not None else None
        return r

    def to_host(self) -> "HostResult":
        return HostResult(self)


class HostResult:
    """Host copy of one solve's outputs, with the oracle's field names."""

    def __init__(self, o: Outputs):
        p = o.problem
        npar, ns = p.net.n_params, p.net.n_species
        shape = tuple(hi - lo + 1 for lo, hi in zip(p.hist_lo, p.hist_hi))
        st = o.stats.cpu().numpy()
        self.hist = o.hist.cpu().numpy().reshape(shape)
        self.hist_w = o.hist_window.cpu().numpy().reshape(shape)
        self.T_s = float(st[ST_T])
        self.outside = float(st[ST_OUTSIDE])
        self.outside_w = float(st[ST_OUTSIDE_W])
        self.fim = st[ST_FIM:ST_FIM + npar * npar].reshape(npar, npar).copy()
        self.rer = st[ST_RER:ST_RER + npar].copy()
        self.y = st[ST_Y:ST_Y + ns].copy()
        self.x_final = o.x_final.cpu().numpy()[:ns].copy()
        self.counters = {k: int(v) for k, v in zip(COUNTER_NAMES, o.counters.cpu().numpy())}
        n = min(self.counters["n_cycle_log"], o.cycle_log_cap)
        self.cycle_log = o.cycle_log.cpu().numpy()[:n].copy() if o.cycle_log_cap > 0 else None

    @property
    def events(self) -> int:
        c = self.counters
        return c["ev_decorr"] + c["ev_dephase"] + c["ev_par_credited"] + c["ev_par_discarded"]


_default_ctx = {}


def context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def parrep_solve(p: W.Problem, ctx: Optional[Context] = None, stream=None,
                 cycle_log_cap: int = 256) -> Outputs:
    """One ParRep solve; returns device outputs (valid after stream sync)."""
    ctx = ctx or context()
    out = Outputs(ctx, p, cycle_log_cap)
    ps = problem_struct(p)
    rs = out.struct()
    _check(lib().parrep_solve(ctx.h, ctx.net(p.net), C.byref(ps), C.byref(rs),
                              _stream_ptr(stream)))
    return out


def parrep_solve_noalloc(p: W.Problem, outputs: "Outputs", ctx: Optional[Context] = None,
                         stream=None) -> "Outputs":
    """parrep_solve with its scratch in the library's fixed device array:
    no device allocation in the call (outputs are allocated by the caller)."""
    ctx = ctx or context()
    ps = problem_struct(p)
    rs = outputs.struct()
    _check(lib().parrep_solve_noalloc(ctx.h, ctx.net(p.net), C.byref(ps), C.byref(rs),
                                      _stream_ptr(stream)))
    return outputs


def parrep_solve_batch(problems: Sequence[W.Problem], ctx: Optional[Context] = None,
                       stream=None, replicas_per_lane: int = 0, waves: int = 0,
                       cycle_log_cap: int = 0, outputs: Optional[List[Outputs]] = None,
                       events=None, workgroups: int = 0, chunk_rounds=(0, 0),
                       barrier_wait_us: int = 0, histogram_staging: int = 0,
                       flush_period: int = 0, persistent: int = 0) -> List[Outputs]:
    """Many independent solves in one launch; returns per-instance device outputs.
    workgroups, chunk_rounds, barrier_wait_us: see parrep_launch (spreading a
    single instance over workgroups)."""
    ctx = ctx or context()
    n = len(problems)
    outs = outputs if outputs is not None else [Outputs(ctx, p, cycle_log_cap) for p in problems]
    nets = (C.c_void_p * n)(*[ctx.net(p.net).value for p in problems])
    ps = (Problem * n)(*[problem_struct(p) for p in problems])
    rs = (Result * n)(*[o.struct() for o in outs])
    la = Launch(replicas_per_lane, waves, None, None, workgroups,
                (C.c_int32 * 2)(*chunk_rounds), barrier_wait_us, histogram_staging, flush_period,
                persistent)
    if events is not None:  # (before, after) torch.cuda.Event pair, already created
        la.event_before, la.event_after = events[0].cuda_event, events[1].cuda_event
    _check(lib().parrep_solve_batch(ctx.h, n, nets, ps, rs, C.byref(la), _stream_ptr(stream)))
    return outs


EST_FIM, EST_FIM_HW, EST_RER, EST_Y, EST_IAF, EST_BOUND, EST_LEN = 0, 64, 72, 80, 84, 88, 120


def parrep_estimate(outputs: Sequence["Outputs"], ctx: Optional[Context] = None, stream=None):
    """Multi-run estimators (Sec. III) of the runs in outputs (one problem's
    independent runs) on the device; returns the PARREP_EST_* buffer (device
    tensor of EST_LEN doubles)."""
    torch = _torch()
    ctx = ctx or context()
    p = outputs[0].problem
    out = torch.empty(EST_LEN, dtype=torch.float64, device=ctx.torch_device)
    ptrs = (C.c_void_p * len(outputs))(*[o.stats.data_ptr() for o in outputs])
    _check(lib().parrep_estimate(ctx.h, len(outputs), ptrs, p.net.n_params, p.net.n_species,
                                 p.T - p.t_burn, C.c_void_p(out.data_ptr()),
                                 _stream_ptr(stream)))
    return out


def split_estimates(est, n_params: int, n_species: int) -> dict:
    """Host view of an estimates buffer, with the oracle's field names."""
    e = est.cpu().numpy() if hasattr(est, "cpu") else np.asarray(est)
    p, s = n_params, n_species
    return dict(fim_mean=e[EST_FIM:EST_FIM + p * p].reshape(p, p).copy(),
                fim_hw=e[EST_FIM_HW:EST_FIM_HW + p].copy(), rer_mean=e[EST_RER:EST_RER + p].copy(),
                y_mean=e[EST_Y:EST_Y + s].copy(), iaf=e[EST_IAF:EST_IAF + s].copy(),
                bound=e[EST_BOUND:EST_BOUND + s * p].reshape(s, p).copy())


def parrep_philox(ctr_key, ctx: Optional[Context] = None, stream=None):
    """Philox4x32-10 blocks on the device: ctr_key (n x 6 uint32 numpy) -> (n x 4) numpy."""
    torch = _torch()
    ctx = ctx or context()
    ck = np.ascontiguousarray(ctr_key, dtype=np.uint32)
    n = ck.shape[0]
    d_in = torch.from_numpy(ck.view(np.int32)).to(ctx.torch_device)
    d_out = torch.empty((n, 4), dtype=torch.int32, device=ctx.torch_device)
    _check(lib().parrep_philox(ctx.h, n, d_in.data_ptr(), d_out.data_ptr(), _stream_ptr(stream)))
    return d_out.cpu().numpy().view(np.uint32)


def parrep_events(net: W.Network, c, states, blocks, ctx: Optional[Context] = None, stream=None):
    """SSA events on the device: returns (a0, tau, J) numpy arrays."""
    torch = _torch()
    ctx = ctx or context()
    st = np.zeros((len(states), MAX_S), dtype=np.int32)
    st[:, :np.asarray(states).shape[1]] = states
    bl = np.ascontiguousarray(blocks, dtype=np.uint32)
    n = st.shape[0]
    dev = ctx.torch_device
    d_st = torch.from_numpy(st).to(dev)
    d_bl = torch.from_numpy(bl.view(np.int32)).to(dev)
    a0 = torch.empty(n, dtype=torch.float64, device=dev)
    tau = torch.empty(n, dtype=torch.float64, device=dev)
    J = torch.empty(n, dtype=torch.int32, device=dev)
    cc = (C.c_double * MAX_P)(*list(c) + [0.0] * (MAX_P - len(c)))
    _check(lib().parrep_events(ctx.h, ctx.net(net), cc, n, d_st.data_ptr(), d_bl.data_ptr(),
                               a0.data_ptr(), tau.data_ptr(), J.data_ptr(), _stream_ptr(stream)))
    return a0.cpu().numpy(), tau.cpu().numpy(), J.cpu().numpy()


def parrep_dephase_only(p: W.Problem, xt, cycle: int = 0, ctx: Optional[Context] = None,
                        stream=None):
    """Dephasing step alone from xt; returns (R x n states, rounds)."""
    torch = _torch()
    ctx = ctx or context()
    dev = ctx.torch_device
    Y = torch.empty((p.R, MAX_S), dtype=torch.int32, device=dev)
    rounds = torch.empty(1, dtype=torch.int64, device=dev)
    xx = (C.c_int32 * MAX_S)(*list(xt) + [0] * (MAX_S - len(xt)))
    ps = problem_struct(p)
    _check(lib().parrep_dephase_only(ctx.h, ctx.net(p.net), C.byref(ps), xx, cycle, Y.data_ptr(),
                                     rounds.data_ptr(), _stream_ptr(stream)))
    return Y.cpu().numpy()[:, :p.net.n_species], int(rounds.cpu().item())


def parrep_parallel_only(p: W.Problem, init, cycle: int = 0, max_rounds: int = -1,
                         ctx: Optional[Context] = None, stream=None):
    """Parallel step alone from init (R x n); returns (N*, K, exit_state, credited)."""
    torch = _torch()
    ctx = ctx or context()
    dev = ctx.torch_device
    st = np.zeros((p.R, MAX_S), dtype=np.int32)
    st[:, :p.net.n_species] = init
    d_init = torch.from_numpy(st).to(dev)
    o64 = torch.empty(2, dtype=torch.int64, device=dev)
    ex = torch.empty(MAX_S, dtype=torch.int32, device=dev)
    cr = torch.empty(1, dtype=torch.float64, device=dev)
    ps = problem_struct(p)
    _check(lib().parrep_parallel_only(ctx.h, ctx.net(p.net), C.byref(ps), d_init.data_ptr(),
                                      cycle, max_rounds, o64.data_ptr(), ex.data_ptr(),
                                      cr.data_ptr(), _stream_ptr(stream)))
    o = o64.cpu().numpy()
    return int(o[0]), int(o[1]), ex.cpu().numpy()[:p.net.n_species], float(cr.cpu().item())


class Plan:
    """A batch prepared once and replayed as one hipGraph launch."""

    def __init__(self, problems: Sequence[W.Problem], ctx: Optional[Context] = None,
                 cycle_log_cap: int = 0, outputs: Optional[List[Outputs]] = None,
                 replicas_per_lane: int = 0, waves: int = 0, histogram_staging: int = 0,
                 flush_period: int = 0, persistent: int = 0):
        self.ctx = ctx or context()
        n = len(problems)
        self.problems = list(problems)
        self.outputs = outputs if outputs is not None else [Outputs(self.ctx, p, cycle_log_cap)
                                                            for p in problems]
        nets = (C.c_void_p * n)(*[self.ctx.net(p.net).value for p in problems])
        ps = (Problem * n)(*[problem_struct(p) for p in problems])
        rs = (Result * n)(*[o.struct() for o in self.outputs])
        la = Launch(replicas_per_lane, waves, None, None)
        la.histogram_staging, la.flush_period = histogram_staging, flush_period
        la.persistent = persistent
        h = C.c_void_p()
        _check(lib().parrep_plan_create(self.ctx.h, n, nets, ps, rs, C.byref(la), C.byref(h)))
        self.h = h

    def launch(self, stream=None):
        _check(lib().parrep_plan_launch(self.h, _stream_ptr(stream)))

    def run(self, stream=None, events=None):
        """The plan's work as individual launches (no graph); events: an
        optional (before, after) torch.cuda.Event pair recorded around the
        instance kernels."""
        eb, ea = (events[0].cuda_event, events[1].cuda_event) if events else (None, None)
        _check(lib().parrep_plan_run(self.h, eb, ea, _stream_ptr(stream)))

    def update(self, index: int, p: W.Problem, stream=None):
        ps = problem_struct(p)
        _check(lib().parrep_plan_update(self.h, index, C.byref(ps), _stream_ptr(stream)))
        self.problems[index] = p
        self.outputs[index].problem = p

    def close(self):
        if getattr(self, "h", None):
            lib().parrep_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def parrep_autotune(p: W.Problem, instances: int = 1024, trial_events: int = 2_000_000,
                    ctx: Optional[Context] = None):
    """Time every compiled launch shape (and histogram staging setting) on
    copies of p; returns (replicas_per_lane, waves, histogram_staging,
    flush_period), which later batches of the same replica-count bucket then
    use."""
    ctx = ctx or context()
    scratch = Outputs(ctx, p, cycle_log_cap=0)
    ps = problem_struct(p)
    rs = scratch.struct()
    la = Launch()
    _check(lib().parrep_autotune(ctx.h, ctx.net(p.net), C.byref(ps), instances, trial_events,
                                 C.byref(rs), C.byref(la)))
    return la.replicas_per_lane, la.waves, la.histogram_staging, la.flush_period


class Server:
    """Request loop with continuous batching (see parrep_server_create)."""

    def __init__(self, ctx: Optional[Context] = None, mem_budget: int = 0, n_streams: int = 4):
        self.ctx = ctx or context()
        h = C.c_void_p()
        _check(lib().parrep_server_create(self.ctx.h, mem_budget, n_streams, C.byref(h)))
        self.h = h
        self._problems = {}

    def submit(self, p: W.Problem, rse_target: float = 0.0, min_runs: int = 1,
               max_runs: Optional[int] = None, event_budget: int = 0) -> int:
        rq = Request(rse_target, min_runs, max_runs if max_runs is not None else min_runs,
                     event_budget)
        ps = problem_struct(p)
        t = C.c_uint64()
        _check(lib().parrep_server_submit(self.h, self.ctx.net(p.net), C.byref(ps), C.byref(rq),
                                          C.byref(t)))
        self._problems[t.value] = p
        return t.value

    def poll(self, ticket: int, wait: bool = True):
        """None while running (wait=False); else (pooled HostResult, info dict)."""
        p = self._problems[ticket]
        out = Outputs(self.ctx, p, cycle_log_cap=0)
        rs = out.struct()
        info = RequestInfo()
        rc = lib().parrep_server_poll(self.h, ticket, C.byref(rs), C.byref(info), 1 if wait else 0)
        if rc == -5:  # PARREP_EBUSY
            return None
        del self._problems[ticket]
        _check(rc)
        return out.to_host(), {"runs": info.runs, "status": info.status, "rse": info.rse,
                               "events": info.events, "latency_s": info.latency_s,
                               "iaf": list(info.iaf)[:p.net.n_species]}

    def cancel(self, ticket: int):
        _check(lib().parrep_server_cancel(self.h, ticket))

    def close(self):
        if getattr(self, "h", None):
            lib().parrep_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
