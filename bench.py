#!/usr/bin/env python3
"""Benchmark the ParRep hot path on one MI355X.

Workload (one step): a batch of independent ParRep trajectories of the
two-gene toggle switch (Omega = 50, a1 = a2 = 3, beta = gamma = 2, R = 1024
replicas, t_c = t_p = 20 time units, horizon T = 2e4, burn-in T/2, 2-D
stationary histogram over [0,400]^2, FIM and RER w.r.t. (a1, a2, beta, gamma)),
seeds = instance ids, all inputs synthetic.  The paper estimates its
stationary and sensitivity quantities from many independent trajectories, so
a step solves a batch of them in one launch.

Prints one JSON line: SSA events/s (all events the method executes:
decorrelation + dephasing + credited and discarded parallel-step events),
the instance kernel's roofline position (VALU-issue bound), and the CPU
oracle timed on the host cores on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SSA events/s on 1 GPU (% VALU peak); batched/served ParRep solves/s + p50/p99"

# Algorithmic VALU work of one SSA event of the toggle switch, in issue
# slots per lane-event (a full-rate op 1 slot; on gfx950 the 32x32->64
# multiply-add is full rate, measured, and the FP64 reciprocal quarter rate,
# 4 slots): Philox4x32-10 10 rounds x (2 multiply-adds + 2 three-way XORs)
# = 40; two 53-bit uniforms 10; -log(u) by table reduction and a degree-7
# log1p 16; four table propensities and their partial sums 9; tau = E/a0 as
# E times the reciprocal of a0 refined by two Newton steps 6; selection 9;
# jump 4; set test 2; replica clock 2.  Total 98.
VALU_SLOTS_PER_EVENT = 98
# FP64 VALU instructions per event in the built kernel (rocprofv3 counters
# SQ_INSTS_VALU_{FMA,ADD,MUL,TRANS}_F64 over events, toggle workload).
FP64_OPS_PER_EVENT_ISA = 25.41
# MI355X: 256 CUs x 4 SIMD16 x 2.4 GHz, a wave64 VALU op takes 4 cycles
# -> 256*4*16*2.4e9 = 3.93e13 lane-op slots per second.
VALU_PEAK_SLOTS = 256 * 4 * 16 * 2.4e9


# HBM traffic of one launch of the instance kernel at the benchmark workload
# (the batch of `instances` trajectories),
# from rocprofv3 FETCH_SIZE / WRITE_SIZE (KiB per dispatch) scaled by what the
# same counters read for a plain device copy of known size; valid only for
# the kernel sources it was measured on (their SHA-256 below).
TRAFFIC = {"instances": 32768,
           "sources_sha256": "609c8a9125eb4e26e72ead6616a26f163b954073dd9fb7963ae222e753e220b9",
           "fetch_kib": 1933805.625, "write_kib": 5687417394.21875,
           "fetch_scale": 524288.0 / 262155.5, "write_scale": 524288.0 / 524288.0}


# The instance kernel is compiled from these files (its translation unit and
# every header it includes).
KERNEL_SOURCES = ("paper_1705_06807_amd/csrc/parrep_instance.hip",
                  "paper_1705_06807_amd/csrc/parrep_device.h",
                  "paper_1705_06807_amd/csrc/parrep_internal.h",
                  "paper_1705_06807_amd/csrc/parrep_neglog.h",
                  "paper_1705_06807_amd/csrc/parrep_fx.h",
                  "include/parrep.h")


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def traffic_bytes(instances: int):
    t = TRAFFIC
    if t["sources_sha256"] is None or t["sources_sha256"] != kernel_sources_sha256():
        return None
    if instances != t["instances"]:
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def copy_calibration(nbytes: int):
    """A plain device-to-device copy of nbytes, three times (for scaling the
    HBM counters: FETCH_SIZE and WRITE_SIZE of this dispatch vs nbytes)."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "copies": 3}), flush=True)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def host_cpus():
    """The host's processor: model name, logical CPUs (nproc), the CPUs this
    process may run on (affinity), and the cgroup's CPU quota when one is
    set (a container's share of the host)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nproc = os.cpu_count() or 1
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = nproc
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, period = f.read().split()[:2]
            if q != "max":
                quota = float(q) / float(period)
    except (OSError, ValueError):
        pass
    usable = affinity if quota is None else max(1, min(affinity, int(quota)))
    return {"model": model, "nproc": nproc, "affinity": affinity, "cgroup_quota": quota,
            "usable": usable}


def cpu_baseline(seconds: float, T_sample: float):
    """Time the CPU oracle (as it stands) on toggle trajectories of the
    benchmark's problem at horizon T_sample, on every CPU this process may
    use: one thread per CPU, each running whole trajectories back to back
    until `seconds` have passed.  The rate is the sum of the threads' own
    rates (events over the time each spent in its trajectories), so the
    last trajectories' tail does not count as idle time."""
    import threading
    from oracle import build as ob
    ob.build(force=False)
    from oracle import oracle as O
    from paper_1705_06807_amd import workloads as W

    cpus = host_cpus()
    threads = cpus["usable"]
    lock = threading.Lock()
    state = {"next": 0}
    per_thread = [[0, 0.0, 0] for _ in range(threads)]  # events, busy seconds, trajectories
    phases = [0, 0, 0, 0]
    t_start = time.perf_counter()

    def worker(k):
        while time.perf_counter() - t_start < seconds:
            with lock:
                i = state["next"]
                state["next"] += 1
            p = W.c2_toggle(seed=0, instance_id=100000 + i, T=T_sample)
            t = time.perf_counter()
            r = O.run(p, cycle_log_cap=0)
            dt = time.perf_counter() - t
            c = r.counters
            ph = (c["ev_decorr"], c["ev_dephase"], c["ev_par_credited"], c["ev_par_discarded"])
            with lock:
                per_thread[k][0] += sum(ph)
                per_thread[k][1] += dt
                per_thread[k][2] += 1
                for j in range(4):
                    phases[j] += ph[j]

    ts = [threading.Thread(target=worker, args=(k,)) for k in range(threads)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    wall = time.perf_counter() - t_start
    rate = sum(e / b for e, b, _ in per_thread if b > 0)
    n = sum(t for _, _, t in per_thread)
    tot = max(1, sum(phases))
    return {"value": rate, "unit": "events/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpus["model"], "nproc": cpus["nproc"], "affinity": cpus["affinity"],
            "cgroup_cpu_quota": cpus["cgroup_quota"],
            "events_by_phase": {"ev_decorr": phases[0] / tot, "ev_dephase": phases[1] / tot,
                                "ev_par_credited": phases[2] / tot,
                                "ev_par_discarded": phases[3] / tot},
            "sample": "%d toggle trajectories of the benchmark problem (Omega=50, R=1024, "
                      "t_c=t_p=20, T=%g), %d threads (one per usable CPU) running whole "
                      "trajectories for %.1f s wall; rate = sum over threads of events / busy "
                      "time" % (n, T_sample, threads, wall)}


def _toggle_law(omega):
    """Exact stationary law of the toggle switch at this Omega on its
    histogram box [0, 8 Omega]^2: a truncated-generator solve on
    [0, 6 Omega]^2 (the mass beyond is below 1e-16; at Omega = 50 it agrees
    with the solve on the whole box to 1.5e-13 in TV), zero outside."""
    import numpy as np
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import exact_laws as E
    n, N = int(round(6 * omega)), int(round(8 * omega))
    _, pi = E.toggle_pi(float(omega), n)
    out = np.zeros((N + 1, N + 1))
    out[:n + 1, :n + 1] = pi.reshape(n + 1, n + 1)
    return out


def start_toggle_laws(problems, workers):
    """Start the exact laws of the toggle instances with Omega <= 50 in a
    process pool (host CPU work that overlaps the GPU measurements)."""
    from concurrent.futures import ProcessPoolExecutor
    oms = sorted({p.hist_hi[0] / 8.0 for p in problems
                  if p.net.name == "toggle" and p.hist_hi[0] <= 400})
    ex = ProcessPoolExecutor(max_workers=max(1, min(workers, len(oms))))
    return ex, {om: ex.submit(_toggle_law, om) for om in oms}


def forms(B, W, ctx, args, laws=None):
    """Batched and served forms at the configured horizons (Schloegl T = 200,
    toggle T = 2e4).  Batched: the 256-instance mix as one hipGraph plan
    launch, against the same 256 instances solved one at a time.  Served: a
    Poisson request stream with continuous batching (p50/p99 latency),
    against the same requests' runs solved one at a time.  Accuracy: every
    batched and served output equals its plain solve (integers exactly,
    floats to 1e-12), and the pooled stationary histogram of the toggle
    instances with Omega <= 50 is compared with the mixture of their exact
    laws in total variation."""
    import numpy as np
    import torch

    Tt = args.forms_T
    probs = W.c3_batch(seed=0, n_schlogl=128, n_toggle=128, T_toggle=Tt)
    law_pool, law_futures = laws if laws is not None else start_toggle_laws(probs, 4)
    plan = B.Plan(probs, ctx=ctx)
    plan.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.launch()
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    batched = len(probs) / t_batch
    bh = [o.to_host() for o in plan.outputs]
    plan.close()
    log("forms: batched %d instances in %.2f s" % (len(probs), t_batch))
    # the same plan in the persistent form (resident workgroups taking each
    # group's instances from a counter), timed the same way
    pplan = B.Plan(probs, ctx=ctx, persistent=1)
    pplan.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pplan.launch()
    torch.cuda.synchronize()
    t_pers = time.perf_counter() - t0
    pers_h = [o.to_host() for o in pplan.outputs]
    pplan.close()
    log("forms: persistent batched %d instances in %.2f s" % (len(probs), t_pers))

    def plain_solves(ps):
        outs = []
        t0 = time.perf_counter()
        for i, p in enumerate(ps):
            o = B.parrep_solve(p, ctx=ctx, cycle_log_cap=0)
            torch.cuda.synchronize()
            outs.append(o)
            if i % 32 == 31:
                log("forms: %d of %d plain solves, %.1f s" % (i + 1, len(ps),
                                                              time.perf_counter() - t0))
        return time.perf_counter() - t0, [o.to_host() for o in outs]

    t_plain, ph = plain_solves(probs)
    plain = len(probs) / t_plain
    log("forms: plain %d instances one at a time in %.2f s" % (len(probs), t_plain))

    def same(a, b):
        if a.counters != b.counters or a.T_s != b.T_s:
            return False
        scale = max(np.abs(b.hist).max(), 1e-300)
        return bool(np.abs(a.hist - b.hist).max() <= 1e-12 * scale)

    batch_equal = all(same(a, b) for a, b in zip(bh, ph))
    # pooled TV of the Omega <= 50 toggle instances against the mixture of exact laws
    laws = {}
    emp = None
    mix = None
    n_tv = 0
    for p, h in zip(probs, bh):
        if p.net.name != "toggle" or p.hist_hi[0] > 400:
            continue
        om = p.hist_hi[0] / 8.0
        if om not in laws:
            laws[om] = law_futures[om].result()
        if emp is None:
            emp = np.zeros((401, 401))
            mix = np.zeros((401, 401))
        n1 = p.hist_hi[0] + 1
        emp[:n1, :n1] += h.hist
        mix[:n1, :n1] += laws[om] * p.T
        n_tv += 1
    tv = tv_well = None
    if n_tv:
        e, m = emp / emp.sum(), mix / mix.sum()
        tv = 0.5 * float(np.abs(e - m).sum())
        # within each well (u > v, u <= v): the error of the sampled
        # quasi-stationary shapes, without the noise of how the few well
        # switches per trajectory split the time
        g = np.arange(401)
        upper = g[:, None] > g[None, :]
        tv_well = 0.0
        for wmask in (upper, ~upper):
            ew, mw = e * wmask, m * wmask
            tv_well += float(mw.sum()) * 0.5 * float(np.abs(ew / ew.sum() - mw / mw.sum()).sum())
    law_pool.shutdown()

    # served: Poisson arrivals at 0.8 x the batched capacity in requests/s
    runs_min, runs_max = args.serve_runs
    rate = 0.8 * batched / (0.5 * (runs_min + runs_max))
    arrivals, reqs = W.c5_requests(seed=0, n=args.serve_requests, rate=rate, T_toggle=Tt)
    srv = B.Server(ctx=ctx, n_streams=4)
    t_start = time.perf_counter()
    tickets = []
    for a, p in zip(arrivals, reqs):
        dt = t_start + a - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        tickets.append(srv.submit(p, rse_target=0.02, min_runs=runs_min, max_runs=runs_max))
    done = [srv.poll(t) for t in tickets]
    t_serve = time.perf_counter() - t_start
    srv.close()
    infos = [d[1] for d in done]
    runs = int(sum(i["runs"] for i in infos))
    log("forms: served %d requests (%d runs) in %.2f s" % (len(reqs), runs, t_serve))
    # the same runs, one plain solve each (instance ids prob.instance_id + k)
    run_probs = [p.replace(instance_id=p.instance_id + k)
                 for p, i in zip(reqs, infos) for k in range(i["runs"])]
    t_plain5, ph5 = plain_solves(run_probs)
    log("forms: plain %d runs one at a time in %.2f s" % (len(run_probs), t_plain5))
    # each pooled request equals the sum of its runs solved alone
    served_equal = True
    k = 0
    for (pooled, info), p in zip(done, reqs):
        alone = ph5[k:k + info["runs"]]
        k += info["runs"]
        hsum = sum(a.hist for a in alone)
        scale = max(np.abs(hsum).max(), 1e-300)
        served_equal &= bool(np.abs(pooled.hist - hsum).max() <= 1e-12 * scale)
        served_equal &= pooled.counters["ev_decorr"] == sum(a.counters["ev_decorr"] for a in alone)
    lat = np.array([i["latency_s"] for i in infos])
    met = sum(1 for i in infos if i["rse"] <= 0.02)
    large = large_single_run(B, W, ctx) if not args.no_large else None
    return {
        "workload": "C3 mix (128 Schloegl c x logU[0.9,1.1] T=200, 128 toggle Omega~U{25..100} "
                    "T=%g, R~logU[64,4096]) and C5 stream (Schloegl T=200 / toggle "
                    "Omega~U{25..150} T=%g, R~logU[256,16384], %d-%d runs per request, "
                    "2%% RSE target)" % (Tt, Tt, runs_min, runs_max),
        "batched_solves_per_s": batched,
        "batched_persistent_solves_per_s": len(probs) / t_pers,
        "batched_persistent_equals_batched": all(same(a, b) for a, b in zip(pers_h, bh)),
        "plain_solves_per_s": plain,
        "batched_over_plain": batched / plain,
        "plain_sample": "all %d instances solved one at a time" % len(probs),
        "batched_equals_plain": batch_equal,
        "tv_pooled_toggle_omega_le_50": tv,
        "tv_within_wells_toggle_omega_le_50": tv_well,
        "tv_instances": n_tv,
        "served": {
            "requests": len(infos), "arrival_rate_per_s": rate,
            "runs": runs, "seconds": t_serve, "solves_per_s": runs / t_serve,
            "plain_solves_per_s": len(run_probs) / t_plain5,
            "plain_sample": "the same %d runs solved one at a time" % len(run_probs),
            "served_over_plain": (runs / t_serve) / (len(run_probs) / t_plain5),
            "served_equals_plain": served_equal,
            "latency_p50_s": float(np.percentile(lat, 50)),
            "latency_p99_s": float(np.percentile(lat, 99)),
            "rse_target": 0.02, "runs_per_request": [runs_min, runs_max],
            "met_target": met,
        },
        "large_single_run": large,
    }


def large_single_run(B, W, ctx):
    """The large single run (toggle Omega = 150, R = 65536, T = 1e5,
    histogram [0, 1200]^2): one instance spread over 256 workgroups (the
    library's choice for R >= 8192), timed after one untimed run, beside the
    same instance on one workgroup of 16 waves; both must agree."""
    import numpy as np
    import torch
    p = W.c4_toggle(seed=0)
    out = B.Outputs(ctx, p, cycle_log_cap=0)
    res = {}
    for name, kw in (("spread", {}), ("one_workgroup", {"workgroups": 1})):
        for rep in range(2 if name == "spread" else 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            B.parrep_solve_batch([p], ctx=ctx, outputs=[out], **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        res[name] = (dt, out.to_host())
    dt, h = res["spread"]
    dt1, h1 = res["one_workgroup"]
    ev = h.events
    same = (h.counters == h1.counters and
            bool(np.abs(h.hist - h1.hist).max() <= 1e-12 * np.abs(h1.hist).max()))
    log("large single run: %.3f s spread, %.2f s on one workgroup" % (dt, dt1))
    return {"workload": "toggle Omega=150, R=65536, t_c=t_p=20, T=1e5, hist [0,1200]^2, one "
                        "instance",
            "launch": "256 workgroups x 4 waves, 1 replica per lane, chunks 512/64 rounds",
            "seconds": dt, "events": int(ev), "events_per_s": ev / dt,
            "one_workgroup_seconds": dt1, "one_workgroup_events_per_s": ev / dt1,
            "spread_equals_one_workgroup": same,
            "cycles": int(h.counters["cycles"]), "reached_T": h.T_s == p.T}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--instances", type=int, default=32768,
                    help="independent trajectories per step")
    ap.add_argument("--T", type=float, default=2e4)
    ap.add_argument("--rpl", type=int, default=0, help="replicas per lane (0 = library choice)")
    ap.add_argument("--waves", type=int, default=0, help="waves per workgroup (0 = library)")
    ap.add_argument("--staging", type=int, default=0, choices=(-1, 0, 1),
                    help="parallel-step histogram staging in LDS (0 = library / autotuned)")
    ap.add_argument("--flush-period", type=int, default=0,
                    help="staged: also flush every this many rounds")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="CPU baseline: start trajectories for this long")
    ap.add_argument("--cpu-T", type=float, default=2e4,
                    help="CPU baseline: horizon of the timed trajectories (the benchmark's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched / served measurement")
    ap.add_argument("--forms-T", type=float, default=2e4,
                    help="toggle horizon of the batched and served forms (Schloegl: 200)")
    ap.add_argument("--serve-requests", type=int, default=24)
    ap.add_argument("--serve-runs", type=int, nargs=2, default=(4, 8), metavar=("MIN", "MAX"),
                    help="runs per served request")
    ap.add_argument("--forms-only", action="store_true",
                    help="measure only the batched / served forms")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the large single run (R = 65536) in the forms section")
    ap.add_argument("--phase-clock", action="store_true",
                    help="report where each trajectory's workgroup spent its time")
    ap.add_argument("--workload", choices=("toggle", "genetic_switch"), default="toggle",
                    help="genetic_switch: the general kernels on Sec. IV B's network (V = 2400, "
                         "R = 100, n_c = n_p = 2e4); no roofline (latency-bound at the paper's "
                         "batch of 100 trajectories)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs each ParRep instance on a single "
              "device and has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    from paper_1705_06807_amd import workloads as W
    laws = None
    if not args.no_forms:
        # forked before this process touches the GPU
        laws = start_toggle_laws(W.c3_batch(seed=0, n_schlogl=128, n_toggle=128,
                                            T_toggle=args.forms_T), 4)

    import torch
    from paper_1705_06807_amd import binding as B

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    B.lib()
    ctx = B.context(0)
    if args.forms_only:
        print(json.dumps({"forms": forms(B, W, ctx, args, laws)}), flush=True)
        return
    toggle = args.workload == "toggle"
    if toggle:
        probs = [W.c2_toggle(seed=0, instance_id=i, T=args.T) for i in range(args.instances)]
    else:
        probs = [W.genetic_switch_problem(seed=0, instance_id=i, T=args.T)
                 for i in range(args.instances)]
    shape = None
    if toggle and args.rpl == 0 and args.waves == 0 and args.staging == 0 and not args.no_autotune:
        # untimed: pick the launch shape and histogram staging for R = 1024 on
        # copies with the horizon cut to T/10 (the same mix of steps: every
        # cycle dephases all replicas, the parallel step credits ~T a0 events).
        # Up to 16384 copies, each with its own histograms (42 GB here): the
        # LDS a staging tile takes lowers the workgroups per CU, which a trial
        # shows only when it fills the device for many waves of workgroups,
        # and copies that share one histogram contend on its bins as the
        # batch's trajectories do not.  (1024 copies, or copies sharing one
        # histogram, picked staging: 2.44e11 events/s at full size against
        # 2.68e11 without it.)
        t = time.perf_counter()
        shape = B.parrep_autotune(probs[0].replace(instance_id=1 << 30, T=args.T / 10,
                                                   t_burn=args.T / 20),
                                  instances=min(args.instances, 16384), trial_events=1 << 40,
                                  ctx=ctx)
        log("autotune: replicas_per_lane=%d waves=%d staging=%d flush=%d (%.1f s)"
            % (shape + (time.perf_counter() - t,)))
    outs = [B.Outputs(ctx, p, cycle_log_cap=0, phase_clock=args.phase_clock) for p in probs]
    ev_b = torch.cuda.Event(enable_timing=True)
    ev_a = torch.cuda.Event(enable_timing=True)
    ev_b.record()
    ev_a.record()
    torch.cuda.synchronize()
    # untimed: the batch's descriptors and scratch go to device memory once; each
    # step enqueues setup / zero / the instance kernels / finalize on them, with
    # the inputs already resident, and the two events on the stream around the
    # instance kernels.
    plan = B.Plan(probs, ctx=ctx, outputs=outs, replicas_per_lane=args.rpl, waves=args.waves,
                  histogram_staging=args.staging, flush_period=args.flush_period)
    stream = torch.cuda.current_stream()

    for i in range(args.warmup):
        t = time.perf_counter()
        plan.run(stream)
        torch.cuda.synchronize()
        log("warmup %d: %.3f s" % (i, time.perf_counter() - t))

    kernel_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        plan.run(stream, events=(ev_b, ev_a))
        ev_a.synchronize()
        kernel_ms.append(ev_b.elapsed_time(ev_a))
        log("step %d: instance kernel %.1f ms" % (i, kernel_ms[-1]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.close()

    counters = torch.stack([o.counters for o in outs]).cpu()
    ev = counters[:, 0:4].sum().item()          # decorr + dephase + credited + discarded
    per_phase = {k: int(counters[:, j].sum().item()) for j, k in enumerate(
        ("ev_decorr", "ev_dephase", "ev_par_credited", "ev_par_discarded", "cycles"))}
    t_end = torch.stack([o.stats[0] for o in outs]).cpu()
    ok = bool((counters[:, 7] == 0).all().item()) and bool((t_end == args.T).all().item())

    ms_per_step = 1e3 * wall / args.steps
    value = ev / (wall / args.steps)
    k_avg = sum(kernel_ms) / len(kernel_ms)
    achieved = ev * VALU_SLOTS_PER_EVENT / (k_avg * 1e-3)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": ("toggle switch Omega=50 (a1=a2=3, beta=gamma=2), R=1024, "
                         "t_c=t_p=20, T=%g, burn-in T/2, hist [0,400]^2, FIM+RER(a1,a2,beta,gamma); "
                         "%d independent trajectories per step" % (args.T, args.instances)
                         if toggle else
                         "genetic switch V=2400, R=100, n_c=n_p=2e4 transitions, T=%g, burn-in "
                         "T/2, FIM+RER of 8 parameters; %d independent trajectories per step"
                         % (args.T, args.instances)),
            "instances": args.instances,
            "launch_shape": ({"replicas_per_lane": shape[0], "waves": shape[1],
                              "histogram_staging": shape[2], "flush_period": shape[3],
                              "autotuned": True}
                             if shape else {"replicas_per_lane": args.rpl, "waves": args.waves,
                                            "histogram_staging": args.staging,
                                            "flush_period": args.flush_period}),
            "replicas": probs[0].R,
            "horizon": args.T,
        },
        "solves_per_s": args.instances / (wall / args.steps),
        "events_per_step": ev,
        "events_by_phase": per_phase,
        "all_runs_reached_T": ok,
        "roofline": None if not toggle else {
            "bound": "alu",
            "kernel": "k_instance",
            "achieved": achieved / 1e12,
            "peak": VALU_PEAK_SLOTS / 1e12,
            "unit": "T VALU lane-slots/s",
            "frac": achieved / VALU_PEAK_SLOTS,
            "traffic": traffic_bytes(args.instances),
            "kernel_ms": k_avg,
            "ops_per_event": VALU_SLOTS_PER_EVENT,
            "fp64_ops_per_event_isa": FP64_OPS_PER_EVENT_ISA,
            "fp64_frac": ev * FP64_OPS_PER_EVENT_ISA / (k_avg * 1e-3) / VALU_PEAK_SLOTS,
        },
    }
    if args.phase_clock:
        hz = B.lib().parrep_wall_clock_hz(ctx.h)
        pc = torch.stack([o.phase_clock for o in outs]).cpu().double() / hz
        tot = pc[:, 3]
        line["phase_seconds_per_trajectory"] = {
            "decorrelation": pc[:, 0].mean().item(), "dephasing": pc[:, 1].mean().item(),
            "parallel": pc[:, 2].mean().item(), "total_mean": tot.mean().item(),
            "total_max": tot.max().item(), "total_min": tot.min().item()}
    if not args.no_forms:
        line["forms"] = forms(B, W, ctx, args, laws)
    if not args.no_cpu_baseline:
        log("cpu baseline: %d threads, >= %.0f s" % (host_cpus()["usable"], args.cpu_seconds))
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds, args.cpu_T)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
