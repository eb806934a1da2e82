// parrep_batch.hip -- the batched form of the C ABI: plans (a batch of
// instances captured once into a hipGraph and replayed, with per-instance
// problem updates between replays) and the launch-shape autotuner.
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "parrep_host.h"

using namespace parrep;
using namespace parrep::host;

struct parrep_plan {
    parrep_ctx* ctx = nullptr;
    std::vector<DevInst> insts;  // grouped order, scratch pointers set
    std::vector<int> slot;       // slot[i]: position of caller instance i in insts
    std::vector<Group> groups;
    std::vector<const parrep_net*> nets;  // caller order
    std::vector<int64_t> nbins;           // caller order
    void* base = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t last = nullptr;  // stream of the latest launch or update
};

namespace {

void destroy_plan(parrep_plan* p) {
    if (!p) return;
    if (set_device(p->ctx) == PARREP_OK) {
        if (p->last) (void)hipStreamSynchronize(p->last);
        if (p->exec) (void)hipGraphExecDestroy(p->exec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        if (p->base) (void)hipFree(p->base);
    }
    delete p;
}

}  // namespace

extern "C" {

int parrep_plan_create(parrep_ctx* ctx, int32_t count, const parrep_net* const* nets,
                       const parrep_problem* probs, const parrep_result* res,
                       const parrep_launch* launch, parrep_plan** out) {
    if (!ctx || !nets || !probs || !res || !out) return fail(PARREP_EINVAL, "NULL argument");
    if (count < 1) return fail(PARREP_EINVAL, "count < 1");
    parrep_plan* p = new (std::nothrow) parrep_plan();
    if (!p) return fail(PARREP_ENOMEM, "plan allocation");
    p->ctx = ctx;
    std::vector<DevInst> insts((size_t)count);
    p->nets.assign(nets, nets + count);
    p->nbins.resize(count);
    int maxR = 1, maxS = 1;
    for (int i = 0; i < count; ++i) {
        if (!nets[i] || nets[i]->ctx != ctx) {
            delete p;
            return fail(PARREP_EINVAL, "NULL net or net of another context");
        }
        int rc = validate_problem(nets[i], &probs[i], &p->nbins[i]);
        if (!rc) rc = check_result(&res[i]);
        if (rc) {
            delete p;
            return rc;
        }
        fill_inst(insts[i], nets[i], &probs[i], p->nbins[i]);
        attach_result(insts[i], &res[i]);
        maxR = std::max(maxR, probs[i].R);
        maxS = std::max(maxS, (int)nets[i]->net.n_species);
    }
    LaunchShape forced{};
    if (launch && (launch->histogram_staging < -1 || launch->histogram_staging > 1 ||
                   launch->flush_period < 0)) {
        delete p;
        return fail(PARREP_EINVAL, "histogram_staging must be -1, 0 or 1 and flush_period >= 0");
    }
    const bool force = launch && (launch->replicas_per_lane > 0 || launch->waves > 0 ||
                                  launch->histogram_staging != 0);
    if (force) {
        forced = choose_shape(maxR, maxS, kMaxM);
        forced.rpl = launch->replicas_per_lane > 0 ? launch->replicas_per_lane : forced.rpl;
        forced.waves = launch->waves > 0 ? launch->waves : forced.waves;
        forced.stage_flush = launch->histogram_staging > 0 ? std::max(0, launch->flush_period) : -1;
        int rc = PARREP_OK;
        if ((int64_t)forced.rpl * forced.waves * 64 < maxR)
            rc = fail(PARREP_EINVAL, "launch shape holds fewer replicas than R");
        else if (!shape_supported(forced))
            rc = fail(PARREP_EUNSUPPORTED, "launch shape not compiled in");
        if (rc) {
            delete p;
            return rc;
        }
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    int rc = set_device(ctx);
    if (rc) {
        delete p;
        return rc;
    }
    std::vector<int> order;
    if (launch && (launch->persistent < 0 || launch->persistent > 1)) {
        delete p;
        return fail(PARREP_EINVAL, "persistent must be 0 or 1");
    }
    p->groups = group_batch(ctx, insts, &order, force ? &forced : nullptr,
                            launch && launch->persistent == 1);
    p->slot.resize(count);
    for (int k = 0; k < count; ++k) p->slot[order[k]] = k;
    hipError_t e = hipMalloc(&p->base, arena_bytes(insts, false));
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipMalloc");
    }
    place_arena(insts, static_cast<char*>(p->base), false);
    p->insts = insts;
    e = hipMemcpy(p->base, insts.data(), insts.size() * sizeof(DevInst), hipMemcpyHostToDevice);
    hipStream_t cap = nullptr;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        destroy_plan(p);
        return hip_fail(e, "plan setup");
    }
    // Capture setup, zero, the group launches (forked over the context's
    // auxiliary streams) and finalize into one graph.
    std::vector<hipEvent_t> keep;
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = enqueue_batch(ctx, static_cast<DevInst*>(p->base), count, p->groups, kModeSolve, 0,
                           -1, cap, nullptr, nullptr, &keep);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cap, &g);
        p->graph = g;
        if (!rc && e2 != hipSuccess) rc = hip_fail(e2, "hipStreamEndCapture");
    } else {
        rc = hip_fail(e, "hipStreamBeginCapture");
    }
    for (hipEvent_t ev : keep)
        if (ev) (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(cap);
    if (!rc) {
        e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = hip_fail(e, "hipGraphInstantiate");
    }
    if (rc) {
        destroy_plan(p);
        return rc;
    }
    *out = p;
    return PARREP_OK;
}

int parrep_plan_update(parrep_plan* p, int32_t index, const parrep_problem* prob, void* stream) {
    if (!p || !prob) return fail(PARREP_EINVAL, "NULL argument");
    if (index < 0 || index >= (int)p->slot.size()) return fail(PARREP_EINVAL, "index out of range");
    int64_t nb = 0;
    int rc = validate_problem(p->nets[index], prob, &nb);
    if (rc) return rc;
    DevInst& cur = p->insts[p->slot[index]];
    DevInst d;
    fill_inst(d, p->nets[index], prob, nb);
    const Group* grp = nullptr;
    for (const Group& g : p->groups)
        if (p->slot[index] >= g.first && p->slot[index] < g.first + g.count) grp = &g;
    if (nb != p->nbins[index] || d.tab_L != cur.tab_L || prob->R > cur.R ||
        (int64_t)grp->shape.rpl * grp->shape.waves * 64 < prob->R)
        return fail(PARREP_EINVAL, "update must keep the histogram box, the table length and "
                                   "at most the planned replica count");
    // keep outputs and scratch
    d.hist = cur.hist;
    d.hist_w = cur.hist_w;
    d.stats = cur.stats;
    d.x_final = cur.x_final;
    d.counters = cur.counters;
    d.cycle_log = cur.cycle_log;
    d.cycle_log_cap = cur.cycle_log_cap;
    d.phase_clock = cur.phase_clock;
    d.tab = cur.tab;
    d.tab_owner = 1;
    d.acc = cur.acc;
    d.spill = cur.spill;
    d.xbuf = cur.xbuf;
    d.sbuf = cur.sbuf;
    cur = d;
    rc = set_device(p->ctx);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(static_cast<DevInst*>(p->base) + p->slot[index], &cur,
                                  sizeof(DevInst), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    p->last = st;
    return PARREP_OK;
}

int parrep_plan_launch(parrep_plan* p, void* stream) {
    if (!p) return fail(PARREP_EINVAL, "NULL plan");
    int rc = set_device(p->ctx);
    if (rc) return rc;
    hipError_t e = hipGraphLaunch(p->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    p->last = (hipStream_t)stream;
    return PARREP_OK;
}

int parrep_plan_run(parrep_plan* p, void* event_before, void* event_after, void* stream) {
    if (!p) return fail(PARREP_EINVAL, "NULL plan");
    std::lock_guard<std::mutex> lk(p->ctx->mu);
    int rc = set_device(p->ctx);
    if (rc) return rc;
    rc = enqueue_batch(p->ctx, static_cast<DevInst*>(p->base), (int)p->insts.size(), p->groups,
                       kModeSolve, 0, -1, (hipStream_t)stream, (hipEvent_t)event_before,
                       (hipEvent_t)event_after);
    if (rc) return rc;
    p->last = (hipStream_t)stream;
    return PARREP_OK;
}

void parrep_plan_destroy(parrep_plan* p) { destroy_plan(p); }

int parrep_autotune(parrep_ctx* ctx, const parrep_net* net, const parrep_problem* prob,
                    int32_t instances, int64_t trial_events, const parrep_result* scratch,
                    parrep_launch* chosen) {
    if (!ctx || !net || !prob || !scratch || !chosen) return fail(PARREP_EINVAL, "NULL argument");
    if (net->ctx != ctx) return fail(PARREP_EINVAL, "net was created in another context");
    if (instances < 1 || trial_events < 1) return fail(PARREP_EINVAL, "instances, trial_events");
    int64_t nb = 0;
    int rc = validate_problem(net, prob, &nb);
    if (!rc) rc = check_result(scratch);
    if (rc) return rc;
    rc = set_device(ctx);
    if (rc) return rc;
    const int R = prob->R;
    const int nsc = net->net.n_species <= 1 ? 1 : (net->net.n_species <= 2 ? 2 : 4);
    const int mc = net->net.n_reactions <= 4 ? 4 : 8;
    hipStream_t st = nullptr;
    hipEvent_t eb = nullptr, ea = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&eb);
    if (e == hipSuccess) e = hipEventCreate(&ea);
    if (e != hipSuccess) return hip_fail(e, "autotune setup");
    // Each trial instance credits its own histogram pair, as the instances of
    // a real batch do: with one shared histogram the trial's credits would
    // contend on the same bins, which favours LDS staging over direct
    // atomics.  Up to 64 GiB of trial histograms; beyond that they share
    // the scratch result's.
    double* trial_hist = nullptr;
    const size_t hist_bytes = (size_t)nb * sizeof(double);
    if (2 * hist_bytes * (size_t)instances <= (size_t)64 << 30) {
        e = hipMalloc(&trial_hist, 2 * hist_bytes * (size_t)instances);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            trial_hist = nullptr;
        }
    }
    float best = -1.0f;
    LaunchShape best_s{};
    const int ropts[4] = {1, 4, 16, 64}, wopts[3] = {1, 4, 16};
    // histogram staging (narrow kernels): off, flushed at the step's end, or
    // also every 64 rounds
    const int sopts[3] = {-1, 0, 64};
    for (int a = 0; a < 4 && !rc; ++a)
        for (int b = 0; b < 3 && !rc; ++b)
        for (int c = 0; c < ((narrow_kernel(nsc, mc) && ropts[a] <= 4 && wopts[b] <= 4) ? 3 : 1) &&
                        !rc;
             ++c) {
            LaunchShape s{ropts[a], wopts[b], nsc, mc};
            s.stage_flush = sopts[c];
            const int64_t cap = (int64_t)s.rpl * s.waves * 64;
            if (cap < R || cap > 16 * (int64_t)std::max(R, 64) || !shape_supported(s)) continue;
            // the trial instances share the scratch result's other outputs:
            // only the time of the launch is kept
            std::vector<DevInst> insts((size_t)instances);
            for (int i = 0; i < instances; ++i) {
                parrep_problem q = *prob;
                q.instance_id = prob->instance_id + (uint32_t)i;
                q.max_events = trial_events;
                fill_inst(insts[i], net, &q, nb);
                attach_result(insts[i], scratch);
                if (trial_hist) {
                    insts[i].hist = trial_hist + (size_t)(2 * i) * (size_t)nb;
                    insts[i].hist_w = trial_hist + (size_t)(2 * i + 1) * (size_t)nb;
                }
                insts[i].cycle_log = nullptr;
                insts[i].cycle_log_cap = 0;
            }
            std::lock_guard<std::mutex> lk(ctx->mu);
            rc = run_batch(ctx, insts, kModeSolve, 0, -1, st, eb, ea, &s);
            if (rc) break;
            e = hipStreamSynchronize(st);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, eb, ea);
            if (e != hipSuccess) {
                rc = hip_fail(e, "autotune trial");
                break;
            }
            if (best < 0.0f || ms < best) {
                best = ms;
                best_s = s;
            }
        }
    (void)hipEventDestroy(eb);
    (void)hipEventDestroy(ea);
    (void)hipStreamDestroy(st);
    if (trial_hist) (void)hipFree(trial_hist);
    if (rc) return rc;
    if (best < 0.0f) return fail(PARREP_EUNSUPPORTED, "no compiled launch shape holds R replicas");
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->tuned[std::make_tuple(shape_bucket(R), nsc, mc)] =
            std::make_tuple(best_s.rpl, best_s.waves, best_s.stage_flush);
    }
    chosen->replicas_per_lane = best_s.rpl;
    chosen->waves = best_s.waves;
    chosen->histogram_staging = best_s.stage_flush >= 0 ? 1 : -1;
    chosen->flush_period = std::max(0, best_s.stage_flush);
    chosen->event_before = nullptr;
    chosen->event_after = nullptr;
    return PARREP_OK;
}

}  // extern "C"
