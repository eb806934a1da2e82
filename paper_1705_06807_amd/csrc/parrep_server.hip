// parrep_server.hip -- the served form of the C ABI: a request loop with
// continuous batching.  A request asks for a ParRep estimate to a relative
// standard error: independent runs of one problem (instance ids id, id+1,
// ...) pooled on the device until the error target, the run cap or the
// event budget is reached.  A worker thread admits requests by device
// memory, launches the runs that are ready as one batch on whichever of the
// server's streams is free (batches on different streams overlap on the
// device), pools finished runs into their request, and decides whether a
// request needs more runs.  Each run's outputs equal a plain solve of the
// same problem; pooling adds histograms (device atomics) and averages the
// per-run FIM, RER and window integrals on the host.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <new>
#include <thread>
#include <vector>

#include "parrep_host.h"

using namespace parrep;
using namespace parrep::host;

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kNS = PARREP_NSTATS, kNC = PARREP_NCOUNTERS;
// Per-run host record copied back after a batch: stats, counters, x_final.
struct RunRec {
    double stats[kNS];
    int64_t counters[kNC];
    int32_t x_final[kMaxS];
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Req {
    uint64_t ticket = 0;
    const parrep_net* net = nullptr;
    parrep_problem prob{};
    parrep_request rq{};
    int64_t nbins = 0;
    enum State { QUEUED, ACTIVE, DONE, CANCELLED, FAILED } state = QUEUED;
    bool forgotten = false;  // polled after a cancel while runs were in flight
    int launched = 0, done = 0, inflight = 0, wave_target = 0;
    int64_t events = 0;
    double* d_pool = nullptr;  // [hist | hist_window], 2 * nbins
    hipEvent_t pool_ready = nullptr;
    size_t pool_bytes = 0, run_bytes = 0;
    double stats_sum[kNS] = {};
    std::vector<double> fim_diag, y;  // per run: n_params, n_species values
    int64_t counters[kNC] = {};
    int32_t x_final[kMaxS] = {};
    double rse = std::numeric_limits<double>::quiet_NaN();
    int status = PARREP_OK;
    Clock::time_point t_submit, t_done;
};

struct Batch {
    int stream = 0;
    std::vector<std::pair<Req*, int>> runs;  // (request, run index)
    size_t mem = 0;
    hipEvent_t done = nullptr;
};

}  // namespace

struct parrep_server {
    parrep_ctx* ctx = nullptr;
    size_t budget = 0, in_use = 0;
    int max_batch = 1024;
    std::vector<hipStream_t> streams;
    std::vector<bool> busy;
    std::vector<RunRec*> pinned;  // per stream, max_batch host-pinned run records
    hipStream_t mem_stream = nullptr;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    uint64_t next = 1;
    std::map<uint64_t, Req*> reqs;
    std::deque<Req*> ready;  // requests with runs to launch
    std::vector<Batch> inflight;
};

namespace {

// Device bytes one run needs while in flight: its outputs and its share of
// the batch arena.
size_t run_bytes(const DevInst& d, int64_t nbins) {
    size_t b = align256(2 * (size_t)nbins * 8) + align256(sizeof(RunRec));
    b += align256(sizeof(DevInst)) + align256((size_t)kMaxM * d.tab_L * 8) +
         align256(kAccLen * 8) + align256(kSpillCap * sizeof(SpillSlot)) +
         align256((size_t)d.R * kMaxS * 4) + align256((size_t)d.R * 32);
    return b;
}

// Relative standard error of the pooled estimates: FIM diagonal entries and
// window integrals of each species, max over those with a nonzero mean.
double pooled_rse(const Req& r) {
    const int n = r.done;
    if (n < 2) return std::numeric_limits<double>::quiet_NaN();
    const int np = r.net->net.n_params, ns = r.net->net.n_species;
    double worst = 0.0;
    auto one = [&](const std::vector<double>& v, int stride, int k) {
        double m = 0.0;
        for (int i = 0; i < n; ++i) m += v[(size_t)i * stride + k];
        m /= n;
        if (m == 0.0) return;
        double s2 = 0.0;
        for (int i = 0; i < n; ++i) {
            const double d = v[(size_t)i * stride + k] - m;
            s2 += d * d;
        }
        s2 /= (n - 1);
        worst = std::max(worst, std::sqrt(s2 / n) / std::fabs(m));
    };
    for (int k = 0; k < np; ++k) one(r.fim_diag, np, k);
    for (int k = 0; k < ns; ++k) one(r.y, ns, k);
    return worst;
}

// Total runs a request should have launched by now: the first min_runs;
// once they have finished and the error is above target, as many as meet it
// at the observed spread (done * (rse/target)^2), within max_runs and the
// event budget.  Follow-up runs start as soon as the first min_runs have
// finished, while later ones may still be running.
int wanted_runs(const Req& r) {
    const parrep_request& q = r.rq;
    if (r.done < q.min_runs) return std::max(r.launched, q.min_runs);
    if (q.event_budget > 0 && r.events >= q.event_budget) return r.launched;
    if (!(q.rse_target > 0.0)) return std::max(r.launched, q.max_runs);
    if (!std::isfinite(r.rse)) return std::max(r.launched, std::min(q.max_runs, 2));
    if (r.rse <= q.rse_target) return r.launched;
    const double ratio = r.rse / q.rse_target;
    const double need = std::ceil(r.done * ratio * ratio);
    return std::max(r.launched, (int)std::min(need, (double)q.max_runs));
}

void finish(parrep_server* s, Req& r, int status) {
    r.state = status == PARREP_OK ? Req::DONE : Req::FAILED;
    r.status = status;
    r.t_done = Clock::now();
    s->cv_done.notify_all();
}

void release_pool(parrep_server* s, Req& r) {
    if (r.d_pool) (void)hipFreeAsync(r.d_pool, s->mem_stream);
    if (r.pool_ready) (void)hipEventDestroy(r.pool_ready);
    r.d_pool = nullptr;
    r.pool_ready = nullptr;
    s->in_use -= r.pool_bytes;
    r.pool_bytes = 0;
}

// A finished batch: fold each run into its request.
void complete(parrep_server* s, Batch& b) {
    const RunRec* rec = s->pinned[b.stream];
    for (size_t k = 0; k < b.runs.size(); ++k) {
        Req& r = *b.runs[k].first;
        const RunRec& x = rec[k];
        r.inflight -= 1;
        if (r.state == Req::ACTIVE) {
            r.done += 1;
            for (int i = 0; i < kNS; ++i) r.stats_sum[i] += x.stats[i];
            for (int i = 0; i < kNC; ++i)
                r.counters[i] = i == PARREP_CNT_STATUS ? std::max(r.counters[i], x.counters[i])
                                                        : r.counters[i] + x.counters[i];
            r.events += x.counters[0] + x.counters[1] + x.counters[2] + x.counters[3];
            std::memcpy(r.x_final, x.x_final, sizeof(r.x_final));
            const int np = r.net->net.n_params, ns = r.net->net.n_species;
            for (int i = 0; i < np; ++i) r.fim_diag.push_back(x.stats[PARREP_ST_FIM + i * np + i]);
            for (int i = 0; i < ns; ++i) r.y.push_back(x.stats[PARREP_ST_Y + i]);
        }
    }
    s->in_use -= b.mem;
    // each request once (a batch may hold several of its runs)
    std::vector<Req*> touched;
    for (auto& pr : b.runs)
        if (std::find(touched.begin(), touched.end(), pr.first) == touched.end())
            touched.push_back(pr.first);
    for (Req* rp : touched) {
        Req& r = *rp;
        if (r.state == Req::ACTIVE) {
            if (r.done >= r.rq.min_runs) r.rse = pooled_rse(r);
            const int w = r.done >= r.rq.min_runs ? wanted_runs(r) : r.wave_target;
            if (w > r.wave_target) {
                r.wave_target = w;
                if (std::find(s->ready.begin(), s->ready.end(), &r) == s->ready.end())
                    s->ready.push_back(&r);
            } else if (r.inflight == 0 && r.launched == r.wave_target) {
                finish(s, r, PARREP_OK);
            }
            continue;
        }
        if (r.inflight > 0) continue;
        if (r.state == Req::CANCELLED || r.state == Req::FAILED) {
            if (r.state == Req::CANCELLED) release_pool(s, r);
            if (r.forgotten) {
                release_pool(s, r);
                s->reqs.erase(r.ticket);
                delete &r;
            }
        }
    }
    s->busy[b.stream] = false;
    (void)hipEventDestroy(b.done);
}

// Admit and launch the runs that fit on stream si; false if there were none.
bool launch(parrep_server* s, int si) {
    hipStream_t st = s->streams[si];
    std::vector<std::pair<Req*, int>> runs;
    std::vector<DevInst> insts;
    size_t mem = 0;
    for (auto it = s->ready.begin(); it != s->ready.end() && (int)runs.size() < s->max_batch;) {
        Req& r = **it;
        if (r.state == Req::QUEUED) {
            const size_t need = align256(2 * (size_t)r.nbins * 8);
            if (s->in_use + mem + need + r.run_bytes > s->budget) break;  // keep arrival order
            double* pool = nullptr;
            hipError_t e = hipMallocAsync(&pool, need, s->mem_stream);
            if (e == hipSuccess) e = hipMemsetAsync(pool, 0, need, s->mem_stream);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&r.pool_ready, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventRecord(r.pool_ready, s->mem_stream);
            if (e != hipSuccess) {
                if (pool) (void)hipFreeAsync(pool, s->mem_stream);
                it = s->ready.erase(it);
                finish(s, r, hip_fail(e, "request admission"));
                continue;
            }
            r.d_pool = pool;
            r.pool_bytes = need;
            s->in_use += need;
            r.state = Req::ACTIVE;
            r.wave_target = std::max(1, r.rq.min_runs);
        }
        bool full = false;
        while (r.launched < r.wave_target && (int)runs.size() < s->max_batch) {
            if (s->in_use + mem + r.run_bytes > s->budget) {
                full = true;
                break;
            }
            parrep_problem q = r.prob;
            q.instance_id = r.prob.instance_id + (uint32_t)r.launched;
            DevInst d;
            fill_inst(d, r.net, &q, r.nbins);
            insts.push_back(d);
            runs.emplace_back(&r, r.launched);
            r.launched += 1;
            r.inflight += 1;
            mem += r.run_bytes;
        }
        if (r.launched >= r.wave_target) it = s->ready.erase(it);
        else ++it;
        if (full) break;
    }
    if (runs.empty()) return false;
    const int n = (int)runs.size();
    // outputs: per run [hist | hist_window] then the run records
    std::vector<size_t> off(n);
    size_t o = 0;
    for (int k = 0; k < n; ++k) {
        off[k] = o;
        o += align256(2 * (size_t)runs[k].first->nbins * 8);
    }
    const size_t rec_off = o;
    o += align256((size_t)n * sizeof(RunRec));
    char* block = nullptr;
    int rc = PARREP_OK;
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&block), o, st);
    if (e != hipSuccess) rc = hip_fail(e, "hipMallocAsync");
    RunRec* drec = reinterpret_cast<RunRec*>(block + rec_off);
    if (!rc) {
        for (int k = 0; k < n; ++k) {
            const Req& r = *runs[k].first;
            DevInst& d = insts[k];
            d.hist = reinterpret_cast<double*>(block + off[k]);
            d.hist_w = d.hist + r.nbins;
            d.stats = drec[k].stats;
            d.counters = drec[k].counters;
            d.x_final = drec[k].x_final;
        }
        // run_batch reorders its copy; the outputs travel with each descriptor
        std::vector<DevInst> launch_insts = insts;
        std::lock_guard<std::mutex> lk(s->ctx->mu);
        rc = run_batch(s->ctx, launch_insts, kModeSolve, 0, -1, st, nullptr, nullptr, nullptr);
    }
    for (int k = 0; !rc && k < n; ++k) {
        Req& r = *runs[k].first;
        e = hipStreamWaitEvent(st, r.pool_ready, 0);
        if (e == hipSuccess) e = launch_accumulate(r.d_pool, insts[k].hist, 2 * r.nbins, st);
        if (e != hipSuccess) rc = hip_fail(e, "pooling");
    }
    Batch b;
    b.stream = si;
    b.runs = runs;
    b.mem = mem;
    if (!rc) {
        e = hipMemcpyAsync(s->pinned[si], drec, (size_t)n * sizeof(RunRec), hipMemcpyDeviceToHost,
                           st);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(b.done, st);
        if (e != hipSuccess) rc = hip_fail(e, "batch completion");
    }
    if (block) (void)hipFreeAsync(block, st);
    if (rc) {
        for (auto& pr : runs) {
            Req& r = *pr.first;
            r.inflight -= 1;
            if (r.state == Req::ACTIVE) finish(s, r, rc);
        }
        if (b.done) (void)hipEventDestroy(b.done);
        return true;
    }
    s->in_use += mem;
    s->busy[si] = true;
    s->inflight.push_back(b);
    return true;
}

void worker_main(parrep_server* s) {
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        for (size_t i = 0; i < s->inflight.size();) {
            if (hipEventQuery(s->inflight[i].done) == hipSuccess) {
                complete(s, s->inflight[i]);
                s->inflight.erase(s->inflight.begin() + i);
            } else {
                ++i;
            }
        }
        if (s->stop && s->inflight.empty()) break;
        bool launched = false;
        if (!s->stop) {
            for (size_t si = 0; si < s->streams.size(); ++si)
                if (!s->busy[si] && !s->ready.empty()) launched = launch(s, (int)si) || launched;
        }
        if (!launched)
            s->cv_work.wait_for(lk, std::chrono::microseconds(s->inflight.empty() ? 2000 : 200));
    }
}

}  // namespace

extern "C" {

int parrep_server_create(parrep_ctx* ctx, size_t mem_budget, int32_t n_streams,
                         parrep_server** out) {
    if (!ctx || !out) return fail(PARREP_EINVAL, "NULL argument");
    if (n_streams < 1 || n_streams > 16) return fail(PARREP_EINVAL, "n_streams must be in [1, 16]");
    int rc = set_device(ctx);
    if (rc) return rc;
    parrep_server* s = new (std::nothrow) parrep_server();
    if (!s) return fail(PARREP_ENOMEM, "server allocation");
    s->ctx = ctx;
    if (mem_budget == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) mem_budget = free_b / 2;
    }
    s->budget = mem_budget;
    hipError_t e = hipStreamCreateWithFlags(&s->mem_stream, hipStreamNonBlocking);
    for (int i = 0; e == hipSuccess && i < n_streams; ++i) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) s->streams.push_back(st);
    }
    if (e != hipSuccess) {
        for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
        if (s->mem_stream) (void)hipStreamDestroy(s->mem_stream);
        delete s;
        return hip_fail(e, "server streams");
    }
    s->busy.assign(s->streams.size(), false);
    s->pinned.assign(s->streams.size(), nullptr);
    for (size_t i = 0; e == hipSuccess && i < s->streams.size(); ++i)
        e = hipHostMalloc(reinterpret_cast<void**>(&s->pinned[i]),
                          (size_t)s->max_batch * sizeof(RunRec), hipHostMallocDefault);
    if (e != hipSuccess) {
        for (size_t i = 0; i < s->streams.size(); ++i) {
            if (s->pinned[i]) (void)hipHostFree(s->pinned[i]);
            (void)hipStreamDestroy(s->streams[i]);
        }
        (void)hipStreamDestroy(s->mem_stream);
        delete s;
        return hip_fail(e, "server host buffers");
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return PARREP_OK;
}

int parrep_server_submit(parrep_server* s, const parrep_net* net, const parrep_problem* prob,
                         const parrep_request* rq, uint64_t* ticket) {
    if (!s || !net || !prob || !rq || !ticket) return fail(PARREP_EINVAL, "NULL argument");
    if (net->ctx != s->ctx) return fail(PARREP_EINVAL, "net was created in another context");
    if (rq->min_runs < 1 || rq->max_runs < rq->min_runs)
        return fail(PARREP_EINVAL, "need 1 <= min_runs <= max_runs");
    Req* r = new (std::nothrow) Req();
    if (!r) return fail(PARREP_ENOMEM, "request allocation");
    int rc = validate_problem(net, prob, &r->nbins);
    if (rc) {
        delete r;
        return rc;
    }
    r->net = net;
    r->prob = *prob;
    r->rq = *rq;
    DevInst d;
    fill_inst(d, net, prob, r->nbins);
    r->run_bytes = run_bytes(d, r->nbins);
    if (align256(2 * (size_t)r->nbins * 8) + r->run_bytes > s->budget) {
        delete r;
        return fail(PARREP_ENOMEM, "one run of this request exceeds the server's memory budget");
    }
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->ticket = s->next++;
        s->reqs[r->ticket] = r;
        s->ready.push_back(r);
        *ticket = r->ticket;
    }
    s->cv_work.notify_one();
    return PARREP_OK;
}

int parrep_server_poll(parrep_server* s, uint64_t ticket, const parrep_result* res,
                       parrep_request_info* info, int32_t wait) {
    if (!s) return fail(PARREP_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(PARREP_EINVAL, "unknown ticket");
    Req* r = it->second;
    if (r->state == Req::CANCELLED) {
        if (r->inflight == 0) {
            s->reqs.erase(it);
            release_pool(s, *r);
            delete r;
        } else {
            r->forgotten = true;
        }
        return fail(PARREP_ECANCELLED, "request was cancelled");
    }
    if (r->state == Req::QUEUED || r->state == Req::ACTIVE) {
        if (!wait) return PARREP_EBUSY;
        s->cv_done.wait(lk, [&] { return r->state == Req::DONE || r->state == Req::FAILED; });
    }
    int rc = r->status;
    // a run whose spill table overflowed left time out of FIM, RER and Y:
    // the pooled outputs are written, and the request reports the overflow
    const bool overflow = rc == PARREP_OK && r->counters[PARREP_CNT_STATUS] == PARREP_RUN_SPILL_OVERFLOW;
    if (r->inflight > 0) {  // failed with runs still in flight: reaped when they finish
        r->forgotten = true;
        return rc;
    }
    if (info) {
        info->runs = r->done;
        info->status = overflow ? PARREP_EOVERFLOW : r->status;
        info->rse = r->rse;
        info->events = r->events;
        info->latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
        const int ns = r->net->net.n_species;
        const double win = r->prob.T - r->prob.t_burn;
        for (int i = 0; i < PARREP_MAX_SPECIES; ++i) {
            double v = std::numeric_limits<double>::quiet_NaN();
            if (i < ns && r->done >= 2) {
                double m = 0.0;
                for (int k = 0; k < r->done; ++k) m += r->y[(size_t)k * ns + i];
                m /= r->done;
                double ss = 0.0;
                for (int k = 0; k < r->done; ++k) {
                    const double d = r->y[(size_t)k * ns + i] - m;
                    ss += d * d;
                }
                v = ss / (win * (r->done - 1));
            }
            info->iaf[i] = v;
        }
    }
    if (rc == PARREP_OK && res) {
        rc = check_result(res);
        if (!rc && r->done > 0) {
            // pooled outputs: histograms and clock / outside-box times summed
            // over runs, FIM, RER and window integrals averaged
            double st[kNS];
            for (int i = 0; i < kNS; ++i)
                st[i] = i < PARREP_ST_FIM ? r->stats_sum[i] : r->stats_sum[i] / r->done;
            hipError_t e = hipStreamSynchronize(s->mem_stream);
            if (e == hipSuccess)
                e = hipMemcpy(res->hist, r->d_pool, r->nbins * 8, hipMemcpyDefault);
            if (e == hipSuccess)
                e = hipMemcpy(res->hist_window, r->d_pool + r->nbins, r->nbins * 8,
                              hipMemcpyDefault);
            if (e == hipSuccess) e = hipMemcpy(res->stats, st, sizeof(st), hipMemcpyDefault);
            if (e == hipSuccess)
                e = hipMemcpy(res->counters, r->counters, sizeof(r->counters), hipMemcpyDefault);
            if (e == hipSuccess)
                e = hipMemcpy(res->x_final, r->x_final, sizeof(r->x_final), hipMemcpyDefault);
            if (e != hipSuccess) rc = hip_fail(e, "result copy");
        }
    }
    s->reqs.erase(ticket);
    release_pool(s, *r);
    delete r;
    if (rc == PARREP_OK && overflow)
        rc = fail(PARREP_EOVERFLOW, "a run's spill table overflowed: FIM, RER and window "
                                    "integrals miss time outside the histogram box");
    return rc;
}

int parrep_server_cancel(parrep_server* s, uint64_t ticket) {
    if (!s) return fail(PARREP_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(PARREP_EINVAL, "unknown ticket");
    Req* r = it->second;
    if (r->state == Req::DONE || r->state == Req::FAILED) return PARREP_OK;
    r->state = Req::CANCELLED;
    auto q = std::find(s->ready.begin(), s->ready.end(), r);
    if (q != s->ready.end()) s->ready.erase(q);
    s->cv_done.notify_all();
    return PARREP_OK;
}

void parrep_server_destroy(parrep_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (auto& kv : s->reqs)
            if (kv.second->state == Req::QUEUED || kv.second->state == Req::ACTIVE)
                kv.second->state = Req::CANCELLED;
        s->ready.clear();
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->ctx->device);
    for (auto& kv : s->reqs) {
        release_pool(s, *kv.second);
        delete kv.second;
    }
    (void)hipStreamSynchronize(s->mem_stream);
    for (size_t i = 0; i < s->streams.size(); ++i) {
        (void)hipStreamSynchronize(s->streams[i]);
        (void)hipStreamDestroy(s->streams[i]);
        if (s->pinned[i]) (void)hipHostFree(s->pinned[i]);
    }
    (void)hipStreamDestroy(s->mem_stream);
    delete s;
}

}  // extern "C"
