// parrep_api.hip -- the C ABI of libparrep (declared in include/parrep.h):
// argument validation, device descriptors, scratch, and kernel launches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "parrep_internal.h"
#include "parrep_neglog.h"

using namespace parrep;

struct parrep_ctx {
    int device = 0;
    std::mutex mu;
    double* logtab = nullptr;  // device copy of the -log(u) reduction table
};

struct parrep_net {
    parrep_ctx* ctx = nullptr;
    DevNet net{};
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return PARREP_EDEVICE;
}

bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

int validate_problem(const parrep_net* net, const parrep_problem* p, int64_t* nbins_out) {
    const DevNet& N = net->net;
    if (p->R < 1 || p->R > PARREP_MAX_REPLICAS)
        return fail(PARREP_EINVAL, "R must be in [1, " + std::to_string(PARREP_MAX_REPLICAS) + "]");
    for (int k = 0; k < N.n_params; ++k) {
        if (!finite_nonneg(p->c[k])) return fail(PARREP_EINVAL, "c must be finite and >= 0");
        if (p->use_rer && !(std::isfinite(p->rer_eps[k]) && p->rer_eps[k] > -1.0))
            return fail(PARREP_EINVAL, "rer_eps must be finite and > -1");
    }
    for (int j = 0; j < N.n_reactions; ++j)
        for (int f = 0; f < N.rx[j].n_factors; ++f)
            if (N.rx[j].f[f].kind == PARREP_HILL_REP) {
                const double h = p->c[N.rx[j].f[f].hill_param];
                if (!(h <= 64.0) || h != std::floor(h))
                    return fail(PARREP_EUNSUPPORTED, "Hill exponents must be integers in [0, 64]");
            }
    if (!(p->T > 0.0) || !(p->T < 0x1.0p51))
        return fail(PARREP_EINVAL, "T must be in (0, 2^51)");
    if (!(p->t_burn >= 0.0) || !(p->t_burn < p->T))
        return fail(PARREP_EINVAL, "t_burn must be in [0, T)");
    if (p->decorr_mode != PARREP_STEPS && p->decorr_mode != PARREP_TIME)
        return fail(PARREP_EINVAL, "decorr_mode");
    if (p->dephase_mode != PARREP_STEPS && p->dephase_mode != PARREP_TIME)
        return fail(PARREP_EINVAL, "dephase_mode");
    if (!(p->decorr >= 0.0) || !(p->decorr <= 0x1.0p62) || !(p->dephase >= 0.0) ||
        !(p->dephase <= 0x1.0p62))
        return fail(PARREP_EINVAL, "decorr/dephase must be in [0, 2^62]");
    int64_t nb = 1;
    for (int i = 0; i < N.n_species; ++i) {
        if (p->hist_hi[i] < p->hist_lo[i]) return fail(PARREP_EINVAL, "hist_hi < hist_lo");
        const int64_t w = (int64_t)p->hist_hi[i] - p->hist_lo[i] + 1;
        nb *= w;
        if (nb > (int64_t(1) << 31)) return fail(PARREP_EINVAL, "histogram box too large");
    }
    *nbins_out = nb;
    return PARREP_OK;
}

void fill_inst(DevInst& d, const parrep_net* net, const parrep_problem* p, int64_t nbins) {
    std::memset(&d, 0, sizeof(d));
    d.net = net->net;
    d.logtab = net->ctx->logtab;
    const int n = d.net.n_species;
    for (int k = 0; k < kMaxP; ++k) {
        d.c[k] = k < d.net.n_params ? p->c[k] : 0.0;
        d.rer_eps[k] = (k < d.net.n_params && p->use_rer) ? p->rer_eps[k] : 0.0;
    }
    d.use_rer = p->use_rer ? 1 : 0;
    d.decorr_mode = p->decorr_mode;
    d.dephase_mode = p->dephase_mode;
    d.R = p->R;
    d.decorr = p->decorr;
    d.dephase = p->dephase;
    d.T = p->T;
    d.t_burn = p->t_burn;
    for (int i = 0; i < kMaxS; ++i) {
        const bool on = i < n;
        d.x0[i] = on ? p->x0[i] : 0;
        d.region_w[i] = on ? p->region_w[i] : 0;
        d.hist_lo[i] = on ? p->hist_lo[i] : 0;
        d.hist_nb[i] = on ? p->hist_hi[i] - p->hist_lo[i] + 1 : 1;
    }
    int64_t st = 1;
    for (int i = kMaxS - 1; i >= 0; --i) {
        d.hist_stride[i] = st;
        st *= d.hist_nb[i];
    }
    d.region_theta = p->region_theta;
    d.nbins = nbins;
    d.seed = p->seed;
    d.instance_id = p->instance_id;
    d.max_events = p->max_events;
    // Hot-path view: reactions with one state-dependent factor read a table
    // of lambda_j over 0..tab_L-1 of that species.
    for (int j = 0; j < kMaxM; ++j) {
        const DevReaction& r = d.net.rx[j];
        uint32_t kind = kRxConst, sp = 0;
        if (j < d.net.n_reactions && r.n_factors == 1) {
            kind = kRxTable;
            sp = (uint32_t)r.f[0].species;
        } else if (j < d.net.n_reactions && r.n_factors > 1) {
            kind = kRxDirect;
        }
        d.jmeta[j] = kind | (sp << 2);
        uint32_t packed = 0;
        for (int i = 0; i < kMaxS; ++i) packed |= ((uint32_t)(r.stoich[i] & 0xFF)) << (8 * i);
        d.jstoich[j] = packed;
    }
    int hi = 0;
    for (int i = 0; i < n; ++i) hi = std::max(hi, std::max(p->hist_hi[i], p->x0[i]));
    d.tab_L = std::min(8192, std::max(256, ((hi + 64 + 63) / 64) * 64));
}

// Device memory for one launch: descriptors plus per-instance scratch.
struct Arena {
    void* base = nullptr;
    size_t bytes = 0;
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Instances with the same network, rate vector and table length share one
// propensity table; the first of them fills it.
std::string table_key(const DevInst& d) {
    std::string k(reinterpret_cast<const char*>(&d.net), sizeof(d.net));
    k.append(reinterpret_cast<const char*>(d.c), sizeof(d.c));
    k.append(reinterpret_cast<const char*>(&d.tab_L), sizeof(d.tab_L));
    return k;
}

int alloc_arena(std::vector<DevInst>& insts, hipStream_t st, Arena& a, DevInst** d_insts) {
    const size_t n = insts.size();
    size_t off = align256(n * sizeof(DevInst));
    std::map<std::string, size_t> tables;
    std::vector<size_t> tab_off(n);
    for (size_t i = 0; i < n; ++i) {
        auto it = tables.find(table_key(insts[i]));
        if (it != tables.end()) {
            tab_off[i] = it->second;
            insts[i].tab_owner = 0;
        } else {
            tab_off[i] = off;
            tables.emplace(table_key(insts[i]), off);
            insts[i].tab_owner = 1;
            off = align256(off + (size_t)kMaxM * insts[i].tab_L * sizeof(double));
        }
    }
    std::vector<size_t> acc_off(n), x_off(n), s_off(n), sp_off(n);
    for (size_t i = 0; i < n; ++i) {
        acc_off[i] = off;
        off = align256(off + kAccLen * sizeof(double));
        sp_off[i] = off;
        off = align256(off + kSpillCap * sizeof(SpillSlot));
        x_off[i] = off;
        off = align256(off + 2 * (size_t)insts[i].R * kMaxS * sizeof(int32_t));
        s_off[i] = off;
        off = align256(off + (size_t)insts[i].R * 4 * sizeof(uint64_t));
    }
    hipError_t e = hipMallocAsync(&a.base, off, st);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync");
    a.bytes = off;
    char* b = static_cast<char*>(a.base);
    for (size_t i = 0; i < n; ++i) {
        insts[i].tab = reinterpret_cast<double*>(b + tab_off[i]);
        insts[i].acc = reinterpret_cast<double*>(b + acc_off[i]);
        insts[i].spill = reinterpret_cast<SpillSlot*>(b + sp_off[i]);
        insts[i].xbuf = reinterpret_cast<int32_t*>(b + x_off[i]);
        insts[i].sbuf = reinterpret_cast<uint64_t*>(b + s_off[i]);
    }
    *d_insts = reinterpret_cast<DevInst*>(b);
    e = hipMemcpyAsync(b, insts.data(), n * sizeof(DevInst), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        (void)hipFreeAsync(a.base, st);
        return hip_fail(e, "hipMemcpyAsync");
    }
    return PARREP_OK;
}

int set_device(parrep_ctx* ctx) {
    hipError_t e = hipSetDevice(ctx->device);
    return e == hipSuccess ? PARREP_OK : hip_fail(e, "hipSetDevice");
}

int run_instances(parrep_ctx* ctx, std::vector<DevInst>& insts, LaunchShape shape, int mode,
                  uint32_t hook_cycle, int64_t hook_max_rounds, hipStream_t st,
                  hipEvent_t ev_before = nullptr, hipEvent_t ev_after = nullptr) {
    if (!shape_supported(shape))
        return fail(PARREP_EUNSUPPORTED, "launch shape not compiled in");
    int rc = set_device(ctx);
    if (rc) return rc;
    Arena a;
    DevInst* d = nullptr;
    rc = alloc_arena(insts, st, a, &d);
    if (rc) return rc;
    const int n = (int)insts.size();
    int max_L = 1, max_m = 1;
    for (const DevInst& di : insts) {
        max_L = std::max(max_L, di.tab_L);
        max_m = std::max(max_m, (int)di.net.n_reactions);
    }
    shape.m = max_m;
    const int tab_Ls = table_lds_states(shape, max_L);
    hipError_t e = launch_setup(d, n, st);
    if (e == hipSuccess && mode == kModeSolve) e = launch_zero(d, n, st);
    if (e == hipSuccess && ev_before) e = hipEventRecord(ev_before, st);
    if (e == hipSuccess)
        e = launch_solve(d, n, shape, mode, hook_cycle, hook_max_rounds, tab_Ls, st);
    if (e == hipSuccess && ev_after) e = hipEventRecord(ev_after, st);
    if (e == hipSuccess && mode == kModeSolve) e = launch_finalize(d, n, st);
    hipError_t ef = hipFreeAsync(a.base, st);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    if (ef != hipSuccess) return hip_fail(ef, "hipFreeAsync");
    return PARREP_OK;
}

int check_result(const parrep_result* r) {
    if (!r || !r->hist || !r->hist_window || !r->stats || !r->counters || !r->x_final)
        return fail(PARREP_EINVAL, "result buffers hist, hist_window, stats, counters and "
                                   "x_final are required");
    if (r->cycle_log_cap < 0) return fail(PARREP_EINVAL, "cycle_log_cap < 0");
    return PARREP_OK;
}

void attach_result(DevInst& d, const parrep_result* r) {
    d.hist = r->hist;
    d.hist_w = r->hist_window;
    d.stats = r->stats;
    d.x_final = r->x_final;
    d.counters = r->counters;
    d.cycle_log = r->cycle_log_cap > 0 ? r->cycle_log : nullptr;
    d.cycle_log_cap = r->cycle_log_cap;
    d.phase_clock = r->phase_clock;
}

}  // namespace

extern "C" {

const char* parrep_last_error(void) { return g_err.c_str(); }

double parrep_wall_clock_hz(parrep_ctx* ctx) {
    if (!ctx || set_device(ctx)) return 0.0;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess)
        return 0.0;
    return 1e3 * khz;
}

int parrep_ctx_create(int device, parrep_ctx** out) {
    if (!out) return fail(PARREP_EINVAL, "out is NULL");
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return fail(PARREP_EDEVICE, "no such device");
    parrep_ctx* c = new (std::nothrow) parrep_ctx();
    if (!c) return fail(PARREP_ENOMEM, "context allocation");
    c->device = device;
    double host_tab[kLogTabLen];
    build_log_table(host_tab);
    int prev = 0;
    e = hipGetDevice(&prev);
    if (e == hipSuccess) e = hipSetDevice(device);
    if (e == hipSuccess) e = hipMalloc(&c->logtab, sizeof(host_tab));
    if (e == hipSuccess) e = hipMemcpy(c->logtab, host_tab, sizeof(host_tab), hipMemcpyHostToDevice);
    hipSetDevice(prev);
    if (e != hipSuccess) {
        if (c->logtab) hipFree(c->logtab);
        delete c;
        return hip_fail(e, "context table upload");
    }
    *out = c;
    return PARREP_OK;
}

void parrep_ctx_destroy(parrep_ctx* ctx) {
    if (!ctx) return;
    if (ctx->logtab) {
        int prev = 0;
        if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(ctx->device) == hipSuccess) {
            hipFree(ctx->logtab);
            hipSetDevice(prev);
        }
    }
    delete ctx;
}

int parrep_net_create(parrep_ctx* ctx, int32_t n_species, int32_t n_reactions, int32_t n_params,
                      const parrep_reaction* rx, parrep_net** out) {
    if (!ctx || !rx || !out) return fail(PARREP_EINVAL, "NULL argument");
    if (n_species < 1 || n_species > kMaxS) return fail(PARREP_EINVAL, "n_species out of range");
    if (n_reactions < 1 || n_reactions > kMaxM)
        return fail(PARREP_EINVAL, "n_reactions out of range");
    if (n_params < 0 || n_params > kMaxP) return fail(PARREP_EINVAL, "n_params out of range");
    parrep_net* net = new (std::nothrow) parrep_net();
    if (!net) return fail(PARREP_ENOMEM, "net allocation");
    net->ctx = ctx;
    DevNet& N = net->net;
    std::memset(&N, 0, sizeof(N));
    N.n_species = n_species;
    N.n_reactions = n_reactions;
    N.n_params = n_params;
    for (int j = 0; j < n_reactions; ++j) {
        const parrep_reaction& r = rx[j];
        DevReaction& d = N.rx[j];
        if (r.rate_param < -1 || r.rate_param >= n_params || r.n_factors < 0 ||
            r.n_factors > kMaxF || !finite_nonneg(r.kappa)) {
            delete net;
            return fail(PARREP_EINVAL, "reaction " + std::to_string(j) + ": bad rate definition");
        }
        d.rate_param = r.rate_param;
        d.n_factors = r.n_factors;
        d.kappa = r.kappa;
        for (int i = 0; i < kMaxS; ++i) {
            d.stoich[i] = i < n_species ? r.stoich[i] : 0;
            if (d.stoich[i] < -128 || d.stoich[i] > 127) {
                delete net;
                return fail(PARREP_EINVAL, "stoichiometric coefficients must be in [-128, 127]");
            }
        }
        for (int f = 0; f < r.n_factors; ++f) {
            const parrep_factor& q = r.factor[f];
            bool ok = q.species >= 0 && q.species < n_species;
            if (q.kind == PARREP_FALLING) ok = ok && q.order >= 0 && q.order <= 8;
            else if (q.kind == PARREP_HILL_REP)
                ok = ok && q.hill_param >= 0 && q.hill_param < n_params && std::isfinite(q.K) &&
                     q.K > 0.0;
            else ok = false;
            if (!ok) {
                delete net;
                return fail(PARREP_EINVAL, "reaction " + std::to_string(j) + ": bad factor");
            }
            d.f[f].kind = q.kind;
            d.f[f].species = q.species;
            d.f[f].order = q.kind == PARREP_FALLING ? q.order : 0;
            d.f[f].hill_param = q.kind == PARREP_HILL_REP ? q.hill_param : 0;
            d.f[f].K = q.kind == PARREP_HILL_REP ? q.K : 1.0;
        }
    }
    *out = net;
    return PARREP_OK;
}

void parrep_net_destroy(parrep_net* net) { delete net; }

int64_t parrep_problem_nbins(const parrep_net* net, const parrep_problem* prob) {
    if (!net || !prob) return fail(PARREP_EINVAL, "NULL argument");
    int64_t nb = 0;
    int rc = validate_problem(net, prob, &nb);
    return rc ? rc : nb;
}

int parrep_solve(parrep_ctx* ctx, const parrep_net* net, const parrep_problem* prob,
                 const parrep_result* res, void* stream) {
    return parrep_solve_batch(ctx, 1, &net, prob, res, nullptr, stream);
}

int parrep_solve_batch(parrep_ctx* ctx, int32_t count, const parrep_net* const* nets,
                       const parrep_problem* probs, const parrep_result* res,
                       const parrep_launch* launch, void* stream) {
    if (!ctx || !nets || !probs || !res) return fail(PARREP_EINVAL, "NULL argument");
    if (count < 1) return fail(PARREP_EINVAL, "count < 1");
    std::vector<DevInst> insts((size_t)count);
    int maxR = 1, maxS = 1;
    for (int i = 0; i < count; ++i) {
        if (!nets[i]) return fail(PARREP_EINVAL, "NULL net");
        if (nets[i]->ctx != ctx) return fail(PARREP_EINVAL, "net was created in another context");
        int64_t nb = 0;
        int rc = validate_problem(nets[i], &probs[i], &nb);
        if (rc) return rc;
        rc = check_result(&res[i]);
        if (rc) return rc;
        fill_inst(insts[i], nets[i], &probs[i], nb);
        attach_result(insts[i], &res[i]);
        maxR = std::max(maxR, probs[i].R);
        maxS = std::max(maxS, (int)nets[i]->net.n_species);
    }
    LaunchShape shape = choose_shape(maxR, maxS, kMaxM);
    hipEvent_t ev_b = launch ? (hipEvent_t)launch->event_before : nullptr;
    hipEvent_t ev_a = launch ? (hipEvent_t)launch->event_after : nullptr;
    if (launch && (launch->replicas_per_lane > 0 || launch->waves > 0)) {
        shape.rpl = launch->replicas_per_lane > 0 ? launch->replicas_per_lane : shape.rpl;
        shape.waves = launch->waves > 0 ? launch->waves : shape.waves;
        if ((int64_t)shape.rpl * shape.waves * 64 < maxR)
            return fail(PARREP_EINVAL, "launch shape holds fewer replicas than R");
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    return run_instances(ctx, insts, shape, kModeSolve, 0, -1, (hipStream_t)stream, ev_b, ev_a);
}

int parrep_philox(parrep_ctx* ctx, int64_t n, const uint32_t* ctr_key, uint32_t* out,
                  void* stream) {
    if (!ctx || n < 0 || (n > 0 && (!ctr_key || !out))) return fail(PARREP_EINVAL, "bad argument");
    int rc = set_device(ctx);
    if (rc) return rc;
    hipError_t e = launch_philox(n, ctr_key, out, (hipStream_t)stream);
    return e == hipSuccess ? PARREP_OK : hip_fail(e, "philox launch");
}

int parrep_events(parrep_ctx* ctx, const parrep_net* net, const double* c_host, int64_t n,
                  const int32_t* states, const uint32_t* blocks, double* a0, double* tau,
                  int32_t* J, void* stream) {
    if (!ctx || !net || !c_host || n < 0 || (n > 0 && (!states || !blocks || !a0 || !tau || !J)))
        return fail(PARREP_EINVAL, "bad argument");
    if (net->ctx != ctx) return fail(PARREP_EINVAL, "net was created in another context");
    parrep_problem p;
    std::memset(&p, 0, sizeof(p));
    for (int k = 0; k < net->net.n_params; ++k) p.c[k] = c_host[k];
    p.R = 1;
    p.T = 1.0;
    for (int i = 0; i < net->net.n_species; ++i) p.hist_hi[i] = 0;
    int64_t nb = 0;
    int rc = validate_problem(net, &p, &nb);
    if (rc) return rc;
    std::vector<DevInst> insts(1);
    fill_inst(insts[0], net, &p, nb);
    insts[0].tab_L = 1024;  // the hook stages states below 512; the rest take the formula path
    rc = set_device(ctx);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    Arena a;
    DevInst* d = nullptr;
    rc = alloc_arena(insts, st, a, &d);
    if (rc) return rc;
    hipError_t e = launch_setup(d, 1, st);
    if (e == hipSuccess) e = launch_events(d, n, states, blocks, a0, tau, J, st);
    hipError_t ef = hipFreeAsync(a.base, st);
    if (e != hipSuccess) return hip_fail(e, "events launch");
    return ef == hipSuccess ? PARREP_OK : hip_fail(ef, "hipFreeAsync");
}

int parrep_dephase_only(parrep_ctx* ctx, const parrep_net* net, const parrep_problem* prob,
                        const int32_t* xt, uint32_t cycle, int32_t* Y_out, int64_t* rounds_out,
                        void* stream) {
    if (!ctx || !net || !prob || !xt || !Y_out || !rounds_out)
        return fail(PARREP_EINVAL, "NULL argument");
    if (net->ctx != ctx) return fail(PARREP_EINVAL, "net was created in another context");
    int64_t nb = 0;
    int rc = validate_problem(net, prob, &nb);
    if (rc) return rc;
    std::vector<DevInst> insts(1);
    fill_inst(insts[0], net, prob, nb);
    for (int i = 0; i < net->net.n_species; ++i) insts[0].x0[i] = xt[i];
    insts[0].hook_states = Y_out;
    insts[0].hook_i64 = rounds_out;
    std::lock_guard<std::mutex> lk(ctx->mu);
    return run_instances(ctx, insts, choose_shape(prob->R, net->net.n_species, net->net.n_reactions), kModeDephaseOnly,
                         cycle, -1, (hipStream_t)stream);
}

int parrep_parallel_only(parrep_ctx* ctx, const parrep_net* net, const parrep_problem* prob,
                         const int32_t* init, uint32_t cycle, int64_t max_rounds,
                         int64_t* out_i64, int32_t* exit_state, double* credited, void* stream) {
    if (!ctx || !net || !prob || !init || !out_i64 || !exit_state || !credited)
        return fail(PARREP_EINVAL, "NULL argument");
    if (net->ctx != ctx) return fail(PARREP_EINVAL, "net was created in another context");
    int64_t nb = 0;
    int rc = validate_problem(net, prob, &nb);
    if (rc) return rc;
    std::vector<DevInst> insts(1);
    fill_inst(insts[0], net, prob, nb);
    insts[0].hook_states = const_cast<int32_t*>(init);  // read only by the kernel
    insts[0].hook_exit = exit_state;
    insts[0].hook_i64 = out_i64;
    insts[0].hook_f64 = credited;
    std::lock_guard<std::mutex> lk(ctx->mu);
    return run_instances(ctx, insts, choose_shape(prob->R, net->net.n_species, net->net.n_reactions), kModeParallelOnly,
                         cycle, max_rounds, (hipStream_t)stream);
}

}  // extern "C"
