// parrep_api.hip -- the C ABI of libparrep (declared in include/parrep.h and
// include/parrep_estimate.h):
// argument validation, device descriptors, scratch, and kernel launches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/parrep_estimate.h"
#include "parrep_host.h"
#include "parrep_neglog.h"

using namespace parrep;

// Scratch of parrep_solve_noalloc: one fixed array per device, held until the
// process ends.  Host code never uses this name as an address (on the host
// it is only a stand-in for the symbol): the device address comes from
// hipGetSymbolAddress, once per device, in noalloc_scratch().
static __device__ __align__(256) char scratch[PARREP_NOALLOC_SCRATCH_BYTES];

namespace parrep {
namespace host {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return PARREP_EDEVICE;
}

namespace {
bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }
}  // namespace

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
            } else if (N.rx[j].f[f].kind == PARREP_HILL_SWITCH) {
                const double K = p->c[N.rx[j].f[f].param3];
                if (!(K > 0.0) || !std::isfinite(K))
                    return fail(PARREP_EINVAL, "switch scales must be positive");
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
    d.stage_flush = -1;
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
    // Hot-path view (kinds described with kRxConst..kRxFall): parameter
    // factors are part of the rate constant; the first state factor indexes
    // a table unless it is a falling factorial of order <= 2 (outside the
    // narrow kernels), and a second state factor is taken as a tail when it
    // is such a falling factorial; anything else takes the formula.
    const bool narrow = narrow_kernel(n, d.net.n_reactions);
    for (int j = 0; j < kMaxM; ++j) {
        const DevReaction& r = d.net.rx[j];
        int st[kMaxF], nstate = 0;
        for (int f = 0; j < d.net.n_reactions && f < r.n_factors; ++f)
            if (r.f[f].kind != PARREP_PARAM) st[nstate++] = f;
        auto small_fall = [&](int f) {
            return r.f[f].kind == PARREP_FALLING && r.f[f].order >= 1 && r.f[f].order <= 2;
        };
        uint32_t meta = jmeta_pack(kRxConst, 0, 0, 0, 0);
        if (nstate >= 1) {
            const DevFactor& f0 = r.f[st[0]];
            const bool tail = nstate == 2 && !narrow && small_fall(st[1]);
            const uint32_t ts = tail ? (uint32_t)r.f[st[1]].species : 0u;
            const uint32_t to = tail ? (uint32_t)r.f[st[1]].order : 0u;
            if (nstate > 2 || (nstate == 2 && !tail))
                meta = jmeta_pack(kRxDirect, 0, 0, 0, 0);
            else if (!narrow && small_fall(st[0]))
                meta = jmeta_pack(kRxFall, (uint32_t)f0.species, (uint32_t)f0.order, ts, to);
            else
                meta = jmeta_pack(kRxTable, (uint32_t)f0.species, 0, ts, to);
        }
        d.jmeta[j] = meta;
        uint32_t packed = 0;
        for (int i = 0; i < kMaxS; ++i) packed |= ((uint32_t)(r.stoich[i] & 0xFF)) << (8 * i);
        d.jstoich[j] = packed;
    }
    // table states per species: the histogram box and the start, plus 64
    d.tab_L = 64;
    for (int i = 0; i < kMaxS; ++i) {
        const int hi = i < n ? std::max(p->hist_hi[i], p->x0[i]) : 0;
        d.tab_Lsp[i] = std::min(8192, std::max(64, ((hi + 64 + 63) / 64) * 64));
        d.tab_L = std::max(d.tab_L, d.tab_Lsp[i]);
    }
}

namespace {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Instances with the same network, rate vector and table length share one
// propensity table; the first of them fills it.
std::string table_key(const DevInst& d) {
    std::string k(reinterpret_cast<const char*>(&d.net), sizeof(d.net));
    k.append(reinterpret_cast<const char*>(d.c), sizeof(d.c));
    k.append(reinterpret_cast<const char*>(&d.tab_L), sizeof(d.tab_L));
    return k;
}

// Offsets of each instance's scratch inside the arena.
struct Layout {
    size_t total = 0;
    std::vector<size_t> tab, acc, spill, xbuf, sbuf, wide;
    std::vector<int> owner;
};

Layout layout(const std::vector<DevInst>& insts, bool share) {
    const size_t n = insts.size();
    Layout L;
    L.tab.resize(n);
    L.acc.resize(n);
    L.spill.resize(n);
    L.xbuf.resize(n);
    L.sbuf.resize(n);
    L.wide.resize(n);
    L.owner.resize(n);
    size_t off = align256(n * sizeof(DevInst));
    std::map<std::string, size_t> tables;
    for (size_t i = 0; i < n; ++i) {
        auto it = share ? tables.find(table_key(insts[i])) : tables.end();
        if (it != tables.end()) {
            L.tab[i] = it->second;
            L.owner[i] = 0;
        } else {
            L.tab[i] = off;
            tables.emplace(table_key(insts[i]), off);
            L.owner[i] = 1;
            off = align256(off + (size_t)kMaxM * insts[i].tab_L * sizeof(double));
        }
    }
    for (size_t i = 0; i < n; ++i) {
        L.acc[i] = off;
        off = align256(off + kAccLen * sizeof(double));
        L.spill[i] = off;
        off = align256(off + kSpillCap * sizeof(SpillSlot));
        L.xbuf[i] = off;
        off = align256(off + (size_t)insts[i].R * kMaxS * sizeof(int32_t));
        L.sbuf[i] = off;
        off = align256(off + (size_t)insts[i].R * 4 * sizeof(uint64_t));
        L.wide[i] = 0;
        if (insts[i].wide_waves > 0) {  // exchange area, per-wave sums, survivor words
            L.wide[i] = off;
            off = align256(off + sizeof(WideSync) + (size_t)insts[i].wide_waves * 16 +
                           (size_t)insts[i].wide_waves * insts[i].wide_rpl * 8);
        }
    }
    L.total = off;
    return L;
}

// Expected work of an instance, for longest-first ordering: replicas times
// horizon (the events of the dephasing and parallel steps scale with both).
double work_estimate(const DevInst& d) { return (double)d.R * d.T; }

}  // namespace

size_t arena_bytes(std::vector<DevInst>& insts, bool share) { return layout(insts, share).total; }

void place_arena(std::vector<DevInst>& insts, char* b, bool share) {
    const Layout L = layout(insts, share);
    for (size_t i = 0; i < insts.size(); ++i) {
        insts[i].tab = reinterpret_cast<double*>(b + L.tab[i]);
        insts[i].tab_owner = L.owner[i];
        insts[i].acc = reinterpret_cast<double*>(b + L.acc[i]);
        insts[i].spill = reinterpret_cast<SpillSlot*>(b + L.spill[i]);
        insts[i].xbuf = reinterpret_cast<int32_t*>(b + L.xbuf[i]);
        insts[i].sbuf = reinterpret_cast<uint64_t*>(b + L.sbuf[i]);
        if (insts[i].wide_waves > 0) {
            char* w = b + L.wide[i];
            insts[i].wide = reinterpret_cast<WideSync*>(w);
            insts[i].wtot = reinterpret_cast<uint64_t*>(w + sizeof(WideSync));
            insts[i].smask = reinterpret_cast<uint64_t*>(w + sizeof(WideSync) +
                                                         (size_t)insts[i].wide_waves * 16);
        } else {
            insts[i].wide = nullptr;
            insts[i].wtot = insts[i].smask = nullptr;
        }
    }
}

// Device address of `scratch` on `device`, which must be current; looked up
// once per device.
int noalloc_scratch(int device, char** out) {
    static std::mutex mu;
    static std::map<int, char*> addr;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(device);
    if (it == addr.end()) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        it = addr.emplace(device, static_cast<char*>(p)).first;
    }
    *out = it->second;
    return PARREP_OK;
}

int set_device(parrep_ctx* ctx) {
    hipError_t e = hipSetDevice(ctx->device);
    return e == hipSuccess ? PARREP_OK : hip_fail(e, "hipSetDevice");
}

int shape_bucket(int R) {
    int b = 64;
    while (b < R) b <<= 1;
    return b;
}

LaunchShape pick_shape(parrep_ctx* ctx, int R, int ns, int m, bool sparse) {
    const int nsc = ns <= 1 ? 1 : (ns <= 2 ? 2 : 4);
    const int mc = m <= 4 ? 4 : 8;
    // A batch that leaves CUs idle is bound by the latency of one event:
    // one replica per lane over several waves beats stacking replicas.
    if (sparse && R > 64 && R <= 256) return LaunchShape{1, 4, nsc, mc};
    auto it = ctx->tuned.find(std::make_tuple(shape_bucket(R), nsc, mc));
    if (it != ctx->tuned.end()) {
        LaunchShape s{std::get<0>(it->second), std::get<1>(it->second), nsc, mc};
        s.stage_flush = std::get<2>(it->second);
        if ((int64_t)s.rpl * s.waves * 64 >= R) return s;
    }
    return choose_shape(R, nsc, mc);
}

std::vector<Group> group_batch(parrep_ctx* ctx, std::vector<DevInst>& insts,
                               std::vector<int>* order, const LaunchShape* forced, bool persist) {
    const int n = (int)insts.size();
    std::vector<LaunchShape> sh(n);
    for (int i = 0; i < n; ++i) {
        const DevInst& d = insts[i];
        if (forced) {
            sh[i] = *forced;
            sh[i].ns = d.net.n_species <= 1 ? 1 : (d.net.n_species <= 2 ? 2 : 4);
            sh[i].m = d.net.n_reactions <= 4 ? 4 : 8;
        } else {
            sh[i] = pick_shape(ctx, d.R, d.net.n_species, d.net.n_reactions, n <= ctx->n_cu);
        }
    }
    auto key = [&](int i) { return std::make_tuple(sh[i].ns, sh[i].m, sh[i].rpl, sh[i].waves); };
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
        if (key(a) != key(b)) return key(a) < key(b);
        return work_estimate(insts[a]) > work_estimate(insts[b]);
    });
    std::vector<DevInst> sorted(n);
    for (int i = 0; i < n; ++i) sorted[i] = insts[ord[i]];
    insts.swap(sorted);
    std::vector<Group> groups;
    for (int i = 0; i < n; ++i) {
        const LaunchShape& s = sh[ord[i]];
        if (groups.empty() || key(ord[i]) != key(ord[groups.back().first])) {
            groups.push_back(Group{s, i, 0, 0});
        }
        groups.back().count += 1;
    }
    for (Group& g : groups) {
        // staging applies to the narrow kernels with at most 4 replicas per
        // lane and at most 4 waves
        if (!narrow_kernel(g.shape.ns, g.shape.m) || g.shape.rpl > 4 || g.shape.waves > 4)
            g.shape.stage_flush = -1;
        // a compiled specialisation when every instance of the group fits
        // it: the species-map kernel (its fixed-stride tables must also fit
        // the LDS budget) or the network-descriptor kernel
        g.shape.spec = -1;
        const bool nk = narrow_kernel(g.shape.ns, g.shape.m);
        auto spec_of = [&](const DevInst& d) -> long long {
            return nk ? (long long)species_map(d, g.shape) : network_desc(d, g.shape);
        };
        long long spec = spec_of(insts[g.first]);
        for (int i = g.first; i < g.first + g.count && spec >= 0; ++i)
            if (spec_of(insts[i]) != spec) spec = -1;
        if (spec >= 0 && nk) {
            LaunchShape t = g.shape;
            t.spec = spec;
            const int need = table_lds_need(insts[g.first], t);
            if (table_lds_doubles(t, need) < need) spec = -1;
        }
        g.shape.spec = spec;
        // the persistent form, when asked for (not with staging)
        g.shape.persist = persist && g.shape.stage_flush < 0 ? 1 : 0;
        int need = 0;
        for (int i = g.first; i < g.first + g.count; ++i) {
            need = std::max(need, table_lds_need(insts[i], g.shape));
            insts[i].stage_flush = g.shape.stage_flush;
        }
        g.tab_lds = table_lds_doubles(g.shape, need);
    }
    if (order) *order = ord;
    return groups;
}

int enqueue_batch(parrep_ctx* ctx, DevInst* d, int n, const std::vector<Group>& groups, int mode,
                  uint32_t hook_cycle, int64_t hook_max_rounds, hipStream_t st, hipEvent_t ev_b,
                  hipEvent_t ev_a, std::vector<hipEvent_t>* keep) {
    for (const Group& g : groups)
        if (!shape_supported(g.shape))
            return fail(PARREP_EUNSUPPORTED, "launch shape not compiled in");
    hipError_t e = launch_setup(d, n, st);
    if (e == hipSuccess && mode == kModeSolve) e = launch_zero(d, n, st);
    if (e == hipSuccess && ev_b) e = hipEventRecord(ev_b, st);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    if (groups.size() == 1) {
        const Group& g = groups[0];
        if (g.shape.wide)
            e = launch_wide(d + g.first, g.shape, g.tab_lds, st);
        else
            e = launch_solve(d + g.first, g.count, g.shape, mode, hook_cycle, hook_max_rounds,
                             g.tab_lds, st);
    } else {
        // Fork: group 0 on st, the others on auxiliary streams; join into st.
        while (ctx->aux.size() + 1 < groups.size()) {
            hipStream_t s = nullptr;
            e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
            ctx->aux.push_back(s);
        }
        hipEvent_t fork = nullptr;
        e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(fork, st);
        std::vector<hipEvent_t> joins(groups.size() - 1, nullptr);
        for (size_t k = 0; e == hipSuccess && k < groups.size(); ++k) {
            const Group& g = groups[k];
            hipStream_t s = k == 0 ? st : ctx->aux[k - 1];
            if (k > 0) e = hipStreamWaitEvent(s, fork, 0);
            if (e == hipSuccess)
                e = launch_solve(d + g.first, g.count, g.shape, mode, hook_cycle,
                                 hook_max_rounds, g.tab_lds, s);
            if (e == hipSuccess && k > 0) {
                e = hipEventCreateWithFlags(&joins[k - 1], hipEventDisableTiming);
                if (e == hipSuccess) e = hipEventRecord(joins[k - 1], s);
                if (e == hipSuccess) e = hipStreamWaitEvent(st, joins[k - 1], 0);
            }
        }
        if (keep) {
            keep->push_back(fork);
            for (hipEvent_t j : joins) keep->push_back(j);
        } else {
            if (fork) (void)hipEventDestroy(fork);
            for (hipEvent_t j : joins)
                if (j) (void)hipEventDestroy(j);
        }
    }
    if (e == hipSuccess && ev_a) e = hipEventRecord(ev_a, st);
    if (e == hipSuccess && mode == kModeSolve) e = launch_finalize(d, n, st);
    return e == hipSuccess ? PARREP_OK : hip_fail(e, "kernel launch");
}

int apply_wide(parrep_ctx* ctx, std::vector<DevInst>& insts, std::vector<Group>& groups,
               const WideReq& w) {
    if (insts.size() != 1 || groups.size() != 1 || w.workgroups == 1) return PARREP_OK;
    DevInst& d = insts[0];
    const int rpl = w.rpl > 0 ? w.rpl : 1;
    if (rpl != 1 && rpl != 4) return fail(PARREP_EINVAL, "spread instances take 1 or 4 replicas per lane");
    const int need = (d.R + 256 * rpl - 1) / (256 * rpl);
    int G = 0;
    if (w.workgroups > 1) {
        if (w.workgroups < need)
            return fail(PARREP_EINVAL, "workgroups x 256 lanes x replicas per lane < R");
        G = w.workgroups;
    } else if (d.R >= kWideMinR) {
        G = need;
    }
    if (G < 2) return PARREP_OK;
    if ((int64_t)G * 256 * rpl > PARREP_MAX_REPLICAS + 256 * rpl - 1)
        return fail(PARREP_EINVAL, "more workgroups than the replica capacity needs");
    if (w.s3 > kWideS3Max) return fail(PARREP_EINVAL, "parallel-step chunk longer than 64 rounds");
    Group& g = groups[0];
    g.shape.rpl = rpl;
    g.shape.waves = 4;
    g.shape.wide = G;
    g.shape.spec = -1;
    g.shape.persist = 0;
    g.tab_lds = table_lds_doubles(g.shape, table_lds_need(d, g.shape));
    d.wide_waves = 4 * G;
    d.wide_rpl = rpl;
    d.wide_s2 = w.s2 > 0 ? w.s2 : kWideChunkS2;
    d.wide_s3 = w.s3 > 0 ? w.s3 : kWideChunkS3;
    const double wait_s = (w.wait_us > 0 ? w.wait_us : 2000000) * 1e-6;
    d.wide_wait_ticks = std::max<int64_t>(1, (int64_t)(wait_s * ctx->wall_hz));
    return PARREP_OK;
}

int run_batch(parrep_ctx* ctx, std::vector<DevInst>& insts, int mode, uint32_t hook_cycle,
              int64_t hook_max_rounds, hipStream_t st, hipEvent_t ev_b, hipEvent_t ev_a,
              const LaunchShape* forced, const WideReq* wide) {
    int rc = set_device(ctx);
    if (rc) return rc;
    std::vector<Group> groups =
        group_batch(ctx, insts, nullptr, forced, mode == kModeSolve && wide && wide->persist);
    if (mode == kModeSolve) {
        rc = apply_wide(ctx, insts, groups, wide ? *wide : WideReq{});
        if (rc) return rc;
    }
    const size_t bytes = arena_bytes(insts);
    void* base = nullptr;
    hipError_t e = hipMallocAsync(&base, bytes, st);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync");
    place_arena(insts, static_cast<char*>(base));
    e = hipMemcpyAsync(base, insts.data(), insts.size() * sizeof(DevInst), hipMemcpyHostToDevice,
                       st);
    if (e != hipSuccess) {
        (void)hipFreeAsync(base, st);
        return hip_fail(e, "hipMemcpyAsync");
    }
    rc = enqueue_batch(ctx, static_cast<DevInst*>(base), (int)insts.size(), groups, mode,
                       hook_cycle, hook_max_rounds, st, ev_b, ev_a);
    hipError_t ef = hipFreeAsync(base, st);
    if (rc) return rc;
    return ef == hipSuccess ? PARREP_OK : hip_fail(ef, "hipFreeAsync");
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

}  // namespace host
}  // namespace parrep

using namespace parrep::host;

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
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount,
                                                   device);
    int wall_khz = 0;
    if (e == hipSuccess &&
        hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, device) == hipSuccess &&
        wall_khz > 0)
        c->wall_hz = 1e3 * wall_khz;
    if (e == hipSuccess) e = hipMalloc(&c->logtab, sizeof(host_tab));
    if (e == hipSuccess) e = hipMemcpy(c->logtab, host_tab, sizeof(host_tab), hipMemcpyHostToDevice);
    int rc = e == hipSuccess ? noalloc_scratch(device, &c->noalloc_scratch)
                             : hip_fail(e, "context table upload");
    if (rc != PARREP_OK && c->logtab) (void)hipFree(c->logtab);
    (void)hipSetDevice(prev);
    if (rc != PARREP_OK) {
        delete c;
        return rc;
    }
    *out = c;
    return PARREP_OK;
}

void parrep_ctx_destroy(parrep_ctx* ctx) {
    if (!ctx) return;
    int prev = 0;
    if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(ctx->device) == hipSuccess) {
        for (hipStream_t s : ctx->aux) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
        if (ctx->logtab) (void)hipFree(ctx->logtab);
        (void)hipSetDevice(prev);
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
            auto par = [&](int32_t i) { return i >= 0 && i < n_params; };
            if (q.kind == PARREP_FALLING) ok = ok && q.order >= 0 && q.order <= 8;
            else if (q.kind == PARREP_HILL_SWITCH)
                ok = ok && q.order >= 1 && q.order <= 8 && par(q.hill_param) && par(q.param2) &&
                     par(q.param3);
            else if (q.kind == PARREP_PARAM)
                ok = par(q.hill_param);
            else if (q.kind == PARREP_HILL_REP)
                ok = ok && q.hill_param >= 0 && q.hill_param < n_params && std::isfinite(q.K) &&
                     q.K > 0.0;
            else ok = false;
            if (!ok) {
                delete net;
                return fail(PARREP_EINVAL, "reaction " + std::to_string(j) + ": bad factor");
            }
            d.f[f].kind = q.kind;
            d.f[f].species = q.kind == PARREP_PARAM ? 0 : q.species;
            d.f[f].order = (q.kind == PARREP_FALLING || q.kind == PARREP_HILL_SWITCH) ? q.order : 0;
            d.f[f].hill_param = q.kind == PARREP_FALLING ? 0 : q.hill_param;
            d.f[f].param2 = q.kind == PARREP_HILL_SWITCH ? q.param2 : 0;
            d.f[f].param3 = q.kind == PARREP_HILL_SWITCH ? q.param3 : 0;
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
    hipEvent_t ev_b = launch ? (hipEvent_t)launch->event_before : nullptr;
    hipEvent_t ev_a = launch ? (hipEvent_t)launch->event_after : nullptr;
    LaunchShape forced{};
    const bool spread = launch && launch->workgroups > 1;
    if (launch && (launch->histogram_staging < -1 || launch->histogram_staging > 1 ||
                   launch->flush_period < 0))
        return fail(PARREP_EINVAL, "histogram_staging must be -1, 0 or 1 and flush_period >= 0");
    const bool force = !spread && launch &&
                       (launch->replicas_per_lane > 0 || launch->waves > 0 ||
                        launch->histogram_staging != 0);
    if (force) {
        forced = choose_shape(maxR, maxS, kMaxM);
        forced.rpl = launch->replicas_per_lane > 0 ? launch->replicas_per_lane : forced.rpl;
        forced.waves = launch->waves > 0 ? launch->waves : forced.waves;
        forced.stage_flush = launch->histogram_staging > 0 ? std::max(0, launch->flush_period) : -1;
        if ((int64_t)forced.rpl * forced.waves * 64 < maxR)
            return fail(PARREP_EINVAL, "launch shape holds fewer replicas than R");
        if (!shape_supported(forced)) return fail(PARREP_EUNSUPPORTED, "launch shape not compiled in");
    }
    WideReq wide;
    if (launch) {
        if (launch->workgroups < 0 || launch->chunk_rounds[0] < 0 || launch->chunk_rounds[1] < 0 ||
            launch->barrier_wait_us < 0)
            return fail(PARREP_EINVAL, "negative workgroups, chunk length or wait");
        wide.workgroups = launch->workgroups;
        // a forced one-workgroup shape stays one workgroup unless spreading is asked for
        if (force && launch->workgroups == 0) wide.workgroups = 1;
        if (launch->workgroups > 1) {
            if (count != 1) return fail(PARREP_EINVAL, "only a single-instance batch is spread over workgroups");
            wide.rpl = launch->replicas_per_lane;
            if (launch->waves != 0 && launch->waves != 4)
                return fail(PARREP_EINVAL, "spread instances run 4 waves per workgroup");
        }
        wide.s2 = launch->chunk_rounds[0];
        wide.s3 = launch->chunk_rounds[1];
        wide.wait_us = launch->barrier_wait_us;
        if (launch->persistent < 0 || launch->persistent > 1)
            return fail(PARREP_EINVAL, "persistent must be 0 or 1");
        wide.persist = launch->persistent;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    return run_batch(ctx, insts, kModeSolve, 0, -1, (hipStream_t)stream, ev_b, ev_a,
                     force ? &forced : nullptr, &wide);
}

int parrep_solve_noalloc(parrep_ctx* ctx, const parrep_net* net, const parrep_problem* prob,
                         const parrep_result* res, void* stream) {
    if (!ctx || !net || !prob || !res) return fail(PARREP_EINVAL, "NULL argument");
    if (net->ctx != ctx) return fail(PARREP_EINVAL, "net was created in another context");
    int64_t nb = 0;
    int rc = validate_problem(net, prob, &nb);
    if (rc) return rc;
    rc = check_result(res);
    if (rc) return rc;
    std::vector<DevInst> insts(1);
    fill_inst(insts[0], net, prob, nb);
    attach_result(insts[0], res);
    std::lock_guard<std::mutex> lk(ctx->mu);
    rc = set_device(ctx);
    if (rc) return rc;
    if (!ctx->noalloc_scratch) return fail(PARREP_EDEVICE, "no scratch array on this device");
    const std::vector<Group> groups = group_batch(ctx, insts, nullptr, nullptr);
    const size_t bytes = arena_bytes(insts);
    if (bytes > PARREP_NOALLOC_SCRATCH_BYTES)
        return fail(PARREP_EINVAL, "the problem needs " + std::to_string(bytes) +
                                       " bytes of scratch; the fixed array holds " +
                                       std::to_string(PARREP_NOALLOC_SCRATCH_BYTES));
    char* base = ctx->noalloc_scratch;
    place_arena(insts, base);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = launch_install(insts[0], reinterpret_cast<DevInst*>(base), st);
    if (e != hipSuccess) return hip_fail(e, "descriptor install");
    return enqueue_batch(ctx, reinterpret_cast<DevInst*>(base), 1, groups, kModeSolve, 0, -1, st,
                         nullptr, nullptr);
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
    // the hook stages 4096 doubles of table in LDS; other states take the formula
    for (int i = 0; i < kMaxS; ++i) insts[0].tab_Lsp[i] = 1024;
    insts[0].tab_L = 1024;
    rc = set_device(ctx);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    void* base = nullptr;
    hipError_t e = hipMallocAsync(&base, arena_bytes(insts), st);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync");
    place_arena(insts, static_cast<char*>(base));
    e = hipMemcpyAsync(base, insts.data(), sizeof(DevInst), hipMemcpyHostToDevice, st);
    DevInst* d = static_cast<DevInst*>(base);
    if (e == hipSuccess) e = launch_setup(d, 1, st);
    if (e == hipSuccess) e = launch_events(d, n, states, blocks, a0, tau, J, st);
    hipError_t ef = hipFreeAsync(base, st);
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
    return run_batch(ctx, insts, kModeDephaseOnly, cycle, -1, (hipStream_t)stream, nullptr,
                     nullptr, nullptr);
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
    return run_batch(ctx, insts, kModeParallelOnly, cycle, max_rounds, (hipStream_t)stream,
                     nullptr, nullptr, nullptr);
}

int parrep_estimate(parrep_ctx* ctx, int32_t n_runs, const double* const* stats_ptrs,
                    int32_t n_params, int32_t n_species, double window, double* out,
                    void* stream) {
    if (!ctx || !stats_ptrs || !out) return fail(PARREP_EINVAL, "NULL argument");
    if (n_runs < 2) return fail(PARREP_EINVAL, "n_runs must be >= 2");
    if (n_params < 1 || n_params > kMaxP || n_species < 1 || n_species > kMaxS)
        return fail(PARREP_EINVAL, "n_params or n_species out of range");
    if (!(window > 0.0) || !std::isfinite(window))
        return fail(PARREP_EINVAL, "window must be positive and finite");
    for (int32_t r = 0; r < n_runs; ++r)
        if (!stats_ptrs[r]) return fail(PARREP_EINVAL, "NULL stats pointer");
    int rc = set_device(ctx);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    void* d_ptrs = nullptr;
    const size_t bytes = sizeof(double*) * (size_t)n_runs;
    hipError_t e = hipMallocAsync(&d_ptrs, bytes, st);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync");
    // from pageable host memory: staged before the call returns
    e = hipMemcpyAsync(d_ptrs, stats_ptrs, bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = launch_estimate(static_cast<const double* const*>(d_ptrs), n_runs, n_params,
                            n_species, window, out, st);
    hipError_t ef = hipFreeAsync(d_ptrs, st);
    if (e != hipSuccess) return hip_fail(e, "estimate launch");
    return ef == hipSuccess ? PARREP_OK : hip_fail(ef, "hipFreeAsync");
}

}  // extern "C"
