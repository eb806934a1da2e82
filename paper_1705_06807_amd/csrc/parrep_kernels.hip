// parrep_kernels.hip -- non-templated kernels of libparrep (accumulator
// zeroing, FIM/RER finalize, test hooks) and the instance-kernel dispatch.
#include "parrep_device.h"
#include "../../include/parrep_estimate.h"

namespace parrep {
namespace dev {

// ---------------------------------------------------------------------------
// Setup: rate constants k_j (c[rate_param] kappa times the parameter factors)
// of every instance, and the tables T_j[x_s] = k_j phi_1(x_s), x_s =
// 0..tab_L-1, of the table reactions (phi_1 the first state factor; the
// formula's own first steps, so a table entry times the tail is
// bit-identical to evaluating the formula at that state).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_setup(DevInst* __restrict__ insts) {
    __shared__ SNet S;
    DevInst* I = insts + blockIdx.x;
    if (threadIdx.x == 0) {
        load_net(S, I);
        for (int j = 0; j < kMaxM; ++j) {
            I->k[j] = S.k[j];
            for (int f = 0; f < kMaxF; ++f) I->hexp[j * kMaxF + f] = S.fhint[j][f];
        }
    }
    __syncthreads();
    if (!I->tab_owner) return;
    const int L = I->tab_L;
    const int m = S.m;
    for (int idx = threadIdx.x; idx < m * L; idx += blockDim.x) {
        const int j = idx / L;
        const int xs = idx - j * L;
        const uint32_t meta = I->jmeta[j];
        if ((meta & 3u) != kRxTable) continue;
        I->tab[idx] = prop_first(S, j, xs);
    }
}

// ---------------------------------------------------------------------------
// Install one descriptor, passed by value, at dst (the allocation-free solve
// writes its descriptor into fixed device memory without a host copy).
// ---------------------------------------------------------------------------
static_assert(sizeof(DevInst) % 8 == 0 && sizeof(DevInst) <= 3072,
              "a descriptor must fit a kernel argument");

__global__ void __launch_bounds__(64) k_install(DevInst d, DevInst* __restrict__ dst) {
    const uint64_t* src = reinterpret_cast<const uint64_t*>(&d);
    uint64_t* out = reinterpret_cast<uint64_t*>(dst);
    for (int i = threadIdx.x; i < (int)(sizeof(DevInst) / 8); i += 64) out[i] = src[i];
}

// ---------------------------------------------------------------------------
// Zero the accumulators of every instance.
// ---------------------------------------------------------------------------
__global__ void k_zero(const DevInst* __restrict__ insts) {
    const DevInst* I = insts + blockIdx.y;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = t0; i < I->nbins; i += stride) {
        I->hist[i] = 0.0;
        I->hist_w[i] = 0.0;
    }
    for (int64_t i = t0; i < kAccLen; i += stride) I->acc[i] = 0.0;
    for (int64_t i = t0; i < kSpillCap; i += stride) {
        I->spill[i].key = 0;
        I->spill[i].full = 0.0;
        I->spill[i].w = 0.0;
    }
    for (int64_t i = t0; i < PARREP_NSTATS; i += stride) I->stats[i] = 0.0;
    for (int64_t i = t0; i < PARREP_NCOUNTERS; i += stride) I->counters[i] = 0;
    if (I->cycle_log)
        for (int64_t i = t0; i < (int64_t)I->cycle_log_cap * PARREP_CYCLE_REC; i += stride)
            I->cycle_log[i] = 0;
    if (I->wide) {
        WideSync* ws = I->wide;
        if (t0 == 0) {
            ws->bar = 0;
            ws->abort = 0;
            ws->rend = -1;
            for (int q = 0; q < 3; ++q) {
                ws->e2[q] = INT64_MAX;
                ws->d2[q] = -1;
                ws->k3[q] = ~0ull;
            }
        }
        for (int64_t i = t0; i < 3 * kWideS3Max * 3; i += stride) (&ws->s3[0][0][0])[i] = 0;
    }
}

// ---------------------------------------------------------------------------
// Finalize: FIM, RER and window integrals from the window histogram
// (the integrands depend on the state only, so int F(X_s) ds over the
// window is sum_x hist_w(x) F(x)), plus the out-of-box accumulators.
// ---------------------------------------------------------------------------
// Finalize: hist += hist_w, then the window FIM, RER and integrals of every
// instance from its window histogram (and the spill slots), divided by the
// window length.  FIM(x) = sum_j lam_j g_j g_j^T with g_j = grad_c log lam_j
// and RER_k(x) = sum_j lam_j log(lam_j/lam'_j) - lam_j + lam'_j (Sec. III,
// Appendix A); the time integrals are sums over visited states, weighted by
// the window time spent there.  Specialised for up to NS species and NP
// parameters (so the per-thread accumulators stay in registers); each of the
// two launches skips the instances of the other.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

template <int NP>
struct WinAcc {
    double fim[NP * NP];
    double rer[NP];
    double y[kMaxS];
};

template <int NS, int NP>
__device__ void fim_rer_point(const SNet& S, const uint32_t* dep, const int (&x)[NS], double w,
                              WinAcc<NP>& A) {
    const int np = S.np;
    double lamv[kMaxM];
    for (int j = 0; j < S.m; ++j) lamv[j] = prop_with<NS>(S, j, x, S.c);
    for (int j = 0; j < S.m; ++j) {
        const double lam = lamv[j];
        if (!(lam > 0.0)) continue;
        double g[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) g[p] = 0.0;
        const int rp = S.rate_param[j];
#pragma unroll
        for (int p = 0; p < NP; ++p)
            if (p == rp) g[p] += 1.0 / S.c[rp];
        for (int f = 0; f < S.nf[j]; ++f) {
            const int kind = S.fkind[j][f];
            const int hp = S.fhp[j][f];
            if (kind == PARREP_PARAM) {
                const double d = 1.0 / S.c[hp];
#pragma unroll
                for (int p = 0; p < NP; ++p)
                    if (p == hp) g[p] += d;
            } else if (kind == PARREP_HILL_SWITCH) {
                // phi = lo + (hi - lo) s: d/dlo = 1 - s, d/dhi = s,
                // d/dK = -(hi - lo) n s (1 - s) / K, each over phi
                const int xs = pick<NS>(x, S.fsp[j][f]);
                const int p2 = S.fp2[j][f], p3 = S.fp3[j][f], n = S.ford[j][f];
                const double lo = S.c[hp], hi = S.c[p2], K = S.c[p3];
                const double phi = switch_val(xs, n, lo, hi, K);
                if (!(phi > 0.0)) continue;
                const double y = (double)xs / K;
                double q = y;
                for (int i = 1; i < n; ++i) q = q * y;
                const double sq = q / (1.0 + q);
                const double dlo = (1.0 - sq) / phi, dhi = sq / phi;
                const double dK = -(hi - lo) * n * sq * (1.0 - sq) / (K * phi);
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    if (p == hp) g[p] += dlo;
                    if (p == p2) g[p] += dhi;
                    if (p == p3) g[p] += dK;
                }
            } else if (kind == PARREP_HILL_REP) {
                const double y = (double)pick<NS>(x, S.fsp[j][f]) / S.fK[j][f];
                if (!(y > 0.0)) continue;
                const double q = hill_pow(y, S.fhint[j][f], S.c[hp]);
                const double d = -q * log(y) / (1.0 + q);
#pragma unroll
                for (int p = 0; p < NP; ++p)
                    if (p == hp) g[p] += d;
            }
        }
#pragma unroll
        for (int a = 0; a < NP; ++a)
#pragma unroll
            for (int bb = 0; bb < NP; ++bb)
                if (a < np && bb < np) A.fim[a * NP + bb] += w * (lam * g[a] * g[bb]);
    }
    if (S.use_rer) {
        // dep[j]: the parameters reaction j reads.  For the others a perturbation
        // of c_k leaves lam'_j = lam_j, and their term lam log 1 - lam + lam is
        // exactly +0, so skipping them changes no bit of the sum.
#pragma unroll
        for (int kp = 0; kp < NP; ++kp) {
            if (kp >= np) continue;
            double cv[kMaxP];
#pragma unroll
            for (int p = 0; p < kMaxP; ++p) cv[p] = (p == kp) ? S.ceps[p] : S.c[p];
            double h = 0.0;
            for (int j = 0; j < S.m; ++j) {
                if (!((dep[j] >> kp) & 1u)) continue;
                const double lam = lamv[j];
                const double lp = prop_with<NS>(S, j, x, cv);
                if (lam > 0.0) h += lam * log(lam / lp) - lam + lp;
                else h += lp;
            }
            A.rer[kp] += w * h;
        }
    }
#pragma unroll
    for (int i = 0; i < NS; ++i)
        if (i < S.n) A.y[i] += w * (double)x[i];
}

template <int NS, int NP>
__global__ void __launch_bounds__(256) k_finalize(const DevInst* __restrict__ insts) {
    __shared__ SNet S;
    __shared__ double acc[kAccLen];
    const DevInst* I = insts + blockIdx.x;
    const bool small = I->net.n_species <= 2 && I->net.n_params <= 4;
    if (small != (NS <= 2)) return;  // the other launch's instance
    __shared__ uint32_t dep[kMaxM];
    const int tid = threadIdx.x;
    if (tid == 0) {
        load_net(S, I);
        for (int j = 0; j < kMaxM; ++j) {
            uint32_t d = 0;
            if (j < S.m) {
                if (S.rate_param[j] >= 0) d |= 1u << S.rate_param[j];
                for (int f = 0; f < S.nf[j]; ++f) {
                    const int kind = S.fkind[j][f];
                    if (kind == PARREP_PARAM || kind == PARREP_HILL_REP ||
                        kind == PARREP_HILL_SWITCH)
                        d |= 1u << S.fhp[j][f];
                    if (kind == PARREP_HILL_SWITCH)
                        d |= (1u << S.fp2[j][f]) | (1u << S.fp3[j][f]);
                }
            }
            dep[j] = d;
        }
    }
    for (int i = tid; i < kAccLen; i += blockDim.x) acc[i] = 0.0;
    __syncthreads();
    WinAcc<NP> A;
#pragma unroll
    for (int i = 0; i < NP * NP; ++i) A.fim[i] = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) A.rer[i] = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxS; ++i) A.y[i] = 0.0;
    // boxes hold fewer than 2^31 bins: 32-bit index arithmetic is exact
    uint32_t stride[NS], nb[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        stride[i] = (uint32_t)S.hist_stride[i];
        nb[i] = (uint32_t)S.hist_nb[i];
    }
    const uint32_t nbins = (uint32_t)I->nbins;
    for (uint32_t idx = tid; idx < nbins; idx += blockDim.x) {
        const double h = I->hist_w[idx];
        if (h == 0.0) continue;
        I->hist[idx] += h;
        int x[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) x[i] = S.hist_lo[i] + (int)((idx / stride[i]) % nb[i]);
        fim_rer_point<NS, NP>(S, dep, x, h, A);
    }
    // states outside the box: their window time sits in the spill table
    for (int i = tid; i < kSpillCap; i += blockDim.x) {
        const SpillSlot sl = I->spill[i];
        if (sl.key == 0ull || !(sl.w > 0.0)) continue;
        int x[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) x[s] = (int)((sl.key >> (15 * s)) & 0x7FFF);
        fim_rer_point<NS, NP>(S, dep, x, sl.w, A);
    }
    const int np = S.np;
    const bool lead = (tid & 63) == 0;
#pragma unroll
    for (int a = 0; a < NP; ++a)
#pragma unroll
        for (int b = 0; b < NP; ++b) {
            if (a >= np || b >= np) continue;
            const double v = wave_sum_f64(A.fim[a * NP + b]);
            if (lead) atomicAdd(&acc[kAccFim + a * np + b], v);
        }
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        if (a >= np) continue;
        const double v = wave_sum_f64(A.rer[a]);
        if (lead) atomicAdd(&acc[kAccRer + a], v);
    }
#pragma unroll
    for (int i = 0; i < kMaxS; ++i) {
        const double v = wave_sum_f64(A.y[i]);
        if (lead) atomicAdd(&acc[kAccY + i], v);
    }
    __syncthreads();
    if (tid == 0) {
        const double win = I->T - I->t_burn;
        I->stats[PARREP_ST_OUTSIDE] = I->acc[kAccOutside];
        I->stats[PARREP_ST_OUTSIDE_W] = I->acc[kAccOutsideW];
        for (int a = 0; a < np * np; ++a) I->stats[PARREP_ST_FIM + a] = acc[kAccFim + a] / win;
        for (int a = 0; a < np; ++a) I->stats[PARREP_ST_RER + a] = acc[kAccRer + a] / win;
        for (int i = 0; i < S.n; ++i) I->stats[PARREP_ST_Y + i] = acc[kAccY + i];
        // time at a state that found no spill slot is missing from FIM, RER
        // and Y: the run reports it in its status
        if (I->counters[PARREP_CNT_SPILL_OVERFLOW] != 0 && I->counters[PARREP_CNT_STATUS] == 0)
            I->counters[PARREP_CNT_STATUS] = PARREP_RUN_SPILL_OVERFLOW;
    }
}

// ---------------------------------------------------------------------------
// Test hooks
// ---------------------------------------------------------------------------
// dst[i] += src[i] (pooling the histograms of a served request's runs;
// runs of one request may finish on different streams, hence the atomics).
__global__ void __launch_bounds__(256) k_accumulate(double* __restrict__ dst,
                                                    const double* __restrict__ src, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double v = src[i];
        if (v != 0.0) atomicAdd(&dst[i], v);
    }
}

__global__ void k_philox(int64_t n, const uint32_t* __restrict__ ck, uint32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t* q = ck + 6 * i;
    const Blk b = philox10<false>(q[0], q[1], q[2], q[3], q[4], q[5]);
    out[4 * i] = b.w0;
    out[4 * i + 1] = b.w1;
    out[4 * i + 2] = b.w2;
    out[4 * i + 3] = b.w3;
}

constexpr int kEventsHookLs = 512;

__global__ void __launch_bounds__(256) k_events(const DevInst* __restrict__ inst, int64_t n,
                                                const int32_t* __restrict__ states,
                                                const uint32_t* __restrict__ blocks, double* a0o,
                                                double* tauo, int32_t* Jo) {
    __shared__ double ltab[kMaxM * kEventsHookLs];
    const TabLayout<kMaxM> tl = tab_layout<kMaxM, false>(inst, kMaxM * kEventsHookLs);
    stage_tables<kMaxM, false>(inst, tl, ltab, threadIdx.x, blockDim.x);
    __shared__ double lgt[kLogTabLen];
    for (int t = threadIdx.x; t < kLogTabLen; t += blockDim.x) lgt[t] = inst->logtab[t];
    __syncthreads();
    const HotNet<kMaxM> hn = load_hot<kMaxM>(inst, tl);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int x[kMaxS];
#pragma unroll
    for (int s = 0; s < kMaxS; ++s) x[s] = states[i * kMaxS + s];
    const Blk b{blocks[4 * i], blocks[4 * i + 1], blocks[4 * i + 2], blocks[4 * i + 3]};
    double tau, a0;
    int J;
    uint32_t dxp;
    ssa_event<kMaxS, kMaxM>(hn, inst, ltab, lgt, x, b, tau, J, dxp, &a0);
    a0o[i] = a0;
    tauo[i] = tau;
    Jo[i] = J;
}

// ---------------------------------------------------------------------------
// Multi-run estimators (Sec. III): one thread per statistic, two-pass sums
// over the runs in run order; then the bounds from the means.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(128) k_estimate(const double* const* __restrict__ st, int n,
                                                  int np, int ns, double window, double* out) {
    __shared__ double fdiag[kMaxP], iafs[kMaxS];
    const int t = threadIdx.x;
    for (int i = t; i < PARREP_EST_LEN; i += blockDim.x) out[i] = 0.0;
    __syncthreads();
    int src = -1;
    if (t < np * np) src = PARREP_ST_FIM + t;
    else if (t < np * np + np) src = PARREP_ST_RER + (t - np * np);
    else if (t < np * np + np + ns) src = PARREP_ST_Y + (t - np * np - np);
    if (src >= 0) {
        double s = 0.0;
        for (int r = 0; r < n; ++r) s += st[r][src];
        const double m = s / (double)n;
        double q = 0.0;
        for (int r = 0; r < n; ++r) {
            const double d = st[r][src] - m;
            q += d * d;
        }
        if (t < np * np) {
            out[PARREP_EST_FIM + t] = m;
            if (t % (np + 1) == 0) {
                const int k = t / (np + 1);
                out[PARREP_EST_FIM_HW + k] =
                    1.96 * (sqrt(q / (double)(n - 1)) / sqrt((double)n));
                fdiag[k] = m;
            }
        } else if (t < np * np + np) {
            out[PARREP_EST_RER + (t - np * np)] = m;
        } else {
            const int i = t - np * np - np;
            const double iaf = q / (window * (double)(n - 1));
            out[PARREP_EST_Y + i] = m;
            out[PARREP_EST_IAF + i] = iaf;
            iafs[i] = iaf;
        }
    }
    __syncthreads();
    if (t < ns * np) out[PARREP_EST_BOUND + t] = sqrt(iafs[t / np] * fdiag[t % np]);
}

}  // namespace dev

using namespace dev;

hipError_t launch_estimate(const double* const* d_stats, int n, int np, int ns, double window,
                           double* out, hipStream_t stream) {
    hipLaunchKernelGGL(k_estimate, dim3(1), dim3(128), 0, stream, d_stats, n, np, ns, window,
                       out);
    return hipGetLastError();
}

bool shape_supported(LaunchShape s) {
    const bool ns_ok = s.ns == 1 || s.ns == 2 || s.ns == 4;
    const bool rpl_ok = s.rpl == 1 || s.rpl == 4 || s.rpl == 16 || (s.rpl == 64 && s.waves == 16);
    const bool w_ok = s.waves == 1 || s.waves == 4 || s.waves == 16;
    const bool m_ok = s.m >= 1 && s.m <= kMaxM;
    return ns_ok && rpl_ok && w_ok && m_ok;
}

LaunchShape choose_shape(int R, int ns, int m) {
    const int nsv = ns <= 1 ? 1 : (ns <= 2 ? 2 : 4);
    if (R <= 64) return {1, 1, nsv, m};
    if (R <= 256) return {4, 1, nsv, m};
    if (R <= 1024) return {4, 4, nsv, m};
    if (R <= 4096) return {4, 16, nsv, m};
    if (R <= 16384) return {16, 16, nsv, m};
    return {64, 16, nsv, m};
}

#define PARREP_DECL(NSv, Wv)                                                                  \
    hipError_t launch_instance_ns##NSv##_w##Wv(const DevInst*, int, int, int, int, uint32_t,     \
                                               int64_t, int, int, long long, int, hipStream_t);
PARREP_DECL(1, 1) PARREP_DECL(1, 4) PARREP_DECL(1, 16)
PARREP_DECL(2, 1) PARREP_DECL(2, 4) PARREP_DECL(2, 16)
PARREP_DECL(4, 1) PARREP_DECL(4, 4) PARREP_DECL(4, 16)
#undef PARREP_DECL

hipError_t launch_solve(const DevInst* d_inst, int n_inst, LaunchShape s, int mode,
                        uint32_t hook_cycle, int64_t hook_max_rounds, int tab_lds,
                        hipStream_t stream) {
    if (!shape_supported(s)) return hipErrorInvalidValue;
#define PARREP_GO(NSv, Wv)                                                                    \
    if (s.ns == NSv && s.waves == Wv)                                                         \
        return launch_instance_ns##NSv##_w##Wv(d_inst, n_inst, s.m, s.rpl, mode, hook_cycle,  \
                                               hook_max_rounds, tab_lds, s.stage_flush >= 0,   \
                                               s.spec, s.persist, stream);
    PARREP_GO(1, 1) PARREP_GO(1, 4) PARREP_GO(1, 16)
    PARREP_GO(2, 1) PARREP_GO(2, 4) PARREP_GO(2, 16)
    PARREP_GO(4, 1) PARREP_GO(4, 4) PARREP_GO(4, 16)
#undef PARREP_GO
    return hipErrorInvalidValue;
}

hipError_t launch_wide_ns1(const DevInst*, int, int, int, int, hipStream_t);
hipError_t launch_wide_ns2(const DevInst*, int, int, int, int, hipStream_t);
hipError_t launch_wide_ns4(const DevInst*, int, int, int, int, hipStream_t);

hipError_t launch_wide(const DevInst* d_inst, LaunchShape s, int tab_lds, hipStream_t stream) {
    if (s.wide < 1 || s.waves != 4 || (s.rpl != 1 && s.rpl != 4)) return hipErrorInvalidValue;
    if (s.ns == 1) return launch_wide_ns1(d_inst, s.wide, s.m, s.rpl, tab_lds, stream);
    if (s.ns == 2) return launch_wide_ns2(d_inst, s.wide, s.m, s.rpl, tab_lds, stream);
    if (s.ns == 4) return launch_wide_ns4(d_inst, s.wide, s.m, s.rpl, tab_lds, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_install(const DevInst& d, DevInst* dst, hipStream_t stream) {
    hipLaunchKernelGGL(k_install, dim3(1), dim3(64), 0, stream, d, dst);
    return hipGetLastError();
}

hipError_t launch_setup(DevInst* d_inst, int n_inst, hipStream_t stream) {
    hipLaunchKernelGGL(k_setup, dim3(n_inst), dim3(256), 0, stream, d_inst);
    return hipGetLastError();
}

int species_map(const DevInst& d, LaunchShape s) {
    if (s.wide || s.ns != 2 || s.m > 4 || d.net.n_species != 2 || d.tab_L > kMapStride) return -1;
    for (int j = 0; j < d.net.n_reactions; ++j) {
        const uint32_t kind = d.jmeta[j] & 3u;
        if (kind == kRxConst) continue;  // a constant row reads the same at any state
        if (kind != kRxTable) return -1;
        if ((int)((d.jmeta[j] >> 2) & 3u) != ((kMapCross >> j) & 1)) return -1;
    }
    return kMapCross;
}

long long network_desc(const DevInst& d, LaunchShape s) {
    // compiled for 4 species, up to 8 reactions and 1 or 4 replicas per lane
    if (s.wide || s.ns != 4 || s.m > 8 || s.rpl > 4 || d.net.n_species > 4 ||
        d.net.n_reactions > kDescMaxM)
        return -1;
    uint32_t meta[kDescMaxM] = {};
    for (int j = 0; j < d.net.n_reactions; ++j) meta[j] = d.jmeta[j];
    const long long mine = desc_pack(meta, d.net.n_reactions);
    return mine == kDescSwitch ? kDescSwitch : -1;
}

int table_lds_need(const DevInst& d, LaunchShape s) {
    const int M = s.m <= 4 ? 4 : 8;
    if (s.spec >= 0 && narrow_kernel(s.ns, s.m)) return M * kMapStride;
    if (narrow_kernel(s.ns, s.m)) return M * d.tab_L;
    int need = 0;
    for (int j = 0; j < d.net.n_reactions; ++j)
        if ((d.jmeta[j] & 3u) == kRxTable) need += d.tab_Lsp[(d.jmeta[j] >> 2) & 3u];
    return need;
}

int table_lds_doubles(LaunchShape s, int max_need) {
    // the wide kernel runs one workgroup per CU and exchanges through HBM;
    // a staging tile takes 8 KiB more
    size_t xb = s.wide ? 0 : xbuf_lds_bytes(s.rpl, s.waves, s.ns);
    if (!s.wide && s.stage_flush >= 0) xb += kTileDoubles * 8;
    // leaves room for the static LDS of the kernel (24 KB more of it with 64
    // replicas per lane: the survivor masks and counts of 1024 slots)
    const size_t budget = (s.rpl == 64 ? 32 : 56) * 1024;
    const size_t fit = xb < budget ? (budget - xb) / 8 : 0;
    return (int)(fit < (size_t)max_need ? fit : (size_t)max_need);
}

hipError_t launch_zero(const DevInst* d_inst, int n_inst, hipStream_t stream) {
    hipLaunchKernelGGL(k_zero, dim3(64, n_inst), dim3(256), 0, stream, d_inst);
    return hipGetLastError();
}

hipError_t launch_finalize(const DevInst* d_inst, int n_inst, hipStream_t stream) {
    // one launch for instances of at most 2 species and 4 parameters, one
    // for the rest; each block of the other class returns at once
    hipLaunchKernelGGL((k_finalize<2, 4>), dim3(n_inst), dim3(256), 0, stream, d_inst);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_finalize<kMaxS, kMaxP>), dim3(n_inst), dim3(256), 0, stream, d_inst);
    return hipGetLastError();
}

hipError_t launch_accumulate(double* dst, const double* src, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t want = (n + 255) / 256;
    const unsigned blocks = (unsigned)(want < 4096 ? want : 4096);
    hipLaunchKernelGGL(k_accumulate, dim3(blocks), dim3(256), 0, stream, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_philox(int64_t n, const uint32_t* ctr_key, uint32_t* out, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_philox, dim3((unsigned)blocks), dim3(256), 0, stream, n, ctr_key, out);
    return hipGetLastError();
}

hipError_t launch_events(const DevInst* d_inst, int64_t n, const int32_t* states,
                         const uint32_t* blocks, double* a0, double* tau, int32_t* J,
                         hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_events, dim3((unsigned)nb), dim3(256), 0, stream, d_inst, n, states,
                       blocks, a0, tau, J);
    return hipGetLastError();
}

}  // namespace parrep
