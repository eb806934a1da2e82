// parrep_wide.h -- one ParRep instance (Alg. 1, Sec. II A) spread over the
// workgroups of a cooperative launch, for large replica counts.
//
// Replica r lives in slot k of lane l of wave v (r = (v RPL + k) 64 + l), so
// every wave holds a contiguous range of replicas.  Between the few points
// where the method couples replicas, the waves run on their own, with no
// barrier per round:
//
//   * decorrelation is serial: every workgroup runs the same chain on one
//     wave (workgroup 0 alone credits it), so all hold the same state after;
//   * dephasing runs in chunks of up to S2 rounds.  A wave stops its chunk at
//     its first round in which a replica left the set.  At the chunk's end
//     the workgroups meet at a grid barrier and agree on E, the first round
//     with an exit, and D, the round after which every replica has dephased
//     (t^r >= t_p, or n_p rounds).  Waves that ran past min(D, E) replay the
//     chunk from its saved start (the counter-based random numbers make the
//     replay exact); an exit round ends with the Fleming-Viot restart from
//     every wave's survivors;
//   * the parallel step runs in chunks of up to S3 rounds: a first pass finds
//     each wave's first exit and the exact 64.64 clock sum of each round; at
//     the grid barrier the workgroups agree on the first exit key R n + r and
//     find the first round that crosses the burn-in time or the horizon; a
//     second pass replays the chunk and credits whole rounds in parallel,
//     and the boundary or exit round is credited by an exact scan in key
//     order (the ParRep-CTMC rule, Sec. II A, properties 1-2: the serial
//     order of the credited events does not depend on how replicas are split).
//
// Every grid-barrier wait is bounded (DevInst::wide_wait_ticks of the
// constant wall clock); a workgroup that gives up sets the abort word, every
// workgroup then leaves, and the run reports PARREP_RUN_ABORTED.
#pragma once
#include "parrep_device.h"

namespace parrep {
namespace dev {
namespace {

constexpr int64_t kNever = INT64_MAX;

struct WideLds {
    uint64_t sums[kWideS3Max][3];  // this workgroup's per-round clock sums of a chunk
    int32_t pre[PARREP_MAX_REPLICAS / 64 + 2];  // survivor prefix counts per 64 replicas
    int32_t part[16];
    int32_t aborted;
    int64_t last_s2, last_s3;  // rounds of the cycle whose parallel step met the horizon
};

// Grid barrier of the cooperative launch.  Every thread releases its writes
// at agent scope, the workgroup meets, thread 0 arrives and waits (bounded)
// for every workgroup's arrival, the workgroup meets again and every thread
// acquires.  Returns false when the run is being aborted.
__device__ __forceinline__ bool grid_sync(WideSync* ws, WideLds& wl, uint32_t& gen,
                                          uint32_t nwg, int64_t wait_ticks) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        gen += 1;
        const uint32_t target = gen * nwg;
        __hip_atomic_fetch_add(&ws->bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t t0 = wall_clock64();
        int ab = 0;
        for (;;) {
            const uint32_t b = __hip_atomic_load(&ws->bar, __ATOMIC_ACQUIRE,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            if ((int32_t)(b - target) >= 0) break;
            if (__hip_atomic_load(&ws->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                ab = 1;
                break;
            }
            if ((int64_t)(wall_clock64() - t0) > wait_ticks) {
                __hip_atomic_store(&ws->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ab = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (!ab && __hip_atomic_load(&ws->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            ab = 1;
        wl.aborted = ab;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return wl.aborted == 0;
}

__device__ __forceinline__ int64_t ld_i64(const int64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_u64(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exact sum of one round's clock over all waves, from the chunk's three
// split sums, saturated at 2^52 (no sum of holding times this large is below
// any horizon).
__device__ __forceinline__ Fx round_total(const uint64_t* s) {
    const uint64_t hi = ld_u64(s), lh = ld_u64(s + 1), ll = ld_u64(s + 2);
    // lo = ll + (lh << 32), carries into hi
    const uint64_t a = lh << 32;
    uint64_t lo = ll + a;
    uint64_t h = hi + (lh >> 32) + (lo < a ? 1u : 0u);
    if (h >= kFxSatHi) return Fx{kFxSatHi, 0};
    return Fx{h, lo};
}

// Reset chunk slot q (workgroup 0, before its next arrival).
__device__ __forceinline__ void reset_slot(WideSync* ws, int q) {
    const int t = threadIdx.x;
    if (t == 0) {
        ws->e2[q] = kNever;
        ws->d2[q] = -1;
        ws->k3[q] = ~0ull;
    }
    for (int i = t; i < kWideS3Max * 3; i += blockDim.x) (&ws->s3[q][0][0])[i] = 0;
}

template <int NS, int M, int RPL, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) k_wide(const DevInst* __restrict__ I, int tab_lds) {
    constexpr int B = 64 * WAVES;
    __shared__ RunState rs;
    __shared__ WideLds wl;
    extern __shared__ int32_t dyn_lds[];

    WideSync* ws = I->wide;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const uint32_t nwg = gridDim.x;
    const int nwv = (int)nwg * WAVES;               // waves in the grid
    const int wv = (int)blockIdx.x * WAVES + wid;   // this wave
    const bool lead = blockIdx.x == 0;
    const int R = I->R;
    const uint32_t key0 = I->seed, key1 = I->instance_id;
    const int64_t wait_ticks = I->wide_wait_ticks;
    const int S2C = I->wide_s2, S3C = I->wide_s3;
    uint32_t gen = 0;   // grid barriers passed
    uint32_t cc = 0;    // chunk barriers passed (chunk slot = cc % 3)

    double* ltab = reinterpret_cast<double*>(dyn_lds);
    const TabLayout<M> tl = tab_layout<M, narrow_kernel(NS, M)>(I, tab_lds);
    stage_tables<M, narrow_kernel(NS, M)>(I, tl, ltab, tid, B);
    __shared__ double lgt[kLogTabLen];
    for (int i = tid; i < kLogTabLen; i += B) lgt[i] = I->logtab[i];
    const HotNet<M> hn = load_hot<M>(I, tl);
    const int64_t max_ev = I->max_events > 0 ? I->max_events : (int64_t(1) << 50);

    if (tid == 0) {
        const Fx Tq0 = fx_from(I->T), tbq0 = fx_from(I->t_burn);
        rs.Tq_hi = Tq0.hi;
        rs.Tq_lo = Tq0.lo;
        rs.tbq_hi = tbq0.hi;
        rs.tbq_lo = tbq0.lo;
        rs.C_hi = rs.C_lo = 0;
        rs.clk[0] = rs.clk[1] = rs.clk[2] = 0;
        rs.clk[3] = wall_clock64();
        rs.clk_mark = rs.clk[3];
        rs.ev_total = 0;
        rs.c_decorr = rs.c_dephase = rs.c_cred = rs.c_disc = rs.c_cycles = 0;
        rs.c_s3 = rs.c_s2 = rs.c_fv = rs.n_log = rs.s1_events = 0;
        rs.cycle = 0;
        rs.stop = rs.end_phase = 0;
        int x[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) x[i] = I->x0[i];
#pragma unroll
        for (int i = 0; i < kMaxS; ++i) rs.xt[i] = rs.xend[i] = i < NS ? x[i] : 0;
        rs.W = region_of<NS>(I, x);
        wl.aborted = 0;
    }
    __syncthreads();

    bool aborted = false;
    bool hit_wait = false;  // the horizon fell in an exact round: its replica is read at the end
    for (;;) {
        // ------------------------------------------------------------------
        // S1, decorrelation: the same serial chain in every workgroup.
        // ------------------------------------------------------------------
        if (wid == 0) {
            if (lane == 0) rs.clk_mark = wall_clock64();
            decorrelate<NS, M>(hn, I, ltab, lgt, rs, Fx{rs.Tq_hi, rs.Tq_lo},
                               Fx{rs.tbq_hi, rs.tbq_lo}, max_ev, key0, key1, lane, lead);
            if (lane == 0) {
                const uint64_t now = wall_clock64();
                rs.clk[0] += now - rs.clk_mark;
                rs.clk_mark = now;
            }
        }
        __syncthreads();
        if (rs.stop) {
            if (tid == 0) {
                rs.end_phase = rs.stop;
                int xe[NS];
#pragma unroll
                for (int i = 0; i < NS; ++i) xe[i] = rs.xend[i];
                if (lead) log_cycle<NS>(I, rs.n_log, rs.cycle, rs.s1_events, 0, 0, 0, rs.stop, xe);
                rs.n_log += 1;
            }
            break;
        }
        const uint32_t cycle = ufl((uint32_t)rs.cycle);
        const int W = ufl(rs.W);
        int xt[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) xt[i] = ufl(rs.xt[i]);

        // ------------------------------------------------------------------
        // S2, dephasing, in chunks.
        // ------------------------------------------------------------------
        int Y[RPL][NS];
        double tr[RPL];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
#pragma unroll
            for (int i = 0; i < NS; ++i) Y[k][i] = xt[i];
            tr[k] = 0.0;
        }
        const bool steps = I->dephase_mode == PARREP_STEPS;
        const int64_t n_p = (int64_t)I->dephase;
        const double t_p = I->dephase;
        const int64_t left2 = (max_ev - rs.ev_total) / R;
        const int64_t budget2 = (int64_t)ufl64((uint64_t)(left2 > 0 ? left2 : 0));
        int64_t n0 = 0, round2 = 0;
        bool budget = false;
        int64_t fv = 0;
        int64_t dw = kNever;  // this wave's first round after which its replicas are all done
        if (!(steps ? (n_p <= 0) : (0.0 >= t_p))) {
            for (;;) {
                if (n0 >= budget2) {
                    budget = true;
                    round2 = n0;
                    break;
                }
                const int64_t end = min(n0 + (int64_t)S2C, budget2) - 1;
                int Y0[RPL][NS];
                double tr0[RPL];
#pragma unroll
                for (int k = 0; k < RPL; ++k) {
#pragma unroll
                    for (int i = 0; i < NS; ++i) Y0[k][i] = Y[k][i];
                    tr0[k] = tr[k];
                }
                int64_t ew = kNever, pos = n0 - 1;
                uint32_t exitbits = 0;
                for (int64_t n = n0; n <= end; ++n) {
                    exitbits = 0;
                    bool nd = false;
#pragma unroll
                    for (int k = 0; k < RPL; ++k) {
                        const int r = (wv * RPL + k) * 64 + lane;
                        if (r < R) {
                            const Blk b = draw((uint64_t)n, (uint32_t)r, cycle, kTagDephase,
                                               key0, key1);
                            double tau;
                            int J;
                            uint32_t dxp;
                            ssa_event<NS, M>(hn, I, ltab, lgt, Y[k], b, tau, J, dxp);
                            apply_dx<NS>(Y[k], dxp);
                            tr[k] = tr[k] + tau;
                            if (region_hot<NS, M>(hn, Y[k]) != W) exitbits |= 1u << k;
                            if (!(tr[k] >= t_p)) nd = true;
                        }
                    }
                    pos = n;
                    if (!steps && dw == kNever && __ballot(nd) == 0ull) dw = n;
                    if (__ballot(exitbits != 0) != 0ull) {
                        ew = n;
                        break;
                    }
                }
                const int q = (int)(cc % 3);
                if (lane == 0) {
                    __hip_atomic_fetch_min(&ws->e2[q], ew, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    const int64_t dpost = steps ? (n_p - 1 <= end ? n_p - 1 : kNever) : dw;
                    __hip_atomic_fetch_max(&ws->d2[q], dpost, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
                if (!grid_sync(ws, wl, gen, nwg, wait_ticks)) {
                    aborted = true;
                    break;
                }
                cc += 1;
                const int64_t E = (int64_t)ufl64((uint64_t)ld_i64(&ws->e2[q]));
                const int64_t D = (int64_t)ufl64((uint64_t)ld_i64(&ws->d2[q]));
                if (lead) reset_slot(ws, (int)((cc + 1) % 3));
                int64_t target;
                bool do_fv, stop;
                if (D != kNever && D >= 0 && D <= end && (E == kNever || D < E)) {
                    target = D;
                    do_fv = false;
                    stop = true;
                } else if (E != kNever) {
                    target = E;
                    do_fv = true;
                    stop = D == E;
                } else {
                    n0 = end + 1;
                    continue;
                }
                if (pos != target) {
                    // replay the chunk from its start up to the target round
#pragma unroll
                    for (int k = 0; k < RPL; ++k) {
#pragma unroll
                        for (int i = 0; i < NS; ++i) Y[k][i] = Y0[k][i];
                        tr[k] = tr0[k];
                    }
                    for (int64_t n = n0; n <= target; ++n) {
                        exitbits = 0;
#pragma unroll
                        for (int k = 0; k < RPL; ++k) {
                            const int r = (wv * RPL + k) * 64 + lane;
                            if (r < R) {
                                const Blk b = draw((uint64_t)n, (uint32_t)r, cycle, kTagDephase,
                                                   key0, key1);
                                double tau;
                                int J;
                                uint32_t dxp;
                                ssa_event<NS, M>(hn, I, ltab, lgt, Y[k], b, tau, J, dxp);
                                apply_dx<NS>(Y[k], dxp);
                                tr[k] = tr[k] + tau;
                                if (region_hot<NS, M>(hn, Y[k]) != W) exitbits |= 1u << k;
                            }
                        }
                    }
                }
                if (dw != kNever && dw > target) dw = kNever;  // found past the target
                if (do_fv) {
                    // Fleming-Viot over every wave's survivors of round `target`:
                    // post the states and survivor words, meet, count.
                    int32_t* xb = I->xbuf;
#pragma unroll
                    for (int k = 0; k < RPL; ++k) {
                        const int r = (wv * RPL + k) * 64 + lane;
                        if (r < R) {
#pragma unroll
                            for (int i = 0; i < NS; ++i) xb[r * NS + i] = Y[k][i];
                        }
                        const uint64_t m = __ballot(r < R && !((exitbits >> k) & 1u));
                        if (lane == 0) I->smask[wv * RPL + k] = m;
                    }
                    if (!grid_sync(ws, wl, gen, nwg, wait_ticks)) {
                        aborted = true;
                        break;
                    }
                    // prefix counts of survivors per word, in LDS
                    const int nwords = nwv * RPL;
                    const int per = (nwords + B - 1) / B;
                    int cnt = 0;
                    for (int w = tid * per; w < (tid + 1) * per && w < nwords; ++w)
                        cnt += __popcll(I->smask[w]);
                    const int incl = wave_incl_scan(cnt, lane);
                    if (lane == 63) wl.part[wid] = incl;
                    __syncthreads();
                    int off = 0;
                    for (int w = 0; w < wid; ++w) off += wl.part[w];
                    int run = off + incl - cnt;
                    for (int w = tid * per; w < (tid + 1) * per && w < nwords; ++w) {
                        wl.pre[w] = run;
                        run += __popcll(I->smask[w]);
                    }
                    if (tid == B - 1) wl.pre[nwords] = off + incl;
                    __syncthreads();
                    const int nS = ufl(wl.pre[nwords]);
#pragma unroll
                    for (int k = 0; k < RPL; ++k) {
                        if (!((exitbits >> k) & 1u)) continue;
                        const int r = (wv * RPL + k) * 64 + lane;
                        if (nS > 0) {
                            const Blk b = draw((uint64_t)target, (uint32_t)r, cycle, kTagFV, key0,
                                               key1);
                            const int idx = (int)(((uint64_t)b.w0 * (uint64_t)nS) >> 32);
                            int lo = 0, hi = nwords;  // pre[lo] <= idx < pre[hi]
                            while (hi - lo > 1) {
                                const int mid = (lo + hi) >> 1;
                                if (wl.pre[mid] <= idx) lo = mid;
                                else hi = mid;
                            }
                            const int l = select_bit(I->smask[lo], idx - wl.pre[lo]);
                            const int rr = lo * 64 + l;
#pragma unroll
                            for (int i = 0; i < NS; ++i) Y[k][i] = xb[rr * NS + i];
                        } else {
#pragma unroll
                            for (int i = 0; i < NS; ++i) Y[k][i] = xt[i];
                        }
                    }
                    fv += R - nS;
                    // the next exchange writes xbuf and smask only after a later
                    // chunk barrier, which every wave reaches after these reads
                }
                n0 = target + 1;
                if (stop) {
                    round2 = n0;
                    break;
                }
            }
        }
        if (aborted) break;
        __syncthreads();
        if (tid == 0) {
            const uint64_t now = wall_clock64();
            rs.clk[1] += now - rs.clk_mark;
            rs.clk_mark = now;
            rs.ev_total += round2 * R;
            rs.c_dephase += round2 * R;
            rs.c_fv += fv;
            if (!budget) rs.c_s2 += round2;
        }
        if (budget) {
            if (tid == 0) {
                rs.end_phase = 9;
#pragma unroll
                for (int i = 0; i < NS; ++i) rs.xend[i] = xt[i];
                if (lead) log_cycle<NS>(I, rs.n_log, cycle, rs.s1_events, 0, 0, 0, 9, xt);
                rs.n_log += 1;
            }
            break;
        }
        __syncthreads();

        // ------------------------------------------------------------------
        // S3, the parallel step, in chunks.
        // ------------------------------------------------------------------
        const int64_t left3 = (max_ev - rs.ev_total) / R;
        const int64_t budget3 = (int64_t)ufl64((uint64_t)(left3 > 0 ? left3 : 0));
        Fx C = ufx(Fx{rs.C_hi, rs.C_lo});
        const Fx Tq = ufx(Fx{rs.Tq_hi, rs.Tq_lo});
        const Fx tbq = ufx(Fx{rs.tbq_hi, rs.tbq_lo});
        int64_t m0 = 0, cred = 0, disc = 0;
        int outcome = -1;  // 1 exit, 0 horizon, -1 budget
        int Kx = 0;
        for (;;) {
            if (m0 >= budget3) {
                outcome = -1;
                break;
            }
            const int64_t end = min(m0 + (int64_t)S3C, budget3) - 1;
            int Z0[RPL][NS];
#pragma unroll
            for (int k = 0; k < RPL; ++k)
#pragma unroll
                for (int i = 0; i < NS; ++i) Z0[k][i] = Y[k][i];
            for (int i = tid; i < kWideS3Max * 3; i += B) (&wl.sums[0][0])[i] = 0;
            __syncthreads();
            // pass 1: first exit of this wave, and its clock sum per round
            uint64_t kw = ~0ull;
            for (int64_t m = m0; m <= end; ++m) {
                Fx lsum{0, 0};
                int firstk = -1, fl = 0;
#pragma unroll
                for (int k = 0; k < RPL; ++k) {
                    const int r = (wv * RPL + k) * 64 + lane;
                    bool ex = false;
                    if (r < R) {
                        const Blk b = draw((uint64_t)m, (uint32_t)r, cycle, kTagParallel, key0,
                                           key1);
                        double tau;
                        int J;
                        uint32_t dxp;
                        ssa_event<NS, M>(hn, I, ltab, lgt, Y[k], b, tau, J, dxp);
                        apply_dx<NS>(Y[k], dxp);
                        ex = region_hot<NS, M>(hn, Y[k]) != W;
                        lsum = fx_add_sat(lsum, fx_from(tau));
                    }
                    const uint64_t bm = __ballot(ex);
                    if (bm && firstk < 0) {
                        firstk = k;
                        fl = __ffsll((unsigned long long)bm) - 1;
                    }
                }
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) lsum = fx_add_sat(lsum, shfl_xor_fx(lsum, off));
                if (lane == 0) {
                    uint64_t* s = wl.sums[m - m0];
                    atomicAdd((unsigned long long*)&s[0], (unsigned long long)lsum.hi);
                    atomicAdd((unsigned long long*)&s[1], (unsigned long long)(lsum.lo >> 32));
                    atomicAdd((unsigned long long*)&s[2],
                              (unsigned long long)(lsum.lo & 0xFFFFFFFFull));
                }
                if (firstk >= 0) {
                    kw = (uint64_t)m * (uint64_t)R + (uint64_t)((wv * RPL + firstk) * 64 + fl);
                    break;
                }
            }
            const int q = (int)(cc % 3);
            if (lane == 0)
                __hip_atomic_fetch_min(&ws->k3[q], kw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            for (int i = tid; i < kWideS3Max * 3; i += B) {
                const uint64_t v = (&wl.sums[0][0])[i];
                if (v) atomicAdd((unsigned long long*)&(&ws->s3[q][0][0])[i], (unsigned long long)v);
            }
            if (!grid_sync(ws, wl, gen, nwg, wait_ticks)) {
                aborted = true;
                break;
            }
            cc += 1;
            const uint64_t kstar = ufl64(ld_u64(&ws->k3[q]));
            const int64_t nstar = kstar == ~0ull ? kNever : (int64_t)(kstar / (uint64_t)R);
            const int64_t last_full = nstar == kNever ? end : (nstar - 1 < end ? nstar - 1 : end);
            // first full round that crosses the burn-in time or the horizon
            int64_t bnd = kNever;
            {
                Fx Cr = C;
                for (int64_t m = m0; m <= last_full; ++m) {
                    const Fx tot = ufx(round_total(ws->s3[q][m - m0]));
                    const Fx Ce = fx_add(Cr, tot);
                    if (fx_ge(Ce, Tq) || (fx_gt(tbq, Cr) && fx_gt(Ce, tbq))) {
                        bnd = m;
                        break;
                    }
                    Cr = Ce;
                }
            }
            // pass 2: replay, crediting whole rounds in parallel
#pragma unroll
            for (int k = 0; k < RPL; ++k)
#pragma unroll
                for (int i = 0; i < NS; ++i) Y[k][i] = Z0[k][i];
            const int64_t full_end = bnd != kNever ? bnd - 1 : last_full;
            for (int64_t m = m0; m <= full_end; ++m) {
                const bool win = fx_ge(C, tbq);
#pragma unroll
                for (int k = 0; k < RPL; ++k) {
                    const int r = (wv * RPL + k) * 64 + lane;
                    if (r < R) {
                        const Blk b = draw((uint64_t)m, (uint32_t)r, cycle, kTagParallel, key0,
                                           key1);
                        double tau;
                        int J;
                        uint32_t dxp;
                        ssa_event<NS, M>(hn, I, ltab, lgt, Y[k], b, tau, J, dxp);
                        credit_side<NS>(I, Y[k], tau, win);
                        apply_dx<NS>(Y[k], dxp);
                    }
                }
                C = fx_add(C, ufx(round_total(ws->s3[q][m - m0])));
                cred += R;
            }
            if (lead) reset_slot(ws, (int)((cc + 1) % 3));
            const int64_t rb = bnd != kNever ? bnd : (nstar <= end ? nstar : kNever);
            if (rb == kNever) {
                m0 = end + 1;
                continue;
            }
            // the boundary or exit round: exact scan in key order
            const bool exit_round = nstar == rb;
            const int K = exit_round ? (int)(kstar % (uint64_t)R) + 1 : R;
            double tauk[RPL];
            uint32_t dxk[RPL];
            Fx run{0, 0};
            Fx pre[RPL];
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                const int r = (wv * RPL + k) * 64 + lane;
                tauk[k] = 0.0;
                dxk[k] = 0;
                Fx v{0, 0};
                if (r < R) {
                    const Blk b = draw((uint64_t)rb, (uint32_t)r, cycle, kTagParallel, key0,
                                       key1);
                    int J;
                    ssa_event<NS, M>(hn, I, ltab, lgt, Y[k], b, tauk[k], J, dxk[k]);
                    if (r < K) v = fx_from(tauk[k]);
                }
                // start of each interval: the (saturating) sum of the ones before
                // it, within the wave in lane order, then across slots; a
                // saturated sum is beyond any horizon, and so is every start after it
                Fx inc = v;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const Fx t = shfl_up_fx(inc, off);
                    if (lane >= off) inc = fx_add_sat(inc, t);
                }
                Fx ex = shfl_up_fx(inc, 1);
                if (lane == 0) ex = Fx{0, 0};
                pre[k] = fx_add_sat(run, ex);
                run = fx_add_sat(run, readlane_fx(inc, 63));
            }
            if (lane == 0) {
                I->wtot[2 * wv] = run.hi;
                I->wtot[2 * wv + 1] = run.lo;
            }
            if (!grid_sync(ws, wl, gen, nwg, wait_ticks)) {
                aborted = true;
                break;
            }
            Fx off{0, 0}, total{0, 0};
            for (int w = 0; w < nwv; ++w) {
                const Fx t = ufx(Fx{ld_u64(&I->wtot[2 * w]), ld_u64(&I->wtot[2 * w + 1])});
                if (w < wv) off = fx_add_sat(off, t);
                total = fx_add_sat(total, t);
            }
            off = fx_add(C, off);
            const Fx Cend = fx_add(C, total);
            const bool hit = fx_ge(Cend, Tq);
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                const int r = (wv * RPL + k) * 64 + lane;
                if (r < K) {
                    const Fx st = fx_add(off, pre[k]);
                    if (!fx_ge(st, Tq)) {
                        Fx dummy;
                        if (credit_event<NS>(I, Y[k], tauk[k], st, Tq, tbq, true, dummy)) {
                            ws->rend = r;
#pragma unroll
                            for (int i = 0; i < NS; ++i) ws->xf[i] = Y[k][i];
                        }
                    }
                }
            }
            if (hit) {
                C = Tq;
                hit_wait = true;
                outcome = 0;
                m0 = rb + 1;
                break;
            }
            C = Cend;
            cred += K;
            if (exit_round) {
                disc += R - K;
#pragma unroll
                for (int k = 0; k < RPL; ++k) {
                    const int r = (wv * RPL + k) * 64 + lane;
                    if (r == K - 1) {
                        int post[NS];
#pragma unroll
                        for (int i = 0; i < NS; ++i) post[i] = Y[k][i];
                        apply_dx<NS>(post, dxk[k]);
#pragma unroll
                        for (int i = 0; i < NS; ++i) ws->xb[i] = post[i];
                    }
                }
                if (!grid_sync(ws, wl, gen, nwg, wait_ticks)) {
                    aborted = true;
                    break;
                }
                if (tid == 0) {
#pragma unroll
                    for (int i = 0; i < NS; ++i)
                        rs.xt[i] = __hip_atomic_load(&ws->xb[i], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                }
                Kx = K;
                outcome = 1;
                m0 = rb + 1;
                break;
            }
#pragma unroll
            for (int k = 0; k < RPL; ++k) apply_dx<NS>(Y[k], dxk[k]);
            m0 = rb + 1;
        }
        if (aborted) break;
        __syncthreads();
        if (tid == 0) {
            const uint64_t now = wall_clock64();
            rs.clk[2] += now - rs.clk_mark;
            rs.clk_mark = now;
            rs.ev_total += m0 * R;
            rs.c_cred += cred;
            rs.c_disc += disc;
            rs.c_s3 += m0;
            rs.C_hi = C.hi;
            rs.C_lo = C.lo;
            if (outcome == 1) {
                int xl[NS];
#pragma unroll
                for (int i = 0; i < NS; ++i) xl[i] = rs.xt[i];
                if (lead) log_cycle<NS>(I, rs.n_log, cycle, rs.s1_events, round2, m0, Kx, 3, xl);
                rs.n_log += 1;
                rs.c_cycles += 1;
                rs.W = region_of<NS>(I, xl);
                rs.cycle = (int32_t)(cycle + 1);
            } else if (outcome == -1) {
                rs.end_phase = 9;
#pragma unroll
                for (int i = 0; i < NS; ++i) rs.xend[i] = xt[i];
                if (lead) log_cycle<NS>(I, rs.n_log, cycle, rs.s1_events, round2, m0, 0, 9, xt);
                rs.n_log += 1;
            } else {
                // the horizon: its replica's state and index are read after the
                // final barrier, then the cycle is logged
                rs.end_phase = 3;
                wl.last_s2 = round2;
                wl.last_s3 = m0;
            }
        }
        __syncthreads();
        if (outcome != 1) break;
    }

    // Final meeting: the horizon replica's record becomes visible to
    // workgroup 0, which writes the outputs.
    if (!aborted && !grid_sync(ws, wl, gen, nwg, wait_ticks)) aborted = true;
    if (!lead || tid != 0) return;
    if (!aborted && hit_wait) {
        const int64_t rend = ld_i64(&ws->rend);
        int xl[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            xl[i] = __hip_atomic_load(&ws->xf[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            rs.xend[i] = xl[i];
        }
        rs.c_cred += rend + 1;
        rs.c_disc += R - (rend + 1);
        log_cycle<NS>(I, rs.n_log, rs.cycle, rs.s1_events, wl.last_s2, wl.last_s3, 0, 3, xl);
        rs.n_log += 1;
    }
    int64_t* cn = I->counters;
    cn[PARREP_CNT_EV_DECORR] = rs.c_decorr;
    cn[PARREP_CNT_EV_DEPHASE] = rs.c_dephase;
    cn[PARREP_CNT_EV_PAR_CREDITED] = rs.c_cred;
    cn[PARREP_CNT_EV_PAR_DISCARDED] = rs.c_disc;
    cn[PARREP_CNT_CYCLES] = rs.c_cycles;
    cn[PARREP_CNT_S3_ROUNDS] = rs.c_s3;
    cn[PARREP_CNT_S2_ROUNDS] = rs.c_s2;
    cn[PARREP_CNT_STATUS] = aborted ? PARREP_RUN_ABORTED
                                    : (rs.end_phase == 9 ? PARREP_RUN_BUDGET : PARREP_RUN_OK);
    cn[PARREP_CNT_FV_RESTARTS] = rs.c_fv;
    cn[PARREP_CNT_END_PHASE] = aborted ? 9 : rs.end_phase;
    cn[PARREP_CNT_N_CYCLE_LOG] = rs.n_log;
#pragma unroll
    for (int i = 0; i < kMaxS; ++i) I->x_final[i] = i < NS ? rs.xend[i] : 0;
    I->stats[PARREP_ST_T] = fx_to_f64(Fx{rs.C_hi, rs.C_lo});
    if (I->phase_clock) {
        I->phase_clock[0] = (int64_t)rs.clk[0];
        I->phase_clock[1] = (int64_t)rs.clk[1];
        I->phase_clock[2] = (int64_t)rs.clk[2];
        I->phase_clock[3] = (int64_t)(wall_clock64() - rs.clk[3]);
    }
}

}  // namespace
}  // namespace dev
}  // namespace parrep
