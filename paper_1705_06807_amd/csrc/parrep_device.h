// parrep_device.h -- device code of libparrep for gfx950: parallel replica dynamics
// (Wang & Plechac, arXiv 1705.06807, Sec. II A, Algorithm 1) on CTMC
// reaction networks.
//
// One workgroup runs one ParRep instance.  Its replicas are spread over the
// lanes: replica r = k*B + tid lives in register slot k of thread tid
// (B = 64*WAVES threads, RPL slots).  Decorrelation is serial and runs on
// thread 0; dephasing and the parallel step advance all replicas one SSA
// event per round.  Per round the workgroup only exchanges what the method
// needs: whether any replica left the metastable set (dephasing), the first
// exiting replica and the credited time (parallel step).  Everything rare --
// Fleming-Viot restarts, the round that crosses the burn-in time or the
// horizon, the exit round -- takes a slower exact path.
//
// Numerics shared with the CPU oracle by definition, not by code:
//   * Philox4x32-10, key (seed, instance), counter (step, replica, cycle,
//     tag<<28 | step>>32); u_open from words 0-1 in (0,1], u_sel from words
//     2-3 in [0,1);
//   * propensities k_j * phi_1 * phi_2 left to right, falling factorials
//     exact in 64-bit integers, Hill powers by repeated multiplication for
//     integral exponents; tau = -log(u_open)/a0; J = first j with
//     u_sel*a0 < S_j; everything built with -ffp-contract=off;
//   * the ParRep clock is an exact 64.64 fixed-point sum of credited
//     holding times (each truncated to 2^-64), so the burn-in time and the
//     horizon are crossed at one event whatever the reduction order.
#pragma once
#include "parrep_fx.h"
#include "parrep_internal.h"
#include "parrep_neglog.h"

#include <climits>
#include <type_traits>
#include <utility>

namespace parrep {
namespace dev {
namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// ---------------------------------------------------------------------------
struct Blk {
    uint32_t w0, w1, w2, w3;
};

// a ^ b ^ k in one VALU op (gfx950 three-input bit operation; 0x96 is the
// truth table of a three-way XOR), k in a scalar register.
__device__ __forceinline__ uint32_t xor3_sk(uint32_t a, uint32_t b, uint32_t k) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

// a * m as one 32x32->64 multiply-add with both halves in a register pair.
__device__ __forceinline__ uint64_t mul_wide_sk(uint32_t a, uint32_t m) {
    uint64_t r, carry;
    asm("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(r), "=s"(carry) : "v"(a), "s"(m));
    return r;
}

// UK: the key is the same in every lane (the instance's).  Its round keys
// are then re-derived in scalar registers at each call (hoisted out of the
// caller's loops, the twenty of them would be spilled to vector lanes and
// read back with one VALU op each), and from the fourth round on, when all
// four words differ between lanes, each round is two multiply-adds and two
// three-way XORs.  With a lane-uniform step, cycle and tag (the replica index
// is the only word that differs), one product of rounds 1 and 2 and both of
// round 0 are lane-uniform: rounds 0-2 are left to the compiler, which keeps
// those words in scalar registers.
template <bool UK = true>
__device__ __forceinline__ Blk philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
    if (UK) asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        uint64_t p0, p1;
        uint32_t n0, n2;
        if (UK && i > 2) {
            p0 = mul_wide_sk(c0, 0xD2511F53u);
            p1 = mul_wide_sk(c2, 0xCD9E8D57u);
            n0 = xor3_sk((uint32_t)(p1 >> 32), c1, k0);
            n2 = xor3_sk((uint32_t)(p0 >> 32), c3, k1);
        } else {
            p0 = (uint64_t)0xD2511F53u * c0;
            p1 = (uint64_t)0xCD9E8D57u * c2;
            n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
            n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        }
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Blk{c0, c1, c2, c3};
}

__device__ __forceinline__ Blk draw(uint64_t step, uint32_t rep, uint32_t cycle, uint32_t tag,
                                    uint32_t k0, uint32_t k1) {
    return philox10((uint32_t)step, rep, cycle,
                    (tag << 28) | ((uint32_t)(step >> 32) & 0x0FFFFFFFu), k0, k1);
}

__device__ __forceinline__ double u_open(const Blk& b) {
    const uint64_t w = ((uint64_t)b.w1 << 32) | b.w0;
    return (double)((w >> 11) + 1) * 0x1.0p-53;
}

__device__ __forceinline__ double u_sel(const Blk& b) {
    // (w >> 11) 2^-53 for w = w3:w2, as w3 2^-32 + (w2 >> 11) 2^-53: both
    // terms and their sum (a 53-bit integer times 2^-53) are exact
    return fma((double)b.w3, 0x1.0p-32, (double)(b.w2 >> 11) * 0x1.0p-53);
}

// -log(u_open(b)); lt: the reduction table in LDS.
__device__ __forceinline__ double neglog_u_open(const Blk& b, const double* __restrict__ lt) {
    return neglog_words53(b.w1, b.w0, lt);
}

// Values known to be equal in all lanes, moved to scalar registers.
__device__ __forceinline__ uint32_t ufl(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ int ufl(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t ufl64(uint64_t v) {
    return ((uint64_t)ufl((uint32_t)(v >> 32)) << 32) | ufl((uint32_t)v);
}
__device__ __forceinline__ Fx ufx(Fx v) { return Fx{ufl64(v.hi), ufl64(v.lo)}; }

// ---------------------------------------------------------------------------
// Network program in LDS
// ---------------------------------------------------------------------------
struct SNet {
    int32_t m, n, np, R;
    int32_t nf[kMaxM];
    int32_t fkind[kMaxM][kMaxF], fsp[kMaxM][kMaxF], ford[kMaxM][kMaxF];
    int32_t fhint[kMaxM][kMaxF], fhp[kMaxM][kMaxF], fp2[kMaxM][kMaxF], fp3[kMaxM][kMaxF];
    int32_t rate_param[kMaxM];
    int32_t stoich[kMaxM][kMaxS];
    int32_t rw[kMaxS];
    int32_t hist_lo[kMaxS], hist_nb[kMaxS];
    int32_t use_rer, pad;
    int64_t theta;
    int64_t hist_stride[kMaxS];
    double k[kMaxM];
    double kappa[kMaxM];
    double fK[kMaxM][kMaxF];
    double c[kMaxP], ceps[kMaxP];
};

__device__ __forceinline__ int small_int_exponent(double h) {
    return (h >= 0.0 && h <= 64.0 && h == floor(h)) ? (int)h : -1;
}

__device__ void load_net(SNet& S, const DevInst* I) {
    const DevNet& N = I->net;
    S.m = N.n_reactions;
    S.n = N.n_species;
    S.np = N.n_params;
    S.R = I->R;
    S.use_rer = I->use_rer;
    S.theta = I->region_theta;
    for (int p = 0; p < kMaxP; ++p) {
        S.c[p] = I->c[p];
        S.ceps[p] = I->c[p] * (1.0 + I->rer_eps[p]);
    }
    for (int i = 0; i < kMaxS; ++i) {
        S.rw[i] = I->region_w[i];
        S.hist_lo[i] = I->hist_lo[i];
        S.hist_nb[i] = I->hist_nb[i];
        S.hist_stride[i] = I->hist_stride[i];
    }
    for (int j = 0; j < kMaxM; ++j) {
        const DevReaction& rx = N.rx[j];
        const bool on = j < N.n_reactions;
        S.nf[j] = on ? rx.n_factors : 0;
        S.rate_param[j] = rx.rate_param;
        S.kappa[j] = rx.kappa;
        // k_j = c_rate kappa, then the parameter factors left to right
        double kj = rx.rate_param >= 0 ? I->c[rx.rate_param] * rx.kappa : rx.kappa;
        for (int f = 0; on && f < rx.n_factors; ++f)
            if (rx.f[f].kind == PARREP_PARAM) kj = kj * I->c[rx.f[f].hill_param];
        S.k[j] = kj;
        for (int i = 0; i < kMaxS; ++i) S.stoich[j][i] = rx.stoich[i];
        for (int f = 0; f < kMaxF; ++f) {
            S.fkind[j][f] = rx.f[f].kind;
            S.fsp[j][f] = rx.f[f].species;
            S.ford[j][f] = rx.f[f].order;
            S.fhp[j][f] = rx.f[f].hill_param;
            S.fp2[j][f] = rx.f[f].param2;
            S.fp3[j][f] = rx.f[f].param3;
            S.fK[j][f] = rx.f[f].K;
            S.fhint[j][f] = (rx.f[f].kind == PARREP_HILL_REP && f < S.nf[j])
                                ? small_int_exponent(I->c[rx.f[f].hill_param])
                                : (rx.f[f].kind == PARREP_HILL_SWITCH ? rx.f[f].order : 0);
        }
    }
}

template <int NS>
__device__ __forceinline__ int pick(const int (&x)[NS], int s) {
    int v = x[0];
#pragma unroll
    for (int i = 1; i < NS; ++i)
        if (s == i) v = x[i];
    return v;
}

__device__ __forceinline__ double hill_pow(double y, int hint, double h) {
    if (hint < 0) return pow(y, h);
    if (hint == 0) return 1.0;
    double q = y;
    for (int i = 1; i < hint; ++i) q = q * y;
    return q;
}

__device__ __forceinline__ double falling(int64_t xs, int order) {
    int64_t p = 1;
    for (int i = 0; i < order; ++i) {
        const int64_t t = xs - i;
        if (t <= 0) return 0.0;
        p *= t;
    }
    return (double)p;
}

// phi of factor f of reaction j at species value xs (main path: exponents from c).
// phi of a switch factor: lo + (hi - lo) q/(1+q), q = (x/K)^n (repeated
// multiplication), with lo, hi, K from cv.
__device__ __forceinline__ double switch_val(int xs, int n, double lo, double hi, double K) {
    const double y = (double)xs / K;
    double q = y;
    for (int i = 1; i < n; ++i) q = q * y;
    const double s = q / (1.0 + q);
    return lo + (hi - lo) * s;
}

__device__ __forceinline__ double factor_val(const SNet& S, int j, int f, int xs) {
    if (S.fkind[j][f] == PARREP_FALLING) return falling(xs, S.ford[j][f]);
    if (S.fkind[j][f] == PARREP_HILL_SWITCH)
        return switch_val(xs, S.ford[j][f], S.c[S.fhp[j][f]], S.c[S.fp2[j][f]],
                          S.c[S.fp3[j][f]]);
    const double y = (double)xs / S.fK[j][f];
    const double q = hill_pow(y, S.fhint[j][f], S.c[S.fhp[j][f]]);
    return 1.0 / (1.0 + q);
}

// lambda_j(x) with an arbitrary parameter vector cv (RER perturbations).
template <int NS>
__device__ double prop_with(const SNet& S, int j, const int (&x)[NS], const double* cv) {
    const int rp = S.rate_param[j];
    double lam = rp >= 0 ? cv[rp] * S.kappa[j] : S.kappa[j];
    for (int f = 0; f < S.nf[j]; ++f)
        if (S.fkind[j][f] == PARREP_PARAM) lam = lam * cv[S.fhp[j][f]];
    for (int f = 0; f < S.nf[j]; ++f) {
        const int kind = S.fkind[j][f];
        if (kind == PARREP_PARAM) continue;
        const int xs = pick<NS>(x, S.fsp[j][f]);
        double phi;
        if (kind == PARREP_FALLING) {
            phi = falling(xs, S.ford[j][f]);
        } else if (kind == PARREP_HILL_SWITCH) {
            phi = switch_val(xs, S.ford[j][f], cv[S.fhp[j][f]], cv[S.fp2[j][f]], cv[S.fp3[j][f]]);
        } else {
            const double h = cv[S.fhp[j][f]];
            const double y = (double)xs / S.fK[j][f];
            phi = 1.0 / (1.0 + hill_pow(y, small_int_exponent(h), h));
        }
        lam = lam * phi;
    }
    return lam;
}

// k_j phi_1(xs): the rate constant times the first state factor at value xs
// (the first steps of prop_with, in its order).
__device__ __forceinline__ double prop_first(const SNet& S, int j, int xs) {
    const int rp = S.rate_param[j];
    double lam = rp >= 0 ? S.c[rp] * S.kappa[j] : S.kappa[j];
    for (int f = 0; f < S.nf[j]; ++f)
        if (S.fkind[j][f] == PARREP_PARAM) lam = lam * S.c[S.fhp[j][f]];
    for (int f = 0; f < S.nf[j]; ++f)
        if (S.fkind[j][f] != PARREP_PARAM) return lam * factor_val(S, j, f, xs);
    return lam;
}

// ---------------------------------------------------------------------------
// Hot-path propensities: uniform per-instance data is read from the
// descriptor (scalar loads); per-lane work is table lookups.
// ---------------------------------------------------------------------------
template <int NS>
__device__ __forceinline__ int xv(const int (&x)[NS], int i) {
    return i < NS ? x[i] : 0;
}

// Add the packed stoichiometric change (int8 per species) to x.
template <int NS>
__device__ __forceinline__ void apply_dx(int (&x)[NS], uint32_t dxp) {
#pragma unroll
    for (int i = 0; i < NS; ++i) x[i] += ((int32_t)(dxp << (24 - 8 * i))) >> 24;
}

// lambda_j(x) by its defining formula (states outside the tables and
// two-factor reactions); exponents are the instance's integral Hill exponents.
template <int NS>
__device__ __forceinline__ double lambda_formula(const DevInst* __restrict__ I, int j,
                                                 const int (&x)[NS]) {
    double lam = I->k[j];  // includes the parameter factors
    const int nf = I->net.rx[j].n_factors;
    for (int f = 0; f < nf; ++f) {
        const DevFactor& fc = I->net.rx[j].f[f];
        if (fc.kind == PARREP_PARAM) continue;
        const int xs = pick<NS>(x, fc.species);
        double phi;
        if (fc.kind == PARREP_FALLING) {
            phi = falling(xs, fc.order);
        } else if (fc.kind == PARREP_HILL_SWITCH) {
            phi = switch_val(xs, fc.order, I->c[fc.hill_param], I->c[fc.param2], I->c[fc.param3]);
        } else {
            const double y = (double)xs / fc.K;
            const int h = I->hexp[j * kMaxF + f];
            double q = 1.0;
            if (h > 0) {
                q = y;
                for (int i = 1; i < h; ++i) q = q * y;
            }
            phi = 1.0 / (1.0 + q);
        }
        lam = lam * phi;
    }
    return lam;
}

// Where the propensity tables of one instance sit in LDS: reaction j's table
// holds states 0..len[j]-1 of its species at ltab[off[j]].
// Narrow kernels (kAll): every reaction has a table of the same length Ls
// (const and padding ones filled with k_j and 0), at off[j] = j Ls, Ls the
// row length cut to what the doubles given to the workgroup allow.
// General kernels: only the table reactions, each with the states of its
// species; when they do not all fit, the longest are cut to a common length
// (bisection on that length).
template <int M>
struct TabLayout {
    int off[M], len[M];
    int Ls;  // narrow kernels: the common length
};

template <int M, bool kAll, long long SPEC = -1>
__device__ __forceinline__ TabLayout<M> tab_layout(const DevInst* __restrict__ I, int avail) {
    TabLayout<M> t;
    if (kAll) {
        const int L = I->tab_L;
        t.Ls = L < avail / M ? L : avail / M;
        // a compiled species map fixes the row stride, so that a lane forms
        // one address per species and every row is an immediate offset
        const int stride = SPEC >= 0 ? kMapStride : t.Ls;
        if (SPEC >= 0 && t.Ls > kMapStride) t.Ls = kMapStride;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            t.off[j] = j * stride;
            t.len[j] = t.Ls;
        }
        return t;
    }
    int need[M];
    int top = 0;
    const int m = I->net.n_reactions;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const uint32_t meta = j < m ? I->jmeta[j] : jmeta_pack(kRxConst, 0, 0, 0, 0);
        need[j] = (meta & 3u) == kRxTable ? I->tab_Lsp[(meta >> 2) & 3u] : 0;
        top = need[j] > top ? need[j] : top;
    }
    auto total_at = [&](int cap) {
        int tot = 0;
#pragma unroll
        for (int j = 0; j < M; ++j) tot += need[j] < cap ? need[j] : cap;
        return tot;
    };
    int cap = top;
    if (total_at(cap) > avail) {
        int lo = 0, hi = top;  // total_at(lo) <= avail < total_at(hi)
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (total_at(mid) <= avail) lo = mid;
            else hi = mid;
        }
        cap = lo;
    }
    int o = 0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        t.off[j] = o;
        t.len[j] = need[j] < cap ? need[j] : cap;
        o += t.len[j];
    }
    t.Ls = 0;
    return t;
}

// Stage the tables in LDS (all threads of the workgroup take part).
template <int M, bool kAll>
__device__ __forceinline__ void stage_tables(const DevInst* __restrict__ I, const TabLayout<M>& t,
                                             double* ltab, int tid, int nthreads) {
    const int L = I->tab_L;
    const int m = I->net.n_reactions;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const uint32_t kind = j < m ? I->jmeta[j] & 3u : kRxConst;
        const double cst = (j < m && kind == kRxConst) ? I->k[j] : 0.0;
        for (int xs = tid; xs < t.len[j]; xs += nthreads)
            ltab[t.off[j] + xs] = kind == kRxTable ? I->tab[j * L + xs] : cst;
    }
}

// Uniform per-instance network data of the event loop, loaded once per
// phase (scalar registers): rate constants, per-reaction kind and species,
// packed stoichiometry, and the LDS propensity tables.  M >= n_reactions;
// reactions m..M-1 are padding with lambda = 0 (adding +0.0 to a partial sum
// changes nothing, so the padding leaves every sum and the selection as is).
template <int M>
struct HotNet {
    uint32_t stoich[M];  // packed eta_j
    uint64_t spack;      // M == 4: eta_j (species 0-1 as int8) in bits 16j..16j+15
    uint32_t species;    // 2 bits per reaction: the species its table is indexed by
    uint32_t kinds;      // 2 bits per reaction: kRxConst..kRxFall
    uint64_t fmeta;      // 8 bits per reaction: first order, tail species, tail order
    int off[M], len[M];  // general kernels: states 0..len[j]-1 of reaction j at ltab[off[j]]
    int Ls;              // narrow kernels: states 0..Ls-1 of every reaction at ltab[j Ls]
    double k[M];         // rate constants (0 for the padding)
    bool any_direct;     // some reaction needs the formula at every state
    int32_t w[kMaxS];    // metastable set: {x : w.x >= theta}
    int64_t theta;
};

template <int M>
__device__ __forceinline__ HotNet<M> load_hot(const DevInst* __restrict__ I,
                                              const TabLayout<M>& t) {
    HotNet<M> h;
    const int m = I->net.n_reactions;
    h.any_direct = false;
    uint32_t sp = 0, kinds = 0;
    uint64_t fm = 0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const uint32_t meta = j < m ? I->jmeta[j] : jmeta_pack(kRxConst, 0, 0, 0, 0);
        h.stoich[j] = j < m ? ufl(I->jstoich[j]) : 0u;
        sp |= ((meta >> 2) & 3u) << (2 * j);
        kinds |= (meta & 3u) << (2 * j);
        fm |= (uint64_t)((meta >> 4) & 0x3Fu) << (8 * j);
        h.any_direct = h.any_direct || ((meta & 3u) == kRxDirect);
        h.off[j] = ufl(t.off[j]);
        h.len[j] = ufl(t.len[j]);
        h.k[j] = j < m ? __longlong_as_double((long long)ufl64(
                             (uint64_t)__double_as_longlong(I->k[j])))
                       : 0.0;
    }
    h.species = ufl(sp);
    h.kinds = ufl(kinds);
    h.fmeta = ufl64(fm);
    h.Ls = ufl(t.Ls);
    uint64_t pk = 0;
#pragma unroll
    for (int j = 0; j < M && j < 4; ++j) pk |= (uint64_t)(h.stoich[j] & 0xFFFFu) << (16 * j);
    h.spack = ufl64(pk);
#pragma unroll
    for (int i = 0; i < kMaxS; ++i) h.w[i] = ufl(I->region_w[i]);
    h.theta = (int64_t)ufl64((uint64_t)I->region_theta);
    return h;
}

// Metastable set of x: 1 if w.x >= theta (one 32x32->64 multiply-add per
// species, weights in scalar registers).
template <int NS, int M>
__device__ __forceinline__ int region_hot(const HotNet<M>& h, const int (&x)[NS]) {
    int64_t d = 0;
#pragma unroll
    for (int i = 0; i < NS; ++i) d += (int64_t)h.w[i] * (int64_t)x[i];
    return d >= h.theta ? 1 : 0;
}

// x_s (order 1) or x_s (x_s - 1) (order 2) as a double: the falling
// factorial of a count x_s >= 0, exact, 0 where it vanishes.
__device__ __forceinline__ double fall12(int xs, uint32_t order) {
    return (double)(order == 2u ? (int64_t)xs * (int64_t)(xs - 1) : (int64_t)xs);
}

// lambda_j(x) on the hot path of the general (not narrow) kernels, by the
// reaction's kind: a constant, a table entry or an inline falling factorial,
// times the tail.  Direct reactions, and table states the LDS does not hold,
// set bit j of *need instead: the caller evaluates the formula for them in
// one rolled loop (rare and divergent; one copy of the formula per event).
template <int NS, int M>
__device__ __forceinline__ double lam_general(const HotNet<M>& h, const double* __restrict__ ltab,
                                              const int (&x)[NS], int j, uint32_t* need) {
    const uint32_t kind = (h.kinds >> (2 * j)) & 3u;
    if (kind == kRxConst) return h.k[j];
    if (kind == kRxDirect) {
        *need |= 1u << j;
        return 0.0;
    }
    const uint32_t fm = (uint32_t)(h.fmeta >> (8 * j)) & 0x3Fu;
    const int xs = pick<NS>(x, (int)((h.species >> (2 * j)) & 3u));
    double lam;
    if (kind == kRxFall) {
        lam = h.k[j] * fall12(xs, fm & 3u);
    } else if ((unsigned)xs < (unsigned)h.len[j]) {
        lam = ltab[h.off[j] + xs];
    } else {
        *need |= 1u << j;
        return 0.0;
    }
    const uint32_t to = (fm >> 4) & 3u;
    if (to != 0u) lam = lam * fall12(pick<NS>(x, (int)((fm >> 2) & 3u)), to);
    return lam;
}

// All M propensities of the general kernels.
template <int NS, int M>
__device__ __forceinline__ void lams_general(const HotNet<M>& h, const DevInst* __restrict__ I,
                                             const double* __restrict__ ltab,
                                             const int (&x)[NS], double (&lam)[M]) {
    uint32_t need = 0;
#pragma unroll
    for (int j = 0; j < M; ++j) lam[j] = lam_general<NS, M>(h, ltab, x, j, &need);
    if (need) {
#pragma unroll 1
        for (int j = 0; j < M; ++j) {
            if (!((need >> j) & 1u)) continue;
            const double v = lambda_formula<NS>(I, j, x);
#pragma unroll
            for (int jj = 0; jj < M; ++jj) lam[jj] = jj == j ? v : lam[jj];
        }
    }
}

// lambda_j(x) of reaction J under the compiled network descriptor D: the
// cases of lam_general with kind, species and tail constants, so that the
// state is read by constant indices (registers, not an indexed private
// array) and the kind dispatch leaves the chain.  Reactions past the
// descriptor's count are the padding (lambda = 0).
template <int NS, int M, long long D, int J>
__device__ __forceinline__ double lam_desc(const HotNet<M>& h, const double* __restrict__ ltab,
                                           const int (&x)[NS], uint32_t* need) {
    constexpr uint32_t meta = desc_meta(D, J);
    constexpr uint32_t kind = meta & 3u;
    constexpr int sp = (int)((meta >> 2) & 3u), ts = (int)((meta >> 6) & 3u);
    constexpr uint32_t o1 = (meta >> 4) & 3u, to = (meta >> 8) & 3u;
    static_assert(sp < NS && ts < NS, "descriptor species beyond the kernel's");
    if constexpr (J >= desc_count(D)) {
        return 0.0;
    } else if constexpr (kind == kRxConst) {
        return h.k[J];
    } else if constexpr (kind == kRxDirect) {
        *need |= 1u << J;
        return 0.0;
    } else {
        const int xs = x[sp];
        double lam;
        if constexpr (kind == kRxFall) {
            lam = h.k[J] * fall12(xs, o1);
        } else {
            const bool in = (unsigned)xs < (unsigned)h.len[J];
            lam = ltab[h.off[J] + (in ? xs : 0)];
            if (!in) *need |= 1u << J;  // replaced by the formula
        }
        if constexpr (to != 0u) lam = lam * fall12(x[ts], to);
        return lam;
    }
}

template <int NS, int M, long long D, int... J>
__device__ __forceinline__ void lams_desc_seq(const HotNet<M>& h, const double* __restrict__ ltab,
                                              const int (&x)[NS], double (&lam)[M],
                                              uint32_t* need, std::integer_sequence<int, J...>) {
    ((lam[J] = lam_desc<NS, M, D, J>(h, ltab, x, need)), ...);
}

// All M propensities under descriptor D (the formula for direct reactions
// and for table states the LDS does not hold, as in lams_general).
template <int NS, int M, long long D>
__device__ __forceinline__ void lams_desc(const HotNet<M>& h, const DevInst* __restrict__ I,
                                          const double* __restrict__ ltab, const int (&x)[NS],
                                          double (&lam)[M]) {
    uint32_t need = 0;
    lams_desc_seq<NS, M, D>(h, ltab, x, lam, &need, std::make_integer_sequence<int, M>{});
    if (need) {
#pragma unroll 1
        for (int j = 0; j < M; ++j) {
            if (!((need >> j) & 1u)) continue;
            const double v = lambda_formula<NS>(I, j, x);
#pragma unroll
            for (int jj = 0; jj < M; ++jj) lam[jj] = jj == j ? v : lam[jj];
        }
    }
}

// lambda_j(x) in the narrow kernels off the fast path: the table when the
// lane's state is inside every table, else the constant or the formula.
template <int NS, int M>
__device__ __forceinline__ double lam_narrow(const HotNet<M>& h, const DevInst* __restrict__ I,
                                             const double* __restrict__ ltab,
                                             const int (&x)[NS], int j, bool inr) {
    const uint32_t kind = j < I->net.n_reactions ? I->jmeta[j] & 3u : (uint32_t)kRxConst;
    if (kind != kRxDirect && inr)
        return ltab[h.off[j] + pick<NS>(x, (int)((h.species >> (2 * j)) & 3u))];
    if (kind == kRxConst) return I->k[j];
    return lambda_formula<NS>(I, j, x);
}

// n / a for the waiting time: n times 1/a, the reciprocal refined from the
// hardware approximation by two Newton steps.  Within 1.5 ulp of the exact
// quotient for the positive, finite a0 of a Gillespie step (the IEEE
// division takes four more instructions for its range scaling and its
// correctly rounded result); with the -log routine's own error the device's
// tau is within 3.5 ulp of the oracle's log(u)/a0.
__device__ __forceinline__ double waiting_time(double n, double a) {
    double r = __builtin_amdgcn_rcp(a);
    double e = fma(-a, r, 1.0);
    r = fma(r, e, r);
    e = fma(-a, r, 1.0);
    r = fma(r, e, r);
    return n * r;
}

// One Gillespie event at x (the "generate tau and J" step of Alg. 1):
// tau = -log(u_open)/a0 (+inf when absorbing) and the packed change of
// channel J = first j with u_sel*a0 < S_j, S_j the left-to-right partial
// sums.  Every propensity equals the defining formula bit for bit (tables
// hold formula values; inline factors repeat its operations).  Narrow
// kernels read every reaction from a table and take the formula for the
// whole wave when a lane's state is outside the tables (rare) or a reaction
// is direct; the general kernels decide per reaction.
template <int NS, int M, long long SPEC = -1>
__device__ __forceinline__ void event_from_uniforms(const HotNet<M>& h,
                                                    const DevInst* __restrict__ I,
                                                    const double* __restrict__ ltab,
                                                    const int (&x)[NS], double neglog_u_open,
                                                    double u_sel_v, double& tau, int& J,
                                                    uint32_t& dxp, double* a0_out = nullptr) {
    constexpr bool kNarrowK = narrow_kernel(NS, M);
    double cum[M];
    double s = 0.0;
    bool inr = true;
    if (kNarrowK) {
#pragma unroll
        for (int i = 0; i < NS; ++i) inr = inr && (unsigned)x[i] < (unsigned)h.Ls;
        if (__builtin_expect(__ballot(!inr) == 0ull && !h.any_direct, 1)) {
            if constexpr (SPEC >= 0 && kNarrowK) {
                // reaction j reads its row at the state of species (SPEC >> j) & 1
                const double* t0 = ltab + x[0];
                const double* t1 = ltab + x[NS > 1 ? 1 : 0];
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    const double lam = (((SPEC >> j) & 1) ? t1 : t0)[j * kMapStride];
                    s = j == 0 ? lam : s + lam;
                    cum[j] = s;
                }
            } else {
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    const int xs = pick<NS>(x, (int)((h.species >> (2 * j)) & 3u));
                    const double lam = ltab[j * h.Ls + xs];
                    s = j == 0 ? lam : s + lam;  // 0 + lam_1 = lam_1 (lam_1 >= 0)
                    cum[j] = s;
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const double lam = lam_narrow<NS, M>(h, I, ltab, x, j, inr);
                s = j == 0 ? lam : s + lam;
                cum[j] = s;
            }
        }
    } else if constexpr (SPEC >= 0) {
        // the padding past the descriptor's count adds nothing (s + 0.0 = s
        // for the non-negative partial sums), so it is left out
        double lam[M];
        lams_desc<NS, M, SPEC>(h, I, ltab, x, lam);
#pragma unroll
        for (int j = 0; j < M; ++j) {
            s = j == 0 ? lam[j] : (j < desc_count(SPEC) ? s + lam[j] : s);
            cum[j] = s;
        }
    } else {
        double lam[M];
        lams_general<NS, M>(h, I, ltab, x, lam);
#pragma unroll
        for (int j = 0; j < M; ++j) {
            s = j == 0 ? lam[j] : s + lam[j];
            cum[j] = s;
        }
    }
    if (a0_out) *a0_out = s;
    tau = waiting_time(neglog_u_open, s);
    const double t = u_sel_v * s;
    // With at most two species and four reactions every eta_j fits 16 bits
    // of one 64-bit scalar: J is found by counting and eta_J by a shift.
    constexpr bool kNarrow = kNarrowK;
    int pj;
    uint32_t d;
    if (kNarrow) {
        // partial sums do not decrease, so the first j with t < S_j is the
        // number of S_j <= t; zero channels (S_j = S_{j-1}) are skipped
        pj = 0;
#pragma unroll
        for (int j = 0; j < M - 1; ++j) pj += t >= cum[j] ? 1 : 0;
        d = (uint32_t)(h.spack >> (16 * pj)) & 0xFFFFu;
    } else {
        pj = -1;
        d = 0;
#pragma unroll
        for (int j = M - 1; j >= 0; --j) {
            if (t < cum[j]) {
                pj = j;
                d = h.stoich[j];
            }
        }
    }
    // Off the common path: no partial sum above t.  For a finite a0 > 0,
    // t = u_sel a0 < a0 always (u_sel <= 1 - 2^-53), so this is a0 = 0 (an
    // absorbing state: tau = +inf and no jump; NaN counts as 0) or a0 not
    // finite (the last channel with lambda > 0).
    if (__builtin_expect(!(t < cum[M - 1]), 0)) {
        if (!(s > 0.0)) {
            tau = __builtin_inf();
            pj = -1;
            d = 0;
        } else {
            uint32_t pos = 0;
            double lam[M];
            if constexpr (kNarrowK) {
#pragma unroll
                for (int j = 0; j < M; ++j) lam[j] = lam_narrow<NS, M>(h, I, ltab, x, j, inr);
            } else if constexpr (SPEC >= 0) {
                lams_desc<NS, M, SPEC>(h, I, ltab, x, lam);
            } else {
                lams_general<NS, M>(h, I, ltab, x, lam);
            }
#pragma unroll
            for (int j = 0; j < M; ++j)
                if (lam[j] > 0.0) pos |= 1u << j;
            pj = 31 - __clz(pos);
            d = I->jstoich[pj];
        }
    }
    J = pj;
    dxp = d;
}

template <int NS, int M, long long SPEC = -1>
__device__ __forceinline__ void ssa_event(const HotNet<M>& h, const DevInst* __restrict__ I,
                                          const double* __restrict__ ltab,
                                          const double* __restrict__ lgt, const int (&x)[NS],
                                          const Blk& b, double& tau, int& J, uint32_t& dxp,
                                          double* a0_out = nullptr) {
    event_from_uniforms<NS, M, SPEC>(h, I, ltab, x, neglog_u_open(b, lgt), u_sel(b), tau, J, dxp,
                               a0_out);
}

// The two uniforms of one Gillespie step: -log(u_open) and u_sel.
struct Uni {
    double nl, us;
};
__device__ __forceinline__ Uni uniforms(const Blk& b, const double* __restrict__ lgt) {
    return Uni{neglog_u_open(b, lgt), u_sel(b)};
}

__device__ __forceinline__ double readlane_f64(double v, int j) {
    const uint64_t bits = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)bits, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(bits >> 32), j);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Metastable set of x: 1 if w.x >= theta, else 0 (weights of +-1 and 0 take
// additions only; the weights are uniform, so the branches are scalar).
template <int NS>
__device__ __forceinline__ int region_of(const DevInst* __restrict__ I, const int (&x)[NS]) {
    int64_t d = 0;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const int w = I->region_w[i];
        const int64_t xi = x[i];
        if (w == 1) d += xi;
        else if (w == -1) d -= xi;
        else if (w != 0) d += (int64_t)w * xi;
    }
    return d >= I->region_theta ? 1 : 0;
}

// Buffers reached through the instance descriptor's pointers are device
// (global) memory.  Saying so with address space 1 makes the compiler issue
// global_* instead of flat_* instructions: a flat access also counts against
// the LDS counter, so every later LDS wait (each barrier of a round) would
// wait for the HBM round trip of the round's histogram atomics.
template <class T>
using gptr_t = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr_t<T> gmem(T* p) {
    return (gptr_t<T>)p;
}
// Relaxed device-scope atomic adds and compare-and-swap in global memory
// (no return value needed for the adds).
__device__ __forceinline__ void gadd(double* p, double v) {
    __hip_atomic_fetch_add(gmem(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gadd(unsigned long long* p, unsigned long long v) {
    __hip_atomic_fetch_add(gmem(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long gcas(unsigned long long* p, unsigned long long expect,
                                                   unsigned long long v) {
    __hip_atomic_compare_exchange_strong(gmem(p), &expect, v, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return expect;
}

template <int NS>
__device__ __forceinline__ int64_t hist_index(const DevInst* __restrict__ I, const int (&x)[NS]) {
    // branch-free, so that the box's parameters load together (one wait)
    int64_t idx = 0;
    bool in = true;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const int64_t o = (int64_t)x[i] - I->hist_lo[i];
        in = in & ((uint64_t)o < (uint64_t)(int64_t)I->hist_nb[i]);
        idx += o * I->hist_stride[i];
    }
    return in ? idx : -1;
}

// Time at a state outside the histogram box: totals plus a slot of the
// instance's spill table; counted in the overflow counter if no slot is free
// (or a species is outside 0..32767).
template <int NS>
__device__ __forceinline__ void spill_credit(const DevInst* __restrict__ I, const int (&x)[NS], double full,
                             double w) {
    gadd(&I->acc[kAccOutside], full);
    if (w > 0.0) gadd(&I->acc[kAccOutsideW], w);
    unsigned long long key = 1ull << 63;
    bool ok = true;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        ok = ok && x[i] >= 0 && x[i] <= 32767;
        key |= (unsigned long long)(x[i] & 0x7FFF) << (15 * i);
    }
    if (ok) {
        uint32_t h = (uint32_t)(key ^ (key >> 29)) * 0x9E3779B1u;
        for (int probe = 0; probe < kSpillCap; ++probe) {
            SpillSlot* sl = &I->spill[(h + probe) & (kSpillCap - 1)];
            const unsigned long long old = gcas(&sl->key, 0ull, key);
            if (old == 0ull || old == key) {
                gadd(&sl->full, full);
                if (w > 0.0) gadd(&sl->w, w);
                return;
            }
        }
    }
    gadd((unsigned long long*)&I->counters[PARREP_CNT_SPILL_OVERFLOW], 1ull);
}

// Credit `full` time at x over [0,T] and `w` of it inside [t_burn, T].
template <int NS>
__device__ __forceinline__ void add_credit(const DevInst* __restrict__ I, const int (&x)[NS],
                                           double full, double w) {
    const int64_t idx = hist_index<NS>(I, x);
    if (idx >= 0) {
        // Until the finalize kernel adds the window histogram to it, hist
        // holds only the time before t_burn: one atomic per credit except
        // for the interval that straddles t_burn (w <= full always).
        if (w > 0.0) {
            gadd(&I->hist_w[idx], w);
            const double pre = full - w;
            if (pre > 0.0) gadd(&I->hist[idx], pre);
        } else {
            gadd(&I->hist[idx], full);
        }
    } else {
        spill_credit<NS>(I, x, full, w);
    }
}

// Credit tau at x wholly on one side of t_burn: to hist_w after it (win),
// to hist before it.  A non-boundary parallel round lies on one side for the
// whole workgroup, so the side is a uniform branch.  Same sums as
// add_credit(x, tau, win ? tau : 0) (a zero tau adds +0 to either).
template <int NS>
__device__ __forceinline__ void credit_side(const DevInst* __restrict__ I, const int (&x)[NS],
                                            double tau, bool win) {
    const int64_t idx = hist_index<NS>(I, x);
    if (idx >= 0) gadd(&(win ? I->hist_w : I->hist)[idx], tau);
    else spill_credit<NS>(I, x, tau, win ? tau : 0.0);
}

// The generic crediting rule for one holding interval [C, C + tau) at x,
// truncated at the horizon; returns true when the horizon is reached.
template <int NS>
__device__ __forceinline__ bool credit_event(const DevInst* __restrict__ I, const int (&x)[NS],
                                             double tau, Fx C, Fx Tq, Fx tbq, bool accum,
                                             Fx& Cout) {
    const Fx tq = fx_from(tau);
    Fx E = fx_add(C, tq);
    bool hit = false;
    double full = tau;
    if (fx_ge(E, Tq)) {
        hit = true;
        E = Tq;
        full = fx_to_f64(fx_sub(E, C));
    }
    double w;
    if (fx_ge(tbq, E)) w = 0.0;
    else if (fx_ge(C, tbq)) w = full;
    else w = fx_to_f64(fx_sub(E, tbq));
    if (accum) add_credit<NS>(I, x, full, w);
    Cout = E;
    return hit;
}


// ---------------------------------------------------------------------------
// Histogram staging tile (LDS)
// ---------------------------------------------------------------------------
// Bins [a0, a0 + n0) x [a1, a1 + n1) of the histogram (absolute states; one
// species: n1 = 1), row-major in LDS; kept for one parallel step.
struct TileWin {
    int a0, a1, n0, n1;
};

template <int NS>
__device__ __forceinline__ int tile_slot(const TileWin& t, const int (&x)[NS]) {
    const int d0 = x[0] - t.a0;
    const int d1 = NS > 1 ? x[NS > 1 ? 1 : 0] - t.a1 : 0;
    return ((unsigned)d0 < (unsigned)t.n0 && (unsigned)d1 < (unsigned)t.n1) ? d0 * t.n1 + d1 : -1;
}

// Add the tile to hist (before the burn-in time) or hist_w (after), one
// atomic per visited bin, consecutive threads on consecutive bins of a row,
// and clear it.  The whole workgroup takes part.
template <int NS>
__device__ __attribute__((noinline)) void flush_tile(const DevInst* __restrict__ I, double* tile, const TileWin& t,
                           bool win, int tid, int nthreads) {
    __syncthreads();
    double* tgt = win ? I->hist_w : I->hist;
    const int64_t s0 = I->hist_stride[0];
    const int64_t s1 = NS > 1 ? I->hist_stride[1] : 0;
    const int64_t base = (int64_t)(t.a0 - I->hist_lo[0]) * s0 +
                         (NS > 1 ? (int64_t)(t.a1 - I->hist_lo[1]) * s1 : 0);
    const int n = t.n0 * t.n1;
    for (int i = tid; i < n; i += nthreads) {
        const double v = tile[i];
        if (v != 0.0) {
            const int d0 = i / t.n1, d1 = i - d0 * t.n1;
            gadd(&tgt[base + d0 * s0 + d1 * s1], v);
            tile[i] = 0.0;
        }
    }
    __syncthreads();
}

// Place the tile for a parallel step on the replicas' states: centred on
// their mean, n1 = 16 bins along the second species when the first spreads
// more (64 otherwise), clamped to the histogram box.  Every thread returns
// the same window (the partial sums are combined in one order).
template <int NS, int RPL, int WAVES>
__device__ __attribute__((noinline)) TileWin place_tile(const DevInst* __restrict__ I, double* tile, const int (&Y)[RPL][NS],
                              int R, int tid, int lane, int wid) {
    constexpr int B = 64 * WAVES;
    constexpr int kUK = RPL <= 16 ? RPL : 1;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll kUK
    for (int k = 0; k < RPL; ++k) {
        if (k * B + tid < R) {
#pragma unroll
            for (int i = 0; i < NS && i < 2; ++i) {
                const double x = (double)Y[k][i];
                s[i] += x;
                s[2 + i] += x * x;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
        for (int off = 32; off >= 1; off >>= 1) s[q] += __shfl_xor(s[q], off);
    if (lane == 0)
        for (int q = 0; q < 4; ++q) tile[wid * 4 + q] = s[q];
    __syncthreads();
    double S[4] = {0.0, 0.0, 0.0, 0.0};
    for (int w = 0; w < WAVES; ++w)
        for (int q = 0; q < 4; ++q) S[q] += tile[w * 4 + q];
    __syncthreads();
    if (lane == 0)
        for (int q = 0; q < 4; ++q) tile[wid * 4 + q] = 0.0;
    const double m0 = S[0] / R, m1 = S[1] / R;
    const double v0 = S[2] / R - m0 * m0, v1 = S[3] / R - m1 * m1;
    const int nb0 = I->hist_nb[0], nb1 = NS > 1 ? I->hist_nb[1] : 1;
    int n1 = NS > 1 ? min(nb1, v0 >= v1 ? 16 : 64) : 1;
    const int n0 = min(nb0, kTileDoubles / n1);
    if (NS > 1) n1 = min(nb1, kTileDoubles / n0);
    const int c0 = (int)floor(m0) - I->hist_lo[0] - n0 / 2;
    const int c1 = NS > 1 ? (int)floor(m1) - I->hist_lo[1] - n1 / 2 : 0;
    TileWin t;
    t.n0 = n0;
    t.n1 = n1;
    t.a0 = I->hist_lo[0] + max(0, min(c0, nb0 - n0));
    t.a1 = NS > 1 ? I->hist_lo[1] + max(0, min(c1, nb1 - n1)) : 0;
    t.a0 = __builtin_amdgcn_readfirstlane(t.a0);
    t.a1 = __builtin_amdgcn_readfirstlane(t.a1);
    t.n0 = __builtin_amdgcn_readfirstlane(t.n0);
    t.n1 = __builtin_amdgcn_readfirstlane(t.n1);
    return t;
}

// ---------------------------------------------------------------------------
// Workgroup communication
// ---------------------------------------------------------------------------
template <int E, int WAVES>
struct Shared {
    int32_t flags[2][WAVES];
    int32_t wmin[2][WAVES];
    uint64_t wsum[2][WAVES][3];
    uint64_t mask[2][E];
    int32_t cnt[2][E];
    int32_t bi[16];
    uint64_t bu[8];
    int64_t e2[2][WAVES];  // chunked dephasing: each wave's first exit round
};

__device__ __forceinline__ Fx shfl_xor_fx(Fx v, int off) {
    return Fx{__shfl_xor(v.hi, off), __shfl_xor(v.lo, off)};
}

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(v, off);
        if (lane >= off) v += t;
    }
    return v;
}

// Position of the k-th (0-based) set bit of m.
__device__ __forceinline__ int select_bit(uint64_t m, int k) {
    int pos = 0;
#pragma unroll
    for (int width = 32; width >= 1; width >>= 1) {
        const uint64_t low = m & ((1ull << width) - 1ull);
        const int c = __popcll(low);
        if (k >= c) {
            k -= c;
            m >>= width;
            pos += width;
        }
    }
    return pos;
}

// Wave-wide reduction by DPP (data moved between lanes by the VALU, no
// LDS round trip): xor 1 and xor 2 within quads, the mirror within 8 and
// within 16 lanes (every lane of a row then holds the row's value), lane 15
// of rows 0 and 2 into rows 1 and 3, lane 31 into rows 2 and 3; lane 63
// ends with the whole wave's.  Lanes of rows a step leaves out combine with
// the identity.  Every lane of the wave must be active.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp32(uint32_t identity, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)identity, (int)v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
    return ((uint64_t)dpp32<CTRL, ROWS>(0u, (uint32_t)(v >> 32)) << 32) |
           dpp32<CTRL, ROWS>(0u, (uint32_t)v);
}

// A minimum and an exact sum of 64.64 times in three parts that cannot
// overflow over 1024 lanes: the high words (each at most 2^52) and the two
// 32-bit halves of the low words.
struct MinSum3 {
    int m;
    uint64_t a, b, c;
};

template <int CTRL, int ROWS>
__device__ __forceinline__ void min_sum_step(MinSum3& r) {
    r.m = min(r.m, (int)dpp32<CTRL, ROWS>((uint32_t)INT_MAX, (uint32_t)r.m));
    r.a += dpp64<CTRL, ROWS>(r.a);
    r.b += dpp64<CTRL, ROWS>(r.b);
    r.c += dpp64<CTRL, ROWS>(r.c);
}

__device__ __forceinline__ MinSum3 wave_min_sum(int vmin, Fx v) {
    MinSum3 r{vmin, v.hi, v.lo >> 32, v.lo & 0xFFFFFFFFull};
    min_sum_step<0xB1, 0xF>(r);   // quad_perm [1,0,3,2]
    min_sum_step<0x4E, 0xF>(r);   // quad_perm [2,3,0,1]
    min_sum_step<0x141, 0xF>(r);  // row_half_mirror
    min_sum_step<0x140, 0xF>(r);  // row_mirror
    min_sum_step<0x142, 0xA>(r);  // row_bcast:15
    min_sum_step<0x143, 0xC>(r);  // row_bcast:31
    return r;
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int j) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}

// Workgroup-wide minimum of vmin and clamped exact sum of vsum (every lane
// of the workgroup takes part; one barrier).
template <int E, int WAVES>
__device__ __forceinline__ void block_min_sum(Shared<E, WAVES>& sh, int& par, int wid, int lane,
                                              int vmin, Fx vsum, int& omin, Fx& osum) {
    const MinSum3 r = wave_min_sum(vmin, vsum);
    const int wm = __builtin_amdgcn_readlane(r.m, 63);
    const uint64_t wa = readlane_u64(r.a, 63), wb = readlane_u64(r.b, 63),
                   wc = readlane_u64(r.c, 63);
    if (WAVES == 1) {
        omin = wm;
        osum = fx_join3(wa, wb, wc);
        return;
    }
    const int p = par;
    par ^= 1;
    if (lane == 0) {
        sh.wmin[p][wid] = wm;
        sh.wsum[p][wid][0] = wa;
        sh.wsum[p][wid][1] = wb;
        sh.wsum[p][wid][2] = wc;
    }
    __syncthreads();
    omin = INT_MAX;
    uint64_t a = 0, b = 0, c = 0;
    // partly unrolled: with 16 waves a full unroll keeps every partial live
#pragma unroll 4
    for (int w = 0; w < WAVES; ++w) {
        omin = min(omin, sh.wmin[p][w]);
        a += sh.wsum[p][w][0];
        b += sh.wsum[p][w][1];
        c += sh.wsum[p][w][2];
    }
    osum = fx_join3(a, b, c);
}

template <int NS>
__device__ void log_cycle(const DevInst* I, int64_t i, int64_t cyc, int64_t s1, int64_t s2,
                          int64_t s3, int64_t K, int64_t phase, const int (&x)[NS]) {
    if (!I->cycle_log || i >= I->cycle_log_cap) return;
    int64_t* rec = I->cycle_log + i * PARREP_CYCLE_REC;
    rec[0] = cyc;
    rec[1] = s1;
    rec[2] = s2;
    rec[3] = s3;
    rec[4] = K;
    rec[5] = phase;
    for (int k = 0; k < 4; ++k) rec[6 + k] = k < NS ? (int64_t)pick<NS>(x, k) : 0;
    rec[10] = 0;
    rec[11] = 0;
}

// ---------------------------------------------------------------------------
// Per-instance run state that only changes between phases or rarely; kept in
// LDS (written by thread 0, read after barriers) so that it does not occupy
// vector registers in the replica loops.
// ---------------------------------------------------------------------------
struct RunState {
    uint64_t C_hi, C_lo;
    uint64_t clk[4], clk_mark;  // phase wall-clock accounting (thread 0)
    uint64_t Tq_hi, Tq_lo, tbq_hi, tbq_lo;  // horizon and burn-in time, 64.64
    int64_t ev_total;
    int64_t c_decorr, c_dephase, c_cred, c_disc, c_cycles, c_s3, c_s2, c_fv, n_log;
    int64_t s1_events;
    int32_t cycle, W, stop, end_phase;
    int32_t xt[kMaxS], xend[kMaxS];
};

// S1, decorrelation (Alg. 1), run by one wave in batches of 64 steps.  Lane
// i draws step k+i's Philox block and -log(u_open).  A uniform chain then
// follows the jump chain alone (propensities, selection, jump, metastable
// set) and leaves event j in lane j: its pre- and post-jump states and a0.
// The lanes take the waiting times tau_j = -log(u_j)/a0_j and the exact 64.64
// clock by an integer prefix scan; the horizon and the time-in-W rule
// (summed in event order, as defined) fix how many of the batch's events
// belong to S1, and those are credited in parallel.  Events past the end of
// S1 leave no trace: the next draw continues at the first unused step.
__device__ __forceinline__ Fx shfl_up_fx(Fx v, int off) {
    return Fx{__shfl_up(v.hi, off), __shfl_up(v.lo, off)};
}
__device__ __forceinline__ Fx readlane_fx(Fx v, int j) {
    const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v.hi >> 32), j);
    const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v.hi, j);
    const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v.lo >> 32), j);
    const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v.lo, j);
    return Fx{((uint64_t)a << 32) | b, ((uint64_t)c << 32) | d};
}

template <int NS, int M, long long SPEC = -1>
__device__ __forceinline__ void decorrelate(const HotNet<M>& h, const DevInst* __restrict__ I,
                                            const double* __restrict__ ltab,
                                            const double* __restrict__ lgt, RunState& rs, Fx Tq,
                                            Fx tbq, int64_t max_ev, uint32_t key0, uint32_t key1,
                                            int lane, bool accum = true) {
    const bool steps = I->decorr_mode == PARREP_STEPS;
    const int64_t n_c = (int64_t)I->decorr;
    const double t_c = I->decorr;
    int x[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) x[i] = rs.xt[i];
    int W = rs.W;
    const uint32_t cycle = (uint32_t)rs.cycle;
    Fx C{rs.C_hi, rs.C_lo};
    int64_t ev = rs.ev_total;
    int64_t Nc = 0, k = 0;
    double e = 0.0;
    int stop = 0;
    for (;;) {
        // before each step: the set kept long enough ends S1; then the budget
        if (steps ? (Nc >= n_c) : (e >= t_c)) break;
        if (ev + 1 > max_ev) {
            stop = 9;
            break;
        }
        const Blk b = draw((uint64_t)(k + lane), 0u, cycle, kTagDecorr, key0, key1);
        const double nl_l = neglog_u_open(b, lgt);
        const double us_l = u_sel(b);

        // The jump chain (uniform): event j's data go to lane j.
        const int W0 = W;
        int nb = 0;
        double a0_l = 0.0;
        int xpre_l[NS], xpost_l[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) xpre_l[i] = xpost_l[i] = x[i];
        uint64_t rgmask = 0;
        for (int j = 0; j < 64; ++j) {
            if (j > 0) {
                if (steps && Nc >= n_c) break;  // (time mode: decided below)
                if (ev + j + 1 > max_ev) break;
            }
            double a0, tau_unused;
            int J;
            uint32_t dxp;
            event_from_uniforms<NS, M, SPEC>(h, I, ltab, x, 0.0, readlane_f64(us_l, j), tau_unused, J,
                                       dxp, &a0);
            const bool me = lane == j;
            a0_l = me ? a0 : a0_l;
#pragma unroll
            for (int i = 0; i < NS; ++i) xpre_l[i] = me ? x[i] : xpre_l[i];
            apply_dx<NS>(x, dxp);
#pragma unroll
            for (int i = 0; i < NS; ++i) xpost_l[i] = me ? x[i] : xpost_l[i];
            const int rg = region_hot<NS, M>(h, x);
            rgmask |= (uint64_t)rg << j;
            if (steps) {
                if (rg == W) {
                    Nc += 1;
                } else {
                    W = rg;
                    Nc = 0;
                }
            }
            nb = j + 1;
            if (!(a0 > 0.0)) break;  // absorbing: the horizon ends the run here
        }

        // Waiting times and the exact clock before / after each event.
        const bool act = lane < nb;
        const double tau_l = act ? (a0_l > 0.0 ? waiting_time(nl_l, a0_l) : __builtin_inf()) : 0.0;
        const Fx fx_l = act ? fx_from(tau_l) : Fx{0, 0};
        Fx inc = fx_l;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const Fx t = shfl_up_fx(inc, off);
            if (lane >= off) inc = fx_add(inc, t);
        }
        const Fx cpost_l = fx_add(C, inc);
        const Fx cpre_l = fx_sub(cpost_l, fx_l);
        const uint64_t hits = __ballot(act && fx_ge(cpost_l, Tq));
        const int jh = hits ? __ffsll((unsigned long long)hits) - 1 : 64;
        int n_eff = jh < nb ? jh + 1 : nb;
        if (!steps) {
            // time in the current set, in event order; the horizon (credited
            // before the jump) comes first within an event
            int Wc = W0;
            for (int j = 0; j < n_eff; ++j) {
                if (j == jh) break;
                const int rg = (int)((rgmask >> j) & 1u);
                if (rg == Wc) {
                    e = e + readlane_f64(tau_l, j);
                } else {
                    Wc = rg;
                    e = 0.0;
                }
                if (e >= t_c) {
                    n_eff = j + 1;
                    break;
                }
            }
        }
        if (lane < n_eff) {
            Fx cn;
            credit_event<NS>(I, xpre_l, tau_l, cpre_l, Tq, tbq, accum, cn);
        }
        const int last = n_eff - 1;
        ev += n_eff;
        k += n_eff;
        if (jh == last) {  // the horizon: the run ends before this event's jump
            C = Tq;
#pragma unroll
            for (int i = 0; i < NS; ++i) x[i] = __builtin_amdgcn_readlane(xpre_l[i], last);
            W = last > 0 ? (int)((rgmask >> (last - 1)) & 1u) : W0;
            stop = 1;
            break;
        }
        C = readlane_fx(cpost_l, last);
#pragma unroll
        for (int i = 0; i < NS; ++i) x[i] = __builtin_amdgcn_readlane(xpost_l[i], last);
        W = (int)((rgmask >> last) & 1u);
    }
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            rs.xt[i] = x[i];
            if (stop) rs.xend[i] = x[i];
        }
        rs.W = W;
        rs.C_hi = C.hi;
        rs.C_lo = C.lo;
        rs.ev_total = ev;
        rs.c_decorr += k;
        rs.s1_events = k;
        rs.stop = stop;
    }
}

// ---------------------------------------------------------------------------
// The instance kernel: one workgroup runs Alg. 1 for one instance.
// ---------------------------------------------------------------------------
// Occupancy target per shape: with 4 replicas per lane and workgroups of at
// most 4 waves the allocator is asked to fit 5 waves per SIMD (at most 96
// VGPRs; the few spills fall outside the per-event path), which is also what
// the LDS of a 4-wave workgroup allows (5 x 28.6 KB).  Other shapes fit their
// natural size: a 16-wave workgroup puts 4 waves on each SIMD, so a 5-wave
// target would only cap its registers (and spill) for no occupancy.
template <int RPL, int WAVES>
constexpr int kMinWavesPerEU = (RPL == 4 && WAVES <= 4) ? 5 : 1;

// SPEC >= 0: a compiled specialisation.  Narrow kernels: one species map
// (bit j: the species that reaction j's table is read at), with rows at a
// fixed stride.  General kernels: one network descriptor (desc_pack).
// STAGE: the histogram-staging build of the parallel step (narrow kernels,
// at most 4 replicas per lane and 4 waves); the other builds carry none of
// its code, whose calls would add register pressure and spills.
template <int NS, int M, int RPL, int WAVES, long long SPEC = -1, bool STAGE = false>
__device__ __forceinline__ void instance_body(const DevInst* __restrict__ I, int mode,
                                              uint32_t hook_cycle, int64_t hook_max_rounds,
                                              int tab_lds) {
    constexpr int B = 64 * WAVES;
    // With one replica per lane a dephasing or parallel round is one
    // dependent chain per wave, so little hides its latency.  The uniforms
    // come from counter-based draws that do not depend on the state: each
    // round takes the next round's a round ahead (Philox and -log(u) then
    // overlap the event), the same numbers as drawn in place.
    constexpr bool kAhead = RPL == 1;
    // Chunked dephasing (STEPS mode) for the same shapes, with several waves.
    constexpr int kChunkS2 = (RPL == 1 && WAVES > 1) ? 32 : 0;
    constexpr int E = RPL * WAVES;
    // Loops over a lane's replica slots are unrolled up to 16 slots (the
    // per-slot state stays in registers); with 64 slots they stay rolled and
    // the per-slot arrays live in the lane's private memory.
    constexpr int kUK = RPL <= 16 ? RPL : 1;
    using SlotMask = typename std::conditional<(RPL > 32), uint64_t, uint32_t>::type;
    __shared__ RunState rs;
    __shared__ Shared<E, WAVES> sh;
    extern __shared__ int32_t dyn_lds[];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const int R = I->R;
    const uint32_t key0 = I->seed, key1 = I->instance_id;
    const bool accum = mode == kModeSolve;
    // Fleming-Viot exchange: in LDS when the shape's slots fit 32 KiB (the
    // launcher sizes dynamic LDS by the same rule), else global scratch.
    constexpr size_t kXbufBytes = xbuf_lds_bytes(RPL, WAVES, NS);
    constexpr int kXbufInts = (int)(kXbufBytes / 4);
    int32_t* xbuf = kXbufBytes ? dyn_lds : I->xbuf;
    // Propensity tables, copied into LDS after the exchange buffer (the
    // launcher reserved tab_lds doubles for them).
    double* ltab = reinterpret_cast<double*>(dyn_lds + ((kXbufInts + 1) & ~1));
    const TabLayout<M> tl = tab_layout<M, narrow_kernel(NS, M), SPEC>(I, tab_lds);
    stage_tables<M, narrow_kernel(NS, M)>(I, tl, ltab, tid, B);
    __shared__ double lgt[kLogTabLen];
    for (int i = tid; i < kLogTabLen; i += B) lgt[i] = I->logtab[i];
    const HotNet<M> hn = load_hot<M>(I, tl);
    const int64_t max_ev = I->max_events > 0 ? I->max_events : (int64_t(1) << 50);
    int par = 0;

    if (tid == 0) {
        Fx Tq0 = fx_from(I->T), tbq0 = fx_from(I->t_burn);
        if (mode == kModeParallelOnly) {
            Tq0 = Fx{~0ull, ~0ull};
            tbq0 = Tq0;
        }
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
        rs.cycle = mode == kModeSolve ? 0 : (int32_t)hook_cycle;
        rs.stop = rs.end_phase = 0;
        int x[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i)
            x[i] = mode == kModeParallelOnly ? I->hook_states[i] : I->x0[i];
#pragma unroll
        for (int i = 0; i < kMaxS; ++i) rs.xt[i] = rs.xend[i] = i < NS ? x[i] : 0;
        rs.W = region_of<NS>(I, x);
    }
    __syncthreads();

    int Y[RPL][NS];
    for (;;) {
        // ------------------------------------------------------------------
        // S1: decorrelation.
        // ------------------------------------------------------------------
        if (mode == kModeSolve) {
            if (wid == 0) {
                if (lane == 0) rs.clk_mark = wall_clock64();
                // The serial chain is this workgroup's critical path while its
                // other waves wait; raise its issue priority over the waves of
                // other workgroups sharing the SIMD.
                __builtin_amdgcn_s_setprio(3);
                decorrelate<NS, M, SPEC>(hn, I, ltab, lgt, rs, Fx{rs.Tq_hi, rs.Tq_lo},
                                   Fx{rs.tbq_hi, rs.tbq_lo}, max_ev, key0, key1, lane);
                __builtin_amdgcn_s_setprio(0);
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
                    log_cycle<NS>(I, rs.n_log, rs.cycle, rs.s1_events, 0, 0, 0, rs.stop, xe);
                    rs.n_log += 1;
                }
                break;
            }
        }
        const uint32_t cycle = ufl((uint32_t)rs.cycle);
        const int W = ufl(rs.W);
        const bool inW1 = W != 0;  // W is set 0 or set 1
        int xt[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) xt[i] = ufl(rs.xt[i]);

        // ------------------------------------------------------------------
        // S2: dephasing, Fleming-Viot restarts from uniformly chosen survivors.
        // ------------------------------------------------------------------
        int64_t round2 = 0;
        if (mode != kModeParallelOnly) {
            double tr[RPL];
#pragma unroll kUK
            for (int k = 0; k < RPL; ++k) {
#pragma unroll
                for (int i = 0; i < NS; ++i) Y[k][i] = xt[i];
                tr[k] = 0.0;
            }
            const bool steps = I->dephase_mode == PARREP_STEPS;
            // uniform (the conversion from double runs on the vector unit)
            const int64_t n_p = (int64_t)ufl64((uint64_t)(int64_t)I->dephase);
            const double t_p = I->dephase;
            const int64_t left2 = (max_ev - rs.ev_total) / R;
            // round 0's uniforms (one replica per lane: see kAhead)
            Uni ahead{0.0, 0.0};
            if (kAhead && tid < R)
                ahead = uniforms(draw(0, (uint32_t)tid, cycle, kTagDephase, key0, key1), lgt);
            const int64_t budget_rounds = (int64_t)ufl64((uint64_t)(left2 > 0 ? left2 : 0));
            bool done = steps ? (n_p <= 0) : (0.0 >= t_p);
            bool budget = false;
            int64_t fv = 0;
            // One dephasing round n of this thread's replicas: the slots whose
            // replica left W; nd is set when one is still short of t_p.
            // full (a std::integral_constant) is true when every slot of every
            // thread holds a replica (R = RPL * B): no per-slot lane masks
            // (instantiated for RPL = 4, below).
            auto dephase_round = [&](int64_t n, bool& nd, auto full) -> SlotMask {
                SlotMask exitbits = 0;
#pragma unroll (RPL <= 16 ? RPL : 1)
                for (int k = 0; k < RPL; ++k) {
                    const int r = k * B + tid;
                    if (decltype(full)::value || r < R) {
                        Uni u;
                        if constexpr (kAhead) {
                            u = ahead;
                            ahead = uniforms(draw((uint64_t)n + 1, (uint32_t)r, cycle,
                                                  kTagDephase, key0, key1),
                                             lgt);
                        } else {
                            u = uniforms(draw((uint64_t)n, (uint32_t)r, cycle, kTagDephase,
                                              key0, key1),
                                         lgt);
                        }
                        double tau;
                        int J;
                        uint32_t dxp;
                        event_from_uniforms<NS, M, SPEC>(hn, I, ltab, Y[k], u.nl, u.us, tau, J,
                                                         dxp);
                        apply_dx<NS>(Y[k], dxp);
                        tr[k] = tr[k] + tau;
                        // left W: the region (0 or 1) differs from W, as an
                        // exclusive or of two conditions
                        const bool out = (region_hot<NS, M>(hn, Y[k]) != 0) != inW1;
                        exitbits |= (SlotMask)(out ? 1 : 0) << k;
                        nd = nd | !(tr[k] >= t_p);
                    }
                }
                return exitbits;
            };
            // Exact Fleming-Viot restart after round n, in which some replica
            // left W (the whole workgroup takes part): survivors keep their
            // post-round state; each exited replica copies the post-round
            // state of survivor floor(u |S| / 2^32), in ascending replica
            // order.  The exchange buffer and masks are single: the next exit
            // round writes them only after that round's agreement barrier,
            // which every wave reaches after its reads here.
            auto fv_restart = [&](int64_t n, SlotMask exitbits) {
                int32_t* xb = xbuf;
#pragma unroll kUK
                for (int k = 0; k < RPL; ++k) {
                    const int r = k * B + tid;
                    if (r < R) {
#pragma unroll
                        for (int i = 0; i < NS; ++i) xb[r * NS + i] = Y[k][i];
                    }
                    const bool surv = (r < R) && !((exitbits >> k) & 1);
                    const uint64_t m = __ballot(surv);
                    if (lane == 0) {
                        sh.mask[0][k * WAVES + wid] = m;
                        sh.cnt[0][k * WAVES + wid] = __popcll(m);
                    }
                }
                __syncthreads();
                int nS = 0;
                for (int e = 0; e < E; ++e) nS += sh.cnt[0][e];
                nS = ufl(nS);
                if (exitbits) {
#pragma unroll kUK
                    for (int k = 0; k < RPL; ++k) {
                        if (!((exitbits >> k) & 1)) continue;
                        const int r = k * B + tid;
                        if (nS > 0) {
                            const Blk b = draw((uint64_t)n, (uint32_t)r, cycle, kTagFV, key0, key1);
                            int idx = (int)(((uint64_t)b.w0 * (uint64_t)nS) >> 32);
                            int e = 0;
                            for (;;) {
                                const int c = sh.cnt[0][e];
                                if (idx < c) break;
                                idx -= c;
                                ++e;
                            }
                            const int l = select_bit(sh.mask[0][e], idx);
                            const int rr = (e / WAVES) * B + (e % WAVES) * 64 + l;
#pragma unroll
                            for (int i = 0; i < NS; ++i) Y[k][i] = xb[rr * NS + i];
                        } else {
#pragma unroll
                            for (int i = 0; i < NS; ++i) Y[k][i] = xt[i];
                        }
                    }
                }
                fv += R - nS;
            };
            // STEPS mode with one replica per lane (a latency-bound shape):
            // between restarts the waves' replicas are independent and every
            // round's uniforms come from counters, so each wave runs a chunk
            // of up to kChunkS2 rounds with no barrier, stopping at its first
            // round with an exit.  The waves then agree on the first such
            // round; those that ran past it rewind to the chunk's start and
            // replay up to it, which leaves every replica where the round-by-
            // round protocol below would have it.  (The phase's end, n_p
            // rounds, is known in advance in STEPS mode.)
            const bool chunked = kChunkS2 && steps;
            int64_t chunk = 0;
            // round2 never passes budget_rounds or (STEPS mode) n_p: it grows by
            // one per round, and a chunk's length is capped by both.  So the
            // loop's tests are equalities of uniform 64-bit values, which the
            // scalar unit takes (it has no ordered 64-bit compare).
            auto s2_rounds = [&](auto full) {
                while (!done) {
                    if (round2 == budget_rounds) {
                        budget = true;
                        break;
                    }
                    if (chunked) {
                        const int64_t c0 = round2;
                        int64_t L = kChunkS2;
                        L = L < n_p - c0 ? L : n_p - c0;
                        L = L < budget_rounds - c0 ? L : budget_rounds - c0;
                        int Y0[RPL][NS];
#pragma unroll
                        for (int k = 0; k < RPL; ++k)
#pragma unroll
                            for (int i = 0; i < NS; ++i) Y0[k][i] = Y[k][i];
                        const Uni ahead0 = ahead;
                        SlotMask exitbits = 0;
                        int64_t ew = INT64_MAX;
                        bool nd = false;
                        for (int64_t n = c0; n < c0 + L; ++n) {
                            exitbits = dephase_round(n, nd, full);
                            if (__ballot(exitbits != 0) != 0ull) {
                                ew = n;
                                break;
                            }
                        }
                        const int q = (int)(chunk & 1);
                        ++chunk;
                        if (lane == 0) sh.e2[q][wid] = ew;
                        __syncthreads();
                        int64_t ef = INT64_MAX;
#pragma unroll
                        for (int w = 0; w < WAVES; ++w) ef = ef < sh.e2[q][w] ? ef : sh.e2[q][w];
                        ef = (int64_t)ufl64((uint64_t)ef);
                        if (ef == INT64_MAX) {
                            round2 = c0 + L;
                        } else {
                            if (ew != ef) {  // this wave ran past the exit round: replay to it
#pragma unroll
                                for (int k = 0; k < RPL; ++k)
#pragma unroll
                                    for (int i = 0; i < NS; ++i) Y[k][i] = Y0[k][i];
                                ahead = ahead0;
                                for (int64_t n = c0; n <= ef; ++n)
                                    exitbits = dephase_round(n, nd, full);
                            }
                            fv_restart(ef, exitbits);
                            round2 = ef + 1;
                        }
                        done = round2 == n_p;
                        continue;
                    }
                    const int p = (int)(round2 & 1);
                    bool nd = false;
                    const SlotMask exitbits = dephase_round(round2, nd, full);
                    // One barrier per round: each wave posts whether one of its
                    // replicas left W and whether one is still short of t_p.  The
                    // flags alternate between two slots, so the posts of round
                    // n+1 never meet a slow wave's reads of round n.
                    const bool wave_exit = __ballot(exitbits != 0) != 0ull;
                    const bool wave_nd = __builtin_amdgcn_ballot_w64(nd) != 0ull;
                    // The flags are uniform, so every lane stores them (a relaxed
                    // atomic store of one value): no lane-0 mask in the round.
                    const int32_t f = (wave_nd ? 1 : 0) | (wave_exit ? 2 : 0);
                    __hip_atomic_store(&sh.flags[p][wid], f, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                    __syncthreads();
                    int fl = 0;
#pragma unroll
                    for (int w = 0; w < WAVES; ++w) fl |= sh.flags[p][w];
                    fl = ufl(fl);
                    if (fl & 2) fv_restart(round2, exitbits);
                    ++round2;
                    done = steps ? (round2 == n_p) : ((fl & 1) == 0);
                }
            };
            // Compiled for 4 replicas per lane only (the throughput shapes):
            // a second copy of the fully unrolled 16-slot round would double
            // the largest kernels' compile time for shapes that rarely run full.
            if constexpr (RPL == 4) {
                if (R >= RPL * B)
                    s2_rounds(std::true_type{});
                else
                    s2_rounds(std::false_type{});
            } else {
                s2_rounds(std::false_type{});
            }
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
                    log_cycle<NS>(I, rs.n_log, cycle, rs.s1_events, 0, 0, 0, 9, xt);
                    rs.n_log += 1;
                }
                if (mode == kModeDephaseOnly && tid == 0) I->hook_i64[0] = -1;
                break;
            }
            if (mode == kModeDephaseOnly) {
#pragma unroll kUK
                for (int k = 0; k < RPL; ++k) {
                    const int r = k * B + tid;
                    if (r < R) {
#pragma unroll
                        for (int i = 0; i < kMaxS; ++i)
                            I->hook_states[r * kMaxS + i] = i < NS ? Y[k][i] : 0;
                    }
                }
                if (tid == 0) I->hook_i64[0] = round2;
                return;
            }
        } else {
#pragma unroll kUK
            for (int k = 0; k < RPL; ++k) {
                const int r = k * B + tid;
#pragma unroll
                for (int i = 0; i < NS; ++i) Y[k][i] = r < R ? I->hook_states[r * kMaxS + i] : 0;
            }
        }
        __syncthreads();

        // ------------------------------------------------------------------
        // S3: parallel step.  Round n credits keys R(n-1)+r for r < K, the
        // first replica outside W, at the pre-jump states (ParRep-CTMC rule).
        // ------------------------------------------------------------------
        const int64_t left3 = (max_ev - rs.ev_total) / R;
        int64_t budget3 = (int64_t)ufl64((uint64_t)(left3 > 0 ? left3 : 0));
        if (mode == kModeParallelOnly && hook_max_rounds >= 0 && hook_max_rounds < budget3)
            budget3 = hook_max_rounds;
        Fx C = ufx(Fx{rs.C_hi, rs.C_lo});
        const Fx Tq = ufx(Fx{rs.Tq_hi, rs.Tq_lo});
        const Fx tbq = ufx(Fx{rs.tbq_hi, rs.tbq_lo});
        int64_t round3 = 0, cred = 0, disc = 0;
        Uni ahead{0.0, 0.0};
        if (kAhead && tid < R)
            ahead = uniforms(draw(0, (uint32_t)tid, cycle, kTagParallel, key0, key1), lgt);
        int outcome = -1;  // 1 exit, 0 horizon, -1 budget
        int Kx = 0;
        double tauk[RPL];
        uint32_t dxk[RPL];
        // Histogram staging (narrow kernels, full solves): credits of whole
        // rounds at states inside a tile of the histogram box go to an LDS
        // copy of that tile (kTileDoubles bins, after the tables; the
        // launcher reserved it) instead of one HBM atomic each; the tile is
        // flushed with one atomic per visited bin.  Decided here, so that
        // nothing of it is live during the other steps.
        const int stage_flush = I->stage_flush;
        constexpr bool kStageable = STAGE && narrow_kernel(NS, M) && RPL <= 4 && WAVES <= 4;
        const bool stage = kStageable && accum && stage_flush >= 0;
        double* tile = ltab + tab_lds;
        TileWin tw{0, 0, 0, 0};
        bool tile_win = false;  // the tile holds time after the burn-in time
        int since = 0;          // rounds credited to the tile since its last flush
        if (stage) {
            for (int i = tid; i < kTileDoubles; i += B) tile[i] = 0.0;
            tw = place_tile<NS, RPL, WAVES>(I, tile, Y, R, tid, lane, wid);
            tile_win = fx_ge(C, tbq);
        }
        for (;;) {
            if (round3 >= budget3) {
                outcome = -1;
                break;
            }
            Fx lsum{0, 0};
            int lfirst = INT_MAX;
#pragma unroll kUK
            for (int k = 0; k < RPL; ++k) {
                const int r = k * B + tid;
                tauk[k] = 0.0;
                dxk[k] = 0;
                if (r < R) {
                    Uni u;
                    if constexpr (kAhead) {
                        u = ahead;
                        ahead = uniforms(draw((uint64_t)round3 + 1, (uint32_t)r, cycle,
                                              kTagParallel, key0, key1),
                                         lgt);
                    } else {
                        u = uniforms(draw((uint64_t)round3, (uint32_t)r, cycle, kTagParallel,
                                          key0, key1),
                                     lgt);
                    }
                    int J;
                    event_from_uniforms<NS, M, SPEC>(hn, I, ltab, Y[k], u.nl, u.us, tauk[k], J,
                                                     dxk[k]);
                    int post[NS];
#pragma unroll
                    for (int i = 0; i < NS; ++i) post[i] = Y[k][i];
                    apply_dx<NS>(post, dxk[k]);
                    if (region_hot<NS, M>(hn, post) != W && lfirst == INT_MAX) lfirst = r;
                    lsum = fx_add_sat(lsum, fx_from(tauk[k]));
                }
            }
            int first;
            Fx total;
            block_min_sum<E, WAVES>(sh, par, wid, lane, lfirst, lsum, first, total);
            first = ufl(first);
            total = ufx(total);
            ++round3;
            const bool ex = first != INT_MAX;
            const int K = ex ? first + 1 : R;
            if (ex) {
                Fx l2{0, 0};
#pragma unroll kUK
                for (int k = 0; k < RPL; ++k) {
                    const int r = k * B + tid;
                    if (r < K) l2 = fx_add_sat(l2, fx_from(tauk[k]));
                }
                int dummy;
                block_min_sum<E, WAVES>(sh, par, wid, lane, INT_MAX, l2, dummy, total);
                total = ufx(total);
            }
            const Fx Cend = fx_add(C, total);
            const bool boundary = fx_ge(Cend, Tq) || (fx_gt(tbq, C) && fx_gt(Cend, tbq));
            int credited;
            bool hit = false;
            if (!boundary) {
                if (accum) {
                    const bool win = fx_ge(C, tbq);
                    if (stage) {
                        // the tile holds one side of the burn-in time; flush it
                        // when that side changes and every stage_flush rounds
                        if (win != tile_win || (stage_flush > 0 && since >= stage_flush)) {
                            flush_tile<NS>(I, tile, tw, tile_win, tid, B);
                            tile_win = win;
                            since = 0;
                        }
#pragma unroll kUK
                        for (int k = 0; k < RPL; ++k) {
                            const int r = k * B + tid;
                            if (r < K) {
                                const int ts = tile_slot<NS>(tw, Y[k]);
                                if (ts >= 0) atomicAdd(&tile[ts], tauk[k]);
                                else credit_side<NS>(I, Y[k], tauk[k], win);
                            }
                        }
                        ++since;
                    } else {
#pragma unroll kUK
                        for (int k = 0; k < RPL; ++k) {
                            const int r = k * B + tid;
                            if (r < K) credit_side<NS>(I, Y[k], tauk[k], win);
                        }
                    }
                }
                C = Cend;
                credited = K;
            } else {
                // Rare: an exact scan in key order finds where the burn-in
                // time and the horizon fall.
                uint64_t* sb = I->sbuf;
#pragma unroll kUK
                for (int k = 0; k < RPL; ++k) {
                    const int r = k * B + tid;
                    if (r < K) {
                        const Fx tq = fx_from(tauk[k]);
                        sb[4 * r] = tq.hi;
                        sb[4 * r + 1] = tq.lo;
                    }
                }
                __syncthreads();
                if (tid == 0) {
                    Fx s = C;
                    int rend = K - 1, h = 0;
                    for (int r = 0; r < K; ++r) {
                        sb[4 * r + 2] = s.hi;
                        sb[4 * r + 3] = s.lo;
                        s = fx_add(s, Fx{sb[4 * r], sb[4 * r + 1]});
                        if (fx_ge(s, Tq)) {
                            rend = r;
                            h = 1;
                            s = Tq;
                            break;
                        }
                    }
                    sh.bi[0] = rend;
                    sh.bi[1] = h;
                    sh.bu[0] = s.hi;
                    sh.bu[1] = s.lo;
                }
                __syncthreads();
                const int rend = ufl(sh.bi[0]);
                hit = sh.bi[1] != 0;
                const Fx Cn = ufx(Fx{sh.bu[0], sh.bu[1]});
                __syncthreads();
#pragma unroll kUK
                for (int k = 0; k < RPL; ++k) {
                    const int r = k * B + tid;
                    if (r <= rend) {
                        const Fx st{sb[4 * r + 2], sb[4 * r + 3]};
                        Fx dummy;
                        credit_event<NS>(I, Y[k], tauk[k], st, Tq, tbq, accum, dummy);
                        if (hit && r == rend) {
#pragma unroll
                            for (int i = 0; i < NS; ++i) rs.xend[i] = Y[k][i];
                        }
                    }
                }
                C = Cn;
                credited = rend + 1;
                __syncthreads();
            }
            cred += credited;
            if (hit || ex) disc += R - credited;
            if (hit) {
                outcome = 0;
                break;
            }
            if (ex) {
                // X~ <- post-jump state of replica K (1-based), then a new cycle.
#pragma unroll kUK
                for (int k = 0; k < RPL; ++k) {
                    const int r = k * B + tid;
                    if (r == K - 1) {
                        int post[NS];
#pragma unroll
                        for (int i = 0; i < NS; ++i) post[i] = Y[k][i];
                        apply_dx<NS>(post, dxk[k]);
#pragma unroll
                        for (int i = 0; i < NS; ++i) rs.xt[i] = post[i];
                    }
                }
                outcome = 1;
                Kx = K;
                break;
            }
#pragma unroll kUK
            for (int k = 0; k < RPL; ++k) apply_dx<NS>(Y[k], dxk[k]);
        }
        __syncthreads();
        if (stage) flush_tile<NS>(I, tile, tw, tile_win, tid, B);
        if (mode == kModeParallelOnly) {
            if (tid == 0) {
                I->hook_i64[0] = outcome == 1 ? round3 : -1;
                I->hook_i64[1] = outcome == 1 ? Kx : 0;
#pragma unroll
                for (int i = 0; i < kMaxS; ++i) I->hook_exit[i] = i < NS ? rs.xt[i] : 0;
                I->hook_f64[0] = fx_to_f64(C);
            }
            return;
        }
        if (tid == 0) {
            const uint64_t now = wall_clock64();
            rs.clk[2] += now - rs.clk_mark;
            rs.clk_mark = now;
            rs.ev_total += round3 * R;
            rs.c_cred += cred;
            rs.c_disc += disc;
            rs.c_s3 += round3;
            rs.C_hi = C.hi;
            rs.C_lo = C.lo;
            int xl[NS];
            if (outcome == 1) {
#pragma unroll
                for (int i = 0; i < NS; ++i) xl[i] = rs.xt[i];
                log_cycle<NS>(I, rs.n_log, cycle, rs.s1_events, round2, round3, Kx, 3, xl);
                rs.c_cycles += 1;
                rs.W = region_of<NS>(I, xl);
                rs.cycle = (int32_t)(cycle + 1);
            } else {
                rs.end_phase = outcome == 0 ? 3 : 9;
                if (outcome != 0) {
#pragma unroll
                    for (int i = 0; i < NS; ++i) rs.xend[i] = xt[i];
                }
#pragma unroll
                for (int i = 0; i < NS; ++i) xl[i] = rs.xend[i];
                log_cycle<NS>(I, rs.n_log, cycle, rs.s1_events, round2, round3, 0, rs.end_phase,
                              xl);
            }
            rs.n_log += 1;
        }
        __syncthreads();
        if (outcome != 1) break;
    }

    if (tid == 0) {
        int64_t* cn = I->counters;
        cn[PARREP_CNT_EV_DECORR] = rs.c_decorr;
        cn[PARREP_CNT_EV_DEPHASE] = rs.c_dephase;
        cn[PARREP_CNT_EV_PAR_CREDITED] = rs.c_cred;
        cn[PARREP_CNT_EV_PAR_DISCARDED] = rs.c_disc;
        cn[PARREP_CNT_CYCLES] = rs.c_cycles;
        cn[PARREP_CNT_S3_ROUNDS] = rs.c_s3;
        cn[PARREP_CNT_S2_ROUNDS] = rs.c_s2;
        cn[PARREP_CNT_STATUS] = rs.end_phase == 9 ? PARREP_RUN_BUDGET : PARREP_RUN_OK;
        cn[PARREP_CNT_FV_RESTARTS] = rs.c_fv;
        cn[PARREP_CNT_END_PHASE] = rs.end_phase;
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
}

// One workgroup per instance: workgroup b runs instance b.
template <int NS, int M, int RPL, int WAVES, long long SPEC = -1, bool STAGE = false>
__global__ void __launch_bounds__(64 * WAVES)
__attribute__((amdgpu_waves_per_eu(kMinWavesPerEU<RPL, WAVES>, 8)))
k_instance(const DevInst* __restrict__ insts, int mode, uint32_t hook_cycle,
           int64_t hook_max_rounds, int tab_lds) {
    instance_body<NS, M, RPL, WAVES, SPEC, STAGE>(insts + blockIdx.x, mode, hook_cycle,
                                                  hook_max_rounds, tab_lds);
}

// Persistent form of a solve launch: a grid of at most as many workgroups as
// the device holds at once, each taking the next instance from the group's
// counter (next, zeroed before the launch) until all n are taken.  Instances
// run in index order of taking, which the host sorts longest first; each
// runs exactly as in k_instance.
template <int NS, int M, int RPL, int WAVES, long long SPEC = -1>
__global__ void __launch_bounds__(64 * WAVES)
__attribute__((amdgpu_waves_per_eu(kMinWavesPerEU<RPL, WAVES>, 8)))
k_persist(const DevInst* __restrict__ insts, int n, int* next, int tab_lds) {
    __shared__ int take;
    for (;;) {
        if (threadIdx.x == 0) take = atomicAdd(next, 1);
        __syncthreads();
        const int i = take;
        __syncthreads();  // every thread has read take before it changes
        if (i >= n) break;
        instance_body<NS, M, RPL, WAVES, SPEC>(insts + i, kModeSolve, 0, -1, tab_lds);
        __syncthreads();  // the instance's last LDS reads before the next one's writes
    }
}

}  // namespace
}  // namespace dev
}  // namespace parrep
