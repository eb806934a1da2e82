// parrep_internal.h -- device-side descriptors shared by the kernels and the
// C-ABI layer of libparrep (not installed; the public interface is parrep.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/parrep.h"

namespace parrep {

constexpr int kMaxS = PARREP_MAX_SPECIES;
constexpr int kMaxM = PARREP_MAX_REACTIONS;
constexpr int kMaxF = PARREP_MAX_FACTORS;
constexpr int kMaxP = PARREP_MAX_PARAMS;

// Philox counter word 3 carries the phase tag in its top nibble.
enum : uint32_t { kTagDecorr = 1, kTagDephase = 2, kTagFV = 3, kTagParallel = 4 };

struct DevFactor {
    int32_t kind, species, order, hill_param, param2, param3;
    double K;
};

struct DevReaction {
    int32_t rate_param, n_factors;
    double kappa;
    int32_t stoich[kMaxS];
    DevFactor f[kMaxF];
};

struct DevNet {
    int32_t n_species, n_reactions, n_params, reserved;
    DevReaction rx[kMaxM];
};

// Everything one ParRep instance needs on the device: the network, the
// problem, its output buffers and its slice of the scratch arena.
// Time spent at states outside the histogram box, keyed by the packed state
// (15 bits per species, bit 63 marks a used slot); the finalize kernel adds
// their FIM, RER and window-integral contributions.
struct SpillSlot {
    unsigned long long key;
    double full;
    double w;
};
constexpr int kSpillCap = 2048;
// Bins of the LDS histogram tile of the instance kernel (8 KiB).
constexpr int kTileDoubles = 1024;
// Row stride (states) of the propensity tables in the narrow kernels compiled
// for one species map, and the maps compiled: two species with reactions 1
// and 4 read at species 1 and reactions 2 and 3 at species 0 (the toggle
// switch's cross-regulated births and linear deaths).
constexpr int kMapStride = 512;
constexpr int kMapCross = 0b1001;

// Exchange area of one instance spread over several workgroups (the wide
// instance kernel): a grid barrier, the chunk results the workgroups agree
// on (triple-buffered by chunk index), and broadcast states.  k_zero
// initialises it before the kernel runs.
constexpr int kWideS3Max = 64;  // longest parallel-step chunk (rounds)
struct WideSync {
    uint32_t bar;     // barrier arrivals (wraps; compared modulo 2^32)
    uint32_t abort;   // a workgroup gave up waiting: every workgroup leaves
    int64_t rend;     // replica whose holding interval holds the horizon
    int64_t e2[3];    // dephasing chunk: first round with an exit (min)
    int64_t d2[3];    // dephasing chunk: round after which every replica is done (max)
    uint64_t k3[3];   // parallel chunk: first exit key R n + r (min)
    int32_t xb[kMaxS], xf[kMaxS];  // broadcast: exit state; state at the horizon
    uint64_t s3[3][kWideS3Max][3];  // parallel chunk: per-round clock sums, 64.64
                                    // split as (hi, lo >> 32, lo & 0xffffffff)
};

struct DevInst {
    DevNet net;
    double c[kMaxP], rer_eps[kMaxP];
    int32_t use_rer, decorr_mode, dephase_mode, R;
    double decorr, dephase, T, t_burn;
    int32_t x0[kMaxS], region_w[kMaxS];
    int64_t region_theta;
    int32_t hist_lo[kMaxS], hist_nb[kMaxS];
    int64_t hist_stride[kMaxS];
    int64_t nbins;
    uint32_t seed, instance_id;
    int64_t max_events;
    // outputs (caller-owned device memory)
    double* hist;
    double* hist_w;
    double* stats;
    int32_t* x_final;
    int64_t* counters;
    int64_t* cycle_log;
    int32_t cycle_log_cap, reserved;
    int64_t* phase_clock;  // optional: ticks in S1, S2, S3, total
    // hot-path network view (jmeta/jstoich/tab_L filled on the host from the
    // network; k and the tables computed on the device by the setup kernel)
    double k[kMaxM];          // k_j = c[rate_param] * kappa * parameter factors
    uint32_t jmeta[kMaxM];    // hot-path kind of reaction j, see jmeta_* below
    uint32_t jstoich[kMaxM];  // eta_j packed as int8 per species (species i in bits 8i..8i+7)
    int32_t hexp[kMaxM * kMaxF];  // integral exponents: HILL_REP from c, HILL_SWITCH order
    int32_t tab_Lsp[kMaxS];   // table states wanted per indexing species (0..tab_Lsp[s]-1)
    int32_t tab_L;            // row length of tab (max of tab_Lsp)
    int32_t tab_owner;        // 1: this instance's setup block fills the table
    double* tab;              // kMaxM * tab_L: row j holds the table of reaction j
    const double* logtab;     // kLogTabLen: reduction table of -log(u) (context-owned)
    // library scratch
    double* acc;         // kAccLen doubles: outside-box accumulators
    SpillSlot* spill;    // kSpillCap slots: time at states outside the histogram box
    int32_t* xbuf;       // 2 * R * kMaxS: Fleming-Viot state exchange (two rounds)
    uint64_t* sbuf;      // R * 4: boundary-round clock scan (tau, start) as 64.64
    // wide instance kernel only (NULL otherwise)
    WideSync* wide;
    uint64_t* wtot;      // per wave: its replicas' clock sum in the exact round (64.64)
    uint64_t* smask;     // per 64 replicas: survivors of a Fleming-Viot round
    int32_t wide_s2, wide_s3;   // chunk lengths (rounds) of dephasing and parallel step
    int64_t wide_wait_ticks;    // wall-clock ticks a workgroup waits at a grid barrier
    int32_t wide_waves, wide_rpl;  // waves of the launch and replicas per lane (0: not wide)
    // parallel-step histogram staging in LDS (narrow kernels): -1 off (one
    // HBM atomic per credit), 0 flush at the end of the step and at the
    // burn-in time, P > 0 also every P rounds
    int32_t stage_flush, reserved2;
    // test-hook outputs (unused by full solves)
    int32_t* hook_states;   // dephase-only: output states; parallel-only: input states
    int32_t* hook_exit;     // parallel-only: exit state
    int64_t* hook_i64;
    double* hook_f64;
};

// acc[] layout: outside, outside_w, fim[kMaxP*kMaxP], rer[kMaxP], y[kMaxS]
constexpr int kAccOutside = 0, kAccOutsideW = 1, kAccFim = 2, kAccRer = 2 + kMaxP * kMaxP,
              kAccY = kAccRer + kMaxP, kAccLen = kAccY + kMaxS;

// Fleming-Viot exchange buffer of the instance kernel: one post-round state
// per replica slot of the launch shape (rpl * 64 * waves slots, ns ints
// each).  It lives in LDS when it fits 32 KiB, else in global scratch
// (DevInst::xbuf); the kernel and its launchers size it by this rule.
constexpr int xbuf_slot_ints(int rpl, int waves, int ns) { return rpl * 64 * waves * ns; }
constexpr size_t xbuf_lds_bytes(int rpl, int waves, int ns) {
    return (size_t)xbuf_slot_ints(rpl, waves, ns) * 4 <= 32768
               ? (size_t)((xbuf_slot_ints(rpl, waves, ns) + 1) & ~1) * 4
               : 0;
}

// Run modes of the instance kernel.
enum : int32_t { kModeSolve = 0, kModeDephaseOnly = 1, kModeParallelOnly = 2 };

// Hot-path reaction kinds (DevInst::jmeta bits 0-1):
//   const  lambda_j = k_j (no state factor; also the padding reactions)
//   table  lambda_j = T_j[x_s] (T_j[x_s] = k_j * phi_1(x_s), the first state
//          factor, computed by the defining formula), times the tail
//   fall   lambda_j = k_j * x_s (order 1) or k_j * x_s (x_s - 1) (order 2),
//          times the tail (no table)
//   direct the defining formula at every event
// The tail is an optional second state factor, a falling factorial of order
// 1 or 2 multiplied last (the formula's own order of operations, so every
// kind gives the formula's value bit for bit).  Kernels specialised for at
// most 2 species and 4 reactions ("narrow") only see const/table without
// tails; there every reaction, const included, reads a table.
enum : uint32_t { kRxConst = 0, kRxTable = 1, kRxDirect = 2, kRxFall = 3 };
// jmeta = kind | species << 2 | first order << 4 | tail species << 6 | tail order << 8
__host__ __device__ constexpr uint32_t jmeta_pack(uint32_t kind, uint32_t sp, uint32_t o1,
                                                  uint32_t ts, uint32_t to) {
    return kind | (sp << 2) | (o1 << 4) | (ts << 6) | (to << 8);
}
__host__ __device__ constexpr bool narrow_kernel(int ns, int m) { return ns <= 2 && m <= 4; }

// Compiled network descriptors of the general kernels: the jmeta of
// reactions 0..5 in bits 10j..10j+9 and the reaction count in bits 60..62.
// With every reaction's kind, species and tail fixed at compile time the
// propensities index the state by constants, so no runtime selection (and
// no indexed private array) sits in the event chain; rate constants, tables
// and stoichiometry stay runtime data.
constexpr int kDescMaxM = 6;
__host__ __device__ constexpr long long desc_pack(const uint32_t (&meta)[kDescMaxM], int m) {
    long long d = (long long)m << 60;
    for (int j = 0; j < kDescMaxM && j < m; ++j) d |= (long long)(meta[j] & 0x3FFu) << (10 * j);
    return d;
}
__host__ __device__ constexpr int desc_count(long long d) { return (int)((d >> 60) & 7); }
__host__ __device__ constexpr uint32_t desc_meta(long long d, int j) {
    return j < desc_count(d) ? (uint32_t)(d >> (10 * j)) & 0x3FFu : jmeta_pack(kRxConst, 0, 0, 0, 0);
}
// The genetic switch of Sec. IV B (species DNA_in, DNA_act, mRNA, protein):
// transcription a x1, mRNA decay gamma x2, translation gamma b x2, protein
// decay x3 (falling factorials), and the switching reactions F(x3) x0 and
// G(x3) x1 (protein tables with a DNA tail).
constexpr uint32_t kDescSwitchMeta[kDescMaxM] = {
    jmeta_pack(kRxFall, 1, 1, 0, 0),  jmeta_pack(kRxFall, 2, 1, 0, 0),
    jmeta_pack(kRxFall, 2, 1, 0, 0),  jmeta_pack(kRxFall, 3, 1, 0, 0),
    jmeta_pack(kRxTable, 3, 0, 0, 1), jmeta_pack(kRxTable, 3, 0, 1, 1)};
constexpr long long kDescSwitch = desc_pack(kDescSwitchMeta, 6);

struct LaunchShape {
    int rpl, waves, ns;
    int m;                 // reactions (the kernel is specialised for m <= 4 and m <= 8)
    int wide = 0;          // > 0: one instance over this many workgroups (4 waves each)
    int stage_flush = -1;  // histogram staging of the group's instances (DevInst::stage_flush)
    // compiled specialisation every instance of the group fits (-1: none):
    // a species map (narrow kernels) or a network descriptor (general kernels)
    long long spec = -1;
    // 1: the persistent form of a solve launch (k_persist: resident
    // workgroups take the group's instances from a counter)
    int persist = 0;
};

// Launchers (parrep_kernels.hip).
hipError_t launch_solve(const DevInst* d_inst, int n_inst, LaunchShape shape, int mode,
                        uint32_t hook_cycle, int64_t hook_max_rounds, int tab_lds,
                        hipStream_t stream);
// Doubles of propensity table an instance of this shape wants in LDS (every
// table whole), and the doubles a workgroup of the shape can give them
// (the kernel shortens the longest tables to fit; states beyond take the
// formula).
int table_lds_need(const DevInst& d, LaunchShape shape);
// The compiled species map (kMapCross) an instance of this shape can run
// with, or -1: two species, four reactions, every reaction a table or a
// constant, tables indexed as the map says, and the table within the map's
// row stride.
int species_map(const DevInst& d, LaunchShape shape);
// The compiled network descriptor (kDescSwitch) an instance of this shape
// can run with, or -1: a 4-species general kernel with at most 4 replicas
// per lane (not spread over workgroups) whose reactions' hot meta equals the
// descriptor's.
long long network_desc(const DevInst& d, LaunchShape shape);
int table_lds_doubles(LaunchShape shape, int max_need);
hipError_t launch_zero(const DevInst* d_inst, int n_inst, hipStream_t stream);
// One instance over s.wide workgroups (cooperative launch; s.rpl 1 or 4).
hipError_t launch_wide(const DevInst* d_inst, LaunchShape s, int tab_lds, hipStream_t stream);
// Replica count from which a single-instance solve is spread over
// workgroups by default, and the default chunk lengths (rounds).
constexpr int kWideMinR = 8192;
constexpr int kWideChunkS2 = 512, kWideChunkS3 = 64;
// Writes descriptor d (a kernel argument) to dst in device memory.
hipError_t launch_install(const DevInst& d, DevInst* dst, hipStream_t stream);
hipError_t launch_setup(DevInst* d_inst, int n_inst, hipStream_t stream);
hipError_t launch_finalize(const DevInst* d_inst, int n_inst, hipStream_t stream);
hipError_t launch_accumulate(double* dst, const double* src, int64_t n, hipStream_t stream);
hipError_t launch_philox(int64_t n, const uint32_t* ctr_key, uint32_t* out, hipStream_t stream);
hipError_t launch_events(const DevInst* d_inst, int64_t n, const int32_t* states,
                         const uint32_t* blocks, double* a0, double* tau, int32_t* J,
                         hipStream_t stream);
bool shape_supported(LaunchShape s);
LaunchShape choose_shape(int R, int ns, int m);

}  // namespace parrep
