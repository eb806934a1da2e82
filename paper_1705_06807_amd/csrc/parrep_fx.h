// parrep_fx.h -- the exact 64.64 fixed-point ParRep clock of libparrep.
//
// The ParRep clock T_s of Alg. 1 (Sec. II A) is the sum of the credited
// holding times.  Kept as an unsigned 64.64 fixed-point number, each time
// truncated to a multiple of 2^-64, the sum is exact: the horizon T and the
// burn-in time are crossed at one well-defined event whatever order the
// replicas' times are added in.  Times of 2^52 or more (and +inf, the
// holding time of an absorbing state) enter as 2^52; every horizon is below
// 2^51, so such a time always reaches it.
//
// Plain C++ so that the host can check it (PARREP_HD is empty there).
#pragma once
#include <cmath>
#include <cstdint>

#ifndef PARREP_HD
#define PARREP_HD __host__ __device__
#endif

namespace parrep {

struct Fx {
    uint64_t hi, lo;
};

// The value every time of 2^52 or more enters as.
constexpr uint64_t kFxSatHi = 1ull << 52;

PARREP_HD inline Fx fx_add(Fx a, Fx b) {
    Fx r;
    r.lo = a.lo + b.lo;
    r.hi = a.hi + b.hi + (r.lo < a.lo ? 1u : 0u);
    return r;
}

// a + b for a, b <= 2^52, clamped to 2^52.  Sums over replicas use it: the
// plain sum of 4096 saturated times (absorbing replicas) would wrap the
// high word to 0 and hide the horizon; clamped, no partial sum exceeds 2^53.
PARREP_HD inline Fx fx_add_sat(Fx a, Fx b) {
    const Fx r = fx_add(a, b);
    return r.hi >= kFxSatHi ? Fx{kFxSatHi, 0} : r;
}

// A sum of times split in three parts that do not overflow over 1024
// terms: a = the sum of the high words (each at most 2^52), b and c = the
// sums of the high and low 32-bit halves of the low words.  Returns the
// 64.64 value a + b 2^-32 + c 2^-64 clamped as fx_add_sat clamps: for
// non-negative terms the clamp of the exact total equals the clamped sum
// taken in any order.
PARREP_HD inline Fx fx_join3(uint64_t a, uint64_t b, uint64_t c) {
    const uint64_t lb = b << 32;
    const uint64_t lo = lb + c;
    const uint64_t hi = a + (b >> 32) + (lo < lb ? 1u : 0u);
    return hi >= kFxSatHi ? Fx{kFxSatHi, 0} : Fx{hi, lo};
}

PARREP_HD inline Fx fx_sub(Fx a, Fx b) {
    Fx r;
    r.lo = a.lo - b.lo;
    r.hi = a.hi - b.hi - (a.lo < b.lo ? 1u : 0u);
    return r;
}

PARREP_HD inline bool fx_ge(Fx a, Fx b) {
    return a.hi > b.hi || (a.hi == b.hi && a.lo >= b.lo);
}
PARREP_HD inline bool fx_gt(Fx a, Fx b) { return !fx_ge(b, a); }

// Correctly rounded uint64 -> double: both halves are exact, one rounding in the sum.
PARREP_HD inline double u64_to_f64(uint64_t v) {
    return (double)(uint32_t)(v >> 32) * 0x1.0p32 + (double)(uint32_t)v;
}
PARREP_HD inline double fx_to_f64(Fx v) {
    return u64_to_f64(v.hi) + u64_to_f64(v.lo) * 0x1.0p-64;
}

// floor(d * 2^64) for 0 <= d < 2^52, by exact steps; +inf and larger saturate.
PARREP_HD inline Fx fx_from(double d) {
    if (!(d < 0x1.0p52)) return Fx{kFxSatHi, 0};
    if (!(d > 0.0)) return Fx{0, 0};
    const double ip = std::floor(d);
    const double a = (d - ip) * 0x1.0p32;
    const double ah = std::floor(a);
    const double b = (a - ah) * 0x1.0p32;
    const double bl = std::floor(b);
    const double iph = std::floor(ip * 0x1.0p-32);
    const double ipl = ip - iph * 0x1.0p32;
    Fx r;
    r.hi = ((uint64_t)(uint32_t)iph << 32) | (uint64_t)(uint32_t)ipl;
    r.lo = ((uint64_t)(uint32_t)ah << 32) | (uint64_t)(uint32_t)bl;
    return r;
}

}  // namespace parrep
