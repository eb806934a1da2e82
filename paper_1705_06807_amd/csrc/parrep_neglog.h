// parrep_neglog.h -- -log(u) for the Gillespie waiting time tau = -log(u)/a0
// (Sec. II A, the "generate tau and J" step of Alg. 1), u = m * 2^-53 with
// integer m in [1, 2^53].  Table-driven, error below one ulp; plain C++ so
// that the host can check it (PARREP_HD is empty there).
//
// Reduction: u = z 2^k with z in [0.6875, 1.375).  The z range is cut into
// kLogTabN sub-intervals by the top seven bits of bits(u) - bits(0.6875); for
// sub-interval i the table holds invc ~ 1/centre, rounded to double, and
// log(1/invc) split as logc_hi (a multiple of 2^-44) + logc_lo.  Then
//     log u = k ln2 + log(1/invc) + log1p(r),  r = z*invc - 1,  |r| < 2^-7,
// with k*ln2_hi + logc_hi exact (all terms multiples of 2^-44 below 2^6) and
// log1p by its Taylor series to r^7 (truncation below 2^-59 absolute),
// evaluated in Estrin form.  The
// two sub-intervals next to z = 1 use invc = 1, log c = 0, so u -> 1 keeps
// full relative accuracy and u = 1 gives -0.0 as the C library log does.
//
// The method is P. T. P. Tang's table-driven logarithm ("Table-driven
// implementation of the logarithm function in IEEE floating-point
// arithmetic", ACM TOMS 16(4), 1990), in the form with the reduction
// interval [0.6875, 1.375) and a 128-entry 1/c, log c table that Arm's
// Optimized Routines use for log.  The table here is computed at run time
// from long double logl, and the polynomial is the plain Taylor series.
#pragma once
#include <cmath>
#include <cstdint>

#ifndef PARREP_HD
#define PARREP_HD __host__ __device__
#endif

namespace parrep {

constexpr int kLogTabN = 128;
constexpr int kLogTabLen = 3 * kLogTabN;  // invc | logc_hi | logc_lo

// ln 2 = kLn2Hi + kLn2Lo, kLn2Hi a multiple of 2^-44
constexpr double kLn2Hi = 0x1.62e42fefa3a00p-1;
constexpr double kLn2Lo = -0x1.0ca86c3898d00p-49;

// d = m as a double (exact), m in [1, 2^53]; returns -log(m * 2^-53).
PARREP_HD inline double neglog_d53(double d, const double* __restrict__ lt) {
    const uint64_t db = __builtin_bit_cast(uint64_t, d);
    const uint32_t dh = (uint32_t)(db >> 32);
    const uint32_t t = dh - 0x3FE60000u;  // high word of bits(d) - bits(0.6875): no borrow
    const int k = (int)(t >> 20) - 53;    // u = d 2^-53 = z 2^k
    const int i = (int)((t >> 13) & (uint32_t)(kLogTabN - 1));
    const double z = __builtin_bit_cast(
        double, ((uint64_t)(dh - (t & 0xFFF00000u)) << 32) | (uint32_t)db);
    const double r = std::fma(z, lt[i], -1.0);
    const double kd = (double)k;
    const double a = std::fma(kd, kLn2Hi, lt[kLogTabN + i]);  // exact
    const double s1 = std::fma(kd, kLn2Lo, lt[2 * kLogTabN + i]);
    // q(r) = -1/2 + r/3 - r^2/4 + r^3/5 - r^4/6 + r^5/7 in Estrin form (the
    // same terms; shorter dependency chains, no accumulator copies)
    const double r2 = r * r;
    const double qa = std::fma(r, 1.0 / 3.0, -0.5);
    const double qb = std::fma(r, 1.0 / 5.0, -0.25);
    const double qc = std::fma(r, 1.0 / 7.0, -1.0 / 6.0);
    const double q = std::fma(r2, std::fma(r2, qc, qb), qa);
    const double p = std::fma(r2, q, r);
    return -(a + (s1 + p));
}

// m in [1, 2^53]; returns -log(m * 2^-53).
PARREP_HD inline double neglog_u53(uint64_t m, const double* __restrict__ lt) {
    return neglog_d53(std::fma((double)(uint32_t)(m >> 32), 0x1.0p32, (double)(uint32_t)m), lt);
}

// The same for m = (hi:lo >> 11) + 1 of two 32-bit words: m = hi 2^21 +
// ((lo >> 11) + 1), both terms exact doubles and their sum (at most 2^53)
// exact, so no 64-bit integer is formed.
PARREP_HD inline double neglog_words53(uint32_t hi, uint32_t lo, const double* __restrict__ lt) {
    return neglog_d53(std::fma((double)hi, 0x1.0p21, (double)((lo >> 11) + 1u)), lt);
}

// Host: fill lt[kLogTabLen].  log(1/invc) in long double (64-bit mantissa:
// absolute error below 2^-65, far under the last bit of any result).
inline void build_log_table(double* lt) {
    const uint64_t base = 0x3FE6000000000000ull;  // bits(0.6875)
    const int i_one = (int)((0x3FF0000000000000ull - base) >> 45);
    for (int i = 0; i < kLogTabN; ++i) {
        double invc = 1.0, hi = 0.0, lo = 0.0;
        if (i != i_one && i != i_one - 1) {
            const uint64_t b0 = base + ((uint64_t)i << 45);
            const double z0 = __builtin_bit_cast(double, b0);
            const double z1 = __builtin_bit_cast(double, b0 + (1ull << 45));
            invc = (double)(2.0L / ((long double)z0 + (long double)z1));
            const long double lc = -logl((long double)invc);
            hi = (double)ldexpl(rintl(ldexpl(lc, 44)), -44);
            lo = (double)(lc - (long double)hi);
        }
        lt[i] = invc;
        lt[kLogTabN + i] = hi;
        lt[2 * kLogTabN + i] = lo;
    }
}

}  // namespace parrep
