// Device-side helpers included by every generated class kernel.
#pragma once
#include "hgp_types.h"

namespace hgp {

// Stage boundary of a staged kernel (no instruction is emitted): a compiler
// memory fence, so values stored to the scratch buffer are reloaded after it
// rather than kept live in registers, and an opaque redefinition of the lane's
// scratch pointer, so the per-slot address arithmetic of a stage is not
// hoisted out of the quartet loop (hundreds of 64-bit addresses would
// otherwise be computed once and spilled).
#define HGP_STAGE(ptr) asm volatile("" : "+v"(ptr)::"memory")
// Opaque redefinition of a per-lane pointer without a memory fence: address
// arithmetic on it cannot be hoisted above this point.
#define HGP_OPAQUE(ptr) asm volatile("" : "+v"(ptr))

// 1/x and 1/sqrt(x) for positive normal x: the hardware estimate refined by
// two Newton-Raphson steps (r <- r + r(1 - x r); y <- y + y(1 - x y^2)/2),
// each roughly doubling the correct bits, which ends within an ulp or two of
// the correctly rounded value -- far cheaper than the IEEE-exact sequences.
__device__ __forceinline__ double hgp_rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ double hgp_rsqrt(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

// True when pred holds on every active lane of the wave.
__device__ __forceinline__ bool hgp_wave_all(bool pred)
{
    return __builtin_amdgcn_ballot_w64(pred) == __builtin_amdgcn_read_exec();
}

// Sum of v over the 64 lanes of a full wave (butterfly: every lane ends with the total).
__device__ __forceinline__ double hgp_wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Segmented wave reductions.  The class lists keep quartets that share a
// digestion target adjacent (same bra pair; same bra pair and ket shell c), so
// the lanes of a wave that add into one J'/K' element form contiguous runs.
// Adding along each run first and letting its last lane issue the atomic
// replaces up to 64 atomics on one address with one.  Lanes that have exited
// are the wave's highest (quartet index past the end of the list).
//
// First lane of the calling lane's run of equal keys (inclusive max-scan of run heads).
__device__ __forceinline__ int hgp_seg_start(long long key)
{
    const int lane = __lane_id();
    const long long prev = __shfl_up(key, 1, 64);
    int s = (lane == 0 || prev != key) ? lane : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(s, o, 64);
        if (lane >= o) s = max(s, t);
    }
    return s;
}

// True on the last active lane of the calling lane's run of equal keys.
__device__ __forceinline__ bool hgp_seg_tail(long long key)
{
    const int lane = __lane_id();
    const long long next = __shfl_down(key, 1, 64);
    const unsigned long long live = __builtin_amdgcn_read_exec();
    return lane == 63 || ((live >> (lane + 1)) & 1ull) == 0 || next != key;
}

// Inclusive sum of v along the run that starts at lane `start` (Hillis-Steele
// steps that only take partial sums from lanes of the same run); the run's
// last lane ends with the run total.
__device__ __forceinline__ double hgp_seg_sum(double v, int start)
{
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double t = __shfl_up(v, o, 64);
        if (lane - o >= start) v += t;
    }
    return v;
}

// Boys function F_m(T) = int_0^1 t^(2m) exp(-T t^2) dt for m = 0..L (L <= 16).
// T < 36: Taylor expansion about the nearest tabulated point T_k (spacing
// 0.05, so |x| = |T_k - T| <= 0.025), F_m(T) = sum_j F_{m+j}(T_k) x^j / j!,
// 8 terms (remainder below 4e-18 F_m).  For L <= 2 every order is expanded
// this way (independent chains, no exponential).  For larger L only the top
// order is, and the downward recurrence F_m = (2T F_{m+1} + exp(-T)) / (2m+1)
// (positive terms only) gives the rest, with exp(-T) = exp(-T_k) exp(x)
// from the table's exp column and a degree-7 Taylor polynomial.
// T >= 36: F_0 = sqrt(pi/T)/2 (erf(sqrt T) = 1 to 2e-17 there) and the
// upward recurrence F_{m+1} = ((2m+1) F_m - exp(-T)) / (2T).
template <int L>
__device__ __forceinline__ void boys_fm(double T, const double *__restrict__ tab, double *F)
{
    constexpr bool kAllTaylor = L <= 2;
    if (T < BOYS_TMAX) {
        const int k = (int)(T * BOYS_INV_STEP + 0.5);
        const double x = (double)k * BOYS_STEP - T;       // -(T - T_k)
        const double *r = tab + k * BOYS_STRIDE;
        const double ek = (!kAllTaylor) ? r[BOYS_NORD] : 0.0;   // exp(-T_k), issued with the coefficients
        const double x2 = x * 0.5, x3 = x * (1.0 / 3.0), x4 = x * 0.25, x5 = x * (1.0 / 5.0),
                     x6 = x * (1.0 / 6.0), x7 = x * (1.0 / 7.0);
#pragma unroll
        for (int m = kAllTaylor ? 0 : L; m <= L; ++m) {
            double s = r[m + 7];
            s = fma(s, x7, r[m + 6]);
            s = fma(s, x6, r[m + 5]);
            s = fma(s, x5, r[m + 4]);
            s = fma(s, x4, r[m + 3]);
            s = fma(s, x3, r[m + 2]);
            s = fma(s, x2, r[m + 1]);
            F[m] = fma(s, x, r[m]);
        }
        if (!kAllTaylor) {
            double p = 1.0 / 5040.0;
            p = fma(p, x, 1.0 / 720.0);
            p = fma(p, x, 1.0 / 120.0);
            p = fma(p, x, 1.0 / 24.0);
            p = fma(p, x, 1.0 / 6.0);
            p = fma(p, x, 0.5);
            p = fma(p, x, 1.0);
            p = fma(p, x, 1.0);                              // exp(x), x = T_k - T
            const double e = ek * p;
            const double t2 = 2.0 * T;
#pragma unroll
            for (int m = L - 1; m >= 0; --m) F[m] = fma(t2, F[m + 1], e) * (1.0 / (double)(2 * m + 1));
        }
    } else {
        // exp(-T) <= 2.4e-16 here: it only corrects F_m by that order, so the
        // single-precision hardware exp2 (relative error ~1e-7, flushing to 0
        // below 1e-38) is far more accurate than needed.
        const double e = L > 0 ? (double)__builtin_amdgcn_exp2f((float)(T * -1.4426950408889634)) : 0.0;
        const double rt = hgp_rcp(T);
        F[0] = 0.88622692545275801365 * hgp_rsqrt(T);      // sqrt(pi)/2 * T^(-1/2)
        const double h = 0.5 * rt;
#pragma unroll
        for (int m = 0; m < L; ++m) F[m + 1] = fma((double)(2 * m + 1), F[m], -e) * h;
    }
}

}  // namespace hgp
