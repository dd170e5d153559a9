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

// Boys function F_m(T) = int_0^1 t^(2m) exp(-T t^2) dt for m = 0..L (L <= 16).
// T < 36: the top order from an 8-term Taylor expansion about the nearest
// tabulated point (spacing 0.05, so |T - T_k| <= 0.025), then the downward
// recurrence F_m = (2T F_{m+1} + exp(-T)) / (2m+1), which only adds positive
// terms.  T >= 36: F_0 = sqrt(pi/T)/2 (erf(sqrt T) = 1 to 2e-17 there) and the
// upward recurrence F_{m+1} = ((2m+1) F_m - exp(-T)) / (2T).
template <int L>
__device__ __forceinline__ void boys_fm(double T, const double *__restrict__ tab, double *F)
{
    const double e = exp(-T);
    if (T < BOYS_TMAX) {
        const int k = (int)(T * BOYS_INV_STEP + 0.5);
        const double x = (double)k * BOYS_STEP - T;       // -(T - T_k)
        const double *r = tab + k * BOYS_NORD + L;
        double s = r[7];
        s = fma(s, x * (1.0 / 7.0), r[6]);
        s = fma(s, x * (1.0 / 6.0), r[5]);
        s = fma(s, x * (1.0 / 5.0), r[4]);
        s = fma(s, x * (1.0 / 4.0), r[3]);
        s = fma(s, x * (1.0 / 3.0), r[2]);
        s = fma(s, x * (1.0 / 2.0), r[1]);
        s = fma(s, x, r[0]);
        F[L] = s;
        const double t2 = 2.0 * T;
#pragma unroll
        for (int m = L - 1; m >= 0; --m) F[m] = fma(t2, F[m + 1], e) * (1.0 / (double)(2 * m + 1));
    } else {
        const double rt = hgp_rcp(T);
        F[0] = 0.88622692545275801365 * hgp_rsqrt(T);      // sqrt(pi)/2 * T^(-1/2)
        const double h = 0.5 * rt;
#pragma unroll
        for (int m = 0; m < L; ++m) F[m + 1] = fma((double)(2 * m + 1), F[m], -e) * h;
    }
}

}  // namespace hgp
