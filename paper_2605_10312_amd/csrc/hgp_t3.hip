// HBM-scratch tier (see hgp_t3.h): generic kernels that run a class's op
// table.  One lane per shell quartet; every intermediate value lives in a
// slot of the lane-interleaved buffer sb[slot * S + lane], so each wave reads
// and writes 512-byte rows.  Op fields are wave-uniform and arrive through
// scalar loads.
#include <map>
#include <mutex>
#include <utility>

#include "hgp_device.h"
#include "hgp_t3.h"

namespace hgp {

struct T3Dev {
    const uint4 *ops;
    const double *coefs;
    const uint16_t *outslots;
};

struct T3Params {
    int L, na, nb, nc, nd, n_hrr, acc0, n_vrr, n_p2;
};

namespace {

// base * F_m(T) for m = 0..L into slots 0..L (the same Boys scheme as
// boys_fm<L>, with L known only at run time: Taylor step for the top order
// and the downward recurrence below T = 36, asymptote and upward recurrence
// above).
__device__ __forceinline__ void t3_boys(double T, int L, const double *__restrict__ tab, double base,
                                        double *__restrict__ sb, uint32_t S, uint32_t li)
{
    if (T < BOYS_TMAX) {
        const int k = (int)(T * BOYS_INV_STEP + 0.5);
        const double x = (double)k * BOYS_STEP - T;
        const double *r = tab + k * BOYS_STRIDE + L;
        const double ek = tab[k * BOYS_STRIDE + BOYS_NORD];
        double f = r[7];
        f = fma(f, x * (1.0 / 7.0), r[6]);
        f = fma(f, x * (1.0 / 6.0), r[5]);
        f = fma(f, x * (1.0 / 5.0), r[4]);
        f = fma(f, x * 0.25, r[3]);
        f = fma(f, x * (1.0 / 3.0), r[2]);
        f = fma(f, x * 0.5, r[1]);
        f = fma(f, x, r[0]);
        sb[(uint32_t)L * S + li] = base * f;
        double p = 1.0 / 5040.0;
        p = fma(p, x, 1.0 / 720.0);
        p = fma(p, x, 1.0 / 120.0);
        p = fma(p, x, 1.0 / 24.0);
        p = fma(p, x, 1.0 / 6.0);
        p = fma(p, x, 0.5);
        p = fma(p, x, 1.0);
        p = fma(p, x, 1.0);
        const double e = ek * p, t2 = 2.0 * T;
        for (int m = L - 1; m >= 0; --m) {
            f = fma(t2, f, e) / (double)(2 * m + 1);
            sb[(uint32_t)m * S + li] = base * f;
        }
    } else {
        const double e = (double)__builtin_amdgcn_exp2f((float)(T * -1.4426950408889634));
        const double h = 0.5 * hgp_rcp(T);
        double f = 0.88622692545275801365 * hgp_rsqrt(T);
        sb[li] = base * f;
        for (int m = 0; m < L; ++m) {
            f = fma((double)(2 * m + 1), f, -e) * h;
            sb[(uint32_t)(m + 1) * S + li] = base * f;
        }
    }
}

// The contracted accumulators of one quartet, then Phase 2: on return the
// quartet's spherical integrals sit in the slots named by outslots.
__device__ void t3_quartet(const T3Params &c, const uint4 *__restrict__ ops, const double *__restrict__ coefs,
                           const PairInfo &pb, const PairGeo &gb, const PairInfo &pk, const PairGeo &gk,
                           const PrimPair *__restrict__ prims, const double *__restrict__ boys,
                           double *__restrict__ sb, uint32_t S, uint32_t li)
{
    auto at = [&](uint32_t slot) -> double & { return sb[slot * S + li]; };
    for (int k = 0; k < c.n_hrr; ++k) at((uint32_t)(c.acc0 + k)) = 0.0;
    const double Ax = gb.ax, Ay = gb.ay, Az = gb.az, Cx = gk.ax, Cy = gk.ay, Cz = gk.az;
    const PrimPair *__restrict__ pbp = prims + pb.prim_off;
    const PrimPair *__restrict__ pkp = prims + pk.prim_off;
    for (int ip = 0; ip < pb.nprim; ++ip) {
        const PrimPair b = pbp[ip];
        for (int jp = 0; jp < pk.nprim; ++jp) {
            const PrimPair q = pkp[jp];
            const double PAx = b.px - Ax, PAy = b.py - Ay, PAz = b.pz - Az;
            const double QCx = q.px - Cx, QCy = q.py - Cy, QCz = q.pz - Cz;
            const double PQx = b.px - q.px, PQy = b.py - q.py, PQz = b.pz - q.pz;
            const double ze = b.zeta + q.zeta, ize = hgp_rcp(ze);
            const double rz = q.zeta * ize, re = b.zeta * ize, o2ze = 0.5 * ize;
            const double T = b.zeta * rz * (PQx * PQx + PQy * PQy + PQz * PQz);
            t3_boys(T, c.L, boys, b.k * q.k * hgp_rsqrt(ze), sb, S, li);
            const double WPx = -rz * PQx, WPy = -rz * PQy, WPz = -rz * PQz;
            const double WQx = re * PQx, WQy = re * PQy, WQz = re * PQz;
            // groups of T3_GROUP independent ops: every operand load of the
            // group is issued before the first result is computed
            for (int g = 0; g < c.n_vrr; g += T3_GROUP) {
                uint4 o[T3_GROUP];
#pragma unroll
                for (int j = 0; j < T3_GROUP; ++j) o[j] = ops[g + j];
                if ((o[0].x & 15u) == T3_ACC) {
                    double x[T3_GROUP], y[T3_GROUP];
#pragma unroll
                    for (int j = 0; j < T3_GROUP; ++j) {
                        if ((o[j].x & 15u) == 0) continue;
                        x[j] = at(o[j].x >> 16);
                        y[j] = at(o[j].y & 0xFFFFu);
                    }
#pragma unroll
                    for (int j = 0; j < T3_GROUP; ++j)
                        if ((o[j].x & 15u) != 0) at(o[j].x >> 16) = x[j] + y[j];
                    continue;
                }
                double v1[T3_GROUP], v2[T3_GROUP], v3[T3_GROUP], v4[T3_GROUP], v5[T3_GROUP];
#pragma unroll
                for (int j = 0; j < T3_GROUP; ++j) {
                    if ((o[j].x & 15u) == 0) continue;
                    const uint32_t w0 = o[j].x & 0xFFFFu;
                    v1[j] = at(o[j].y & 0xFFFFu);
                    v2[j] = at(o[j].y >> 16);
                    if ((w0 >> 6) & 31u) {
                        v3[j] = at(o[j].z & 0xFFFFu);
                        v4[j] = at(o[j].z >> 16);
                    }
                    if ((w0 >> 11) & 31u) v5[j] = at(o[j].w & 0xFFFFu);
                }
#pragma unroll
                for (int j = 0; j < T3_GROUP; ++j) {
                    const uint32_t w0 = o[j].x & 0xFFFFu;
                    const uint32_t code = w0 & 15u, axis = (w0 >> 4) & 3u;
                    if (code == 0) continue;
                    const uint32_t ks = (w0 >> 6) & 31u, kc = (w0 >> 11) & 31u;
                    double X, Y, o2, r;
                    if (code == T3_VRR_BRA) {
                        X = axis == 0 ? PAx : (axis == 1 ? PAy : PAz);
                        Y = axis == 0 ? WPx : (axis == 1 ? WPy : WPz);
                        o2 = b.o2z;
                        r = rz;
                    } else {
                        X = axis == 0 ? QCx : (axis == 1 ? QCy : QCz);
                        Y = axis == 0 ? WQx : (axis == 1 ? WQy : WQz);
                        o2 = q.o2z;
                        r = re;
                    }
                    double v = fma(X, v1[j], Y * v2[j]);
                    if (ks) v = fma((double)ks * o2, fma(-r, v4[j], v3[j]), v);
                    if (kc) v = fma((double)kc * o2ze, v5[j], v);
                    at(o[j].x >> 16) = v;
                }
            }
        }
    }
    // Phase 2: HRR and the stepwise transforms (Eq. hrr, Eqs. bra-sph .. stepwise-sph)
    const double ABx = gb.abx, ABy = gb.aby, ABz = gb.abz, CDx = gk.abx, CDy = gk.aby, CDz = gk.abz;
    for (int g = c.n_vrr; g < c.n_vrr + c.n_p2; g += T3_GROUP) {
        uint4 o[T3_GROUP];
#pragma unroll
        for (int j = 0; j < T3_GROUP; ++j) o[j] = ops[g + j];
        const uint32_t gcode = o[0].x & 15u;
        if (gcode == T3_HRR_BRA || gcode == T3_HRR_KET) {
            double hi[T3_GROUP], lo[T3_GROUP];
#pragma unroll
            for (int j = 0; j < T3_GROUP; ++j) {
                if ((o[j].x & 15u) == 0) continue;
                hi[j] = at(o[j].y & 0xFFFFu);
                lo[j] = at(o[j].y >> 16);
            }
#pragma unroll
            for (int j = 0; j < T3_GROUP; ++j) {
                const uint32_t code = o[j].x & 15u, axis = (o[j].x >> 4) & 3u;
                if (code == 0) continue;
                const double d = code == T3_HRR_BRA ? (axis == 0 ? ABx : (axis == 1 ? ABy : ABz))
                                                    : (axis == 0 ? CDx : (axis == 1 ? CDy : CDz));
                at(o[j].x >> 16) = fma(d, lo[j], hi[j]);
            }
        } else {
            double x1[T3_GROUP], x2[T3_GROUP], x3[T3_GROUP], acc[T3_GROUP];
#pragma unroll
            for (int j = 0; j < T3_GROUP; ++j) {
                const uint32_t code = o[j].x & 15u;
                if (code == 0) continue;
                x1[j] = at(o[j].y & 0xFFFFu);
                if ((o[j].y >> 16) != T3_NONE) x2[j] = at(o[j].y >> 16);
                if ((o[j].z & 0xFFFFu) != T3_NONE) x3[j] = at(o[j].z & 0xFFFFu);
                if (code == T3_LIN_ACC) acc[j] = at(o[j].x >> 16);
            }
#pragma unroll
            for (int j = 0; j < T3_GROUP; ++j) {
                const uint32_t code = o[j].x & 15u;
                if (code == 0) continue;
                double v = code == T3_LIN_ACC ? acc[j] : 0.0;
                v = fma(coefs[o[j].z >> 16], x1[j], v);
                if ((o[j].y >> 16) != T3_NONE) v = fma(coefs[o[j].w & 0xFFFFu], x2[j], v);
                if ((o[j].z & 0xFFFFu) != T3_NONE) v = fma(coefs[o[j].w >> 16], x3[j], v);
                at(o[j].x >> 16) = v;
            }
        }
    }
}

__global__ __launch_bounds__(64) void t3_jk_kernel(T3Params c, const uint4 *__restrict__ ops, const double *__restrict__ coefs,
                             const uint16_t *__restrict__ outslots, JKArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.nq) return;
    double *__restrict__ sb = a.scratch;
    const uint32_t S = (uint32_t)a.stride, li = (uint32_t)i;
    const int2 pq = a.quartets[i];
    const PairInfo pb = a.pairs[pq.x], pk = a.pairs[pq.y];
    const PairGeo gb = a.geo[pq.x], gk = a.geo[pq.y];
    t3_quartet(c, ops, coefs, pb, gb, pk, gk, a.prims, a.boys, sb, S, li);
    auto I = [&](int mu, int nu, int lam, int sig) -> double {
        return sb[(uint32_t)outslots[((mu * c.nb + nu) * c.nc + lam) * c.nd + sig] * S + li];
    };
    const double *__restrict__ D = a.D;
    const int64_t N = a.nbf;
    const int fa = pb.fa, fb = pb.fb, fc = pk.fa, fd = pk.fb;
    const double s = (pb.same ? 0.5 : 1.0) * (pk.same ? 0.5 : 1.0) * (pq.x == pq.y ? 0.5 : 1.0);
    // J'[ab] += 2s sum_cd I D_cd, J'[cd] += 2s sum_ab I D_ab (unsymmetrised, degeneracy-scaled)
    if (a.want_j) {
        for (int mu = 0; mu < c.na; ++mu)
            for (int nu = 0; nu < c.nb; ++nu) {
                double t = 0.0;
                for (int lam = 0; lam < c.nc; ++lam)
                    for (int sig = 0; sig < c.nd; ++sig) t = fma(I(mu, nu, lam, sig), D[(fc + lam) * N + fd + sig], t);
                atomicAdd(a.J + (fa + mu) * N + fb + nu, 2.0 * s * t);
            }
        for (int lam = 0; lam < c.nc; ++lam)
            for (int sig = 0; sig < c.nd; ++sig) {
                double t = 0.0;
                for (int mu = 0; mu < c.na; ++mu)
                    for (int nu = 0; nu < c.nb; ++nu) t = fma(I(mu, nu, lam, sig), D[(fa + mu) * N + fb + nu], t);
                atomicAdd(a.J + (fc + lam) * N + fd + sig, 2.0 * s * t);
            }
    }
    // K'[ac] += s sum I D_bd, K'[bc] += s sum I D_ad, K'[ad] += s sum I D_bc, K'[bd] += s sum I D_ac
    if (a.want_k) {
        for (int mu = 0; mu < c.na; ++mu)
            for (int lam = 0; lam < c.nc; ++lam) {
                double t = 0.0;
                for (int nu = 0; nu < c.nb; ++nu)
                    for (int sig = 0; sig < c.nd; ++sig) t = fma(I(mu, nu, lam, sig), D[(fb + nu) * N + fd + sig], t);
                atomicAdd(a.K + (fa + mu) * N + fc + lam, s * t);
            }
        for (int nu = 0; nu < c.nb; ++nu)
            for (int lam = 0; lam < c.nc; ++lam) {
                double t = 0.0;
                for (int mu = 0; mu < c.na; ++mu)
                    for (int sig = 0; sig < c.nd; ++sig) t = fma(I(mu, nu, lam, sig), D[(fa + mu) * N + fd + sig], t);
                atomicAdd(a.K + (fb + nu) * N + fc + lam, s * t);
            }
        for (int mu = 0; mu < c.na; ++mu)
            for (int sig = 0; sig < c.nd; ++sig) {
                double t = 0.0;
                for (int nu = 0; nu < c.nb; ++nu)
                    for (int lam = 0; lam < c.nc; ++lam) t = fma(I(mu, nu, lam, sig), D[(fb + nu) * N + fc + lam], t);
                atomicAdd(a.K + (fa + mu) * N + fd + sig, s * t);
            }
        for (int nu = 0; nu < c.nb; ++nu)
            for (int sig = 0; sig < c.nd; ++sig) {
                double t = 0.0;
                for (int mu = 0; mu < c.na; ++mu)
                    for (int lam = 0; lam < c.nc; ++lam) t = fma(I(mu, nu, lam, sig), D[(fa + mu) * N + fc + lam], t);
                atomicAdd(a.K + (fb + nu) * N + fd + sig, s * t);
            }
    }
}

__global__ __launch_bounds__(64) void t3_eri_kernel(T3Params c, const uint4 *__restrict__ ops, const double *__restrict__ coefs,
                              const uint16_t *__restrict__ outslots, EriArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.ntask) return;
    double *__restrict__ sb = a.scratch;
    const uint32_t S = (uint32_t)a.stride, li = (uint32_t)i;
    const EriTask t = a.tasks[i];
    const PairInfo pb = a.pairs[t.bra], pk = a.pairs[t.ket];
    const PairGeo gb = a.geo[t.bra], gk = a.geo[t.ket];
    t3_quartet(c, ops, coefs, pb, gb, pk, gk, a.prims, a.boys, sb, S, li);
    auto slot = [&](int mu, int nu, int lam, int sig) -> uint32_t {
        return outslots[((mu * c.nb + nu) * c.nc + lam) * c.nd + sig];
    };
    if (a.mode == 1) {                       // Schwarz factor of a diagonal quartet
        double m = 0.0;
        for (int mu = 0; mu < c.na; ++mu)
            for (int nu = 0; nu < c.nb; ++nu) m = fmax(m, fabs(sb[slot(mu, nu, mu, nu) * S + li]));
        a.out[i] = sqrt(m);
        return;
    }
    double *__restrict__ o = a.out + t.off;
    for (int mu = 0; mu < c.na; ++mu)
        for (int nu = 0; nu < c.nb; ++nu)
            for (int lam = 0; lam < c.nc; ++lam)
                for (int sig = 0; sig < c.nd; ++sig)
                    o[mu * t.s0 + nu * t.s1 + lam * t.s2 + sig * t.s3] = sb[slot(mu, nu, lam, sig) * S + li];
}

// ---------------------------------------------------------------------------
// Wave-cooperative LDS variant.  One 64-lane workgroup per quartet; LDS holds
// [slots | Z | sink | coefficients | six D blocks] as doubles, then the
// uint16 output-slot map.  Lane j runs ops j and j + 64 of every group.  A
// group's ops are independent of one another, so each lane reads its
// operands before any lane of the group writes; successive groups see each other's writes
// because LDS instructions of one wavefront execute in issue order.  The
// wave barrier below only stops the compiler from moving LDS accesses
// across a group boundary (it emits no instruction).

struct T3WParams {
    int L, na, nb, nc, nd, n_hrr, acc0, n_vrr, n_p2, nslots, ncoef, maxblk, nint;
    int deriv;      // 1: derivative tables, whose ACC_W ops read 2a, 2b, 2c from slots L + 1 .. L + 3
    int nseg;       // Phase 2 only: partial accumulators per accumulator (segments of the primitive loop)
};

// G = false: slots in LDS; a compiler-level barrier suffices.  G = true: slots
// in the quartet's region of global memory; a workgroup-scope release and
// acquire (the workgroup is this one wave) make each group's stores visible
// to the next group's loads.
template <bool G>
__device__ __forceinline__ void t3w_sync()
{
    if (G) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Lane m <= L writes base * F_m(T) to slot m.  Below T = 36 each order is its
// own 8-term Taylor expansion about the nearest table point (the table holds
// orders 0..23, so m + 7 <= 23 for L <= 16); above, the asymptote and the
// upward recurrence, evaluated by every lane up to its own order.
__device__ __forceinline__ void t3w_boys(double T, int L, const double *__restrict__ tab, double base,
                                         double *__restrict__ S, int lane)
{
    if (lane > L) return;
    if (T < BOYS_TMAX) {
        const int k = (int)(T * BOYS_INV_STEP + 0.5);
        const double x = (double)k * BOYS_STEP - T;
        const double *r = tab + k * BOYS_STRIDE + lane;
        double f = r[7];
        f = fma(f, x * (1.0 / 7.0), r[6]);
        f = fma(f, x * (1.0 / 6.0), r[5]);
        f = fma(f, x * (1.0 / 5.0), r[4]);
        f = fma(f, x * 0.25, r[3]);
        f = fma(f, x * (1.0 / 3.0), r[2]);
        f = fma(f, x * 0.5, r[1]);
        f = fma(f, x, r[0]);
        S[lane] = base * f;
    } else {
        const double e = (double)__builtin_amdgcn_exp2f((float)(T * -1.4426950408889634));
        const double h = 0.5 * hgp_rcp(T);
        double f = 0.88622692545275801365 * hgp_rsqrt(T);
        for (int m = 0; m < lane; ++m) f = fma((double)(2 * m + 1), f, -e) * h;
        S[lane] = base * f;
    }
}

// One group of ops, o = this lane's op.  Per-primitive quantities come in
// through q (bra values then ket values).
struct T3WPrim {
    double PAx, PAy, PAz, WPx, WPy, WPz, o2z, rz;
    double QCx, QCy, QCz, WQx, WQy, WQz, o2e, re;
    double o2ze;
};

// Each lane runs T3W_K ops of a group of T3W_OPS: ops lane, lane + 64, ...
// All operand reads of its ops are issued before any result is computed, so
// one memory latency covers them all; the results are written last.
constexpr int T3W_K = T3W_OPS / T3W_GROUP;

// The per-primitive constants of the VRR as an LDS record R (16 doubles):
// (X, Y) = (P-A, W-P) or (Q-C, W-Q) along axis a at R[2 (3 side + a)], and
// (1/(2 zeta), rho/zeta) or (1/(2 eta), rho/eta) at R[12 + 2 side], side 0
// for the bra.  An op reads its pairs with two 16-byte loads instead of
// selecting among twelve values.
__device__ __forceinline__ void t3w_vrr_group(const uint4 *o, const double *__restrict__ R, double o2ze,
                                              double *__restrict__ S)
{
    double v[T3W_K][5];
    double2 xy[T3W_K], or_[T3W_K];
#pragma unroll
    for (int k = 0; k < T3W_K; ++k) {
        const uint32_t side = (o[k].x & 15u) == (uint32_t)T3_VRR_BRA ? 0u : 1u, axis = (o[k].x >> 4) & 3u;
        v[k][0] = S[o[k].y & 0xFFFFu];
        v[k][1] = S[o[k].y >> 16];
        v[k][2] = S[o[k].z & 0xFFFFu];
        v[k][3] = S[o[k].z >> 16];
        v[k][4] = S[o[k].w & 0xFFFFu];
        xy[k] = *(const double2 *)(R + 2 * (3 * side + axis));
        or_[k] = *(const double2 *)(R + 12 + 2 * side);
    }
    double r[T3W_K];
#pragma unroll
    for (int k = 0; k < T3W_K; ++k) {
        const uint32_t w0 = o[k].x;
        double t = fma(xy[k].x, v[k][0], xy[k].y * v[k][1]);
        t = fma((double)((w0 >> 6) & 31u) * or_[k].x, fma(-or_[k].y, v[k][3], v[k][2]), t);
        r[k] = fma((double)((w0 >> 11) & 31u) * o2ze, v[k][4], t);
    }
#pragma unroll
    for (int k = 0; k < T3W_K; ++k) S[o[k].x >> 16] = r[k];
}

// ACC: dst += src; ACC_W: dst += S[w] * src (w: a per-primitive weight slot).
__device__ __forceinline__ void t3w_acc_group(const uint4 *o, double *__restrict__ S)
{
    double x[T3W_K], y[T3W_K], w[T3W_K];
#pragma unroll
    for (int k = 0; k < T3W_K; ++k) {
        x[k] = S[o[k].x >> 16];
        y[k] = S[o[k].y & 0xFFFFu];
        w[k] = (o[k].x & 15u) == (uint32_t)T3_ACC_W ? S[o[k].y >> 16] : 1.0;
    }
#pragma unroll
    for (int k = 0; k < T3W_K; ++k) S[o[k].x >> 16] = fma(w[k], y[k], x[k]);
}

struct T3WHrr {
    double abx, aby, abz, cdx, cdy, cdz;
};

__device__ __forceinline__ double t3w_hrr_d(const uint4 o, const T3WHrr &h)
{
    const uint32_t code = o.x & 15u, axis = (o.x >> 4) & 3u;
    const bool bra = code == (uint32_t)T3_HRR_BRA;
    const double d0 = bra ? +h.abx : +h.cdx, d1 = bra ? +h.aby : +h.cdy, d2 = bra ? +h.abz : +h.cdz;
    return axis == 0 ? d0 : (axis == 1 ? d1 : d2);
}

__device__ __forceinline__ void t3w_hrr_group(const uint4 *o, const T3WHrr &h, double *__restrict__ S)
{
    double hi[T3W_K], lo[T3W_K];
#pragma unroll
    for (int k = 0; k < T3W_K; ++k) {
        hi[k] = S[o[k].y & 0xFFFFu];
        lo[k] = S[o[k].y >> 16];
    }
#pragma unroll
    for (int k = 0; k < T3W_K; ++k) S[o[k].x >> 16] = fma(t3w_hrr_d(o[k], h), lo[k], hi[k]);
}

__device__ __forceinline__ void t3w_lin_group(const uint4 *o, const double *__restrict__ C, double *__restrict__ S)
{
    double x[T3W_K][4], c[T3W_K][3];
#pragma unroll
    for (int k = 0; k < T3W_K; ++k) {
        x[k][0] = S[o[k].y & 0xFFFFu];
        x[k][1] = S[o[k].y >> 16];
        x[k][2] = S[o[k].z & 0xFFFFu];
        x[k][3] = (o[k].x & 15u) == (uint32_t)T3_LIN_ACC ? S[o[k].x >> 16] : 0.0;
        c[k][0] = C[o[k].z >> 16];
        c[k][1] = C[o[k].w & 0xFFFFu];
        c[k][2] = C[o[k].w >> 16];
    }
#pragma unroll
    for (int k = 0; k < T3W_K; ++k)
        S[o[k].x >> 16] = fma(c[k][2], x[k][2], fma(c[k][1], x[k][1], fma(c[k][0], x[k][0], x[k][3])));
}

// The quartet's integrals into their output slots (LDS), as t3_quartet.
// P2: the accumulators come in from acc_in[k * acc_stride] (a staged form's
// Phase 1) and only Phase 2 runs.
template <bool G, bool P2 = false>
__device__ __forceinline__ void t3w_quartet(const T3WParams &c, const uint4 *__restrict__ ops, const PairInfo &pb,
                            const PairGeo &gb, const PairInfo &pk, const PairGeo &gk,
                            const PrimPair *__restrict__ prims, const double *__restrict__ boys, double *__restrict__ S,
                            const double *__restrict__ C, double *__restrict__ R, int lane,
                            const double *__restrict__ acc_in = nullptr, int64_t acc_stride = 0)
{
    if (P2) {
        for (int k = lane; k < c.n_hrr; k += T3W_GROUP) {
            double x = acc_in[(int64_t)k * acc_stride];
            for (int sg = 1; sg < c.nseg; ++sg) x += acc_in[((int64_t)sg * c.n_hrr + k) * acc_stride];
            S[c.acc0 + k] = x;
        }
    } else {
        for (int k = lane; k < c.n_hrr; k += T3W_GROUP) S[c.acc0 + k] = 0.0;
    }
    if (lane == 0) S[c.nslots] = 0.0;                       // the zero slot
    t3w_sync<G>();
    const uint4 *__restrict__ myops = ops + lane;
    const PrimPair *__restrict__ pbp = prims + pb.prim_off;
    const PrimPair *__restrict__ pkp = prims + pk.prim_off;
    for (int ip = 0; ip < (P2 ? 0 : pb.nprim); ++ip) {
        const PrimPair b = pbp[ip];
        for (int jp = 0; jp < pk.nprim; ++jp) {
            const PrimPair e = pkp[jp];
            T3WPrim q;
            q.PAx = b.px - gb.ax; q.PAy = b.py - gb.ay; q.PAz = b.pz - gb.az;
            q.QCx = e.px - gk.ax; q.QCy = e.py - gk.ay; q.QCz = e.pz - gk.az;
            const double PQx = b.px - e.px, PQy = b.py - e.py, PQz = b.pz - e.pz;
            const double ze = b.zeta + e.zeta, ize = hgp_rcp(ze);
            q.rz = e.zeta * ize;
            q.re = b.zeta * ize;
            q.o2ze = 0.5 * ize;
            q.o2z = b.o2z;
            q.o2e = e.o2z;
            q.WPx = -q.rz * PQx; q.WPy = -q.rz * PQy; q.WPz = -q.rz * PQz;
            q.WQx = q.re * PQx; q.WQy = q.re * PQy; q.WQz = q.re * PQz;
            const double T = b.zeta * q.rz * (PQx * PQx + PQy * PQy + PQz * PQz);
            t3w_boys(T, c.L, boys, b.k * e.k * hgp_rsqrt(ze), S, lane);
            if (c.deriv && lane >= 61) {                    // derivative weights 2a, 2b, 2c (slots past the Boys values)
                const double wv = lane == 61 ? b.ea : (lane == 62 ? b.eb : e.ea);
                S[c.L + lane - 60] = 2.0 * wv;
            }
            if (lane < 16) {                                // the constants record, one value a lane
                const double rv[16] = {q.PAx, q.WPx, q.PAy, q.WPy, q.PAz, q.WPz, q.QCx, q.WQx,
                                       q.QCy, q.WQy, q.QCz, q.WQz, q.o2z, q.rz,  q.o2e, q.re};
                double x = rv[0];
#pragma unroll
                for (int j = 1; j < 16; ++j) x = lane == j ? rv[j] : x;
                R[lane] = x;
            }
            t3w_sync<G>();
            // groups of T3W_OPS ops, two per lane; the next group's ops are
            // loaded while this one runs (the table ends in a padding group)
            const int ng = c.n_vrr / T3W_OPS;
            uint4 nx[T3W_K];
#pragma unroll
            for (int k = 0; k < T3W_K; ++k) nx[k] = myops[k * T3W_GROUP];
            for (int g = 0; g < ng; ++g) {
                uint4 o[T3W_K];
#pragma unroll
                for (int k = 0; k < T3W_K; ++k) {
                    o[k] = nx[k];
                    nx[k] = myops[(size_t)(g + 1) * T3W_OPS + k * T3W_GROUP];
                }
                const uint32_t kind = __builtin_amdgcn_readfirstlane(o[0].x) & 15u;
                if (kind == (uint32_t)T3_ACC || kind == (uint32_t)T3_ACC_W)
                    t3w_acc_group(o, S);
                else
                    t3w_vrr_group(o, R, q.o2ze, S);
                t3w_sync<G>();
            }
        }
    }
    // Phase 2: HRR and the stepwise transforms (Eq. hrr, Eqs. bra-sph .. stepwise-sph)
    const T3WHrr h{gb.abx, gb.aby, gb.abz, gk.abx, gk.aby, gk.abz};
    const uint4 *__restrict__ p2 = myops + (size_t)c.n_vrr;
    const int ng = c.n_p2 / T3W_OPS;
    uint4 nx[T3W_K];
#pragma unroll
    for (int k = 0; k < T3W_K; ++k) nx[k] = p2[k * T3W_GROUP];
    for (int g = 0; g < ng; ++g) {
        uint4 o[T3W_K];
#pragma unroll
        for (int k = 0; k < T3W_K; ++k) {
            o[k] = nx[k];
            nx[k] = p2[(size_t)(g + 1) * T3W_OPS + k * T3W_GROUP];
        }
        const uint32_t cls = __builtin_amdgcn_readfirstlane(o[0].x) & 15u;
        if (cls == (uint32_t)T3_HRR_BRA || cls == (uint32_t)T3_HRR_KET)
            t3w_hrr_group(o, h, S);
        else
            t3w_lin_group(o, C, S);
        t3w_sync<G>();
    }
}

// LDS of one workgroup: S (slots, Z, sink; in global memory when G),
// C (coefficients), Db (six D blocks), O (output slot of integral
// (mu, nu, lam, sig), row-major), R (the 16 per-primitive VRR constants).
struct T3WLds {
    double *S, *C, *Db, *R;
    uint16_t *O;
};

template <bool G>
__device__ __forceinline__ T3WLds t3w_lds(const T3WParams &c, double *base, double *gslots,
                                          const double *__restrict__ coefs, const uint16_t *__restrict__ outslots,
                                          int lane)
{
    T3WLds l;
    l.S = G ? gslots : base;
    l.C = G ? base : base + c.nslots + 2;
    l.Db = l.C + c.ncoef;
    l.O = (uint16_t *)(l.Db + 6 * c.maxblk);
    l.R = (double *)((char *)l.O + ((2 * c.nint + 15) / 16) * 16);      // 16-byte aligned
    for (int k = lane; k < c.ncoef; k += T3W_GROUP) l.C[k] = coefs[k];
    for (int k = lane; k < c.nint; k += T3W_GROUP) l.O[k] = outslots[k];
    return l;
}

extern __shared__ double t3w_smem[];

// G: the quartet's slots are a.scratch[blockIdx.x * (nslots + 2) ...].
template <bool G>
__global__ __launch_bounds__(64) void t3w_jk_kernel(T3WParams c, const uint4 *__restrict__ ops,
                                                    const double *__restrict__ coefs,
                                                    const uint16_t *__restrict__ outslots, JKArgs a)
{
    const int64_t i = blockIdx.x;
    if (i >= a.nq) return;
    const int lane = threadIdx.x;
    const T3WLds l = t3w_lds<G>(c, t3w_smem, G ? a.scratch + (size_t)i * (size_t)(c.nslots + 2) : nullptr, coefs,
                                outslots, lane);
    const int2 pq = a.quartets[i];
    const PairInfo pb = a.pairs[pq.x], pk = a.pairs[pq.y];
    const PairGeo gb = a.geo[pq.x], gk = a.geo[pq.y];
    // the six D blocks (global reads, overlapping the quartet's evaluation)
    const double *__restrict__ D = a.D;
    const int64_t N = a.nbf;
    const int fa = pb.fa, fb = pb.fb, fc = pk.fa, fd = pk.fb;
    const int na = c.na, nb = c.nb, nc = c.nc, nd = c.nd, M = c.maxblk;
    double *Dcd = l.Db, *Dab = l.Db + M, *Dbd = l.Db + 2 * M, *Dad = l.Db + 3 * M, *Dbc = l.Db + 4 * M,
           *Dac = l.Db + 5 * M;
    for (int k = lane; k < nc * nd; k += T3W_GROUP) Dcd[k] = D[(fc + k / nd) * N + fd + k % nd];
    for (int k = lane; k < na * nb; k += T3W_GROUP) Dab[k] = D[(fa + k / nb) * N + fb + k % nb];
    if (a.want_k) {
        for (int k = lane; k < nb * nd; k += T3W_GROUP) Dbd[k] = D[(fb + k / nd) * N + fd + k % nd];
        for (int k = lane; k < na * nd; k += T3W_GROUP) Dad[k] = D[(fa + k / nd) * N + fd + k % nd];
        for (int k = lane; k < nb * nc; k += T3W_GROUP) Dbc[k] = D[(fb + k / nc) * N + fc + k % nc];
        for (int k = lane; k < na * nc; k += T3W_GROUP) Dac[k] = D[(fa + k / nc) * N + fc + k % nc];
    }
    t3w_quartet<G>(c, ops, pb, gb, pk, gk, a.prims, a.boys, l.S, l.C, l.R, lane);
    const double *__restrict__ S = l.S;
    const uint16_t *__restrict__ O = l.O;
    auto I = [&](int mu, int nu, int lam, int sig) -> double {
        return S[O[((mu * nb + nu) * nc + lam) * nd + sig]];
    };
    const double s = (pb.same ? 0.5 : 1.0) * (pk.same ? 0.5 : 1.0) * (pq.x == pq.y ? 0.5 : 1.0);
    // J'[ab] += 2s sum_cd I D_cd, J'[cd] += 2s sum_ab I D_ab; K'[ac] += s sum I D_bd,
    // K'[bc] += s sum I D_ad, K'[ad] += s sum I D_bc, K'[bd] += s sum I D_ac
    // (unsymmetrised, degeneracy-scaled); one output element per lane
    if (a.want_j) {
        for (int k = lane; k < na * nb; k += T3W_GROUP) {
            const int mu = k / nb, nu = k % nb;
            double t = 0.0;
            for (int lam = 0; lam < nc; ++lam)
                for (int sig = 0; sig < nd; ++sig) t = fma(I(mu, nu, lam, sig), Dcd[lam * nd + sig], t);
            atomicAdd(a.J + (fa + mu) * N + fb + nu, 2.0 * s * t);
        }
        for (int k = lane; k < nc * nd; k += T3W_GROUP) {
            const int lam = k / nd, sig = k % nd;
            double t = 0.0;
            for (int mu = 0; mu < na; ++mu)
                for (int nu = 0; nu < nb; ++nu) t = fma(I(mu, nu, lam, sig), Dab[mu * nb + nu], t);
            atomicAdd(a.J + (fc + lam) * N + fd + sig, 2.0 * s * t);
        }
    }
    if (a.want_k) {
        for (int k = lane; k < na * nc; k += T3W_GROUP) {
            const int mu = k / nc, lam = k % nc;
            double t = 0.0;
            for (int nu = 0; nu < nb; ++nu)
                for (int sig = 0; sig < nd; ++sig) t = fma(I(mu, nu, lam, sig), Dbd[nu * nd + sig], t);
            atomicAdd(a.K + (fa + mu) * N + fc + lam, s * t);
        }
        for (int k = lane; k < nb * nc; k += T3W_GROUP) {
            const int nu = k / nc, lam = k % nc;
            double t = 0.0;
            for (int mu = 0; mu < na; ++mu)
                for (int sig = 0; sig < nd; ++sig) t = fma(I(mu, nu, lam, sig), Dad[mu * nd + sig], t);
            atomicAdd(a.K + (fb + nu) * N + fc + lam, s * t);
        }
        for (int k = lane; k < na * nd; k += T3W_GROUP) {
            const int mu = k / nd, sig = k % nd;
            double t = 0.0;
            for (int nu = 0; nu < nb; ++nu)
                for (int lam = 0; lam < nc; ++lam) t = fma(I(mu, nu, lam, sig), Dbc[nu * nc + lam], t);
            atomicAdd(a.K + (fa + mu) * N + fd + sig, s * t);
        }
        for (int k = lane; k < nb * nd; k += T3W_GROUP) {
            const int nu = k / nd, sig = k % nd;
            double t = 0.0;
            for (int mu = 0; mu < na; ++mu)
                for (int lam = 0; lam < nc; ++lam) t = fma(I(mu, nu, lam, sig), Dac[mu * nc + lam], t);
            atomicAdd(a.K + (fb + nu) * N + fd + sig, s * t);
        }
    }
}

template <bool G>
__global__ __launch_bounds__(64) void t3w_eri_kernel(T3WParams c, const uint4 *__restrict__ ops,
                                                     const double *__restrict__ coefs,
                                                     const uint16_t *__restrict__ outslots, EriArgs a)
{
    const int64_t i = blockIdx.x;
    if (i >= a.ntask) return;
    const int lane = threadIdx.x;
    const T3WLds l = t3w_lds<G>(c, t3w_smem, G ? a.scratch + (size_t)i * (size_t)(c.nslots + 2) : nullptr, coefs,
                                outslots, lane);
    const EriTask t = a.tasks[i];
    const PairInfo pb = a.pairs[t.bra], pk = a.pairs[t.ket];
    const PairGeo gb = a.geo[t.bra], gk = a.geo[t.ket];
    t3w_quartet<G>(c, ops, pb, gb, pk, gk, a.prims, a.boys, l.S, l.C, l.R, lane);
    const int na = c.na, nb = c.nb, nc = c.nc, nd = c.nd;
    if (a.mode == 1) {                       // Schwarz factor of a diagonal quartet
        double m = 0.0;
        for (int k = lane; k < na * nb; k += T3W_GROUP) {
            const int mu = k / nb, nu = k % nb;
            m = fmax(m, fabs(l.S[l.O[((mu * nb + nu) * nc + mu) * nd + nu]]));
        }
        for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
        if (lane == 0) a.out[i] = sqrt(m);
        return;
    }
    double *__restrict__ o = a.out + t.off;
    const int ncd = nc * nd;
    for (int mu = 0; mu < na; ++mu)
        for (int nu = 0; nu < nb; ++nu)
            for (int k = lane; k < ncd; k += T3W_GROUP) {
                const int lam = k / nd, sig = k % nd;
                o[mu * t.s0 + nu * t.s1 + lam * t.s2 + sig * t.s3] = l.S[l.O[(mu * nb + nu) * ncd + k]];
            }
}

// First-derivative integrals of quartet i (tables from gen/emit_deriv.py):
// the 12 blocks [centre][axis] of the canonical class, canonical centre r's
// written to the requested centre (code[t.bra / 2] >> 2r) & 3 of the
// shell-quartet classifier.
// P2: Phase 2 only, from the accumulators a.scratch[k * a.stride + i].
template <bool G, bool P2 = false>
__global__ __launch_bounds__(64) void t3w_deriv_kernel(T3WParams c, const uint4 *__restrict__ ops,
                                                       const double *__restrict__ coefs,
                                                       const uint16_t *__restrict__ outslots, EriArgs a,
                                                       const int32_t *__restrict__ code)
{
    const int64_t i = blockIdx.x;
    if (i >= a.ntask) return;
    const int lane = threadIdx.x;
    const T3WLds l = t3w_lds<G>(c, t3w_smem, G ? a.scratch + (size_t)i * (size_t)(c.nslots + 2) : nullptr, coefs,
                                outslots, lane);
    const EriTask t = a.tasks[i];
    const PairInfo pb = a.pairs[t.bra], pk = a.pairs[t.ket];
    const PairGeo gb = a.geo[t.bra], gk = a.geo[t.ket];
    t3w_quartet<G, P2>(c, ops, pb, gb, pk, gk, a.prims, a.boys, l.S, l.C, l.R, lane, P2 ? a.scratch + i : nullptr,
                       a.stride);
    const int na = c.na, nb = c.nb, nc = c.nc, nd = c.nd;
    const int nint = na * nb * nc * nd;
    const int32_t pos = code[t.bra >> 1];
    double *__restrict__ o = a.out + t.off;
    for (int k = lane; k < 12 * nint; k += T3W_GROUP) {
        const int blk = k / nint, r = k - blk * nint;          // blk = 3 * centre + axis
        const int centre = blk / 3, axis = blk - 3 * centre;
        const int req = (pos >> (2 * centre)) & 3;
        const int sig = r % nd, lam = (r / nd) % nc, nu = (r / (nd * nc)) % nb, mu = r / (nd * nc * nb);
        o[(int64_t)(3 * req + axis) * nint + mu * t.s0 + nu * t.s1 + lam * t.s2 + sig * t.s3] = l.S[l.O[k]];
    }
}

// Device copies of a class's tables, uploaded on first use on each device
// and kept until the process ends.
std::mutex g_t3_mutex;
std::map<std::pair<const T3Class *, int>, T3Dev> g_t3_dev;

hipError_t t3_device_tables(const T3Class &c, T3Dev *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_t3_mutex);
    auto it = g_t3_dev.find({&c, dev});
    if (it != g_t3_dev.end()) {
        *out = it->second;
        return hipSuccess;
    }
    // zero groups past the end: the wave variant loads group g + 1 while it runs group g
    const size_t nops = (size_t)(c.n_vrr + c.n_p2),
                 nout = (size_t)c.na * c.nb * c.nc * c.nd * (size_t)(c.out_blocks > 1 ? c.out_blocks : 1);
    const size_t npad = (size_t)T3W_PREFETCH * T3W_OPS;
    void *ops = nullptr, *coefs = nullptr, *outs = nullptr;
    if ((e = hipMalloc(&ops, (nops + npad) * 16)) != hipSuccess ||
        (e = hipMemset(ops, 0, (nops + npad) * 16)) != hipSuccess ||
        (e = hipMalloc(&coefs, sizeof(double) * c.ncoef)) != hipSuccess ||
        (e = hipMalloc(&outs, sizeof(uint16_t) * nout)) != hipSuccess ||
        (e = hipMemcpy(ops, c.ops, nops * 16, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(coefs, c.coefs, sizeof(double) * c.ncoef, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(outs, c.outslots, sizeof(uint16_t) * nout, hipMemcpyHostToDevice)) != hipSuccess) {
        (void)hipFree(ops);
        (void)hipFree(coefs);
        (void)hipFree(outs);
        return e;
    }
    T3Dev d{(const uint4 *)ops, (const double *)coefs, (const uint16_t *)outs};
    g_t3_dev[{&c, dev}] = d;
    *out = d;
    return hipSuccess;
}

T3Params params(const T3Class &c)
{
    return T3Params{c.L, c.na, c.nb, c.nc, c.nd, c.n_hrr, c.acc0, c.n_vrr, c.n_p2};
}

}  // namespace

// Wave-variant classes: the workgroup's LDS must fit the device's per-block
// limit (160 KB on gfx950); launches above 64 KB need the kernels' dynamic
// LDS limit raised once per device.
int t3_prepare(const T3Class &c)
{
    if (c.lane) {
        const int e = t3_prepare(*c.lane);
        if (e != 0) return e;
    }
    if (c.lds_bytes > 0) {
        int dev = 0, maxlds = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (e != hipSuccess) return (int)e;
        if (c.lds_bytes > maxlds) return (int)hipErrorInvalidConfiguration;
        if (c.lds_bytes > 65536) {
            static std::mutex mu;
            static bool raised[64] = {};
            std::lock_guard<std::mutex> lock(mu);
            if (dev < 0 || dev >= 64) return (int)hipErrorInvalidDevice;
            if (!raised[dev]) {
                if ((e = hipFuncSetAttribute((const void *)t3w_jk_kernel<false>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, maxlds)) != hipSuccess ||
                    (e = hipFuncSetAttribute((const void *)t3w_eri_kernel<false>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, maxlds)) != hipSuccess ||
                    (e = hipFuncSetAttribute((const void *)t3w_deriv_kernel<false>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, maxlds)) != hipSuccess ||
                    (e = hipFuncSetAttribute((const void *)t3w_deriv_kernel<false, true>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, maxlds)) != hipSuccess)
                    return (int)e;
                raised[dev] = true;
            }
        }
    }
    T3Dev d;
    return (int)t3_device_tables(c, &d);
}

// The runtime calls t3_prepare before it launches a class, so the lookup
// below only finds tables that are already on the device.
void t3_launch_jk(const T3Class &c, const JKArgs &a, hipStream_t s)
{
    T3Dev d;
    if (a.nq <= 0 || t3_device_tables(c, &d) != hipSuccess) return;
    hipLaunchKernelGGL(t3_jk_kernel, dim3((unsigned)((a.nq + c.block - 1) / c.block)), dim3(c.block), 0, s, params(c),
                       d.ops, d.coefs, d.outslots, a);
}

namespace {
T3WParams wparams(const T3Class &c)
{
    return T3WParams{c.L,      c.na,    c.nb,        c.nc,    c.nd,     c.n_hrr, c.acc0,
                     c.n_vrr,  c.n_p2,  c.nslots,    c.ncoef, c.maxblk, c.na * c.nb * c.nc * c.nd};
}
}  // namespace

// One workgroup per quartet; the runtime keeps a launch under 2^26 quartets
// (and, for the global-slot variant, within the batch its buffer holds).
void t3w_launch_jk(const T3Class &c, const JKArgs &a, hipStream_t s)
{
    T3Dev d;
    if (a.nq <= 0 || c.lds_bytes <= 0 || t3_device_tables(c, &d) != hipSuccess) return;
    if (c.gslots) {
        if (a.nq >= T3G_LANE_MIN && c.lane) {      // large batch: one lane per quartet, stride a.stride
            t3_launch_jk(*c.lane, a, s);
            return;
        }
        // launches of at most T3G_CHUNK quartets, each reusing the first regions of the buffer
        for (int64_t q0 = 0; q0 < a.nq; q0 += T3G_CHUNK) {
            JKArgs b = a;
            b.quartets = a.quartets + q0;
            b.nq = std::min<int64_t>(T3G_CHUNK, a.nq - q0);
            hipLaunchKernelGGL(t3w_jk_kernel<true>, dim3((unsigned)b.nq), dim3(T3W_GROUP), (unsigned)c.lds_bytes, s,
                               wparams(c), d.ops, d.coefs, d.outslots, b);
        }
    } else
        hipLaunchKernelGGL(t3w_jk_kernel<false>, dim3((unsigned)a.nq), dim3(T3W_GROUP), (unsigned)c.lds_bytes, s,
                           wparams(c), d.ops, d.coefs, d.outslots, a);
}

void t3w_launch_eri(const T3Class &c, const EriArgs &a, hipStream_t s)
{
    T3Dev d;
    if (a.ntask <= 0 || c.lds_bytes <= 0 || t3_device_tables(c, &d) != hipSuccess) return;
    if (c.gslots) {
        if (a.ntask >= T3G_LANE_MIN && c.lane) {
            t3_launch_eri(*c.lane, a, s);
            return;
        }
        for (int64_t q0 = 0; q0 < a.ntask; q0 += T3G_CHUNK) {
            EriArgs b = a;
            b.tasks = a.tasks + q0;
            b.ntask = std::min<int64_t>(T3G_CHUNK, a.ntask - q0);
            if (a.mode == 1) b.out = a.out + q0;
            hipLaunchKernelGGL(t3w_eri_kernel<true>, dim3((unsigned)b.ntask), dim3(T3W_GROUP), (unsigned)c.lds_bytes,
                               s, wparams(c), d.ops, d.coefs, d.outslots, b);
        }
    } else
        hipLaunchKernelGGL(t3w_eri_kernel<false>, dim3((unsigned)a.ntask), dim3(T3W_GROUP), (unsigned)c.lds_bytes, s,
                           wparams(c), d.ops, d.coefs, d.outslots, a);
}

void t3w_launch_deriv(const T3Class &c, const EriArgs &a, const int32_t *code, hipStream_t s)
{
    T3Dev d;
    if (a.ntask <= 0 || c.lds_bytes <= 0 || c.gslots || c.out_blocks != 12 || t3_device_tables(c, &d) != hipSuccess)
        return;
    T3WParams p = wparams(c);
    p.nint *= 12;
    p.deriv = 1;
    hipLaunchKernelGGL(t3w_deriv_kernel<false>, dim3((unsigned)a.ntask), dim3(T3W_GROUP), (unsigned)c.lds_bytes, s, p,
                       d.ops, d.coefs, d.outslots, a, code);
}

void t3w_launch_deriv_p2(const T3Class &c, const EriArgs &a, const int32_t *code, int nseg, hipStream_t s)
{
    T3Dev d;
    if (a.ntask <= 0 || nseg < 1 || c.lds_bytes <= 0 || c.gslots || c.out_blocks != 12 || !a.scratch ||
        t3_device_tables(c, &d) != hipSuccess)
        return;
    T3WParams p = wparams(c);
    p.nint *= 12;
    p.deriv = 1;
    p.nseg = nseg;
    hipLaunchKernelGGL((t3w_deriv_kernel<false, true>), dim3((unsigned)a.ntask), dim3(T3W_GROUP),
                       (unsigned)c.lds_bytes, s, p, d.ops, d.coefs, d.outslots, a, code);
}

void t3_launch_eri(const T3Class &c, const EriArgs &a, hipStream_t s)
{
    T3Dev d;
    if (a.ntask <= 0 || t3_device_tables(c, &d) != hipSuccess) return;
    hipLaunchKernelGGL(t3_eri_kernel, dim3((unsigned)((a.ntask + c.block - 1) / c.block)), dim3(c.block), 0, s,
                       params(c), d.ops, d.coefs, d.outslots, a);
}

}  // namespace hgp
