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
    const size_t nops = (size_t)(c.n_vrr + c.n_p2), nout = (size_t)c.na * c.nb * c.nc * c.nd;
    void *ops = nullptr, *coefs = nullptr, *outs = nullptr;
    if ((e = hipMalloc(&ops, nops * 16)) != hipSuccess || (e = hipMalloc(&coefs, sizeof(double) * c.ncoef)) != hipSuccess ||
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

int t3_prepare(const T3Class &c)
{
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

void t3_launch_eri(const T3Class &c, const EriArgs &a, hipStream_t s)
{
    T3Dev d;
    if (a.ntask <= 0 || t3_device_tables(c, &d) != hipSuccess) return;
    hipLaunchKernelGGL(t3_eri_kernel, dim3((unsigned)((a.ntask + c.block - 1) / c.block)), dim3(c.block), 0, s,
                       params(c), d.ops, d.coefs, d.outslots, a);
}

}  // namespace hgp
