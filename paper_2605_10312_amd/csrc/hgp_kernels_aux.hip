// Hand-written device kernels around the generated class kernels: the Boys
// table, contraction normalisation, shell-pair / primitive-pair precompute,
// Schwarz screening with class-list compaction, zero fill and J/K
// symmetrisation.
#include "hgp_aux.h"

namespace hgp {

// ---------------------------------------------------------------------------
// Boys table: F_m(k h) for m = 0 .. BOYS_NORD-1 from the series
// F_m(T) = exp(-T) sum_j (2T)^j / ((2m+1)(2m+3)...(2m+2j+1)) for the top
// order, then the downward recurrence.  One thread per grid point.
// ---------------------------------------------------------------------------
__global__ void boys_table_kernel(double *tab)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= BOYS_NPTS) return;
    const double T = k * BOYS_STEP;
    const int top = BOYS_NORD - 1;
    double term = 1.0 / (2 * top + 1), sum = term;
    for (int j = 1; j < 2000; ++j) {
        term *= 2.0 * T / (double)(2 * top + 2 * j + 1);
        sum += term;
        if (term < sum * 1e-18) break;
    }
    const double e = exp(-T);
    double f = e * sum;
    tab[k * BOYS_STRIDE + top] = f;
    for (int m = top - 1; m >= 0; --m) {
        f = (2.0 * T * f + e) / (double)(2 * m + 1);
        tab[k * BOYS_STRIDE + m] = f;
    }
    tab[k * BOYS_STRIDE + BOYS_NORD] = e;
}

// ---------------------------------------------------------------------------
// Contraction normalisation, one thread per shell:
// c_k = d_k N(a_k, l) / sqrt(sum_kk' d_k d_k' [2 sqrt(a_k a_k')/(a_k + a_k')]^(l+3/2)),
// N(a, l) = (2a/pi)^(3/4) (4a)^(l/2) / sqrt((2l-1)!!).
// ---------------------------------------------------------------------------
__global__ void normalize_kernel(int nshell, const int *l, const int *nprim, const int *poff, const double *exps,
                                 const double *coefs, double *out)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nshell) return;
    const int L = l[s], n = nprim[s], o = poff[s];
    double ovl = 0.0;
    for (int k = 0; k < n; ++k)
        for (int q = 0; q < n; ++q) {
            const double a = exps[o + k], b = exps[o + q];
            ovl += coefs[o + k] * coefs[o + q] * pow(2.0 * sqrt(a * b) / (a + b), L + 1.5);
        }
    double df = 1.0;
    for (int k = 2 * L - 1; k > 1; k -= 2) df *= k;
    const double scale = 1.0 / sqrt(ovl);
    for (int k = 0; k < n; ++k) {
        const double a = exps[o + k];
        const double nrm = pow(2.0 * a / 3.14159265358979323846, 0.75) * pow(4.0 * a, 0.5 * L) / sqrt(df);
        out[o + k] = coefs[o + k] * nrm * scale;
    }
}

// ---------------------------------------------------------------------------
// Pair precompute (Alg. 2's GaussianPairs hoisted out of the quartet loops),
// one thread per shell pair: geometry and one PrimPair record per primitive
// pair.
// ---------------------------------------------------------------------------
__global__ void pair_kernel(int npair, const PairInfo *pairs, const double *cen, const int *poff,
                            const double *exps, const double *ncoef, PairGeo *geo, PrimPair *prims)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npair) return;
    const PairInfo pi = pairs[p];
    const double Ax = cen[3 * pi.sh_a], Ay = cen[3 * pi.sh_a + 1], Az = cen[3 * pi.sh_a + 2];
    const double Bx = cen[3 * pi.sh_b], By = cen[3 * pi.sh_b + 1], Bz = cen[3 * pi.sh_b + 2];
    const double abx = Ax - Bx, aby = Ay - By, abz = Az - Bz;
    const double ab2 = abx * abx + aby * aby + abz * abz;
    PairGeo g;
    g.ax = Ax; g.ay = Ay; g.az = Az;
    g.abx = abx; g.aby = aby; g.abz = abz;
    g.q = 0.0; g.pad = 0.0;
    geo[p] = g;
    const int oa = poff[pi.sh_a], ob = poff[pi.sh_b];
    const int nb = poff[pi.sh_b + 1] - ob;
    const double pref = sqrt(2.0) * pow(3.14159265358979323846, 1.25);   // sqrt(2) pi^(5/4)
    for (int r = 0; r < pi.nprim; ++r) {
        const int ka = r / nb, kb = r % nb;
        const double a = exps[oa + ka], b = exps[ob + kb];
        const double z = a + b, iz = 1.0 / z;
        PrimPair pp;
        pp.zeta = z;
        pp.o2z = 0.5 * iz;
        pp.px = (a * Ax + b * Bx) * iz;
        pp.py = (a * Ay + b * By) * iz;
        pp.pz = (a * Az + b * Bz) * iz;
        pp.k = ncoef[oa + ka] * ncoef[ob + kb] * exp(-a * b * iz * ab2) * pref * iz;
        pp.ea = a; pp.eb = b;
        prims[pi.prim_off + r] = pp;
    }
}

// Primitive-quartet microbench input: quartet q uses pairs 2q (bra) and 2q+1
// (ket), one primitive pair each; role r of the canonical class reads the
// caller's centre/exponent slot perm[r]; coefficient N(a, l).
__global__ void prim_quartet_pair_kernel(int64_t n, const double *centers, const double *exps, int la, int lb, int lc,
                                         int ld, int4 perm, int4 strides, int64_t block, PairInfo *pairs,
                                         PairGeo *geo, PrimPair *prims, EriTask *tasks)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int slot[4] = {perm.x, perm.y, perm.z, perm.w};
    const int ls[4] = {la, lb, lc, ld};
    for (int side = 0; side < 2; ++side) {
        const int r0 = 2 * side, r1 = 2 * side + 1;
        const double *A = centers + 12 * q + 3 * slot[r0];
        const double *B = centers + 12 * q + 3 * slot[r1];
        const double a = exps[4 * q + slot[r0]], b = exps[4 * q + slot[r1]];
        double nrm[2];
        for (int t = 0; t < 2; ++t) {
            const int L = ls[r0 + t];
            const double x = t ? b : a;
            double df = 1.0;
            for (int k = 2 * L - 1; k > 1; k -= 2) df *= k;
            nrm[t] = pow(2.0 * x / 3.14159265358979323846, 0.75) * pow(4.0 * x, 0.5 * L) / sqrt(df);
        }
        const int64_t p = 2 * q + side;
        PairInfo pi;
        pi.sh_a = pi.sh_b = -1;
        pi.prim_off = (int32_t)p;
        pi.nprim = 1;
        pi.fa = pi.fb = 0;
        pi.same = 0;
        pi.cls = 0;
        pairs[p] = pi;
        const double abx = A[0] - B[0], aby = A[1] - B[1], abz = A[2] - B[2];
        PairGeo g;
        g.ax = A[0]; g.ay = A[1]; g.az = A[2];
        g.abx = abx; g.aby = aby; g.abz = abz;
        g.q = 0.0; g.pad = 0.0;
        geo[p] = g;
        const double z = a + b, iz = 1.0 / z;
        PrimPair pp;
        pp.zeta = z;
        pp.o2z = 0.5 * iz;
        pp.px = (a * A[0] + b * B[0]) * iz;
        pp.py = (a * A[1] + b * B[1]) * iz;
        pp.pz = (a * A[2] + b * B[2]) * iz;
        pp.k = nrm[0] * nrm[1] * exp(-a * b * iz * (abx * abx + aby * aby + abz * abz)) * sqrt(2.0) *
               pow(3.14159265358979323846, 1.25) * iz;
        pp.ea = a; pp.eb = b;
        prims[p] = pp;
    }
    EriTask t;
    t.bra = (int32_t)(2 * q);
    t.ket = (int32_t)(2 * q + 1);
    t.off = q * block;
    t.s0 = strides.x; t.s1 = strides.y; t.s2 = strides.z; t.s3 = strides.w;
    tasks[q] = t;
}

// ---------------------------------------------------------------------------
// Screening and class lists.  For one class, bra pairs are rows
// [b0, b0+nb) and ket pairs [k0, k0+nk) of the global pair arrays; when
// the bra and ket pair classes coincide only ket <= bra is a unique quartet.
// A quartet is kept when tau <= Q_bra * Q_ket < hi.  One block per row.
// Bra rows b0 .. b0 + nb - 1 of one pair class; the ket candidates of a row
// are the ket class's pairs of the same system, kbeg[sys] .. kbeg[sys] +
// kcnt[sys] - 1 (psys: system of each pair); within one class (sym) only
// those up to the row itself.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void ket_range(int row, int sym, const int *psys, const int *kbeg, const int *kcnt,
                                          int *k0, int *len)
{
    const int sy = psys[row];
    *k0 = kbeg[sy];
    *len = sym ? (row - kbeg[sy] + 1) : kcnt[sy];
}

// Per bra row: the kets kept (counts) and the sum of their primitive-pair
// counts (pcounts, the row's primitive quartets divided by its own count).
__global__ void screen_count_kernel(int b0, int nb, int sym, const double *Q, double tau, double hi,
                                    const int *psys, const int *kbeg, const int *kcnt, const int *npr,
                                    int64_t *counts, int64_t *pcounts)
{
    const int row = b0 + blockIdx.x;
    int k0, len;
    ket_range(row, sym, psys, kbeg, kcnt, &k0, &len);
    const double qb = Q[row];
    int c = 0;
    int64_t pc = 0;
    for (int j = threadIdx.x; j < len; j += blockDim.x) {
        const double qq = qb * Q[k0 + j];
        const bool keep = qq >= tau && qq < hi;
        c += keep ? 1 : 0;
        pc += keep ? npr[k0 + j] : 0;
    }
    __shared__ int part[1024 / 64];
    __shared__ int64_t ppart[1024 / 64];
    // wave reduction
    for (int off = 32; off > 0; off >>= 1) {
        c += __shfl_down(c, off, 64);
        pc += __shfl_down(pc, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        part[threadIdx.x >> 6] = c;
        ppart[threadIdx.x >> 6] = pc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        int64_t pt = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            t += part[w];
            pt += ppart[w];
        }
        counts[blockIdx.x] = t;
        pcounts[blockIdx.x] = pt;
    }
}

// ---------------------------------------------------------------------------
// Shell quartets given on the device (integrals out, any shell order).
// Classify: one thread per quartet validates its shells and offset, puts the
// four shells in the canonical order of the class kernels (the larger l
// first within each pair, then the pair of higher pair class as bra), looks
// up the class and counts it.  code = class << 8 | pos[0] | pos[1] << 2 |
// pos[2] << 4 | pos[3] << 6, pos[r] = requested position of canonical role r.
// ---------------------------------------------------------------------------
__device__ inline int dev_pair_class(int la, int lb) { return la * (la + 1) / 2 + lb; }

__global__ __launch_bounds__(256) void sq_classify_kernel(int64_t nq, const int32_t *quartets,
                                                           const int64_t *offsets, int nshell, const int *l,
                                                           const int *nprim, ClassOf class_of, int nkeys,
                                                           int32_t *code, int64_t *primcnt,
                                                           unsigned long long *counts, unsigned long long *err)
{
    // per-key counts of the block in LDS, then one global atomic per key present
    extern __shared__ unsigned sq_hist[];
    for (int j = threadIdx.x; j < nkeys; j += blockDim.x) sq_hist[j] = 0u;
    __syncthreads();
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nq) {
        int sh[4];
        bool bad = offsets[q] < 0;
        for (int r = 0; r < 4; ++r) {
            sh[r] = quartets[4 * q + r];
            bad = bad || sh[r] < 0 || sh[r] >= nshell;
        }
        int key = -1;
        if (bad) {
            atomicOr(err, 1ull);
        } else {
            int L[4];
            for (int r = 0; r < 4; ++r) L[r] = l[sh[r]];
            int pos[4] = {0, 1, 2, 3};
            if (L[0] < L[1]) { pos[0] = 1; pos[1] = 0; }
            if (L[2] < L[3]) { pos[2] = 3; pos[3] = 2; }
            if (dev_pair_class(L[pos[0]], L[pos[1]]) < dev_pair_class(L[pos[2]], L[pos[3]])) {
                int t = pos[0]; pos[0] = pos[2]; pos[2] = t;
                t = pos[1]; pos[1] = pos[3]; pos[3] = t;
            }
            const int ci = class_of.c[((L[pos[0]] * 5 + L[pos[1]]) * 5 + L[pos[2]]) * 5 + L[pos[3]]];
            if (ci < 0) {
                atomicOr(err, 2ull);
            } else {
                const int64_t nb = (int64_t)nprim[sh[0]] * nprim[sh[1]], nk = (int64_t)nprim[sh[2]] * nprim[sh[3]];
                // most primitive quartets first: bucket floor(log2(n_bra n_ket)), reversed
                const int lg = 63 - __builtin_clzll((unsigned long long)(nb * nk));
                key = ci * SQ_BUCKETS + (SQ_BUCKETS - 1 - min(lg, SQ_BUCKETS - 1));
                atomicAdd(&sq_hist[key], 1u);
                code[q] = key << 8 | pos[0] | pos[1] << 2 | pos[2] << 4 | pos[3] << 6;
                primcnt[q] = nb + nk;
            }
        }
        if (key < 0) {
            code[q] = -1;
            primcnt[q] = 0;
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < nkeys; j += blockDim.x)
        if (sq_hist[j]) atomicAdd(&counts[j], (unsigned long long)sq_hist[j]);
}

// Scatter: the two pair records of quartet q (2q bra, 2q + 1 ket, primitive
// records from prim_off[q], an exclusive scan of the classify counts) and its
// task, placed in its class's range (class_base, an exclusive scan of the
// class counts) at a slot taken from that class's cursor.
__global__ __launch_bounds__(256) void sq_scatter_kernel(int64_t nq, const int32_t *quartets, const int64_t *offsets,
                                                          const int *l, const int *nprim, const int *foff,
                                                          const int32_t *code, const int64_t *prim_off,
                                                          const int64_t *key_base, int nkeys,
                                                          unsigned long long *cursor, PairInfo *pairs, EriTask *tasks)
{
    // a quartet's slot: its key's base + the block's share of the key's
    // cursor (one global atomic per key present) + its rank in the block
    extern __shared__ unsigned long long sq_blk[];
    unsigned *hist = (unsigned *)(sq_blk + nkeys);
    for (int j = threadIdx.x; j < nkeys; j += blockDim.x) hist[j] = 0u;
    __syncthreads();
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t c = q < nq ? code[q] : -1;
    const int key = c >> 8;             // -1 for no quartet (the runtime scatters only valid codes)
    unsigned rank = 0u;
    EriTask t;
    if (c >= 0) {
        rank = atomicAdd(&hist[key], 1u);
        int sh[4], pos[4], n[4], stride[4];
        for (int r = 0; r < 4; ++r) {
            sh[r] = quartets[4 * q + r];
            pos[r] = (c >> (2 * r)) & 3;
            n[r] = 2 * l[sh[r]] + 1;
        }
        stride[3] = 1; stride[2] = n[3]; stride[1] = n[2] * n[3]; stride[0] = n[1] * n[2] * n[3];
        int64_t po = prim_off[q];
        for (int side = 0; side < 2; ++side) {
            PairInfo pi;
            pi.sh_a = sh[pos[2 * side]];
            pi.sh_b = sh[pos[2 * side + 1]];
            pi.prim_off = (int32_t)po;
            pi.nprim = nprim[pi.sh_a] * nprim[pi.sh_b];
            pi.fa = foff[pi.sh_a];
            pi.fb = foff[pi.sh_b];
            pi.same = pi.sh_a == pi.sh_b;
            pi.cls = dev_pair_class(l[pi.sh_a], l[pi.sh_b]);
            po += pi.nprim;
            pairs[2 * q + side] = pi;
        }
        t.bra = (int32_t)(2 * q);
        t.ket = (int32_t)(2 * q + 1);
        t.off = offsets[q];
        t.s0 = stride[pos[0]]; t.s1 = stride[pos[1]]; t.s2 = stride[pos[2]]; t.s3 = stride[pos[3]];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < nkeys; j += blockDim.x)
        if (hist[j]) sq_blk[j] = atomicAdd(&cursor[j], (unsigned long long)hist[j]);
    __syncthreads();
    if (c >= 0) tasks[key_base[key] + (int64_t)sq_blk[key] + rank] = t;
}

// Exclusive scan of the 1024-element block b of v in place (LDS), its sum into bsum[b].
__global__ __launch_bounds__(1024) void scan_block_kernel(int64_t *v, int64_t n, int64_t *bsum)
{
    __shared__ int64_t buf[1024];
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    const int64_t x = i < n ? v[i] : 0;
    buf[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t y = threadIdx.x >= (unsigned)off ? buf[threadIdx.x - off] : 0;
        __syncthreads();
        buf[threadIdx.x] += y;
        __syncthreads();
    }
    if (i < n) v[i] = buf[threadIdx.x] - x;
    if (threadIdx.x == 1023) bsum[blockIdx.x] = buf[1023];
}

// Adds boff[b] (the exclusive scan of the block sums) to block b of v.
__global__ __launch_bounds__(1024) void scan_add_kernel(int64_t *v, int64_t n, const int64_t *boff)
{
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    if (i < n) v[i] += boff[blockIdx.x];
}

// exclusive scan of n counts in place (single block), total into *total
__global__ void scan_kernel(int64_t *v, int n, int64_t *total)
{
    __shared__ int64_t buf[1024];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += blockDim.x) {
        const int i = base + threadIdx.x;
        const int64_t x = (i < n) ? v[i] : 0;
        buf[threadIdx.x] = x;
        __syncthreads();
        for (int off = 1; off < (int)blockDim.x; off <<= 1) {
            const int64_t y = (threadIdx.x >= (unsigned)off) ? buf[threadIdx.x - off] : 0;
            __syncthreads();
            buf[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < n) v[i] = carry + buf[threadIdx.x] - x;
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) carry += buf[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// Writes the kept (bra, ket) pairs of rows b0 .. b0 + nb - 1, row r's at
// out[offsets[r - b0] - shift ...] (shift: the first row's offset when out
// holds only a chunk of the class list).
__global__ void screen_write_kernel(int b0, int nb, int sym, const double *Q, double tau, double hi,
                                    const int *psys, const int *kbeg, const int *kcnt, const int64_t *offsets,
                                    int64_t shift, int2 *out)
{
    const int row = b0 + blockIdx.x;
    int k0, len;
    ket_range(row, sym, psys, kbeg, kcnt, &k0, &len);
    const double qb = Q[row];
    __shared__ int wcount[1024 / 64];
    __shared__ int64_t base;
    if (threadIdx.x == 0) base = offsets[blockIdx.x] - shift;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int j0 = 0; j0 < len; j0 += blockDim.x) {
        const int j = j0 + threadIdx.x;
        const double qq = j < len ? qb * Q[k0 + j] : 0.0;
        const bool keep = (j < len) && qq >= tau && qq < hi;
        const unsigned long long m = __ballot(keep);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wcount[wv] = __popcll(m);
        __syncthreads();
        int woff = 0, tot = 0;
        for (int w = 0; w < nw; ++w) {
            if (w < wv) woff += wcount[w];
            tot += wcount[w];
        }
        if (keep) out[base + woff + before] = make_int2(row, k0 + j);
        __syncthreads();
        if (threadIdx.x == 0) base += tot;
        __syncthreads();
    }
}

// Q[p] for every pair from the Schwarz tasks' outputs, also into the geometry
__global__ void store_q_kernel(int npair, const double *qv, PairGeo *geo, double *Q)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npair) return;
    Q[p] = qv[p];
    geo[p].q = qv[p];
}

__global__ void fill_zero_kernel(double *x, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = 0.0;
}

// out[i][j] = acc[i][j] + acc[j][i] for an n x n block; acc rows astride apart
__global__ void symmetrize_kernel(const double *acc, int64_t astride, double *out, int n)
{
    const int i = blockIdx.y * 16 + threadIdx.y, j = blockIdx.x * 16 + threadIdx.x;
    if (i >= n || j >= n) return;
    out[(int64_t)i * n + j] = acc[(int64_t)i * astride + j] + acc[(int64_t)j * astride + i];
}

// dst[i * dstride + j] = src[i * n + j] (an n x n block into a strided layout)
__global__ void block_in_kernel(const double *src, int n, double *dst, int64_t dstride)
{
    const int i = blockIdx.y * 16 + threadIdx.y, j = blockIdx.x * 16 + threadIdx.x;
    if (i >= n || j >= n) return;
    dst[(int64_t)i * dstride + j] = src[(int64_t)i * n + j];
}

// zero an n x n block of a strided layout
__global__ void block_zero_kernel(double *dst, int n, int64_t dstride)
{
    const int i = blockIdx.y * 16 + threadIdx.y, j = blockIdx.x * 16 + threadIdx.x;
    if (i >= n || j >= n) return;
    dst[(int64_t)i * dstride + j] = 0.0;
}

// ---------------------------------------------------------------------------
// host launch wrappers
// ---------------------------------------------------------------------------
void launch_boys_table(double *tab, hipStream_t s)
{
    hipLaunchKernelGGL(boys_table_kernel, dim3((BOYS_NPTS + 127) / 128), dim3(128), 0, s, tab);
}
void launch_normalize(int nshell, const int *l, const int *nprim, const int *poff, const double *exps,
                      const double *coefs, double *out, hipStream_t s)
{
    if (nshell > 0)
        hipLaunchKernelGGL(normalize_kernel, dim3((nshell + 127) / 128), dim3(128), 0, s, nshell, l, nprim, poff,
                           exps, coefs, out);
}
void launch_pairs(int npair, const PairInfo *pairs, const double *cen, const int *poff, const double *exps,
                  const double *ncoef, PairGeo *geo, PrimPair *prims, hipStream_t s)
{
    if (npair > 0)
        hipLaunchKernelGGL(pair_kernel, dim3((npair + 127) / 128), dim3(128), 0, s, npair, pairs, cen, poff, exps,
                           ncoef, geo, prims);
}
void launch_prim_quartet_pairs(int64_t n, const double *centers, const double *exps, const int ls[4],
                               const int perm[4], const int strides[4], int64_t block, PairInfo *pairs,
                               PairGeo *geo, PrimPair *prims, EriTask *tasks, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(prim_quartet_pair_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, centers,
                           exps, ls[0], ls[1], ls[2], ls[3], make_int4(perm[0], perm[1], perm[2], perm[3]),
                           make_int4(strides[0], strides[1], strides[2], strides[3]), block, pairs, geo, prims,
                           tasks);
}
void launch_screen_count(int b0, int nb, int sym, const double *Q, double tau, double hi, const int *psys,
                         const int *kbeg, const int *kcnt, const int *npr, int64_t *counts, int64_t *pcounts,
                         hipStream_t s)
{
    if (nb > 0)
        hipLaunchKernelGGL(screen_count_kernel, dim3(nb), dim3(256), 0, s, b0, nb, sym, Q, tau, hi, psys, kbeg, kcnt,
                           npr, counts, pcounts);
}
void launch_screen_write(int b0, int nb, int sym, const double *Q, double tau, double hi, const int *psys,
                         const int *kbeg, const int *kcnt, const int64_t *offsets, int64_t shift, int2 *out,
                         hipStream_t s)
{
    if (nb > 0)
        hipLaunchKernelGGL(screen_write_kernel, dim3(nb), dim3(256), 0, s, b0, nb, sym, Q, tau, hi, psys, kbeg, kcnt,
                           offsets, shift, out);
}
void launch_scan(int64_t *v, int n, int64_t *total, int64_t *tmp, hipStream_t s)
{
    const int nb = (n + 1023) / 1024;
    if (nb <= 1 || !tmp) {
        hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, v, n, total);
        return;
    }
    hipLaunchKernelGGL(scan_block_kernel, dim3((unsigned)nb), dim3(1024), 0, s, v, (int64_t)n, tmp);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, tmp, nb, total);
    hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)nb), dim3(1024), 0, s, v, (int64_t)n, (const int64_t *)tmp);
}
void launch_sq_classify(int64_t nq, const int32_t *quartets, const int64_t *offsets, int nshell, const int *l,
                        const int *nprim, const ClassOf &class_of, int nkeys, int32_t *code, int64_t *primcnt,
                        unsigned long long *counts, unsigned long long *err, hipStream_t s)
{
    if (nq > 0)
        hipLaunchKernelGGL(sq_classify_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256),
                           (unsigned)(sizeof(unsigned) * nkeys), s, nq, quartets, offsets, nshell, l, nprim, class_of,
                           nkeys, code, primcnt, counts, err);
}
void launch_sq_scatter(int64_t nq, const int32_t *quartets, const int64_t *offsets, const int *l, const int *nprim,
                       const int *foff, const int32_t *code, const int64_t *prim_off, const int64_t *key_base,
                       int nkeys, unsigned long long *cursor, PairInfo *pairs, EriTask *tasks, hipStream_t s)
{
    if (nq > 0)
        hipLaunchKernelGGL(sq_scatter_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256),
                           (unsigned)((sizeof(unsigned long long) + sizeof(unsigned)) * nkeys), s, nq, quartets,
                           offsets, l, nprim, foff, code, prim_off, key_base, nkeys, cursor, pairs, tasks);
}
void launch_store_q(int npair, const double *qv, PairGeo *geo, double *Q, hipStream_t s)
{
    if (npair > 0) hipLaunchKernelGGL(store_q_kernel, dim3((npair + 255) / 256), dim3(256), 0, s, npair, qv, geo, Q);
}
void launch_fill_zero(double *x, int64_t n, hipStream_t s)
{
    if (n > 0) {
        int64_t blocks = (n + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, n);
    }
}
void launch_symmetrize(const double *acc, int64_t astride, double *out, int n, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(symmetrize_kernel, dim3((n + 15) / 16, (n + 15) / 16), dim3(16, 16), 0, s, acc, astride,
                           out, n);
}
void launch_block_in(const double *src, int n, double *dst, int64_t dstride, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(block_in_kernel, dim3((n + 15) / 16, (n + 15) / 16), dim3(16, 16), 0, s, src, n, dst,
                           dstride);
}
void launch_block_zero(double *dst, int n, int64_t dstride, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(block_zero_kernel, dim3((n + 15) / 16, (n + 15) / 16), dim3(16, 16), 0, s, dst, n, dstride);
}

}  // namespace hgp
