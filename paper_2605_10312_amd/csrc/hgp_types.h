// Data layout shared by the host runtime and the generated class kernels.
// Everything lives in HBM; sizes are per plan.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hgp {

// One shell pair (a, b) with l_a >= l_b, in the role of a bra or a ket.
// 32 bytes.  prim_off/nprim index the primitive-pair records.
struct PairInfo {
    int32_t sh_a, sh_b;     // shell indices
    int32_t prim_off;       // first primitive-pair record
    int32_t nprim;          // number of primitive pairs (n_a * n_b)
    int32_t fa, fb;         // first spherical function of shell a and b
    int32_t same;           // 1 if sh_a == sh_b
    int32_t cls;            // pair class index
};

// Per-pair geometry, 64 bytes: centre A, A - B, Schwarz factor Q.
struct PairGeo {
    double ax, ay, az;
    double abx, aby, abz;
    double q;
    double pad;
};

// Per primitive pair, 64 bytes (one half cache line):
// zeta = a + b, 1/(2 zeta), P = (a A + b B)/zeta and
// K = c_a c_b exp(-a b |AB|^2 / zeta) * sqrt(2) pi^(5/4) / zeta, so that the
// base integral of a primitive quartet is K_ab K_cd / sqrt(zeta + eta) * F_m(T);
// the exponents a and b themselves (the weights of derivative integrals).
struct PrimPair {
    double zeta, o2z;
    double px, py, pz;
    double k;
    double ea, eb;
};

// Integrals-out work item: canonical (bra, ket) pair indices and where each
// canonical element (m, n, l, s) lands: out[off + m*s0 + n*s1 + l*s2 + s*s3].
struct EriTask {
    int32_t bra, ket;
    int64_t off;
    int32_t s0, s1, s2, s3;
};

struct JKArgs {
    const int2 *quartets;   // (bra pair, ket pair) per unique quartet of the class
    int64_t nq;
    const PairInfo *pairs;
    const PairGeo *geo;
    const PrimPair *prims;
    const double *boys;     // Boys table
    const double *D;        // N x N, symmetric
    double *J;              // unsymmetrised accumulators, N x N
    double *K;
    int32_t nbf;
    int32_t want_j, want_k;
    double *scratch;        // staged classes: slot k of batch quartet i at scratch[k * stride + i]
    int64_t stride;         // slot stride of the staged buffer (>= quartets in the batch)
};

struct EriArgs {
    const EriTask *tasks;
    int64_t ntask;
    const PairInfo *pairs;
    const PairGeo *geo;
    const PrimPair *prims;
    const double *boys;
    double *out;
    int32_t mode;           // 0: write blocks, 1: Schwarz factor of a diagonal quartet into out[task]
    double *scratch;
    int64_t stride;
};

// Phase-1 kernel of a staged class: items i < n, pair indices at idx[i*istride]
// (bra) and idx[i*istride + 1] (ket); accumulators to scratch[slot*stride + i]
// (slot-major), or, with qmajor set (row-form classes in integrals-out mode),
// to scratch[i*slots + slot] (the quartet's values contiguous).
struct P1Args {
    const int32_t *idx;
    int64_t istride;
    int64_t n;
    const PairInfo *pairs;
    const PairGeo *geo;
    const PrimPair *prims;
    const double *boys;
    double *scratch;
    int64_t stride;
    int32_t qmajor;
};

// Boys table: F_m(T_k) for T_k = k * BOYS_STEP, k = 0 .. BOYS_NPTS-1, m = 0 .. BOYS_NORD-1,
// stored [k][m] (row stride BOYS_STRIDE) so that the orders one evaluation reads
// are contiguous; column BOYS_NORD of row k holds exp(-T_k).
constexpr double BOYS_STEP = 0.05;
constexpr double BOYS_INV_STEP = 20.0;
constexpr double BOYS_TMAX = 36.0;
constexpr int BOYS_NPTS = 722;
constexpr int BOYS_NORD = 24;      // orders needed: L + 7 <= 23 for L <= 16
constexpr int BOYS_STRIDE = 25;    // per point: F_0 .. F_23, then exp(-T_k)

// Largest staged-tier buffer a plan allocates (doubles): 4 GiB.  Classes whose
// quartets do not fit in one batch are processed in several.
constexpr int64_t SCRATCH_MAX_DOUBLES = (int64_t)1 << 29;
// The HBM-scratch tier keeps every value of a quartet in the buffer (23 k
// doubles per (gg|gg) quartet), so it may take up to 16 GiB to keep enough
// quartets in flight; slot offsets stay below 2^32.
constexpr int64_t T3_SCRATCH_MAX_DOUBLES = (int64_t)1 << 31;
// HBM-scratch classes with both a wave-cooperative (slots in the buffer, at
// most max_batch quartets per launch) and a lane-per-quartet form: batches of
// at least this many quartets take the lane form, smaller ones the wave form.
// The lane form runs in rounds of one wave per SIMD (65 536 quartets on 256
// CUs); from half a round on it beats the wave form.
constexpr int64_t T3G_LANE_MIN = 32768;

// Launchers run one lane per work item (nq or ntask): the register tier's
// whole evaluation, or a staged class's Phase 2 + digestion; p1 launchers run
// a staged class's Phase 1 over (item, chunk).
typedef void (*launch_jk_fn)(const JKArgs &, hipStream_t);
typedef void (*launch_eri_fn)(const EriArgs &, hipStream_t);
typedef void (*launch_p1_fn)(const P1Args &, hipStream_t);

typedef int (*prepare_fn)();

struct ClassKernels {
    int la, lb, lc, ld;
    int tier;               // 0 register, 1 staged (chunked Phase 1 + Phase 2), 2 HBM scratch (op tables),
                            // 3 wave-cooperative LDS (op tables)
    launch_jk_fn jk;
    launch_eri_fn eri;
    launch_p1_fn p1;        // staged tier only (nullptr otherwise)
    prepare_fn prepare;     // HBM-scratch tier: uploads the class tables to the current device (0 on success)
    launch_jk_fn jk32;      // register tier: VRR and contraction in FP32, HRR and digestion in FP64 (mixed plans), or nullptr
    int block;              // threads per block
    double vrr_flops;       // per primitive quartet (generator count)
    double p2_flops;        // per contracted quartet: HRR + transform
    int n_hrr;
    int peak_live;
    int scratch_slots;      // doubles of buffer per quartet (0 for the register tier)
    int chunks;             // Phase-1 target chunks
    int max_batch;          // > 0: wave-cooperative launches of at most this many quartets (see T3G_LANE_MIN)
    int eri_wave;           // 1: row-form class whose integrals-out kernel runs one wave per quartet over a
                            // quartet-major buffer (Phase 1 with qmajor set)
    launch_eri_fn eri_tiles;  // row form, integrals out: ket stage of the tiled rows, before eri (or nullptr)
    launch_p1_fn p1_32;     // row form: Phase 1 with the VRR and contraction in FP32 (mixed precision), or nullptr
    launch_eri_fn eri32;    // register tier: integrals out with the VRR and contraction in FP32, or nullptr
};

}  // namespace hgp
