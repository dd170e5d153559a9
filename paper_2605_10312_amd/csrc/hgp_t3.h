// HBM-scratch tier: one generic kernel per mode runs a class's op table (the
// generator's VRR and Phase-2 programs with slot-packed operands) over a
// lane-interleaved buffer; the wave-cooperative variant runs the same kind
// of table with the slots of one quartet in LDS.  A generated class file holds only the tables
// (host data) and two launchers.
#pragma once
#include "hgp_types.h"

namespace hgp {

// Op codes of the tables (eight uint16 words per op; see gen/emit_t3.py).
enum : int {
    T3_VRR_BRA = 1, T3_VRR_KET = 2, T3_ACC = 3, T3_HRR_BRA = 4, T3_HRR_KET = 5, T3_LIN = 6, T3_LIN_ACC = 7,
    T3_ACC_W = 8    // weighted accumulation (derivative tables, wave form only)
};
constexpr uint16_t T3_NONE = 0xFFFF;
// Ops come in groups of T3_GROUP (padded with op code 0): no op of a group
// reads a slot another op of the group writes, so a group issues all its
// operand loads before it computes (the generator's bundling, gen/emit_t3.py).
constexpr int T3_GROUP = 8;

struct T3Class {
    int la, lb, lc, ld, L;
    int na, nb, nc, nd;          // spherical functions per shell
    int nslots;                  // doubles of buffer per lane
    int n_hrr, acc0;             // accumulators [e0|f0] in slots acc0 .. acc0 + n_hrr - 1
    int n_vrr, n_p2;             // ops per primitive quartet, ops of Phase 2
    const uint16_t *ops;         // host: 8 words per op, VRR part first
    int ncoef;
    const double *coefs;         // host: transform coefficients
    const uint16_t *outslots;    // host: slot of integral (mu, nu, lam, sig), row-major
    int block;                   // threads per block
    // wave-cooperative LDS variant only (0 for the HBM-scratch variant):
    int maxblk;                  // largest of the six D/J/K blocks of a quartet
    int lds_bytes;               // LDS per workgroup (slots, zero and sink slots, coefficients, D blocks, outslots)
    int gslots;                  // 1: the slots (nslots + 2 per quartet) live in the scratch buffer, not in LDS
    const T3Class *lane;         // gslots: the lane-per-quartet tables, run for batches of T3G_LANE_MIN or more
    int out_blocks;              // output blocks per quartet: 0 or 1 for integrals, 12 for first derivatives
};

// Wave-cooperative variant (tier 3): the same tables regrouped T3W_OPS ops a
// group; one wavefront per quartet holds every slot in LDS and lane j runs
// ops j and j + 64 of each group.  Absent operands name the zero slot nslots; padding ops
// write the sink slot nslots + 1.  A class whose slots do not fit in LDS
// (gslots = 1, tier 2) keeps them in a per-quartet region of the scratch
// buffer instead, quartet i of a batch at scratch[i * (nslots + 2)].
constexpr int T3W_GROUP = 64;    // lanes of the wavefront that runs one quartet
constexpr int T3W_OPS = 128;     // ops per group: each lane runs ops lane and lane + 64 (four a lane measured slower: more padding)
constexpr int T3W_PREFETCH = 1;  // groups whose ops are in flight ahead of the running one
constexpr int T3G_CHUNK = 1024;  // quartets per launch of the wave form with its slots in the buffer

// 0 (hipSuccess) once the class's tables are on the current device (uploaded
// on first call), else the hipError_t of the step that failed.
int t3_prepare(const T3Class &c);
void t3_launch_jk(const T3Class &c, const JKArgs &a, hipStream_t s);
void t3_launch_eri(const T3Class &c, const EriArgs &a, hipStream_t s);
void t3w_launch_jk(const T3Class &c, const JKArgs &a, hipStream_t s);
void t3w_launch_eri(const T3Class &c, const EriArgs &a, hipStream_t s);

// First-derivative integrals (tables of gen/emit_deriv.py, wave form with the
// slots in LDS): per task the 12 blocks [centre][axis] of n_a n_b n_c n_d
// values at a.out + t.off + (3 * centre + axis) * n_a n_b n_c n_d, elements
// placed by the task's strides, where centre is the requested position of
// the canonical shell: bits 2r, 2r + 1 of code[t.bra / 2] for canonical shell r.
void t3w_launch_deriv(const T3Class &c, const EriArgs &a, const int32_t *code, hipStream_t s);

// The same from the weighted accumulators of Phase 1 (the staged form), Phase
// 2 only: accumulator k of task i is the sum over segments s < nseg, in that
// order, of a.scratch[(s * n_acc + k) * a.stride + i] (n_acc = c.n_hrr).
void t3w_launch_deriv_p2(const T3Class &c, const EriArgs &a, const int32_t *code, int nseg, hipStream_t s);

// The derivative classes built into the library: per canonical class its
// tables; for classes whose values fit in registers, the register form (one
// lane per quartet; same task layout and centre code; nseg unused), or
// nullptr; and the staged form's Phase 1 (partial accumulators of nseg
// segments of each quartet's primitive quartets into a.scratch as above,
// then t3w_launch_deriv_p2), or nullptr.
typedef void (*launch_deriv_fn)(const EriArgs &, const int32_t *code, int nseg, hipStream_t);
struct DerivClass {
    int la, lb, lc, ld;
    const T3Class *t;
    launch_deriv_fn reg;
    launch_deriv_fn p1;
    int p1_chunks;      // chunks per Phase-1 launch (the largest part)
};
// Staged derivative classes: doubles of accumulator buffer at most (1 GiB).
constexpr int64_t DERIV_STAGE_DOUBLES = (int64_t)1 << 27;
// A class with both forms takes the register form from this many quartets on
// (a wave a SIMD at one wave per SIMD), the staged form below.
constexpr int64_t DERIV_REG_MIN = 65536;
extern const DerivClass g_deriv_table[];
extern const int g_num_deriv;

}  // namespace hgp
