// Launchers of the hand-written auxiliary kernels (hgp_kernels_aux.hip).
#pragma once
#include "hgp_types.h"

namespace hgp {

void launch_boys_table(double *tab, hipStream_t s);
void launch_normalize(int nshell, const int *l, const int *nprim, const int *poff, const double *exps,
                      const double *coefs, double *out, hipStream_t s);
void launch_pairs(int npair, const PairInfo *pairs, const double *cen, const int *poff, const double *exps,
                  const double *ncoef, PairGeo *geo, PrimPair *prims, hipStream_t s);
void launch_prim_quartet_pairs(int64_t n, const double *centers, const double *exps, const int ls[4],
                               const int perm[4], const int strides[4], int64_t block, PairInfo *pairs,
                               PairGeo *geo, PrimPair *prims, EriTask *tasks, hipStream_t s);
void launch_screen_count(int b0, int nb, int sym, const double *Q, double tau, double hi, const int *psys,
                         const int *kbeg, const int *kcnt, const int *npr, int64_t *counts, int64_t *pcounts,
                         hipStream_t s);
void launch_screen_write(int b0, int nb, int sym, const double *Q, double tau, double hi, const int *psys,
                         const int *kbeg, const int *kcnt, const int64_t *offsets, int64_t shift, int2 *out,
                         hipStream_t s);
// Exclusive scan of v[0 .. n) in place, the sum into *total; tmp (at least
// (n + 1023) / 1024 values, or nullptr for one workgroup) holds block sums.
void launch_scan(int64_t *v, int n, int64_t *total, int64_t *tmp, hipStream_t s);
// class of each (la, lb, lc, ld) in canonical order, index ((la*5 + lb)*5 + lc)*5 + ld, -1 if not built;
// passed by value to the classify kernel
struct ClassOf {
    int16_t c[625];
};
// Shell quartets are keyed by class and, within a class, by primitive-quartet
// count: key = class * SQ_BUCKETS + (SQ_BUCKETS - 1 - min(floor(log2(n_bra n_ket)),
// SQ_BUCKETS - 1)), so a class's quartets are contiguous, the costliest first,
// and the lanes of a wave loop over similar counts.  code[q] = key << 8 | the
// four canonical positions (2 bits each); counts[key] per key.
constexpr int SQ_BUCKETS = 16;
void launch_sq_classify(int64_t nq, const int32_t *quartets, const int64_t *offsets, int nshell, const int *l,
                        const int *nprim, const ClassOf &class_of, int nkeys, int32_t *code, int64_t *primcnt,
                        unsigned long long *counts, unsigned long long *err, hipStream_t s);
// Pair records and tasks: quartet q's task at key_base[key] + its rank in the key.
void launch_sq_scatter(int64_t nq, const int32_t *quartets, const int64_t *offsets, const int *l, const int *nprim,
                       const int *foff, const int32_t *code, const int64_t *prim_off, const int64_t *key_base,
                       int nkeys, unsigned long long *cursor, PairInfo *pairs, EriTask *tasks, hipStream_t s);
void launch_store_q(int npair, const double *qv, PairGeo *geo, double *Q, hipStream_t s);
void launch_fill_zero(double *x, int64_t n, hipStream_t s);
void launch_symmetrize(const double *acc, int64_t astride, double *out, int n, hipStream_t s);
void launch_block_in(const double *src, int n, double *dst, int64_t dstride, hipStream_t s);
void launch_block_zero(double *dst, int n, int64_t dstride, hipStream_t s);

extern const ClassKernels g_class_table[];
extern const int g_num_classes;

}  // namespace hgp
