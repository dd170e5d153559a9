/*
 * hgp.h -- C ABI of the MI355X (gfx950) Head-Gordon-Pople ERI / J-K library.
 *
 * What it computes (the paper's statement of the problem, Sec. II-A and
 * Alg. 2's input/output): contracted two-electron repulsion integrals
 *     (mn|ls) = int int phi_m(r1) phi_n(r1) phi_l(r2) phi_s(r2) / |r1 - r2|
 * (Eq. eri-def) over shells of contracted Cartesian Gaussians, transformed to
 * pure spherical functions (Sec. III-B, Eq. cart2sph), and their digestion
 * into the Coulomb and exchange matrices
 *     J_mn = sum_ls (mn|ls) D_ls,     K_mn = sum_ls (ml|ns) D_ls
 * for a symmetric density D.  Evaluation follows the HGP scheme: Boys
 * function, vertical recurrence (Eq. vrr) per primitive quartet with the
 * contraction accumulated before the horizontal recurrence (Eq. hrr), which
 * is fused with the spherical transform index by index (Eq. stepwise-sph).
 *
 * Conventions
 *   - Units: bohr for coordinates, bohr^-2 for exponents, hartree for integrals.
 *   - Shells: l = 0..4.  Contraction coefficients are raw: the library scales
 *     them so that x^l exp(-a r^2) components are normalised (each primitive
 *     carries N(a,l) = (2a/pi)^(3/4) (4a)^(l/2) / sqrt((2l-1)!!)) and the
 *     contracted x^l component has unit norm.
 *   - Spherical functions per shell: s: 1; p: x, y, z (untransformed);
 *     l >= 2: 2l+1 real solid harmonics, m = -l .. l, unit norm, leading
 *     monomial coefficient positive (no Condon-Shortley phase).
 *   - Basis function order: shell by shell, in the order given.
 *   - Matrices: N x N, row-major, FP64, N = number of spherical functions.
 *
 * Memory and streams
 *   - Host pointers are read during the call and copied; device pointers
 *     (marked "device") are borrowed for the call and must stay valid until
 *     the work enqueued on the stream has completed.
 *   - hip_stream is a hipStream_t passed as void* (0: the null stream).
 *     Calls that enqueue work return after enqueueing; the caller
 *     synchronises the stream before reading results.
 *   - Handles own their device allocations; *_destroy frees them.  A handle
 *     must not be used from two host threads at once; distinct plans may run
 *     on distinct streams concurrently.
 *
 * Errors
 *   - Every call returns an hgp_status.  Argument errors are detected before
 *     any work is enqueued.  hgp_last_error() returns a thread-local message
 *     describing the last non-OK status.
 *   - A device or launch failure returns HGP_E_DEVICE and marks the plan
 *     unusable (later calls on it return HGP_E_STATE).
 */
#ifndef HGP_H
#define HGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HGP_OK = 0,
    HGP_E_INVALID = -1,        /* bad argument (null pointer, bad size, non-finite or non-positive exponent) */
    HGP_E_UNSUPPORTED_L = -2,  /* a shell with l > 4, or a class not built into this library */
    HGP_E_OOM = -3,            /* device allocation failed or the plan exceeds hbm_budget_bytes */
    HGP_E_DEVICE = -4,         /* HIP runtime or launch failure */
    HGP_E_STATE = -5           /* handle unusable after an earlier device failure */
} hgp_status;

typedef struct hgp_basis hgp_basis;  /* validated shells, normalised coefficients, device copies */
typedef struct hgp_plan hgp_plan;    /* pair data, Schwarz factors and screened class quartet lists */

#define HGP_NORMALIZE 1           /* hgp_basis_create: normalise the raw contraction coefficients */
#define HGP_FP64 0
#define HGP_MIXED 1               /* FP32 VRR and primitive contraction where a class has that form; Boys, HRR, J/K in FP64 */
#define HGP_MIXED_THETA_DEFAULT 1e-10

/* Library version and the highest l built into this library's class kernels (the per-class
 * kernel library of Sec. IV: one generated kernel set per canonical (la lb|lc ld), 120 for l <= 4). */
int32_t hgp_version(void);
int32_t hgp_max_l(void);

/*
 * hgp_basis_create -- ingest nshell shells (Alg. 2's input: shells with
 * primitives {(alpha_i, c_i)}, Sec. II-A) onto the current HIP device.
 *   l[nshell]         angular momentum per shell, 0..4              (host)
 *   nprim[nshell]     primitives per shell, 1..64                   (host)
 *   centers[3*nshell] x, y, z per shell, bohr                       (host)
 *   exps[sum nprim]   exponents, shell by shell, > 0                (host)
 *   coefs[sum nprim]  contraction coefficients                      (host)
 *   flags             HGP_NORMALIZE: coefs are raw; a device kernel scales
 *                     them by N(alpha, l) and the contraction norm (see
 *                     Conventions).  0: coefs are used as given, i.e. they are
 *                     already those scaled coefficients (what HGP_NORMALIZE
 *                     would compute); the functions are then whatever they
 *                     define.  Anything else: HGP_E_INVALID.
 * nshell = 0 is allowed (N = 0).  The host arrays are copied.
 */
hgp_status hgp_basis_create(int32_t nshell, const int32_t *l, const int32_t *nprim, const double *centers,
                            const double *exps, const double *coefs, int32_t flags, hgp_basis **out);
/* Number of spherical functions (2l+1 per shell, Sec. III-B, Eq. cart2sph); shell_offsets[nshell+1]
 * (host, may be NULL) gets each shell's first function. */
hgp_status hgp_basis_nbf(const hgp_basis *b, int32_t *nbf, int32_t *shell_offsets);
/* Frees the basis's device copies (handle plumbing: no passage of the paper). NULL is accepted. */
hgp_status hgp_basis_destroy(hgp_basis *b);

/*
 * hgp_plan_create -- everything a J/K build reuses across density updates:
 * shell-pair and primitive-pair data (the Gaussian-product quantities of
 * Alg. 2's GaussianPairs), Schwarz factors Q_ab = sqrt(max |(mn|mn)|), and per
 * canonical class (la lb|lc ld) (the l-configurations of Sec. IV) the list of
 * unique quartets with Q_ab Q_cd >= schwarz_tau (0: keep all).  The screen
 * is not part of the paper's text: it is the Cauchy-Schwarz bound
 * |(ab|cd)| <= Q_ab Q_cd applied to the unique quartets of Eq. eri-def.  All of it is computed by device
 * kernels on hip_stream; the call waits for the stream before returning.
 * With schwarz_tau > 0 the plan also drops primitive pairs: with q_r the
 * Schwarz factor of primitive pair r (contraction coefficients included),
 * Qmax the largest q over the basis and P the largest primitive-pair count of
 * a shell pair, pair r is left out when q_r Qmax < 0.1 schwarz_tau / P^2, so
 * the part dropped from any one integral is below 0.1 schwarz_tau.  With
 * schwarz_tau = 0 nothing is dropped and every integral is the exact sum.
 *   precision         HGP_FP64, or HGP_MIXED (= hgp_plan_create_mixed with
 *                     theta = HGP_MIXED_THETA_DEFAULT)
 *   hbm_budget_bytes  device bytes the plan may hold; 0 = half the device
 *                     memory free at creation for the quartet lists.  The
 *                     kept (bra pair, ket pair) lists of the classes (8 B a
 *                     quartet) are stored while they fit; past that the
 *                     largest lists are streamed: the plan keeps per bra row
 *                     the offset of its first kept quartet and every build
 *                     re-screens those rows, chunk by chunk, into one buffer
 *                     (same quartets, same order, an extra screening pass per
 *                     build; the streamed lists then run on hip_stream only).
 *                     HGP_E_OOM if the pair data, accumulators, staged-tier
 *                     buffer and one chunk holding the longest row exceed it.
 */
hgp_status hgp_plan_create(const hgp_basis *b, double schwarz_tau, int32_t precision, size_t hbm_budget_bytes,
                           void *hip_stream, hgp_plan **out);
/*
 * hgp_plan_create_mixed -- a plan whose register-tier classes evaluate the
 * quartets with schwarz_tau <= Q_ab Q_cd < theta with the VRR and the
 * contraction over primitives in FP32 (an extension: the paper's method is
 * FP64 throughout; here Eq. vrr and the accumulation of Alg. 2 run in FP32).  The pair quantities, the
 * Boys function, the horizontal recurrence and transforms (which cancel
 * between large intermediates) and the J/K digestion stay FP64.
 * Larger-bound quartets and the staged, wave-LDS and HBM-scratch classes run
 * wholly in FP64: for the staged row-form classes the HRR's cancellation
 * lifts the FP32 rounding of the VRR values beyond what the Schwarz bound
 * controls.  theta <= schwarz_tau gives an FP64 plan.  The deviation from the
 * FP64 result grows roughly in proportion to theta and depends on the basis
 * (tight, high-l primitives raise it): 1e-8 keeps it near 3e-10 on a
 * 3s2p1d molecule but gives ~3e-8 on small 5s4p3d2f1g molecules, so the
 * default is 1e-10.  Other arguments as hgp_plan_create.
 */
hgp_status hgp_plan_create_mixed(const hgp_basis *b, double schwarz_tau, double theta, size_t hbm_budget_bytes,
                                 void *hip_stream, hgp_plan **out);
/* Frees the plan's device data and streams after its pending work (handle plumbing). NULL is accepted. */
hgp_status hgp_plan_destroy(hgp_plan *p);
/* Plan statistics: unique quartets kept after screening, candidate quartets, device bytes held
 * (the quartet counts are those of Eq. eri-def's unique quartets before and after the screen). */
hgp_status hgp_plan_stats(const hgp_plan *p, int64_t *quartets_kept, int64_t *quartets_total, int64_t *device_bytes);
/* Primitive pairs (Alg. 2's GaussianPairs records) held by the plan's shell pairs after and before
 * primitive-pair screening. */
hgp_status hgp_plan_prim_stats(const hgp_plan *p, int64_t *prim_pairs_kept, int64_t *prim_pairs_total);
/* Streamed class lists (see hgp_plan_create): kept quartets in them, chunks per build over all of
 * them, and the chunk buffer's capacity in quartets (0 when nothing is streamed). */
hgp_status hgp_plan_stream_stats(const hgp_plan *p, int64_t *quartets_streamed, int64_t *chunks,
                                 int64_t *chunk_capacity);
/* Per class list c (0 .. n-1, n = hgp_plan_num_classes, in launch order; a mixed plan can hold two
 * lists of one class): angular momenta ls[4], quartets kept, primitive quartets they hold, the
 * generator's FLOP counts per primitive quartet (VRR + accumulate, unchunked) and per contracted
 * quartet (Phase 2), and the tier (0 register, 1 staged, 2 HBM scratch, 3 wave-cooperative LDS; the
 * register-only and buffered tiers of Sec. III-C, the last two this library's forms past them). */
int32_t hgp_plan_num_classes(const hgp_plan *p);
hgp_status hgp_plan_class_info(const hgp_plan *p, int32_t c, int32_t *ls, int64_t *nquartets, int64_t *nprim_quartets,
                               double *vrr_flops, double *phase2_flops, int32_t *tier);
/* Arithmetic width of class list c's VRR and primitive contraction: 64, or 32 for the FP32 part of a
 * mixed plan (HRR, transforms, Boys and digestion are FP64 in both). */
hgp_status hgp_plan_class_precision(const hgp_plan *p, int32_t c, int32_t *bits);

/* The plan's Schwarz factors by shell (the Cauchy-Schwarz screen above): Q[i*nshell + j] = Q[j*nshell + i] =
 * sqrt(max |(mn|mn)|) over m in shell i, n in shell j (host array, nshell^2),
 * from the primitive pairs the plan kept; 0 for a shell pair with none kept
 * (and for shells of different systems of a multi-system plan, whose shells
 * are numbered over the bases in the order given). */
hgp_status hgp_plan_schwarz(const hgp_plan *p, double *Q);

/*
 * Kernel timing for profiling (the per-kernel times of Sec. V's measurements): with timing enabled,
 * hgp_jk records a pair of
 * HIP events on its stream around each class kernel (the work enqueued is
 * unchanged).  hgp_plan_set_timing(p, 1) also resets the counters.
 * hgp_plan_class_timing waits for the recorded events and returns, for class
 * c and kernel k, the number of timed launches and their summed duration in
 * milliseconds.  k = 0: the one kernel of a register, wave-LDS or HBM-scratch
 * class, or a staged class's Phase-1 kernel; k = 1: a staged class's Phase-2 +
 * digestion kernel.  hgp_jk_multi records the same events.
 */
hgp_status hgp_plan_set_timing(hgp_plan *p, int32_t enable);
hgp_status hgp_plan_class_timing(hgp_plan *p, int32_t c, int32_t kernel, int64_t *launches, double *total_ms);

/*
 * hgp_jk -- J and K for density D (Alg. 2's Scatter step, 8-fold symmetry;
 * for buffered classes the separate contraction kernel of Sec. III-C.2).
 *   D   N x N symmetric density (device; symmetry is assumed, not checked)
 *   J   N x N output (device, overwritten) or NULL to skip J
 *   K   N x N output (device, overwritten) or NULL to skip K
 * Enqueues: zeroing of the plan's accumulators, one kernel per class, and
 * the symmetrisation J = J' + J'^T, K = K' + K'^T into the outputs.
 */
hgp_status hgp_jk(hgp_plan *p, const double *D, double *J, double *K, void *hip_stream);

/*
 * Several systems in one plan (the batched-systems growth of the method, not
 * in the paper, which evaluates one molecule at a time; the integrals and J/K
 * of each system are those of Eq. eri-def and Alg. 2):
 * the n bases are independent systems; the plan keeps only shell pairs
 * within a system and quartets whose two pairs are in the same system, so
 * each class is one launch over the quartets of every system at once
 * instead of n small launches.  Every screening decision (primitive pairs
 * included) is taken per system exactly as the system's own plan would, so
 * each system's J and K equal its own plan's up to the order of the FP64
 * additions.  Arguments as hgp_plan_create_mixed
 * (theta = 0: FP64).  The plan holds a copy of the bases (they may be
 * destroyed afterwards) and, besides the usual plan data, three buffers of
 * N_tot * (N_max + 1) doubles (N_tot = sum of the systems' N, N_max the
 * largest): system s's block of D, J' and K' sits at row offset R_s and
 * column offset R_s with row stride N_max, so blocks never overlap.
 * HGP_E_INVALID if N_tot * (N_max + 1) reaches 2^31.
 */
hgp_status hgp_plan_create_multi(const hgp_basis *const *bases, int32_t n, double schwarz_tau, double theta,
                                 size_t hbm_budget_bytes, void *hip_stream, hgp_plan **out);
/*
 * hgp_jk_multi -- J and K of every system of a multi-system plan.
 *   D[n], J[n], K[n]  device pointers, N_s x N_s row-major per system (J or K
 *                     may be NULL as a whole to skip it)
 * Stream-ordered like hgp_jk.  hgp_jk on a multi-system plan returns
 * HGP_E_INVALID; hgp_jk_multi on a one-system plan is hgp_jk.
 */
hgp_status hgp_jk_multi(hgp_plan *p, const double *const *D, double *const *J, double *const *K, void *hip_stream);

/*
 * Batched J/K over many systems (the batched-systems growth of the method, not
 * in the paper; each system's J/K as hgp_jk computes it, Alg. 2):
 * the J/K builds of n plans, each with its own D, J and K, captured once as
 * one HIP graph in which every system is an independent branch, so the
 * device overlaps the classes of small and large systems instead of running
 * them one launch at a time.
 *   plans[n]          built plans (same device), distinct from one another
 *   D[n], J[n], K[n]  device pointers per system, N_i x N_i; J[i] or K[i] may
 *                     be NULL to skip; captured by address, so later runs read
 *                     the current contents of D[i] and overwrite J[i], K[i]
 * hgp_batch_create checks the arguments, captures the builds on streams of
 * its own (so the caller's stream is neither needed nor touched) and
 * instantiates the graph; nothing runs yet.  Systems are spread over up to 8
 * branches, largest first, each to the branch with the least estimated work.
 * Plans with kernel timing on are rejected (events cannot be captured), and
 * so is a plan given twice (its accumulators would be shared).
 * hgp_batch_run enqueues one replay on hip_stream (any stream, the null
 * stream included); J and K are complete when that stream reaches the end of
 * the replay.  A plan in a batch must not be used concurrently with the
 * batch's runs.  hgp_batch_destroy frees the graph and the batch's streams,
 * not the plans or buffers.  Errors: HGP_E_INVALID for bad arguments,
 * HGP_E_STATE for a broken plan, HGP_E_DEVICE if capture or instantiation
 * fails (nothing is left allocated).
 */
typedef struct hgp_batch hgp_batch;
hgp_status hgp_batch_create(hgp_plan *const *plans, int32_t n, const double *const *D, double *const *J,
                            double *const *K, hgp_batch **out);
hgp_status hgp_batch_run(hgp_batch *b, void *hip_stream);
hgp_status hgp_batch_destroy(hgp_batch *b);

/*
 * hgp_eri_shell_quartets -- integrals out, any shell order: the contracted
 * spherical integrals (ij|kl) of the basis's shells (Sec. II-A, the
 * definition of the ERI and of contracted shells).
 *   quartets[4*nq]  shell indices (i, j, k, l) per quartet          (device)
 *   offsets[nq]     element offset of each block in out             (device)
 *   out             blocks [n_i][n_j][n_k][n_l] row-major at out + offsets[q] (device)
 * The quartets are classified on the device (class and canonical order per
 * quartet); the call then waits once for hip_stream, to read the per-class
 * counts that size the class launches, enqueues the pair precompute and the
 * class kernels, and returns.  Part of the class kernels runs on side streams
 * the library keeps per device, forked from and joined back into hip_stream,
 * so out is complete when hip_stream reaches the end of that work; quartets
 * and offsets must stay valid until then.  Calls on one device from several
 * host threads enqueue one at a time.
 * Temporary buffers are taken from and returned to the device's default
 * memory pool on hip_stream.  Blocks must not overlap (each is written, not
 * accumulated).  Errors: HGP_E_INVALID for NULL pointers, nq < 0 or beyond
 * 2^28, a shell index out of range or a negative offset (nothing written);
 * HGP_E_OOM if the pool cannot supply the buffers.
 */
hgp_status hgp_eri_shell_quartets(const hgp_basis *b, int64_t nq, const int32_t *quartets, const int64_t *offsets,
                                  double *out, void *hip_stream);

/*
 * hgp_eri_deriv_shell_quartets -- first derivatives of the contracted
 * spherical integrals with respect to the shell centres, the adjacent step
 * for nuclear gradients (the paper counts first-derivative kernel variants
 * in Sec. IV and names derivative integrals as the next step in Sec. VII):
 * d(ij|kl)/dR_p,x for each position p = 0..3 (the centre of the shell at that
 * position) and axis x.  Per primitive, the derivative of a Gaussian in its
 * centre is 2 alpha times the function with that Cartesian index raised
 * minus the index times the function with it lowered; the contraction,
 * Eq. hrr and Eq. cart2sph then apply as for the integrals, and the fourth
 * position follows from translational invariance.
 *   quartets[4*nq], offsets[nq]  as hgp_eri_shell_quartets       (device)
 *   out   per quartet 12 blocks [position 0..3][axis x, y, z][n_i][n_j][n_k][n_l],
 *         row-major, 12 n_i n_j n_k n_l doubles at out + offsets[q] (device)
 * A shell given at two positions gets a block per position (their sum is
 * the derivative in its centre).  Shells up to l = hgp_deriv_max_l();
 * HGP_E_UNSUPPORTED_L beyond.  Stream behaviour and other errors as
 * hgp_eri_shell_quartets; the call also holds, stream-ordered, a buffer of
 * at most 1 GiB for the partial accumulators of its larger classes.
 */
hgp_status hgp_eri_deriv_shell_quartets(const hgp_basis *b, int64_t nq, const int32_t *quartets,
                                        const int64_t *offsets, double *out, void *hip_stream);
/* Highest shell l for which hgp_eri_deriv_shell_quartets is built (-1: none). */
int32_t hgp_deriv_max_l(void);

/*
 * hgp_eri_prim_quartets -- n independent primitive quartets of class
 * (la lb|lc ld), each primitive normalised (coefficient N(a,l)): Eq. eri-def
 * for one-primitive shells, evaluated as Alg. 2 does (Boys, Eq. vrr, Eq. hrr
 * with the stepwise spherical transform, Eq. stepwise-sph).
 *   centers[12*n]  A, B, C, D per quartet, bohr                      (device)
 *   exps[4*n]      a, b, c, d per quartet                            (device)
 *   out[n * nsph(la) nsph(lb) nsph(lc) nsph(ld)]  spherical blocks   (device)
 *   precision      HGP_FP64, or HGP_MIXED: the VRR and the contraction in
 *                  FP32 for the classes that have that form (hgp_class_form;
 *                  register tier and the staged row form), with the pair
 *                  quantities, Boys function, HRR and transforms in FP64;
 *                  other classes wholly FP64.  The FP32 error is the FP64
 *                  path's own rounding error scaled by about 2^29 (the ratio
 *                  of the unit roundoffs): about 1e-6 of the largest integral
 *                  for low-l register classes, 1e-4 for (dd|dd), and for
 *                  high-l classes with distant centres (HRR cancellation)
 *                  more than the integrals; see hgp_plan_create_mixed for the
 *                  screened form used in J/K builds.
 * Stream-ordered; returns after enqueueing.  Its temporary buffers come from
 * the device's default memory pool, whose release threshold the library
 * raises on the first call (freed blocks stay in the pool for the next call).
 */
hgp_status hgp_eri_prim_quartets(int32_t la, int32_t lb, int32_t lc, int32_t ld, int64_t n, const double *centers,
                                 const double *exps, double *out, int32_t precision, void *hip_stream);

/*
 * hgp_class_form -- how this library evaluates class (la lb|lc ld) (any
 * order of the four; the tier routing of Sec. III-C, decided per class at
 * build time): *tier 0 register, 1 staged, 2 HBM-scratch op tables,
 * 3 wave-LDS op tables; *has_fp32 1 if the class has the FP32
 * VRR-and-contraction form that HGP_MIXED uses.  Either pointer may be NULL.
 * Errors: HGP_E_INVALID for negative l, HGP_E_UNSUPPORTED_L beyond l = 4.
 */
hgp_status hgp_class_form(int32_t la, int32_t lb, int32_t lc, int32_t ld, int32_t *tier, int32_t *has_fp32);

/*
 * hgp_eri_prim_quartets_noalloc -- hgp_eri_prim_quartets for callers that
 * cannot allocate device memory during the call (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, layout and results.  The pair and task records and the staged
 * tier's batch buffer come from one fixed 64 MiB device buffer that the
 * library holds per device until the process ends (set up on the first call
 * on a device, together with the Boys table; no call allocates).
 * Limits: register- and staged-tier classes only (HGP_E_UNSUPPORTED_L for a
 * class on an op-table tier); n at most hgp_eri_prim_quartets_noalloc_max for
 * the class (about 190 000 for register-tier classes), HGP_E_INVALID beyond.
 * Every call on a device shares that device's buffer: calls that overlap on
 * one device (two streams, two host threads) race and must be serialised by
 * the caller; the buffer keeps the last call's contents.
 */
hgp_status hgp_eri_prim_quartets_noalloc(int32_t la, int32_t lb, int32_t lc, int32_t ld, int64_t n,
                                         const double *centers, const double *exps, double *out, int32_t precision,
                                         void *hip_stream);
/* Largest n hgp_eri_prim_quartets_noalloc accepts for class (la lb|lc ld); -1 if it cannot run the class. */
int64_t hgp_eri_prim_quartets_noalloc_max(int32_t la, int32_t lb, int32_t lc, int32_t ld);

/* Thread-local description of the last non-OK status (never NULL; error plumbing, no passage). */
const char *hgp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HGP_H */
