// Host runtime behind the C ABI in include/hgp.h: validation, basis ingest,
// plan construction (pairs, Schwarz factors, screened class lists) and the
// per-class dispatch of the generated kernels.  All arithmetic of the method
// runs in device kernels; the host only does index bookkeeping.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <limits>
#include <vector>

#include "hgp.h"
#include "hgp_aux.h"
#include "hgp_t3.h"

using namespace hgp;

namespace {

thread_local std::string g_err = "no error";

hgp_status fail(hgp_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

#define HGP_HIP(call)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess) return fail(HGP_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

int nsph(int l) { return 2 * l + 1; }
int pair_class_of(int la, int lb) { return la * (la + 1) / 2 + lb; }   // la >= lb

std::mutex g_mu;
double *g_boys[64] = {};

// The Boys table lives in a file-scope device array, one copy per device, so
// building it allocates nothing.  Host code uses the address returned by
// hipGetSymbolAddress on that device, never the array's name.
__device__ __align__(256) double boys_store[BOYS_NPTS * BOYS_STRIDE];

// Runs fn with device dev current, then restores the caller's device.
template <class F>
hipError_t on_device(int dev, F fn)
{
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    e = fn();
    if (cur != dev) {
        const hipError_t r = hipSetDevice(cur);
        if (e == hipSuccess) e = r;
    }
    return e;
}

hgp_status boys_table(int dev, const double **out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (dev < 0 || dev >= 64) return fail(HGP_E_DEVICE, "device index out of range");
    if (!g_boys[dev]) {
        double *t = nullptr;
        HGP_HIP(on_device(dev, [&]() {
            hipError_t e = hipGetSymbolAddress((void **)&t, HIP_SYMBOL(boys_store));
            if (e != hipSuccess) return e;
            launch_boys_table(t, 0);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            return hipStreamSynchronize(0);
        }));
        g_boys[dev] = t;
    }
    *out = g_boys[dev];
    return HGP_OK;
}

// The stream-ordered buffers of hgp_eri_prim_quartets (up to several GB for
// high-l classes) come from the device's default memory pool.  With the
// pool's default release threshold of zero every synchronisation hands that
// memory back to the driver and the next call maps it again, which cost more
// than the kernels themselves; the library raises the threshold once per
// device so freed blocks stay in the pool for reuse.
bool g_pool_kept[64] = {};

hgp_status keep_pool(int dev)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (dev < 0 || dev >= 64) return fail(HGP_E_DEVICE, "device index out of range");
    if (!g_pool_kept[dev]) {
        hipMemPool_t pool = nullptr;
        HGP_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
        uint64_t thr = UINT64_MAX;
        HGP_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr));
        g_pool_kept[dev] = true;
    }
    return HGP_OK;
}

// Staged derivative class of cnt quartets: segments of each quartet's
// primitive loop, enough for about 2^17 lanes per Phase-1 launch (two waves
// a SIMD), at most 16; then quartets per batch, whose partial accumulators
// (nseg n_hrr per quartet) stay within DERIV_STAGE_DOUBLES, at most 2^20.
int deriv_nseg(const DerivClass &dc, int64_t cnt)
{
    const int64_t lanes = (int64_t)std::max(1, dc.p1_chunks) * std::max<int64_t>(1, cnt);
    return (int)std::min<int64_t>(16, std::max<int64_t>(1, (((int64_t)1 << 17) + lanes - 1) / lanes));
}

// The register form (one lane per quartet, no Phase-1 buffer) where the class
// has one and its quartets alone fill the device; else the staged form, whose
// segments fill it.
bool deriv_use_reg(const DerivClass &dc, int64_t cnt)
{
    return dc.reg && (!dc.p1 || cnt >= DERIV_REG_MIN);
}

int64_t deriv_batch(const DerivClass &dc, int64_t cnt, int nseg)
{
    const int64_t per = std::max<int64_t>(1, DERIV_STAGE_DOUBLES / ((int64_t)nseg * std::max(1, dc.t->n_hrr)));
    return std::max<int64_t>(1, std::min({cnt, per, (int64_t)1 << 20}));
}

// Highest l of the derivative classes built into the library (-1: none).
int max_deriv_l()
{
    int m = -1;
    for (int c = 0; c < g_num_deriv; ++c)
        m = std::max({m, g_deriv_table[c].la, g_deriv_table[c].lb, g_deriv_table[c].lc, g_deriv_table[c].ld});
    return m;
}

int class_index(int la, int lb, int lc, int ld)
{
    for (int c = 0; c < g_num_classes; ++c) {
        const ClassKernels &k = g_class_table[c];
        if (k.la == la && k.lb == lb && k.lc == lc && k.ld == ld) return c;
    }
    return -1;
}

int built_max_l()
{
    int m = -1;
    for (int c = 0; c < g_num_classes; ++c) m = std::max(m, g_class_table[c].la);
    return m;
}

// Batch size of a staged class over a buffer of `doubles`: a multiple of 64.
// Quartets of one round of the lane-per-quartet op-table form on the current
// device: one wave of 64 lanes per SIMD (its kernel runs at one wave per SIMD).
int64_t lane_round()
{
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess || cu <= 0)
        return 0;
    return (int64_t)cu * 4 * 64;
}

// A class with both op-table forms (max_batch > 0): a batch holding more than
// one lane-form round is cut to whole rounds, so that no batch ends in a
// partly filled round (the remainder then runs as a batch of its own).
int64_t staged_batch(const ClassKernels &k, int64_t doubles)
{
    int64_t b = doubles / (k.scratch_slots > 0 ? k.scratch_slots : 1);
    b = (b / 64) * 64;
    if (k.max_batch > 0) {
        const int64_t r = lane_round();
        if (r > 0 && b > r) b = (b / r) * r;
    }
    return b < 64 ? 64 : b;
}

// Buffer a staged class needs to run all n items in one batch (capped).
int64_t staged_need(const ClassKernels &k, int64_t n)
{
    if (k.tier == 0 || k.tier == 3 || n <= 0) return 0;      // no HBM buffer
    if (k.max_batch > 0 && n < T3G_LANE_MIN) n = std::min(n, (int64_t)k.max_batch);   // wave form only
    const int64_t want = (int64_t)k.scratch_slots * (((n + 63) / 64) * 64);
    const int64_t floor64 = (int64_t)k.scratch_slots * 64;
    return std::max(floor64, std::min(want, k.tier == 2 ? T3_SCRATCH_MAX_DOUBLES : SCRATCH_MAX_DOUBLES));
}

// The HBM-scratch tier's tables must be on the device before its first launch.
hgp_status prepare_class(const ClassKernels &k)
{
    const int e = k.prepare ? k.prepare() : 0;
    if (e != 0)
        return fail(HGP_E_DEVICE, std::string("preparing the op tables of an HBM-scratch or wave-LDS class failed "
                                              "(upload, or LDS beyond the device's per-block limit): ") +
                                      hipGetErrorString((hipError_t)e));
    return HGP_OK;
}

// Integrals-out work of one class: register and wave-LDS tiers in launches of
// at most 2^20 blocks; staged tier in batches (Phase 1 then Phase 2);
// HBM-scratch tier in batches of one kernel each.  f32: the class's FP32
// VRR-and-contraction kernels where it has them (register tier, row form).
void run_eri_class(const ClassKernels &k, EriArgs a, int64_t scratch_doubles, hipStream_t s, bool f32 = false)
{
    const int64_t ntask = a.ntask;
    if (k.tier == 0 || k.tier == 3) {
        const launch_eri_fn run = f32 && k.eri32 ? k.eri32 : k.eri;
        const int64_t chunk = (int64_t)k.block << 20;
        for (int64_t q0 = 0; q0 < ntask; q0 += chunk) {
            EriArgs b = a;
            b.tasks = a.tasks + q0;
            b.ntask = std::min(chunk, ntask - q0);
            if (a.mode == 1) b.out = a.out + q0;
            run(b, s);
        }
        return;
    }
    const launch_p1_fn p1 = f32 && k.p1_32 ? k.p1_32 : k.p1;
    const int64_t B = staged_batch(k, scratch_doubles);
    for (int64_t q0 = 0; q0 < ntask; q0 += B) {
        const int64_t nb = std::min(B, ntask - q0);
        if (k.tier == 1) {
            // row-form classes run their integrals-out kernel one wave per
            // quartet over a quartet-major buffer
            P1Args pa{(const int32_t *)(a.tasks + q0), (int64_t)(sizeof(EriTask) / sizeof(int32_t)), nb, a.pairs,
                      a.geo, a.prims, a.boys, a.scratch, B, k.eri_wave};
            p1(pa, s);
        }
        EriArgs b = a;
        b.tasks = a.tasks + q0;
        b.ntask = nb;
        if (a.mode == 1) b.out = a.out + q0;
        b.stride = B;
        if (k.eri_tiles) k.eri_tiles(b, s);
        k.eri(b, s);
    }
}

template <class T>
hgp_status dalloc(T **p, size_t n, int64_t *bytes = nullptr)
{
    *p = nullptr;
    if (n == 0) return HGP_OK;
    hipError_t e = hipMalloc((void **)p, n * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(HGP_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    if (bytes) *bytes += (int64_t)(n * sizeof(T));
    return HGP_OK;
}

template <class T>
hgp_status upload(T **p, const std::vector<T> &v, int64_t *bytes = nullptr)
{
    hgp_status s = dalloc(p, v.size(), bytes);
    if (s != HGP_OK) return s;
    if (!v.empty()) HGP_HIP(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return HGP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
struct hgp_basis {
    int device = 0;
    int flags = HGP_NORMALIZE;  // coefficients normalised by the library (else used as given)
    int nshell = 0, nbf = 0, lmax = 0;
    std::vector<int32_t> l, nprim, poff, foff;
    std::vector<double> cen, exps, coefs;
    int *d_l = nullptr, *d_nprim = nullptr, *d_poff = nullptr, *d_foff = nullptr;
    double *d_cen = nullptr, *d_exps = nullptr, *d_coefs = nullptr, *d_ncoef = nullptr;
};

struct ClassList {
    int cls;          // index into g_class_table
    int bits = 64;    // 64: FP64 kernel; 32: VRR and contraction in FP32 (mixed plans, Q_ab Q_cd below theta)
    int64_t nq = 0;   // unique quartets kept
    int64_t nprimq = 0;
    int2 *d_q = nullptr;   // the kept (bra, ket) pairs, or nullptr for a streamed list
    // screening parameters: bra rows b0 .. b0 + nb - 1 of pair class bc against
    // the kets of pair class kc, Q_ab Q_cd in [lo, hi)
    int b0 = 0, nb = 0, sym = 0, kc = 0;
    double lo = 0.0, hi = 0.0;
    // streamed list (its pairs re-screened into the plan's chunk buffer on every
    // build): per-row first-quartet offsets (device, nb) and the row ranges of
    // the chunks with their first offsets
    int64_t *d_off = nullptr;
    std::vector<int> chunk_row;            // chunk k: rows chunk_row[k] .. chunk_row[k + 1] - 1
    std::vector<int64_t> chunk_off;        // chunk k: quartets chunk_off[k] .. chunk_off[k + 1] - 1
    int64_t launches[2] = {0, 0};   // timed launches: [0] whole / Phase-1 kernel, [1] Phase-2 kernel
    double ms[2] = {0.0, 0.0};      // their summed durations
};

struct PendingTiming {
    int list, kernel;
    hipEvent_t start, stop;
};

struct hgp_plan {
    const hgp_basis *b = nullptr;
    int device = 0;
    bool broken = false;
    int npair = 0;
    std::vector<int> pc_begin, pc_count;
    std::vector<PairInfo> pairs;           // host copy, same order as d_pairs
    PairInfo *d_pairs = nullptr;
    PairGeo *d_geo = nullptr;
    PrimPair *d_prims = nullptr;
    double *d_Q = nullptr;
    double *d_Jacc = nullptr, *d_Kacc = nullptr;
    double *d_scratch = nullptr;           // staged classes: slot-major batch buffer
    int64_t scratch_doubles = 0;
    int *d_npr = nullptr;                  // primitive pairs of each pair
    int2 *d_chunk = nullptr;               // streamed lists: one chunk of kept pairs at a time
    int64_t chunk_cap = 0;                 // its capacity in quartets
    std::vector<ClassList> lists;
    int64_t kept = 0, total = 0, bytes = 0;
    int64_t prim_total = 0, prim_kept = 0;   // primitive pairs before / after primitive screening
    double theta = 0.0;                      // mixed plans: quartets with Q_ab Q_cd < theta use FP32 VRR and contraction
    bool timing = false;
    std::vector<PendingTiming> pending;
    std::vector<hipEvent_t> event_pool;
    // several systems in one plan (hgp_plan_create_multi): pairs and quartets
    // stay within a system; system s's functions are R_s .. R_s + N_s - 1 of
    // the union basis, and D and the accumulators hold its block at
    // (R_s + i) * stride + R_s + j with stride = max N_s, so blocks of
    // different systems never overlap
    hgp_basis *owned = nullptr;              // the union basis
    std::vector<int> shell_sys;              // system of each shell (empty: one system)
    int nsys = 1;
    std::vector<int> sys_R, sys_N;
    int64_t stride = 0;                      // row stride of D and the accumulators
    int64_t acc_len = 0;                     // doubles per accumulator
    double *d_Dunion = nullptr;              // several systems: the densities in the accumulators' layout
    int *d_psys = nullptr;                   // system of each pair
    int *d_cbeg = nullptr, *d_ccnt = nullptr;   // [pair class][system]: first pair and count
    // register- and wave-tier class lists run concurrently on these side
    // streams (forked from and joined back into the caller's stream)
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> side_ev;         // [0] fork, [1 + k] join of side stream k
};

static hipEvent_t take_event(hgp_plan *p)
{
    if (!p->event_pool.empty()) {
        hipEvent_t e = p->event_pool.back();
        p->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

static hgp_status collect_timing(hgp_plan *p)
{
    for (const PendingTiming &t : p->pending) {
        float ms = 0.f;
        HGP_HIP(hipEventSynchronize(t.stop));
        HGP_HIP(hipEventElapsedTime(&ms, t.start, t.stop));
        p->lists[t.list].ms[t.kernel] += ms;
        p->lists[t.list].launches[t.kernel] += 1;
        p->event_pool.push_back(t.start);
        p->event_pool.push_back(t.stop);
    }
    p->pending.clear();
    return HGP_OK;
}

extern "C" {

int32_t hgp_version(void) { return 1; }
int32_t hgp_max_l(void) { return built_max_l(); }
const char *hgp_last_error(void) { return g_err.c_str(); }

hgp_status hgp_basis_destroy(hgp_basis *b)
{
    if (!b) return HGP_OK;
    hipFree(b->d_l); hipFree(b->d_nprim); hipFree(b->d_poff); hipFree(b->d_foff);
    hipFree(b->d_cen); hipFree(b->d_exps); hipFree(b->d_coefs); hipFree(b->d_ncoef);
    delete b;
    return HGP_OK;
}

hgp_status hgp_basis_create(int32_t nshell, const int32_t *l, const int32_t *nprim, const double *centers,
                            const double *exps, const double *coefs, int32_t flags, hgp_basis **out)
{
    if (!out) return fail(HGP_E_INVALID, "out is NULL");
    *out = nullptr;
    if (nshell < 0) return fail(HGP_E_INVALID, "nshell < 0");
    if (flags != 0 && flags != HGP_NORMALIZE) return fail(HGP_E_INVALID, "flags: HGP_NORMALIZE or 0");
    if (nshell > 0 && (!l || !nprim || !centers || !exps || !coefs)) return fail(HGP_E_INVALID, "NULL shell array");
    auto *b = new hgp_basis();
    b->nshell = nshell;
    b->flags = flags;
    b->poff.assign(1, 0);
    b->foff.assign(1, 0);
    for (int s = 0; s < nshell; ++s) {
        if (l[s] < 0) { hgp_basis_destroy(b); return fail(HGP_E_INVALID, "negative l"); }
        if (l[s] > 4) { hgp_basis_destroy(b); return fail(HGP_E_UNSUPPORTED_L, "shell with l > 4"); }
        if (nprim[s] < 1 || nprim[s] > 64) { hgp_basis_destroy(b); return fail(HGP_E_INVALID, "nprim outside 1..64"); }
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(centers[3 * s + k])) { hgp_basis_destroy(b); return fail(HGP_E_INVALID, "non-finite centre"); }
        b->l.push_back(l[s]);
        b->nprim.push_back(nprim[s]);
        b->poff.push_back(b->poff.back() + nprim[s]);
        b->foff.push_back(b->foff.back() + nsph(l[s]));
        b->lmax = std::max(b->lmax, (int)l[s]);
    }
    b->nbf = b->foff.back();
    const int np = b->poff.back();
    for (int k = 0; k < np; ++k) {
        if (!(exps[k] > 0.0) || !std::isfinite(exps[k]) || !std::isfinite(coefs[k])) {
            hgp_basis_destroy(b);
            return fail(HGP_E_INVALID, "exponents must be finite and > 0, coefficients finite");
        }
    }
    b->cen.assign(centers, centers + 3 * nshell);
    b->exps.assign(exps, exps + np);
    b->coefs.assign(coefs, coefs + np);
    const hipError_t de = hipGetDevice(&b->device);
    if (de != hipSuccess) {
        hgp_basis_destroy(b);
        return fail(HGP_E_DEVICE, std::string("hipGetDevice failed: ") + hipGetErrorString(de));
    }
    hgp_status st;
    if ((st = upload(&b->d_l, b->l)) || (st = upload(&b->d_nprim, b->nprim)) || (st = upload(&b->d_poff, b->poff)) ||
        (st = upload(&b->d_foff, b->foff)) ||
        (st = upload(&b->d_cen, b->cen)) || (st = upload(&b->d_exps, b->exps)) || (st = upload(&b->d_coefs, b->coefs)) ||
        (st = dalloc(&b->d_ncoef, (size_t)std::max(np, 1)))) {
        hgp_basis_destroy(b);
        return st;
    }
    if (flags & HGP_NORMALIZE)
        launch_normalize(nshell, b->d_l, b->d_nprim, b->d_poff, b->d_exps, b->d_coefs, b->d_ncoef, 0);
    else if (np > 0 && hipMemcpy(b->d_ncoef, b->d_coefs, sizeof(double) * np, hipMemcpyDeviceToDevice) != hipSuccess) {
        hgp_basis_destroy(b);
        return fail(HGP_E_DEVICE, "copying the coefficients failed");
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(0) != hipSuccess) {
        hgp_basis_destroy(b);
        return fail(HGP_E_DEVICE, "normalisation kernel failed");
    }
    *out = b;
    return HGP_OK;
}

hgp_status hgp_basis_nbf(const hgp_basis *b, int32_t *nbf, int32_t *shell_offsets)
{
    if (!b || !nbf) return fail(HGP_E_INVALID, "NULL argument");
    *nbf = b->nbf;
    if (shell_offsets) std::memcpy(shell_offsets, b->foff.data(), sizeof(int32_t) * b->foff.size());
    return HGP_OK;
}

hgp_status hgp_plan_destroy(hgp_plan *p)
{
    if (!p) return HGP_OK;
    for (const PendingTiming &t : p->pending) {
        hipEventSynchronize(t.stop);
        p->event_pool.push_back(t.start);
        p->event_pool.push_back(t.stop);
    }
    for (hipEvent_t e : p->event_pool) hipEventDestroy(e);
    for (hipEvent_t e : p->side_ev) hipEventDestroy(e);
    for (hipStream_t st : p->side) hipStreamDestroy(st);
    hipFree(p->d_pairs); hipFree(p->d_geo); hipFree(p->d_prims); hipFree(p->d_Q);
    hipFree(p->d_Jacc); hipFree(p->d_Kacc); hipFree(p->d_scratch);
    hipFree(p->d_Dunion); hipFree(p->d_psys); hipFree(p->d_cbeg); hipFree(p->d_ccnt);
    for (auto &c : p->lists) { hipFree(c.d_q); hipFree(c.d_off); }
    hipFree(p->d_npr); hipFree(p->d_chunk);
    if (p->owned) hgp_basis_destroy(p->owned);
    delete p;
    return HGP_OK;
}

// Schwarz factors sqrt(max |(mn|mn)|) of npair pairs grouped by pair class
// (class c occupies [begin[c], begin[c] + count[c])), from the diagonal quartets
// (p|p) run through the class kernels' integrals-out mode.  q: device, npair.
static hgp_status schwarz_factors(const PairInfo *d_pairs, const PairGeo *d_geo, const PrimPair *d_prims,
                                  const std::vector<int> &begin, const std::vector<int> &count, int npair,
                                  const double *boys, double *q, hipStream_t s)
{
    if (npair <= 0) return HGP_OK;
    const int npc = (int)begin.size();
    EriTask *tasks = nullptr;
    double *sscr = nullptr;
    int64_t sneed = 0;
    std::vector<int> cls(npc, -1);
    for (int c = 0; c < npc; ++c) {
        if (!count[c]) continue;
        int la = 0;
        while (pair_class_of(la + 1, 0) <= c) ++la;
        const int lb = c - pair_class_of(la, 0);
        cls[c] = class_index(la, lb, la, lb);
        if (cls[c] < 0) return fail(HGP_E_UNSUPPORTED_L, "class kernel not built");
        hgp_status ps = prepare_class(g_class_table[cls[c]]);
        if (ps) return ps;
        sneed = std::max(sneed, staged_need(g_class_table[cls[c]], count[c]));
    }
    hgp_status st;
    if ((st = dalloc(&tasks, (size_t)npair)) || (st = dalloc(&sscr, (size_t)sneed))) { hipFree(tasks); return st; }
    std::vector<EriTask> th((size_t)npair);
    for (int i = 0; i < npair; ++i) th[i] = EriTask{i, i, 0, 0, 0, 0, 0};
    hipError_t e = hipMemcpyAsync(tasks, th.data(), th.size() * sizeof(EriTask), hipMemcpyHostToDevice, s);
    for (int c = 0; c < npc && e == hipSuccess; ++c) {
        if (!count[c]) continue;
        EriArgs a{};
        a.tasks = tasks + begin[c];
        a.ntask = count[c];
        a.pairs = d_pairs; a.geo = d_geo; a.prims = d_prims; a.boys = boys;
        a.out = q + begin[c];
        a.mode = 1;
        a.scratch = sscr;
        run_eri_class(g_class_table[cls[c]], a, sneed, s);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(tasks);
    hipFree(sscr);
    if (e != hipSuccess) return fail(HGP_E_DEVICE, std::string("Schwarz kernels: ") + hipGetErrorString(e));
    return HGP_OK;
}

// Primitive-pair screening.  The contribution of one primitive quartet (r|s)
// to any integral of its contracted quartet is bounded by q_r q_s <= q_r Qmax,
// with q_r the Schwarz factor of primitive pair r (contraction coefficients
// included) and Qmax the largest over the basis.  A primitive pair is dropped
// when q_r Qmax < PRIM_SCREEN_FRACTION * tau / P^2, where P is the largest
// primitive-pair count of any shell pair, so P^2 bounds the primitive quartets
// of a contracted quartet: what is dropped from one integral stays below a
// tenth of the Schwarz threshold tau.
constexpr double PRIM_SCREEN_FRACTION = 0.1;
// Register- and wave-tier class lists of one J/K build run on the caller's
// stream and this many more (the device runs four hardware queues a process).
constexpr int HGP_SIDE_STREAMS = 3;

static hgp_status plan_build(hgp_plan *p, double tau, size_t budget, hipStream_t s)
{
    const hgp_basis *b = p->b;
    const int lmax = b->lmax;
    const int npc = pair_class_of(lmax, lmax) + 1;
    // ---- pair lists per pair class, sorted by primitive-pair count (descending)
    std::vector<std::vector<PairInfo>> per(npc);
    auto sysof = [&](int sh) { return p->shell_sys.empty() ? 0 : p->shell_sys[(size_t)sh]; };
    // within a pair class: by system, then by primitive-pair count (descending),
    // so the lanes of a wavefront run primitive loops of equal length (ordering
    // by first shell instead, for longer K'[ac] reduction runs, measured 1.8x
    // slower on the benchmark workload)
    auto pair_order = [&](const PairInfo &x, const PairInfo &y) {
        const int sx = sysof(x.sh_a), sy = sysof(y.sh_a);
        return sx != sy ? sx < sy : x.nprim > y.nprim;
    };
    for (int i = 0; i < b->nshell; ++i)
        for (int j = 0; j < b->nshell; ++j) {
            const int li = b->l[i], lj = b->l[j];
            if (li < lj || (li == lj && j > i)) continue;
            if (sysof(i) != sysof(j)) continue;       // no pair across systems
            PairInfo pi{};
            pi.sh_a = i; pi.sh_b = j;
            pi.nprim = b->nprim[i] * b->nprim[j];
            pi.fa = b->foff[i]; pi.fb = b->foff[j];
            pi.same = (i == j);
            pi.cls = pair_class_of(li, lj);
            per[pi.cls].push_back(pi);
        }
    auto layout = [&](std::vector<std::vector<PairInfo>> &groups, std::vector<PairInfo> &flat) {
        flat.clear();
        p->pc_begin.assign(npc, 0);
        p->pc_count.assign(npc, 0);
        int off = 0;
        for (int c = 0; c < npc; ++c) {
            std::stable_sort(groups[c].begin(), groups[c].end(), pair_order);
            p->pc_begin[c] = (int)flat.size();
            p->pc_count[c] = (int)groups[c].size();
            for (auto &pi : groups[c]) {
                pi.prim_off = off;
                off += pi.nprim;
                flat.push_back(pi);
            }
        }
        return off;
    };
    std::vector<PairInfo> pairs;
    int prim_off = layout(per, pairs);
    // candidate unique quartets over all shell pairs (within each system), before any screening
    const int nsys = p->nsys;
    {
        std::vector<int64_t> cnt((size_t)npc * nsys, 0);
        for (const PairInfo &x : pairs) ++cnt[(size_t)x.cls * nsys + sysof(x.sh_a)];
        p->total = 0;
        for (int bc = 0; bc < npc; ++bc)
            for (int kc = 0; kc <= bc; ++kc)
                for (int sy = 0; sy < nsys; ++sy) {
                    const int64_t nb = cnt[(size_t)bc * nsys + sy], nk = cnt[(size_t)kc * nsys + sy];
                    p->total += (bc == kc) ? nb * (nb + 1) / 2 : nb * nk;
                }
    }
    const int64_t nbf = b->nbf;
    if (nsys == 1) {
        p->stride = nbf;
        p->acc_len = nbf * nbf;
    } else {
        p->stride = std::max(1, *std::max_element(p->sys_N.begin(), p->sys_N.end()));
        p->acc_len = nbf * (p->stride + 1);
    }
    if (p->acc_len >= ((int64_t)1 << 31))   // the kernels index D, J and K with 32-bit offsets
        return fail(HGP_E_INVALID, "basis too large: D/J/K offsets exceed 32 bits");
    const int64_t need = (int64_t)pairs.size() * (sizeof(PairInfo) + sizeof(PairGeo) + 2 * sizeof(double)) +
                         (int64_t)prim_off * sizeof(PrimPair) +
                         (nsys == 1 ? 2 : 3) * p->acc_len * (int64_t)sizeof(double);
    if (budget && (size_t)need > budget) return fail(HGP_E_OOM, "plan exceeds the HBM budget (pair data and accumulators)");
    hgp_status st;
    PairInfo *d_pairs = nullptr;
    PairGeo *d_geo = nullptr;
    PrimPair *d_prims = nullptr;
    auto free_tmp = [&]() { hipFree(d_pairs); hipFree(d_geo); hipFree(d_prims); d_pairs = nullptr; d_geo = nullptr; d_prims = nullptr; };
    if ((st = upload(&d_pairs, pairs)) || (st = dalloc(&d_geo, pairs.size())) || (st = dalloc(&d_prims, (size_t)prim_off))) {
        free_tmp();
        return st;
    }
    launch_pairs((int)pairs.size(), d_pairs, b->d_cen, b->d_poff, b->d_exps, b->d_ncoef, d_geo, d_prims, s);
    HGP_HIP(hipGetLastError());
    const double *boys = nullptr;
    if ((st = boys_table(p->device, &boys))) { free_tmp(); return st; }

    // ---- primitive-pair screening (skipped when tau = 0: the path stays exact)
    if (tau > 0 && prim_off > 0) {
        std::vector<PairGeo> geo(pairs.size());
        std::vector<PrimPair> recs((size_t)prim_off);
        HGP_HIP(hipMemcpyAsync(geo.data(), d_geo, geo.size() * sizeof(PairGeo), hipMemcpyDeviceToHost, s));
        HGP_HIP(hipMemcpyAsync(recs.data(), d_prims, recs.size() * sizeof(PrimPair), hipMemcpyDeviceToHost, s));
        HGP_HIP(hipStreamSynchronize(s));
        // one single-primitive pair per record; records of a class are contiguous
        std::vector<PairInfo> pp((size_t)prim_off);
        std::vector<PairGeo> pg((size_t)prim_off);
        std::vector<int> pbeg(npc, 0), pcnt(npc, 0);
        for (int c = 0; c < npc; ++c) {
            for (int k = 0; k < p->pc_count[c]; ++k) {
                const int pi = p->pc_begin[c] + k;
                if (k == 0) pbeg[c] = pairs[pi].prim_off;
                pcnt[c] += pairs[pi].nprim;
                for (int r = 0; r < pairs[pi].nprim; ++r) {
                    PairInfo x = pairs[pi];
                    x.prim_off = pairs[pi].prim_off + r;
                    x.nprim = 1;
                    pp[(size_t)x.prim_off] = x;
                    pg[(size_t)x.prim_off] = geo[pi];
                }
            }
        }
        PairInfo *d_pp = nullptr;
        PairGeo *d_pg = nullptr;
        double *d_qp = nullptr;
        if ((st = upload(&d_pp, pp)) || (st = upload(&d_pg, pg)) || (st = dalloc(&d_qp, (size_t)prim_off)) ||
            (st = schwarz_factors(d_pp, d_pg, d_prims, pbeg, pcnt, prim_off, boys, d_qp, s))) {
            hipFree(d_pp); hipFree(d_pg); hipFree(d_qp); free_tmp();
            return st;
        }
        std::vector<double> qp((size_t)prim_off);
        hipError_t e = hipMemcpy(qp.data(), d_qp, qp.size() * sizeof(double), hipMemcpyDeviceToHost);
        hipFree(d_pp); hipFree(d_pg); hipFree(d_qp);
        if (e != hipSuccess) { free_tmp(); return fail(HGP_E_DEVICE, "copying primitive Schwarz factors"); }
        // largest primitive Schwarz factor and primitive-pair count per system (a
        // multi-system plan drops exactly what each system's own plan would)
        std::vector<double> qmax((size_t)nsys, 0.0);
        std::vector<int> pmax((size_t)nsys, 1);
        for (const PairInfo &x : pairs) {
            const int sy = sysof(x.sh_a);
            pmax[(size_t)sy] = std::max(pmax[(size_t)sy], x.nprim);
            for (int r = 0; r < x.nprim; ++r) qmax[(size_t)sy] = std::max(qmax[(size_t)sy], qp[(size_t)(x.prim_off + r)]);
        }
        // rebuild the pairs with only the primitive pairs that matter
        std::vector<std::vector<PairInfo>> kept(npc);
        std::vector<std::vector<int>> keep_recs(pairs.size());
        std::vector<PairGeo> kgeo_by_pair(pairs.size());
        for (size_t pi = 0; pi < pairs.size(); ++pi) {
            const int sy = sysof(pairs[pi].sh_a);
            const double cut = PRIM_SCREEN_FRACTION * tau / ((double)pmax[(size_t)sy] * (double)pmax[(size_t)sy]);
            for (int r = 0; r < pairs[pi].nprim; ++r) {
                const int rr = pairs[pi].prim_off + r;
                if (qp[(size_t)rr] * qmax[(size_t)sy] >= cut) keep_recs[pi].push_back(rr);
            }
            if (keep_recs[pi].empty()) continue;   // no primitive quartet of this pair matters
            PairInfo x = pairs[pi];
            x.nprim = (int)keep_recs[pi].size();
            x.prim_off = (int)pi;                   // temporarily: index of the original pair
            kept[x.cls].push_back(x);
        }
        std::vector<PairInfo> np;
        int noff = 0;
        {
            // keep the original pair index to gather records and geometry
            std::vector<std::vector<PairInfo>> groups = kept;
            std::vector<int> orig;
            p->pc_begin.assign(npc, 0);
            p->pc_count.assign(npc, 0);
            for (int c = 0; c < npc; ++c) {
                std::stable_sort(groups[c].begin(), groups[c].end(), pair_order);
                p->pc_begin[c] = (int)np.size();
                p->pc_count[c] = (int)groups[c].size();
                for (auto &x : groups[c]) {
                    orig.push_back(x.prim_off);
                    x.prim_off = noff;
                    noff += x.nprim;
                    np.push_back(x);
                }
            }
            std::vector<PrimPair> nrec((size_t)noff);
            std::vector<PairGeo> ngeo(np.size());
            for (size_t k = 0; k < np.size(); ++k) {
                ngeo[k] = geo[(size_t)orig[k]];
                const auto &rs = keep_recs[(size_t)orig[k]];
                for (size_t t = 0; t < rs.size(); ++t) nrec[(size_t)np[k].prim_off + t] = recs[(size_t)rs[t]];
            }
            free_tmp();
            if ((st = upload(&d_pairs, np)) || (st = upload(&d_geo, ngeo)) || (st = upload(&d_prims, nrec))) {
                free_tmp();
                return st;
            }
        }
        p->prim_total = prim_off;
        pairs = np;
        prim_off = noff;
    } else {
        p->prim_total = prim_off;
    }
    p->prim_kept = prim_off;
    p->npair = (int)pairs.size();
    p->pairs = pairs;
    p->d_pairs = d_pairs; p->d_geo = d_geo; p->d_prims = d_prims;
    p->bytes += (int64_t)pairs.size() * (sizeof(PairInfo) + sizeof(PairGeo)) + (int64_t)prim_off * sizeof(PrimPair);
    if ((st = dalloc(&p->d_Q, pairs.size(), &p->bytes)) || (st = dalloc(&p->d_Jacc, (size_t)p->acc_len, &p->bytes)) ||
        (st = dalloc(&p->d_Kacc, (size_t)p->acc_len, &p->bytes)))
        return st;
    if (nsys > 1 && (st = dalloc(&p->d_Dunion, (size_t)p->acc_len, &p->bytes))) return st;
    // the system of each pair, and per pair class and system the range of its pairs
    {
        std::vector<int> psys(std::max<size_t>(pairs.size(), 1), 0), cbeg((size_t)npc * nsys, 0),
            ccnt((size_t)npc * nsys, 0);
        for (int c = 0; c < npc; ++c)
            for (int k = p->pc_begin[c]; k < p->pc_begin[c] + p->pc_count[c]; ++k) {
                const int sy = sysof(pairs[(size_t)k].sh_a);
                psys[(size_t)k] = sy;
                if (ccnt[(size_t)c * nsys + sy]++ == 0) cbeg[(size_t)c * nsys + sy] = k;
            }
        if ((st = upload(&p->d_psys, psys, &p->bytes)) || (st = upload(&p->d_cbeg, cbeg, &p->bytes)) ||
            (st = upload(&p->d_ccnt, ccnt, &p->bytes)))
            return st;
    }

    // ---- Schwarz factors of the contracted pairs
    if (p->npair > 0) {
        double *qv = nullptr;
        if ((st = dalloc(&qv, pairs.size()))) return st;
        st = schwarz_factors(p->d_pairs, p->d_geo, p->d_prims, p->pc_begin, p->pc_count, p->npair, boys, qv, s);
        if (st) { hipFree(qv); return st; }
        launch_store_q(p->npair, qv, p->d_geo, p->d_Q, s);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        hipFree(qv);
        if (e != hipSuccess) return fail(HGP_E_DEVICE, std::string("storing Schwarz factors: ") + hipGetErrorString(e));
    }

    // ---- screened unique-quartet lists per canonical class
    // First every list is counted (per bra row: kets kept and their primitive
    // pairs).  Lists are then materialised as (bra, ket) pairs while they fit
    // the budget, smallest first; the rest are streamed: each build re-screens
    // their rows chunk by chunk into one buffer (same pairs, same order).
    {
        std::vector<int> npr(std::max<size_t>(pairs.size(), 1), 0);
        for (size_t k = 0; k < pairs.size(); ++k) npr[k] = pairs[k].nprim;
        if ((st = upload(&p->d_npr, npr, &p->bytes))) return st;
    }
    int64_t *d_counts = nullptr, *d_pcounts = nullptr;
    int maxrows = 1;
    for (int c = 0; c < npc; ++c) maxrows = std::max(maxrows, p->pc_count[c]);
    if ((st = dalloc(&d_counts, (size_t)maxrows + 1)) || (st = dalloc(&d_pcounts, (size_t)maxrows + 1))) {
        hipFree(d_counts);
        return st;
    }
    auto free_counts = [&]() { hipFree(d_counts); hipFree(d_pcounts); };
    std::vector<std::vector<int64_t>> row_off;     // per list: nb + 1 exclusive offsets
    std::vector<int64_t> hc(maxrows), hp(maxrows);
    for (int bc = 0; bc < npc; ++bc) {
        for (int kc = 0; kc <= bc; ++kc) {
            const int nb = p->pc_count[bc], nk = p->pc_count[kc];
            if (!nb || !nk) continue;
            int la = 0, lc = 0;
            while (pair_class_of(la + 1, 0) <= bc) ++la;
            while (pair_class_of(lc + 1, 0) <= kc) ++lc;
            const int lb = bc - pair_class_of(la, 0), ld = kc - pair_class_of(lc, 0);
            const int ci = class_index(la, lb, lc, ld);
            if (ci < 0) { free_counts(); return fail(HGP_E_UNSUPPORTED_L, "class kernel not built"); }
            if ((st = prepare_class(g_class_table[ci]))) { free_counts(); return st; }
            const int sym = (bc == kc);
            const int b0 = p->pc_begin[bc];
            const double t = tau > 0 ? tau : -1.0;
            // bands of Q_ab Q_cd: [t, theta) in FP32 where the class has a
            // register-tier FP32 kernel and the plan is mixed, the rest in FP64.
            // The row-form classes' FP32 Phase 1 stays out of J/K plans: their
            // HRR cancels between intermediates far larger than the integrals,
            // which lifts the FP32 rounding of the VRR values (per primitive
            // quartet about 1e-4 of the block's largest integral for (dd|dd),
            // more than the integrals themselves for (ff|ff))
            struct Band { double lo, hi; int bits; };
            std::vector<Band> bands;
            const double inf = std::numeric_limits<double>::infinity();
            if (p->theta > t && g_class_table[ci].jk32) {
                bands.push_back({t, p->theta, 32});
                bands.push_back({p->theta, inf, 64});
            } else {
                bands.push_back({t, inf, 64});
            }
            for (const Band &bd : bands) {
                launch_screen_count(b0, nb, sym, p->d_Q, bd.lo, bd.hi, p->d_psys, p->d_cbeg + (size_t)kc * nsys,
                                    p->d_ccnt + (size_t)kc * nsys, p->d_npr, d_counts, d_pcounts, s);
                HGP_HIP(hipGetLastError());
                HGP_HIP(hipMemcpyAsync(hc.data(), d_counts, sizeof(int64_t) * nb, hipMemcpyDeviceToHost, s));
                HGP_HIP(hipMemcpyAsync(hp.data(), d_pcounts, sizeof(int64_t) * nb, hipMemcpyDeviceToHost, s));
                HGP_HIP(hipStreamSynchronize(s));
                ClassList cl;
                cl.cls = ci;
                cl.bits = bd.bits;
                cl.b0 = b0; cl.nb = nb; cl.sym = sym; cl.kc = kc;
                cl.lo = bd.lo; cl.hi = bd.hi;
                std::vector<int64_t> off((size_t)nb + 1, 0);
                int64_t np = 0;
                for (int r = 0; r < nb; ++r) {
                    off[(size_t)r + 1] = off[(size_t)r] + hc[(size_t)r];
                    np += (int64_t)pairs[(size_t)(b0 + r)].nprim * hp[(size_t)r];
                }
                cl.nq = off[(size_t)nb];
                cl.nprimq = np;
                p->kept += cl.nq;
                p->lists.push_back(cl);
                row_off.push_back(std::move(off));
            }
        }
    }
    free_counts();
    // staged-tier buffer: one batch per class where it fits under the cap
    int64_t sbuf = 0;
    for (const ClassList &cl : p->lists) sbuf = std::max(sbuf, staged_need(g_class_table[cl.cls], cl.nq));
    if (budget && (size_t)(p->bytes + sbuf * (int64_t)sizeof(double)) > budget)
        return fail(HGP_E_OOM, "plan exceeds the HBM budget (staged-tier buffer)");
    if ((st = dalloc(&p->d_scratch, (size_t)sbuf, &p->bytes))) return st;
    p->scratch_doubles = sbuf;
    // the budget for the lists: the caller's, else half the device memory free now
    int64_t room = 0;
    if (budget) {
        room = (int64_t)budget - p->bytes;
    } else {
        size_t fr = 0, tot = 0;
        HGP_HIP(hipMemGetInfo(&fr, &tot));
        room = (int64_t)(fr / 2);
    }
    std::vector<size_t> order(p->lists.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return p->lists[x].nq < p->lists[y].nq; });
    int64_t all = 0, longest_row = 0;
    for (const ClassList &cl : p->lists) all += cl.nq;
    // what materialising fits; a streamed list needs its row offsets and a chunk
    // buffer that holds its longest row
    std::vector<char> stream(p->lists.size(), 0);
    int64_t used = 0;
    for (size_t k : order) {
        const int64_t need = p->lists[k].nq * (int64_t)sizeof(int2);
        if (all * (int64_t)sizeof(int2) <= room || used + need <= room / 2) {
            used += need;
        } else {
            stream[k] = 1;
            used += (int64_t)(p->lists[k].nb + 1) * (int64_t)sizeof(int64_t);
            for (int r = 0; r < p->lists[k].nb; ++r)
                longest_row = std::max(longest_row, row_off[k][(size_t)r + 1] - row_off[k][(size_t)r]);
        }
    }
    if (longest_row > 0) {
        p->chunk_cap = std::max<int64_t>(longest_row, (room - used) / (int64_t)sizeof(int2));
        p->chunk_cap = std::min<int64_t>(p->chunk_cap, (int64_t)1 << 27);      // 1 GiB of pairs per chunk
        if (p->chunk_cap < longest_row || (room - used) < longest_row * (int64_t)sizeof(int2))
            return fail(HGP_E_OOM, "plan exceeds the HBM budget (a streamed row does not fit)");
        if ((st = dalloc(&p->d_chunk, (size_t)p->chunk_cap, &p->bytes))) return st;
    }
    for (size_t k = 0; k < p->lists.size(); ++k) {
        ClassList &cl = p->lists[k];
        if (cl.nq == 0) continue;
        int64_t *d_off = nullptr;
        if ((st = upload(&d_off, std::vector<int64_t>(row_off[k].begin(), row_off[k].end() - 1),
                         stream[k] ? &p->bytes : nullptr)))
            return st;
        if (stream[k]) {
            cl.d_off = d_off;
            // rows into chunks of at most chunk_cap quartets
            cl.chunk_row.push_back(0);
            cl.chunk_off.push_back(0);
            for (int r = 0; r < cl.nb; ++r)
                if (row_off[k][(size_t)r + 1] - cl.chunk_off.back() > p->chunk_cap) {
                    cl.chunk_row.push_back(r);
                    cl.chunk_off.push_back(row_off[k][(size_t)r]);
                }
            cl.chunk_row.push_back(cl.nb);
            cl.chunk_off.push_back(cl.nq);
            continue;
        }
        st = dalloc(&cl.d_q, (size_t)cl.nq, &p->bytes);
        if (!st) {
            launch_screen_write(cl.b0, cl.nb, cl.sym, p->d_Q, cl.lo, cl.hi, p->d_psys,
                                p->d_cbeg + (size_t)cl.kc * nsys, p->d_ccnt + (size_t)cl.kc * nsys, d_off, 0, cl.d_q,
                                s);
            const hipError_t e = hipStreamSynchronize(s);
            if (e != hipSuccess) st = fail(HGP_E_DEVICE, std::string("writing a quartet list: ") + hipGetErrorString(e));
        }
        hipFree(d_off);
        if (st) return st;
    }
    // side streams for concurrent class lists (default priority, non-blocking)
    for (int k = 0; k < HGP_SIDE_STREAMS; ++k) {
        hipStream_t ss = nullptr;
        HGP_HIP(hipStreamCreateWithFlags(&ss, hipStreamNonBlocking));
        p->side.push_back(ss);
    }
    for (int k = 0; k <= HGP_SIDE_STREAMS; ++k) {
        hipEvent_t e = nullptr;
        HGP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        p->side_ev.push_back(e);
    }
    // heaviest classes first
    std::stable_sort(p->lists.begin(), p->lists.end(), [](const ClassList &x, const ClassList &y) {
        const double cx = x.nprimq * g_class_table[x.cls].vrr_flops + x.nq * g_class_table[x.cls].p2_flops;
        const double cy = y.nprimq * g_class_table[y.cls].vrr_flops + y.nq * g_class_table[y.cls].p2_flops;
        return cx > cy;
    });
    HGP_HIP(hipStreamSynchronize(s));
    return HGP_OK;
}

hgp_status hgp_plan_create_mixed(const hgp_basis *b, double schwarz_tau, double theta, size_t hbm_budget_bytes,
                                 void *hip_stream, hgp_plan **out)
{
    if (!out) return fail(HGP_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!b) return fail(HGP_E_INVALID, "basis is NULL");
    if (!(schwarz_tau >= 0.0) || !std::isfinite(schwarz_tau)) return fail(HGP_E_INVALID, "schwarz_tau must be >= 0");
    if (!(theta >= 0.0) || !std::isfinite(theta)) return fail(HGP_E_INVALID, "theta must be >= 0 and finite");
    if (b->lmax > built_max_l()) return fail(HGP_E_UNSUPPORTED_L, "basis has l above the classes built into this library");
    auto *p = new hgp_plan();
    p->b = b;
    p->device = b->device;
    p->theta = theta > schwarz_tau ? theta : 0.0;
    hgp_status st = plan_build(p, schwarz_tau, hbm_budget_bytes, (hipStream_t)hip_stream);
    if (st != HGP_OK) {
        hgp_plan_destroy(p);
        return st;
    }
    *out = p;
    return HGP_OK;
}

hgp_status hgp_plan_create(const hgp_basis *b, double schwarz_tau, int32_t precision, size_t hbm_budget_bytes,
                           void *hip_stream, hgp_plan **out)
{
    if (out) *out = nullptr;
    if (precision != HGP_FP64 && precision != HGP_MIXED) return fail(HGP_E_INVALID, "precision must be HGP_FP64 or HGP_MIXED");
    return hgp_plan_create_mixed(b, schwarz_tau, precision == HGP_MIXED ? HGP_MIXED_THETA_DEFAULT : 0.0,
                                 hbm_budget_bytes, hip_stream, out);
}

hgp_status hgp_plan_create_multi(const hgp_basis *const *bases, int32_t n, double schwarz_tau, double theta,
                                 size_t hbm_budget_bytes, void *hip_stream, hgp_plan **out)
{
    if (!out) return fail(HGP_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n < 1 || !bases) return fail(HGP_E_INVALID, "need n >= 1 bases");
    if (!(schwarz_tau >= 0.0) || !std::isfinite(schwarz_tau)) return fail(HGP_E_INVALID, "schwarz_tau must be >= 0");
    if (!(theta >= 0.0) || !std::isfinite(theta)) return fail(HGP_E_INVALID, "theta must be >= 0 and finite");
    std::vector<int32_t> l, nprim, sys;
    std::vector<double> cen, exps, coefs;
    std::vector<int> R, N;
    int dev = -1, nbf = 0;
    for (int k = 0; k < n; ++k) {
        const hgp_basis *b = bases[k];
        if (!b) return fail(HGP_E_INVALID, "a basis is NULL");
        if (dev >= 0 && b->device != dev) return fail(HGP_E_INVALID, "all bases must be on one device");
        if (b->flags != bases[0]->flags) return fail(HGP_E_INVALID, "all bases must be created with the same flags");
        dev = b->device;
        l.insert(l.end(), b->l.begin(), b->l.end());
        nprim.insert(nprim.end(), b->nprim.begin(), b->nprim.end());
        cen.insert(cen.end(), b->cen.begin(), b->cen.end());
        exps.insert(exps.end(), b->exps.begin(), b->exps.end());
        coefs.insert(coefs.end(), b->coefs.begin(), b->coefs.end());
        sys.insert(sys.end(), (size_t)b->nshell, k);
        R.push_back(nbf);
        N.push_back(b->nbf);
        nbf += b->nbf;
    }
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || cur != dev) return fail(HGP_E_INVALID, "the bases' device is not current");
    hgp_basis *u = nullptr;
    hgp_status st = hgp_basis_create((int32_t)l.size(), l.data(), nprim.data(), cen.data(), exps.data(), coefs.data(),
                                     bases[0]->flags, &u);
    if (st) return st;
    if (u->lmax > built_max_l()) {
        hgp_basis_destroy(u);
        return fail(HGP_E_UNSUPPORTED_L, "basis has l above the classes built into this library");
    }
    auto *p = new hgp_plan();
    p->b = u;
    p->owned = u;
    p->device = u->device;
    p->theta = theta > schwarz_tau ? theta : 0.0;
    p->nsys = n;
    p->shell_sys.assign(sys.begin(), sys.end());
    p->sys_R = R;
    p->sys_N = N;
    st = plan_build(p, schwarz_tau, hbm_budget_bytes, (hipStream_t)hip_stream);
    if (st != HGP_OK) {
        hgp_plan_destroy(p);
        return st;
    }
    *out = p;
    return HGP_OK;
}

hgp_status hgp_plan_stats(const hgp_plan *p, int64_t *kept, int64_t *total, int64_t *bytes)
{
    if (!p) return fail(HGP_E_INVALID, "plan is NULL");
    if (kept) *kept = p->kept;
    if (total) *total = p->total;
    if (bytes) *bytes = p->bytes;
    return HGP_OK;
}

hgp_status hgp_plan_prim_stats(const hgp_plan *p, int64_t *prim_pairs_kept, int64_t *prim_pairs_total)
{
    if (!p) return fail(HGP_E_INVALID, "plan is NULL");
    if (prim_pairs_kept) *prim_pairs_kept = p->prim_kept;
    if (prim_pairs_total) *prim_pairs_total = p->prim_total;
    return HGP_OK;
}

hgp_status hgp_plan_stream_stats(const hgp_plan *p, int64_t *quartets_streamed, int64_t *chunks,
                                 int64_t *chunk_capacity)
{
    if (!p) return fail(HGP_E_INVALID, "plan is NULL");
    int64_t q = 0, c = 0;
    for (const ClassList &cl : p->lists)
        if (!cl.d_q && cl.nq > 0) {
            q += cl.nq;
            c += (int64_t)cl.chunk_row.size() - 1;
        }
    if (quartets_streamed) *quartets_streamed = q;
    if (chunks) *chunks = c;
    if (chunk_capacity) *chunk_capacity = p->chunk_cap;
    return HGP_OK;
}

int32_t hgp_plan_num_classes(const hgp_plan *p) { return p ? (int32_t)p->lists.size() : 0; }

hgp_status hgp_plan_class_precision(const hgp_plan *p, int32_t c, int32_t *bits)
{
    if (!p || c < 0 || c >= (int32_t)p->lists.size() || !bits) return fail(HGP_E_INVALID, "bad plan or class index");
    *bits = p->lists[c].bits;
    return HGP_OK;
}

hgp_status hgp_plan_class_info(const hgp_plan *p, int32_t c, int32_t *ls, int64_t *nq, int64_t *npq, double *vf,
                               double *pf, int32_t *tier)
{
    if (!p || c < 0 || c >= (int32_t)p->lists.size()) return fail(HGP_E_INVALID, "bad plan or class index");
    const ClassList &cl = p->lists[c];
    const ClassKernels &k = g_class_table[cl.cls];
    if (ls) { ls[0] = k.la; ls[1] = k.lb; ls[2] = k.lc; ls[3] = k.ld; }
    if (nq) *nq = cl.nq;
    if (npq) *npq = cl.nprimq;
    if (vf) *vf = k.vrr_flops;
    if (pf) *pf = k.p2_flops;
    if (tier) *tier = k.tier;
    return HGP_OK;
}

hgp_status hgp_plan_schwarz(const hgp_plan *p, double *Q)
{
    if (!p || !Q) return fail(HGP_E_INVALID, "NULL argument");
    const int ns = p->b->nshell;
    std::vector<double> q((size_t)p->npair);
    if (p->npair) HGP_HIP(hipMemcpy(q.data(), p->d_Q, sizeof(double) * q.size(), hipMemcpyDeviceToHost));
    std::fill(Q, Q + (size_t)ns * ns, 0.0);
    for (int i = 0; i < p->npair; ++i) {
        const PairInfo &pi = p->pairs[i];
        Q[(size_t)pi.sh_a * ns + pi.sh_b] = Q[(size_t)pi.sh_b * ns + pi.sh_a] = q[i];
    }
    return HGP_OK;
}

hgp_status hgp_plan_set_timing(hgp_plan *p, int32_t enable)
{
    if (!p) return fail(HGP_E_INVALID, "plan is NULL");
    hgp_status st = collect_timing(p);
    if (st) return st;
    for (ClassList &cl : p->lists) {
        cl.ms[0] = cl.ms[1] = 0.0;
        cl.launches[0] = cl.launches[1] = 0;
    }
    p->timing = enable != 0;
    return HGP_OK;
}

hgp_status hgp_plan_class_timing(hgp_plan *p, int32_t c, int32_t kernel, int64_t *launches, double *total_ms)
{
    if (!p || c < 0 || c >= (int32_t)p->lists.size() || kernel < 0 || kernel > 1)
        return fail(HGP_E_INVALID, "bad plan, class or kernel index");
    hgp_status st = collect_timing(p);
    if (st) return st;
    if (launches) *launches = p->lists[c].launches[kernel];
    if (total_ms) *total_ms = p->lists[c].ms[kernel];
    return HGP_OK;
}

// The class lists of a plan over D (laid out like the accumulators) into the
// unsymmetrised accumulators, which the caller has cleared.
static hgp_status jk_classes(hgp_plan *p, const double *D, bool want_j, bool want_k, hipStream_t s0)
{
    const double *boys = nullptr;
    hgp_status st = boys_table(p->device, &boys);
    if (st) return st;
    // class lists that use no scratch buffer go to the least-loaded of the
    // caller's stream and the side streams (lists come heaviest first).  Not
    // while kernel timing is on (concurrent kernels would stretch each
    // other's timed intervals) and not while the stream is being captured
    // into a graph (the side-stream fork and join under capture crashed the
    // HIP runtime on the host): then every list runs on the caller's stream.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    const bool capturing = hipStreamIsCapturing(s0, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone;
    const int nside = (p->timing || capturing) ? 0 : (int)p->side.size();
    std::vector<double> load((size_t)nside + 1, 0.0);
    std::vector<int> where(p->lists.size(), 0);
    bool any_side = false;
    for (size_t li = 0; li < p->lists.size(); ++li) {
        const ClassList &cl = p->lists[li];
        const ClassKernels &k = g_class_table[cl.cls];
        const double c = cl.nprimq * k.vrr_flops + cl.nq * k.p2_flops;
        int w = 0;
        if (cl.nq > 0 && cl.d_q && (k.tier == 0 || k.tier == 3))      // streamed lists share the chunk buffer
            w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[(size_t)w] += c;
        where[li] = w;
        any_side = any_side || w > 0;
    }
    if (any_side) {
        HGP_HIP(hipEventRecord(p->side_ev[0], s0));
        for (int k = 0; k < nside; ++k) HGP_HIP(hipStreamWaitEvent(p->side[(size_t)k], p->side_ev[0], 0));
    }
    hipStream_t s = s0;
    auto mark = [&](hipEvent_t *e) -> hgp_status {
        *e = nullptr;
        if (!p->timing) return HGP_OK;
        *e = take_event(p);
        if (!*e) return fail(HGP_E_DEVICE, "hipEventCreate failed");
        HGP_HIP(hipEventRecord(*e, s));
        return HGP_OK;
    };
    auto done = [&](int li, int kernel, hipEvent_t a, hipEvent_t b) {
        if (p->timing) p->pending.push_back(PendingTiming{li, kernel, a, b});
    };
    for (size_t li = 0; li < p->lists.size(); ++li) {
        const ClassList &cl = p->lists[li];
        if (cl.nq == 0) continue;
        const ClassKernels &k = g_class_table[cl.cls];
        s = where[li] == 0 ? s0 : p->side[(size_t)where[li] - 1];
        JKArgs a{};
        a.pairs = p->d_pairs; a.geo = p->d_geo; a.prims = p->d_prims; a.boys = boys;
        a.D = D; a.J = p->d_Jacc; a.K = p->d_Kacc; a.nbf = (int32_t)p->stride;
        a.want_j = want_j; a.want_k = want_k;
        hipEvent_t e0, e1, e2, e3;
        // a streamed list runs chunk by chunk: its rows re-screened into the chunk buffer
        const int nchunk = cl.d_q ? 1 : (int)cl.chunk_row.size() - 1;
        for (int ch = 0; ch < nchunk; ++ch) {
            const int2 *qbase = cl.d_q;
            int64_t nq = cl.nq;
            if (!cl.d_q) {
                const int r0 = cl.chunk_row[(size_t)ch], r1 = cl.chunk_row[(size_t)ch + 1];
                nq = cl.chunk_off[(size_t)ch + 1] - cl.chunk_off[(size_t)ch];
                if (nq == 0) continue;
                launch_screen_write(cl.b0 + r0, r1 - r0, cl.sym, p->d_Q, cl.lo, cl.hi, p->d_psys,
                                    p->d_cbeg + (size_t)cl.kc * p->nsys, p->d_ccnt + (size_t)cl.kc * p->nsys, cl.d_off + r0,
                                    cl.chunk_off[(size_t)ch], p->d_chunk, s);
                qbase = p->d_chunk;
            }
            if (k.tier == 0 || k.tier == 3) {                // register or wave-cooperative LDS tier
                if ((st = mark(&e0))) return st;
                const int64_t chunk = (int64_t)k.block << 20;
                const launch_jk_fn run = cl.bits == 32 ? k.jk32 : k.jk;
                for (int64_t q0 = 0; q0 < nq; q0 += chunk) {
                    a.quartets = qbase + q0;
                    a.nq = std::min(chunk, nq - q0);
                    run(a, s);
                }
                if ((st = mark(&e1))) return st;
                done((int)li, 0, e0, e1);
            } else {
                const int64_t B = staged_batch(k, p->scratch_doubles);
                for (int64_t q0 = 0; q0 < nq; q0 += B) {
                    const int64_t nb = std::min(B, nq - q0);
                    a.quartets = qbase + q0;
                    a.nq = nb;
                    a.scratch = p->d_scratch;
                    a.stride = B;
                    if (k.tier == 2) {                     // HBM-scratch tier: one kernel per batch
                        if ((st = mark(&e0))) return st;
                        k.jk(a, s);
                        if ((st = mark(&e1))) return st;
                        done((int)li, 0, e0, e1);
                        continue;
                    }
                    P1Args pa{(const int32_t *)(qbase + q0), 2, nb, p->d_pairs, p->d_geo, p->d_prims, boys,
                              p->d_scratch, B, 0};
                    if ((st = mark(&e0))) return st;
                    k.p1(pa, s);
                    if ((st = mark(&e1)) || (st = mark(&e2))) return st;
                    k.jk(a, s);
                    if ((st = mark(&e3))) return st;
                    done((int)li, 0, e0, e1);
                    done((int)li, 1, e2, e3);
                }
            }
        }
    }
    if (any_side) {
        for (int k = 0; k < nside; ++k) {
            HGP_HIP(hipEventRecord(p->side_ev[(size_t)k + 1], p->side[(size_t)k]));
            HGP_HIP(hipStreamWaitEvent(s0, p->side_ev[(size_t)k + 1], 0));
        }
    }
    return HGP_OK;
}

static hgp_status launch_status(hgp_plan *p)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        p->broken = true;
        return fail(HGP_E_DEVICE, std::string("J/K launch failed: ") + hipGetErrorString(e));
    }
    return HGP_OK;
}

hgp_status hgp_jk(hgp_plan *p, const double *D, double *J, double *K, void *hip_stream)
{
    if (!p) return fail(HGP_E_INVALID, "plan is NULL");
    if (p->broken) return fail(HGP_E_STATE, "plan unusable after an earlier device failure");
    if (p->nsys > 1) return fail(HGP_E_INVALID, "the plan covers several systems: use hgp_jk_multi");
    const int n = p->b->nbf;
    if (n == 0) return HGP_OK;                       // empty basis: J and K are 0 x 0
    if (!D) return fail(HGP_E_INVALID, "D is NULL");
    if (!J && !K) return fail(HGP_E_INVALID, "both J and K are NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    if (J) launch_fill_zero(p->d_Jacc, p->acc_len, s);
    if (K) launch_fill_zero(p->d_Kacc, p->acc_len, s);
    hgp_status st = jk_classes(p, D, J != nullptr, K != nullptr, s);
    if (st) return st;
    if (J) launch_symmetrize(p->d_Jacc, n, J, n, s);
    if (K) launch_symmetrize(p->d_Kacc, n, K, n, s);
    return launch_status(p);
}

hgp_status hgp_jk_multi(hgp_plan *p, const double *const *D, double *const *J, double *const *K, void *hip_stream)
{
    if (!p) return fail(HGP_E_INVALID, "plan is NULL");
    if (p->broken) return fail(HGP_E_STATE, "plan unusable after an earlier device failure");
    if (!D) return fail(HGP_E_INVALID, "D is NULL");
    const bool want_j = J != nullptr, want_k = K != nullptr;
    if (!want_j && !want_k) return fail(HGP_E_INVALID, "both J and K are NULL");
    for (int sy = 0; sy < p->nsys; ++sy) {
        if (p->sys_N[(size_t)sy] == 0) continue;
        if (!D[sy] || (want_j && !J[sy]) || (want_k && !K[sy]))
            return fail(HGP_E_INVALID, "a system of the plan has no D, J or K");
    }
    if (p->b->nbf == 0) return HGP_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    if (p->nsys == 1) {                          // a one-system plan: the plain path
        if (want_j) launch_fill_zero(p->d_Jacc, p->acc_len, s);
        if (want_k) launch_fill_zero(p->d_Kacc, p->acc_len, s);
        hgp_status st = jk_classes(p, D[0], want_j, want_k, s);
        if (st) return st;
        const int n = p->b->nbf;
        if (want_j) launch_symmetrize(p->d_Jacc, n, J[0], n, s);
        if (want_k) launch_symmetrize(p->d_Kacc, n, K[0], n, s);
        return launch_status(p);
    }
    // each system's density into its block; its accumulator blocks cleared
    const int64_t S = p->stride;
    for (int sy = 0; sy < p->nsys; ++sy) {
        const int n = p->sys_N[(size_t)sy];
        const int64_t base = (int64_t)p->sys_R[(size_t)sy] * (S + 1);
        launch_block_in(D[sy], n, p->d_Dunion + base, S, s);
        if (want_j) launch_block_zero(p->d_Jacc + base, n, S, s);
        if (want_k) launch_block_zero(p->d_Kacc + base, n, S, s);
    }
    hgp_status st = jk_classes(p, p->d_Dunion, want_j, want_k, s);
    if (st) return st;
    for (int sy = 0; sy < p->nsys; ++sy) {
        const int n = p->sys_N[(size_t)sy];
        const int64_t base = (int64_t)p->sys_R[(size_t)sy] * (S + 1);
        if (want_j) launch_symmetrize(p->d_Jacc + base, S, J[sy], n, s);
        if (want_k) launch_symmetrize(p->d_Kacc + base, S, K[sy], n, s);
    }
    return launch_status(p);
}

}  // extern "C"

namespace {

// Side streams of the shell-quartet calls, one set per device, created on
// first use (default priority) and kept until the process ends.  A call holds
// its device's set while it enqueues; its classes go to the caller's stream
// and these, forked and joined with the set's events (derivative classes with
// a region of the accumulator buffer per stream).
constexpr int SQ_NSIDE = 3;
struct SqSide {
    std::mutex m;
    bool ok = false;
    hipStream_t st[SQ_NSIDE] = {};
    hipEvent_t fork = nullptr, join[SQ_NSIDE] = {};
};

SqSide *sq_side(int dev)
{
    static std::mutex mm;
    static std::map<int, SqSide *> sets;
    std::lock_guard<std::mutex> lock(mm);
    SqSide *&x = sets[dev];
    if (!x) x = new SqSide;
    return x;
}

// Shell quartets given on the device, integrals (deriv = false) or their
// first derivatives (deriv = true: 12 blocks a quartet, from the register form
// of the class where it has one, else from its wave-form tables).
hgp_status shell_quartets(const hgp_basis *b, int64_t nq, const int32_t *quartets, const int64_t *offsets,
                          double *out, void *hip_stream, bool deriv)
{
    if (!b) return fail(HGP_E_INVALID, "basis is NULL");
    if (nq < 0) return fail(HGP_E_INVALID, "nq < 0");
    if (nq == 0) return HGP_OK;
    if (!quartets || !offsets || !out) return fail(HGP_E_INVALID, "NULL argument");
    if (nq > (int64_t)1 << 28) return fail(HGP_E_INVALID, "too many quartets in one call");
    hipStream_t s = (hipStream_t)hip_stream;
    const double *boys = nullptr;
    hgp_status st = boys_table(b->device, &boys);
    if (st) return st;
    if ((st = keep_pool(b->device))) return st;
    ClassOf cof;
    for (int k = 0; k < 625; ++k) cof.c[k] = -1;
    const int ncls = deriv ? g_num_deriv : g_num_classes;
    for (int c = 0; c < ncls; ++c) {
        const int la = deriv ? g_deriv_table[c].la : g_class_table[c].la, lb = deriv ? g_deriv_table[c].lb : g_class_table[c].lb;
        const int lc = deriv ? g_deriv_table[c].lc : g_class_table[c].lc, ld = deriv ? g_deriv_table[c].ld : g_class_table[c].ld;
        cof.c[((la * 5 + lb) * 5 + lc) * 5 + ld] = (int16_t)c;
    }
    // stream-ordered temporaries; every exit below frees them on the stream
    int32_t *d_code = nullptr;
    int64_t *d_poff = nullptr, *d_ptotal = nullptr, *d_base = nullptr, *d_btotal = nullptr, *d_stmp = nullptr;
    unsigned long long *d_counts = nullptr, *d_cursor = nullptr, *d_err = nullptr;
    PairInfo *d_pairs = nullptr;
    PairGeo *d_geo = nullptr;
    PrimPair *d_prims = nullptr;
    EriTask *d_tasks = nullptr;
    double *d_scr = nullptr;
    std::vector<void *> held;
    auto get = [&](void **p, size_t bytes) {
        const hipError_t e = hipMallocAsync(p, bytes, s);
        if (e == hipSuccess) held.push_back(*p);
        return e;
    };
    auto release = [&]() {
        for (void *p : held) hipFreeAsync(p, s);
        held.clear();
    };
    const size_t nc8 = (size_t)ncls, nk8 = nc8 * SQ_BUCKETS;      // keys: (class, primitive-count bucket)
    hipError_t e = get((void **)&d_code, sizeof(int32_t) * nq);
    if (e == hipSuccess) e = get((void **)&d_poff, sizeof(int64_t) * nq);
    if (e == hipSuccess) e = get((void **)&d_ptotal, sizeof(int64_t));
    if (e == hipSuccess) e = get((void **)&d_base, sizeof(int64_t) * nk8);
    if (e == hipSuccess) e = get((void **)&d_btotal, sizeof(int64_t));
    if (e == hipSuccess) e = get((void **)&d_stmp, sizeof(int64_t) * (size_t)((nq + 1023) / 1024));
    // counts, cursors and the error word in one zeroed block
    if (e == hipSuccess) e = get((void **)&d_counts, sizeof(unsigned long long) * (2 * nk8 + 1));
    if (e != hipSuccess) {
        release();
        return fail(HGP_E_OOM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
    }
    d_cursor = d_counts + nk8;
    d_err = d_counts + 2 * nk8;
    launch_fill_zero((double *)d_counts, (int64_t)(2 * nk8 + 1), s);      // all-zero bits
    launch_sq_classify(nq, quartets, offsets, b->nshell, b->d_l, b->d_nprim, cof, (int)nk8, d_code, d_poff, d_counts,
                       d_err, s);
    launch_scan(d_poff, (int)nq, d_ptotal, d_stmp, s);
    e = hipMemcpyAsync(d_base, d_counts, sizeof(int64_t) * nk8, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) {
        release();
        return fail(HGP_E_DEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    }
    launch_scan(d_base, (int)nk8, d_btotal, nullptr, s);
    // the one wait: per-key counts, the error word and the primitive total size the launches
    std::vector<unsigned long long> hk(nk8 + 1);
    int64_t ptotal = 0;
    e = hipMemcpyAsync(hk.data(), d_counts, sizeof(unsigned long long) * nk8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&hk[nk8], d_err, sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&ptotal, d_ptotal, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        release();
        return fail(HGP_E_DEVICE, std::string("classifying the quartets: ") + hipGetErrorString(e));
    }
    // per class (its keys are contiguous), then the error word
    std::vector<unsigned long long> h(nc8 + 1, 0ull);
    for (size_t k = 0; k < nk8; ++k) h[k / SQ_BUCKETS] += hk[k];
    h[nc8] = hk[nk8];
    if (h[nc8] & 1ull) { release(); return fail(HGP_E_INVALID, "shell index out of range or negative offset"); }
    if (h[nc8] & 2ull) {
        release();
        return fail(HGP_E_UNSUPPORTED_L, deriv ? "derivative integrals are built for shells up to l = " +
                                                     std::to_string(max_deriv_l())
                                               : std::string("class kernel not built"));
    }
    if (ptotal > INT32_MAX) { release(); return fail(HGP_E_INVALID, "too many primitive pairs in one call"); }
    int64_t sneed = 0;
    // classes over the caller's stream (0) and the side streams (1 ..
    // SQ_NSIDE), largest estimated work first, each to the least loaded:
    // every derivative class (each stream gets its own buffer region), and of
    // the integral classes those that use no buffer (register and wave-LDS
    // tiers); staged and HBM-scratch integral classes share the buffer on 0
    std::vector<int> lane((size_t)ncls, 0);
    int64_t need[1 + SQ_NSIDE] = {0}, roff[1 + SQ_NSIDE] = {0};
    {
        std::vector<std::pair<double, int>> est;
        double load[1 + SQ_NSIDE] = {0.0};
        for (int c = 0; c < ncls; ++c) {
            if (!h[(size_t)c]) continue;
            const double n = (double)h[(size_t)c];
            // primitive quartets from the keys' log2 buckets (bucket b: about 1.5 * 2^(SQ_BUCKETS - 1 - b) each)
            double np = 0.0;
            for (int bk = 0; bk < SQ_BUCKETS; ++bk)
                np += (double)hk[(size_t)c * SQ_BUCKETS + bk] * 1.5 * std::ldexp(1.0, SQ_BUCKETS - 1 - bk);
            if (deriv) {
                est.push_back({np * g_deriv_table[c].t->n_vrr + n * g_deriv_table[c].t->n_p2, c});
            } else {
                const ClassKernels &k = g_class_table[c];
                const double w = np * k.vrr_flops + n * k.p2_flops;
                if (k.tier == 0 || k.tier == 3)
                    est.push_back({w, c});
                else
                    load[0] += w;
            }
        }
        std::sort(est.begin(), est.end(), [](const std::pair<double, int> &a, const std::pair<double, int> &b) {
            return a.first > b.first || (a.first == b.first && a.second < b.second);
        });
        for (const auto &x : est) {
            int k = 0;
            for (int j = 1; j <= SQ_NSIDE; ++j)
                if (load[j] < load[k]) k = j;
            lane[(size_t)x.second] = k;
            load[k] += x.first;
        }
    }
    for (int c = 0; c < ncls; ++c)
        if (h[(size_t)c]) {
            if (deriv) {
                const DerivClass &dc = g_deriv_table[c];
                if (deriv_use_reg(dc, (int64_t)h[(size_t)c])) continue;
                const int pe = t3_prepare(*dc.t);
                if (pe != 0) {
                    release();
                    return fail(HGP_E_DEVICE, std::string("preparing derivative tables: ") +
                                                  hipGetErrorString((hipError_t)pe));
                }
                if (dc.p1) {
                    const int64_t n = (int64_t)h[(size_t)c];
                    const int ns = deriv_nseg(dc, n);
                    int64_t &nd = need[lane[(size_t)c]];
                    nd = std::max(nd, deriv_batch(dc, n, ns) * ns * (int64_t)dc.t->n_hrr);
                }
                continue;
            }
            if ((st = prepare_class(g_class_table[c]))) { release(); return st; }
            sneed = std::max(sneed, staged_need(g_class_table[c], (int64_t)h[(size_t)c]));
        }
    if (deriv) {
        for (int k = 0; k <= SQ_NSIDE; ++k) {
            roff[k] = sneed;
            sneed += need[k];
        }
    }
    e = get((void **)&d_pairs, sizeof(PairInfo) * 2 * nq);
    if (e == hipSuccess) e = get((void **)&d_geo, sizeof(PairGeo) * 2 * nq);
    if (e == hipSuccess) e = get((void **)&d_prims, sizeof(PrimPair) * (size_t)std::max<int64_t>(ptotal, 1));
    if (e == hipSuccess) e = get((void **)&d_tasks, sizeof(EriTask) * nq);
    if (e == hipSuccess && sneed) e = get((void **)&d_scr, sizeof(double) * sneed);
    if (e != hipSuccess) {
        release();
        return fail(HGP_E_OOM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
    }
    launch_sq_scatter(nq, quartets, offsets, b->d_l, b->d_nprim, b->d_foff, d_code, d_poff, d_base, (int)nk8, d_cursor,
                      d_pairs, d_tasks, s);
    launch_pairs((int)(2 * nq), d_pairs, b->d_cen, b->d_poff, b->d_exps, b->d_ncoef, d_geo, d_prims, s);
    // fork the side streams, which read what the stream has written so far
    SqSide *sd = nullptr;
    std::unique_lock<std::mutex> side_lock;
    bool used[1 + SQ_NSIDE] = {true, false, false, false};
    for (int c = 0; c < ncls; ++c)
        if (h[(size_t)c]) used[lane[(size_t)c]] = true;
    if (used[1] || used[2] || used[3]) {
        int dev = 0;
        e = hipGetDevice(&dev);
        if (e == hipSuccess) {
            sd = sq_side(dev);
            side_lock = std::unique_lock<std::mutex>(sd->m);
            for (int k = 0; k < SQ_NSIDE && !sd->ok && e == hipSuccess; ++k) {
                e = hipStreamCreateWithFlags(&sd->st[k], hipStreamNonBlocking);
                if (e == hipSuccess) e = hipEventCreateWithFlags(&sd->join[k], hipEventDisableTiming);
            }
            if (!sd->ok && e == hipSuccess) e = hipEventCreateWithFlags(&sd->fork, hipEventDisableTiming);
            if (e == hipSuccess) sd->ok = true;
        }
        if (e == hipSuccess) e = hipEventRecord(sd->fork, s);
        for (int k = 0; k < SQ_NSIDE && e == hipSuccess; ++k)
            if (used[k + 1]) e = hipStreamWaitEvent(sd->st[k], sd->fork, 0);
        if (e != hipSuccess) {
            release();
            return fail(HGP_E_DEVICE, std::string("side streams: ") + hipGetErrorString(e));
        }
    }
    int64_t begin = 0;
    for (int c = 0; c < ncls; ++c) {
        const int64_t cnt = (int64_t)h[(size_t)c];
        if (!cnt) continue;
        EriArgs a{};
        a.tasks = d_tasks + begin;
        a.ntask = cnt;
        a.pairs = d_pairs; a.geo = d_geo; a.prims = d_prims; a.boys = boys;
        a.out = out;
        a.mode = 0;
        a.scratch = d_scr;
        if (deriv) {
            // launches of at most 2^20 quartets (a workgroup each in the table form); the
            // staged form in batches whose accumulators fit the buffer, slot stride = batch
            const DerivClass &dc = g_deriv_table[c];
            const int k = lane[(size_t)c];
            hipStream_t ss = k ? sd->st[k - 1] : s;
            const bool reg = deriv_use_reg(dc, cnt);
            const int nseg = dc.p1 && !reg ? deriv_nseg(dc, cnt) : 1;
            const int64_t step = reg || !dc.p1 ? (int64_t)1 << 20 : deriv_batch(dc, cnt, nseg);
            for (int64_t q0 = 0; q0 < cnt; q0 += step) {
                EriArgs x = a;
                x.tasks = a.tasks + q0;
                x.ntask = std::min<int64_t>(step, cnt - q0);
                if (reg) {
                    dc.reg(x, d_code, 1, ss);
                } else if (dc.p1) {
                    x.stride = x.ntask;
                    x.scratch = d_scr + roff[k];
                    dc.p1(x, d_code, nseg, ss);
                    t3w_launch_deriv_p2(*dc.t, x, d_code, nseg, ss);
                } else {
                    t3w_launch_deriv(*dc.t, x, d_code, ss);
                }
            }
        } else {
            run_eri_class(g_class_table[c], a, sneed, lane[(size_t)c] ? sd->st[lane[(size_t)c] - 1] : s);
        }
        begin += cnt;
    }
    e = hipGetLastError();
    // join the side streams before the temporaries are freed on the caller's stream
    for (int k = 0; sd && k < SQ_NSIDE; ++k)
        if (used[k + 1]) {
            hipError_t j = hipEventRecord(sd->join[k], sd->st[k]);
            if (j == hipSuccess) j = hipStreamWaitEvent(s, sd->join[k], 0);
            if (j != hipSuccess && e == hipSuccess) e = j;
        }
    release();
    if (e != hipSuccess) return fail(HGP_E_DEVICE, std::string("integral kernels: ") + hipGetErrorString(e));
    return HGP_OK;
}

}  // namespace

extern "C" {

hgp_status hgp_eri_shell_quartets(const hgp_basis *b, int64_t nq, const int32_t *quartets, const int64_t *offsets,
                                  double *out, void *hip_stream)
{
    return shell_quartets(b, nq, quartets, offsets, out, hip_stream, false);
}

hgp_status hgp_eri_deriv_shell_quartets(const hgp_basis *b, int64_t nq, const int32_t *quartets,
                                        const int64_t *offsets, double *out, void *hip_stream)
{
    return shell_quartets(b, nq, quartets, offsets, out, hip_stream, true);
}

int32_t hgp_deriv_max_l(void) { return max_deriv_l(); }

}  // extern "C"

namespace {

// Validated class and layout of one hgp_eri_prim_quartets call.
struct PrimCall {
    int ci = -1;              // class table index
    int ls[4], pos[4], cs[4];
    int64_t blk = 0;          // integrals per quartet
    bool f32 = false;         // HGP_MIXED: FP32 VRR and contraction where the class has that form
};

hgp_status prim_call_setup(int32_t la, int32_t lb, int32_t lc, int32_t ld, int64_t n, const double *centers,
                           const double *exps, double *out, int32_t precision, PrimCall *c)
{
    const int lin[4] = {la, lb, lc, ld};
    for (int r = 0; r < 4; ++r) {
        if (lin[r] < 0) return fail(HGP_E_INVALID, "negative l");
        if (lin[r] > 4) return fail(HGP_E_UNSUPPORTED_L, "l > 4");
    }
    if (precision != HGP_FP64 && precision != HGP_MIXED) return fail(HGP_E_INVALID, "precision must be HGP_FP64 or HGP_MIXED");
    c->f32 = precision == HGP_MIXED;
    if (n < 0) return fail(HGP_E_INVALID, "n < 0");
    if (n > 0 && (!centers || !exps || !out)) return fail(HGP_E_INVALID, "NULL argument");
    if (n > (int64_t)1 << 30) return fail(HGP_E_INVALID, "n too large for one call");
    int *pos = c->pos;
    for (int r = 0; r < 4; ++r) pos[r] = r;
    if (lin[0] < lin[1]) std::swap(pos[0], pos[1]);
    if (lin[2] < lin[3]) std::swap(pos[2], pos[3]);
    if (pair_class_of(lin[pos[0]], lin[pos[1]]) < pair_class_of(lin[pos[2]], lin[pos[3]])) {
        std::swap(pos[0], pos[2]);
        std::swap(pos[1], pos[3]);
    }
    int nn[4], stride[4];
    for (int r = 0; r < 4; ++r) { c->ls[r] = lin[pos[r]]; nn[r] = nsph(lin[r]); }
    c->ci = class_index(c->ls[0], c->ls[1], c->ls[2], c->ls[3]);
    if (c->ci < 0) return fail(HGP_E_UNSUPPORTED_L, "class kernel not built into this library");
    stride[3] = 1; stride[2] = nn[3]; stride[1] = nn[2] * nn[3]; stride[0] = nn[1] * nn[2] * nn[3];
    for (int r = 0; r < 4; ++r) c->cs[r] = stride[pos[r]];
    c->blk = (int64_t)nn[0] * nn[1] * nn[2] * nn[3];
    return HGP_OK;
}

// Pair records of the n quartets, then the class kernels (in batches through
// the scratch buffer for the staged and op-table tiers).
void prim_call_run(const PrimCall &c, int64_t n, const double *centers, const double *exps, double *out,
                   const double *boys, PairInfo *d_pairs, PairGeo *d_geo, PrimPair *d_prims, EriTask *d_tasks,
                   double *d_scr, int64_t scr_doubles, hipStream_t s)
{
    launch_prim_quartet_pairs(n, centers, exps, c.ls, c.pos, c.cs, c.blk, d_pairs, d_geo, d_prims, d_tasks, s);
    EriArgs a{};
    a.tasks = d_tasks; a.ntask = n; a.pairs = d_pairs; a.geo = d_geo; a.prims = d_prims; a.boys = boys;
    a.out = out; a.mode = 0;
    a.scratch = d_scr;
    run_eri_class(g_class_table[c.ci], a, scr_doubles, s, c.f32);
}

// hgp_eri_prim_quartets_noalloc's buffer: file-scope device memory, one copy
// per device, held until the process ends.  Host code reaches it only through
// the per-device address hipGetSymbolAddress returns (g_scratch_ptr).
constexpr size_t NOALLOC_BYTES = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
unsigned char *g_scratch_ptr[64] = {};

hgp_status noalloc_scratch(int dev, unsigned char **out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (dev < 0 || dev >= 64) return fail(HGP_E_DEVICE, "device index out of range");
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HGP_HIP(on_device(dev, [&]() { return hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)); }));
        if (!ptr) return fail(HGP_E_DEVICE, "hipGetSymbolAddress returned no address for the scratch buffer");
        g_scratch_ptr[dev] = (unsigned char *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return HGP_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Bytes of the fixed buffer that n quartets of class k take: pair and task
// records, plus room for one 64-quartet batch of a staged class.
size_t noalloc_need(const ClassKernels &k, int64_t n)
{
    const size_t rec = align256(sizeof(PairInfo) * 2 * n) + align256(sizeof(PairGeo) * 2 * n) +
                       align256(sizeof(PrimPair) * 2 * n) + align256(sizeof(EriTask) * n);
    return rec + (k.tier == 1 ? sizeof(double) * (size_t)k.scratch_slots * 64 : 0);
}

}  // namespace

extern "C" {

hgp_status hgp_eri_prim_quartets(int32_t la, int32_t lb, int32_t lc, int32_t ld, int64_t n, const double *centers,
                                 const double *exps, double *out, int32_t precision, void *hip_stream)
{
    PrimCall c;
    if (hgp_status st = prim_call_setup(la, lb, lc, ld, n, centers, exps, out, precision, &c)) return st;
    if (n == 0) return HGP_OK;
    if (hgp_status pst = prepare_class(g_class_table[c.ci])) return pst;
    hipStream_t s = (hipStream_t)hip_stream;
    int dev = 0;
    HGP_HIP(hipGetDevice(&dev));
    if (hgp_status kst = keep_pool(dev)) return kst;
    const double *boys = nullptr;
    hgp_status st = boys_table(dev, &boys);
    if (st) return st;
    PairInfo *d_pairs = nullptr;
    PairGeo *d_geo = nullptr;
    PrimPair *d_prims = nullptr;
    EriTask *d_tasks = nullptr;
    double *d_scr = nullptr;
    const int64_t sneed = staged_need(g_class_table[c.ci], n);
    hipError_t e = hipMallocAsync((void **)&d_pairs, sizeof(PairInfo) * 2 * n, s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&d_geo, sizeof(PairGeo) * 2 * n, s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&d_prims, sizeof(PrimPair) * 2 * n, s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&d_tasks, sizeof(EriTask) * n, s);
    if (e == hipSuccess && sneed) e = hipMallocAsync((void **)&d_scr, sizeof(double) * sneed, s);
    if (e != hipSuccess) {
        if (d_pairs) hipFreeAsync(d_pairs, s);
        if (d_geo) hipFreeAsync(d_geo, s);
        if (d_prims) hipFreeAsync(d_prims, s);
        if (d_tasks) hipFreeAsync(d_tasks, s);
        return fail(HGP_E_OOM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
    }
    prim_call_run(c, n, centers, exps, out, boys, d_pairs, d_geo, d_prims, d_tasks, d_scr, sneed, s);
    e = hipGetLastError();
    if (d_scr) hipFreeAsync(d_scr, s);
    hipFreeAsync(d_pairs, s);
    hipFreeAsync(d_geo, s);
    hipFreeAsync(d_prims, s);
    hipFreeAsync(d_tasks, s);
    if (e != hipSuccess) return fail(HGP_E_DEVICE, std::string("microbench launch: ") + hipGetErrorString(e));
    return HGP_OK;
}

hgp_status hgp_class_form(int32_t la, int32_t lb, int32_t lc, int32_t ld, int32_t *tier, int32_t *has_fp32)
{
    PrimCall c;
    double dummy = 0.0;
    if (hgp_status st = prim_call_setup(la, lb, lc, ld, 0, &dummy, &dummy, &dummy, HGP_FP64, &c)) return st;
    const ClassKernels &k = g_class_table[c.ci];
    if (tier) *tier = k.tier;
    if (has_fp32) *has_fp32 = (k.tier == 0 && k.eri32) || (k.tier == 1 && k.p1_32) ? 1 : 0;
    return HGP_OK;
}

int64_t hgp_eri_prim_quartets_noalloc_max(int32_t la, int32_t lb, int32_t lc, int32_t ld)
{
    PrimCall c;
    double dummy = 0.0;
    if (prim_call_setup(la, lb, lc, ld, 0, &dummy, &dummy, &dummy, HGP_FP64, &c)) return -1;
    const ClassKernels &k = g_class_table[c.ci];
    if (k.tier != 0 && k.tier != 1) return -1;
    int64_t lo = 0, hi = (int64_t)(NOALLOC_BYTES / 64);
    while (lo < hi) {                       // largest n whose records fit
        const int64_t mid = (lo + hi + 1) / 2;
        if (noalloc_need(k, mid) <= NOALLOC_BYTES) lo = mid; else hi = mid - 1;
    }
    return lo;
}

hgp_status hgp_eri_prim_quartets_noalloc(int32_t la, int32_t lb, int32_t lc, int32_t ld, int64_t n,
                                         const double *centers, const double *exps, double *out, int32_t precision,
                                         void *hip_stream)
{
    PrimCall c;
    if (hgp_status st = prim_call_setup(la, lb, lc, ld, n, centers, exps, out, precision, &c)) return st;
    const ClassKernels &k = g_class_table[c.ci];
    if (k.tier != 0 && k.tier != 1)
        return fail(HGP_E_UNSUPPORTED_L, "this class runs on an op-table tier, whose tables are uploaded to the "
                                         "device on first use; use hgp_eri_prim_quartets");
    const size_t need = noalloc_need(k, n);
    if (need > NOALLOC_BYTES)
        return fail(HGP_E_INVALID, "n = " + std::to_string(n) + " needs " + std::to_string(need) +
                                       " bytes of the fixed buffer (" + std::to_string(NOALLOC_BYTES) +
                                       "); at most " + std::to_string(hgp_eri_prim_quartets_noalloc_max(la, lb, lc, ld)) +
                                       " quartets of this class per call");
    if (n == 0) return HGP_OK;
    int dev = 0;
    HGP_HIP(hipGetDevice(&dev));
    const double *boys = nullptr;
    if (hgp_status st = boys_table(dev, &boys)) return st;
    unsigned char *base = nullptr;
    if (hgp_status st = noalloc_scratch(dev, &base)) return st;
    size_t off = 0;
    auto carve = [&](size_t bytes) { unsigned char *p = base + off; off += align256(bytes); return p; };
    PairInfo *d_pairs = (PairInfo *)carve(sizeof(PairInfo) * 2 * n);
    PairGeo *d_geo = (PairGeo *)carve(sizeof(PairGeo) * 2 * n);
    PrimPair *d_prims = (PrimPair *)carve(sizeof(PrimPair) * 2 * n);
    EriTask *d_tasks = (EriTask *)carve(sizeof(EriTask) * n);
    double *d_scr = nullptr;
    int64_t scr_doubles = 0;
    if (k.tier == 1) {
        d_scr = (double *)(base + off);
        scr_doubles = std::min((int64_t)((NOALLOC_BYTES - off) / sizeof(double)), staged_need(k, n));
    }
    prim_call_run(c, n, centers, exps, out, boys, d_pairs, d_geo, d_prims, d_tasks, d_scr, scr_doubles,
                  (hipStream_t)hip_stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(HGP_E_DEVICE, std::string("microbench launch: ") + hipGetErrorString(e));
    return HGP_OK;
}

struct hgp_batch {
    int device = 0;
    hipStream_t origin = nullptr;                 // the capture's origin stream
    std::vector<hipStream_t> branches;
    std::vector<hipEvent_t> events;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

hgp_status hgp_batch_destroy(hgp_batch *b)
{
    if (!b) return HGP_OK;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
    for (hipStream_t st : b->branches) (void)hipStreamDestroy(st);
    if (b->origin) (void)hipStreamDestroy(b->origin);
    delete b;
    return HGP_OK;
}

hgp_status hgp_batch_create(hgp_plan *const *plans, int32_t n, const double *const *D, double *const *J,
                            double *const *K, hgp_batch **out)
{
    if (!out) return fail(HGP_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n < 1 || !plans || !D || !J || !K) return fail(HGP_E_INVALID, "need n >= 1 and the plans, D, J, K arrays");
    int dev = 0;
    HGP_HIP(hipGetDevice(&dev));
    std::vector<std::pair<double, int>> cost((size_t)n);
    for (int i = 0; i < n; ++i) {
        const hgp_plan *p = plans[i];
        if (!p) return fail(HGP_E_INVALID, "a plan is NULL");
        if (p->broken) return fail(HGP_E_STATE, "a plan is unusable after an earlier device failure");
        if (p->timing) return fail(HGP_E_INVALID, "kernel timing must be off for plans in a batch");
        if (p->device != dev) return fail(HGP_E_INVALID, "all plans of a batch must be on the current device");
        for (int j = 0; j < i; ++j)
            if (plans[j] == p) return fail(HGP_E_INVALID, "a plan appears twice in the batch");
        if (p->b->nbf > 0 && (!D[i] || (!J[i] && !K[i]))) return fail(HGP_E_INVALID, "a system has no D or no output");
        double c = 0.0;                           // work estimate: VRR + Phase-2 FLOPs of its lists
        for (const ClassList &cl : p->lists)
            c += cl.nprimq * g_class_table[cl.cls].vrr_flops + cl.nq * g_class_table[cl.cls].p2_flops;
        cost[i] = {c, i};
    }
    const double *boys = nullptr;                  // the table is built (and allocated) outside the capture
    if (hgp_status bst = boys_table(dev, &boys)) return bst;
    auto *b = new hgp_batch();
    b->device = dev;
    const int nbranch = std::min(n, 8);
    auto bail = [&](hgp_status st) { hgp_batch_destroy(b); return st; };
    if (hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(HGP_E_DEVICE, "creating the capture stream failed"));
    hipStream_t s = b->origin;
    for (int k = 0; k < nbranch; ++k) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(HGP_E_DEVICE, "creating a branch stream failed"));
        b->branches.push_back(st);
    }
    for (int k = 0; k <= nbranch; ++k) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return bail(fail(HGP_E_DEVICE, "creating a branch event failed"));
        b->events.push_back(e);
    }
    // largest systems first, each to the branch with the least work so far
    std::sort(cost.begin(), cost.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
    std::vector<double> load((size_t)nbranch, 0.0);
    std::vector<int> branch_of((size_t)n, 0);
    for (const auto &ci : cost) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        branch_of[(size_t)ci.second] = k;
        load[(size_t)k] += ci.first + 1.0;
    }
    if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess)
        return bail(fail(HGP_E_DEVICE, "hipStreamBeginCapture failed"));
    hgp_status st = HGP_OK;
    hipError_t e = hipEventRecord(b->events[0], s);
    for (int k = 0; k < nbranch && e == hipSuccess; ++k) e = hipStreamWaitEvent(b->branches[k], b->events[0], 0);
    for (const auto &ci : cost) {
        if (e != hipSuccess || st != HGP_OK) break;
        const int i = ci.second;
        st = hgp_jk(plans[i], D[i], J[i], K[i], b->branches[(size_t)branch_of[(size_t)i]]);
    }
    for (int k = 0; k < nbranch && e == hipSuccess; ++k) {
        e = hipEventRecord(b->events[k + 1], b->branches[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, b->events[k + 1], 0);
    }
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &g);
    b->graph = g;
    if (st != HGP_OK) return bail(st);
    if (e != hipSuccess || ec != hipSuccess)
        return bail(fail(HGP_E_DEVICE, std::string("capturing the batch failed: ") + hipGetErrorString(e != hipSuccess ? e : ec)));
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
        return bail(fail(HGP_E_DEVICE, "hipGraphInstantiate failed"));
    *out = b;
    return HGP_OK;
}

hgp_status hgp_batch_run(hgp_batch *b, void *hip_stream)
{
    if (!b || !b->exec) return fail(HGP_E_INVALID, "batch is NULL");
    const hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(HGP_E_DEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    return HGP_OK;
}

}  // extern "C"
