/*
 * CPU oracle for contracted electron-repulsion integrals and Coulomb/exchange
 * matrices.  TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
 * benchmark's CPU-baseline leg are its only callers; the HIP library never
 * links or calls it, and it shares no code, header or table with that library.
 *
 * It computes, plainly and slowly, what the HGP method reaches up to rounding:
 *   - the integral definition (Sec. II-A, Eq. eri-def) over contracted,
 *     normalised Cartesian Gaussian shells, transformed to pure spherical
 *     functions (Sec. III-B, Eq. cart2sph);
 *   - by the Obara-Saika vertical recurrence (Eq. vrr; the ket form is its
 *     mirror image) with a fixed x->y->z, bra-then-ket axis order, contraction
 *     over primitives, then the horizontal recurrence (Eq. hrr and its ket
 *     mirror) fully in the Cartesian basis, and only then the four shell
 *     transformations (materialise-then-transform, Eq. materialize-sph);
 *   - J_mn = sum_ls (mn|ls) D_ls and K_mn = sum_ls (ml|ns) D_ls, from the
 *     unique shell quartets by adding every distinct index image once
 *     (the 8-fold permutational symmetry, Sec. III-C.2 and Sec. IV).
 *
 * Conventions the paper leaves open (Sec. III-B cites the standard shell
 * transformation without printing it):
 *   - primitives x^i y^j z^k exp(-a r^2) all carry N(a,l), the factor that
 *     normalises x^l exp(-a r^2); contraction coefficients are rescaled so
 *     that the x^l component of the contracted shell has unit norm;
 *   - Cartesian order within a shell: x power descending, then y descending;
 *   - s and p shells are kept as is (p in x, y, z order); l >= 2 shells use
 *     real solid harmonics ordered m = -l .. l, no Condon-Shortley phase
 *     (leading monomial coefficient positive), each unit-normalised;
 *   - Boys function: F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt.
 *
 * Built twice: as double (symbols oracle_*) and as long double with
 * -DORACLE_LD (symbols oracle_ld_*), so the oracle's own rounding error can be
 * estimated.  All entry points take and return double arrays and return 0 on
 * success, -1 on invalid arguments, -2 for l > 4, -3 when out of memory.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef ORACLE_LD
typedef long double real;
#define EXP expl
#define SQRT sqrtl
#define ERF erfl
#define FABS fabsl
#define POW powl
#define PFX(n) oracle_ld_##n
#define SERIES_EPS 1e-22L
#else
typedef double real;
#define EXP exp
#define SQRT sqrt
#define ERF erf
#define FABS fabs
#define POW pow
#define PFX(n) oracle_##n
#define SERIES_EPS 1e-18
#endif

#define PI_R ((real)3.14159265358979323846264338327950288L)
#define LMAX 4                 /* highest shell angular momentum accepted   */
#define LINT (LMAX + 1)        /* highest l evaluated inside (first derivatives raise one shell by one) */
#define NMAX (2 * LINT)        /* highest |e| in a pair, la + lb            */
#define NGMAX 286              /* monomials of degree <= NMAX: ncum(NMAX+1) */

/* ------------------------------------------------------------------ */
/* Cartesian bookkeeping                                               */
/* ------------------------------------------------------------------ */

static int ncart(int l) { return (l + 1) * (l + 2) / 2; }
static int nsph(int l) { return 2 * l + 1; }
/* number of Cartesian monomials of total degree < n */
static int ncum(int n) { return n * (n + 1) * (n + 2) / 6; }
/* position of (x,y,z) inside its own shell (x descending, then y descending) */
static int cidx(int y, int z) { int jk = y + z; return jk * (jk + 1) / 2 + z; }
/* position of (x,y,z) among all monomials of degree <= NMAX, degree-major */
static int gidx(int x, int y, int z) { return ncum(x + y + z) + cidx(y, z); }

/* component table: monomial g has exponents CMP[g][0..2] */
static int CMP[NGMAX][3];
static void init_tables(void)
{
    int g = 0;
    for (int n = 0; n <= NMAX; ++n)
        for (int x = n; x >= 0; --x)
            for (int y = n - x; y >= 0; --y) {
                CMP[g][0] = x; CMP[g][1] = y; CMP[g][2] = n - x - y;
                ++g;
            }
}
static int deg(int g) { return CMP[g][0] + CMP[g][1] + CMP[g][2]; }
/* first axis (x, then y, then z) with a nonzero exponent */
static int first_axis(int g) { return CMP[g][0] ? 0 : (CMP[g][1] ? 1 : 2); }
static int shift(int g, int axis, int by)
{
    int c[3] = {CMP[g][0], CMP[g][1], CMP[g][2]};
    c[axis] += by;
    if (c[axis] < 0) return -1;
    return gidx(c[0], c[1], c[2]);
}

static real dfact(int n) /* n!! with (-1)!! = 1 */
{
    real r = 1;
    for (int k = n; k > 1; k -= 2) r *= (real)k;
    return r;
}
static real binom(int n, int k)
{
    if (k < 0 || k > n) return 0;
    real r = 1;
    for (int i = 1; i <= k; ++i) r = r * (real)(n - k + i) / (real)i;
    return r;
}

/* ------------------------------------------------------------------ */
/* Boys function F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt                */
/* ------------------------------------------------------------------ */

/* F[0..mmax].  T = 0: 1/(2m+1) exactly.  T < 40: the series
 * F_m = exp(-T) sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1)) for the top order,
 * then the downward recurrence F_m = (2T F_{m+1} + exp(-T)) / (2m+1).
 * T >= 40: F_0 = sqrt(pi/T) erf(sqrt T) / 2 and the upward recurrence
 * F_{m+1} = ((2m+1) F_m - exp(-T)) / (2T), stable there for m <= 20. */
static void boys(int mmax, real T, real *F)
{
    if (T == 0) {
        for (int m = 0; m <= mmax; ++m) F[m] = (real)1 / (real)(2 * m + 1);
        return;
    }
    real e = EXP(-T);
    if (T < 40) {
        real term = (real)1 / (real)(2 * mmax + 1), sum = term;
        for (int k = 1; k < 100000; ++k) {
            term *= 2 * T / (real)(2 * mmax + 2 * k + 1);
            sum += term;
            if (term < sum * SERIES_EPS) break;
        }
        F[mmax] = e * sum;
        for (int m = mmax - 1; m >= 0; --m) F[m] = (2 * T * F[m + 1] + e) / (real)(2 * m + 1);
    } else {
        F[0] = SQRT(PI_R / T) * ERF(SQRT(T)) / 2;
        for (int m = 0; m < mmax; ++m) F[m + 1] = ((real)(2 * m + 1) * F[m] - e) / (2 * T);
    }
}

/* ------------------------------------------------------------------ */
/* Normalisation and the Cartesian -> pure spherical matrices          */
/* ------------------------------------------------------------------ */

/* N(a,l) normalises x^l exp(-a r^2) */
static real prim_norm(real a, int l)
{
    return POW(2 * a / PI_R, (real)0.75) * POW(4 * a, (real)l / 2) / SQRT(dfact(2 * l - 1));
}

/* c_k = d_k N(a_k,l) / sqrt(sum_kk' d_k d_k' [2 sqrt(a_k a_k')/(a_k+a_k')]^(l+3/2)) */
static void norm_coefs(int l, int np, const double *a, const double *d, real *out)
{
    real s = 0;
    for (int k = 0; k < np; ++k)
        for (int q = 0; q < np; ++q) {
            real ak = a[k], aq = a[q];
            s += (real)d[k] * (real)d[q] * POW(2 * SQRT(ak * aq) / (ak + aq), (real)l + (real)1.5);
        }
    real sc = 1 / SQRT(s);
    for (int k = 0; k < np; ++k) out[k] = (real)d[k] * prim_norm(a[k], l) * sc;
}

/* <c|c'> between two monomials of one shell, both carrying N(a,l):
 * prod_axes (p+p'-1)!! / (2l-1)!!, zero unless every exponent sum is even. */
static real cart_metric(int l, const int *c1, const int *c2)
{
    real r = 1;
    for (int ax = 0; ax < 3; ++ax) {
        int s = c1[ax] + c2[ax];
        if (s & 1) return 0;
        r *= dfact(s - 1);
    }
    return r / dfact(2 * l - 1);
}

/* T^(l): (2l+1) x ncart(l), row-major.  s, p: identity.  l >= 2: real solid
 * harmonics from the closed form (Helgaker, Jorgensen & Olsen, Molecular
 * Electronic-Structure Theory, Eqs. 6.4.47-50), rows then unit-normalised
 * in the metric above. */
static void sph_matrix(int l, real *t)
{
    int nc = ncart(l), ns = nsph(l);
    memset(t, 0, sizeof(real) * (size_t)nc * (size_t)ns);
    if (l <= 1) {
        for (int i = 0; i < nc; ++i) t[i * nc + i] = 1;
        return;
    }
    for (int row = 0; row < ns; ++row) {
        int m = row - l, am = m < 0 ? -m : m, km = m < 0 ? 1 : 0;
        real *r = t + row * nc;
        for (int tt = 0; tt <= (l - am) / 2; ++tt)
            for (int u = 0; u <= tt; ++u)
                for (int k = km; k <= am; k += 2) {          /* k = 2v */
                    int sgn = ((tt + (k - km) / 2) & 1) ? -1 : 1;
                    real c = sgn * POW((real)0.25, (real)tt) * binom(l, tt) * binom(l - tt, am + tt) *
                             binom(tt, u) * binom(am, k);
                    int py = 2 * u + k, pz = l - 2 * tt - am;   /* x power: l - py - pz */
                    r[cidx(py, pz)] += c;
                }
        /* unit norm */
        int cs[64][3], n = 0;
        for (int x = l; x >= 0; --x)
            for (int y = l - x; y >= 0; --y) { cs[n][0] = x; cs[n][1] = y; cs[n][2] = l - x - y; ++n; }
        real nn = 0;
        for (int i = 0; i < nc; ++i)
            for (int j = 0; j < nc; ++j) nn += r[i] * r[j] * cart_metric(l, cs[i], cs[j]);
        real sc = 1 / SQRT(nn);
        for (int i = 0; i < nc; ++i) r[i] *= sc;
    }
}

/* ------------------------------------------------------------------ */
/* One contracted shell quartet                                        */
/* ------------------------------------------------------------------ */

typedef struct {
    int nshell, nbf;
    const int *l, *nprim;
    const double *cen, *exps;
    int *poff, *foff;
    real *c;                 /* normalised contraction coefficients */
} basis_t;

static int basis_make(basis_t *b, int nshell, const int *l, const int *nprim, const double *cen,
                      const double *exps, const double *coefs)
{
    init_tables();
    memset(b, 0, sizeof(*b));
    if (nshell < 0) return -1;
    b->nshell = nshell; b->l = l; b->nprim = nprim; b->cen = cen; b->exps = exps;
    b->poff = malloc(sizeof(int) * (size_t)(nshell + 1));
    b->foff = malloc(sizeof(int) * (size_t)(nshell + 1));
    if (!b->poff || !b->foff) return -3;
    b->poff[0] = 0; b->foff[0] = 0;
    for (int s = 0; s < nshell; ++s) {
        if (l[s] < 0 || nprim[s] <= 0) return -1;
        if (l[s] > LMAX) return -2;
        b->poff[s + 1] = b->poff[s] + nprim[s];
        b->foff[s + 1] = b->foff[s] + nsph(l[s]);
    }
    b->nbf = b->foff[nshell];
    b->c = malloc(sizeof(real) * (size_t)(b->poff[nshell] + 1));
    if (!b->c) return -3;
    for (int s = 0; s < nshell; ++s) {
        for (int k = 0; k < nprim[s]; ++k)
            if (!(exps[b->poff[s] + k] > 0) || !isfinite(coefs[b->poff[s] + k])) return -1;
        norm_coefs(l[s], nprim[s], exps + b->poff[s], coefs + b->poff[s], b->c + b->poff[s]);
    }
    return 0;
}
static void basis_free(basis_t *b) { free(b->poff); free(b->foff); free(b->c); }

/* per-thread work arrays, sized for the quartet at hand */
typedef struct {
    real *V, *H, *X, *B, *Y, *C, *S1, *S2;
    size_t nV, nH, nX, nB, nY, nC, nS1, nS2;
} work_t;

static int grow(real **p, size_t *have, size_t need)
{
    if (*have >= need) return 0;
    real *q = realloc(*p, sizeof(real) * need);
    if (!q) return -3;
    *p = q; *have = need;
    return 0;
}
static void work_free(work_t *w)
{
    free(w->V); free(w->H); free(w->X); free(w->B); free(w->Y); free(w->C); free(w->S1); free(w->S2);
    memset(w, 0, sizeof(*w));
}

/* Cartesian contracted block (ab|cd), [ncart(la)][ncart(lb)][ncart(lc)][ncart(ld)].
 * Primitive data: exponents ea[na] with coefficients ca[na], and so on. */
static int quartet_cart(work_t *w, const int L4[4], const double *cen4[4], const double *e4[4],
                        const real *c4[4], const int n4[4], real *out)
{
    int la = L4[0], lb = L4[1], lc = L4[2], ld = L4[3];
    int Lab = la + lb, Lcd = lc + ld, L = Lab + Lcd;
    int NE = ncum(Lab + 1), NF = ncum(Lcd + 1);
    real A[3], B[3], C[3], D[3], AB[3], CD[3];
    for (int i = 0; i < 3; ++i) {
        A[i] = cen4[0][i]; B[i] = cen4[1][i]; C[i] = cen4[2][i]; D[i] = cen4[3][i];
        AB[i] = A[i] - B[i]; CD[i] = C[i] - D[i];
    }
    real AB2 = AB[0] * AB[0] + AB[1] * AB[1] + AB[2] * AB[2];
    real CD2 = CD[0] * CD[0] + CD[1] * CD[1] + CD[2] * CD[2];
    if (grow(&w->V, &w->nV, (size_t)(L + 1) * NE * NF) || grow(&w->H, &w->nH, (size_t)NE * NF)) return -3;
    real *V = w->V, *H = w->H;
    memset(H, 0, sizeof(real) * (size_t)NE * NF);
#define VV(m, e, f) V[((size_t)(m) * NE + (e)) * NF + (f)]
    real F[4 * LINT + 2];

    /* ---- Phase 1: primitive loops, OS vertical recurrence, contraction ---- */
    for (int pa = 0; pa < n4[0]; ++pa)
    for (int pb = 0; pb < n4[1]; ++pb)
    for (int pc = 0; pc < n4[2]; ++pc)
    for (int pd = 0; pd < n4[3]; ++pd) {
        real a = e4[0][pa], b = e4[1][pb], c = e4[2][pc], d = e4[3][pd];
        real zeta = a + b, eta = c + d, ze = zeta + eta, rho = zeta * eta / ze;
        real P[3], Q[3], W[3], PA[3], WP[3], QC[3], WQ[3];
        real PQ2 = 0;
        for (int i = 0; i < 3; ++i) {
            P[i] = (a * A[i] + b * B[i]) / zeta;
            Q[i] = (c * C[i] + d * D[i]) / eta;
            W[i] = (zeta * P[i] + eta * Q[i]) / ze;
            PA[i] = P[i] - A[i]; WP[i] = W[i] - P[i]; QC[i] = Q[i] - C[i]; WQ[i] = W[i] - Q[i];
            PQ2 += (P[i] - Q[i]) * (P[i] - Q[i]);
        }
        real T = rho * PQ2;
        real pref = 2 * POW(PI_R, (real)2.5) / (zeta * eta * SQRT(ze)) * EXP(-a * b / zeta * AB2) *
                    EXP(-c * d / eta * CD2) * c4[0][pa] * c4[1][pb] * c4[2][pc] * c4[3][pd];
        boys(L, T, F);
        for (int m = 0; m <= L; ++m) VV(m, 0, 0) = pref * F[m];
        real o2z = 1 / (2 * zeta), o2e = 1 / (2 * eta), o2ze = 1 / (2 * ze), rz = rho / zeta, re = rho / eta;
        /* bra build: [e+1_i 0|0 0]^(m) */
        for (int g = 1; g < NE; ++g) {
            int n = deg(g), i = first_axis(g), e1 = shift(g, i, -1), e2 = shift(g, i, -2);
            int ei = CMP[g][i];
            for (int m = 0; m <= L - n; ++m) {
                real v = PA[i] * VV(m, e1, 0) + WP[i] * VV(m + 1, e1, 0);
                if (ei >= 2) v += (real)(ei - 1) * o2z * (VV(m, e2, 0) - rz * VV(m + 1, e2, 0));
                VV(m, g, 0) = v;
            }
        }
        /* ket build: [e 0|f+1_i 0]^(m) */
        for (int h = 1; h < NF; ++h) {
            int nf = deg(h), i = first_axis(h), f1 = shift(h, i, -1), f2 = shift(h, i, -2);
            int fi = CMP[h][i];
            for (int g = 0; g < NE; ++g) {
                int ne = deg(g), ei = CMP[g][i], em = ei ? shift(g, i, -1) : -1;
                for (int m = 0; m <= L - ne - nf; ++m) {
                    real v = QC[i] * VV(m, g, f1) + WQ[i] * VV(m + 1, g, f1);
                    if (fi >= 2) v += (real)(fi - 1) * o2e * (VV(m, g, f2) - re * VV(m + 1, g, f2));
                    if (ei >= 1) v += (real)ei * o2ze * VV(m + 1, em, f1);
                    VV(m, g, h) = v;
                }
            }
        }
        /* contraction: H[e][f] += [e0|f0]^(0) for la<=|e|<=Lab, lc<=|f|<=Lcd */
        for (int g = ncum(la); g < NE; ++g)
            for (int h = ncum(lc); h < NF; ++h) H[(size_t)g * NF + h] += VV(0, g, h);
    }
#undef VV

    /* ---- Phase 2: bra HRR (ab+1_i| = (a+1_i b| + AB_i (ab| ---- */
    int NB = ncum(lb + 1);
    if (grow(&w->X, &w->nX, (size_t)NE * NB * NF)) return -3;
    real *X = w->X;
#define XX(a, b, f) X[((size_t)(a) * NB + (b)) * NF + (f)]
    for (int g = ncum(la); g < NE; ++g)
        for (int h = ncum(lc); h < NF; ++h) XX(g, 0, h) = H[(size_t)g * NF + h];
    for (int gb = 1; gb < NB; ++gb) {
        int k = deg(gb), i = first_axis(gb), b1 = shift(gb, i, -1);
        for (int g = ncum(la); g < ncum(Lab - k + 1); ++g) {
            int a1 = shift(g, i, +1);
            for (int h = ncum(lc); h < NF; ++h) XX(g, gb, h) = XX(a1, b1, h) + AB[i] * XX(g, b1, h);
        }
    }
    /* ket HRR (ab|c d+1_i) = (ab|c+1_i d) + CD_i (ab|cd), per final (a,b) */
    int nca = ncart(la), ncb = ncart(lb), ncc = ncart(lc), ncd = ncart(ld), ND = ncum(ld + 1);
    if (grow(&w->Y, &w->nY, (size_t)NF * ND)) return -3;
    real *Y = w->Y;
#define YY(c, d) Y[(size_t)(c) * ND + (d)]
    for (int ia = 0; ia < nca; ++ia)
        for (int ib = 0; ib < ncb; ++ib) {
            int ga = ncum(la) + ia, gb = ncum(lb) + ib;
            for (int h = ncum(lc); h < NF; ++h) YY(h, 0) = XX(ga, gb, h);
            for (int gd = 1; gd < ND; ++gd) {
                int k = deg(gd), i = first_axis(gd), d1 = shift(gd, i, -1);
                for (int h = ncum(lc); h < ncum(Lcd - k + 1); ++h) {
                    int c1 = shift(h, i, +1);
                    YY(h, gd) = YY(c1, d1) + CD[i] * YY(h, d1);
                }
            }
            for (int ic = 0; ic < ncc; ++ic)
                for (int id = 0; id < ncd; ++id)
                    out[((size_t)(ia * ncb + ib) * ncc + ic) * ncd + id] = YY(ncum(lc) + ic, ncum(ld) + id);
        }
#undef XX
#undef YY
    return 0;
}

/* apply T^(l) to one index of a 4-index tensor: dims n[4] -> n'[4] */
static void transform_index(const real *in, real *out, const int n[4], int which, int l)
{
    real t[9 * 15];
    sph_matrix(l, t);
    int ns = nsph(l), nc = n[which];
    int pre = 1, post = 1;
    for (int k = 0; k < which; ++k) pre *= n[k];
    for (int k = which + 1; k < 4; ++k) post *= n[k];
    for (int p = 0; p < pre; ++p)
        for (int s = 0; s < ns; ++s)
            for (int q = 0; q < post; ++q) {
                real acc = 0;
                for (int c = 0; c < nc; ++c) acc += t[s * nc + c] * in[((size_t)p * nc + c) * post + q];
                out[((size_t)p * ns + s) * post + q] = acc;
            }
}

/* spherical block of shells (i j|k l) of basis b */
static int quartet_sph(work_t *w, const basis_t *b, int i, int j, int k, int l, real *out)
{
    int sh[4] = {i, j, k, l}, L4[4], n4[4];
    const double *cen4[4], *e4[4];
    const real *c4[4];
    for (int q = 0; q < 4; ++q) {
        L4[q] = b->l[sh[q]]; n4[q] = b->nprim[sh[q]];
        cen4[q] = b->cen + 3 * sh[q]; e4[q] = b->exps + b->poff[sh[q]]; c4[q] = b->c + b->poff[sh[q]];
    }
    size_t ncc = (size_t)ncart(L4[0]) * ncart(L4[1]) * ncart(L4[2]) * ncart(L4[3]);
    if (grow(&w->C, &w->nC, ncc) || grow(&w->S1, &w->nS1, ncc) || grow(&w->S2, &w->nS2, ncc)) return -3;
    int rc = quartet_cart(w, L4, cen4, e4, c4, n4, w->C);
    if (rc) return rc;
    /* materialise-then-transform: T(la) x T(lb) x T(lc) x T(ld) on the Cartesian block */
    int n[4] = {ncart(L4[0]), ncart(L4[1]), ncart(L4[2]), ncart(L4[3])};
    real *src = w->C, *dst = w->S1;
    for (int q = 0; q < 4; ++q) {
        transform_index(src, dst, n, q, L4[q]);
        n[q] = nsph(L4[q]);
        src = dst;
        dst = (dst == w->S1) ? w->S2 : w->S1;
    }
    memcpy(out, src, sizeof(real) * (size_t)n[0] * n[1] * n[2] * n[3]);
    return 0;
}

/* First derivatives of the spherical block (i j|k l) with respect to the
 * centre coordinates of each of its four shells.  Differentiating a Cartesian
 * primitive (x - A_x)^a_x ... exp(-alpha |r - A|^2) with respect to A_t gives
 * 2 alpha times the primitive with a + 1_t minus a_t times the primitive with
 * a - 1_t, so for the contracted shell (coefficients c_k, exponents alpha_k)
 *   d/dA_t (a b|c d) = (a+1_t b|c d)_w - a_t (a-1_t b|c d),
 * where the subscript w marks the contraction of that shell with weights
 * 2 alpha_k c_k; likewise for the other three centres.  Each Cartesian
 * derivative block is then transformed to spherical functions (materialise
 * then transform).  out: [4 centres][3 axes][nsph(li)][nsph(lj)][nsph(lk)][nsph(ll)]. */
static int quartet_deriv_sph(work_t *w, const basis_t *b, int i, int j, int k, int l, real *out)
{
    int sh[4] = {i, j, k, l}, L4[4], n4[4];
    const double *cen4[4], *e4[4];
    const real *c4[4];
    for (int q = 0; q < 4; ++q) {
        L4[q] = b->l[sh[q]]; n4[q] = b->nprim[sh[q]];
        cen4[q] = b->cen + 3 * sh[q]; e4[q] = b->exps + b->poff[sh[q]]; c4[q] = b->c + b->poff[sh[q]];
    }
    int nc[4], ns[4];
    size_t ncc = 1, nss = 1;
    for (int q = 0; q < 4; ++q) { nc[q] = ncart(L4[q]); ns[q] = nsph(L4[q]); ncc *= nc[q]; nss *= ns[q]; }
    if (grow(&w->C, &w->nC, ncc) || grow(&w->S1, &w->nS1, ncc) || grow(&w->S2, &w->nS2, ncc)) return -3;
    int rc = 0;
    for (int r = 0; r < 4 && !rc; ++r) {
        int Lp[4], Lm[4], np_[4], nm_[4];
        size_t sp = 1, sm = 1;
        for (int q = 0; q < 4; ++q) { Lp[q] = Lm[q] = L4[q]; }
        Lp[r] += 1; Lm[r] -= 1;
        for (int q = 0; q < 4; ++q) { np_[q] = ncart(Lp[q]); sp *= np_[q]; nm_[q] = Lm[r] >= 0 ? ncart(Lm[q]) : 0; }
        if (Lm[r] >= 0) for (int q = 0; q < 4; ++q) sm *= nm_[q]; else sm = 0;
        real *cw = malloc(sizeof(real) * (size_t)n4[r]);
        real *Xp = malloc(sizeof(real) * sp);
        real *Xm = sm ? malloc(sizeof(real) * sm) : NULL;
        if (!cw || !Xp || (sm && !Xm)) rc = -3;
        if (!rc) {
            for (int kk = 0; kk < n4[r]; ++kk) cw[kk] = 2 * (real)e4[r][kk] * c4[r][kk];
            const real *c4p[4] = {c4[0], c4[1], c4[2], c4[3]};
            c4p[r] = cw;
            rc = quartet_cart(w, Lp, cen4, e4, c4p, n4, Xp);
            if (!rc && sm) rc = quartet_cart(w, Lm, cen4, e4, c4, n4, Xm);
        }
        for (int t = 0; t < 3 && !rc; ++t) {
            /* Cartesian derivative block along axis t of centre r */
            real *Dc = w->C;
            int q4[4];
            for (q4[0] = 0; q4[0] < nc[0]; ++q4[0])
            for (q4[1] = 0; q4[1] < nc[1]; ++q4[1])
            for (q4[2] = 0; q4[2] < nc[2]; ++q4[2])
            for (q4[3] = 0; q4[3] < nc[3]; ++q4[3]) {
                /* exponents of shell r's component q4[r] (x descending, then y descending) */
                int cnt = 0, ex[3] = {0, 0, 0};
                for (int x = L4[r]; x >= 0 && cnt <= q4[r]; --x)
                    for (int y = L4[r] - x; y >= 0; --y, ++cnt)
                        if (cnt == q4[r]) { ex[0] = x; ex[1] = y; ex[2] = L4[r] - x - y; }
                int up[3] = {ex[0], ex[1], ex[2]};
                up[t] += 1;
                int pidx[4] = {q4[0], q4[1], q4[2], q4[3]};
                pidx[r] = cidx(up[1], up[2]);
                size_t op = (((size_t)pidx[0] * np_[1] + pidx[1]) * np_[2] + pidx[2]) * np_[3] + pidx[3];
                real v = Xp[op];
                if (ex[t] > 0) {
                    int dn[3] = {ex[0], ex[1], ex[2]};
                    dn[t] -= 1;
                    int midx[4] = {q4[0], q4[1], q4[2], q4[3]};
                    midx[r] = cidx(dn[1], dn[2]);
                    size_t om = (((size_t)midx[0] * nm_[1] + midx[1]) * nm_[2] + midx[2]) * nm_[3] + midx[3];
                    v -= (real)ex[t] * Xm[om];
                }
                Dc[(((size_t)q4[0] * nc[1] + q4[1]) * nc[2] + q4[2]) * nc[3] + q4[3]] = v;
            }
            int n[4] = {nc[0], nc[1], nc[2], nc[3]};
            real *src = w->C, *dst = w->S1;
            for (int q = 0; q < 4; ++q) {
                transform_index(src, dst, n, q, L4[q]);
                n[q] = ns[q];
                src = dst;
                dst = (dst == w->S1) ? w->S2 : w->S1;
            }
            memcpy(out + (size_t)(r * 3 + t) * nss, src, sizeof(real) * nss);
        }
        free(cw); free(Xp); free(Xm);
    }
    return rc;
}

/* ------------------------------------------------------------------ */
/* Exported entry points                                               */
/* ------------------------------------------------------------------ */

int PFX(boys)(int mmax, double T, double *F)
{
    if (mmax < 0 || mmax > 40 || !(T >= 0)) return -1;
    real f[41];
    boys(mmax, (real)T, f);
    for (int m = 0; m <= mmax; ++m) F[m] = (double)f[m];
    return 0;
}

int PFX(sph_matrix)(int l, double *t)
{
    if (l < 0) return -1;
    if (l > LMAX) return -2;
    real r[9 * 15];
    sph_matrix(l, r);
    for (int i = 0; i < nsph(l) * ncart(l); ++i) t[i] = (double)r[i];
    return 0;
}

int PFX(norm_coefs)(int l, int np, const double *exps, const double *coefs, double *out)
{
    if (l < 0 || np <= 0) return -1;
    if (l > LMAX) return -2;
    real r[64];
    if (np > 64) return -1;
    norm_coefs(l, np, exps, coefs, r);
    for (int k = 0; k < np; ++k) out[k] = (double)r[k];
    return 0;
}

/* unnormalised primitive Cartesian block: unit coefficients, no N(a,l) */
int PFX(prim_cart_eri)(int la, int lb, int lc, int ld, const double *centers /*12*/,
                       const double *alpha /*4*/, double *out)
{
    int L4[4] = {la, lb, lc, ld}, n4[4] = {1, 1, 1, 1};
    for (int q = 0; q < 4; ++q) {
        if (L4[q] < 0) return -1;
        if (L4[q] > LMAX) return -2;
    }
    init_tables();
    const double *cen4[4] = {centers, centers + 3, centers + 6, centers + 9};
    const double *e4[4] = {alpha, alpha + 1, alpha + 2, alpha + 3};
    real one = 1;
    const real *c4[4] = {&one, &one, &one, &one};
    work_t w; memset(&w, 0, sizeof(w));
    size_t n = (size_t)ncart(la) * ncart(lb) * ncart(lc) * ncart(ld);
    real *tmp = malloc(sizeof(real) * n);
    if (!tmp) return -3;
    int rc = quartet_cart(&w, L4, cen4, e4, c4, n4, tmp);
    for (size_t i = 0; i < n && !rc; ++i) out[i] = (double)tmp[i];
    free(tmp);
    work_free(&w);
    return rc;
}

/* contracted spherical block of shells (i j|k l) in any order */
int PFX(eri_shell_quartet)(int nshell, const int *l, const int *nprim, const double *centers,
                           const double *exps, const double *coefs, int i, int j, int k, int ll,
                           double *out)
{
    basis_t b;
    int rc = basis_make(&b, nshell, l, nprim, centers, exps, coefs);
    if (!rc && (i < 0 || j < 0 || k < 0 || ll < 0 || i >= nshell || j >= nshell || k >= nshell || ll >= nshell))
        rc = -1;
    if (rc) { basis_free(&b); return rc; }
    size_t n = (size_t)nsph(l[i]) * nsph(l[j]) * nsph(l[k]) * nsph(l[ll]);
    real *tmp = malloc(sizeof(real) * n);
    work_t w; memset(&w, 0, sizeof(w));
    rc = tmp ? quartet_sph(&w, &b, i, j, k, ll, tmp) : -3;
    for (size_t q = 0; q < n && !rc; ++q) out[q] = (double)tmp[q];
    free(tmp); work_free(&w); basis_free(&b);
    return rc;
}

/* First derivatives of the contracted spherical block of shells (i j|k l)
 * with respect to the centre of each shell: out[4][3][ni][nj][nk][nl]
 * (centre of shell i, j, k, l; axis x, y, z), bohr^-1 hartree. */
int PFX(eri_deriv_shell_quartet)(int nshell, const int *l, const int *nprim, const double *centers,
                                 const double *exps, const double *coefs, int i, int j, int k, int ll,
                                 double *out)
{
    basis_t b;
    int rc = basis_make(&b, nshell, l, nprim, centers, exps, coefs);
    if (!rc && (i < 0 || j < 0 || k < 0 || ll < 0 || i >= nshell || j >= nshell || k >= nshell || ll >= nshell))
        rc = -1;
    if (rc) { basis_free(&b); return rc; }
    size_t n = 12 * (size_t)nsph(l[i]) * nsph(l[j]) * nsph(l[k]) * nsph(l[ll]);
    real *tmp = malloc(sizeof(real) * n);
    work_t w; memset(&w, 0, sizeof(w));
    rc = tmp ? quartet_deriv_sph(&w, &b, i, j, k, ll, tmp) : -3;
    for (size_t q = 0; q < n && !rc; ++q) out[q] = (double)tmp[q];
    free(tmp); work_free(&w); basis_free(&b);
    return rc;
}

/* Config-style primitive quartets: n quartets of class (la lb|lc ld), centres
 * [n][4][3], exponents [n][4]; normalised primitives (coefficient N(a,l));
 * output spherical blocks [n][nsph(la)][nsph(lb)][nsph(lc)][nsph(ld)]. */
int PFX(eri_prim_quartets)(int la, int lb, int lc, int ld, int64_t n, const double *centers,
                           const double *exps, double *out)
{
    int L4[4] = {la, lb, lc, ld};
    for (int q = 0; q < 4; ++q) {
        if (L4[q] < 0) return -1;
        if (L4[q] > LMAX) return -2;
    }
    if (n < 0) return -1;
    init_tables();
    size_t blk = (size_t)nsph(la) * nsph(lb) * nsph(lc) * nsph(ld);
    int err = 0;
#pragma omp parallel
    {
        work_t w; memset(&w, 0, sizeof(w));
        real *tmp = malloc(sizeof(real) * blk);
        int lrc = tmp ? 0 : -3;
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < n; ++q) {
            if (lrc) continue;
            int l4[4] = {la, lb, lc, ld}, np4[4] = {1, 1, 1, 1}, nshell = 4;
            double one[4] = {1, 1, 1, 1};
            basis_t b;
            lrc = basis_make(&b, nshell, l4, np4, centers + 12 * q, exps + 4 * q, one);
            if (!lrc) lrc = quartet_sph(&w, &b, 0, 1, 2, 3, tmp);
            basis_free(&b);
            for (size_t i = 0; i < blk && !lrc; ++i) out[(size_t)q * blk + i] = (double)tmp[i];
        }
        if (lrc) {
#pragma omp atomic write
            err = lrc;
        }
        free(tmp); work_free(&w);
    }
    return err;
}

/* Schwarz factors Q[s*nshell+t] = sqrt(max |(mn|mn)|) over m in s, n in t */
static int schwarz(const basis_t *b, real *Qm)
{
    int ns = b->nshell, err = 0;
#pragma omp parallel
    {
        work_t w; memset(&w, 0, sizeof(w));
        real *blk = malloc(sizeof(real) * 9 * 9 * 9 * 9);
        int lrc = blk ? 0 : -3;
#pragma omp for schedule(dynamic, 1)
        for (int s = 0; s < ns; ++s)
            for (int t = 0; t <= s; ++t) {
                if (lrc) continue;
                lrc = quartet_sph(&w, b, s, t, s, t, blk);
                int n1 = nsph(b->l[s]), n2 = nsph(b->l[t]);
                real mx = 0;
                for (int m = 0; m < n1; ++m)
                    for (int n = 0; n < n2; ++n) {
                        real v = FABS(blk[((size_t)(m * n2 + n) * n1 + m) * n2 + n]);
                        if (v > mx) mx = v;
                    }
                Qm[(size_t)s * ns + t] = Qm[(size_t)t * ns + s] = SQRT(mx);
            }
        if (lrc) {
#pragma omp atomic write
            err = lrc;
        }
        free(blk); work_free(&w);
    }
    return err;
}

int PFX(schwarz)(int nshell, const int *l, const int *nprim, const double *centers, const double *exps,
                 const double *coefs, double *Q)
{
    basis_t b;
    int rc = basis_make(&b, nshell, l, nprim, centers, exps, coefs);
    real *Qm = rc ? NULL : malloc(sizeof(real) * (size_t)nshell * nshell + 1);
    if (!rc && !Qm) rc = -3;
    if (!rc) rc = schwarz(&b, Qm);
    for (size_t i = 0; !rc && i < (size_t)nshell * nshell; ++i) Q[i] = (double)Qm[i];
    free(Qm); basis_free(&b);
    return rc;
}

/* J and K from the unique shell quartets (i>=j, k>=l, ij>=kl), each adding
 * every distinct image among its 8 index permutations once.  Quartets with
 * Q_ij Q_kl < tau are skipped (tau = 0: no screening).  D is used as given
 * (it need not be symmetric); J, K are N x N row-major and overwritten. */
int PFX(jk)(int nshell, const int *l, const int *nprim, const double *centers, const double *exps,
            const double *coefs, const double *D, double tau, double *J, double *K)
{
    basis_t b;
    int rc = basis_make(&b, nshell, l, nprim, centers, exps, coefs);
    if (rc) { basis_free(&b); return rc; }
    int N = b.nbf, ns = nshell;
    size_t NN = (size_t)N * N;
    real *Qm = malloc(sizeof(real) * ((size_t)ns * ns + 1));
    real *Jt = calloc(NN + 1, sizeof(real)), *Kt = calloc(NN + 1, sizeof(real));
    if (!Qm || !Jt || !Kt) rc = -3;
    if (!rc && tau > 0) rc = schwarz(&b, Qm);
    long npair = (long)ns * (ns + 1) / 2;
    static const int perm[8][4] = {{0, 1, 2, 3}, {1, 0, 2, 3}, {0, 1, 3, 2}, {1, 0, 3, 2},
                                   {2, 3, 0, 1}, {3, 2, 0, 1}, {2, 3, 1, 0}, {3, 2, 1, 0}};
    int err = rc;
    if (!rc) {
#pragma omp parallel
        {
            work_t w; memset(&w, 0, sizeof(w));
            real *blk = malloc(sizeof(real) * 9 * 9 * 9 * 9);
            real *Jl = calloc(NN + 1, sizeof(real)), *Kl = calloc(NN + 1, sizeof(real));
            int lrc = (blk && Jl && Kl) ? 0 : -3;
#pragma omp for schedule(dynamic, 1)
            for (long p = 0; p < npair; ++p) {
                if (lrc) continue;
                int i = (int)((sqrt(8.0 * (double)p + 1.0) - 1.0) / 2.0);
                while ((long)i * (i + 1) / 2 > p) --i;
                while ((long)(i + 1) * (i + 2) / 2 <= p) ++i;
                int j = (int)(p - (long)i * (i + 1) / 2);
                for (long r = 0; r <= p && !lrc; ++r) {
                    int k = (int)((sqrt(8.0 * (double)r + 1.0) - 1.0) / 2.0);
                    while ((long)k * (k + 1) / 2 > r) --k;
                    while ((long)(k + 1) * (k + 2) / 2 <= r) ++k;
                    int ll = (int)(r - (long)k * (k + 1) / 2);
                    if (tau > 0 && Qm[(size_t)i * ns + j] * Qm[(size_t)k * ns + ll] < (real)tau) continue;
                    lrc = quartet_sph(&w, &b, i, j, k, ll, blk);
                    if (lrc) break;
                    int sh[4] = {i, j, k, ll};
                    /* walk every function quartet of the block and every distinct image */
                    int n0 = nsph(l[i]), n1 = nsph(l[j]), n2 = nsph(l[k]), n3 = nsph(l[ll]);
                    int o[4] = {b.foff[i], b.foff[j], b.foff[k], b.foff[ll]};
                    int used[8], nu = 0;
                    for (int q = 0; q < 8; ++q) {
                        int t[4] = {sh[perm[q][0]], sh[perm[q][1]], sh[perm[q][2]], sh[perm[q][3]]};
                        int dup = 0;
                        for (int u = 0; u < nu; ++u) {
                            const int *pu = perm[used[u]];
                            if (sh[pu[0]] == t[0] && sh[pu[1]] == t[1] && sh[pu[2]] == t[2] && sh[pu[3]] == t[3]) dup = 1;
                        }
                        if (!dup) used[nu++] = q;
                    }
                    for (int a0 = 0; a0 < n0; ++a0)
                    for (int a1 = 0; a1 < n1; ++a1)
                    for (int a2 = 0; a2 < n2; ++a2)
                    for (int a3 = 0; a3 < n3; ++a3) {
                        real v = blk[((size_t)(a0 * n1 + a1) * n2 + a2) * n3 + a3];
                        int f[4] = {o[0] + a0, o[1] + a1, o[2] + a2, o[3] + a3};
                        for (int u = 0; u < nu; ++u) {
                            const int *pq = perm[used[u]];
                            int w0 = f[pq[0]], w1 = f[pq[1]], w2 = f[pq[2]], w3 = f[pq[3]];
                            Jl[(size_t)w0 * N + w1] += v * (real)D[(size_t)w2 * N + w3];
                            Kl[(size_t)w0 * N + w2] += v * (real)D[(size_t)w1 * N + w3];
                        }
                    }
                }
            }
#pragma omp critical
            {
                for (size_t q = 0; q < NN; ++q) { Jt[q] += Jl[q]; Kt[q] += Kl[q]; }
                if (lrc) err = lrc;
            }
            free(blk); free(Jl); free(Kl); work_free(&w);
        }
    }
    if (!err) {
        for (size_t q = 0; q < NN; ++q) {
            if (J) J[q] = (double)Jt[q];
            if (K) K[q] = (double)Kt[q];
        }
    }
    free(Qm); free(Jt); free(Kt); basis_free(&b);
    return err;
}

/* Direct J and K blocks for the listed shell pairs (P,Q), from the definitions
 * without any permutational symmetry:
 *   J[m in P][n in Q] = sum over all ordered shell pairs (R,S) of (PQ|RS) D_RS,
 *   K[m in P][n in Q] = sum over all ordered (R,S) of (PR|QS) D_RS,
 * skipping a quartet when its Schwarz product is below tau (tau = 0: none).
 * Block t is stored row-major at offset sum_{u<t} nsph(P_u) nsph(Q_u). */
int PFX(jk_blocks)(int nshell, const int *l, const int *nprim, const double *centers, const double *exps,
                   const double *coefs, const double *D, double tau, int npairs, const int *pairs,
                   double *Jout, double *Kout)
{
    basis_t b;
    int rc = basis_make(&b, nshell, l, nprim, centers, exps, coefs);
    for (int t = 0; !rc && t < npairs; ++t)
        if (pairs[2 * t] < 0 || pairs[2 * t] >= nshell || pairs[2 * t + 1] < 0 || pairs[2 * t + 1] >= nshell) rc = -1;
    if (rc) { basis_free(&b); return rc; }
    int N = b.nbf, ns = nshell;
    real *Qm = malloc(sizeof(real) * ((size_t)ns * ns + 1));
    if (!Qm) rc = -3;
    if (!rc && tau > 0) rc = schwarz(&b, Qm);
    size_t off = 0;
    for (int t = 0; t < npairs && !rc; ++t) {
        int P = pairs[2 * t], Qs = pairs[2 * t + 1];
        int np_ = nsph(l[P]), nq = nsph(l[Qs]);
        real accJ[81], accK[81];
        memset(accJ, 0, sizeof(accJ)); memset(accK, 0, sizeof(accK));
        int err = 0;
#pragma omp parallel
        {
            work_t w; memset(&w, 0, sizeof(w));
            real *blk = malloc(sizeof(real) * 9 * 9 * 9 * 9);
            real lJ[81], lK[81];
            memset(lJ, 0, sizeof(lJ)); memset(lK, 0, sizeof(lK));
            int lrc = blk ? 0 : -3;
#pragma omp for schedule(dynamic, 1)
            for (int R = 0; R < ns; ++R)
                for (int S = 0; S < ns && !lrc; ++S) {
                    int nr = nsph(l[R]), nsS = nsph(l[S]);
                    int oR = b.foff[R], oS = b.foff[S];
                    if (!(tau > 0) || Qm[(size_t)P * ns + Qs] * Qm[(size_t)R * ns + S] >= (real)tau) {
                        lrc = quartet_sph(&w, &b, P, Qs, R, S, blk);   /* (PQ|RS) */
                        for (int m = 0; m < np_ && !lrc; ++m)
                            for (int n = 0; n < nq; ++n)
                                for (int r = 0; r < nr; ++r)
                                    for (int s = 0; s < nsS; ++s)
                                        lJ[m * nq + n] += blk[((size_t)(m * nq + n) * nr + r) * nsS + s] *
                                                          (real)D[(size_t)(oR + r) * N + oS + s];
                    }
                    if (!lrc && (!(tau > 0) || Qm[(size_t)P * ns + R] * Qm[(size_t)Qs * ns + S] >= (real)tau)) {
                        lrc = quartet_sph(&w, &b, P, R, Qs, S, blk);   /* (PR|QS) */
                        for (int m = 0; m < np_ && !lrc; ++m)
                            for (int r = 0; r < nr; ++r)
                                for (int n = 0; n < nq; ++n)
                                    for (int s = 0; s < nsS; ++s)
                                        lK[m * nq + n] += blk[((size_t)(m * nr + r) * nq + n) * nsS + s] *
                                                          (real)D[(size_t)(oR + r) * N + oS + s];
                    }
                }
#pragma omp critical
            {
                for (int q = 0; q < 81; ++q) { accJ[q] += lJ[q]; accK[q] += lK[q]; }
                if (lrc) err = lrc;
            }
            free(blk); work_free(&w);
        }
        rc = err;
        for (int q = 0; q < np_ * nq && !rc; ++q) {
            if (Jout) Jout[off + q] = (double)accJ[q];
            if (Kout) Kout[off + q] = (double)accK[q];
        }
        off += (size_t)np_ * nq;
    }
    free(Qm); basis_free(&b);
    return rc;
}

/* The full spherical tensor (mn|ls), N^4 row-major, from every ordered shell
 * quartet (small bases only). */
int PFX(eri_tensor)(int nshell, const int *l, const int *nprim, const double *centers, const double *exps,
                    const double *coefs, double *out)
{
    basis_t b;
    int rc = basis_make(&b, nshell, l, nprim, centers, exps, coefs);
    if (rc) { basis_free(&b); return rc; }
    size_t N = (size_t)b.nbf;
    int err = 0;
#pragma omp parallel
    {
        work_t w; memset(&w, 0, sizeof(w));
        real *blk = malloc(sizeof(real) * 9 * 9 * 9 * 9);
        int lrc = blk ? 0 : -3;
#pragma omp for schedule(dynamic, 1) collapse(2)
        for (int i = 0; i < nshell; ++i)
            for (int j = 0; j < nshell; ++j)
                for (int k = 0; k < nshell && !lrc; ++k)
                    for (int q = 0; q < nshell && !lrc; ++q) {
                        lrc = quartet_sph(&w, &b, i, j, k, q, blk);
                        int n0 = nsph(l[i]), n1 = nsph(l[j]), n2 = nsph(l[k]), n3 = nsph(l[q]);
                        for (int a = 0; a < n0 && !lrc; ++a)
                            for (int c = 0; c < n1; ++c)
                                for (int e = 0; e < n2; ++e)
                                    for (int g = 0; g < n3; ++g)
                                        out[(((size_t)(b.foff[i] + a) * N + b.foff[j] + c) * N + b.foff[k] + e) * N +
                                            b.foff[q] + g] = (double)blk[((size_t)(a * n1 + c) * n2 + e) * n3 + g];
                    }
        if (lrc) {
#pragma omp atomic write
            err = lrc;
        }
        free(blk); work_free(&w);
    }
    basis_free(&b);
    return err;
}

/* Spherical blocks of the nq listed shell quartets (4 shell indices each),
 * evaluated in parallel; *count gets the number of integrals evaluated and
 * *checksum the sum of all their values (the blocks are not kept). */
int PFX(eri_quartet_list)(int nshell, const int *l, const int *nprim, const double *centers, const double *exps,
                          const double *coefs, int64_t nq, const int *quartets, int64_t *count, double *checksum)
{
    basis_t b;
    int rc = basis_make(&b, nshell, l, nprim, centers, exps, coefs);
    for (int64_t q = 0; !rc && q < 4 * nq; ++q)
        if (quartets[q] < 0 || quartets[q] >= nshell) rc = -1;
    if (rc) { basis_free(&b); return rc; }
    int64_t cnt = 0;
    real sum = 0;
    int err = 0;
#pragma omp parallel reduction(+ : cnt, sum)
    {
        work_t w; memset(&w, 0, sizeof(w));
        real *blk = malloc(sizeof(real) * 9 * 9 * 9 * 9);
        int lrc = blk ? 0 : -3;
#pragma omp for schedule(dynamic, 4)
        for (int64_t q = 0; q < nq; ++q) {
            if (lrc) continue;
            const int *s = quartets + 4 * q;
            lrc = quartet_sph(&w, &b, s[0], s[1], s[2], s[3], blk);
            int64_t n = (int64_t)nsph(l[s[0]]) * nsph(l[s[1]]) * nsph(l[s[2]]) * nsph(l[s[3]]);
            for (int64_t i = 0; i < n && !lrc; ++i) sum += blk[i];
            cnt += n;
        }
        if (lrc) {
#pragma omp atomic write
            err = lrc;
        }
        free(blk); work_free(&w);
    }
    if (count) *count = cnt;
    if (checksum) *checksum = (double)sum;
    basis_free(&b);
    return err;
}

/* threads an OpenMP parallel region of the oracle uses */
int PFX(num_threads)(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
