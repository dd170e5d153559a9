/*
 * Driver for the oracle's AddressSanitizer / UndefinedBehaviorSanitizer
 * build (test infrastructure, host code only).  It compiles oracle.c into
 * itself and runs every exported entry point once on small inputs: a
 * two-atom basis with shells up to l = 4 and several primitives, plus the
 * argument errors.  Any out-of-bounds access, leak or undefined operation
 * aborts with a non-zero status; the values themselves are checked by the
 * Python pins, here only their finiteness.
 *
 *   gcc -fsanitize=address,undefined -fno-sanitize-recover=all -g -O1 \
 *       [-DORACLE_LD] oracle/sanitize_main.c -lm -o oracle_asan
 */
#include "oracle.c"

#include <stdio.h>

static int check_finite(const double *v, size_t n, const char *what)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) {
            fprintf(stderr, "%s: non-finite value at %zu\n", what, i);
            return 1;
        }
    return 0;
}

#define CHECK(call, want)                                                               \
    do {                                                                                \
        int rc_ = (call);                                                               \
        if (rc_ != (want)) {                                                            \
            fprintf(stderr, "%s returned %d, expected %d\n", #call, rc_, (want));       \
            return 1;                                                                   \
        }                                                                               \
    } while (0)

int main(void)
{
    /* shells: atom 0: s(3) p(2) d(1) g(2); atom 1: s(1) f(2) p(1) */
    const int nshell = 7;
    const int l[7] = {0, 1, 2, 4, 0, 3, 1};
    const int np[7] = {3, 2, 1, 2, 1, 2, 1};
    double cen[21];
    for (int s = 0; s < 7; ++s) {
        const double *c = s < 4 ? (const double[3]){0.1, -0.2, 0.3} : (const double[3]){1.4, 0.9, -0.7};
        for (int k = 0; k < 3; ++k) cen[3 * s + k] = c[k];
    }
    const double exps[12] = {13.0, 2.0, 0.4, 1.7, 0.35, 0.8, 2.2, 0.6, 0.5, 3.1, 0.9, 0.45};
    const double coefs[12] = {0.2, 0.5, 0.7, 0.6, 0.4, 1.0, 0.3, 0.9, 1.0, 0.5, 0.8, 1.0};
    int N = 0;
    for (int s = 0; s < nshell; ++s) N += 2 * l[s] + 1;

    double F[20];
    CHECK(PFX(boys)(16, 0.0, F), 0);
    CHECK(PFX(boys)(16, 7.5, F), 0);
    CHECK(PFX(boys)(16, 80.0, F), 0);
    if (check_finite(F, 17, "boys")) return 1;

    double T[9 * 15];
    for (int ll = 0; ll <= 4; ++ll) {
        CHECK(PFX(sph_matrix)(ll, T), 0);
        if (check_finite(T, (size_t)(2 * ll + 1) * ((ll + 1) * (ll + 2) / 2), "sph_matrix")) return 1;
    }
    CHECK(PFX(sph_matrix)(5, T), -2);

    double nc[3];
    CHECK(PFX(norm_coefs)(2, 3, exps, coefs, nc), 0);

    const double c12[12] = {0, 0, 0, 0.5, 0, 0, 0, 0.7, 0, 0.2, 0.1, 0.3};
    const double a4[4] = {1.1, 0.6, 2.0, 0.9};
    double cart[15 * 15 * 15 * 15];
    CHECK(PFX(prim_cart_eri)(4, 4, 4, 4, c12, a4, cart), 0);
    if (check_finite(cart, 15 * 15 * 15 * 15, "prim_cart_eri")) return 1;

    double blk[9 * 7 * 5 * 9];
    CHECK(PFX(eri_shell_quartet)(nshell, l, np, cen, exps, coefs, 3, 5, 2, 3, blk), 0);
    if (check_finite(blk, 9 * 7 * 5 * 9, "eri_shell_quartet")) return 1;
    CHECK(PFX(eri_shell_quartet)(nshell, l, np, cen, exps, coefs, 0, 1, 2, 7, blk), -1);

    double *dblk = malloc(sizeof(double) * 12 * 9 * 7 * 5 * 9);
    if (!dblk) return 1;
    CHECK(PFX(eri_deriv_shell_quartet)(nshell, l, np, cen, exps, coefs, 3, 5, 2, 3, dblk), 0);
    if (check_finite(dblk, 12 * 9 * 7 * 5 * 9, "eri_deriv_shell_quartet")) return 1;
    free(dblk);

    const double pc[24] = {0, 0, 0, 0.3, 0, 0, 0, 0.4, 0, 0, 0, 0.5, 1, 1, 1, 1.2, 1, 1, 1, 1.3, 1, 1, 1, 1.4};
    const double pe[8] = {0.5, 1.5, 2.5, 3.5, 0.7, 1.1, 4.0, 0.2};
    double pq[2 * 7 * 5 * 3 * 9];
    CHECK(PFX(eri_prim_quartets)(3, 2, 1, 4, 2, pc, pe, pq), 0);
    if (check_finite(pq, 2 * 7 * 5 * 3 * 9, "eri_prim_quartets")) return 1;
    CHECK(PFX(eri_prim_quartets)(5, 0, 0, 0, 1, pc, pe, pq), -2);

    double *Q = malloc(sizeof(double) * nshell * nshell);
    double *D = malloc(sizeof(double) * N * N), *J = malloc(sizeof(double) * N * N), *K = malloc(sizeof(double) * N * N);
    if (!Q || !D || !J || !K) return 1;
    CHECK(PFX(schwarz)(nshell, l, np, cen, exps, coefs, Q), 0);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) D[i * N + j] = 1.0 / (1.0 + i + j);
    CHECK(PFX(jk)(nshell, l, np, cen, exps, coefs, D, 0.0, J, K), 0);
    if (check_finite(J, (size_t)N * N, "J") || check_finite(K, (size_t)N * N, "K")) return 1;
    CHECK(PFX(jk)(nshell, l, np, cen, exps, coefs, D, 1e-10, J, K), 0);

    const int pairs[6] = {3, 5, 0, 0, 6, 2};
    double Jb[9 * 7 + 1 + 3 * 5], Kb[9 * 7 + 1 + 3 * 5];
    CHECK(PFX(jk_blocks)(nshell, l, np, cen, exps, coefs, D, 0.0, 3, pairs, Jb, Kb), 0);
    if (check_finite(Jb, 9 * 7 + 1 + 15, "jk_blocks J")) return 1;

    /* the full tensor of a smaller basis (shells 0..2 and 4, 6) */
    const int l2[4] = {0, 1, 0, 1};
    const int np2[4] = {3, 2, 1, 1};
    const double cen2[12] = {0, 0, 0, 0, 0, 0, 1, 0.5, 0, 1, 0.5, 0};
    const double e2[7] = {13.0, 2.0, 0.4, 1.7, 0.35, 0.5, 0.9};
    const double co2[7] = {0.2, 0.5, 0.7, 0.6, 0.4, 1.0, 1.0};
    double *E = malloc(sizeof(double) * 8 * 8 * 8 * 8);
    if (!E) return 1;
    CHECK(PFX(eri_tensor)(4, l2, np2, cen2, e2, co2, E), 0);

    const int ql[8] = {3, 3, 3, 3, 5, 1, 2, 0};
    int64_t cnt = 0;
    double chk = 0.0;
    CHECK(PFX(eri_quartet_list)(nshell, l, np, cen, exps, coefs, 2, ql, &cnt, &chk), 0);
    if (cnt != 9 * 9 * 9 * 9 + 7 * 3 * 5 * 1) {
        fprintf(stderr, "eri_quartet_list counted %lld\n", (long long)cnt);
        return 1;
    }

    /* argument errors */
    const int lbad[1] = {5};
    CHECK(PFX(schwarz)(1, lbad, np, cen, exps, coefs, Q), -2);

    free(Q); free(D); free(J); free(K); free(E);
    printf("oracle sanitizer driver: ok (N = %d, threads %d)\n", N, PFX(num_threads)());
    return 0;
}
