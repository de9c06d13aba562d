/* oracle_driver.c -- runs the CPU oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer (test infrastructure).  Small tensors of every
 * supported form (2D-4D groups, outer and inner spectators, index pairs,
 * chains, in place, zero extents) go through the forward chain and its
 * adjoint; besides the sanitizers' own checks it verifies that in place
 * equals out of place and that <S x, y> = <x, S^T y>.  Prints PASSED or the
 * failed checks; exit status 0 when every check held. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_spinsum_chain_ex(int ndim, const int64_t* extents, int group_first, int d, int pairs,
                            int nstages, const int* nterms, const int* perms, const double* alpha,
                            const double* in, double* out, int nthreads);
int oracle_spinsum_chain_adjoint_ex(int ndim, const int64_t* extents, int group_first, int d,
                                    int pairs, int nstages, const int* nterms, const int* perms,
                                    const double* alpha, const double* grad_out, double* grad_in,
                                    int nthreads);

static int fails = 0;
static uint64_t rng = 0x9E3779B97F4A7C15ull;

static double uni(void) {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

/* every permutation of d in lexicographic order, random coefficient each */
static int all_perms(int d, int* perms, double* alpha) {
    int p[4], n = 0;
    for (int i = 0; i < d; ++i) p[i] = i;
    for (;;) {
        memcpy(perms + n * d, p, sizeof(int) * d);
        alpha[n] = (double)((int)(uni() * 4.0));
        ++n;
        int i = d - 2;
        while (i >= 0 && p[i] > p[i + 1]) --i;
        if (i < 0) break;
        int j = d - 1;
        while (p[j] < p[i]) --j;
        int t = p[i]; p[i] = p[j]; p[j] = t;
        for (int a = i + 1, b = d - 1; a < b; ++a, --b) { t = p[a]; p[a] = p[b]; p[b] = t; }
    }
    return n;
}

static void run(const char* name, int ndim, const int64_t* ext, int gf, int d, int pairs,
                int nstages) {
    int64_t n = 1;
    for (int i = 0; i < ndim; ++i) n *= ext[i];
    int perms[2 * 24 * 4], nterms[2];
    double alpha[2 * 24];
    int off = 0;
    for (int s = 0; s < nstages; ++s) {
        nterms[s] = all_perms(d, perms + off * d, alpha + off);
        off += nterms[s];
    }
    size_t bytes = (size_t)(n > 0 ? n : 1) * sizeof(double);
    double* x = malloc(bytes);
    double* y = malloc(bytes);
    double* z = malloc(bytes);
    double* g = malloc(bytes);
    for (int64_t i = 0; i < n; ++i) { x[i] = uni(); y[i] = uni(); }
    int st = oracle_spinsum_chain_ex(ndim, ext, gf, d, pairs, nstages, nterms, perms, alpha, x, z, 2);
    if (st != 0) { printf("FAIL %s: forward status %d\n", name, st); ++fails; }
    memcpy(g, x, n * sizeof(double));
    st = oracle_spinsum_chain_ex(ndim, ext, gf, d, pairs, nstages, nterms, perms, alpha, g, g, 1);
    if (st != 0 || (n > 0 && memcmp(g, z, n * sizeof(double)) != 0)) {
        printf("FAIL %s: in place differs\n", name);
        ++fails;
    }
    st = oracle_spinsum_chain_adjoint_ex(ndim, ext, gf, d, pairs, nstages, nterms, perms, alpha, y,
                                         g, 2);
    if (st != 0) { printf("FAIL %s: adjoint status %d\n", name, st); ++fails; }
    double lhs = 0, rhs = 0, scale = 0;
    for (int64_t i = 0; i < n; ++i) {
        lhs += z[i] * y[i];
        rhs += x[i] * g[i];
        scale += fabs(z[i] * y[i]);
    }
    if (fabs(lhs - rhs) > 1e-12 * (scale + 1.0)) {
        printf("FAIL %s: adjoint identity %g vs %g\n", name, lhs, rhs);
        ++fails;
    }
    free(x); free(y); free(z); free(g);
    printf("ok %s\n", name);
}

int main(void) {
    const int64_t a[] = {3, 5, 5, 5};
    const int64_t b[] = {2, 4, 4, 4, 4, 2};
    const int64_t c[] = {7, 7};
    const int64_t e[] = {2, 3, 3, 3, 4, 4, 4, 2};
    const int64_t f[] = {1, 2, 2, 2, 2, 3, 3, 3, 3};
    const int64_t z0[] = {0, 4, 4, 4};
    const int64_t z1[] = {2, 3, 3, 3, 0};
    const int64_t one[] = {4, 1, 1, 1};
    run("3d outer", 4, a, 1, 3, 0, 1);
    run("3d chain", 4, a, 1, 3, 0, 2);
    run("4d outer+inner", 6, b, 1, 4, 0, 2);
    run("2d", 2, c, 0, 2, 0, 1);
    run("3d pairs + inner", 8, e, 4, 3, 1, 2);
    run("4d pairs", 9, f, 5, 4, 1, 1);
    run("empty outer", 4, z0, 1, 3, 0, 1);
    run("empty inner", 5, z1, 1, 3, 0, 1);
    run("extent one", 4, one, 1, 3, 0, 2);
    /* refused arguments */
    int bad[3] = {0, 0, 1}, nt = 1;
    double al = 1.0, buf[48];
    if (oracle_spinsum_chain_ex(4, a, 1, 3, 0, 1, &nt, bad, &al, buf, buf, 1) == 0) {
        printf("FAIL non-bijection accepted\n");
        ++fails;
    }
    printf("%s\n", fails ? "FAILED" : "PASSED");
    return fails ? 1 : 0;
}
