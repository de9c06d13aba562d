/*
 * spinsum_oracle.c -- plain, slow CPU reference for spin summations.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so and is
 * loaded exclusively by the test-suite, by the smoke check and by the CPU
 * baseline leg of the benchmark.  The GPU library never includes, links or
 * calls anything in here, and nothing in here is shared with it.
 *
 * What it computes (Springer, Matthews, Bientinesi, "Spin Summations: A
 * High-Performance Perspective"):
 *
 *   Def. 1 / Eq. 1-2   a permutation pi_{phi(1)..phi(d)} sends the index tuple
 *                      (i_1..i_d) to (i_phi(1) .. i_phi(d)).  Here a
 *                      permutation is stored 0-based: p[m] = phi(m+1) - 1.
 *   Def. 2 / Eq. 3     B_i <- A_{pi(i)}: output element i reads the input at
 *                      the permuted tuple.
 *   Def. 3 / Eq. 4     B <- sum_t alpha_t * omega_t(A).
 *   Def. 4 / Eq. 5-6   a factorised sum is a chain of such sums; the inner
 *                      factor is applied first, into a full temporary (the
 *                      two-pass form of Alg. 3).
 *
 * The permuted index group is a contiguous run of d dimensions of a
 * row-major (last index fastest) tensor of shape
 *     [outer spectators ..., N x d, inner spectators ...];
 * spectator indices are carried through unchanged.  All group extents must
 * be equal (hyper-square, Sec. 3.1).
 *
 * Index-pair form: the coupled-cluster quantities whose spin summations the
 * paper targets (Sec. 1) carry indices in pairs, e.g. T[a,b,c,i,j,k] with
 * (a,i), (b,j), (c,k) belonging together.  With `pairs` set, the d
 * dimensions right before the group (extent V each) are permuted by the
 * same permutation as the group:
 *     B[.., a_0..a_{d-1}, i_0..i_{d-1}, ..] +=
 *         alpha_t * A[.., a_{p[0]}..a_{p[d-1]}, i_{p[0]}..i_{p[d-1]}, ..].
 * Here this is evaluated literally, on the 2d-tuple (a, i).
 *
 * Arithmetic: each output element is accumulated in long double (x87
 * extended precision on x86-64) with no reordering beyond the term order,
 * and rounded to double once at the end.  Chain temporaries are kept in
 * long double.  Terms whose coefficient is exactly zero are skipped, so a
 * zero-weight term contributes nothing even when the input holds Inf/NaN
 * (reading of a sum with zero weight).
 *
 * The adjoint (transpose) is computed by its plain definition as a scatter:
 * for every output position i and term t, grad_in[source(i,t)] +=
 * alpha_t * grad_out[i].  It does not use inverse permutations, so it is an
 * independent route from any code that does.
 *
 * Parallelism: an optional OpenMP loop over the outer spectator index, used
 * only so the CPU baseline can be timed on several cores.  Results do not
 * depend on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_ERR_ARG (-1)
#define ORACLE_ERR_PERM (-2)
#define ORACLE_ERR_EXTENT (-3)
#define ORACLE_ERR_NOMEM (-7)

#define ORACLE_MAX_D 8

typedef struct {
    int64_t outer;   /* product of the extents before the permuted dims */
    int64_t inner;   /* product of the extents after the group          */
    int64_t group;   /* product of the permuted extents (N^d, or V^d N^d) */
    int64_t ext[2 * ORACLE_MAX_D];  /* extents of the permuted dims     */
    int d;
    int nidx;        /* permuted dims: d, or 2d in the index-pair form  */
} layout_t;

static int make_layout(int ndim, const int64_t* extents, int group_first, int d, int pairs,
                       layout_t* L) {
    if (ndim < 1 || extents == NULL || d < 1 || d > ORACLE_MAX_D) return ORACLE_ERR_ARG;
    if (group_first < 0 || group_first + d > ndim) return ORACLE_ERR_ARG;
    if (pairs && group_first < d) return ORACLE_ERR_ARG;
    for (int k = 0; k < ndim; ++k)
        if (extents[k] < 0) return ORACLE_ERR_ARG;
    const int first = pairs ? group_first - d : group_first;
    L->d = d;
    L->nidx = pairs ? 2 * d : d;
    for (int m = 0; m < L->nidx; ++m) L->ext[m] = extents[first + m];
    for (int m = 1; m < d; ++m)
        if (extents[group_first + m] != extents[group_first]) return ORACLE_ERR_EXTENT;
    if (pairs)
        for (int m = 1; m < d; ++m)
            if (extents[first + m] != extents[first]) return ORACLE_ERR_EXTENT;
    L->outer = 1;
    for (int k = 0; k < first; ++k) L->outer *= extents[k];
    L->inner = 1;
    for (int k = group_first + d; k < ndim; ++k) L->inner *= extents[k];
    L->group = 1;
    for (int m = 0; m < L->nidx; ++m) L->group *= L->ext[m];
    return ORACLE_OK;
}

/* Position read for permuted dim m by a term with group permutation p: the
 * group part (and the partner part of the index-pair form) follow p. */
static int read_pos(const layout_t* L, const int* p, int m) {
    if (L->nidx == L->d) return p[m];
    return (m < L->d) ? p[m] : L->d + p[m - L->d];
}

static int check_perms(int d, int nterms, const int* perms) {
    if (nterms < 0 || (nterms > 0 && perms == NULL)) return ORACLE_ERR_ARG;
    for (int t = 0; t < nterms; ++t) {
        int seen[ORACLE_MAX_D] = {0};
        for (int m = 0; m < d; ++m) {
            int v = perms[t * d + m];
            if (v < 0 || v >= d || seen[v]) return ORACLE_ERR_PERM;
            seen[v] = 1;
        }
    }
    return ORACLE_OK;
}

/* Offset (in units of the inner block) of the permuted-dims tuple
 * idx[0..nidx-1] inside one outer slice: row-major, last fastest. */
static int64_t group_offset(const layout_t* L, const int64_t* idx) {
    int64_t off = 0;
    for (int m = 0; m < L->nidx; ++m) off = off * L->ext[m] + idx[m];
    return off;
}

/* One summation stage, long double in and out (Def. 3, evaluated in the
 * output-linear order of Alg. 1). */
static void stage_ld(const layout_t* L, int nterms, const int* perms,
                     const double* alpha, const long double* src,
                     long double* dst, int nthreads) {
    const int d = L->d, nidx = L->nidx;
    (void)nthreads;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
#endif
    for (int64_t b = 0; b < L->outer; ++b) {
        int64_t idx[2 * ORACLE_MAX_D];
        int64_t read[2 * ORACLE_MAX_D];
        const long double* s = src + b * L->group * L->inner;
        long double* o = dst + b * L->group * L->inner;
        for (int m = 0; m < nidx; ++m) idx[m] = 0;
        for (int64_t g = 0; g < L->group; ++g) {
            /* idx is the tuple of permuted indices of linear index g */
            for (int64_t r = 0; r < L->inner; ++r) {
                long double acc = 0.0L;
                for (int t = 0; t < nterms; ++t) {
                    if (alpha[t] == 0.0) continue;
                    const int* p = perms + t * d;
                    for (int m = 0; m < nidx; ++m) read[m] = idx[read_pos(L, p, m)];
                    acc += (long double)alpha[t] * s[group_offset(L, read) * L->inner + r];
                }
                o[g * L->inner + r] = acc;
            }
            /* advance the odometer, last index fastest */
            for (int m = nidx - 1; m >= 0; --m) {
                if (++idx[m] < L->ext[m]) break;
                idx[m] = 0;
            }
        }
    }
}

/* Transpose of one stage, by its definition as a scatter. */
static void stage_adjoint_ld(const layout_t* L, int nterms, const int* perms,
                             const double* alpha, const long double* gout,
                             long double* gin, int nthreads) {
    const int d = L->d, nidx = L->nidx;
    (void)nthreads;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
#endif
    for (int64_t b = 0; b < L->outer; ++b) {
        int64_t idx[2 * ORACLE_MAX_D];
        int64_t read[2 * ORACLE_MAX_D];
        const long double* go = gout + b * L->group * L->inner;
        long double* gi = gin + b * L->group * L->inner;
        for (int64_t e = 0; e < L->group * L->inner; ++e) gi[e] = 0.0L;
        for (int m = 0; m < nidx; ++m) idx[m] = 0;
        for (int64_t g = 0; g < L->group; ++g) {
            for (int64_t r = 0; r < L->inner; ++r) {
                for (int t = 0; t < nterms; ++t) {
                    if (alpha[t] == 0.0) continue;
                    const int* p = perms + t * d;
                    for (int m = 0; m < nidx; ++m) read[m] = idx[read_pos(L, p, m)];
                    gi[group_offset(L, read) * L->inner + r] +=
                        (long double)alpha[t] * go[g * L->inner + r];
                }
            }
            for (int m = nidx - 1; m >= 0; --m) {
                if (++idx[m] < L->ext[m]) break;
                idx[m] = 0;
            }
        }
    }
}

static int run_chain(int adjoint, int ndim, const int64_t* extents, int group_first,
                     int d, int pairs, int nstages, const int* nterms, const int* perms,
                     const double* alpha, const double* in, double* out,
                     int nthreads) {
    layout_t L;
    int st = make_layout(ndim, extents, group_first, d, pairs, &L);
    if (st != ORACLE_OK) return st;
    if (nstages < 1 || nterms == NULL || in == NULL || out == NULL) return ORACLE_ERR_ARG;
    int total = 0;
    for (int k = 0; k < nstages; ++k) {
        if (nterms[k] < 0) return ORACLE_ERR_ARG;
        total += nterms[k];
    }
    if (total > 0 && alpha == NULL) return ORACLE_ERR_ARG;
    st = check_perms(d, total, perms);
    if (st != ORACLE_OK) return st;

    const int64_t nel = L.outer * L.group * L.inner;
    if (nel == 0) return ORACLE_OK;
    long double* a = (long double*)malloc((size_t)nel * sizeof(long double));
    long double* b = (long double*)malloc((size_t)nel * sizeof(long double));
    if (!a || !b) {
        free(a);
        free(b);
        return ORACLE_ERR_NOMEM;
    }
    for (int64_t e = 0; e < nel; ++e) a[e] = (long double)in[e];

    /* term offsets of every stage */
    int offs[64];
    if (nstages > 64) {
        free(a);
        free(b);
        return ORACLE_ERR_ARG;
    }
    offs[0] = 0;
    for (int k = 1; k < nstages; ++k) offs[k] = offs[k - 1] + nterms[k - 1];

    for (int s = 0; s < nstages; ++s) {
        /* forward: stage 0 (innermost factor) first; adjoint: last stage first */
        int k = adjoint ? (nstages - 1 - s) : s;
        if (adjoint)
            stage_adjoint_ld(&L, nterms[k], perms + offs[k] * d, alpha + offs[k], a, b,
                             nthreads);
        else
            stage_ld(&L, nterms[k], perms + offs[k] * d, alpha + offs[k], a, b, nthreads);
        long double* tmp = a;
        a = b;
        b = tmp;
    }
    for (int64_t e = 0; e < nel; ++e) out[e] = (double)a[e];
    free(a);
    free(b);
    return ORACLE_OK;
}

/* Out = S_K( ... S_1(In)), every S_k = sum_t alpha_t pi_t (Def. 3-4).
 * perms: sum(nterms) x d, 0-based; in/out: double, row-major, may alias
 * (the result is formed in a private buffer and copied at the end). */
int oracle_spinsum_chain(int ndim, const int64_t* extents, int group_first, int d,
                         int nstages, const int* nterms, const int* perms,
                         const double* alpha, const double* in, double* out,
                         int nthreads) {
    return run_chain(0, ndim, extents, group_first, d, 0, nstages, nterms, perms, alpha,
                     in, out, nthreads);
}

/* The same with the index-pair form selectable (pairs = 1: the d dims before
 * the group are permuted along with it). */
int oracle_spinsum_chain_ex(int ndim, const int64_t* extents, int group_first, int d,
                            int pairs, int nstages, const int* nterms, const int* perms,
                            const double* alpha, const double* in, double* out,
                            int nthreads) {
    return run_chain(0, ndim, extents, group_first, d, pairs != 0, nstages, nterms, perms,
                     alpha, in, out, nthreads);
}

/* Single stage convenience form. */
int oracle_spinsum(int ndim, const int64_t* extents, int group_first, int d,
                   int nterms, const int* perms, const double* alpha,
                   const double* in, double* out, int nthreads) {
    return run_chain(0, ndim, extents, group_first, d, 0, 1, &nterms, perms, alpha, in, out,
                     nthreads);
}

/* grad_in = S^T grad_out for the chain, S^T = S_1^T ( ... S_K^T (grad_out)). */
int oracle_spinsum_chain_adjoint(int ndim, const int64_t* extents, int group_first,
                                 int d, int nstages, const int* nterms,
                                 const int* perms, const double* alpha,
                                 const double* grad_out, double* grad_in,
                                 int nthreads) {
    return run_chain(1, ndim, extents, group_first, d, 0, nstages, nterms, perms, alpha,
                     grad_out, grad_in, nthreads);
}

int oracle_spinsum_chain_adjoint_ex(int ndim, const int64_t* extents, int group_first,
                                    int d, int pairs, int nstages, const int* nterms,
                                    const int* perms, const double* alpha,
                                    const double* grad_out, double* grad_in,
                                    int nthreads) {
    return run_chain(1, ndim, extents, group_first, d, pairs != 0, nstages, nterms, perms,
                     alpha, grad_out, grad_in, nthreads);
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
