/*
 * Plain C twin of oracle/fsi_oracle.py (same algorithm, for speed at d = 20).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py; never by the product library. It shares no
 * code, header or table generator with the HIP implementation.
 *
 * Computes the FSI closed form (paper Sec. 2.2, Eq. 3 + Eq. 4; weights Eq. 7)
 * by the paper's "Baseline" method (Sec. 4.6): a direct Moebius butterfly
 * followed by brute-force sums over every superset T of each output S.
 * The weight table W[s][t] (shape (l+1) x (d+1), row-major) is passed in; the
 * Python oracle builds it from exact rationals (W[s][s] = 1, W[s][t] = w(s,t)
 * for t > l and s >= 1, 0 otherwise).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC fsi_oracle_c.c -o liboracle.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* In-place Moebius butterfly over all d bit axes (Sec. 4.2 / Appendix B). */
void oracle_mobius(double *a, int d)
{
    const int64_t n = (int64_t)1 << d;
    for (int i = 0; i < d; ++i) {
        const int64_t bit = (int64_t)1 << i;
        for (int64_t m = 0; m < n; ++m)
            if (m & bit)
                a[m] -= a[m ^ bit];
    }
}

/*
 * E[k] = sum over supersets T of masks[k] of W[|S|][|T|] * a[T].
 * masks: n_out output masks; a: Moebius vector of length 2^d.
 * Supersets are enumerated as S | sub for every sub of the complement, in
 * ascending order of sub. nthreads <= 0 means one thread.
 */
void oracle_superset_sums(const double *a, int d, int l, const double *W,
                          const int64_t *masks, int64_t n_out, double *E,
                          int nthreads)
{
    const int64_t full = ((int64_t)1 << d) - 1;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
    #pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int64_t k = 0; k < n_out; ++k) {
        const int64_t S = masks[k];
        const int s = __builtin_popcountll((unsigned long long)S);
        const double *Wrow = W + (int64_t)s * (d + 1);
        const int64_t comp = full & ~S;
        double acc = 0.0;
        int64_t sub = 0;
        for (;;) {
            const int64_t T = S | sub;
            const int t = __builtin_popcountll((unsigned long long)T);
            acc += Wrow[t] * a[T];
            if (sub == comp) break;
            sub = (sub - comp) & comp; /* next subset of comp, ascending */
        }
        E[k] = acc;
    }
    (void)l;
}

/* Full oracle: copies v, runs the butterfly, then the superset sums. */
int oracle_fsi(const double *v, int d, int l, const double *W,
               const int64_t *masks, int64_t n_out, double *E, int nthreads)
{
    const int64_t n = (int64_t)1 << d;
    double *a = (double *)malloc(sizeof(double) * (size_t)n);
    if (!a) return 1;
    memcpy(a, v, sizeof(double) * (size_t)n);
    oracle_mobius(a, d);
    oracle_superset_sums(a, d, l, W, masks, n_out, E, nthreads);
    free(a);
    return 0;
}

/*
 * Exact variant for integer-valued v (e.g. the +/-1 vectors): the Moebius
 * transform in int64 (exact while |v| * 2^d < 2^63) and, for every output S,
 * the ranked superset sums A[k][t] = sum over supersets T of S with |T| = t
 * of a(T), also in int64. The caller combines E_S = a(S) +
 * sum_{t > l} w(|S|, t) A[k][t] in exact rational arithmetic.
 * A has n_out rows of d + 1 entries; a_S receives a(S) per output.
 */
int oracle_ranked_sums_int(const int64_t *v, int d, const int64_t *masks,
                           int64_t n_out, int64_t *A, int64_t *a_S, int nthreads)
{
    const int64_t n = (int64_t)1 << d;
    const int64_t full = n - 1;
    int64_t *a = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!a) return 1;
    memcpy(a, v, sizeof(int64_t) * (size_t)n);
    for (int i = 0; i < d; ++i) {
        const int64_t bit = (int64_t)1 << i;
        for (int64_t m = 0; m < n; ++m)
            if (m & bit)
                a[m] -= a[m ^ bit];
    }
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
    #pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int64_t k = 0; k < n_out; ++k) {
        const int64_t S = masks[k];
        int64_t *row = A + k * (d + 1);
        for (int t = 0; t <= d; ++t) row[t] = 0;
        const int64_t comp = full & ~S;
        int64_t sub = 0;
        for (;;) {
            const int64_t T = S | sub;
            row[__builtin_popcountll((unsigned long long)T)] += a[T];
            if (sub == comp) break;
            sub = (sub - comp) & comp;
        }
        a_S[k] = a[S];
    }
    free(a);
    (void)nthreads;
    return 0;
}
