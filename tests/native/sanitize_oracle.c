/* The CPU oracle's C routines on small inputs, built with AddressSanitizer
 * and UndefinedBehaviorSanitizer; checks a few exact values:
 *  - the all-ones triangle sums n (n-1) (n-2) ordered distinct triples;
 *  - the exact integer path agrees with the fp64 path;
 *  - the rank-1 all-ones low-rank DP gives the same count;
 *  - a 5-cycle's closed walks of length 5 (tr A^5) equal 10. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_sum_tuples(int m, int ne, const int *eu, const int *ev, const double *const *T, long n,
                      int distinct, long item_lo, long item_hi, double *out);
int oracle_sum_tuples_i64(int m, int ne, const int *eu, const int *ev, const int64_t *const *T, long n,
                          int distinct, long lo, long hi, int64_t *out_hi, uint64_t *out_lo);
int oracle_lowrank_dp(int m, int ne, const int *eu, const int *ev, long n, int r,
                      const double *const *F, const double *const *G, double *out);
int oracle_cycle_walks(long n, const int64_t *rowptr, const int32_t *col, int64_t *out);

int main(void) {
    enum { N = 11 };
    int fails = 0;
    double *T = malloc(sizeof(double) * N * N);
    int64_t *Ti = malloc(sizeof(int64_t) * N * N);
    for (int i = 0; i < N * N; ++i) {
        T[i] = 1.0;
        Ti[i] = 1;
    }
    const int eu[3] = {0, 1, 2}, ev[3] = {1, 2, 0};
    const double *Ts[3] = {T, T, T};
    const int64_t *Tis[3] = {Ti, Ti, Ti};
    double u = 0;
    if (oracle_sum_tuples(3, 3, eu, ev, Ts, N, 1, 0, (long)N * N, &u) || u != N * (N - 1) * (N - 2)) ++fails;
    int64_t hi = 0;
    uint64_t lo = 0;
    if (oracle_sum_tuples_i64(3, 3, eu, ev, Tis, N, 1, 0, N, &hi, &lo) || hi != 0 || (double)lo != u) ++fails;
    double *F = malloc(sizeof(double) * N);
    for (int i = 0; i < N; ++i) F[i] = 1.0;
    const double *Fs[3] = {F, F, F};
    double d = 0;
    if (oracle_lowrank_dp(3, 3, eu, ev, N, 1, Fs, Fs, &d) || d != u) ++fails;
    /* the 5-cycle graph as CSR */
    int64_t rowptr[6];
    int32_t col[10];
    for (int v = 0; v < 5; ++v) {
        rowptr[v] = 2 * v;
        col[2 * v] = (v + 4) % 5;
        col[2 * v + 1] = (v + 1) % 5;
    }
    rowptr[5] = 10;
    int64_t walks[6] = {0, 0, 0, 0, 0, 0};
    if (oracle_cycle_walks(5, rowptr, col, walks) || walks[0] != 0 || walks[1] != 10) ++fails;
    if (oracle_sum_tuples(3, 3, eu, ev, Ts, N, 1, 5, 3, &u) != -1) ++fails;  /* bad range rejected */
    free(T);
    free(Ti);
    free(F);
    printf("sanitized oracle run: %d failures\n", fails);
    return fails ? 1 : 0;
}
