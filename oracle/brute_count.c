/* Brute-force clause counting for large n (oracle, test infrastructure only).
 *
 * For every assignment z in [0, 2^n) this counts the clauses that z leaves
 * unsatisfied, by the definition of App. B: with lit = 2*var + neg, a literal
 * is false iff bit var of z equals neg; a clause is unsatisfied iff all three
 * of its literals are false. It then tallies the level histogram
 * N_k = #{z : C(z) = k} (App. C, "Optimization"). Plain loops, no blocking;
 * threads split the z range and each keeps its own histogram.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int clause_cost(uint64_t z, int m, const int32_t *lits) {
    int c = 0;
    for (int i = 0; i < m; ++i) {
        int unsat = 1;
        for (int j = 0; j < 3; ++j) {
            int lit = lits[3 * i + j];
            uint64_t bit = (z >> (lit >> 1)) & 1u;
            if (bit != (uint64_t)(lit & 1)) { unsat = 0; break; }
        }
        c += unsat;
    }
    return c;
}

/* hist[0..m] receives N_k. Returns 0, or -1 on bad arguments. */
int oracle_level_histogram(int n, int m, const int32_t *lits, uint64_t *hist) {
    if (n < 1 || n > 40 || m < 1 || m > 255 || !lits || !hist) return -1;
    memset(hist, 0, sizeof(uint64_t) * (size_t)(m + 1));
    const uint64_t N = (uint64_t)1 << n;
#pragma omp parallel
    {
        uint64_t local[256];
        memset(local, 0, sizeof(local));
#pragma omp for schedule(static)
        for (int64_t z = 0; z < (int64_t)N; ++z)
            local[clause_cost((uint64_t)z, m, lits)] += 1;
#pragma omp critical
        for (int k = 0; k <= m; ++k) hist[k] += local[k];
    }
    return 0;
}

/* out[i] = C(z0 + i) for i in [0, count). */
int oracle_cost_range(int n, int m, const int32_t *lits, uint64_t z0, uint64_t count,
                      uint8_t *out) {
    if (n < 1 || n > 40 || m < 1 || m > 255 || !lits || !out) return -1;
    if (z0 + count > ((uint64_t)1 << n)) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)count; ++i)
        out[i] = (uint8_t)clause_cost(z0 + (uint64_t)i, m, lits);
    return 0;
}
