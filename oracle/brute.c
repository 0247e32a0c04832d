/*
 * ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Brute-force definition of induced subgraph counts: for every k-subset S of
 * vertices (k = 3, 4 or 5), read the induced edge set as a bitmask over the
 * C(k,2) vertex pairs and look up its isomorphism class in a table supplied by
 * the caller (the table is built in Python from the pattern drawings).  This is
 * the plain definition the paper starts from (Sec. 2.1): C_X is the number of
 * vertex subsets whose induced subgraph is X.
 *
 * Pair bit order for a subset s0 < s1 < ... : (0,1),(0,2),...,(0,k-1),(1,2),...
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* adjacency as bitset rows, n <= 4096 */
int brute_count(int32_t n, const int32_t *rp, const int32_t *ci, int k,
                const int32_t *lut, int nclass, int threads, uint64_t *counts) {
    if (k < 3 || k > 5 || n > 4096) return -1;
    if (threads > 0) omp_set_num_threads(threads);
    int words = (n + 63) / 64;
    uint64_t *adj = (uint64_t *)calloc((size_t)n * words + 1, sizeof(uint64_t));
    if (!adj) return -1;
    for (int32_t u = 0; u < n; u++)
        for (int32_t p = rp[u]; p < rp[u + 1]; p++) {
            int32_t v = ci[p];
            adj[(size_t)u * words + (v >> 6)] |= 1ULL << (v & 63);
        }
#define A(u, v) ((adj[(size_t)(u) * words + ((v) >> 6)] >> ((v) & 63)) & 1ULL)
    memset(counts, 0, sizeof(uint64_t) * nclass);
    #pragma omp parallel
    {
        uint64_t *local = (uint64_t *)calloc((size_t)nclass, sizeof(uint64_t));
        #pragma omp for schedule(dynamic, 1)
        for (int32_t a = 0; a < n; a++) {
            for (int32_t b = a + 1; b < n; b++) {
                unsigned mab = (unsigned)A(a, b);
                for (int32_t c = b + 1; c < n; c++) {
                    unsigned mc = mab | (unsigned)A(a, c) << 1;
                    if (k == 3) { local[lut[mc | (unsigned)A(b, c) << 2]]++; continue; }
                    for (int32_t d = c + 1; d < n; d++) {
                        if (k == 4) {
                            /* pairs: 01 02 03 12 13 23 */
                            unsigned mk = mc | (unsigned)A(a, d) << 2 | (unsigned)A(b, c) << 3 |
                                          (unsigned)A(b, d) << 4 | (unsigned)A(c, d) << 5;
                            local[lut[mk]]++;
                            continue;
                        }
                        /* k == 5, pairs: 01 02 03 04 12 13 14 23 24 34 */
                        unsigned md = mc | (unsigned)A(a, d) << 2 | (unsigned)A(b, c) << 4 |
                                      (unsigned)A(b, d) << 5 | (unsigned)A(c, d) << 7;
                        for (int32_t e = d + 1; e < n; e++) {
                            unsigned mk = md | (unsigned)A(a, e) << 3 | (unsigned)A(b, e) << 6 |
                                          (unsigned)A(c, e) << 8 | (unsigned)A(d, e) << 9;
                            local[lut[mk]]++;
                        }
                    }
                }
            }
        }
        #pragma omp critical
        for (int c = 0; c < nclass; c++) counts[c] += local[c];
        free(local);
    }
#undef A
    free(adj);
    return 0;
}
