/*
 * CPU oracle for the exact Hamming kNN graph -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the checker, not the product. Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg load it. It shares no code,
 * header or table with the GPU library.
 *
 * What it computes (the plain definition, no blocking or reordering):
 *
 *   The data are binary codes y_i in {0,1}^b (Sec. 3.1). The distance between
 *   two codes is the Hamming distance (Sec. 3 notation, "l_h"), i.e. the number
 *   of bit positions in which they differ; on {0,1} vectors it equals the
 *   squared Euclidean distance of Eq. 1. For row i the kNN set B(l_i)
 *   (Sec. 3 notation) is taken exhaustively, the way the reduce step searches a
 *   partition and the way the paper's "binary linear search" ground truth is
 *   defined (Sec. 3.2 and Sec. 4.5):
 *
 *     row i = the first K elements of { (ham(i, j), j) : j in C, j != i }
 *             in lexicographic order (distance, then index),
 *
 *   where C is the candidate column range [c0, c1). Readings where the paper
 *   is silent: a point is not its own neighbour; ties go to the smaller index;
 *   rows are ascending; with fewer than K candidates the row is padded with
 *   index 0xFFFFFFFF and distance 0xFFFF.
 *
 * How: for one row, every candidate distance is computed with a word-by-word
 * popcount of the XOR, then a stable counting sort on the distance (a textbook
 * sort on small integer keys; candidates are visited in increasing index, so
 * each distance bucket is in index order) is cut at K.
 *
 * Parity pins: a pure-Python per-bit brute force on tiny inputs, the hypercube
 * closed form, degenerate inputs and invariants (tests of the oracle).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_NO_IDX 0xFFFFFFFFu
#define ORACLE_NO_DIST 0xFFFFu

static unsigned hamming_words(const uint64_t *a, const uint64_t *b, unsigned words)
{
    unsigned d = 0;
    for (unsigned w = 0; w < words; ++w)
        d += (unsigned)__builtin_popcountll(a[w] ^ b[w]);
    return d;
}

/* Number of OpenMP threads the oracle will use (1 without OpenMP). */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0)
        omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/*
 * Exact kNN rows against the candidate columns [c0, c1) of the same code set.
 *   codes    [n][words] uint64, little-endian bit order
 *   rows     query row ids (NULL: rows 0..nrows-1)
 *   out_idx  [nrows][K] uint32, out_dist [nrows][K] uint16
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int oracle_knn_rows(const uint64_t *codes, uint32_t n, uint32_t words, uint32_t K,
                    uint32_t c0, uint32_t c1, const uint32_t *rows, uint32_t nrows,
                    uint32_t *out_idx, uint16_t *out_dist)
{
    if (!codes || !out_idx || !out_dist || words == 0 || K == 0 || c0 > c1 || c1 > n)
        return -1;
    const unsigned bits = 64u * words;
    int failed = 0;
#pragma omp parallel
    {
        uint32_t *count = (uint32_t *)malloc((bits + 1) * sizeof(uint32_t));
        uint32_t *pos = (uint32_t *)malloc((bits + 1) * sizeof(uint32_t));
        uint16_t *dist = (uint16_t *)malloc((size_t)(c1 - c0 + 1) * sizeof(uint16_t));
        if (!count || !pos || !dist) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < (int64_t)nrows; ++r) {
            if (failed)
                continue;
            const uint32_t i = rows ? rows[r] : (uint32_t)r;
            uint32_t *oi = out_idx + (size_t)r * K;
            uint16_t *od = out_dist + (size_t)r * K;
            for (uint32_t k = 0; k < K; ++k) {
                oi[k] = ORACLE_NO_IDX;
                od[k] = ORACLE_NO_DIST;
            }
            if (i >= n)
                continue;
            const uint64_t *qi = codes + (size_t)i * words;
            memset(count, 0, (bits + 1) * sizeof(uint32_t));
            for (uint32_t j = c0; j < c1; ++j) {
                if (j == i)
                    continue;
                unsigned d = hamming_words(qi, codes + (size_t)j * words, words);
                dist[j - c0] = (uint16_t)d;
                count[d]++;
            }
            /* bucket start positions; stop assigning once K slots are used */
            uint32_t start = 0;
            for (unsigned d = 0; d <= bits; ++d) {
                pos[d] = start;
                start += count[d];
            }
            for (uint32_t j = c0; j < c1; ++j) {
                if (j == i)
                    continue;
                unsigned d = dist[j - c0];
                uint32_t p = pos[d]++;
                if (p < K) {
                    oi[p] = j;
                    od[p] = (uint16_t)d;
                }
            }
        }
        free(count);
        free(pos);
        free(dist);
    }
    return failed ? -1 : 0;
}

/* Hamming distance of explicit pairs (a[t], b[t]) -- for certificate checks. */
void oracle_pair_distances(const uint64_t *codes, uint32_t words, const uint32_t *a,
                           const uint32_t *b, uint64_t npairs, uint16_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < (int64_t)npairs; ++t)
        out[t] = (uint16_t)hamming_words(codes + (size_t)a[t] * words,
                                         codes + (size_t)b[t] * words, words);
}
