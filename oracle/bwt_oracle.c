/*
 * bwt_oracle.c -- plain, slow, obviously correct CPU oracle for the BWT of a
 * string set (Pantaleoni, "A massively parallel algorithm for constructing the
 * BWT of large string sets", arXiv:1410.0562).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no code with the GPU path.
 *
 * Text encoding used throughout: one byte per symbol, 0 = a terminator, and
 * 1..4 = the bases A,C,G,T in alphabet order.  A string set S_0..S_{m-1} is
 * laid out as T = S_0 $_0 S_1 $_1 ... S_{m-1} $_{m-1} (Section 2, the
 * definition of the BWT of a string set), so every terminator is a 0 byte and
 * the i-th 0 byte from the left is $_i.
 *
 * Order (Section 2): $_0 < $_1 < ... < $_{m-1} < A < C < G < T.  Two suffixes
 * are compared symbol by symbol; at the first pair that differs the byte value
 * decides; if both walks reach a terminator at the same offset, the terminators
 * are distinct symbols and the one further left is the smaller (its index is
 * lower).  A walk never passes a terminator, so it never reads past T[n-1],
 * which is always $_{m-1}.
 *
 * Functions (all single-threaded unless stated):
 *   oracle_sa            suffix array by comparison sort (definition of SA,
 *                        Section 2)
 *   oracle_sa_threads    the same comparison sort, run as `threads` sorted
 *                        runs merged pairwise (same comparator, same result)
 *   oracle_bwt           B[i] = T[(SA[i]-1) mod n]   (Eq. 1)
 *   oracle_count_smaller number of suffixes of T smaller than T^p, by brute
 *                        force against every suffix (rank of one row, O(n))
 *   oracle_lf_invert     walks B backwards from row j with C[c] + rank(c,r),
 *                        the LF step of Lemma 1 applied inside one BWT; spells
 *                        each string reversed.  Used as an invariant check.
 *   oracle_count_old_smaller  brute-force definition of what ComputeRanks
 *                        returns: for a new suffix, the number of old suffixes
 *                        smaller than it (hypothesis of Lemma 1)
 *   oracle_pattern_rows  for a pattern P over the bases, by a scan over every
 *                        suffix: how many suffixes are smaller than P and how
 *                        many start with P (the rows of the sorted suffixes
 *                        prefixed by P, i.e. the FM-index interval of P)
 *
 * What ComputeRanks returns for a whole block is computed in oracle.py from
 * its definition (old suffixes smaller than each new one, read off one suffix
 * array of the old and new text together); nothing here walks LF steps to
 * produce it.
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Compare suffixes a and b of T under the order stated above. */
static int cmp_suffix_at(const uint8_t *T, uint64_t a, uint64_t b)
{
    if (a == b) return 0;
    for (uint64_t t = 0;; ++t) {
        uint8_t x = T[a + t], y = T[b + t];
        if (x != y) return x < y ? -1 : 1;
        if (x == 0) return (a + t) < (b + t) ? -1 : 1;
    }
}

static int qsort_cmp(const void *pa, const void *pb, void *text)
{
    uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    return cmp_suffix_at((const uint8_t *)text, a, b);
}

/* Suffix array of T[0..n) (T[n-1] must be 0). */
void oracle_sa(const uint8_t *T, uint64_t n, uint64_t *sa)
{
    for (uint64_t i = 0; i < n; ++i) sa[i] = i;
    qsort_r(sa, (size_t)n, sizeof(uint64_t), qsort_cmp, (void *)T);
}

/* ---- the same sort on several threads ----------------------------------
 * The positions are cut into `threads` contiguous runs; each run is sorted
 * by qsort_r with the comparator above, then neighbouring runs are merged
 * pairwise, round by round, until one run is left.  The suffixes are all
 * distinct, so the merged order is the one oracle_sa gives. */
struct sort_job {
    const uint8_t *T;
    uint64_t *a;
    uint64_t n;
};

static void *sort_run(void *p)
{
    struct sort_job *j = (struct sort_job *)p;
    qsort_r(j->a, (size_t)j->n, sizeof(uint64_t), qsort_cmp, (void *)j->T);
    return NULL;
}

struct merge_job {
    const uint8_t *T;
    const uint64_t *x, *y;
    uint64_t nx, ny;
    uint64_t *out;
};

static void *merge_runs(void *p)
{
    struct merge_job *j = (struct merge_job *)p;
    uint64_t i = 0, k = 0, o = 0;
    while (i < j->nx && k < j->ny) {
        if (cmp_suffix_at(j->T, j->x[i], j->y[k]) < 0) j->out[o++] = j->x[i++];
        else j->out[o++] = j->y[k++];
    }
    while (i < j->nx) j->out[o++] = j->x[i++];
    while (k < j->ny) j->out[o++] = j->y[k++];
    return NULL;
}

/* Returns 0, or -1 when memory or threads could not be had (sa is then
 * unspecified). */
int oracle_sa_threads(const uint8_t *T, uint64_t n, uint64_t *sa, int threads)
{
    if (threads < 1) threads = 1;
    if ((uint64_t)threads > n) threads = n ? (int)n : 1;
    if (threads == 1) {
        oracle_sa(T, n, sa);
        return 0;
    }
    for (uint64_t i = 0; i < n; ++i) sa[i] = i;
    uint64_t *bound = (uint64_t *)malloc(sizeof(uint64_t) * (threads + 1));
    uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
    struct sort_job *sj = (struct sort_job *)malloc(sizeof(struct sort_job) * threads);
    struct merge_job *mj = (struct merge_job *)malloc(sizeof(struct merge_job) * threads);
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * threads);
    int rc = -1;
    if (!bound || !tmp || !sj || !mj || !th) goto done;
    for (int t = 0; t <= threads; ++t) bound[t] = n * (uint64_t)t / (uint64_t)threads;
    for (int t = 0; t < threads; ++t) {
        sj[t].T = T;
        sj[t].a = sa + bound[t];
        sj[t].n = bound[t + 1] - bound[t];
        if (pthread_create(&th[t], NULL, sort_run, &sj[t]) != 0) {
            for (int u = 0; u < t; ++u) pthread_join(th[u], NULL);
            goto done;
        }
    }
    for (int t = 0; t < threads; ++t) pthread_join(th[t], NULL);
    {
        uint64_t *src = sa, *dst = tmp;
        int runs = threads;
        while (runs > 1) {
            int pairs = runs / 2, started = 0, ok = 1;
            for (int q = 0; q < pairs; ++q) {
                uint64_t a0 = bound[2 * q], a1 = bound[2 * q + 1], a2 = bound[2 * q + 2];
                mj[q].T = T;
                mj[q].x = src + a0;
                mj[q].nx = a1 - a0;
                mj[q].y = src + a1;
                mj[q].ny = a2 - a1;
                mj[q].out = dst + a0;
                if (pthread_create(&th[q], NULL, merge_runs, &mj[q]) != 0) {
                    ok = 0;
                    break;
                }
                ++started;
            }
            for (int q = 0; q < started; ++q) pthread_join(th[q], NULL);
            if (!ok) goto done;
            if (runs & 1) {  /* the odd last run is carried over as it is */
                uint64_t a0 = bound[runs - 1], a1 = bound[runs];
                memcpy(dst + a0, src + a0, (size_t)(a1 - a0) * sizeof(uint64_t));
            }
            int nr = 0;
            for (int q = 0; q < runs; q += 2) bound[nr++] = bound[q];
            bound[nr] = n;
            runs = nr;
            uint64_t *sw = src;
            src = dst;
            dst = sw;
        }
        if (src != sa) memcpy(sa, src, (size_t)n * sizeof(uint64_t));
    }
    rc = 0;
done:
    free(bound);
    free(tmp);
    free(sj);
    free(mj);
    free(th);
    return rc;
}

/* Eq. 1: B[i] = T[(SA[i]-1) mod n], written as ASCII with every terminator
 * printed as '$'. */
void oracle_bwt(const uint8_t *T, uint64_t n, const uint64_t *sa, uint8_t *B)
{
    static const char ascii[5] = {'$', 'A', 'C', 'G', 'T'};
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t prev = (sa[i] + n - 1) % n;
        B[i] = (uint8_t)ascii[T[prev]];
    }
}

/* Number of suffixes q of T with T^q < T^p: one row of the suffix array,
 * computed without sorting anything. */
uint64_t oracle_count_smaller(const uint8_t *T, uint64_t n, uint64_t p)
{
    uint64_t c = 0;
    for (uint64_t q = 0; q < n; ++q)
        if (cmp_suffix_at(T, q, p) < 0) ++c;
    return c;
}

/* Symbol code of an ASCII BWT byte: '$'->0, A->1, C->2, G->3, T->4, else 255. */
static int code_of(uint8_t ch)
{
    switch (ch) {
    case '$': return 0;
    case 'A': return 1;
    case 'C': return 2;
    case 'G': return 3;
    case 'T': return 4;
    default: return 255;
    }
}

/* Occurrence table used by the LF walks below: occ[r*5 + c] = number of code c
 * in B[0..r) for r a multiple of OCC_STEP; the rest is counted by a scan. */
#define OCC_STEP 64

static uint64_t *build_occ(const uint8_t *B, uint64_t n)
{
    uint64_t ns = n / OCC_STEP + 1;
    uint64_t *occ = (uint64_t *)calloc((size_t)ns * 5, sizeof(uint64_t));
    if (!occ) return NULL;
    uint64_t run[5] = {0, 0, 0, 0, 0};
    for (uint64_t i = 0; i <= n; ++i) {
        if (i % OCC_STEP == 0) memcpy(occ + (i / OCC_STEP) * 5, run, sizeof run);
        if (i < n) run[code_of(B[i])]++;
    }
    return occ;
}

/* rank(c, k, B) of Eq. 2 from the sampled table plus a short scan. */
static uint64_t occ_rank(const uint8_t *B, const uint64_t *occ, int c, uint64_t k)
{
    uint64_t s = k / OCC_STEP;
    uint64_t r = occ[s * 5 + c];
    for (uint64_t i = s * OCC_STEP; i < k; ++i)
        if (code_of(B[i]) == c) ++r;
    return r;
}

/*
 * Invert the BWT B (ASCII, n symbols, m terminators) for the rows listed in
 * `rows`: from row j, emit B[r] and step r <- C[B[r]] + rank(B[r], r, B) until
 * B[r] is '$'.  Row j of the BWT of a string set is the suffix $_j..., whose
 * preceding symbol is the last symbol of S_j, so the walk spells S_j reversed.
 * Output for row rows[t] goes to out + out_off[t] (ASCII, reversed string),
 * with at most out_off[t+1]-out_off[t] symbols; lens[t] receives the walk
 * length (or UINT64_MAX when the walk overran its slot or hit a bad byte).
 * Returns 0, or -1 on allocation failure.
 */
int oracle_lf_invert(const uint8_t *B, uint64_t n, const uint64_t *rows,
                     uint64_t nrows, const uint64_t *out_off, uint8_t *out,
                     uint64_t *lens)
{
    uint64_t *occ = build_occ(B, n);
    if (!occ) return -1;
    uint64_t cnt[5];
    for (int c = 0; c < 5; ++c) cnt[c] = occ_rank(B, occ, c, n);
    uint64_t C[5];
    C[0] = 0;
    for (int c = 1; c < 5; ++c) C[c] = C[c - 1] + cnt[c - 1];
    for (uint64_t t = 0; t < nrows; ++t) {
        uint64_t r = rows[t], cap = out_off[t + 1] - out_off[t], len = 0;
        for (;;) {
            if (r >= n) { len = UINT64_MAX; break; }
            int c = code_of(B[r]);
            if (c == 255) { len = UINT64_MAX; break; }
            if (c == 0) break;
            if (len == cap) { len = UINT64_MAX; break; }
            out[out_off[t] + len] = B[r];
            ++len;
            r = C[c] + occ_rank(B, occ, c, r);
        }
        lens[t] = len;
    }
    free(occ);
    return 0;
}

/*
 * What ComputeRanks must return, from the definition: the number of old
 * suffixes smaller than the new suffix starting at text position p.  The old
 * and new strings are compared inside one global text G = old strings then new
 * strings (the order in which their terminators are numbered), so this is
 * simply a count over the first n_old positions of G.
 */
uint64_t oracle_count_old_smaller(const uint8_t *G, uint64_t n_old, uint64_t p)
{
    uint64_t c = 0;
    for (uint64_t q = 0; q < n_old; ++q)
        if (cmp_suffix_at(G, q, p) < 0) ++c;
    return c;
}

/*
 * The rows of the suffix array whose suffix starts with P (codes 1..4, L >= 0
 * symbols): *below = the number of suffixes smaller than P, where a suffix
 * that reaches a terminator before it differs from P is smaller (a terminator
 * is smaller than every base), and *count = the number of suffixes that start
 * with P, i.e. the occurrences of P in the strings (P holds no terminator, so
 * an occurrence never crosses one).  Those suffixes are consecutive in sorted
 * order, so they are the rows [below, below + count).  One scan over all n
 * suffixes, stopping each comparison at the first difference.
 */
void oracle_pattern_rows(const uint8_t *T, uint64_t n, const uint8_t *P, uint64_t L,
                         uint64_t *below, uint64_t *count)
{
    uint64_t lo = 0, cnt = 0;
    for (uint64_t q = 0; q < n; ++q) {
        int cmp = 0;
        for (uint64_t t = 0; t < L; ++t) {
            uint8_t x = T[q + t];
            if (x != P[t]) {
                cmp = x < P[t] ? -1 : 1;
                break;
            }
            /* x == P[t] is a base, so the walk has not met a terminator and
             * T[q + t + 1] exists (T ends with one) */
        }
        if (cmp < 0) ++lo;
        else if (cmp == 0) ++cnt;
    }
    *below = lo;
    *count = cnt;
}
