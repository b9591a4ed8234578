/*
 * Definitional CPU oracle for multi-string BWT construction, SA-interval
 * counting and SMEM finding (Li, "BWT construction and search at the terabase
 * scale", arXiv 2409.00613).
 *
 * THIS IS TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg call it. The GPU library never links, loads or
 * calls anything here, and nothing here shares code with the GPU library.
 *
 * Every routine computes the plain definition, slowly:
 *   - orc_expand       double-strand string list (Sec. 2.5, the DS concatenation)
 *   - orc_bwt          suffix array by comparison sort of every suffix of the
 *                      sentinel-terminated concatenation, then B[i] = T[S(i)-1]
 *                      (Sec. 2.1; the m+5 integer alphabet of Sec. 2.2)
 *   - orc_verify       inverse BWT: LF-walk every string back out of a candidate
 *                      BWT (the LF relation of Sec. 2.1 / Table 1); also in
 *                      parts (orc_verifier_new / _walk / _free) for lists too
 *                      large to walk in one call
 *   - orc_count        SA interval [lo, hi) of a pattern by scanning every
 *                      suffix (Sec. 2.3 definition of lo/occ/hi)
 *   - orc_sa_interval  the same interval by binary search over a sorted SA
 *   - orc_smem         SMEMs of length >= min_len occurring >= min_occ times,
 *                      from the definition of Sec. 2.6 (see the function)
 *
 * Symbol codes: $=0 A=1 C=2 G=3 T=4 N=5 (the order $ < A < C < G < T < N of
 * Sec. 2.2). All positions and counts are int64.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_THREADS 256

/* ------------------------------------------------------------------------ */
/* Alphabet                                                                   */
/* ------------------------------------------------------------------------ */

static int orc_code_of(uint8_t ch)
{
    switch (ch) {
    case 'A': case 'a': return 1;
    case 'C': case 'c': return 2;
    case 'G': case 'g': return 3;
    case 'T': case 't': return 4;
    case 'N': case 'n': return 5;
    default: return -1;
    }
}

/* Watson-Crick complement on codes (Sec. 2.5): $->$, A<->T, C<->G, N->N. */
static uint8_t orc_comp(uint8_t c)
{
    static const uint8_t tab[6] = {0, 4, 3, 2, 1, 5};
    return tab[c];
}

/*
 * Encode ASCII strings and expand them to the ordered list
 * P0, rc(P0), P1, rc(P1), ... when both != 0 (Sec. 2.5), or P0, P1, ...
 * otherwise. codes receives the concatenated strands without sentinels,
 * lens_out one length per strand. Returns 0, or -1 on a byte outside
 * ACGTNacgtn, or -2 on a string of length 0 unless allow_empty (patterns
 * may be empty; strings of the text may not).
 */
int orc_expand(const uint8_t *seq, const int64_t *lens, int64_t m_in, int both,
               int allow_empty, uint8_t *codes, int64_t *lens_out)
{
    int64_t in = 0, out = 0, s = 0;
    for (int64_t j = 0; j < m_in; ++j) {
        int64_t L = lens[j];
        if (L < 0 || (L == 0 && !allow_empty)) return -2;
        for (int64_t t = 0; t < L; ++t) {
            int c = orc_code_of(seq[in + t]);
            if (c < 0) return -1;
            codes[out + t] = (uint8_t)c;
        }
        lens_out[s++] = L;
        if (both) {
            for (int64_t t = 0; t < L; ++t)
                codes[out + L + t] = orc_comp(codes[out + L - 1 - t]);
            lens_out[s++] = L;
            out += 2 * L;
        } else {
            out += L;
        }
        in += L;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The concatenated text T over the m+5 integer alphabet (Sec. 2.2)           */
/* ------------------------------------------------------------------------ */

/*
 * T = P_0 $_0 P_1 $_1 ... P_{m-1} $_{m-1} with $_0 < ... < $_{m-1} < A < C < G
 * < T < N. Encoded as int32: sentinel $_j -> j, base code c (1..5) -> m-1+c.
 * Two distinct suffixes always differ at or before the first sentinel either
 * reaches, because sentinel values are unique.
 */
static int32_t *orc_make_text(const uint8_t *codes, const int64_t *lens, int64_t m,
                              int64_t *n_out)
{
    int64_t n = 0;
    for (int64_t j = 0; j < m; ++j) n += lens[j] + 1;
    int32_t *T = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!T) return NULL;
    int64_t p = 0, q = 0;
    for (int64_t j = 0; j < m; ++j) {
        for (int64_t t = 0; t < lens[j]; ++t) T[p++] = (int32_t)(m - 1 + codes[q++]);
        T[p++] = (int32_t)j;
    }
    *n_out = n;
    return T;
}

static int orc_cmp_suffix(const int32_t *T, int64_t a, int64_t b)
{
    if (a == b) return 0;
    for (;;) {
        int32_t x = T[a], y = T[b];
        if (x != y) return x < y ? -1 : 1;
        ++a;
        ++b;
    }
}

/* top-down merge sort of suffix start positions */
static void orc_msort(const int32_t *T, int64_t *a, int64_t *tmp, int64_t n)
{
    if (n < 2) return;
    if (n <= 16) {
        for (int64_t i = 1; i < n; ++i) {
            int64_t v = a[i], j = i;
            while (j > 0 && orc_cmp_suffix(T, a[j - 1], v) > 0) { a[j] = a[j - 1]; --j; }
            a[j] = v;
        }
        return;
    }
    int64_t h = n / 2;
    orc_msort(T, a, tmp, h);
    orc_msort(T, a + h, tmp + h, n - h);
    int64_t i = 0, j = h, k = 0;
    while (i < h && j < n) tmp[k++] = (orc_cmp_suffix(T, a[j], a[i]) < 0) ? a[j++] : a[i++];
    while (i < h) tmp[k++] = a[i++];
    while (j < n) tmp[k++] = a[j++];
    memcpy(a, tmp, (size_t)n * sizeof(int64_t));
}

typedef struct {
    const int32_t *T;
    int64_t *a, *tmp;
    int64_t n;
} orc_sort_job;

static void *orc_sort_worker(void *p)
{
    orc_sort_job *jb = (orc_sort_job *)p;
    orc_msort(jb->T, jb->a, jb->tmp, jb->n);
    return NULL;
}

typedef struct {
    const int32_t *T;
    const int64_t *src;
    int64_t *dst;
    int64_t a0, a1, b1; /* merge src[a0,a1) with src[a1,b1) into dst[a0,b1) */
} orc_merge_job;

static void *orc_merge_worker(void *p)
{
    orc_merge_job *jb = (orc_merge_job *)p;
    int64_t i = jb->a0, j = jb->a1, k = jb->a0;
    while (i < jb->a1 && j < jb->b1)
        jb->dst[k++] = (orc_cmp_suffix(jb->T, jb->src[j], jb->src[i]) < 0) ? jb->src[j++] : jb->src[i++];
    while (i < jb->a1) jb->dst[k++] = jb->src[i++];
    while (j < jb->b1) jb->dst[k++] = jb->src[j++];
    return NULL;
}

/* Sort every suffix start of T (the suffix array S of Sec. 2.1). */
static int orc_suffix_sort(const int32_t *T, int64_t n, int nthreads, int64_t *S)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > ORC_MAX_THREADS) nthreads = ORC_MAX_THREADS;
    if (n < (int64_t)nthreads * 1024) nthreads = 1;
    int64_t *tmp = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!tmp) return -1;
    for (int64_t i = 0; i < n; ++i) S[i] = i;
    int64_t bounds[ORC_MAX_THREADS + 1];
    for (int t = 0; t <= nthreads; ++t) bounds[t] = n * t / nthreads;
    pthread_t th[ORC_MAX_THREADS];
    orc_sort_job jobs[ORC_MAX_THREADS];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].T = T;
        jobs[t].a = S + bounds[t];
        jobs[t].tmp = tmp + bounds[t];
        jobs[t].n = bounds[t + 1] - bounds[t];
        pthread_create(&th[t], NULL, orc_sort_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    /* pairwise merge rounds of the sorted runs */
    int runs = nthreads;
    int64_t *src = S, *dst = tmp;
    while (runs > 1) {
        orc_merge_job mj[ORC_MAX_THREADS];
        int nj = 0, nr = 0;
        int64_t nb[ORC_MAX_THREADS + 1];
        for (int r = 0; r < runs; r += 2) {
            if (r + 1 < runs) {
                mj[nj].T = T; mj[nj].src = src; mj[nj].dst = dst;
                mj[nj].a0 = bounds[r]; mj[nj].a1 = bounds[r + 1]; mj[nj].b1 = bounds[r + 2];
                pthread_create(&th[nj], NULL, orc_merge_worker, &mj[nj]);
                ++nj;
            } else {
                memcpy(dst + bounds[r], src + bounds[r],
                       (size_t)(bounds[r + 1] - bounds[r]) * sizeof(int64_t));
            }
            nb[nr++] = bounds[r];
        }
        for (int t = 0; t < nj; ++t) pthread_join(th[t], NULL);
        nb[nr] = n;
        for (int r = 0; r <= nr; ++r) bounds[r] = nb[r];
        runs = nr;
        int64_t *sw = src; src = dst; dst = sw;
    }
    if (src != S) memcpy(S, src, (size_t)n * sizeof(int64_t));
    free(tmp);
    return 0;
}

/*
 * BWT of the ordered list (Sec. 2.1): sort all n = sum(L_j + 1) suffixes of T
 * and output B[i] = T[S(i) - 1] with T[-1] = T[n-1]; every sentinel prints as
 * code 0. If S_out is not NULL it receives the suffix array (positions in T).
 * Returns 0, or -1 on allocation failure.
 */
int orc_bwt(const uint8_t *codes, const int64_t *lens, int64_t m, int nthreads,
            uint8_t *B, int64_t *S_out)
{
    int64_t n = 0;
    int32_t *T = orc_make_text(codes, lens, m, &n);
    if (!T) return -1;
    int64_t *S = S_out ? S_out : (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!S) { free(T); return -1; }
    if (orc_suffix_sort(T, n, nthreads, S) != 0) {
        if (!S_out) free(S);
        free(T);
        return -1;
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t p = S[i] == 0 ? n - 1 : S[i] - 1;
        int32_t v = T[p];
        B[i] = (v < m) ? 0 : (uint8_t)(v - (m - 1));
    }
    if (!S_out) free(S);
    free(T);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Inverse-BWT verifier                                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    const uint8_t *B;
    const int64_t *occ; /* counts of each code before every 64th position */
    const int64_t *C;
    const uint8_t *codes;
    const int64_t *lens, *start; /* start offset of each string in codes */
    int64_t m;
    int64_t j0, j1;
    int64_t bad; /* first failing string + 1, or 0 */
} orc_walk_job;

/* Occurrences of c in B[0, k): the table entry of k's 64-symbol block plus
 * the matching bytes of the block before k, eight at a time (a byte of
 * w ^ c8 is zero exactly where B holds c). */
static int64_t orc_rank(const uint8_t *B, const int64_t *occ, int c, int64_t k)
{
    int64_t i = k & ~(int64_t)63, r = occ[(k >> 6) * 6 + c];
    const uint64_t c8 = 0x0101010101010101ULL * (uint64_t)c, lo7 = 0x7F7F7F7F7F7F7F7FULL;
    for (; i + 8 <= k; i += 8) {
        uint64_t w;
        memcpy(&w, B + i, 8);
        const uint64_t x = w ^ c8;
        const uint64_t z = ~(((x & lo7) + lo7) | x | lo7); /* high bit of each zero byte */
        r += __builtin_popcountll(z);
    }
    for (; i < k; ++i) r += (B[i] == c);
    return r;
}

/* Walks the job's strings, several at a time in turn, so that the memory
 * reads of independent walks overlap. Each walk is the LF walk of one
 * string: row j holds the sentinel-only suffix of string j, its BWT symbol
 * is the string's last base, and LF steps the string right to left. */
#define ORC_WALKS 8
static void *orc_walk_worker(void *p)
{
    orc_walk_job *jb = (orc_walk_job *)p;
    jb->bad = 0;
    int64_t wj[ORC_WALKS], wt[ORC_WALKS], wk[ORC_WALKS];
    int nw = 0;
    int64_t next = jb->j0;
    for (;;) {
        while (nw < ORC_WALKS && next < jb->j1) {
            wj[nw] = next;
            wt[nw] = jb->lens[next] - 1;
            wk[nw] = next;
            ++nw;
            ++next;
        }
        if (nw == 0) break;
        for (int a = 0; a < nw;) {
            const int64_t j = wj[a], k = wk[a], t = wt[a];
            if (t < 0) {
                /* the walk is back at the string's start: its row's symbol is $ */
                if (jb->B[k] != 0 && (!jb->bad || j + 1 < jb->bad)) jb->bad = j + 1;
                --nw;
                wj[a] = wj[nw]; wt[a] = wt[nw]; wk[a] = wk[nw];
                continue;
            }
            const int c = jb->B[k];
            if (c != jb->codes[jb->start[j] + t]) {
                if (!jb->bad || j + 1 < jb->bad) jb->bad = j + 1;
                --nw;
                wj[a] = wj[nw]; wt[a] = wt[nw]; wk[a] = wk[nw];
                continue;
            }
            wk[a] = jb->C[c] + orc_rank(jb->B, jb->occ, c, k);
            wt[a] = t - 1;
            ++a;
        }
    }
    return NULL;
}

/*
 * The verifier in two parts, so that a very large list can be walked a few
 * strings at a time: orc_verifier_new checks the length and the symbol
 * counts and builds C and the occurrence table (it keeps pointers to B,
 * codes and lens, which must outlive it); orc_verifier_walk LF-walks strings
 * [j0, j1). The list passes when the counts pass and every string in
 * [0, m) is walked without failure.
 */
typedef struct {
    const uint8_t *B;
    int64_t n;
    const uint8_t *codes;
    const int64_t *lens;
    int64_t m;
    int64_t C[6];
    int64_t *occ;
    int64_t *start;
} orc_verifier;

void orc_verifier_free(void *h)
{
    orc_verifier *v = (orc_verifier *)h;
    if (!v) return;
    free(v->occ);
    free(v->start);
    free(v);
}

/* The occurrence table in parallel: each thread counts its range of B
 * (ranges start at multiples of 64), then writes the running counts of its
 * range's 64-symbol blocks from the counts of the ranges before it. */
typedef struct {
    const uint8_t *B;
    int64_t *occ;
    int64_t i0, i1, n;
    int64_t cnt[8];   /* pass 1: symbols 0..5 of the range, [6] = codes above 5 */
    int64_t base[6];  /* pass 2: counts before the range */
    int pass;
} orc_occ_job;

static void *orc_occ_worker(void *p)
{
    orc_occ_job *jb = (orc_occ_job *)p;
    if (jb->pass == 1) {
        int64_t c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t i = jb->i0; i < jb->i1; ++i) c[jb->B[i] < 6 ? jb->B[i] : 6]++;
        memcpy(jb->cnt, c, sizeof(c));
        return NULL;
    }
    int64_t run[6];
    memcpy(run, jb->base, sizeof(run));
    for (int64_t i = jb->i0; i < jb->i1; ++i) {
        if ((i & 63) == 0) memcpy(jb->occ + (i >> 6) * 6, run, sizeof(run));
        run[jb->B[i]]++;
    }
    if (jb->i1 == jb->n && (jb->n & 63) == 0) memcpy(jb->occ + (jb->n >> 6) * 6, run, sizeof(run));
    return NULL;
}

/* *status: 0 ok, -1 wrong n, -2 symbol counts differ, -3 allocation failure
 * (the handle is NULL unless *status is 0). */
void *orc_verifier_new_mt(const uint8_t *B, int64_t n, const uint8_t *codes, const int64_t *lens,
                          int64_t m, int nthreads, int64_t *status)
{
    int64_t want = 0;
    int64_t cnt[6] = {0, 0, 0, 0, 0, 0}, got[7] = {0, 0, 0, 0, 0, 0, 0};
    int64_t q = 0;
    for (int64_t j = 0; j < m; ++j) {
        want += lens[j] + 1;
        for (int64_t t = 0; t < lens[j]; ++t) cnt[codes[q++]]++;
    }
    cnt[0] = m;
    if (want != n) { *status = -1; return NULL; }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > ORC_MAX_THREADS) nthreads = ORC_MAX_THREADS;
    orc_verifier *v = (orc_verifier *)calloc(1, sizeof(orc_verifier));
    if (!v) { *status = -3; return NULL; }
    v->B = B; v->n = n; v->codes = codes; v->lens = lens; v->m = m;
    const int64_t nb = (n >> 6) + 1;
    v->occ = (int64_t *)malloc((size_t)nb * 6 * sizeof(int64_t));
    v->start = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    if (!v->occ || !v->start) { orc_verifier_free(v); *status = -3; return NULL; }
    pthread_t th[ORC_MAX_THREADS];
    orc_occ_job jobs[ORC_MAX_THREADS];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].B = B; jobs[t].occ = v->occ; jobs[t].n = n; jobs[t].pass = 1;
        jobs[t].i0 = ((n >> 6) * t / nthreads) << 6;
        jobs[t].i1 = t == nthreads - 1 ? n : ((n >> 6) * (t + 1) / nthreads) << 6;
        pthread_create(&th[t], NULL, orc_occ_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    for (int t = 0; t < nthreads; ++t)
        for (int c = 0; c < 7; ++c) got[c] += jobs[t].cnt[c];
    int ok = got[6] == 0;
    for (int c = 0; c < 6; ++c) ok &= got[c] == cnt[c];
    if (!ok) { orc_verifier_free(v); *status = -2; return NULL; }
    int64_t run[6] = {0, 0, 0, 0, 0, 0};
    for (int t = 0; t < nthreads; ++t) {
        memcpy(jobs[t].base, run, sizeof(run));
        for (int c = 0; c < 6; ++c) run[c] += jobs[t].cnt[c];
        jobs[t].pass = 2;
        pthread_create(&th[t], NULL, orc_occ_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    v->C[0] = 0;
    for (int c = 1; c < 6; ++c) v->C[c] = v->C[c - 1] + cnt[c - 1];
    q = 0;
    for (int64_t j = 0; j < m; ++j) { v->start[j] = q; q += lens[j]; }
    *status = 0;
    return v;
}

void *orc_verifier_new(const uint8_t *B, int64_t n, const uint8_t *codes, const int64_t *lens,
                       int64_t m, int64_t *status)
{
    return orc_verifier_new_mt(B, n, codes, lens, m, 1, status);
}

/* 0 when strings [j0, j1) are all recovered, else the first failing j + 1. */
int64_t orc_verifier_walk(void *h, int64_t j0, int64_t j1, int nthreads)
{
    orc_verifier *v = (orc_verifier *)h;
    if (j0 < 0) j0 = 0;
    if (j1 > v->m) j1 = v->m;
    if (j1 <= j0) return 0;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > ORC_MAX_THREADS) nthreads = ORC_MAX_THREADS;
    if (nthreads > j1 - j0) nthreads = (int)(j1 - j0);
    pthread_t th[ORC_MAX_THREADS];
    orc_walk_job jobs[ORC_MAX_THREADS];
    const int64_t k = j1 - j0;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].B = v->B; jobs[t].occ = v->occ; jobs[t].C = v->C; jobs[t].codes = v->codes;
        jobs[t].lens = v->lens; jobs[t].start = v->start; jobs[t].m = v->m;
        jobs[t].j0 = j0 + k * t / nthreads; jobs[t].j1 = j0 + k * (t + 1) / nthreads;
        pthread_create(&th[t], NULL, orc_walk_worker, &jobs[t]);
    }
    int64_t bad = 0;
    for (int t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        if (jobs[t].bad && (!bad || jobs[t].bad < bad)) bad = jobs[t].bad;
    }
    return bad;
}

/*
 * Check that candidate codes B (length n) are the BWT of the list (codes,
 * lens, m). Returns 0 when every string is recovered by LF walks from rows
 * 0..m-1 and the symbol counts match; -1 when n is wrong; -2 when symbol
 * counts differ; -3 on allocation failure; j+1 when string j is not recovered.
 */
int64_t orc_verify(const uint8_t *B, int64_t n, const uint8_t *codes, const int64_t *lens,
                   int64_t m, int nthreads)
{
    int64_t status = 0;
    void *h = orc_verifier_new_mt(B, n, codes, lens, m, nthreads, &status);
    if (!h) return status;
    int64_t bad = orc_verifier_walk(h, 0, m, nthreads);
    orc_verifier_free(h);
    return bad;
}

/* ------------------------------------------------------------------------ */
/* SA intervals                                                               */
/* ------------------------------------------------------------------------ */

/*
 * Compare the suffix of T starting at g with the pattern P (codes 1..5):
 * -1 if the suffix is smaller than P and P is not its prefix, 0 if P is a
 * prefix of the suffix, +1 if the suffix is larger. A sentinel is smaller
 * than every base.
 */
static int orc_cmp_pattern(const int32_t *T, int64_t m, int64_t g, const uint8_t *P, int64_t len)
{
    for (int64_t d = 0; d < len; ++d) {
        int32_t v = T[g + d];
        if (v < m) return -1;
        int c = (int)(v - (m - 1));
        if (c != P[d]) return c < P[d] ? -1 : 1;
    }
    return 0;
}

typedef struct {
    const int32_t *T;
    int64_t n, m;
    const uint8_t *q;
    const int64_t *qoff, *qlens;
    int64_t i0, i1;
    int64_t *lo, *hi;
} orc_count_job;

static void *orc_count_worker(void *p)
{
    orc_count_job *jb = (orc_count_job *)p;
    for (int64_t i = jb->i0; i < jb->i1; ++i) {
        const uint8_t *P = jb->q + jb->qoff[i];
        int64_t len = jb->qlens[i], lo = 0, occ = 0;
        for (int64_t g = 0; g < jb->n; ++g) {
            int r = orc_cmp_pattern(jb->T, jb->m, g, P, len);
            if (r < 0) ++lo;
            else if (r == 0) ++occ;
        }
        jb->lo[i] = lo;
        jb->hi[i] = lo + occ;
    }
    return NULL;
}

/*
 * SA interval of each query by brute force (Sec. 2.3): lo = number of
 * suffixes smaller than P, occ = number of suffixes with prefix P, hi = lo +
 * occ. Query codes are 1..5 concatenated; an empty query gives [0, n).
 */
int orc_count(const uint8_t *codes, const int64_t *lens, int64_t m, const uint8_t *qcodes,
              const int64_t *qlens, int64_t nq, int nthreads, int64_t *lo, int64_t *hi)
{
    int64_t n = 0;
    int32_t *T = orc_make_text(codes, lens, m, &n);
    int64_t *qoff = (int64_t *)malloc((size_t)(nq > 0 ? nq : 1) * sizeof(int64_t));
    if (!T || !qoff) { free(T); free(qoff); return -1; }
    int64_t s = 0;
    for (int64_t i = 0; i < nq; ++i) { qoff[i] = s; s += qlens[i]; }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > ORC_MAX_THREADS) nthreads = ORC_MAX_THREADS;
    pthread_t th[ORC_MAX_THREADS];
    orc_count_job jobs[ORC_MAX_THREADS];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].T = T; jobs[t].n = n; jobs[t].m = m; jobs[t].q = qcodes;
        jobs[t].qoff = qoff; jobs[t].qlens = qlens;
        jobs[t].i0 = nq * t / nthreads; jobs[t].i1 = nq * (t + 1) / nthreads;
        jobs[t].lo = lo; jobs[t].hi = hi;
        pthread_create(&th[t], NULL, orc_count_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(qoff);
    free(T);
    return 0;
}

/* [lo, hi) of P by binary search over the sorted suffix array S of T. */
static void orc_interval(const int32_t *T, int64_t n, int64_t m, const int64_t *S,
                         const uint8_t *P, int64_t len, int64_t *lo, int64_t *hi)
{
    int64_t a = 0, b = n;
    while (a < b) { /* first row whose suffix is not below P */
        int64_t mid = a + (b - a) / 2;
        if (orc_cmp_pattern(T, m, S[mid], P, len) < 0) a = mid + 1; else b = mid;
    }
    *lo = a;
    b = n;
    while (a < b) { /* first row whose suffix is above P */
        int64_t mid = a + (b - a) / 2;
        if (orc_cmp_pattern(T, m, S[mid], P, len) <= 0) a = mid + 1; else b = mid;
    }
    *hi = a;
}

typedef struct {
    int32_t *T;
    int64_t n, m;
} orc_text;

/* Build the integer text once so that interval and SMEM calls can reuse it. */
void *orc_text_new(const uint8_t *codes, const int64_t *lens, int64_t m)
{
    orc_text *x = (orc_text *)malloc(sizeof(orc_text));
    if (!x) return NULL;
    x->T = orc_make_text(codes, lens, m, &x->n);
    x->m = m;
    if (!x->T) { free(x); return NULL; }
    return x;
}

void orc_text_free(void *h)
{
    orc_text *x = (orc_text *)h;
    if (!x) return;
    free(x->T);
    free(x);
}

int orc_sa_interval(void *h, const int64_t *S, const uint8_t *P, int64_t len, int64_t *lo,
                    int64_t *hi)
{
    orc_text *x = (orc_text *)h;
    orc_interval(x->T, x->n, x->m, S, P, len, lo, hi);
    return 0;
}

/*
 * SMEMs of P no shorter than min_len that occur at least min_occ times
 * (Sec. 2.6, with the min-occurrence generalisation cited there).
 *
 * Definition used: let e(i) be the largest e <= |P| with occ(P[i,e)) >=
 * min_occ (e(i) = i when even P[i] is too rare). occ only falls as a
 * substring grows, so e(.) is non-decreasing, and the exact matches that no
 * other match on P contains are exactly [i, e(i)) with i = 0 or e(i) >
 * e(i-1), whenever that interval is non-empty. The ones of length >= min_len
 * are reported, in increasing i, as five int64 each: start, end,
 * occ(P[start,end)), lo(P[start,end)), lo(rc(P[start,end))).
 *
 * S is the suffix array of the text (from orc_bwt). Returns the number of
 * SMEMs found; only the first cap are written.
 */
int64_t orc_smem(void *h, const int64_t *S, const uint8_t *P, int64_t len, int64_t min_len,
                 int64_t min_occ, int64_t *out, int64_t cap)
{
    orc_text *x = (orc_text *)h;
    int64_t found = 0, eprev = -1;
    uint8_t *rc = (uint8_t *)malloc((size_t)(len > 0 ? len : 1));
    if (!rc) return -1;
    for (int64_t i = 0; i < len; ++i) {
        int64_t e = eprev > i ? eprev : i;
        int64_t lo, hi;
        /* e(i) >= e(i-1): P[i, e(i-1)) is inside P[i-1, e(i-1)) */
        if (e > i) {
            orc_interval(x->T, x->n, x->m, S, P + i, e - i, &lo, &hi);
        } else {
            lo = 0;
            hi = x->n;
        }
        if (hi - lo < min_occ) {
            /* only possible when e == i and the whole text is too small */
            eprev = e;
            continue;
        }
        while (e < len) {
            int64_t lo2, hi2;
            orc_interval(x->T, x->n, x->m, S, P + i, e + 1 - i, &lo2, &hi2);
            if (hi2 - lo2 < min_occ) break;
            lo = lo2;
            hi = hi2;
            ++e;
        }
        if ((i == 0 || e > eprev) && e - i >= min_len && e > i) {
            if (found < cap) {
                int64_t L = e - i, klo, khi;
                for (int64_t t = 0; t < L; ++t) rc[t] = orc_comp(P[e - 1 - t]);
                orc_interval(x->T, x->n, x->m, S, rc, L, &klo, &khi);
                int64_t *o = out + found * 5;
                o[0] = i; o[1] = e; o[2] = hi - lo; o[3] = lo; o[4] = klo;
            }
            ++found;
        }
        eprev = e;
    }
    free(rc);
    return found;
}

/* ------------------------------------------------------------------------ */
/* SA intervals of many patterns in one pass over every suffix               */
/* ------------------------------------------------------------------------ */

/*
 * The same [lo, hi) as orc_count (Sec. 2.3: lo = number of suffixes below P,
 * hi = lo + number of suffixes with prefix P), for a batch of patterns,
 * with one pass over the suffixes instead of one per pattern.
 *
 * Each pattern P gives two probes: P followed by a symbol below every
 * symbol (lo counts the suffixes below it) and P followed by a symbol above
 * every symbol (hi counts the suffixes below that one). A suffix never
 * equals a probe, so with the probes sorted, the probes above a suffix x
 * are exactly those from the g(x)-th on, where g(x) is the number of probes
 * below x; a histogram of g over all suffixes, summed up to a probe's place,
 * gives the number of suffixes below that probe.
 *
 * g(x) comes from the first ORC_SCAN_K symbols of x when they are all bases
 * A..T: the probes whose first ORC_SCAN_K symbols are smaller all lie below
 * x, the larger ones above, and only the probes sharing x's prefix are
 * compared in full (binary search). Any other suffix (a sentinel or an N
 * among its first ORC_SCAN_K symbols) is compared with every probe by
 * binary search; those comparisons end within ORC_SCAN_K symbols.
 *
 * Precondition: every pattern is at least ORC_SCAN_K long and its first
 * ORC_SCAN_K symbols are A..T (codes 1..4). Returns 0, -1 on allocation
 * failure, -4 when a pattern breaks the precondition.
 */
#define ORC_SCAN_K 12
#define ORC_SCAN_NB (1u << (2 * ORC_SCAN_K))

typedef struct {
    const uint8_t *codes;       /* text strands, concatenated, no sentinels */
    const int64_t *lens, *start;
    int64_t m;
    const uint8_t *pc;          /* pattern codes */
    const int64_t *poff, *plen;
    const int64_t *probe;       /* sorted probes: pattern index * 2 + (0: lo, 1: hi) */
    int64_t np2;                /* number of probes */
    const uint32_t *first;      /* probes with a smaller K-prefix code, per code */
} orc_scan_ctx;

/* 1 if the suffix at offset t of strand j is below probe pr, else 0. */
static int orc_suffix_below(const orc_scan_ctx *x, int64_t j, int64_t t, int64_t pr)
{
    const uint8_t *S = x->codes + x->start[j];
    const int64_t L = x->lens[j];
    const int64_t pi = pr >> 1;
    const uint8_t *P = x->pc + x->poff[pi];
    const int64_t pl = x->plen[pi];
    for (int64_t d = 0;; ++d) {
        if (d == pl) return (int)(pr & 1);     /* past P: below the "above all" probe only */
        if (t + d == L) return 1;              /* the suffix's sentinel is below every base */
        const uint8_t s = S[t + d];
        if (s != P[d]) return s < P[d];
    }
}

/* Probe order: compare the patterns, then the terminal symbol (lo < hi). */
static int orc_probe_cmp(const orc_scan_ctx *x, int64_t a, int64_t b)
{
    const uint8_t *A = x->pc + x->poff[a >> 1], *B = x->pc + x->poff[b >> 1];
    const int64_t la = x->plen[a >> 1], lb = x->plen[b >> 1];
    const int64_t n = la < lb ? la : lb;
    for (int64_t d = 0; d < n; ++d)
        if (A[d] != B[d]) return A[d] < B[d] ? -1 : 1;
    if (la == lb) return (int)(a & 1) - (int)(b & 1);
    /* the shorter one ends in its terminal, below or above every symbol */
    if (la < lb) return (a & 1) ? 1 : -1;
    return (b & 1) ? -1 : 1;
}

static void orc_probe_sort(const orc_scan_ctx *x, int64_t *a, int64_t *tmp, int64_t n)
{
    if (n < 2) return;
    if (n <= 16) {
        for (int64_t i = 1; i < n; ++i) {
            int64_t v = a[i], j = i;
            while (j > 0 && orc_probe_cmp(x, a[j - 1], v) > 0) { a[j] = a[j - 1]; --j; }
            a[j] = v;
        }
        return;
    }
    int64_t h = n / 2;
    orc_probe_sort(x, a, tmp, h);
    orc_probe_sort(x, a + h, tmp + h, n - h);
    int64_t i = 0, j = h, k = 0;
    while (i < h && j < n) tmp[k++] = (orc_probe_cmp(x, a[j], a[i]) < 0) ? a[j++] : a[i++];
    while (i < h) tmp[k++] = a[i++];
    while (j < n) tmp[k++] = a[j++];
    memcpy(a, tmp, (size_t)n * sizeof(int64_t));
}

/* Number of probes in [f0, f1) below the suffix (t of strand j), given that
 * the probes before f0 are below it and those from f1 on above it. */
static int64_t orc_probes_below(const orc_scan_ctx *x, int64_t j, int64_t t, int64_t f0, int64_t f1)
{
    while (f0 < f1) { /* first probe the suffix is below */
        int64_t mid = f0 + (f1 - f0) / 2;
        if (orc_suffix_below(x, j, t, x->probe[mid])) f1 = mid; else f0 = mid + 1;
    }
    return f0;
}

typedef struct {
    const orc_scan_ctx *x;
    int64_t j0, t0, j1, t1;   /* suffixes from (j0, t0) up to, not including, (j1, t1) */
    int64_t *hist;            /* np2 + 1 */
} orc_scan_job;

static void *orc_scan_worker(void *p)
{
    orc_scan_job *jb = (orc_scan_job *)p;
    const orc_scan_ctx *x = jb->x;
    const uint32_t mask = ORC_SCAN_NB - 1;
    for (int64_t j = jb->j0; j <= jb->j1 && j < x->m; ++j) {
        const int64_t L = x->lens[j];
        const int64_t a = j == jb->j0 ? jb->t0 : 0;
        const int64_t b = j == jb->j1 ? jb->t1 : L + 1; /* offsets [a, b), L = the sentinel */
        if (a >= b) continue;
        const uint8_t *S = x->codes + x->start[j];
        /* the window of K symbols starting at b: its 2-bit code and how many
         * of its leading symbols are A..T */
        uint32_t code = 0;
        int run = 0;
        for (int d = ORC_SCAN_K - 1; d >= 0; --d) {
            const int64_t q = b + d;
            const int s = q < L ? S[q] : 0;
            if (s >= 1 && s <= 4) {
                code = (code >> 2) | ((uint32_t)(s - 1) << (2 * ORC_SCAN_K - 2));
                run = run < ORC_SCAN_K ? run + 1 : ORC_SCAN_K;
            } else {
                run = 0;
            }
        }
        for (int64_t t = b - 1; t >= a; --t) {
            const int s = t < L ? S[t] : 0;
            if (s >= 1 && s <= 4) {
                code = ((code >> 2) | ((uint32_t)(s - 1) << (2 * ORC_SCAN_K - 2))) & mask;
                run = run < ORC_SCAN_K ? run + 1 : ORC_SCAN_K;
            } else {
                run = 0;
            }
            int64_t g;
            if (run >= ORC_SCAN_K) {
                const int64_t f0 = x->first[code], f1 = x->first[code + 1];
                g = f0 < f1 ? orc_probes_below(x, j, t, f0, f1) : f0;
            } else {
                g = orc_probes_below(x, j, t, 0, x->np2);
            }
            jb->hist[g]++;
        }
    }
    return NULL;
}

int orc_scan_intervals(const uint8_t *codes, const int64_t *lens, int64_t m, const uint8_t *pcodes,
                       const int64_t *plens, int64_t np, int nthreads, int64_t *lo, int64_t *hi)
{
    if (np == 0) return 0;
    for (int64_t i = 0, o = 0; i < np; o += plens[i], ++i) {
        if (plens[i] < ORC_SCAN_K) return -4;
        for (int d = 0; d < ORC_SCAN_K; ++d)
            if (pcodes[o + d] < 1 || pcodes[o + d] > 4) return -4;
    }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > ORC_MAX_THREADS) nthreads = ORC_MAX_THREADS;
    const int64_t np2 = 2 * np;
    int64_t *start = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    int64_t *poff = (int64_t *)malloc((size_t)np * sizeof(int64_t));
    int64_t *probe = (int64_t *)malloc((size_t)np2 * sizeof(int64_t));
    int64_t *tmp = (int64_t *)malloc((size_t)np2 * sizeof(int64_t));
    int64_t *place = (int64_t *)malloc((size_t)np2 * sizeof(int64_t));
    uint32_t *first = (uint32_t *)calloc((size_t)ORC_SCAN_NB + 1, sizeof(uint32_t));
    int64_t *hist = (int64_t *)calloc((size_t)nthreads * (size_t)(np2 + 1), sizeof(int64_t));
    int rc = -1;
    if (!start || !poff || !probe || !tmp || !place || !first || !hist) goto done;
    int64_t nsuf = 0;
    for (int64_t j = 0, s = 0; j < m; s += lens[j], ++j) { start[j] = s; nsuf += lens[j] + 1; }
    for (int64_t i = 0, o = 0; i < np; o += plens[i], ++i) poff[i] = o;
    orc_scan_ctx x = {codes, lens, start, m, pcodes, poff, plens, probe, np2, first};
    for (int64_t i = 0; i < np2; ++i) probe[i] = i;
    orc_probe_sort(&x, probe, tmp, np2);
    /* first[c] = probes whose K-prefix code is below c */
    for (int64_t i = 0; i < np2; ++i) {
        const uint8_t *P = pcodes + poff[probe[i] >> 1];
        uint32_t c = 0;
        for (int d = 0; d < ORC_SCAN_K; ++d) c = (c << 2) | (uint32_t)(P[d] - 1);
        first[c + 1]++;
    }
    for (uint32_t c = 0; c < ORC_SCAN_NB; ++c) first[c + 1] += first[c];
    /* the suffixes, cut into nthreads equal ranges */
    pthread_t th[ORC_MAX_THREADS];
    orc_scan_job jobs[ORC_MAX_THREADS];
    {
        int64_t j = 0, before = 0; /* suffixes of strands before j */
        for (int t = 0; t < nthreads; ++t) {
            const int64_t g0 = nsuf * t / nthreads, g1 = nsuf * (t + 1) / nthreads;
            while (j < m && before + lens[j] + 1 <= g0) { before += lens[j] + 1; ++j; }
            jobs[t].j0 = j;
            jobs[t].t0 = g0 - before;
            int64_t jj = j, bb = before;
            while (jj < m && bb + lens[jj] + 1 <= g1) { bb += lens[jj] + 1; ++jj; }
            jobs[t].j1 = jj;
            jobs[t].t1 = g1 - bb;
            jobs[t].x = &x;
            jobs[t].hist = hist + (size_t)t * (size_t)(np2 + 1);
        }
    }
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, orc_scan_worker, &jobs[t]);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    /* suffixes below sorted probe k: histogram summed over g <= k */
    int64_t run = 0;
    for (int64_t k = 0; k < np2; ++k) {
        for (int t = 0; t < nthreads; ++t) run += hist[(size_t)t * (size_t)(np2 + 1) + k];
        place[probe[k]] = run;
    }
    for (int64_t i = 0; i < np; ++i) {
        lo[i] = place[2 * i];
        hi[i] = place[2 * i + 1];
    }
    rc = 0;
done:
    free(start); free(poff); free(probe); free(tmp); free(place); free(first); free(hist);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* SMEMs by a seeded scan of the text                                        */
/* ------------------------------------------------------------------------ */

/*
 * The SMEMs of orc_smem (length >= min_len, occurring >= min_occ times;
 * Sec. 2.6), for a batch of queries, found without a suffix array, by one
 * pass over the text:
 *
 *   1. every min_len-mer of every query is hashed;
 *   2. one pass over the text hashes each min_len-mer of it; a text window
 *      equal to query window (q, i) is a hit, and the hits of one query on
 *      one diagonal (text position - query position) at consecutive i form
 *      a run; a hit whose left neighbours also match is inside a run, so
 *      only a run's first hit is extended, to the right, once: the run
 *      starting at i is the exact match P[i, r) of the text at that
 *      diagonal, with r as far as the match goes;
 *   3. an occurrence of P[i, e) with e - i >= min_len contains the hit of
 *      P[i, i + min_len), so occ(P[i, e)) is the number of runs covering
 *      query position i (as a hit) with r >= e. So e(i) (largest e with
 *      occ >= min_occ) is the min_occ-th largest r of those runs, and the
 *      SMEMs are [i, e(i)) with i = 0 or e(i) > e(i-1), as in orc_smem (a
 *      position with fewer covering runs has e(i) < i + min_len, so it
 *      starts no SMEM and any longer e(i+1) exceeds it);
 *   4. k and krc, the lo of P[i, e) and of its reverse complement, come
 *      from orc_scan_intervals, whose hi - lo must equal the run count.
 *
 * out: 5 int64 per SMEM (start, end, occ, k, krc), query by query in
 * increasing start; qoff (nq + 1) the offsets. Returns the number of SMEMs
 * (only the first cap are written); -1 allocation failure; -4 min_len below
 * ORC_SCAN_K or an SMEM whose first ORC_SCAN_K symbols (or those of its
 * reverse complement) are not all A..T; -5 when the two counts of an SMEM
 * disagree (an internal inconsistency).
 */
static uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

#define ORC_HASH_B 0x9E3779B97F4A7C15ULL

typedef struct {
    uint64_t key;
    int64_t q, i;
} orc_seed;

typedef struct {
    int64_t q, i, r; /* query q matches the text on [i, r) at one diagonal */
} orc_run;

typedef struct {
    const uint8_t *codes;
    const int64_t *lens, *start;
    const uint8_t *qc;
    const int64_t *qoff, *qlen;
    int64_t ell;
    const orc_seed *seed;
    const int64_t *bstart;
    int bshift;
    int64_t j0, j1; /* strands [j0, j1) */
    orc_run *runs;
    int64_t nruns, cap;
    int failed;
} orc_seedscan_job;

static void orc_push_run(orc_seedscan_job *jb, int64_t q, int64_t i, int64_t r)
{
    if (jb->nruns == jb->cap) {
        int64_t nc = jb->cap ? 2 * jb->cap : 4096;
        orc_run *nr = (orc_run *)realloc(jb->runs, (size_t)nc * sizeof(orc_run));
        if (!nr) { jb->failed = 1; return; }
        jb->runs = nr;
        jb->cap = nc;
    }
    jb->runs[jb->nruns].q = q;
    jb->runs[jb->nruns].i = i;
    jb->runs[jb->nruns].r = r;
    jb->nruns++;
}

static void *orc_seedscan_worker(void *p)
{
    orc_seedscan_job *jb = (orc_seedscan_job *)p;
    const int64_t ell = jb->ell;
    uint64_t bpow = 1; /* B^(ell-1) */
    for (int64_t d = 1; d < ell; ++d) bpow *= ORC_HASH_B;
    for (int64_t j = jb->j0; j < jb->j1 && !jb->failed; ++j) {
        const int64_t L = jb->lens[j];
        if (L < ell) continue;
        const uint8_t *T = jb->codes + jb->start[j];
        uint64_t h = 0;
        for (int64_t d = 0; d < ell; ++d) h = h * ORC_HASH_B + T[d];
        for (int64_t t = 0;; ++t) {
            const uint64_t key = orc_mix64(h);
            const int64_t b = (int64_t)(key >> jb->bshift);
            for (int64_t e = jb->bstart[b]; e < jb->bstart[b + 1]; ++e) {
                if (jb->seed[e].key != key) continue;
                const int64_t q = jb->seed[e].q, i = jb->seed[e].i;
                const uint8_t *P = jb->qc + jb->qoff[q];
                /* inside a run that starts further left */
                if (i > 0 && t > 0 && P[i - 1] == T[t - 1]) continue;
                if (memcmp(P + i, T + t, (size_t)ell) != 0) continue;
                int64_t r = i + ell;
                while (r < jb->qlen[q] && t + (r - i) < L && P[r] == T[t + (r - i)]) ++r;
                orc_push_run(jb, q, i, r);
            }
            if (t + ell >= L) break;
            h = (h - T[t] * bpow) * ORC_HASH_B + T[t + ell];
        }
    }
    return NULL;
}

static int orc_seed_cmp(const void *a, const void *b)
{
    const uint64_t x = ((const orc_seed *)a)->key, y = ((const orc_seed *)b)->key;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static int orc_run_cmp(const void *a, const void *b)
{
    const orc_run *x = (const orc_run *)a, *y = (const orc_run *)b;
    if (x->q != y->q) return x->q < y->q ? -1 : 1;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    return x->r < y->r ? -1 : (x->r > y->r ? 1 : 0);
}

int64_t orc_smem_scan(const uint8_t *codes, const int64_t *lens, int64_t m, const uint8_t *qcodes,
                      const int64_t *qlens, int64_t nq, int64_t min_len, int64_t min_occ, int nthreads,
                      int64_t *out, int64_t cap, int64_t *qoff_out)
{
    if (min_len < ORC_SCAN_K) return -4;
    if (min_occ < 1) min_occ = 1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > ORC_MAX_THREADS) nthreads = ORC_MAX_THREADS;
    const int64_t ell = min_len;
    int64_t rc = -1;
    int64_t *start = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    int64_t *qoff = (int64_t *)malloc((size_t)(nq + 1) * sizeof(int64_t));
    orc_seed *seed = NULL;
    int64_t *bstart = NULL;
    orc_run *runs = NULL;
    int64_t *sm = NULL;      /* SMEMs: q, start, end, occ */
    uint8_t *pat = NULL;     /* the SMEM strings and their reverse complements */
    int64_t *plen = NULL, *plo = NULL, *phi = NULL;
    int64_t *act = NULL;
    orc_seedscan_job jobs[ORC_MAX_THREADS];
    memset(jobs, 0, sizeof(jobs));
    if (!start || !qoff) goto done;
    int64_t ntext = 0;
    for (int64_t j = 0; j < m; ++j) { start[j] = ntext; ntext += lens[j]; }
    qoff[0] = 0;
    for (int64_t q = 0; q < nq; ++q) qoff[q + 1] = qoff[q] + qlens[q];
    /* 1. seeds */
    int64_t nseed = 0;
    for (int64_t q = 0; q < nq; ++q) if (qlens[q] >= ell) nseed += qlens[q] - ell + 1;
    seed = (orc_seed *)malloc((size_t)(nseed > 0 ? nseed : 1) * sizeof(orc_seed));
    if (!seed) goto done;
    {
        uint64_t bpow = 1;
        for (int64_t d = 1; d < ell; ++d) bpow *= ORC_HASH_B;
        int64_t k = 0;
        for (int64_t q = 0; q < nq; ++q) {
            if (qlens[q] < ell) continue;
            const uint8_t *P = qcodes + qoff[q];
            uint64_t h = 0;
            for (int64_t d = 0; d < ell; ++d) h = h * ORC_HASH_B + P[d];
            for (int64_t i = 0;; ++i) {
                seed[k].key = orc_mix64(h);
                seed[k].q = q;
                seed[k].i = i;
                ++k;
                if (i + ell >= qlens[q]) break;
                h = (h - P[i] * bpow) * ORC_HASH_B + P[i + ell];
            }
        }
    }
    qsort(seed, (size_t)nseed, sizeof(orc_seed), orc_seed_cmp);
    int bbits = 10;
    while (bbits < 30 && ((int64_t)1 << bbits) < 2 * nseed) ++bbits;
    const int bshift = 64 - bbits;
    const int64_t nb = (int64_t)1 << bbits;
    bstart = (int64_t *)malloc((size_t)(nb + 1) * sizeof(int64_t));
    if (!bstart) goto done;
    for (int64_t b = 0, e = 0; b <= nb; ++b) {
        while (e < nseed && (int64_t)(seed[e].key >> bshift) < b) ++e;
        bstart[b] = e;
    }
    /* 2. the text, strands dealt to threads in nearly equal symbol counts */
    {
        int64_t j = 0, acc = 0;
        for (int t = 0; t < nthreads; ++t) {
            const int64_t goal = ntext * (t + 1) / nthreads;
            jobs[t].j0 = j;
            while (j < m && (acc < goal || t == nthreads - 1)) acc += lens[j++];
            jobs[t].j1 = j;
            jobs[t].codes = codes; jobs[t].lens = lens; jobs[t].start = start;
            jobs[t].qc = qcodes; jobs[t].qoff = qoff; jobs[t].qlen = qlens; jobs[t].ell = ell;
            jobs[t].seed = seed; jobs[t].bstart = bstart; jobs[t].bshift = bshift;
        }
        pthread_t th[ORC_MAX_THREADS];
        for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, orc_seedscan_worker, &jobs[t]);
        for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    }
    int64_t nrun = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (jobs[t].failed) goto done;
        nrun += jobs[t].nruns;
    }
    runs = (orc_run *)malloc((size_t)(nrun > 0 ? nrun : 1) * sizeof(orc_run));
    if (!runs) goto done;
    {
        int64_t k = 0;
        for (int t = 0; t < nthreads; ++t) {
            memcpy(runs + k, jobs[t].runs, (size_t)jobs[t].nruns * sizeof(orc_run));
            k += jobs[t].nruns;
        }
    }
    qsort(runs, (size_t)nrun, sizeof(orc_run), orc_run_cmp);
    /* 3. e(i) per query from the runs covering i, then the SMEMs */
    int64_t nsm = 0, smcap = 1024;
    sm = (int64_t *)malloc((size_t)smcap * 4 * sizeof(int64_t));
    if (!sm) goto done;
    int64_t actcap = 1024;
    act = (int64_t *)malloc((size_t)actcap * sizeof(int64_t)); /* run ends r */
    if (!act) goto done;
    for (int64_t q = 0, ri = 0; q < nq; ++q) {
        qoff_out[q] = nsm;
        const int64_t len = qlens[q];
        int64_t na = 0, eprev = -1; /* eprev: e(i-1), or -1 when below i-1+ell */
        for (int64_t i = 0; i + ell <= len; ++i) {
            /* drop runs that no longer cover i (their last hit is at r - ell) */
            int64_t w = 0;
            for (int64_t a = 0; a < na; ++a)
                if (act[a] - ell >= i) act[w++] = act[a];
            na = w;
            while (ri < nrun && runs[ri].q == q && runs[ri].i == i) {
                if (na == actcap) {
                    actcap *= 2;
                    int64_t *nw = (int64_t *)realloc(act, (size_t)actcap * sizeof(int64_t));
                    if (!nw) goto done;
                    act = nw;
                }
                act[na++] = runs[ri++].r;
            }
            int64_t e = -1, occ = 0;
            if (na >= min_occ) {
                /* the min_occ-th largest end: the largest e with occ >= min_occ */
                int64_t lo_ = i + ell, hi_ = len;
                while (lo_ < hi_) { /* largest e in [i+ell, len] with count(r >= e) >= min_occ */
                    const int64_t mid = hi_ - (hi_ - lo_) / 2;
                    int64_t c = 0;
                    for (int64_t a = 0; a < na; ++a) c += act[a] >= mid;
                    if (c >= min_occ) lo_ = mid; else hi_ = mid - 1;
                }
                e = lo_;
                for (int64_t a = 0; a < na; ++a) occ += act[a] >= e;
            }
            if (e >= 0 && (i == 0 || e > eprev)) {
                if (nsm == smcap) {
                    smcap *= 2;
                    int64_t *nw = (int64_t *)realloc(sm, (size_t)smcap * 4 * sizeof(int64_t));
                    if (!nw) goto done;
                    sm = nw;
                }
                sm[nsm * 4 + 0] = q; sm[nsm * 4 + 1] = i; sm[nsm * 4 + 2] = e; sm[nsm * 4 + 3] = occ;
                ++nsm;
            }
            eprev = e;
        }
        while (ri < nrun && runs[ri].q == q) ++ri;
    }
    qoff_out[nq] = nsm;
    /* 4. intervals of each SMEM and of its reverse complement */
    {
        int64_t tot = 0;
        for (int64_t s = 0; s < nsm; ++s) tot += 2 * (sm[s * 4 + 2] - sm[s * 4 + 1]);
        pat = (uint8_t *)malloc((size_t)(tot > 0 ? tot : 1));
        plen = (int64_t *)malloc((size_t)(2 * nsm + 1) * sizeof(int64_t));
        plo = (int64_t *)malloc((size_t)(2 * nsm + 1) * sizeof(int64_t));
        phi = (int64_t *)malloc((size_t)(2 * nsm + 1) * sizeof(int64_t));
        if (!pat || !plen || !plo || !phi) goto done;
        int64_t o = 0;
        for (int64_t s = 0; s < nsm; ++s) {
            const uint8_t *P = qcodes + qoff[sm[s * 4]];
            const int64_t a = sm[s * 4 + 1], b = sm[s * 4 + 2], L = b - a;
            memcpy(pat + o, P + a, (size_t)L);
            for (int64_t d = 0; d < L; ++d) pat[o + L + d] = orc_comp(P[b - 1 - d]);
            plen[2 * s] = L;
            plen[2 * s + 1] = L;
            o += 2 * L;
        }
        const int r2 = orc_scan_intervals(codes, lens, m, pat, plen, 2 * nsm, nthreads, plo, phi);
        if (r2 != 0) { rc = r2; goto done; }
        for (int64_t s = 0; s < nsm; ++s) {
            const int64_t occ = sm[s * 4 + 3];
            if (phi[2 * s] - plo[2 * s] != occ || phi[2 * s + 1] - plo[2 * s + 1] != occ) { rc = -5; goto done; }
            if (s < cap) {
                int64_t *w = out + s * 5;
                w[0] = sm[s * 4 + 1]; w[1] = sm[s * 4 + 2]; w[2] = occ; w[3] = plo[2 * s]; w[4] = plo[2 * s + 1];
            }
        }
    }
    rc = nsm;
done:
    for (int t = 0; t < ORC_MAX_THREADS; ++t) free(jobs[t].runs);
    free(start); free(qoff); free(seed); free(bstart); free(runs); free(sm); free(pat);
    free(plen); free(plo); free(phi); free(act);
    return rc;
}
