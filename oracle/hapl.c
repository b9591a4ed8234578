/*
 * Local haplotype enumeration (Sec. 2.8): semi-global alignment of a query P
 * to the prefix DAWG G_T of the indexed text by the revised BWA-SW recurrences
 * (Sec. 2.7, Algorithm 5), then the bi-interval redundancy filter.
 *
 * THIS IS TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg call it. The GPU library never links, loads or
 * calls anything here, and nothing here shares code with the GPU library.
 *
 * Readings of the paper used (the same ones the library documents):
 *   - G_P is the path graph of P taken from its end: node u_i follows u_{i+1}
 *     along the edge labelled P[i]; u_{|P|} is the start, u_0 the end.
 *   - A node v of G_T is an SA interval; its children are the non-empty
 *     intervals of bS for b in {A, C, G, T} (prepending b: backward search).
 *     The root is the empty string, interval [0, n).
 *   - The start cell (u_{|P|}, root) has H = 0 and is propagated although it
 *     is not positive; every other cell is kept only when H > 0.
 *   - Scores: s(a, b) = match if a = b else -mismatch (a query N mismatches
 *     every symbol); a gap of length L costs gap_open + L * gap_ext.
 *   - At each u: the match and insertion steps from the cells of u', then
 *     the deletion step repeated until no cell of u improves (chains of
 *     deletions), then the cells with H <= 0 are dropped and, with band W >
 *     0, only the W cells of largest H are kept (ties: smaller k, then
 *     smaller s).
 *   - Result: the cells of u_0, by decreasing H (ties: smaller k, then
 *     smaller s); a cell is dropped when its interval [k, k+s), or its
 *     reverse-complement interval [k', k'+s), lies inside the corresponding
 *     interval of a cell kept before it.
 *   - A node holds every string with its SA interval (X and XZ when each
 *     occurrence of X is followed by Z), and those strings' reverse
 *     complements have different intervals. A cell's k' is that of a
 *     representative string: among the strings of the node whose alignment
 *     attains the cell's H, the one whose reverse complement's interval
 *     starts first. Each of H, E and F keeps such a representative: a match,
 *     insertion or deletion passes on the string of the score it extends
 *     (b prepended for a match or a deletion), and an offer replaces a
 *     score's representative when it scores higher, or equal with a
 *     smaller k'.
 *
 * Here a node is found as the SA interval of a string of it, by binary
 * search over the oracle's own suffix array, and a string's
 * reverse-complement interval as the SA interval of its reverse complement:
 * no backward-extension formula is used.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int orc_sa_interval(void *h, const int64_t *S, const uint8_t *P, int64_t len, int64_t *lo, int64_t *hi);

#define HP_NEG (-1000000000)

/* a score with its representative string (codes, len symbols) and the start
 * kr of its reverse complement's SA interval */
typedef struct {
    int v;
    uint8_t *str;
    int len;
    int64_t kr;
} hp_score;

typedef struct {
    int64_t k, s;
    hp_score H, E, F;
} hp_cell;

typedef struct {
    hp_cell *c;
    int n, cap;
} hp_table;

static int hp_find(const hp_table *t, int64_t k, int64_t s)
{
    for (int i = 0; i < t->n; ++i)
        if (t->c[i].k == k && t->c[i].s == s) return i;
    return -1;
}

static void hp_free_cell(hp_cell *c)
{
    free(c->H.str);
    free(c->E.str);
    free(c->F.str);
}

static void hp_clear(hp_table *t)
{
    for (int i = 0; i < t->n; ++i) hp_free_cell(&t->c[i]);
    t->n = 0;
}

/* the cell of interval (k, s), created with all scores at minus infinity
 * and no representatives when absent; -1 on allocation failure */
static int hp_get(hp_table *t, int64_t k, int64_t s)
{
    int i = hp_find(t, k, s);
    if (i >= 0) return i;
    if (t->n == t->cap) {
        int nc = t->cap ? 2 * t->cap : 64;
        hp_cell *nn = (hp_cell *)realloc(t->c, (size_t)nc * sizeof(hp_cell));
        if (!nn) return -1;
        t->c = nn;
        t->cap = nc;
    }
    hp_cell *c = &t->c[t->n];
    memset(c, 0, sizeof(*c));
    c->k = k;
    c->s = s;
    c->H.v = c->E.v = c->F.v = HP_NEG;
    return t->n++;
}

/* start of the SA interval of the reverse complement of str */
static int64_t hp_rc_start(const uint8_t *str, int len, void *h, const int64_t *S)
{
    static const uint8_t comp[6] = {0, 4, 3, 2, 1, 5};
    uint8_t *rc = (uint8_t *)malloc((size_t)(len > 0 ? len : 1));
    int64_t lo, hi;
    if (!rc) return -1;
    for (int j = 0; j < len; ++j) rc[j] = comp[str[len - 1 - j]];
    orc_sa_interval(h, S, rc, len, &lo, &hi);
    free(rc);
    return lo;
}

/* offer value v through string str to score x: it wins when higher, or
 * equal with a reverse complement whose interval starts first. Returns 1
 * when x changed, 0 when not, -1 on an allocation failure. */
static int hp_offer(hp_score *x, int v, const uint8_t *str, int len, void *h, const int64_t *S)
{
    if (v < x->v) return 0;
    const int64_t kr = hp_rc_start(str, len, h, S);
    if (kr < 0) return -1;
    if (v == x->v && x->str && kr >= x->kr) return 0;
    uint8_t *cp = (uint8_t *)malloc((size_t)(len > 0 ? len : 1));
    if (!cp) return -1;
    memcpy(cp, str, (size_t)len);
    free(x->str);
    x->str = cp;
    x->len = len;
    x->kr = kr;
    x->v = v;
    return 1;
}

/* the representative a gap passes on: that of the higher of a (opening
 * from H) and b (extending the gap), at a tie the one with the smaller kr */
static const hp_score *hp_gap_rep(const hp_score *H, int a, const hp_score *G, int b)
{
    if (a != b || !G->str) return a >= b ? H : G;
    return G->kr < H->kr ? G : H;
}

/* b prepended to str (len symbols), into buf; the SA interval of the
 * result (s = 0 if it does not occur) */
static void hp_child(const uint8_t *str, int len, int b, void *h, const int64_t *S, uint8_t *buf, int64_t *k,
                     int64_t *s)
{
    int64_t lo, hi;
    buf[0] = (uint8_t)b;
    memcpy(buf + 1, str, (size_t)len);
    orc_sa_interval(h, S, buf, len + 1, &lo, &hi);
    *k = lo;
    *s = hi - lo;
}

static int hp_better(const hp_cell *a, const hp_cell *b)
{
    if (a->H.v != b->H.v) return a->H.v > b->H.v;
    if (a->k != b->k) return a->k < b->k;
    return a->s < b->s;
}

static int hp_cmp(const void *x, const void *y)
{
    const hp_cell *a = (const hp_cell *)x, *b = (const hp_cell *)y;
    if (hp_better(a, b)) return -1;
    if (hp_better(b, a)) return 1;
    return 0;
}

static int hp_max(int a, int b) { return a > b ? a : b; }

/*
 * P (codes 1..5, length len) against the text handle h with suffix array S
 * of n rows. out: up to cap records of 5 int64 (k, kr, s, score, 0), in the
 * order of the result. *nraw gets the number of cells of u_0 before the
 * filter (raw: when non-NULL, those cells are written there instead, up to
 * cap, unfiltered). Returns the number of records after the filter, -1 on
 * an allocation failure.
 */
int64_t orc_hapl(void *h, const int64_t *S, int64_t n, const uint8_t *P, int64_t len, int match, int mismatch,
                 int gap_open, int gap_ext, int band, int64_t *out, int64_t cap, int64_t *nraw, int raw)
{
    hp_table A = {0, 0, 0}, B = {0, 0, 0};
    uint8_t *buf = (uint8_t *)calloc((size_t)(len + 4096), 1);
    uint8_t *rbuf = (uint8_t *)calloc((size_t)(len + 4096), 1);
    int64_t result = -1;
    int ok = buf != NULL && rbuf != NULL, maxlen = 4000;
    if (ok) {
        int r = hp_get(&A, 0, n); /* the root, interval [0, n), the empty string */
        if (r < 0 || hp_offer(&A.c[r].H, 0, buf, 0, h, S) < 0) ok = 0;
    }
    for (int64_t i = len - 1; ok && i >= 0; --i) {
        const int a = P[i];
        hp_clear(&B);
        /* match / mismatch and insertion from the cells of u' (A is not
         * changed meanwhile, so c's strings stay valid) */
        for (int x = 0; ok && x < A.n; ++x) {
            const hp_cell c = A.c[x];
            if (c.H.len >= maxlen) continue;
            for (int b = 1; ok && b <= 4; ++b) {
                int64_t k, s;
                hp_child(c.H.str, c.H.len, b, h, S, buf, &k, &s);
                if (s <= 0) continue;
                const int v = c.H.v + (a == b ? match : -mismatch);
                if (v <= 0) continue;
                int j = hp_get(&B, k, s);
                if (j < 0 || hp_offer(&B.c[j].H, v, buf, c.H.len + 1, h, S) < 0) ok = 0;
            }
            if (!ok) break;
            {
                const int eh = c.H.v - gap_open, ee = c.E.v;
                const int e = hp_max(eh, ee) - gap_ext;
                if (e > 0) {
                    const hp_score *rep = hp_gap_rep(&c.H, eh, &c.E, ee);
                    int j = hp_get(&B, c.k, c.s);
                    if (j < 0 || hp_offer(&B.c[j].E, e, rep->str, rep->len, h, S) < 0 ||
                        hp_offer(&B.c[j].H, e, rep->str, rep->len, h, S) < 0)
                        ok = 0;
                }
            }
        }
        /* deletion, repeated until no score of u improves (a higher score,
         * or the same with a representative of smaller k') */
        int changed = 1;
        while (ok && changed) {
            changed = 0;
            for (int x = 0; ok && x < B.n; ++x) {
                if (B.c[x].H.v <= 0) continue;
                const int fh = B.c[x].H.v - gap_open, ff = B.c[x].F.v;
                const int f = hp_max(fh, ff) - gap_ext;
                if (f <= 0) continue;
                const hp_score *rep = hp_gap_rep(&B.c[x].H, fh, &B.c[x].F, ff);
                const int rl = rep->len;
                if (rl >= maxlen) continue;
                memcpy(rbuf, rep->str, (size_t)rl); /* hp_get may move B's cells */
                for (int b = 1; ok && b <= 4; ++b) {
                    int64_t k, s;
                    hp_child(rbuf, rl, b, h, S, buf, &k, &s);
                    if (s <= 0) continue;
                    int j = hp_get(&B, k, s);
                    if (j < 0) { ok = 0; break; }
                    const int r1 = hp_offer(&B.c[j].F, f, buf, rl + 1, h, S);
                    const int r2 = hp_offer(&B.c[j].H, f, buf, rl + 1, h, S);
                    if (r1 < 0 || r2 < 0) ok = 0;
                    if (r1 > 0 || r2 > 0) changed = 1;
                }
            }
        }
        if (!ok) break;
        /* keep H > 0, then the band */
        int w = 0;
        for (int x = 0; x < B.n; ++x) {
            if (B.c[x].H.v > 0) B.c[w++] = B.c[x];
            else hp_free_cell(&B.c[x]);
        }
        B.n = w;
        qsort(B.c, (size_t)B.n, sizeof(hp_cell), hp_cmp);
        if (band > 0 && B.n > band) {
            for (int x = band; x < B.n; ++x) hp_free_cell(&B.c[x]);
            B.n = band;
        }
        hp_table t = A;
        A = B;
        B = t;
    }
    if (ok) {
        /* A holds the cells of u_0 (ordered; the root of an empty query has
         * H = 0 and is not a result) */
        int64_t w = 0;
        {
            int z = 0;
            for (int x = 0; x < A.n; ++x) {
                if (A.c[x].H.v > 0) A.c[z++] = A.c[x];
                else hp_free_cell(&A.c[x]);
            }
            A.n = z;
        }
        if (nraw) *nraw = A.n;
        if (raw) {
            for (int x = 0; x < A.n && x < cap; ++x) {
                out[5 * x] = A.c[x].k;
                out[5 * x + 1] = A.c[x].H.kr;
                out[5 * x + 2] = A.c[x].s;
                out[5 * x + 3] = A.c[x].H.v;
                out[5 * x + 4] = 0;
            }
            w = A.n;
        } else {
            char *drop = (char *)calloc((size_t)(A.n > 0 ? A.n : 1), 1);
            if (!drop) ok = 0;
            for (int x = 0; ok && x < A.n; ++x) {
                for (int y = 0; y < x && !drop[x]; ++y) {
                    if (drop[y]) continue;
                    const hp_cell *p = &A.c[y], *q = &A.c[x];
                    if ((q->k >= p->k && q->k + q->s <= p->k + p->s) ||
                        (q->H.kr >= p->H.kr && q->H.kr + q->s <= p->H.kr + p->s))
                        drop[x] = 1;
                }
                if (!drop[x]) {
                    if (w < cap) {
                        out[5 * w] = A.c[x].k;
                        out[5 * w + 1] = A.c[x].H.kr;
                        out[5 * w + 2] = A.c[x].s;
                        out[5 * w + 3] = A.c[x].H.v;
                        out[5 * w + 4] = 0;
                    }
                    ++w;
                }
            }
            free(drop);
        }
        if (ok) result = w;
    }
    hp_clear(&A);
    hp_clear(&B);
    free(A.c);
    free(B.c);
    free(buf);
    free(rbuf);
    return result;
}
