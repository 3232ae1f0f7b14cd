/*
 * Seeded synthetic bipartite-graph generators (CSC, int32).
 *
 * This file holds no matching arithmetic: it only draws sparsity patterns.
 * Both the matching library's tests/benchmarks and the CPU reference take
 * their inputs from here, so both sides always see byte-identical graphs.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  The i-th output of a
 * stream seeded with s is fmix(s + (i+1)*GAMMA); that makes every stream
 * counter-based, so the large generators can draw in parallel and still be
 * deterministic.
 *
 * Conventions of every generated graph:
 *   colptr[nc+1], colptr[0] = 0, rowind[colptr[c] .. colptr[c+1]) are the
 *   rows of column c, sorted ascending, without duplicates.
 *
 * Memory returned through gg_graph is malloc'ed here and released with
 * gg_free().  Functions return 0 on success, -1 on bad arguments, -2 when
 * an allocation fails.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define GG_GAMMA 0x9e3779b97f4a7c15ULL

typedef struct {
    int32_t nc, nr;
    int64_t nnz;
    int32_t *colptr; /* [nc+1] */
    int32_t *rowind; /* [nnz]  */
} gg_graph;

static inline uint64_t gg_fmix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* i-th output (i >= 0) of the SplitMix64 stream seeded with `seed`. */
static inline uint64_t gg_at(uint64_t seed, uint64_t i) { return gg_fmix(seed + (i + 1) * GG_GAMMA); }

typedef struct { uint64_t s; } gg_rng;
static inline uint64_t gg_next(gg_rng *g) { g->s += GG_GAMMA; return gg_fmix(g->s); }
/* uniform integer in [0, n), n < 2^32 (multiply-shift; bias < n / 2^32) */
static inline uint32_t gg_below(uint64_t x, uint32_t n) { return (uint32_t)(((x >> 32) * (uint64_t)n) >> 32); }
/* uniform double in [0, 1) with 53 random bits */
static inline double gg_unit(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

/* Derived seed for sub-stream b of master seed a (used per graph / per request). */
uint64_t gg_seed_mix(uint64_t a, uint64_t b) { return gg_fmix(gg_fmix(a + GG_GAMMA) ^ (b * 0xd1b54a32d192ed03ULL + 0x632be59bd9b4e019ULL)); }

void gg_free(gg_graph *g)
{
    if (!g) return;
    free(g->colptr);
    free(g->rowind);
    g->colptr = g->rowind = NULL;
    g->nnz = 0;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static void isort(int32_t *a, int64_t n)
{
    if (n > 48) { qsort(a, (size_t)n, sizeof(int32_t), cmp_i32); return; }
    for (int64_t i = 1; i < n; ++i) {
        int32_t v = a[i];
        int64_t j = i - 1;
        while (j >= 0 && a[j] > v) { a[j + 1] = a[j]; --j; }
        a[j + 1] = v;
    }
}

/* Sort every column in place, drop duplicates, compact; colptr rewritten. */
static void sort_dedup_compact(int32_t nc, int64_t *cptr64, int32_t *rowind, int32_t *colptr_out)
{
    int64_t w = 0;
    for (int32_t c = 0; c < nc; ++c) {
        int64_t b = cptr64[c], e = cptr64[c + 1];
        isort(rowind + b, e - b);
        colptr_out[c] = (int32_t)w;
        for (int64_t j = b; j < e; ++j)
            if (j == b || rowind[j] != rowind[j - 1]) rowind[w++] = rowind[j];
    }
    colptr_out[nc] = (int32_t)w;
}

/* -------- uniform: every column draws `deg` rows uniformly ------------- */
/* replace=1: with replacement then deduplicated (degree <= deg);
 * replace=0: `min(deg, nr)` distinct rows (rejection of repeats).       */
int gg_uniform(int32_t nc, int32_t nr, int32_t deg, int replace, uint64_t seed, gg_graph *out)
{
    if (nc < 0 || nr < 0 || deg < 0 || !out) return -1;
    memset(out, 0, sizeof *out);
    out->nc = nc; out->nr = nr;
    int32_t d = (nr == 0) ? 0 : deg;
    if (!replace && d > nr) d = nr;
    int64_t cap = (int64_t)nc * d;
    int64_t *cp = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nc + 1));
    out->colptr = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nc + 1));
    out->rowind = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
    if (!cp || !out->colptr || !out->rowind) { free(cp); gg_free(out); return -2; }
    gg_rng g = { seed };
    int64_t k = 0;
    for (int32_t c = 0; c < nc; ++c) {
        cp[c] = k;
        int64_t b = k;
        while (k - b < d) {
            int32_t r = (int32_t)gg_below(gg_next(&g), (uint32_t)nr);
            if (!replace) {
                int dup = 0;
                for (int64_t j = b; j < k; ++j) if (out->rowind[j] == r) { dup = 1; break; }
                if (dup) continue;
            }
            out->rowind[k++] = r;
        }
    }
    cp[nc] = k;
    sort_dedup_compact(nc, cp, out->rowind, out->colptr);
    out->nnz = out->colptr[nc];
    free(cp);
    return 0;
}

/* Draw k distinct values of [0, n) by a partial Fisher-Yates shuffle. */
static int sample_without_replacement(int64_t n, int64_t k, gg_rng *g, uint8_t *mark)
{
    int32_t *a = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!a) return -2;
    for (int64_t i = 0; i < n; ++i) a[i] = (int32_t)i;
    for (int64_t i = 0; i < k; ++i) {
        int64_t j = i + gg_below(gg_next(g), (uint32_t)(n - i));
        int32_t t = a[i]; a[i] = a[j]; a[j] = t;
        mark[a[i]] = 1;
    }
    free(a);
    return 0;
}

/* -------- 5-point grid with deleted columns and rows ------------------- */
/* Vertex (i,j) of a k x k grid has id i*k+j on both sides.  Column (i,j)
 * holds rows (i-1,j), (i,j-1), (i,j), (i,j+1), (i+1,j) that lie inside the
 * grid.  `ndel_cols` columns and, independently, `ndel_rows` rows are
 * picked uniformly without replacement (columns first) and every entry in a
 * picked column or row is removed; the dimensions stay k*k.  If del_cols /
 * del_rows are non-NULL they receive the 0/1 masks of picked ids.          */
int gg_grid5(int32_t k, int64_t ndel_cols, int64_t ndel_rows, uint64_t seed, gg_graph *out,
             uint8_t *del_cols, uint8_t *del_rows)
{
    if (k < 0 || !out) return -1;
    int64_t n = (int64_t)k * k;
    if (n > INT32_MAX || ndel_cols < 0 || ndel_rows < 0 || ndel_cols > n || ndel_rows > n) return -1;
    memset(out, 0, sizeof *out);
    out->nc = out->nr = (int32_t)n;
    uint8_t *dc = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    uint8_t *dr = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    out->colptr = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    out->rowind = (int32_t *)malloc(sizeof(int32_t) * (size_t)(5 * n + 1));
    if (!dc || !dr || !out->colptr || !out->rowind) { free(dc); free(dr); gg_free(out); return -2; }
    gg_rng g = { seed };
    if (sample_without_replacement(n, ndel_cols, &g, dc) || sample_without_replacement(n, ndel_rows, &g, dr)) {
        free(dc); free(dr); gg_free(out); return -2;
    }
    int64_t w = 0;
    for (int64_t c = 0; c < n; ++c) {
        out->colptr[c] = (int32_t)w;
        if (dc[c]) continue;
        int64_t i = c / k, j = c % k;
        int64_t cand[5]; int nc5 = 0;
        if (i > 0) cand[nc5++] = c - k;
        if (j > 0) cand[nc5++] = c - 1;
        cand[nc5++] = c;
        if (j + 1 < k) cand[nc5++] = c + 1;
        if (i + 1 < k) cand[nc5++] = c + k;
        for (int t = 0; t < nc5; ++t)
            if (!dr[cand[t]]) out->rowind[w++] = (int32_t)cand[t];
    }
    out->colptr[n] = (int32_t)w;
    out->nnz = w;
    if (del_cols) memcpy(del_cols, dc, (size_t)n);
    if (del_rows) memcpy(del_rows, dr, (size_t)n);
    free(dc); free(dr);
    return 0;
}

/* -------- R-MAT ---------------------------------------------------------- */
/* `nsamples` edges, each from `scale` quadrant choices (MSB first) with
 * probabilities a: (row bit 0, col bit 0), b: (0, 1), c: (1, 0),
 * d = 1-a-b-c: (1, 1).  Sample s uses draws s*scale .. s*scale+scale-1 of
 * the counter stream.  Samples with row or column >= n_limit are dropped
 * (n_limit <= 0 means 2^scale).  Duplicates removed.  With permute=1 a
 * uniformly random permutation is applied to the rows and then to the
 * columns (Fisher-Yates on a stream derived from the seed).              */
int gg_rmat(int32_t scale, int64_t nsamples, double a, double b, double c, int32_t n_limit,
            int permute, uint64_t seed, gg_graph *out)
{
    if (scale < 0 || scale > 30 || nsamples < 0 || !out) return -1;
    int64_t n = (int64_t)1 << scale;
    if (n_limit > 0 && n_limit < n) n = n_limit;
    memset(out, 0, sizeof *out);
    out->nc = out->nr = (int32_t)n;
    const double ab = a + b, abc = a + b + c;
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cnt) return -2;

    /* pass 1: column counts */
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < nsamples; ++s) {
        uint64_t base = (uint64_t)s * (uint64_t)scale;
        int64_t row = 0, col = 0;
        for (int32_t t = 0; t < scale; ++t) {
            double u = gg_unit(gg_at(seed, base + t));
            int64_t bit = (int64_t)1 << (scale - 1 - t);
            if (u < a) {}
            else if (u < ab) col |= bit;
            else if (u < abc) row |= bit;
            else { row |= bit; col |= bit; }
        }
        if (row >= n || col >= n) continue;
        #pragma omp atomic
        cnt[col + 1]++;
    }
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    int64_t total = cnt[n];
    int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!rows || !cur) { free(cnt); free(rows); free(cur); return -2; }
    memcpy(cur, cnt, sizeof(int64_t) * (size_t)n);

    /* pass 2: scatter rows into their column buckets (order inside a
     * bucket is irrelevant: buckets are sorted afterwards)              */
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < nsamples; ++s) {
        uint64_t base = (uint64_t)s * (uint64_t)scale;
        int64_t row = 0, col = 0;
        for (int32_t t = 0; t < scale; ++t) {
            double u = gg_unit(gg_at(seed, base + t));
            int64_t bit = (int64_t)1 << (scale - 1 - t);
            if (u < a) {}
            else if (u < ab) col |= bit;
            else if (u < abc) row |= bit;
            else { row |= bit; col |= bit; }
        }
        if (row >= n || col >= n) continue;
        int64_t pos;
        #pragma omp atomic capture
        pos = cur[col]++;
        rows[pos] = (int32_t)row;
    }
    free(cur);

    int32_t *pr = NULL, *pc = NULL;
    if (permute) {
        pr = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        pc = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        if (!pr || !pc) { free(cnt); free(rows); free(pr); free(pc); return -2; }
        gg_rng g = { gg_seed_mix(seed, 0x5045524dULL) };
        for (int64_t i = 0; i < n; ++i) { pr[i] = (int32_t)i; pc[i] = (int32_t)i; }
        for (int64_t i = n - 1; i > 0; --i) { int64_t j = gg_below(gg_next(&g), (uint32_t)(i + 1)); int32_t t = pr[i]; pr[i] = pr[j]; pr[j] = t; }
        for (int64_t i = n - 1; i > 0; --i) { int64_t j = gg_below(gg_next(&g), (uint32_t)(i + 1)); int32_t t = pc[i]; pc[i] = pc[j]; pc[j] = t; }
        #pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < total; ++j) rows[j] = pr[rows[j]];
    }

    /* sort + dedup each (old) column in place */
    int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!deg) { free(cnt); free(rows); free(pr); free(pc); return -2; }
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t col = 0; col < n; ++col) {
        int64_t b0 = cnt[col], e0 = cnt[col + 1];
        isort(rows + b0, e0 - b0);
        int64_t w = b0;
        for (int64_t j = b0; j < e0; ++j)
            if (j == b0 || rows[j] != rows[j - 1]) rows[w++] = rows[j];
        deg[col] = w - b0;
    }
    /* new column of old column `col` is pc[col] (identity without permute) */
    int64_t *ncp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!ncp) { free(cnt); free(rows); free(pr); free(pc); free(deg); return -2; }
    for (int64_t col = 0; col < n; ++col) ncp[(pc ? pc[col] : col) + 1] = deg[col];
    for (int64_t i = 0; i < n; ++i) ncp[i + 1] += ncp[i];
    int64_t nnz = ncp[n];
    if (nnz > INT32_MAX) { free(cnt); free(rows); free(pr); free(pc); free(deg); free(ncp); return -1; }
    out->colptr = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    out->rowind = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!out->colptr || !out->rowind) { free(cnt); free(rows); free(pr); free(pc); free(deg); free(ncp); gg_free(out); return -2; }
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t col = 0; col < n; ++col) {
        int64_t dst = ncp[pc ? pc[col] : col];
        memcpy(out->rowind + dst, rows + cnt[col], sizeof(int32_t) * (size_t)deg[col]);
    }
    for (int64_t i = 0; i <= n; ++i) out->colptr[i] = (int32_t)ncp[i];
    out->nnz = nnz;
    free(cnt); free(rows); free(pr); free(pc); free(deg); free(ncp);
    return 0;
}

/* -------- one member of the uneven batch -------------------------------- */
/* Graph g of a batch with master seed `seed`: sub-seed s = gg_seed_mix(seed, g).
 * nc and nr are each round(exp(U[ln lo, ln hi])); every column draws a
 * degree uniform in {dmin..dmax} capped at nr.  Even g: rows uniform
 * without replacement.  Odd g: banded, centre floor(c*nr/nc), window
 * [centre-halfband, centre+halfband] intersected with [0, nr), and
 * min(degree, window size) rows drawn without replacement from it.  Then
 * floor(empty_frac*nc) columns, drawn without replacement, are emptied.   */
int gg_batch_member(uint64_t seed, int64_t gidx, int32_t lo, int32_t hi, int32_t dmin, int32_t dmax,
                    int32_t halfband, double empty_frac, gg_graph *out)
{
    if (!out || lo < 1 || hi < lo || dmin < 0 || dmax < dmin || halfband < 0) return -1;
    memset(out, 0, sizeof *out);
    gg_rng g = { gg_seed_mix(seed, (uint64_t)gidx) };
    double llo = log((double)lo), lhi = log((double)hi);
    int32_t nc = (int32_t)llround(exp(llo + (lhi - llo) * gg_unit(gg_next(&g))));
    int32_t nr = (int32_t)llround(exp(llo + (lhi - llo) * gg_unit(gg_next(&g))));
    out->nc = nc; out->nr = nr;
    int banded = (int)(gidx & 1);
    int64_t cap = (int64_t)nc * dmax;
    int64_t *cp = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nc + 1));
    out->colptr = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nc + 1));
    out->rowind = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
    uint8_t *empty = (uint8_t *)calloc((size_t)nc + 1, 1);
    if (!cp || !out->colptr || !out->rowind || !empty) { free(cp); free(empty); gg_free(out); return -2; }
    int64_t k = 0;
    for (int32_t c = 0; c < nc; ++c) {
        cp[c] = k;
        int32_t d = dmin + (int32_t)gg_below(gg_next(&g), (uint32_t)(dmax - dmin + 1));
        if (d > nr) d = nr;
        int32_t wlo = 0, wsz = nr;
        if (banded) {
            int64_t centre = ((int64_t)c * nr) / nc;
            int64_t a0 = centre - halfband, b0 = centre + halfband;
            if (a0 < 0) a0 = 0;
            if (b0 > nr - 1) b0 = nr - 1;
            wlo = (int32_t)a0; wsz = (int32_t)(b0 - a0 + 1);
            if (d > wsz) d = wsz;
        }
        int64_t b = k;
        while (k - b < d) {
            int32_t r = wlo + (int32_t)gg_below(gg_next(&g), (uint32_t)wsz);
            int dup = 0;
            for (int64_t j = b; j < k; ++j) if (out->rowind[j] == r) { dup = 1; break; }
            if (!dup) out->rowind[k++] = r;
        }
    }
    cp[nc] = k;
    int64_t ne = (int64_t)floor(empty_frac * (double)nc);
    if (sample_without_replacement(nc, ne, &g, empty)) { free(cp); free(empty); gg_free(out); return -2; }
    /* empty the picked columns, then sort/dedup/compact */
    int64_t w = 0;
    for (int32_t c = 0; c < nc; ++c) {
        int64_t b = cp[c], e = cp[c + 1];
        isort(out->rowind + b, e - b);
        out->colptr[c] = (int32_t)w;
        if (!empty[c])
            for (int64_t j = b; j < e; ++j)
                if (j == b || out->rowind[j] != out->rowind[j - 1]) out->rowind[w++] = out->rowind[j];
    }
    out->colptr[nc] = (int32_t)w;
    out->nnz = w;
    free(cp); free(empty);
    return 0;
}

/* -------- helpers ---------------------------------------------------------- */
/* CSR (row -> columns, columns ascending) of a CSC graph. */
/* -------- random row and column permutation of a pattern ---------------- */
/* The RCP transform: new row of old row r is pr[r], new column of old
 * column c is pc[c], both drawn by Fisher-Yates from `seed` (rows first);
 * rows sorted within each new column.  Matching sizes are invariant under
 * it; the structure the BFS sees is not.                                  */
int gg_permute(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind, uint64_t seed, gg_graph *out)
{
    if (!out || nc < 0 || nr < 0 || !colptr) return -1;
    memset(out, 0, sizeof *out);
    const int64_t nnz = colptr[nc];
    int32_t *pr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nr > 0 ? nr : 1));
    int32_t *pc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
    out->colptr = (int32_t *)calloc((size_t)nc + 1, sizeof(int32_t));
    out->rowind = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!pr || !pc || !out->colptr || !out->rowind) { free(pr); free(pc); gg_free(out); return -2; }
    gg_rng g = { gg_seed_mix(seed, 0x52435050ULL) };
    for (int32_t i = 0; i < nr; ++i) pr[i] = i;
    for (int32_t i = 0; i < nc; ++i) pc[i] = i;
    for (int64_t i = (int64_t)nr - 1; i > 0; --i) { int64_t j = gg_below(gg_next(&g), (uint32_t)(i + 1)); int32_t t = pr[i]; pr[i] = pr[j]; pr[j] = t; }
    for (int64_t i = (int64_t)nc - 1; i > 0; --i) { int64_t j = gg_below(gg_next(&g), (uint32_t)(i + 1)); int32_t t = pc[i]; pc[i] = pc[j]; pc[j] = t; }
    for (int32_t c = 0; c < nc; ++c) out->colptr[pc[c] + 1] = colptr[c + 1] - colptr[c];
    for (int32_t i = 0; i < nc; ++i) out->colptr[i + 1] += out->colptr[i];
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int32_t c = 0; c < nc; ++c) {
        int32_t *dst = out->rowind + out->colptr[pc[c]];
        const int32_t b = colptr[c], e = colptr[c + 1];
        for (int32_t j = b; j < e; ++j) dst[j - b] = pr[rowind[j]];
        isort(dst, e - b);
    }
    out->nc = nc;
    out->nr = nr;
    out->nnz = nnz;
    free(pr);
    free(pc);
    return 0;
}

int gg_transpose(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind,
                 int32_t *rowptr, int32_t *colind)
{
    if (nc < 0 || nr < 0) return -1;
    memset(rowptr, 0, sizeof(int32_t) * ((size_t)nr + 1));
    int64_t nnz = colptr[nc];
    for (int64_t j = 0; j < nnz; ++j) rowptr[rowind[j] + 1]++;
    for (int32_t r = 0; r < nr; ++r) rowptr[r + 1] += rowptr[r];
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nr + 1));
    if (!cur) return -2;
    memcpy(cur, rowptr, sizeof(int32_t) * (size_t)nr);
    for (int32_t c = 0; c < nc; ++c)
        for (int64_t j = colptr[c]; j < colptr[c + 1]; ++j) colind[cur[rowind[j]]++] = c;
    free(cur);
    return 0;
}

/* 64-bit FNV-1a over colptr bytes then rowind bytes: identifies an input
 * on both machines. */
uint64_t gg_fnv1a(int32_t nc, const int32_t *colptr, const int32_t *rowind)
{
    uint64_t h = 0xcbf29ce484222325ULL;
    const uint8_t *p = (const uint8_t *)colptr;
    size_t n1 = sizeof(int32_t) * ((size_t)nc + 1);
    for (size_t i = 0; i < n1; ++i) { h ^= p[i]; h *= 0x100000001b3ULL; }
    p = (const uint8_t *)rowind;
    size_t n2 = sizeof(int32_t) * (size_t)colptr[nc];
    for (size_t i = 0; i < n2; ++i) { h ^= p[i]; h *= 0x100000001b3ULL; }
    return h;
}

/* Exponential inter-arrival gaps (seconds) of a Poisson stream with rate
 * `lambda`, and per-request size draws for a mixed request trace:
 * n = round(exp(U[ln lo, ln hi])), degree uniform {dmin..dmax}, kind 0 =
 * uniform, 1 = R-MAT with probability 1/2, per-request seed.              */
int gg_request_trace(uint64_t seed, int64_t count, double lambda, int32_t lo, int32_t hi,
                     int32_t dmin, int32_t dmax, double *gap, int32_t *n, int32_t *deg,
                     int32_t *kind, uint64_t *rseed)
{
    if (count < 0 || lambda <= 0 || lo < 1 || hi < lo || dmax < dmin) return -1;
    gg_rng g = { seed };
    double llo = log((double)lo), lhi = log((double)hi);
    for (int64_t i = 0; i < count; ++i) {
        double u = gg_unit(gg_next(&g));
        gap[i] = -log(1.0 - u) / lambda;
        n[i] = (int32_t)llround(exp(llo + (lhi - llo) * gg_unit(gg_next(&g))));
        deg[i] = dmin + (int32_t)gg_below(gg_next(&g), (uint32_t)(dmax - dmin + 1));
        kind[i] = (int32_t)(gg_next(&g) >> 63);
        rseed[i] = gg_seed_mix(seed, (uint64_t)i + 1);
    }
    return 0;
}
