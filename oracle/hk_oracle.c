/*
 * CPU reference ("oracle") for maximum-cardinality bipartite matching.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the matching library calls, links
 * or loads this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the GPU path.
 *
 * Problem (paper, section 2): a matching M of a bipartite graph is a set of
 * edges no two of which share a vertex; its cardinality |M| is the number
 * of edges; M is maximum when no matching is larger.  By Berge's theorem M
 * is maximum iff it admits no M-augmenting path (an alternating path whose
 * two end vertices are unmatched).
 *
 * Graph layout (paper, section 3, problem statement of Algorithm 1): the
 * adjacency of the column vertices in compressed form, colptr[nc+1] and
 * rowind[nnz]; the rows of column c are rowind[colptr[c] .. colptr[c+1]).
 * A matching is given by cmatch[nc] and rmatch[nr]: cmatch[c] = r and
 * rmatch[r] = c when (c, r) is in M, -1 for an unmatched vertex.
 *
 * Functions:
 *   orc_check_csc        the input is well formed
 *   orc_check_matching   (cmatch, rmatch) is a matching of the graph
 *   orc_cheap_init       the greedy initial matching used before every run
 *                        (paper, section 4, experimental setup)
 *   orc_hopcroft_karp    Hopcroft-Karp from a given matching (section 2)
 *   orc_konig_cover      minimum vertex cover from the final alternating BFS
 *   orc_verify_cover     independent certificate check (weak duality)
 *   orc_brute_force      maximum matching size by exhaustive search (tiny)
 *   orc_alt_bfs_levels   alternating-BFS levels from all unmatched columns
 *
 * All sizes fit int32 except nnz sums, kept in int64.  Return codes: >= 0
 * a result, -1 bad argument or malformed input, -2 out of memory.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_INF INT32_MAX

/* colptr monotone from 0, every row index in [0, nr). */
int orc_check_csc(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind)
{
    if (nc < 0 || nr < 0 || !colptr) return -1;
    if (colptr[0] != 0) return -1;
    for (int32_t c = 0; c < nc; ++c)
        if (colptr[c + 1] < colptr[c]) return -1;
    for (int64_t j = 0; j < colptr[nc]; ++j)
        if (rowind[j] < 0 || rowind[j] >= nr) return -1;
    return 0;
}

static int has_edge(const int32_t *colptr, const int32_t *rowind, int32_t c, int32_t r)
{
    for (int64_t j = colptr[c]; j < colptr[c + 1]; ++j)
        if (rowind[j] == r) return 1;
    return 0;
}

/* 0 if cmatch/rmatch describe a matching of the graph (symmetric, on
 * edges, values in range or -1), else -1.  Returns |M| through *card.  */
int orc_check_matching(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind,
                       const int32_t *cmatch, const int32_t *rmatch, int64_t *card)
{
    int64_t m = 0;
    for (int32_t c = 0; c < nc; ++c) {
        int32_t r = cmatch[c];
        if (r == -1) continue;
        if (r < 0 || r >= nr) return -1;
        if (rmatch[r] != c) return -1;
        if (!has_edge(colptr, rowind, c, r)) return -1;
        ++m;
    }
    int64_t mr = 0;
    for (int32_t r = 0; r < nr; ++r) {
        int32_t c = rmatch[r];
        if (c == -1) continue;
        if (c < 0 || c >= nc) return -1;
        if (cmatch[c] != r) return -1;
        ++mr;
    }
    if (m != mr) return -1;
    if (card) *card = m;
    return 0;
}

/* Greedy initial matching: columns in index order, each takes the first
 * row of its stored adjacency that is still unmatched.  Starts from empty. */
void orc_cheap_init(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind,
                    int32_t *cmatch, int32_t *rmatch)
{
    for (int32_t c = 0; c < nc; ++c) cmatch[c] = -1;
    for (int32_t r = 0; r < nr; ++r) rmatch[r] = -1;
    for (int32_t c = 0; c < nc; ++c) {
        for (int64_t j = colptr[c]; j < colptr[c + 1]; ++j) {
            int32_t r = rowind[j];
            if (rmatch[r] == -1) {
                cmatch[c] = r;
                rmatch[r] = c;
                break;
            }
        }
    }
}

/*
 * Hopcroft-Karp, starting from the matching in (cmatch, rmatch), which it
 * updates in place.  Each phase:
 *   1. BFS layering from every unmatched column (distance 0), through
 *      matched edges; `limit` becomes the length (in columns) of the
 *      shortest augmenting path, the search stops expanding at that layer.
 *   2. DFS restricted to the layered graph from every unmatched column,
 *      augmenting along vertex-disjoint shortest paths (columns used by an
 *      augmentation or found dead leave the layered graph).
 * Stops when the BFS reaches no unmatched row.  Returns |M|; the number of
 * phases that augmented is stored in *phases.
 */
int64_t orc_hopcroft_karp_ex(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind,
                             int32_t *cmatch, int32_t *rmatch, int64_t max_phases, int64_t *phases,
                             int64_t *edges_scanned);

int64_t orc_hopcroft_karp(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind,
                          int32_t *cmatch, int32_t *rmatch, int64_t *phases)
{
    return orc_hopcroft_karp_ex(nc, nr, colptr, rowind, cmatch, rmatch, INT64_MAX, phases, NULL);
}

/* Same, stopping after at most max_phases augmenting phases (the matching
 * is then valid but possibly not maximum); *edges_scanned (if non-NULL)
 * receives the number of adjacency entries read by the BFS and DFS steps. */
int64_t orc_hopcroft_karp_ex(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind,
                             int32_t *cmatch, int32_t *rmatch, int64_t max_phases, int64_t *phases,
                             int64_t *edges_scanned)
{
    (void)nr;
    int64_t nedges = 0;
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nc + 1));
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nc + 1));
    int64_t *it = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nc + 1));
    int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nc + 1));
    if (!dist || !queue || !it || !stack) {
        free(dist); free(queue); free(it); free(stack);
        return -2;
    }
    int64_t nph = 0;
    for (;;) {
        /* 1. layered BFS */
        int64_t qh = 0, qt = 0;
        for (int32_t c = 0; c < nc; ++c) {
            if (cmatch[c] == -1) { dist[c] = 0; queue[qt++] = c; }
            else dist[c] = ORC_INF;
        }
        int32_t limit = ORC_INF;
        while (qh < qt) {
            int32_t c = queue[qh++];
            if (dist[c] >= limit) continue;
            nedges += colptr[c + 1] - colptr[c];
            for (int64_t j = colptr[c]; j < colptr[c + 1]; ++j) {
                int32_t r = rowind[j];
                int32_t m = rmatch[r];
                if (m == -1) {
                    if (limit == ORC_INF) limit = dist[c] + 1;
                } else if (dist[m] == ORC_INF) {
                    dist[m] = dist[c] + 1;
                    queue[qt++] = m;
                }
            }
        }
        if (limit == ORC_INF) break;

        /* 2. DFS over the layered graph, one root at a time */
        for (int32_t c = 0; c < nc; ++c) it[c] = colptr[c];
        int64_t augmented = 0;
        for (int32_t root = 0; root < nc; ++root) {
            if (cmatch[root] != -1 || dist[root] != 0) continue;
            int32_t top = 0;
            stack[0] = root;
            while (top >= 0) {
                int32_t u = stack[top];
                if (it[u] == colptr[u + 1]) {     /* exhausted: dead end */
                    dist[u] = ORC_INF;
                    --top;
                    continue;
                }
                int32_t r = rowind[it[u]++];
                ++nedges;
                int32_t m = rmatch[r];
                if (m == -1) {
                    if (dist[u] + 1 != limit) continue;
                    /* augment: stack[k] takes the row it last advanced over */
                    int32_t row = r;
                    for (int32_t k = top; k >= 0; --k) {
                        int32_t col = stack[k];
                        int32_t prev = cmatch[col];
                        cmatch[col] = row;
                        rmatch[row] = col;
                        dist[col] = ORC_INF; /* leaves the layered graph */
                        row = prev;
                    }
                    ++augmented;
                    break;
                }
                if (dist[m] != ORC_INF && dist[m] == dist[u] + 1)
                    stack[++top] = m;
            }
        }
        ++nph;
        if (augmented == 0) break; /* cannot happen when limit < INF; kept as a guard */
        if (nph >= max_phases) break;
    }
    int64_t card = 0;
    for (int32_t c = 0; c < nc; ++c) card += (cmatch[c] >= 0);
    if (phases) *phases = nph;
    if (edges_scanned) *edges_scanned = nedges;
    free(dist); free(queue); free(it); free(stack);
    return card;
}

/*
 * Konig's theorem: from a maximum matching, let Z_C be the columns reached
 * by the alternating BFS from all unmatched columns and Z_R the rows
 * adjacent to Z_C.  K = (C \ Z_C) u Z_R is a vertex cover with |K| = |M|.
 * Fills col_in_cover[nc] and row_in_cover[nr] with 0/1 and returns |K|,
 * or -3 if the BFS reaches an unmatched row (the matching is not maximum).
 */
int64_t orc_konig_cover(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind,
                        const int32_t *cmatch, const int32_t *rmatch,
                        uint8_t *col_in_cover, uint8_t *row_in_cover)
{
    uint8_t *zc = (uint8_t *)calloc((size_t)nc + 1, 1);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nc + 1));
    if (!zc || !queue) { free(zc); free(queue); return -2; }
    int64_t qh = 0, qt = 0;
    for (int32_t c = 0; c < nc; ++c)
        if (cmatch[c] == -1) { zc[c] = 1; queue[qt++] = c; }
    memset(row_in_cover, 0, (size_t)nr);
    int64_t bad = 0;
    while (qh < qt) {
        int32_t c = queue[qh++];
        for (int64_t j = colptr[c]; j < colptr[c + 1]; ++j) {
            int32_t r = rowind[j];
            row_in_cover[r] = 1;
            int32_t m = rmatch[r];
            if (m == -1) { bad = 1; continue; }
            if (!zc[m]) { zc[m] = 1; queue[qt++] = m; }
        }
    }
    int64_t k = 0;
    for (int32_t c = 0; c < nc; ++c) {
        col_in_cover[c] = (uint8_t)(cmatch[c] != -1 && !zc[c]);
        k += col_in_cover[c];
    }
    for (int32_t r = 0; r < nr; ++r) k += row_in_cover[r];
    free(zc); free(queue);
    return bad ? -3 : k;
}

/*
 * Independent certificate check.  Returns 0 when
 *   (i)   cmatch/rmatch is a matching of the graph,
 *   (ii)  every edge has an endpoint in the cover, and
 *   (iii) |cover| == |M|;
 * then M is maximum by weak duality (no matching exceeds any cover).
 * Otherwise returns 1, 2 or 3, the first property that fails.
 */
int orc_verify_cover(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind,
                     const int32_t *cmatch, const int32_t *rmatch,
                     const uint8_t *col_in_cover, const uint8_t *row_in_cover)
{
    int64_t m = 0, k = 0;
    for (int32_t c = 0; c < nc; ++c) {
        int32_t r = cmatch[c];
        if (r == -1) continue;
        if (r < 0 || r >= nr || rmatch[r] != c) return 1;
        int on_edge = 0;
        for (int64_t j = colptr[c]; j < colptr[c + 1]; ++j) on_edge |= (rowind[j] == r);
        if (!on_edge) return 1;
        ++m;
    }
    for (int32_t r = 0; r < nr; ++r) {
        int32_t c = rmatch[r];
        if (c != -1 && (c < 0 || c >= nc || cmatch[c] != r)) return 1;
    }
    for (int32_t c = 0; c < nc; ++c)
        for (int64_t j = colptr[c]; j < colptr[c + 1]; ++j)
            if (!col_in_cover[c] && !row_in_cover[rowind[j]]) return 2;
    for (int32_t c = 0; c < nc; ++c) k += (col_in_cover[c] != 0);
    for (int32_t r = 0; r < nr; ++r) k += (row_in_cover[r] != 0);
    return (k == m) ? 0 : 3;
}

/*
 * Exhaustive maximum matching size for tiny graphs (nr <= 20): best[mask]
 * over columns processed so far, mask = set of rows already used.
 * Column c either stays unmatched or takes one unused neighbour.
 */
int64_t orc_brute_force(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind)
{
    if (nr < 0 || nr > 20 || nc < 0) return -1;
    size_t states = (size_t)1 << nr;
    int8_t *cur = (int8_t *)malloc(states), *nxt = (int8_t *)malloc(states);
    if (!cur || !nxt) { free(cur); free(nxt); return -2; }
    memset(cur, -1, states);
    cur[0] = 0;
    for (int32_t c = 0; c < nc; ++c) {
        memcpy(nxt, cur, states);
        for (size_t mask = 0; mask < states; ++mask) {
            if (cur[mask] < 0) continue;
            for (int64_t j = colptr[c]; j < colptr[c + 1]; ++j) {
                size_t bit = (size_t)1 << rowind[j];
                if (mask & bit) continue;
                if (nxt[mask | bit] < cur[mask] + 1) nxt[mask | bit] = (int8_t)(cur[mask] + 1);
            }
        }
        int8_t *t = cur; cur = nxt; nxt = t;
    }
    int64_t best = 0;
    for (size_t mask = 0; mask < states; ++mask)
        if (cur[mask] > best) best = cur[mask];
    free(cur); free(nxt);
    return best;
}

/*
 * Exhaustive maximum matching size by enumerating every subset of edges
 * (nnz <= 24) and keeping the largest one in which no two edges share a
 * vertex: the definition of a maximum matching, written out.
 */
int64_t orc_brute_force_subsets(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind)
{
    int64_t nnz = colptr[nc];
    if (nnz > 24 || nc > 64 || nr > 64) return -1;
    int32_t ec[24], er[24];
    int64_t e = 0;
    for (int32_t c = 0; c < nc; ++c)
        for (int64_t j = colptr[c]; j < colptr[c + 1]; ++j) { ec[e] = c; er[e] = rowind[j]; ++e; }
    int64_t best = 0;
    for (uint32_t s = 0; s < ((uint32_t)1 << nnz); ++s) {
        uint64_t usedc = 0, usedr = 0;
        int ok = 1, size = 0;
        for (int64_t i = 0; i < nnz && ok; ++i) {
            if (!(s >> i & 1u)) continue;
            uint64_t bc = (uint64_t)1 << ec[i], br = (uint64_t)1 << er[i];
            if ((usedc & bc) || (usedr & br)) ok = 0;
            usedc |= bc; usedr |= br; ++size;
        }
        if (ok && size > best) best = size;
    }
    return best;
}

/*
 * Alternating BFS from all unmatched columns without any early stop:
 * clevel[c] = number of matched edges on a shortest alternating path from
 * an unmatched column to c (0 for unmatched columns), -1 if unreachable;
 * rlevel[r] = level of the first column that reaches row r (the column
 * level at which r is discovered), -1 if r is not adjacent to any reached
 * column.  Returns the number of unmatched rows reached.
 */
int64_t orc_alt_bfs_levels(int32_t nc, int32_t nr, const int32_t *colptr, const int32_t *rowind,
                           const int32_t *cmatch, const int32_t *rmatch, int32_t *clevel, int32_t *rlevel)
{
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nc + 1));
    if (!queue) return -2;
    int64_t qh = 0, qt = 0, free_found = 0;
    for (int32_t c = 0; c < nc; ++c) {
        clevel[c] = -1;
        if (cmatch[c] == -1) { clevel[c] = 0; queue[qt++] = c; }
    }
    for (int32_t r = 0; r < nr; ++r) rlevel[r] = -1;
    while (qh < qt) {
        int32_t c = queue[qh++];
        for (int64_t j = colptr[c]; j < colptr[c + 1]; ++j) {
            int32_t r = rowind[j];
            if (rlevel[r] == -1) {
                rlevel[r] = clevel[c];
                if (rmatch[r] == -1) ++free_found;
            }
            int32_t m = rmatch[r];
            if (m >= 0 && clevel[m] == -1) {
                clevel[m] = clevel[c] + 1;
                queue[qt++] = m;
            }
        }
    }
    free(queue);
    return free_found;
}
