/*
 * gom_oracle.c -- plain CPU oracle for parallel Gene-pool Optimal Mixing (GOM) with partial
 * evaluations on weighted Max-Cut, parallelised by colouring the linkage-model interaction
 * graph (Bouter & Bosman, "GPU-Accelerated Parallel Gene-pool Optimal Mixing in a Gray-Box
 * Optimization Setting", arXiv 2203.08680).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker that the GPU library is compared
 * against.  It is slow on purpose: one byte per gene, explicit edge loops, explicit donor
 * scans.  Only the tests, the package's smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code, header, table or helper with the GPU library.
 *
 * What each function follows (sections, equations and algorithms of the paper):
 *   or_philox4x32_10 / or_philox4x64_10  counter-based RNG of Salmon, Moraes, Dror & Shaw,
 *       "Parallel random numbers: as easy as 1, 2, 3" (SC'11); the paper names no RNG.
 *       Pinned: the published known-answer vectors of Philox4x32-10 (Random123
 *       distribution), and the 4x64 instance against numpy.random.Philox.
 *   or_maxcut          Section 6.2, the Max-Cut objective: sum of weights of edges whose
 *       endpoints are on different sides.  Pinned: brute force, closed forms.
 *   or_fos_build       Section 4.1 (a FOS is a family of variable subsets that covers every
 *       variable); univariate {v} and neighbourhood {v} + N(v).  Pinned: tests.
 *   or_lmig_pairwise   Section 5.2, the LMIG: two linkage sets are dependent when they share a
 *       variable or when a VIG edge joins them.  Pinned: the 22 edges of Fig. 3.
 *   or_colour          Section 5.2, greedy Welsh-Powell colouring of the LMIG (classic
 *       colour-by-colour sweep over vertices sorted by degree).  Pinned: Fig. 3 example,
 *       validity, Welsh-Powell bound, torus closed forms.
 *   or_new/or_generation/or_run   Algorithm 3 (Par-GOMEA) with the step of Algorithm 2 (GOM)
 *       and the partial evaluation of Algorithm 4 / Section 2.2, under the readings listed
 *       at the top of or_generation.  Pinned: partial delta equals full re-evaluation after
 *       every step (debug flag), the whole-class reference with full evaluations,
 *       hand-worked two-solution examples, invariants (monotone
 *       fitness, converged fixed point, univariate donor independence, in-class order
 *       invariance).  There are no published trajectories to compare against.
 *   or_linkage_tree    Section 4.1: the Linkage Tree by UPGMA (pairwise merges of the two
 *       clusters with the largest average similarity), optionally bounded in set size (the
 *       Bounded Fixed Linkage Tree); Section 6.1 takes the graph's weights as the similarity.
 *       Dense similarity matrix, every pair rescanned at every merge.  Pinned: the tree of
 *       Fig. 2 from weights chosen to produce it, merge-by-merge maximality against an
 *       exact recomputation, non-increasing merge similarities, tree structure, bound.
 *   or_local_search    the colouring-parallel local search of the paper's conclusion (future
 *       work there): improving single-bit flips, a colour class of the graph at a time.
 *       Pinned: every solution ends at a local optimum (brute force over all single flips),
 *       fitness equals the full evaluation, a literal reading that computes a class's gains
 *       first and flips them together agrees pass by pass, a second search changes nothing.
 *   or_iterated_local_search  the iterated form of that search (also named as future work
 *       there): per round a perturbation of random single-bit flips, the search, and a keep-
 *       or-revert decision per solution.  Pinned: the flipped variable of a one-flip round
 *       against the definition of the draw, a literal reading built on the literal search,
 *       zero-flip rounds equal the plain search, invariants (full-evaluation fitness, no
 *       solution gets worse, local optima kept, counters unchanged).
 *   or_stop_after_class  a generation of Algorithm 3 cut after a given position of the class
 *       order (a debugging view of the offspring between two groups).  Pinned: the
 *       whole-class reference (every pair of a class decided on the class-start offspring,
 *       full evaluations) stopped after the same class.
 *   or_hash            a 64-bit summary of the state (not from the paper): the sum modulo 2^64
 *       of SplitMix64's output mixer (Steele, Lea & Flood, OOPSLA 2014) applied to
 *       256 * k + b_k for every byte b_k at position k of a canonical byte string.  Pinned: a
 *       numpy evaluation of the same definition on the bytes the accessors return.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------------------------
 * Philox (SC'11): a Feistel-like network over 4 words; each round multiplies words 0 and 2
 * by fixed odd constants, keeps the low halves and mixes the high halves with the two other
 * words and the round key; the key is advanced by Weyl constants between rounds.
 * One macro defines both word widths so the 4x64 check covers the 4x32 rounds.
 * ---------------------------------------------------------------------------------------- */
static inline void mulhilo_u32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}
static inline void mulhilo_u64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

#define OR_DEFINE_PHILOX4(NAME, T, MULHILO, M0, M1, W0, W1)                                \
    void NAME(const T key_in[2], const T ctr[4], T out[4]) {                               \
        T x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];                              \
        T k0 = key_in[0], k1 = key_in[1];                                                  \
        for (int r = 0; r < 10; ++r) {                                                     \
            if (r > 0) { k0 = (T)(k0 + (W0)); k1 = (T)(k1 + (W1)); }                       \
            T hi0, lo0, hi1, lo1;                                                          \
            MULHILO((T)(M0), x0, &hi0, &lo0);                                              \
            MULHILO((T)(M1), x2, &hi1, &lo1);                                              \
            T y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;                  \
            x0 = y0; x1 = y1; x2 = y2; x3 = y3;                                            \
        }                                                                                  \
        out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;                                \
    }

OR_DEFINE_PHILOX4(or_philox4x32_10, uint32_t, mulhilo_u32, 0xD2511F53u, 0xCD9E8D57u,
                  0x9E3779B9u, 0xBB67AE85u)
OR_DEFINE_PHILOX4(or_philox4x64_10, uint64_t, mulhilo_u64, 0xD2E7470EE14C6C93ull,
                  0xCA5A826395121157ull, 0x9E3779B97F4A7C15ull, 0xBB67AE8584CAA73Bull)

/* Philox4x32-10 keyed by a 64-bit seed: key = (low word, high word). */
static void draw4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                  uint32_t out[4]) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {c0, c1, c2, c3};
    or_philox4x32_10(key, ctr, out);
}

/* ------------------------------------------------------------------------------------------
 * Max-Cut objective (Section 6.2).  With x in {-1,1} the objective is half the sum over
 * vertex pairs of w_ij (1 - x_i x_j); mapped to bits it is the total weight of the edges
 * whose two endpoints carry different bits, each edge counted once.
 * ---------------------------------------------------------------------------------------- */
int64_t or_maxcut(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                  const int32_t *ew, const uint8_t *x) {
    (void)n;
    int64_t f = 0;
    for (int64_t e = 0; e < m; ++e)
        if (x[eu[e]] != x[ev[e]]) f += ew[e];
    return f;
}

/* ------------------------------------------------------------------------------------------
 * Plain adjacency: for each vertex the list of incident edge ids, in edge order.
 * ---------------------------------------------------------------------------------------- */
typedef struct {
    int32_t n;
    int64_t m;
    int32_t *eu, *ev, *ew;
    int64_t *inc_ptr; /* n+1 */
    int64_t *inc;     /* 2m edge ids */
} or_graph;

static int graph_init(or_graph *g, int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                      const int32_t *ew) {
    g->n = n;
    g->m = m;
    g->eu = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    g->ev = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    g->ew = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    g->inc_ptr = calloc((size_t)n + 1, sizeof(int64_t));
    g->inc = malloc(sizeof(int64_t) * (size_t)(2 * m + 1));
    if (!g->eu || !g->ev || !g->ew || !g->inc_ptr || !g->inc) return -1;
    memcpy(g->eu, eu, sizeof(int32_t) * (size_t)m);
    memcpy(g->ev, ev, sizeof(int32_t) * (size_t)m);
    if (ew) memcpy(g->ew, ew, sizeof(int32_t) * (size_t)m);
    else for (int64_t e = 0; e < m; ++e) g->ew[e] = 1;
    for (int64_t e = 0; e < m; ++e) {
        g->inc_ptr[eu[e] + 1]++;
        g->inc_ptr[ev[e] + 1]++;
    }
    for (int32_t v = 0; v < n; ++v) g->inc_ptr[v + 1] += g->inc_ptr[v];
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!fill) return -1;
    memcpy(fill, g->inc_ptr, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t e = 0; e < m; ++e) {
        g->inc[fill[eu[e]]++] = e;
        g->inc[fill[ev[e]]++] = e;
    }
    free(fill);
    return 0;
}

static void graph_free(or_graph *g) {
    free(g->eu); free(g->ev); free(g->ew); free(g->inc_ptr); free(g->inc);
}

static inline int32_t other_end(const or_graph *g, int64_t e, int32_t u) {
    return g->eu[e] == u ? g->ev[e] : g->eu[e];
}

/* ------------------------------------------------------------------------------------------
 * FOS (Section 4.1).  kind 0: univariate {v}; kind 1: neighbourhood {v} + N(v), ascending.
 * Writes set_ptr[n+1] and, when set_vars is non-NULL, the member lists; returns the total
 * member count.
 * ---------------------------------------------------------------------------------------- */
static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

int64_t or_fos_build(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev, int kind,
                     int32_t *set_ptr, int32_t *set_vars) {
    or_graph g;
    if (graph_init(&g, n, m, eu, ev, NULL)) return -1;
    int64_t total = 0;
    set_ptr[0] = 0;
    for (int32_t v = 0; v < n; ++v) {
        int64_t sz = 1 + (kind == 1 ? (g.inc_ptr[v + 1] - g.inc_ptr[v]) : 0);
        if (set_vars) {
            int32_t *s = set_vars + total;
            s[0] = v;
            if (kind == 1)
                for (int64_t t = g.inc_ptr[v]; t < g.inc_ptr[v + 1]; ++t)
                    s[1 + (t - g.inc_ptr[v])] = other_end(&g, g.inc[t], v);
            qsort(s, (size_t)sz, sizeof(int32_t), cmp_i32);
        }
        total += sz;
        set_ptr[v + 1] = (int32_t)total;
    }
    graph_free(&g);
    return total;
}

/* ------------------------------------------------------------------------------------------
 * LMIG, literal pairwise form (Section 5.2): sets j < k are joined when they share a
 * variable or some edge (u, v) has u in F_j and v in F_k.  For small instances only: it
 * looks at every pair of sets.  Writes up to max_edges pairs (j, k), returns the count.
 * ---------------------------------------------------------------------------------------- */
int64_t or_lmig_pairwise(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                         int32_t nsets, const int32_t *set_ptr, const int32_t *set_vars,
                         int64_t max_edges, int32_t *out_pairs) {
    uint8_t *in_j = calloc((size_t)n, 1), *in_k = calloc((size_t)n, 1);
    if (!in_j || !in_k) return -1;
    int64_t cnt = 0;
    for (int32_t j = 0; j < nsets; ++j) {
        for (int32_t t = set_ptr[j]; t < set_ptr[j + 1]; ++t) in_j[set_vars[t]] = 1;
        for (int32_t k = j + 1; k < nsets; ++k) {
            for (int32_t t = set_ptr[k]; t < set_ptr[k + 1]; ++t) in_k[set_vars[t]] = 1;
            int dep = 0;
            for (int32_t v = 0; v < n && !dep; ++v) dep = in_j[v] && in_k[v];
            for (int64_t e = 0; e < m && !dep; ++e)
                dep = (in_j[eu[e]] && in_k[ev[e]]) || (in_j[ev[e]] && in_k[eu[e]]);
            if (dep) {
                if (cnt < max_edges) {
                    out_pairs[2 * cnt] = j;
                    out_pairs[2 * cnt + 1] = k;
                }
                ++cnt;
            }
            for (int32_t t = set_ptr[k]; t < set_ptr[k + 1]; ++t) in_k[set_vars[t]] = 0;
        }
        for (int32_t t = set_ptr[j]; t < set_ptr[j + 1]; ++t) in_j[set_vars[t]] = 0;
    }
    free(in_j);
    free(in_k);
    return cnt;
}

/* ------------------------------------------------------------------------------------------
 * Welsh-Powell colouring of the LMIG (Section 5.2).  The LMIG neighbours of set j are the
 * sets that contain a variable of the closed neighbourhood N[F_j] = F_j + N(F_j); they are
 * enumerated on demand from an inverse index (variable -> sets containing it) instead of
 * storing the LMIG.  Vertices are sorted by LMIG degree, largest first (ties: smaller index
 * first).  Then colour after colour: walk the sorted list and give the current colour to
 * every uncoloured set that has no neighbour already holding that colour.
 * ---------------------------------------------------------------------------------------- */
typedef struct {
    const or_graph *g;
    int32_t nsets;
    const int32_t *set_ptr, *set_vars;
    int64_t *vs_ptr; /* variable -> sets containing it */
    int32_t *vs;
} or_lmig;

static int lmig_init(or_lmig *L, const or_graph *g, int32_t nsets, const int32_t *set_ptr,
                     const int32_t *set_vars) {
    L->g = g;
    L->nsets = nsets;
    L->set_ptr = set_ptr;
    L->set_vars = set_vars;
    L->vs_ptr = calloc((size_t)g->n + 1, sizeof(int64_t));
    L->vs = malloc(sizeof(int32_t) * (size_t)(set_ptr[nsets] + 1));
    if (!L->vs_ptr || !L->vs) return -1;
    for (int32_t t = 0; t < set_ptr[nsets]; ++t) L->vs_ptr[set_vars[t] + 1]++;
    for (int32_t v = 0; v < g->n; ++v) L->vs_ptr[v + 1] += L->vs_ptr[v];
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(g->n + 1));
    if (!fill) return -1;
    memcpy(fill, L->vs_ptr, sizeof(int64_t) * (size_t)(g->n + 1));
    for (int32_t j = 0; j < nsets; ++j)
        for (int32_t t = set_ptr[j]; t < set_ptr[j + 1]; ++t) L->vs[fill[set_vars[t]]++] = j;
    free(fill);
    return 0;
}

static void lmig_free(or_lmig *L) {
    free(L->vs_ptr);
    free(L->vs);
}

/* Calls visit(k, ctx) for every set k != j that touches N[F_j] (k may repeat). */
static void lmig_visit(const or_lmig *L, int32_t j, void (*visit)(int32_t, void *), void *ctx) {
    const or_graph *g = L->g;
    for (int32_t t = L->set_ptr[j]; t < L->set_ptr[j + 1]; ++t) {
        int32_t u = L->set_vars[t];
        for (int64_t a = L->vs_ptr[u]; a < L->vs_ptr[u + 1]; ++a)
            if (L->vs[a] != j) visit(L->vs[a], ctx);
        for (int64_t q = g->inc_ptr[u]; q < g->inc_ptr[u + 1]; ++q) {
            int32_t v = other_end(g, g->inc[q], u);
            for (int64_t a = L->vs_ptr[v]; a < L->vs_ptr[v + 1]; ++a)
                if (L->vs[a] != j) visit(L->vs[a], ctx);
        }
    }
}

typedef struct { int32_t *stamp; int32_t tag; int64_t count; } count_ctx;
static void count_visit(int32_t k, void *p) {
    count_ctx *c = p;
    if (c->stamp[k] != c->tag) { c->stamp[k] = c->tag; c->count++; }
}
typedef struct { int32_t *blocked; int32_t colour; } block_ctx;
static void block_visit(int32_t k, void *p) {
    block_ctx *b = p;
    b->blocked[k] = b->colour;
}

static const int64_t *g_sort_deg; /* qsort comparator context (single-threaded oracle) */
static int cmp_wp(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    if (g_sort_deg[x] != g_sort_deg[y]) return g_sort_deg[x] > g_sort_deg[y] ? -1 : 1;
    return (x > y) - (x < y);
}

/* Returns the number of colours k; colour_out[nsets]; degree_out (optional) the LMIG degree. */
static int32_t colour_sets(const or_graph *g, int32_t nsets, const int32_t *set_ptr,
                           const int32_t *set_vars, int32_t *colour_out, int64_t *degree_out) {
    or_lmig L;
    if (lmig_init(&L, g, nsets, set_ptr, set_vars)) return -1;
    int64_t *deg = malloc(sizeof(int64_t) * (size_t)nsets);
    int32_t *stamp = malloc(sizeof(int32_t) * (size_t)nsets);
    int32_t *order = malloc(sizeof(int32_t) * (size_t)nsets);
    if (!deg || !stamp || !order) return -1;
    for (int32_t j = 0; j < nsets; ++j) stamp[j] = -1;
    for (int32_t j = 0; j < nsets; ++j) {
        count_ctx c = {stamp, j, 0};
        lmig_visit(&L, j, count_visit, &c);
        deg[j] = c.count;
        order[j] = j;
    }
    g_sort_deg = deg;
    qsort(order, (size_t)nsets, sizeof(int32_t), cmp_wp);
    for (int32_t j = 0; j < nsets; ++j) { colour_out[j] = -1; stamp[j] = -1; }
    int32_t remaining = nsets, k = 0;
    while (remaining > 0) {
        int32_t colour = k++;
        block_ctx b = {stamp, colour};
        for (int32_t t = 0; t < nsets; ++t) {
            int32_t j = order[t];
            if (colour_out[j] != -1 || stamp[j] == colour) continue;
            colour_out[j] = colour;
            --remaining;
            lmig_visit(&L, j, block_visit, &b);
        }
    }
    if (degree_out) memcpy(degree_out, deg, sizeof(int64_t) * (size_t)nsets);
    free(deg);
    free(stamp);
    free(order);
    lmig_free(&L);
    return k;
}

int32_t or_colour(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev, int32_t nsets,
                  const int32_t *set_ptr, const int32_t *set_vars, int32_t *colour_out,
                  int64_t *degree_out) {
    or_graph g;
    if (graph_init(&g, n, m, eu, ev, NULL)) return -1;
    int32_t k = colour_sets(&g, nsets, set_ptr, set_vars, colour_out, degree_out);
    graph_free(&g);
    return k;
}

/* ------------------------------------------------------------------------------------------
 * Linkage tree by UPGMA (Section 4.1).  Readings where the paper is silent:
 *   - similarity of variables a, b = |w(a, b)|, 0 without an edge (Section 6.1 uses the
 *     weights as the similarity; the sign of a weight does not make two variables less
 *     dependent);
 *   - ties between pairs with equal average similarity: smaller combined size first, then the
 *     pair with the lower smaller cluster id, then the lower larger id; the variables are
 *     clusters 0..n-1 and each merge creates the next id;
 *   - bounded: only pairs whose union has at most `bound` variables are candidates; the tree
 *     stops when no candidate is left (pairs of average 0 are candidates too);
 *   - the union of all variables is not a set of the tree.
 * Output: sets 0..n-1 are the variables, then one set per merge in merge order, members
 * ascending.  Returns the number of sets, or -1 on bad input or allocation failure.
 * set_ptr needs 2n entries, set_vars n*n (enough for any tree).
 * ---------------------------------------------------------------------------------------- */
int32_t or_linkage_tree(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                        const int32_t *ew, int32_t bound, int32_t *set_ptr,
                        int32_t *set_vars) {
    if (n < 1 || bound < 0 || bound == 1) return -1;
    const int64_t cap = bound ? bound : n;
    int64_t *S = calloc((size_t)n * (size_t)n, sizeof(int64_t));
    int32_t *cid = malloc(sizeof(int32_t) * (size_t)n);  /* cluster id of each variable */
    int32_t *size = malloc(sizeof(int32_t) * (size_t)(2 * n));
    char *alive = calloc((size_t)(2 * n), 1);
    if (!S || !cid || !size || !alive) {
        free(S); free(cid); free(size); free(alive);
        return -1;
    }
    for (int64_t e = 0; e < m; ++e) {
        int64_t w = ew[e] < 0 ? -(int64_t)ew[e] : (int64_t)ew[e];
        S[(size_t)eu[e] * n + ev[e]] += w;
        S[(size_t)ev[e] * n + eu[e]] += w;
    }
    set_ptr[0] = 0;
    for (int32_t v = 0; v < n; ++v) {
        cid[v] = v;
        size[v] = 1;
        alive[v] = 1;
        set_vars[v] = v;
        set_ptr[v + 1] = v + 1;
    }
    int32_t next = n;
    for (;;) {
        /* best allowed pair (i < j): largest W / (|i| |j|), then smallest size sum, then the
           smallest (i, j) */
        int32_t bi = -1, bj = -1;
        int64_t bW = 0, bsz = 1, bsum = 0;
        for (int32_t i = 0; i < next; ++i) {
            if (!alive[i]) continue;
            for (int32_t j = i + 1; j < next; ++j) {
                if (!alive[j]) continue;
                int64_t sum = (int64_t)size[i] + size[j];
                if (sum > cap || sum >= n) continue;
                int64_t W = 0; /* summed similarity over member pairs */
                for (int32_t a = 0; a < n; ++a) {
                    if (cid[a] != i) continue;
                    for (int32_t b = 0; b < n; ++b)
                        if (cid[b] == j) W += S[(size_t)a * n + b];
                }
                int64_t sz = (int64_t)size[i] * size[j];
                int better;
                if (bi < 0) {
                    better = 1;
                } else {
                    __int128 x = (__int128)W * bsz, y = (__int128)bW * sz;
                    better = x > y || (x == y && sum < bsum);
                }
                if (better) { bi = i; bj = j; bW = W; bsz = sz; bsum = sum; }
            }
        }
        if (bi < 0) break;
        int32_t c = next++;
        size[c] = size[bi] + size[bj];
        alive[c] = 1;
        alive[bi] = alive[bj] = 0;
        int32_t at = set_ptr[c];
        for (int32_t a = 0; a < n; ++a)
            if (cid[a] == bi || cid[a] == bj) {
                cid[a] = c;
                set_vars[at++] = a;
            }
        set_ptr[c + 1] = at;
    }
    free(S); free(cid); free(size); free(alive);
    return next;
}

/* ------------------------------------------------------------------------------------------
 * Par-GOMEA state (Algorithm 3).
 * ---------------------------------------------------------------------------------------- */
enum { OR_NEUTRAL_PAPER = 0, OR_NEUTRAL_ALWAYS = 1 };
enum { OR_ORDER_RANDOM = 0, OR_ORDER_FIXED = 1 };
enum { OR_FLAG_DEBUG = 1, OR_FLAG_REVERSE = 2, OR_FLAG_FI = 4 };

typedef struct or_state {
    or_graph g;
    int32_t nsets;
    int32_t *set_ptr, *set_vars;
    int32_t k;
    int32_t *class_ptr, *class_elems;
    int32_t N;
    uint64_t seed, donor_seed;
    int rule, order, flags;
    uint8_t *P, *O, *E, *eq, *acc_any;
    int64_t *f, fE;
    int32_t gen;
    int32_t open_next;        /* -1, or the next class position of an unfinished generation */
    int64_t attempted, evaluated, accepted;
    int64_t debug_mismatches;
    int32_t *perm;
    /* working memory: one block per worker thread (one unless or_set_workers asks for more) */
    int32_t nwork;
    struct or_work *work;
} or_state;

/* Working memory of one worker: the donor list of a step, stamps that mark the vertices and
   edges a step touches, and the step counters it adds up (folded into the state after each
   class). */
typedef struct or_work {
    int32_t *donors, *vstamp;
    int64_t *estamp;
    int32_t stamp;
    int64_t attempted, evaluated, accepted, debug_mismatches;
} or_work;

static void work_free(or_work *w) {
    free(w->donors); free(w->vstamp); free(w->estamp);
    memset(w, 0, sizeof(*w));
}

static int work_init(or_work *w, int32_t n, int64_t m, int32_t pop) {
    memset(w, 0, sizeof(*w));
    w->donors = malloc(sizeof(int32_t) * (size_t)pop);
    w->vstamp = malloc(sizeof(int32_t) * (size_t)n);
    w->estamp = malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
    if (!w->donors || !w->vstamp || !w->estamp) { work_free(w); return -1; }
    for (int32_t v = 0; v < n; ++v) w->vstamp[v] = -1;
    for (int64_t e = 0; e < m; ++e) w->estamp[e] = -1;
    return 0;
}

/* Add the workers' step counters to the state's and clear them. */
static void fold_counters(or_state *s) {
    for (int32_t t = 0; t < s->nwork; ++t) {
        or_work *w = &s->work[t];
        s->attempted += w->attempted;
        s->evaluated += w->evaluated;
        s->accepted += w->accepted;
        s->debug_mismatches += w->debug_mismatches;
        w->attempted = w->evaluated = w->accepted = w->debug_mismatches = 0;
    }
}

static int worker_id(void) {
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

void or_free(or_state *s) {
    if (!s) return;
    graph_free(&s->g);
    free(s->set_ptr); free(s->set_vars); free(s->class_ptr); free(s->class_elems);
    free(s->P); free(s->O); free(s->E); free(s->eq); free(s->acc_any); free(s->f);
    free(s->perm);
    for (int32_t t = 0; t < s->nwork; ++t) work_free(&s->work[t]);
    free(s->work);
    free(s);
}

/* Number of worker threads over which the solutions of a class are spread (1 = serial).
   The solutions of a class only write their own offspring and fitness and read the
   generation-start population, so the result is the same for any number.  Returns the
   number set (1 without OpenMP), or -1 when memory ran out (the state is then unchanged). */
int32_t or_set_workers(or_state *s, int32_t nwork) {
#ifndef _OPENMP
    nwork = 1;
#endif
    if (nwork < 1) nwork = 1;
    if (nwork == s->nwork) return nwork;
    or_work *w = calloc((size_t)nwork, sizeof(or_work));
    if (!w) return -1;
    for (int32_t t = 0; t < nwork; ++t)
        if (work_init(&w[t], s->g.n, s->g.m, s->N)) {
            for (int32_t u = 0; u < t; ++u) work_free(&w[u]);
            free(w);
            return -1;
        }
    fold_counters(s);
    for (int32_t t = 0; t < s->nwork; ++t) work_free(&s->work[t]);
    free(s->work);
    s->work = w;
    s->nwork = nwork;
    return nwork;
}

static void full_fitness_all(or_state *s) {
    for (int32_t i = 0; i < s->N; ++i)
        s->f[i] = or_maxcut(s->g.n, s->g.m, s->g.eu, s->g.ev, s->g.ew,
                            s->P + (size_t)i * s->g.n);
}

/* Elitist = the best solution; ties go to the lowest index. */
static int32_t best_index(const or_state *s) {
    int32_t b = 0;
    for (int32_t i = 1; i < s->N; ++i)
        if (s->f[i] > s->f[b]) b = i;
    return b;
}

or_state *or_new(int32_t n, int64_t m, const int32_t *eu, const int32_t *ev, const int32_t *ew,
                 int32_t nsets, const int32_t *set_ptr, const int32_t *set_vars, int32_t pop,
                 uint64_t seed, uint64_t donor_salt, int rule, int order, int flags) {
    if (n < 1 || pop < 2 || nsets < 1) return NULL;
    or_state *s = calloc(1, sizeof(or_state));
    if (!s) return NULL;
    if (graph_init(&s->g, n, m, eu, ev, ew)) { or_free(s); return NULL; }
    s->nsets = nsets;
    s->set_ptr = malloc(sizeof(int32_t) * (size_t)(nsets + 1));
    s->set_vars = malloc(sizeof(int32_t) * (size_t)(set_ptr[nsets] + 1));
    memcpy(s->set_ptr, set_ptr, sizeof(int32_t) * (size_t)(nsets + 1));
    memcpy(s->set_vars, set_vars, sizeof(int32_t) * (size_t)set_ptr[nsets]);
    s->N = pop;
    s->seed = seed;
    s->donor_seed = seed ^ donor_salt;
    s->rule = rule;
    s->order = order;
    s->flags = flags;
    size_t genes = (size_t)pop * (size_t)n;
    s->P = malloc(genes);
    s->O = malloc(genes);
    s->E = malloc((size_t)n);
    s->eq = malloc((size_t)pop);
    s->acc_any = calloc((size_t)pop, 1);
    s->f = malloc(sizeof(int64_t) * (size_t)pop);
    s->work = calloc(1, sizeof(or_work));
    int32_t *colour = malloc(sizeof(int32_t) * (size_t)nsets);
    if (!s->P || !s->O || !s->E || !s->eq || !s->acc_any || !s->f || !s->work || !colour) {
        free(colour); or_free(s); return NULL;
    }
    if (work_init(&s->work[0], n, m, pop)) { free(colour); or_free(s); return NULL; }
    s->nwork = 1;

    /* Groups G_1..G_k: colour classes, members ascending by set index. */
    s->k = colour_sets(&s->g, nsets, s->set_ptr, s->set_vars, colour, NULL);
    if (s->k < 1) { free(colour); or_free(s); return NULL; }
    s->class_ptr = calloc((size_t)s->k + 1, sizeof(int32_t));
    s->class_elems = malloc(sizeof(int32_t) * (size_t)nsets);
    s->perm = malloc(sizeof(int32_t) * (size_t)s->k);
    for (int32_t j = 0; j < nsets; ++j) s->class_ptr[colour[j] + 1]++;
    for (int32_t c = 0; c < s->k; ++c) s->class_ptr[c + 1] += s->class_ptr[c];
    int32_t *fill = malloc(sizeof(int32_t) * (size_t)s->k);
    memcpy(fill, s->class_ptr, sizeof(int32_t) * (size_t)s->k);
    for (int32_t j = 0; j < nsets; ++j) s->class_elems[fill[colour[j]]++] = j;
    free(fill);
    free(colour);

    /* InitializePopulation: gene v of solution i is bit (v mod 32) of output word
       ((v / 32) mod 4) of Philox(seed; counter = (0xFFFFFFFF, i, v / 128, 0)). */
    for (int32_t i = 0; i < pop; ++i)
        for (int32_t v = 0; v < n; ++v) {
            uint32_t out[4];
            draw4(seed, 0xFFFFFFFFu, (uint32_t)i, (uint32_t)(v >> 7), 0u, out);
            s->P[(size_t)i * n + v] = (uint8_t)((out[(v >> 5) & 3] >> (v & 31)) & 1u);
        }
    memcpy(s->O, s->P, genes);
    full_fitness_all(s);
    int32_t b = best_index(s);
    memcpy(s->E, s->P + (size_t)b * n, (size_t)n);
    s->fE = s->f[b];
    s->open_next = -1;
    return s;
}

/* One GOM step (Algorithm 2) for solution i and set j at position p of class c. */
/* Insert donor genes D[F_j] into O_i when the partial evaluation (Section 2.2, Algorithm 4)
   allows it: every subfunction (edge) that depends on a variable of F_j is evaluated before
   and after the insertion.  Accepts improvements, and equal fitness unless P_i equals the
   elitist (or always, under the ALWAYS rule).  *delta receives the change; returns whether
   the step was accepted. */
static int try_insert(or_state *s, or_work *w, int32_t i, int32_t j, const uint8_t *D,
                      int64_t *delta_out) {
    const int32_t n = s->g.n;
    uint8_t *Oi = s->O + (size_t)i * n;
    const int32_t *F = s->set_vars + s->set_ptr[j];
    const int32_t sz = s->set_ptr[j + 1] - s->set_ptr[j];
    int32_t tag = ++w->stamp;
    for (int32_t q = 0; q < sz; ++q) w->vstamp[F[q]] = tag;
    int64_t delta = 0;
    for (int32_t q = 0; q < sz; ++q) {
        int32_t u = F[q];
        for (int64_t t = s->g.inc_ptr[u]; t < s->g.inc_ptr[u + 1]; ++t) {
            int64_t e = s->g.inc[t];
            if (w->estamp[e] == tag) continue;
            w->estamp[e] = tag;
            int32_t a = s->g.eu[e], b = s->g.ev[e];
            uint8_t xa = Oi[a], xb = Oi[b];
            uint8_t ya = w->vstamp[a] == tag ? D[a] : xa;
            uint8_t yb = w->vstamp[b] == tag ? D[b] : xb;
            int64_t before = xa != xb ? s->g.ew[e] : 0;
            int64_t after = ya != yb ? s->g.ew[e] : 0;
            delta += after - before;
        }
    }
    int accept = delta > 0 || (delta == 0 && (s->rule == OR_NEUTRAL_ALWAYS || !s->eq[i]));
    if (accept) {
        for (int32_t q = 0; q < sz; ++q) Oi[F[q]] = D[F[q]];
        s->f[i] += delta;
        w->accepted++;
    }
    if (s->flags & OR_FLAG_DEBUG) {
        int64_t full = or_maxcut(n, s->g.m, s->g.eu, s->g.ev, s->g.ew, Oi);
        if (full != s->f[i]) w->debug_mismatches++;
    }
    *delta_out = delta;
    return accept;
}

/* One GOM step (Algorithm 2) for solution i and set j at position p of class c. */
static void gom_step(or_state *s, or_work *w, int32_t c, int32_t p, int32_t j, int32_t i) {
    const int32_t n = s->g.n;
    uint8_t *Oi = s->O + (size_t)i * n;
    const int32_t *F = s->set_vars + s->set_ptr[j];
    const int32_t sz = s->set_ptr[j + 1] - s->set_ptr[j];
    w->attempted++;

    /* SelectDonorFromPopulation: candidates are the other members of the population P (as
       it was at the start of the generation) whose genes on F_j differ from those of O_i. */
    int32_t nd = 0;
    for (int32_t d = 0; d < s->N; ++d) {
        if (d == i) continue;
        const uint8_t *Pd = s->P + (size_t)d * n;
        for (int32_t q = 0; q < sz; ++q)
            if (Pd[F[q]] != Oi[F[q]]) { w->donors[nd++] = d; break; }
    }
    if (nd == 0) return; /* no donor differs: this step is skipped */
    w->evaluated++;

    /* Uniform choice among the nd candidates from a 16-bit Philox field. */
    uint32_t out[4];
    draw4(s->donor_seed, (uint32_t)s->gen, (uint32_t)c, (uint32_t)i, (uint32_t)(p >> 3), out);
    uint32_t h = (out[(p & 7) >> 1] >> (16 * (p & 1))) & 0xFFFFu;
    int32_t d = w->donors[((uint64_t)h * (uint64_t)nd) >> 16];
    int64_t delta;
    if (try_insert(s, w, i, j, s->P + (size_t)d * n, &delta)) s->acc_any[i] = 1;
}

/* Forced improvement, in a form that runs class by class (Section 4 describes the serial
   procedure; Section 5.4 leaves a parallel form open).  For every solution that had no
   accepted GOM step in this generation: GOM steps with the elitist (of the generation start)
   as the donor, over the classes in the generation's order, all sets of a class together;
   the solution stops after the first class in which a step raised its fitness.  A solution
   that never improved becomes a copy of the elitist.  With one set per class this is the
   serial procedure visiting the sets in class order. */
static void forced_improvement(or_state *s) {
    const int32_t n = s->g.n;
    for (int32_t i = 0; i < s->N; ++i) {
        if (s->acc_any[i]) continue;
        int improved = 0;
        for (int32_t t = 0; t < s->k && !improved; ++t) {
            int32_t c = s->perm[t];
            for (int32_t q = s->class_ptr[c]; q < s->class_ptr[c + 1]; ++q) {
                int32_t j = s->class_elems[q];
                const int32_t *F = s->set_vars + s->set_ptr[j];
                const int32_t sz = s->set_ptr[j + 1] - s->set_ptr[j];
                const uint8_t *Oi = s->O + (size_t)i * n;
                int differs = 0;
                for (int32_t r = 0; r < sz; ++r) differs |= s->E[F[r]] != Oi[F[r]];
                if (!differs) continue;
                s->evaluated++;
                int64_t delta;
                if (try_insert(s, &s->work[0], i, j, s->E, &delta) && delta > 0) improved = 1;
            }
        }
        if (!improved) {
            memcpy(s->O + (size_t)i * n, s->E, (size_t)n);
            s->f[i] = s->fE;
        }
    }
    fold_counters(s);
}

/*
 * One generation of Par-GOMEA (Algorithm 3).  Readings of the paper taken here:
 *  - donors are drawn from P, the population at the start of the generation; the steps are
 *    applied to the offspring O, which starts as a copy of P;
 *  - "equal to the elitist" compares P_i (start of generation) with the elitist;
 *  - the groups (colour classes) are visited in a random order drawn per generation by a
 *    Fisher-Yates shuffle (FIXED order: ascending class index);
 *  - within a group, every (solution, set) pair is one GOM step; the groups' independence
 *    makes their order irrelevant (the REVERSE flag visits them backwards to check that);
 *  - no forced improvement (Section 5.4) unless the FI flag asks for the class-by-class form
 *    of forced_improvement, run after the groups;
 *  - after the groups, P <- O and the elitist is replaced when the best solution (lowest index
 *    on ties) is strictly better.
 */
/* Generation start: equality with the elitist, the class order, O <- P. */
static void begin_generation(or_state *s) {
    const int32_t n = s->g.n, N = s->N;
    for (int32_t i = 0; i < N; ++i)
        s->eq[i] = memcmp(s->P + (size_t)i * n, s->E, (size_t)n) == 0;

    for (int32_t c = 0; c < s->k; ++c) s->perm[c] = c;
    if (s->order == OR_ORDER_RANDOM)
        for (int32_t t = s->k - 1; t >= 1; --t) {
            uint32_t out[4];
            draw4(s->seed, (uint32_t)s->gen, 0xFFFFFFFFu, (uint32_t)t, 0u, out);
            int32_t r = (int32_t)(((uint64_t)out[0] * (uint64_t)(t + 1)) >> 32);
            int32_t tmp = s->perm[t];
            s->perm[t] = s->perm[r];
            s->perm[r] = tmp;
        }

    memcpy(s->O, s->P, (size_t)N * n);
    memset(s->acc_any, 0, (size_t)N);
    s->open_next = 0;
}

/* Every (solution, set) pair of the class at position t of the order.  A solution's steps
   write only its own offspring, fitness and flag and read the generation-start population, so
   the solutions may be spread over worker threads. */
static void run_class(or_state *s, int32_t t) {
    const int32_t N = s->N;
    const int rev = (s->flags & OR_FLAG_REVERSE) != 0;
    int32_t c = s->perm[t];
    int32_t size = s->class_ptr[c + 1] - s->class_ptr[c];
#pragma omp parallel for num_threads(s->nwork) schedule(static) if (s->nwork > 1)
    for (int32_t ii = 0; ii < N; ++ii) {
        or_work *w = &s->work[worker_id()];
        int32_t i = rev ? N - 1 - ii : ii;
        for (int32_t pp = 0; pp < size; ++pp) {
            int32_t p = rev ? size - 1 - pp : pp;
            gom_step(s, w, c, p, s->class_elems[s->class_ptr[c] + p], i);
        }
    }
    fold_counters(s);
}

/* Generation end: P <- O, then the elitist on strict improvement. */
static void end_generation(or_state *s) {
    const int32_t n = s->g.n;
    memcpy(s->P, s->O, (size_t)s->N * n);
    int32_t b = best_index(s);
    if (s->f[b] > s->fE) {
        memcpy(s->E, s->P + (size_t)b * n, (size_t)n);
        s->fE = s->f[b];
    }
    s->gen++;
    s->open_next = -1;
}

/* One generation of Algorithm 3 (or the rest of one left open by or_stop_after_class). */
void or_generation(or_state *s) {
    if (s->open_next < 0) begin_generation(s);
    for (int32_t t = s->open_next; t < s->k; ++t) run_class(s, t);
    if (s->flags & OR_FLAG_FI) forced_improvement(s);
    end_generation(s);
}

/*
 * Colouring-parallel local search: the hybrid that the paper's conclusion names as future work
 * (graph colouring yields sets of independent variables, so single-bit flips of one colour
 * class can be made together).  Defined for a univariate FOS, whose colour classes are the
 * colour classes of the graph itself.  Reading: for every solution of the population, a pass
 * visits the classes in ascending class index and flips each variable of the class whose
 * flip strictly raises the solution's fitness (variables of one class share no edge, so the
 * order inside a class does not matter); passes repeat until one flips nothing anywhere or
 * max_passes have run.  Then P <- O and the elitist is replaced when the best solution
 * (lowest index on ties) is strictly better, as at a generation end; the generation and the
 * GOM counters do not change.  Returns the passes run, or -1 when the FOS is not univariate
 * or a generation is open.
 */
/* Change of solution i's cut when variable u of O_i flips: an uncut incident edge becomes
   cut (+w), a cut one uncut (-w). */
static int64_t flip_gain(const or_state *s, const uint8_t *Oi, int32_t u) {
    int64_t gain = 0;
    for (int64_t t = s->g.inc_ptr[u]; t < s->g.inc_ptr[u + 1]; ++t) {
        const int64_t e = s->g.inc[t];
        const int32_t v = s->g.eu[e] == u ? s->g.ev[e] : s->g.eu[e];
        gain += Oi[u] == Oi[v] ? (int64_t)s->g.ew[e] : -(int64_t)s->g.ew[e];
    }
    return gain;
}

/* Passes of the local search over the offspring O with fitness `fit`: per pass the classes
   in ascending index, per class every solution, per variable of the class the flip when it
   strictly raises the cut.  Returns the number of passes. */
static int32_t ls_passes(or_state *s, int64_t *fit, int32_t max_passes) {
    const int32_t n = s->g.n;
    int32_t passes = 0;
    while (passes < max_passes) {
        int any = 0;
        for (int32_t c = 0; c < s->k; ++c)
            for (int32_t i = 0; i < s->N; ++i) {
                uint8_t *Oi = s->O + (size_t)i * n;
                for (int32_t q = s->class_ptr[c]; q < s->class_ptr[c + 1]; ++q) {
                    const int32_t u = s->set_vars[s->set_ptr[s->class_elems[q]]];
                    const int64_t gain = flip_gain(s, Oi, u);
                    if (gain > 0) {
                        Oi[u] ^= 1u;
                        fit[i] += gain;
                        any = 1;
                    }
                }
            }
        ++passes;
        if (!any) break;
    }
    return passes;
}

static void update_elitist(or_state *s) {
    const int32_t b = best_index(s);
    if (s->f[b] > s->fE) {
        memcpy(s->E, s->P + (size_t)b * s->g.n, (size_t)s->g.n);
        s->fE = s->f[b];
    }
}

static int univariate_fos(const or_state *s) {
    for (int32_t j = 0; j < s->nsets; ++j)
        if (s->set_ptr[j + 1] - s->set_ptr[j] != 1) return 0;
    return 1;
}

int32_t or_local_search(or_state *s, int32_t max_passes) {
    if (s->open_next >= 0 || max_passes < 0 || !univariate_fos(s)) return -1;
    memcpy(s->O, s->P, (size_t)s->N * s->g.n);  /* between generations the offspring is P */
    const int32_t passes = ls_passes(s, s->f, max_passes);
    memcpy(s->P, s->O, (size_t)s->N * s->g.n);
    update_elitist(s);
    return passes;
}

/* Iterated local search, rounds round0 .. round0 + rounds - 1.  A round, for every solution
   i at once:
     perturbation: for t = 0 .. flips - 1, the word t mod 4 of
       Philox(seed, (generation, 0xFFFFFFFE, i, 16 r + t / 4)), scaled to a class position
       q = (word * |F|) >> 32, names the set at position q of the class-ordered list; its
       variable flips in a copy of P_i (one after another, the fitness following each flip);
     search: passes of the local search over the copies (as or_local_search);
     acceptance: solution i takes its copy when the copy's fitness is at least f_i, else it
       stays as it was;
   then the elitist updates as at a generation end.  The generation and the GOM counters do
   not change.  Returns the passes summed over the rounds, or -1 (nothing done) for a
   non-univariate FOS, an open generation or arguments out of range. */
int32_t or_iterated_local_search(or_state *s, int32_t round0, int32_t rounds, int32_t flips,
                                 int32_t max_passes) {
    if (s->open_next >= 0 || !univariate_fos(s) || round0 < 0 || rounds < 0 ||
        (int64_t)round0 + rounds > (1 << 27) || flips < 0 || flips > 64 || max_passes < 0)
        return -1;
    const int32_t n = s->g.n;
    int64_t *fo = malloc(sizeof(int64_t) * (size_t)s->N);
    if (!fo) return -1;
    int32_t total = 0;
    for (int32_t r = round0; r < round0 + rounds; ++r) {
        memcpy(s->O, s->P, (size_t)s->N * n);
        for (int32_t i = 0; i < s->N; ++i) {
            uint8_t *Oi = s->O + (size_t)i * n;
            fo[i] = s->f[i];
            for (int32_t t = 0; t < flips; ++t) {
                uint32_t out[4];
                draw4(s->seed, (uint32_t)s->gen, 0xFFFFFFFEu, (uint32_t)i,
                      (uint32_t)r * 16u + (uint32_t)t / 4u, out);
                const int32_t q = (int32_t)(((uint64_t)out[t % 4] * (uint64_t)s->nsets) >> 32);
                const int32_t u = s->set_vars[s->set_ptr[s->class_elems[q]]];
                fo[i] += flip_gain(s, Oi, u);
                Oi[u] ^= 1u;
            }
        }
        total += ls_passes(s, fo, max_passes);
        for (int32_t i = 0; i < s->N; ++i)
            if (fo[i] >= s->f[i]) {
                memcpy(s->P + (size_t)i * n, s->O + (size_t)i * n, (size_t)n);
                s->f[i] = fo[i];
            }
        update_elitist(s);
    }
    memcpy(s->O, s->P, (size_t)s->N * n);
    free(fo);
    return total;
}

/* Start a generation if none is open, then run the classes up to order position `pos`
   (inclusive) and leave the generation open.  Returns -1 (nothing done) when pos is out of
   range or the open generation has already passed it. */
int32_t or_stop_after_class(or_state *s, int32_t pos) {
    if (pos < 0 || pos >= s->k) return -1;
    if (s->open_next >= 0 && pos < s->open_next) return -1;
    if (s->open_next < 0) begin_generation(s);
    for (int32_t t = s->open_next; t <= pos; ++t) run_class(s, t);
    s->open_next = pos + 1;
    return 0;
}

/* The canonical byte string: per solution its n genes (the offspring while a generation is
   open), each fitness as 8 little-endian bytes, the n elitist genes, the elitist fitness (8),
   the generation (4), then attempted, evaluated and accepted (8 each). */
static uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static void hash_bytes(uint64_t *h, uint64_t *k, const uint8_t *b, size_t len) {
    for (size_t t = 0; t < len; ++t, ++*k) *h += mix64((*k << 8) | b[t]);
}

static void hash_int(uint64_t *h, uint64_t *k, uint64_t x, int bytes) {
    for (int t = 0; t < bytes; ++t, ++*k) *h += mix64((*k << 8) | ((x >> (8 * t)) & 0xFFu));
}

uint64_t or_hash(const or_state *s) {
    const size_t n = (size_t)s->g.n;
    const uint8_t *X = s->open_next >= 0 ? s->O : s->P;
    uint64_t h = 0, k = 0;
    hash_bytes(&h, &k, X, (size_t)s->N * n);
    for (int32_t i = 0; i < s->N; ++i) hash_int(&h, &k, (uint64_t)s->f[i], 8);
    hash_bytes(&h, &k, s->E, n);
    hash_int(&h, &k, (uint64_t)s->fE, 8);
    hash_int(&h, &k, (uint64_t)(uint32_t)s->gen, 4);
    hash_int(&h, &k, (uint64_t)s->attempted, 8);
    hash_int(&h, &k, (uint64_t)s->evaluated, 8);
    hash_int(&h, &k, (uint64_t)s->accepted, 8);
    return h;
}

/* Generations until the elitist reaches target or max_gens generations have run in total;
   returns the number of generations run by this call. */
int32_t or_run(or_state *s, int64_t target, int32_t max_gens) {
    int32_t start = s->gen;
    while (s->fE < target && s->gen < max_gens) or_generation(s);
    return s->gen - start;
}

/* ------------------------------------------------------------------------------------------
 * Accessors.
 * ---------------------------------------------------------------------------------------- */
int32_t or_num_classes(const or_state *s) { return s->k; }

void or_get_classes(const or_state *s, int32_t *class_ptr, int32_t *class_elems) {
    memcpy(class_ptr, s->class_ptr, sizeof(int32_t) * (size_t)(s->k + 1));
    memcpy(class_elems, s->class_elems, sizeof(int32_t) * (size_t)s->nsets);
}

/* genes: N x n bytes (or NULL; the offspring while a generation is open); fitness: N (running
   values while a generation is open); elite: n (or NULL); counters: attempted, evaluated,
   accepted, debug mismatches. */
void or_get(const or_state *s, uint8_t *genes, int64_t *fitness, uint8_t *elite,
            int64_t *elite_fitness, int32_t *generation, int64_t counters[4]) {
    const size_t n = (size_t)s->g.n;
    if (genes) memcpy(genes, s->open_next >= 0 ? s->O : s->P, (size_t)s->N * n);
    if (fitness) memcpy(fitness, s->f, sizeof(int64_t) * (size_t)s->N);
    if (elite) memcpy(elite, s->E, n);
    if (elite_fitness) *elite_fitness = s->fE;
    if (generation) *generation = s->gen;
    if (counters) {
        counters[0] = s->attempted;
        counters[1] = s->evaluated;
        counters[2] = s->accepted;
        counters[3] = s->debug_mismatches;
    }
}

/* Replace the population (fitness recomputed in full), elitist and counters; resume point. */
void or_set(or_state *s, const uint8_t *genes, const uint8_t *elite, int64_t elite_fitness,
            int32_t generation, const int64_t counters[3]) {
    const size_t n = (size_t)s->g.n;
    memcpy(s->P, genes, (size_t)s->N * n);
    memcpy(s->O, genes, (size_t)s->N * n);
    full_fitness_all(s);
    memcpy(s->E, elite, n);
    s->fE = elite_fitness;
    s->gen = generation;
    s->attempted = counters[0];
    s->evaluated = counters[1];
    s->accepted = counters[2];
    s->open_next = -1;
}
