/*
 * CPU oracle for exact triangle counting. TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the package's smoke check and the benchmark's CPU-baseline
 * leg may load this library. It shares no code, header or helper with the GPU
 * library: it is a plain, slow, obviously correct restatement of what the
 * paper's method computes, in the paper's order of steps.
 *
 * Problem (Section 3): exact triangle count of an undirected simple graph.
 * Input pairs are unordered; self-loops are dropped and repeated pairs count
 * once (the dataset table of Section 5 counts de-duplicated edges).
 *
 *   T    = number of vertex triples {a,b,c} with all three edges present
 *   t[v] = number of triangles that contain v
 *
 * Functions:
 *  - oracle_count_forward: the forward algorithm (Section 3.2, "TC using set
 *    intersection", Algorithm 2; orientation by degree order, Section 4.2):
 *    keep each edge once, directed along a strict total order of the
 *    vertices, and intersect the two out-neighbour lists of every kept edge.
 *    oracle_count_forward_timed is the same with the wall time of its two
 *    stages (orientation + out-lists, intersections) reported;
 *    oracle_count_forward_rows restricts the intersections to every k-th row.
 *  - oracle_forward_edge_counts: the per-edge intersection sizes of the
 *    forward algorithm (Algorithm 2), in canonical pair order.
 *  - oracle_vertex_triangles: t[v] by definition, the number of edges among
 *    the neighbours of v. Written independently of the forward algorithm.
 *  - oracle_oriented_edge_counts: per kept edge (a -> b), the number of
 *    common neighbours w that follow both a and b in the (degree, id) order.
 *    This is the per-edge intersection size of Section 3.2.
 *  - oracle_edge_support: per edge, the number of triangles through it
 *    (the per-edge triangle support used by k-truss, Section 1).
 *  - oracle_matrix_rows: the matrix formulation (Section 3.3, Algorithm 3),
 *    row by row: C = A o (L U) without forming L U, per-row sums of C.
 *  - oracle_full_sum: the full-list variant of the intersection method
 *    (each edge once, whole neighbour lists; Section 4.2 without the induced
 *    subgraph): the sum of |N(a) intersected with N(b)| over the edges.
 *
 * Integers only; every count is accumulated in uint64_t, so there is no
 * rounding anywhere.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>

#include <algorithm>
#include <parallel/algorithm>
#include <vector>

namespace {

struct Graph {
    int32_t n = 0;
    int64_t m = 0;
    std::vector<uint64_t> keys;       // canonical pairs (min << 32 | max), sorted, unique
    std::vector<int32_t> deg;         // degree in the simple graph
    std::vector<int64_t> deg_input;   // input pairs incident to v (loops dropped, repeats counted)
    std::vector<int64_t> adj_off;     // symmetric adjacency, rows sorted by id
    std::vector<int32_t> adj;
};

int pick_threads(int threads) { return threads > 0 ? threads : omp_get_max_threads(); }

// (degree, id) ascending: the strict total order used to orient edges.
inline bool precedes_deg_id(const Graph& g, int32_t a, int32_t b) {
    return g.deg[a] < g.deg[b] || (g.deg[a] == g.deg[b] && a < b);
}
// The same order with the degree counted over the input pairs (repeats included).
inline bool precedes_input_deg_id(const Graph& g, int32_t a, int32_t b) {
    return g.deg_input[a] < g.deg_input[b] || (g.deg_input[a] == g.deg_input[b] && a < b);
}
// The paper's literal filter keeps e(u,v) with d(u) > d(v), ties to the
// smaller id: degree descending, id ascending.
inline bool precedes_paper(const Graph& g, int32_t a, int32_t b) {
    return g.deg[a] > g.deg[b] || (g.deg[a] == g.deg[b] && a < b);
}
inline bool precedes(const Graph& g, int mode, int32_t a, int32_t b) {
    if (mode == 1) return precedes_paper(g, a, b);
    if (mode == 2) return a < b;
    return precedes_deg_id(g, a, b);
}

// Size of the intersection of two ascending lists (two-pointer merge).
inline uint64_t merge_count(const int32_t* a, int64_t na, const int32_t* b, int64_t nb) {
    uint64_t c = 0;
    int64_t i = 0, j = 0;
    while (i < na && j < nb) {
        if (a[i] < b[j]) ++i;
        else if (a[i] > b[j]) ++j;
        else { ++c; ++i; ++j; }
    }
    return c;
}

}  // namespace

extern "C" {

/*
 * Status codes: 0 ok, 1 invalid argument, 2 vertex id outside [0, n).
 * seconds (may be NULL) receives wall times: [0] canonicalisation (range
 * check, loops, sort, de-duplication), [1] the degrees, [2] the symmetric
 * adjacency (used by the definition-level functions, not by the forward
 * algorithm).
 */
int oracle_graph_build_timed(const int32_t* edges, int64_t num_edges, int32_t n, int threads, void** out,
                             double* seconds) {
    if (!out || num_edges < 0 || n < 0 || (num_edges > 0 && !edges)) return 1;
    *out = nullptr;
    const double t0 = omp_get_wtime();
    for (int64_t i = 0; i < 2 * num_edges; ++i)
        if (edges[i] < 0 || edges[i] >= n) return 2;
    Graph* g = new Graph;
    g->n = n;
    // Canonicalise: unordered pair -> (min, max); self-loops dropped.
    g->keys.reserve((size_t)num_edges);
    g->deg_input.assign((size_t)n, 0);
    for (int64_t i = 0; i < num_edges; ++i) {
        uint32_t a = (uint32_t)edges[2 * i], b = (uint32_t)edges[2 * i + 1];
        if (a == b) continue;
        g->deg_input[a]++;
        g->deg_input[b]++;
        if (a > b) std::swap(a, b);
        g->keys.push_back(((uint64_t)a << 32) | b);
    }
    // De-duplicate: sort, then keep one of each run of equal pairs.
    omp_set_num_threads(pick_threads(threads));
    __gnu_parallel::sort(g->keys.begin(), g->keys.end());
    g->keys.erase(std::unique(g->keys.begin(), g->keys.end()), g->keys.end());
    g->m = (int64_t)g->keys.size();
    const double t1 = omp_get_wtime();
    // Degrees and the symmetric adjacency (rows ascending by id).
    g->deg.assign((size_t)n, 0);
    for (uint64_t k : g->keys) { g->deg[k >> 32]++; g->deg[(uint32_t)k]++; }
    const double t2 = omp_get_wtime();
    g->adj_off.assign((size_t)n + 1, 0);
    for (int32_t v = 0; v < n; ++v) g->adj_off[v + 1] = g->adj_off[v] + g->deg[v];
    g->adj.resize((size_t)(2 * g->m));
    std::vector<int64_t> fill(g->adj_off.begin(), g->adj_off.end() - 1);
    for (uint64_t k : g->keys) {
        int32_t a = (int32_t)(k >> 32), b = (int32_t)(uint32_t)k;
        g->adj[fill[a]++] = b;
        g->adj[fill[b]++] = a;
    }
#pragma omp parallel for schedule(dynamic, 1024) num_threads(pick_threads(threads))
    for (int32_t v = 0; v < n; ++v)
        std::sort(g->adj.begin() + g->adj_off[v], g->adj.begin() + g->adj_off[v + 1]);
    if (seconds) {
        seconds[0] = t1 - t0;
        seconds[1] = t2 - t1;
        seconds[2] = omp_get_wtime() - t2;
    }
    *out = g;
    return 0;
}

int oracle_graph_build(const int32_t* edges, int64_t num_edges, int32_t n, int threads, void** out) {
    return oracle_graph_build_timed(edges, num_edges, n, threads, out, nullptr);
}

void oracle_graph_free(void* h) { delete (Graph*)h; }

int64_t oracle_graph_num_edges(const void* h) { return ((const Graph*)h)->m; }

/* Canonical pairs (a < b), ascending, as int32 [m][2]. */
void oracle_graph_edges(const void* h, int32_t* out) {
    const Graph* g = (const Graph*)h;
    for (int64_t i = 0; i < g->m; ++i) {
        out[2 * i] = (int32_t)(g->keys[i] >> 32);
        out[2 * i + 1] = (int32_t)(uint32_t)g->keys[i];
    }
}

void oracle_graph_degrees(const void* h, int32_t* out) {
    const Graph* g = (const Graph*)h;
    for (int32_t v = 0; v < g->n; ++v) out[v] = g->deg[v];
}

/*
 * Forward algorithm (Section 3.2, Algorithm 2; filter of Section 4.2).
 *   order_mode 0: orient along (degree, id) ascending (the reading used by
 *                 the GPU path), 1: the paper's literal filter (degree
 *                 descending, id ascending), 2: plain id order.
 * Every strict total order finds each triangle exactly once, at the edge
 * joining its two smallest vertices, so T and t do not depend on the mode.
 * per_vertex (length n, may be NULL) receives t[v]: each thread adds its
 * matches into an array of its own, and the arrays are summed at the end.
 * seconds (may be NULL): [0] orientation and out-lists, [1] intersections.
 * oracle_count_forward_rows runs the intersections of the rows u with
 * u % row_stride == 0 only (the CPU baseline's bounded sample; stride 1 is
 * the whole algorithm): it returns the triangles whose earliest vertex is such
 * a u, and rows_edges (may be NULL) receives the kept edges of those rows.
 */
uint64_t oracle_count_forward_rows(const void* h, int order_mode, int32_t row_stride, uint64_t* per_vertex,
                                   int threads, double* seconds, int64_t* rows_edges) {
    const Graph* g = (const Graph*)h;
    const int32_t n = g->n;
    const int nth = pick_threads(threads);
    const double t0 = omp_get_wtime();
    // Form the filtered edge list: each edge once, from the earlier to the later endpoint.
    std::vector<int64_t> off((size_t)n + 1, 0);
    for (uint64_t k : g->keys) {
        int32_t a = (int32_t)(k >> 32), b = (int32_t)(uint32_t)k;
        off[(precedes(*g, order_mode, a, b) ? a : b) + 1]++;
    }
    for (int32_t v = 0; v < n; ++v) off[v + 1] += off[v];
    std::vector<int32_t> out_adj((size_t)g->m);
    std::vector<int64_t> fill(off.begin(), off.end() - 1);
    for (uint64_t k : g->keys) {
        int32_t a = (int32_t)(k >> 32), b = (int32_t)(uint32_t)k;
        if (precedes(*g, order_mode, a, b)) out_adj[fill[a]++] = b;
        else out_adj[fill[b]++] = a;
    }
    // Out-lists sorted by vertex id (keys are ascending, but sort to be explicit).
#pragma omp parallel for schedule(dynamic, 1024) num_threads(nth)
    for (int32_t v = 0; v < n; ++v) std::sort(out_adj.begin() + off[v], out_adj.begin() + off[v + 1]);
    const double t1 = omp_get_wtime();
    // Intersect the two out-lists of every kept edge; reduce the counts.
    uint64_t total = 0;
    std::vector<std::vector<uint64_t>> local(per_vertex ? (size_t)nth : 0);
#pragma omp parallel num_threads(nth)
    {
        uint64_t* t = nullptr;
        if (per_vertex) {
            std::vector<uint64_t>& mine = local[(size_t)omp_get_thread_num()];
            mine.assign((size_t)n, 0);
            t = mine.data();
        }
#pragma omp for schedule(dynamic, 64) reduction(+ : total)
        for (int32_t u = 0; u < n; ++u) {
            if (u % row_stride != 0) continue;
            const int32_t* nu = out_adj.data() + off[u];
            const int64_t du = off[u + 1] - off[u];
            for (int64_t p = 0; p < du; ++p) {
                int32_t v = nu[p];
                const int32_t* nv = out_adj.data() + off[v];
                const int64_t dv = off[v + 1] - off[v];
                if (!t) {
                    total += merge_count(nu, du, nv, dv);
                    continue;
                }
                int64_t i = 0, j = 0;
                while (i < du && j < dv) {
                    if (nu[i] < nv[j]) ++i;
                    else if (nu[i] > nv[j]) ++j;
                    else {
                        ++total;
                        t[u]++;
                        t[v]++;
                        t[nu[i]]++;
                        ++i; ++j;
                    }
                }
            }
        }
    }
    if (per_vertex) {
#pragma omp parallel for schedule(static) num_threads(nth)
        for (int32_t v = 0; v < n; ++v) {
            uint64_t s = 0;
            for (const std::vector<uint64_t>& l : local) s += l[v];
            per_vertex[v] = s;
        }
    }
    if (seconds) {
        seconds[0] = t1 - t0;
        seconds[1] = omp_get_wtime() - t1;
    }
    if (rows_edges) {
        int64_t c = 0;
        for (int32_t u = 0; u < n; u += row_stride) c += off[u + 1] - off[u];
        *rows_edges = c;
    }
    return total;
}

uint64_t oracle_count_forward_timed(const void* h, int order_mode, uint64_t* per_vertex, int threads,
                                    double* seconds) {
    return oracle_count_forward_rows(h, order_mode, 1, per_vertex, threads, seconds, nullptr);
}

uint64_t oracle_count_forward(const void* h, int order_mode, uint64_t* per_vertex, int threads) {
    return oracle_count_forward_timed(h, order_mode, per_vertex, threads, nullptr);
}

/*
 * One call from the edge list to T (Section 3.2, Algorithm 2): canonicalise,
 * orient by (degree, id), count by the forward algorithm. h_per_vertex (may
 * be NULL) receives t[v] for v in [0, num_vertices). A null or negative
 * argument, or an id outside [0, num_vertices), returns UINT64_MAX and writes
 * nothing. threads <= 0: all cores.
 */
uint64_t tc_oracle_count(const int32_t* h_edges, int64_t num_edges, int32_t num_vertices, uint64_t* h_per_vertex,
                         int threads) {
    void* h = nullptr;
    if (oracle_graph_build(h_edges, num_edges, num_vertices, threads, &h) != 0) return UINT64_MAX;
    const uint64_t T = oracle_count_forward(h, 0, h_per_vertex, threads);
    oracle_graph_free(h);
    return T;
}

/*
 * The forward algorithm's per-edge intersection sizes (Algorithm 2): for each kept edge
 * x -> y of the (degree, id) orientation, |N+(x) intersected with N+(y)| by a
 * two-pointer merge of the two out-lists, written at the index of the edge's
 * canonical pair (ascending order of oracle_graph_edges). degree_mode 0: the
 * simple graph's degree; 1: input pairs at the vertex. The definition-level
 * oracle_oriented_edge_counts gives the same values by another route.
 */
void oracle_forward_edge_counts(const void* h, int degree_mode, uint32_t* out, int threads) {
    const Graph* g = (const Graph*)h;
    const int32_t n = g->n;
    struct Out {
        int32_t w;        // out-neighbour
        int64_t pair;     // index of the canonical pair
    };
    auto before = [&](int32_t a, int32_t b) {
        return degree_mode ? precedes_input_deg_id(*g, a, b) : precedes_deg_id(*g, a, b);
    };
    std::vector<int64_t> off((size_t)n + 1, 0);
    for (uint64_t k : g->keys) {
        int32_t a = (int32_t)(k >> 32), b = (int32_t)(uint32_t)k;
        off[(before(a, b) ? a : b) + 1]++;
    }
    for (int32_t v = 0; v < n; ++v) off[v + 1] += off[v];
    std::vector<Out> lst((size_t)g->m);
    std::vector<int64_t> fill(off.begin(), off.end() - 1);
    for (int64_t i = 0; i < g->m; ++i) {
        int32_t a = (int32_t)(g->keys[i] >> 32), b = (int32_t)(uint32_t)g->keys[i];
        if (before(a, b)) lst[fill[a]++] = {b, i};
        else lst[fill[b]++] = {a, i};
    }
#pragma omp parallel for schedule(dynamic, 1024) num_threads(pick_threads(threads))
    for (int32_t v = 0; v < n; ++v)
        std::sort(lst.begin() + off[v], lst.begin() + off[v + 1], [](const Out& x, const Out& y) { return x.w < y.w; });
#pragma omp parallel for schedule(dynamic, 64) num_threads(pick_threads(threads))
    for (int32_t u = 0; u < n; ++u) {
        const Out* nu = lst.data() + off[u];
        const int64_t du = off[u + 1] - off[u];
        for (int64_t p = 0; p < du; ++p) {
            const Out* nv = lst.data() + off[nu[p].w];
            const int64_t dv = off[nu[p].w + 1] - off[nu[p].w];
            uint32_t c = 0;
            int64_t i = 0, j = 0;
            while (i < du && j < dv) {
                if (nu[i].w < nv[j].w) ++i;
                else if (nu[i].w > nv[j].w) ++j;
                else { ++c; ++i; ++j; }
            }
            out[nu[p].pair] = c;
        }
    }
}

/*
 * t[v] for the k vertices vs[0..k): by definition, the number of edges whose
 * two endpoints are both neighbours of v. Neighbours of v are marked in a
 * byte map; each edge {a,b} with a, b in N(v) is seen twice (from a and b).
 */
void oracle_vertex_triangles(const void* h, const int32_t* vs, int64_t k, uint64_t* out, int threads) {
    const Graph* g = (const Graph*)h;
#pragma omp parallel num_threads(pick_threads(threads))
    {
        std::vector<uint8_t> mark((size_t)g->n, 0);
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < k; ++q) {
            int32_t v = vs[q];
            for (int64_t p = g->adj_off[v]; p < g->adj_off[v + 1]; ++p) mark[g->adj[p]] = 1;
            uint64_t twice = 0;
            for (int64_t p = g->adj_off[v]; p < g->adj_off[v + 1]; ++p) {
                int32_t a = g->adj[p];
                for (int64_t r = g->adj_off[a]; r < g->adj_off[a + 1]; ++r) twice += mark[g->adj[r]];
            }
            for (int64_t p = g->adj_off[v]; p < g->adj_off[v + 1]; ++p) mark[g->adj[p]] = 0;
            out[q] = twice / 2;
        }
    }
}

/*
 * Per-edge intersection sizes for the (degree, id) orientation. For the
 * canonical pair i (a < b, ascending order of oracle_graph_edges), out[i] =
 * |{ w : w ~ a, w ~ b, a < w and b < w in (degree, id) order }|, the size of
 * N+(x) intersected with N+(y) for the kept edge x -> y on {a, b}.
 * degree_mode 0: degree in the simple graph; 1: number of input pairs at the
 * vertex (self-loops dropped, repeated pairs counted). The two agree on
 * inputs without repeats.
 */
void oracle_oriented_edge_counts(const void* h, int degree_mode, uint32_t* out, int threads) {
    const Graph* g = (const Graph*)h;
#pragma omp parallel for schedule(dynamic, 4096) num_threads(pick_threads(threads))
    for (int64_t i = 0; i < g->m; ++i) {
        int32_t a = (int32_t)(g->keys[i] >> 32), b = (int32_t)(uint32_t)g->keys[i];
        const int32_t* na = g->adj.data() + g->adj_off[a];
        const int32_t* nb = g->adj.data() + g->adj_off[b];
        int64_t da = g->adj_off[a + 1] - g->adj_off[a], db = g->adj_off[b + 1] - g->adj_off[b];
        uint32_t c = 0;
        int64_t x = 0, y = 0;
        while (x < da && y < db) {
            if (na[x] < nb[y]) ++x;
            else if (na[x] > nb[y]) ++y;
            else {
                int32_t w = na[x];
                const bool after_a = degree_mode ? precedes_input_deg_id(*g, a, w) : precedes_deg_id(*g, a, w);
                const bool after_b = degree_mode ? precedes_input_deg_id(*g, b, w) : precedes_deg_id(*g, b, w);
                if (after_a && after_b) ++c;
                ++x; ++y;
            }
        }
        out[i] = c;
    }
}

/*
 * The oriented per-edge count of oracle_oriented_edge_counts for k given
 * pairs (a_q, b_q) (any order; each must be an edge of the graph, else the
 * count is 0): the number of common neighbours w after both a_q and b_q in
 * (degree, id) order, degree_mode as above.
 */
void oracle_pair_counts(const void* h, const int32_t* pairs, int64_t k, int degree_mode, uint32_t* out,
                        int threads) {
    const Graph* g = (const Graph*)h;
#pragma omp parallel for schedule(dynamic, 16) num_threads(pick_threads(threads))
    for (int64_t q = 0; q < k; ++q) {
        const int32_t a = pairs[2 * q], b = pairs[2 * q + 1];
        const int32_t* na = g->adj.data() + g->adj_off[a];
        const int32_t* nb = g->adj.data() + g->adj_off[b];
        const int64_t da = g->adj_off[a + 1] - g->adj_off[a], db = g->adj_off[b + 1] - g->adj_off[b];
        if (!std::binary_search(na, na + da, b)) { out[q] = 0; continue; }
        uint32_t c = 0;
        int64_t x = 0, y = 0;
        while (x < da && y < db) {
            if (na[x] < nb[y]) ++x;
            else if (na[x] > nb[y]) ++y;
            else {
                const int32_t w = na[x];
                const bool after_a = degree_mode ? precedes_input_deg_id(*g, a, w) : precedes_deg_id(*g, a, w);
                const bool after_b = degree_mode ? precedes_input_deg_id(*g, b, w) : precedes_deg_id(*g, b, w);
                if (after_a && after_b) ++c;
                ++x; ++y;
            }
        }
        out[q] = c;
    }
}

/* Per-edge triangle support |N(a) intersected with N(b)| for canonical pair i. */
void oracle_edge_support(const void* h, uint32_t* out, int threads) {
    const Graph* g = (const Graph*)h;
#pragma omp parallel for schedule(dynamic, 4096) num_threads(pick_threads(threads))
    for (int64_t i = 0; i < g->m; ++i) {
        int32_t a = (int32_t)(g->keys[i] >> 32), b = (int32_t)(uint32_t)g->keys[i];
        out[i] = (uint32_t)merge_count(g->adj.data() + g->adj_off[a], g->adj_off[a + 1] - g->adj_off[a],
                                       g->adj.data() + g->adj_off[b], g->adj_off[b + 1] - g->adj_off[b]);
    }
}

/*
 * Full-list variant: the edge list is filtered (each undirected edge once,
 * here the canonical pairs) but every intersection takes the whole
 * neighbour lists, N(a) with N(b). A triangle is found once at each of its
 * three edges, so the returned sum is 3T.
 */
uint64_t oracle_full_sum(const void* h, int threads) {
    const Graph* g = (const Graph*)h;
    uint64_t total = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : total) num_threads(pick_threads(threads))
    for (int64_t i = 0; i < g->m; ++i) {
        int32_t a = (int32_t)(g->keys[i] >> 32), b = (int32_t)(uint32_t)g->keys[i];
        total += merge_count(g->adj.data() + g->adj_off[a], g->adj_off[a + 1] - g->adj_off[a],
                             g->adj.data() + g->adj_off[b], g->adj_off[b + 1] - g->adj_off[b]);
    }
    return total;
}

/*
 * Matrix formulation (Section 3.3, Algorithm 3), row by row:
 *   1. order the rows (and columns) by increasing number of nonzeros, ties
 *      by id (order_mode 0), or keep the id order (order_mode 2);
 *   2. L holds the entries (i, k) with k before i in that order, U the
 *      entries (k, j) with k before j, so that A = L + U;
 *   3-4. row i of C = A o (L U): for every k in row i of L and every j in
 *      row k of U, C(i, j) gains one if A(i, j) is set (a dense marker of
 *      row i of A stands in for the Hadamard product; B = L U is not stored);
 *   5. T = (1/2) sum C (the sum of C, as the worked example of Figure 4
 *      states; the printed last line sums A).
 * upper = 1 keeps only the entries of C above the diagonal (j after i; the
 * first optimisation of the matrix implementation in Section 3.3): their
 * sum is T itself.
 * row_sums (length n, original ids, may be NULL) receives sum_j C(i, j);
 * returns sum C.
 */
uint64_t oracle_matrix_rows(const void* h, int order_mode, int upper, uint64_t* row_sums, int threads) {
    const Graph* g = (const Graph*)h;
    const int32_t n = g->n;
    std::vector<int64_t> pos((size_t)n);   // place of each vertex in the row order
    {
        std::vector<int32_t> perm((size_t)n);
        for (int32_t v = 0; v < n; ++v) perm[v] = v;
        if (order_mode == 0)
            std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return g->deg[a] < g->deg[b]; });
        for (int32_t q = 0; q < n; ++q) pos[perm[q]] = q;
    }
    uint64_t total = 0;
#pragma omp parallel num_threads(pick_threads(threads))
    {
        std::vector<uint8_t> mask((size_t)n, 0);
#pragma omp for schedule(dynamic, 256) reduction(+ : total)
        for (int32_t i = 0; i < n; ++i) {
            const int64_t a0 = g->adj_off[i], a1 = g->adj_off[i + 1];
            for (int64_t p = a0; p < a1; ++p) {   // row i of A (cut to the upper triangle if asked)
                const int32_t j = g->adj[p];
                if (!upper || pos[j] > pos[i]) mask[j] = 1;
            }
            uint64_t row = 0;
            for (int64_t p = a0; p < a1; ++p) {
                const int32_t k = g->adj[p];
                if (pos[k] >= pos[i]) continue;   // L(i, k) needs k before i
                for (int64_t r = g->adj_off[k]; r < g->adj_off[k + 1]; ++r) {
                    const int32_t j = g->adj[r];
                    if (pos[j] > pos[k]) row += mask[j];   // U(k, j) needs k before j
                }
            }
            for (int64_t p = a0; p < a1; ++p) mask[g->adj[p]] = 0;
            if (row_sums) row_sums[i] = row;
            total += row;
        }
    }
    return total;
}

}  // extern "C"
