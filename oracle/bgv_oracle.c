/*
 * BigGraphVis CPU ORACLE -- test infrastructure, not part of the product.
 *
 * A plain, slow, obviously correct CPU implementation of what the GPU path computes,
 * written from the paper (Moradi & Mondal, "BigGraphVis", arXiv 2108.00529):
 *   - streaming community detection (Section 3.2 and Section 3.2.1, Algorithm 3),
 *     in its batch-synchronous form: fixed chunks of the edge stream read the label
 *     snapshot taken at the chunk start, and the smallest edge index wins a conflict;
 *   - community sizes and supergraph by count-min sketch (Section 3.3, Algorithm 2,
 *     Section 4.1);
 *   - ForceAtlas2 layout of the supergraph (Section 3.1, Algorithm 1), in the force
 *     and speed forms of the ForceAtlas2 publication the paper cites, with exact
 *     O(K^2) repulsion or a Barnes-Hut tree;
 *   - the ForceAtlas2 energy whose negative gradient is that force field.
 * Floating point is FP64 throughout.  No blocking, fusion or reordering beyond the
 * definitions.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library; the GPU path never does.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC bgv_oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------------ */
/* Community detection                                                             */
/* ------------------------------------------------------------------------------ */

/* Threshold of pass p (0-based): D1 * growth^p, saturating at INT32_MAX
 * (Section 3.2.1: the threshold is multiplied by a constant factor each round). */
static int32_t orc_threshold(int32_t D1, int32_t growth, int32_t p)
{
    int64_t D = D1;
    for (int32_t k = 0; k < p; ++k) {
        D *= growth;
        if (D > INT32_MAX) return INT32_MAX;
    }
    return (int32_t)D;
}

/*
 * Batch-synchronous streaming community detection.
 *
 * Rule (Section 3.2): every streamed edge raises the degree of both endpoints; if
 * both degrees are at most the threshold, the endpoint of smaller degree joins the
 * community of the endpoint of larger degree; equal degrees do nothing (the nesting
 * of the conditions in Algorithm 3), or, with tie = 1 (the variant where the stream's
 * first endpoint joins the second's community on a tie), the first endpoint joins.  Degrees are never reset between passes
 * (Algorithm 3 initialises them once, before the round loop).  Self-loops are ignored.
 *
 * Batch-synchronous reading: within each pass the stream is cut into chunks of
 * `chunk` edges.  For each chunk: (a) all degree increments of the chunk are applied;
 * (b) every edge of the chunk is tested with those chunk-end degrees and with the
 * labels as they were when the chunk started; (c) each node that received proposals
 * takes the label proposed by the edge of smallest index.  chunk == 1 is exactly the
 * sequential rule.
 *
 * rule = 1: the community-volume rule of the SCoDA algorithm the paper adopts, in the
 * same batch-synchronous form.  V[c] = sum of the counters of the nodes labelled c (a
 * node's increments add to its community's V; a move carries its counter along).  An
 * edge whose endpoints both have counters at most D and different chunk-start labels
 * proposes: u joins v's community if V[label u] <= V[label v], else v joins u's (V and
 * counters as at the end of the chunk's increments).  Endpoints already sharing a
 * label make no proposal.  (tie must be 0 with rule 1.)
 *
 * label[n] (out), counter[n] (out: degree counter after all passes = passes * d(v)).
 * Returns 0, or -1 on bad arguments.
 */
int orc_bs_community(int32_t n, int64_t m, const int32_t *edges, int32_t D1,
                     int32_t passes, int32_t growth, int64_t chunk, int32_t tie, int32_t rule,
                     int32_t *label, int32_t *counter)
{
    if (n <= 0 || m < 0 || passes < 1 || growth < 1 || chunk < 1 || D1 < 0 || tie < 0 || tie > 1) return -1;
    if (rule < 0 || rule > 1 || (rule == 1 && tie)) return -1;
    int64_t *prop_edge = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int32_t *prop_label = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)(chunk < m ? chunk : (m > 0 ? m : 1)));
    if (!prop_edge || !prop_label || !touched) { free(prop_edge); free(prop_label); free(touched); return -1; }
    int64_t *vol = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    if (!vol) { free(prop_edge); free(prop_label); free(touched); return -1; }
    for (int32_t v = 0; v < n; ++v) { label[v] = v; counter[v] = 0; prop_edge[v] = -1; }

    for (int32_t p = 0; p < passes; ++p) {
        const int32_t D = orc_threshold(D1, growth, p);
        for (int64_t s = 0; s < m; s += chunk) {
            const int64_t e = (s + chunk < m) ? s + chunk : m;
            /* (a) degree increments of the whole chunk */
            for (int64_t i = s; i < e; ++i) {
                const int32_t u = edges[2 * i], v = edges[2 * i + 1];
                if (u == v) continue;
                counter[u] += 1;
                counter[v] += 1;
                vol[label[u]] += 1;
                vol[label[v]] += 1;
            }
            /* (b) decisions on chunk-end degrees and chunk-start labels */
            int64_t nt = 0;
            for (int64_t i = s; i < e; ++i) {
                const int32_t u = edges[2 * i], v = edges[2 * i + 1];
                if (u == v) continue;
                const int32_t du = counter[u], dv = counter[v];
                if (du > D || dv > D) continue;
                int32_t x, y;
                if (rule == 0) {
                    if (du == dv && !tie) continue;
                    /* lower degree joins the higher's community; on a tie (tie = 1) u joins v */
                    x = (du <= dv) ? u : v;
                    y = (du <= dv) ? v : u;
                } else {
                    if (label[u] == label[v]) continue;
                    /* the endpoint of the smaller (or equal) community volume moves */
                    x = (vol[label[u]] <= vol[label[v]]) ? u : v;
                    y = (x == u) ? v : u;
                }
                if (prop_edge[x] < 0) {                /* first (smallest) index wins */
                    prop_edge[x] = i;
                    prop_label[x] = label[y];
                    touched[nt++] = x;
                }
            }
            /* (c) apply */
            for (int64_t t = 0; t < nt; ++t) {
                const int32_t x = touched[t];
                vol[label[x]] -= counter[x];   /* the move carries x's counter along */
                vol[prop_label[x]] += counter[x];
                label[x] = prop_label[x];
                prop_edge[x] = -1;
            }
        }
    }
    free(prop_edge); free(prop_label); free(touched); free(vol);
    return 0;
}

/* True degree d(v) = counter[v] / passes (each pass adds exactly d(v)) and the exact
 * community volume vol[c] = sum of d(v) over L[v] = c, i.e. the supernode weight the
 * paper estimates with the sketch (Section 4.1: twice the edges of the community). */
void orc_degree_volume(int32_t n, int32_t passes, const int32_t *counter,
                       const int32_t *label, int32_t *degree, int64_t *volume)
{
    for (int32_t v = 0; v < n; ++v) volume[v] = 0;
    for (int32_t v = 0; v < n; ++v) {
        degree[v] = counter[v] / passes;
        volume[label[v]] += degree[v];
    }
}

/* ------------------------------------------------------------------------------ */
/* Count-min sketch (Section 3.3, Algorithm 2; supernode weights Section 4.1)      */
/* ------------------------------------------------------------------------------ */

/* Row hash of a 32-bit key: multiply-add-shift (Dietzfelbinger) to a 32-bit value,
 * then Lemire's multiply-high reduction to [0, cols).  Arithmetic mod 2^64. */
static uint32_t orc_col_key(uint64_t A, uint64_t B, uint32_t x, uint32_t cols)
{
    uint64_t t = A * (uint64_t)x + B;
    return (uint32_t)(((t >> 32) * (uint64_t)cols) >> 32);
}

/* Row hash of an unordered pair key (a < b): vector multiply-add-shift. */
static uint32_t orc_col_pair(uint64_t A, uint64_t B, uint64_t C, uint32_t a, uint32_t b,
                             uint32_t cols)
{
    uint64_t t = A * (uint64_t)a + C * (uint64_t)b + B;
    return (uint32_t)(((t >> 32) * (uint64_t)cols) >> 32);
}

/* Exported for the hash test vectors. coef = (A, B, C) of one row. */
uint32_t orc_hash_key(const uint64_t *coef, uint32_t x, uint32_t cols)
{
    return orc_col_key(coef[0], coef[1], x, cols);
}
uint32_t orc_hash_pair(const uint64_t *coef, uint32_t a, uint32_t b, uint32_t cols)
{
    return orc_col_pair(coef[0], coef[1], coef[2], a, b, cols);
}

static int orc_cmp_u64(const void *pa, const void *pb)
{
    uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    return (a > b) - (a < b);
}

/*
 * Supergraph (Algorithm 3, last steps; Section 4.1).
 *
 * Supernodes: the distinct labels, numbered by ascending label (sid).
 * Sketch 1: for every node v and row r, M1[r][h_r(L[v])] += d(v); the size of a
 * community c is min_r M1[r][h_r(c)].
 * Sketch 2: for every non-loop edge whose endpoints carry different labels a != b,
 * with key (min(a,b), max(a,b)), M2[r][g_r(key)] += 1.
 * Superedges: the sorted set of distinct pairs (sid(min), sid(max)); weight = the
 * sketch-2 estimate min_r M2[r][g_r(key)]; count = the exact number of edges.
 *
 * coef: uint64 [rows][3]; sketch 1 uses coef1, sketch 2 uses coef2.
 * Outputs have capacity n (supernodes) and m (superedges).  Returns E_S (>= 0) or -1.
 */
int64_t orc_supergraph(int32_t n, int64_t m, const int32_t *edges, const int32_t *label,
                       const int32_t *degree, int32_t rows, int32_t cols,
                       const uint64_t *coef1, const uint64_t *coef2,
                       int32_t *K_out, int32_t *sid_of_label, int32_t *super_label,
                       uint32_t *super_size, int32_t *se, uint32_t *se_weight,
                       uint32_t *se_count, uint32_t *M1, uint32_t *M2)
{
    if (n <= 0 || m < 0 || rows < 1 || cols < 1) return -1;
    /* supernode numbering */
    for (int32_t c = 0; c < n; ++c) sid_of_label[c] = 0;
    for (int32_t v = 0; v < n; ++v) sid_of_label[label[v]] = 1;
    int32_t K = 0;
    for (int32_t c = 0; c < n; ++c) {
        if (sid_of_label[c]) { super_label[K] = c; sid_of_label[c] = K; ++K; }
        else sid_of_label[c] = -1;
    }
    *K_out = K;
    /* sketch 1 */
    memset(M1, 0, sizeof(uint32_t) * (size_t)rows * (size_t)cols);
    for (int32_t v = 0; v < n; ++v)
        for (int32_t r = 0; r < rows; ++r)
            M1[(size_t)r * cols + orc_col_key(coef1[3 * r], coef1[3 * r + 1], (uint32_t)label[v], (uint32_t)cols)] += (uint32_t)degree[v];
    for (int32_t k = 0; k < K; ++k) {
        uint32_t best = UINT32_MAX;
        for (int32_t r = 0; r < rows; ++r) {
            uint32_t val = M1[(size_t)r * cols + orc_col_key(coef1[3 * r], coef1[3 * r + 1], (uint32_t)super_label[k], (uint32_t)cols)];
            if (val < best) best = val;
        }
        super_size[k] = best;
    }
    /* sketch 2 and inter-community keys */
    memset(M2, 0, sizeof(uint32_t) * (size_t)rows * (size_t)cols);
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
    if (!keys) return -1;
    int64_t nk = 0;
    for (int64_t i = 0; i < m; ++i) {
        const int32_t u = edges[2 * i], v = edges[2 * i + 1];
        if (u == v) continue;
        const int32_t a = label[u], b = label[v];
        if (a == b) continue;
        const uint32_t lo = (uint32_t)(a < b ? a : b), hi = (uint32_t)(a < b ? b : a);
        for (int32_t r = 0; r < rows; ++r)
            M2[(size_t)r * cols + orc_col_pair(coef2[3 * r], coef2[3 * r + 1], coef2[3 * r + 2], lo, hi, (uint32_t)cols)] += 1u;
        keys[nk++] = ((uint64_t)(uint32_t)sid_of_label[lo] << 32) | (uint32_t)sid_of_label[hi];
    }
    qsort(keys, (size_t)nk, sizeof(uint64_t), orc_cmp_u64);
    int64_t E = 0;
    for (int64_t i = 0; i < nk;) {
        int64_t j = i;
        while (j < nk && keys[j] == keys[i]) ++j;
        const int32_t sa = (int32_t)(keys[i] >> 32), sb = (int32_t)(keys[i] & 0xffffffffu);
        se[2 * E] = sa; se[2 * E + 1] = sb;
        se_count[E] = (uint32_t)(j - i);
        uint32_t best = UINT32_MAX;
        for (int32_t r = 0; r < rows; ++r) {
            uint32_t val = M2[(size_t)r * cols + orc_col_pair(coef2[3 * r], coef2[3 * r + 1], coef2[3 * r + 2],
                                                               (uint32_t)super_label[sa], (uint32_t)super_label[sb], (uint32_t)cols)];
            if (val < best) best = val;
        }
        se_weight[E] = best;
        ++E;
        i = j;
    }
    free(keys);
    return E;
}

/* ------------------------------------------------------------------------------ */
/* ForceAtlas2 (Section 3.1, Algorithm 1; forces and speeds of the cited FA2 paper) */
/* ------------------------------------------------------------------------------ */

/* Node mass m_i = (number of distinct incident superedges) + 1, the (deg + 1) of the
 * ForceAtlas2 repulsion and gravity laws. */
void orc_fa2_mass(int32_t K, int64_t E, const int32_t *se, double *mass)
{
    for (int32_t i = 0; i < K; ++i) mass[i] = 1.0;
    for (int64_t e = 0; e < E; ++e) { mass[se[2 * e]] += 1.0; mass[se[2 * e + 1]] += 1.0; }
}

/* Attraction (linear in distance, weight a_e, a_e = 1 when aw is NULL) and gravity
 * (strength kg * m_i towards the origin, zero at the origin). */
static void orc_attract_gravity(int32_t K, const double *x, const double *mass, int64_t E,
                                const int32_t *se, const double *aw, double kg, double *F)
{
    for (int64_t e = 0; e < E; ++e) {
        const int32_t i = se[2 * e], j = se[2 * e + 1];
        const double a = aw ? aw[e] : 1.0;
        const double dx = x[2 * j] - x[2 * i], dy = x[2 * j + 1] - x[2 * i + 1];
        F[2 * i] += a * dx; F[2 * i + 1] += a * dy;
        F[2 * j] -= a * dx; F[2 * j + 1] -= a * dy;
    }
    for (int32_t i = 0; i < K; ++i) {
        const double r = sqrt(x[2 * i] * x[2 * i] + x[2 * i + 1] * x[2 * i + 1]);
        if (r > 0.0) {
            F[2 * i] -= kg * mass[i] * x[2 * i] / r;
            F[2 * i + 1] -= kg * mass[i] * x[2 * i + 1] / r;
        }
    }
}

/* Exact repulsion: F_i += kr m_i m_j (x_i - x_j) / d^2 over all j != i with d > 0. */
static void orc_repulse_exact(int32_t K, const double *x, const double *mass, double kr, double *F)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < K; ++i) {
        double fx = 0.0, fy = 0.0;
        for (int32_t j = 0; j < K; ++j) {
            if (j == i) continue;
            const double dx = x[2 * i] - x[2 * j], dy = x[2 * i + 1] - x[2 * j + 1];
            const double d2 = dx * dx + dy * dy;
            if (d2 > 0.0) {
                const double f = kr * mass[i] * mass[j] / d2;
                fx += f * dx; fy += f * dy;
            }
        }
        F[2 * i] += fx; F[2 * i + 1] += fy;
    }
}

/* ---- Barnes-Hut quadtree (Section 3.1 body repulsion) ---------------------------
 * Section 3.1 approximates far groups of bodies through a hierarchical partition of
 * the plane (the GPU quadtree of Burtscher and Pingali it cites).  The quadtree here:
 * bodies are placed in the bounding square of their FP32 positions (side s0 = the
 * larger extent, 1 if zero) and quantised to a 2^16 x 2^16 grid in FP32 arithmetic; a
 * cell of depth d is a square of side s0 / 2^d, split into its four quadrants at
 * depth d + 1.  The tree is the compressed quadtree: every node is the smallest cell
 * that holds its bodies, so an internal node's bodies occupy at least two of its
 * quadrants, and its children are the nodes of the occupied quadrants.  Bodies that
 * share one grid point form a leaf (depth 16); so does a single body.  The node mass
 * is the sum of the body masses and the centre of mass their weighted mean.
 * (A chain of cells with one occupied quadrant has one body set and one centre of
 * mass, and its smallest cell passes the opening test whenever a larger one does, so
 * the uncompressed quadtree takes the same decisions.)
 *
 * Construction: bodies sorted by 32-bit Morton code of the grid point (x bits at the
 * even positions), ties by body index; a cell is then a contiguous run of the sorted
 * order, and the quadrant of a body at depth d + 1 is the two code bits below the
 * cell's 2d-bit prefix. */
typedef struct {
    int32_t lo, hi;        /* body range in sorted order */
    int32_t child0;        /* first child in the child list, -1 for a leaf */
    int32_t nchild;        /* 2..4 for an internal node, 0 for a leaf */
    int32_t depth;         /* cell depth: side s0 / 2^depth */
    double size, mx, my, mass;
} orc_qt_node;

typedef struct {
    int32_t K;
    int32_t *order;        /* sorted position -> body */
    int32_t *rank;         /* body -> sorted position */
    uint32_t *code;        /* code in sorted order */
    orc_qt_node *nodes;
    int32_t nnodes;
    int32_t *child;        /* child lists */
    int32_t nchildren;
    float s0;
} orc_qt;

static uint32_t orc_spread16(uint32_t v)
{
    uint32_t r = 0;
    for (int b = 0; b < 16; ++b) r |= ((v >> b) & 1u) << (2 * b);
    return r;
}

/* Quantise and encode (the FP32 operation sequence is part of the tree definition). */
void orc_bh_codes(int32_t K, const float *pos, uint32_t *code_out, float *s0_out, float *xmin_out, float *ymin_out)
{
    float xmin = pos[0], xmax = pos[0], ymin = pos[1], ymax = pos[1];
    for (int32_t i = 1; i < K; ++i) {
        if (pos[2 * i] < xmin) xmin = pos[2 * i];
        if (pos[2 * i] > xmax) xmax = pos[2 * i];
        if (pos[2 * i + 1] < ymin) ymin = pos[2 * i + 1];
        if (pos[2 * i + 1] > ymax) ymax = pos[2 * i + 1];
    }
    float ex = xmax - xmin, ey = ymax - ymin;
    float s0 = ex > ey ? ex : ey;
    if (!(s0 > 0.0f)) s0 = 1.0f;
    for (int32_t i = 0; i < K; ++i) {
        volatile float tx = (pos[2 * i] - xmin) / s0;
        volatile float ty = (pos[2 * i + 1] - ymin) / s0;
        volatile float fx = tx * 65536.0f, fy = ty * 65536.0f;
        int32_t qx = (int32_t)fx, qy = (int32_t)fy;
        if (qx > 65535) qx = 65535;
        if (qy > 65535) qy = 65535;
        code_out[i] = orc_spread16((uint32_t)qx) | (orc_spread16((uint32_t)qy) << 1);
    }
    *s0_out = s0; *xmin_out = xmin; *ymin_out = ymin;
}

static const uint32_t *orc_sort_codes;
static int orc_cmp_body(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    uint32_t ca = orc_sort_codes[a], cb = orc_sort_codes[b];
    if (ca != cb) return (ca > cb) - (ca < cb);
    return (a > b) - (a < b);
}

/* The node of the smallest cell holding sorted bodies [lo, hi), and its subtree. */
static int32_t orc_qt_build_rec(orc_qt *t, const double *x, const double *mass, int32_t lo, int32_t hi)
{
    const int32_t id = t->nnodes++;
    const uint32_t a = t->code[lo], b = t->code[hi - 1];
    int32_t depth = 16;
    if (a != b) {
        int prefix = 0;   /* leading bits shared by all codes of the range (sorted: first and last) */
        while (((a ^ b) >> (31 - prefix) & 1u) == 0) ++prefix;
        depth = prefix / 2;
    }
    orc_qt_node nd;
    nd.lo = lo; nd.hi = hi; nd.depth = depth; nd.child0 = -1; nd.nchild = 0;
    nd.size = (double)t->s0 / (double)(1u << depth);
    double M = 0.0, sx = 0.0, sy = 0.0;
    for (int32_t k = lo; k < hi; ++k) {
        const int32_t j = t->order[k];
        M += mass[j]; sx += mass[j] * x[2 * j]; sy += mass[j] * x[2 * j + 1];
    }
    nd.mass = M; nd.mx = sx / M; nd.my = sy / M;
    if (a != b) {
        /* occupied quadrants at depth + 1: runs of equal 2-bit digit below the prefix */
        const int shift = 30 - 2 * depth;
        int32_t runs[5], nr = 0;
        runs[nr++] = lo;
        for (int32_t k = lo + 1; k < hi; ++k)
            if (((t->code[k] >> shift) & 3u) != ((t->code[k - 1] >> shift) & 3u)) runs[nr++] = k;
        runs[nr] = hi;
        nd.child0 = t->nchildren;
        nd.nchild = nr;
        t->nchildren += nr;
        for (int32_t q = 0; q < nr; ++q) t->child[nd.child0 + q] = -1;
        t->nodes[id] = nd;
        for (int32_t q = 0; q < nr; ++q) {
            const int32_t c = orc_qt_build_rec(t, x, mass, runs[q], runs[q + 1]);
            t->child[t->nodes[id].child0 + q] = c;
        }
    } else {
        t->nodes[id] = nd;
    }
    return id;
}

static void orc_qt_build(orc_qt *t, int32_t K, const double *x, const double *mass)
{
    t->K = K;
    float *pf = (float *)malloc(sizeof(float) * 2 * (size_t)K);
    uint32_t *codes = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)K);
    t->order = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    t->rank = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    t->code = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)K);
    t->nodes = (orc_qt_node *)malloc(sizeof(orc_qt_node) * (size_t)(2 * K));
    t->child = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * K));
    t->nnodes = 0;
    t->nchildren = 0;
    for (int32_t i = 0; i < 2 * K; ++i) pf[i] = (float)x[i];
    float xmin, ymin;
    orc_bh_codes(K, pf, codes, &t->s0, &xmin, &ymin);
    for (int32_t i = 0; i < K; ++i) t->order[i] = i;
    orc_sort_codes = codes;
    qsort(t->order, (size_t)K, sizeof(int32_t), orc_cmp_body);
    for (int32_t k = 0; k < K; ++k) { t->code[k] = codes[t->order[k]]; t->rank[t->order[k]] = k; }
    orc_qt_build_rec(t, x, mass, 0, K);
    free(pf); free(codes);
}

static void orc_qt_free(orc_qt *t)
{
    free(t->order); free(t->rank); free(t->code); free(t->nodes); free(t->child);
}

/* Repulsion on body i (Barnes-Hut): a node whose cell holds i is opened; a leaf is
 * summed body by body (skipping i); any other node is replaced by its centre of mass
 * when size / dist < theta (as size^2 < theta^2 dist^2, dist > 0), else opened.
 *
 * Borderline decisions: a single-precision implementation computes the distance from
 * single-precision positions and a centre of mass rounded to single precision, so its
 * test can fall the other way when size / dist lies within its rounding of theta.  A
 * decision is flagged borderline when |size^2 - theta^2 dist^2| <= theta^2 dist^2 tol,
 * tol = 1e-5 + 2 * eps32 * (|x_i| + |y_i| + |cx| + |cy|) * 4 / dist, eps32 = 2^-24:
 * twice the relative change of dist from a rounding of every coordinate, with a
 * factor 4 to spare. */
static void orc_qt_visit(const orc_qt *t, const double *x, const double *mass, int32_t i,
                         int32_t nid, double theta2, double kr, double *fx, double *fy, int32_t *border)
{
    const orc_qt_node *nd = &t->nodes[nid];
    if (nd->nchild == 0) {
        for (int32_t k = nd->lo; k < nd->hi; ++k) {
            const int32_t j = t->order[k];
            if (j == i) continue;
            const double dx = x[2 * i] - x[2 * j], dy = x[2 * i + 1] - x[2 * j + 1];
            const double d2 = dx * dx + dy * dy;
            if (d2 > 0.0) {
                const double f = kr * mass[i] * mass[j] / d2;
                *fx += f * dx; *fy += f * dy;
            }
        }
        return;
    }
    const int32_t ri = t->rank[i];
    if (ri < nd->lo || ri >= nd->hi) {
        const double dx = x[2 * i] - nd->mx, dy = x[2 * i + 1] - nd->my;
        const double d2 = dx * dx + dy * dy;
        if (border && d2 > 0.0) {
            const double eps32 = 1.0 / 16777216.0;
            const double tol = 1e-5 + 8.0 * eps32 * (fabs(x[2 * i]) + fabs(x[2 * i + 1]) + fabs(nd->mx) +
                                                     fabs(nd->my)) / sqrt(d2);
            if (fabs(nd->size * nd->size - theta2 * d2) <= theta2 * d2 * tol) *border = 1;
        }
        if (d2 > 0.0 && nd->size * nd->size < theta2 * d2) {
            const double f = kr * mass[i] * nd->mass / d2;
            *fx += f * dx; *fy += f * dy;
            return;
        }
    }
    for (int32_t q = 0; q < nd->nchild; ++q)
        orc_qt_visit(t, x, mass, i, t->child[nd->child0 + q], theta2, kr, fx, fy, border);
}

/* Barnes-Hut repulsion added into F; border (optional, K entries) receives 1 for the
 * bodies with a borderline opening decision, else 0. */
void orc_bh_repulsion(int32_t K, const double *x, const double *mass, double kr, double theta, double *F,
                      int32_t *border)
{
    orc_qt t;
    orc_qt_build(&t, K, x, mass);
    const double theta2 = theta * theta;
#pragma omp parallel for schedule(dynamic, 64)
    for (int32_t i = 0; i < K; ++i) {
        double fx = 0.0, fy = 0.0;
        int32_t b = 0;
        orc_qt_visit(&t, x, mass, i, 0, theta2, kr, &fx, &fy, border ? &b : NULL);
        F[2 * i] += fx; F[2 * i + 1] += fy;
        if (border) border[i] = b;
    }
    orc_qt_free(&t);
}

static void orc_repulse_bh(int32_t K, const double *x, const double *mass, double kr, double theta, double *F)
{
    orc_bh_repulsion(K, x, mass, kr, theta, F, NULL);
}

/* Tree export for the structure tests: order[K]; per node (lo, hi, first child in
 * child[], number of children, depth) and (size, mass, cx, cy); child[] (<= 2K
 * entries).  Returns the node count (<= 2K - 1). */
int32_t orc_bh_tree_export(int32_t K, const double *x, const double *mass, int32_t *order,
                           int32_t *node_i5, double *node_d4, int32_t *child)
{
    orc_qt t;
    orc_qt_build(&t, K, x, mass);
    for (int32_t k = 0; k < K; ++k) order[k] = t.order[k];
    for (int32_t n = 0; n < t.nnodes; ++n) {
        node_i5[5 * n] = t.nodes[n].lo; node_i5[5 * n + 1] = t.nodes[n].hi;
        node_i5[5 * n + 2] = t.nodes[n].child0; node_i5[5 * n + 3] = t.nodes[n].nchild;
        node_i5[5 * n + 4] = t.nodes[n].depth;
        node_d4[4 * n] = t.nodes[n].size; node_d4[4 * n + 1] = t.nodes[n].mass;
        node_d4[4 * n + 2] = t.nodes[n].mx; node_d4[4 * n + 3] = t.nodes[n].my;
    }
    for (int32_t c = 0; c < t.nchildren; ++c) child[c] = t.child[c];
    int32_t nn = t.nnodes;
    orc_qt_free(&t);
    return nn;
}

/* Net force F(x) = repulsion + attraction + gravity (F is overwritten).
 * exact != 0: O(K^2) repulsion; else Barnes-Hut with opening parameter theta. */
void orc_fa2_forces(int32_t K, const double *x, const double *mass, int64_t E, const int32_t *se,
                    const double *aw, double kr, double kg, int32_t exact, double theta, double *F)
{
    for (int32_t i = 0; i < 2 * K; ++i) F[i] = 0.0;
    if (exact) orc_repulse_exact(K, x, mass, kr, F);
    else orc_repulse_bh(K, x, mass, kr, theta, F);
    orc_attract_gravity(K, x, mass, E, se, aw, kg, F);
}

/*
 * ForceAtlas2 iterations.  state: Fprev[2K] (force of the previous iteration, zero
 * at the start) and speed[1] (global speed, 1 at the start, Algorithm 1).  Per
 * iteration:
 *   swing_i = |F_i - F'_i|, traction_i = |F_i + F'_i| / 2,
 *   S = sum m_i swing_i, T = sum m_i traction_i,
 *   global speed s = min(tau * T / S, 1.5 * s) when S > 0 (unchanged otherwise),
 *   local speed s_i = ks * s / (1 + s * sqrt(swing_i)), capped so s_i |F_i| <= ksmax,
 *   x_i += s_i F_i, F' = F.
 */
void orc_fa2_layout(int32_t K, int64_t E, const int32_t *se, const double *aw, const double *mass,
                    double *x, double *Fprev, double *speed, int32_t iters, int32_t exact,
                    double theta, double kr, double kg, double tau, double ks, double ksmax)
{
    double *F = (double *)malloc(sizeof(double) * 2 * (size_t)(K > 0 ? K : 1));
    double *sw = (double *)malloc(sizeof(double) * (size_t)(K > 0 ? K : 1));
    for (int32_t it = 0; it < iters; ++it) {
        orc_fa2_forces(K, x, mass, E, se, aw, kr, kg, exact, theta, F);
        double S = 0.0, T = 0.0;
        for (int32_t i = 0; i < K; ++i) {
            const double ax = F[2 * i] - Fprev[2 * i], ay = F[2 * i + 1] - Fprev[2 * i + 1];
            const double bx = F[2 * i] + Fprev[2 * i], by = F[2 * i + 1] + Fprev[2 * i + 1];
            sw[i] = sqrt(ax * ax + ay * ay);
            S += mass[i] * sw[i];
            T += mass[i] * 0.5 * sqrt(bx * bx + by * by);
        }
        if (S > 0.0) {
            const double target = tau * T / S, cap = 1.5 * speed[0];
            speed[0] = target < cap ? target : cap;
        }
        const double s = speed[0];
        for (int32_t i = 0; i < K; ++i) {
            double si = ks * s / (1.0 + s * sqrt(sw[i]));
            const double fn = sqrt(F[2 * i] * F[2 * i] + F[2 * i + 1] * F[2 * i + 1]);
            if (fn > 0.0 && si > ksmax / fn) si = ksmax / fn;
            x[2 * i] += si * F[2 * i];
            x[2 * i + 1] += si * F[2 * i + 1];
            Fprev[2 * i] = F[2 * i];
            Fprev[2 * i + 1] = F[2 * i + 1];
        }
    }
    free(F); free(sw);
}

/* ------------------------------------------------------------------------------ */
/* ForceAtlas2 energy: its negative gradient is the force field above              */
/*   E = sum_e a_e d_e^2 / 2 - kr sum_{i<j, d>0} m_i m_j ln d_ij + kg sum_i m_i |x_i| */
/* ------------------------------------------------------------------------------ */
double orc_fa2_energy(int32_t K, const double *x, const double *mass, int64_t E, const int32_t *se,
                      const double *aw, double kr, double kg)
{
    double e_att = 0.0, e_rep = 0.0, e_grav = 0.0;
    for (int64_t e = 0; e < E; ++e) {
        const int32_t i = se[2 * e], j = se[2 * e + 1];
        const double a = aw ? aw[e] : 1.0;
        const double dx = x[2 * i] - x[2 * j], dy = x[2 * i + 1] - x[2 * j + 1];
        e_att += 0.5 * a * (dx * dx + dy * dy);
    }
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : e_rep)
    for (int32_t i = 0; i < K; ++i) {
        double acc = 0.0;
        for (int32_t j = i + 1; j < K; ++j) {
            const double dx = x[2 * i] - x[2 * j], dy = x[2 * i + 1] - x[2 * j + 1];
            const double d2 = dx * dx + dy * dy;
            if (d2 > 0.0) acc += mass[i] * mass[j] * 0.5 * log(d2);
        }
        e_rep += acc;
    }
    for (int32_t i = 0; i < K; ++i)
        e_grav += mass[i] * sqrt(x[2 * i] * x[2 * i] + x[2 * i + 1] * x[2 * i + 1]);
    return e_att - kr * e_rep + kg * e_grav;
}

/* The terms of E that involve node i (for finite differences in x_i). */
double orc_fa2_node_energy(int32_t K, const double *x, const double *mass, int64_t E,
                           const int32_t *se, const double *aw, double kr, double kg, int32_t i)
{
    double acc = 0.0;
    for (int64_t e = 0; e < E; ++e) {
        const int32_t a0 = se[2 * e], b0 = se[2 * e + 1];
        if (a0 != i && b0 != i) continue;
        const double a = aw ? aw[e] : 1.0;
        const double dx = x[2 * a0] - x[2 * b0], dy = x[2 * a0 + 1] - x[2 * b0 + 1];
        acc += 0.5 * a * (dx * dx + dy * dy);
    }
    for (int32_t j = 0; j < K; ++j) {
        if (j == i) continue;
        const double dx = x[2 * i] - x[2 * j], dy = x[2 * i + 1] - x[2 * j + 1];
        const double d2 = dx * dx + dy * dy;
        if (d2 > 0.0) acc -= kr * mass[i] * mass[j] * 0.5 * log(d2);
    }
    acc += kg * mass[i] * sqrt(x[2 * i] * x[2 * i] + x[2 * i + 1] * x[2 * i + 1]);
    return acc;
}
