/*
 * bgv.h -- C ABI of the MI355X (gfx950) BigGraphVis hot path.
 *
 * The library implements the data-parallel core of BigGraphVis (Moradi & Mondal,
 * arXiv 2108.00529): an edge list goes in; community labels, a count-min-sketch
 * weighted supergraph and 2-D ForceAtlas2 positions of that supergraph come out
 * (Algorithm 3 and Section 4.1).  Every step runs in hand-written HIP kernels.
 *
 * Conventions shared by every entry point
 *   - Pointers marked "dev" are device memory (hipMalloc'd, e.g. a torch tensor's
 *     data_ptr()); pointers marked "host" are host memory.  Every buffer is owned by
 *     the caller and is never freed or reallocated by the library.
 *   - Scratch memory comes only from the caller's workspace `ws` (dev), at least the
 *     size returned by the matching *_workspace() query, 256-byte aligned, except for
 *     bgv_fa2_layout_static, which uses a fixed device array of the library.  The
 *     library itself never calls hipMalloc.
 *   - Work is enqueued on `stream` and is asynchronous, except where an entry point
 *     says it synchronises.  Calls on distinct streams need distinct workspaces.
 *   - Arguments are validated on the host before any HIP call; a rejected call
 *     touches no device memory.  No C++ exception crosses this boundary.
 *   - Integer results are identical for every launch configuration; floating-point
 *     results are identical run to run (fixed reduction orders, no FP atomics).
 *   - Edge lists are int32 (m, 2) row-major: edge i is (edges[2i], edges[2i+1]), and
 *     i is its position in the stream.  Node ids must lie in [0, n).
 *   - Ids are not checked on the device by default: an id outside its range makes the
 *     kernels read and write outside the caller's arrays.  With the environment
 *     variable BGV_CHECK=1, every entry point that takes ids first scans them with a
 *     read-only kernel (edges, and labels for bgv_supergraph; superedge ids against K;
 *     the batched form's offsets, local ids and order), synchronises its stream, and
 *     returns BGV_E_RANGE before any kernel indexes by them.  bgv_validate_edges runs
 *     the same scan on request.
 */
#ifndef BGV_H
#define BGV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *bgv_stream_t; /* a hipStream_t; NULL = the null stream */

typedef int32_t bgv_status;
#define BGV_OK 0
#define BGV_E_INVALID (-1)     /* an argument is out of its documented range      */
#define BGV_E_RANGE (-2)       /* an id lies outside its range (device check)     */
#define BGV_E_WORKSPACE (-3)   /* ws is NULL, misaligned or smaller than required */
#define BGV_E_HIP (-4)         /* a HIP call failed; see bgv_last_error()          */

/* Human-readable name of a status code (static storage). */
const char *bgv_status_string(bgv_status s);
/* Message of the last failing call on this host thread ("" if none). */
const char *bgv_last_error(void);

/* ---------------------------------------------------------------------------- */
/* Streaming community detection                                                 */
/* ---------------------------------------------------------------------------- */
/*
 * Paper: Section 3.2 (the streaming rule), Section 3.2.1 and Algorithm 3 (parallel
 * passes with a growing threshold).  Every streamed edge raises the degree counter
 * of both endpoints; when both counters are at most the pass threshold, the endpoint
 * with the smaller counter joins the community of the other; equal counters do
 * nothing; self-loops are ignored.  Counters accumulate over passes (Algorithm 3
 * initialises them once).  Pass p (0-based) uses threshold D1 * growth^p, saturating
 * at INT32_MAX.
 *
 * Parallel semantics (batch-synchronous): each pass is cut into chunks of `chunk`
 * consecutive edges.  Within a chunk all counter increments happen first; then every
 * edge decides with the chunk-end counters and the labels as they stood when the
 * chunk began; a node proposed to by several edges takes the label from the edge of
 * smallest stream index.  chunk = 1 is the sequential rule; `chunk` is part of the
 * result's definition, not a tuning knob.
 *
 * Two methods compute these same integers.  Chunk by chunk (method 1): two launches
 * per chunk and pass.  Back-pointer resolution (method 2): decisions depend only on
 * counters, which follow in closed form from the stream, so every pass's proposals are
 * formed at once; a chunk's winner for a target is its proposal of smallest stream
 * index, and the label it carries is the one its source got from its own latest winner
 * in an earlier chunk; pointer jumping over those links resolves all labels in about
 * 20 + log2(passes * chunks) launches, whatever the chunk size (chunk = 1 included).
 * Method 2 needs m >= 1 and passes * m < 2^31 (method 2 otherwise: BGV_E_INVALID) and
 * more workspace.
 *
 * rule = 1 (the volume rule of SCoDA, the streaming algorithm Section 3.2 adopts), in
 * the same batch-synchronous form: V[c] = the sum of the counters of the nodes labelled
 * c (increments raise the V of the chunk-start label; a move carries the node's counter
 * from its old community's V to the new one's).  An edge whose counters are both at most
 * the threshold and whose endpoints' chunk-start labels differ proposes: the endpoint
 * whose community has the smaller or equal V joins the other's; endpoints that share a
 * label propose nothing.  Decisions then depend on labels, so rule 1 runs chunk by chunk
 * on per-node records with device atomics (method 0 or 1; tie must be 0); its
 * workspace is 24 bytes per node and 4 per edge of a chunk.  Method 0 picks 2 when it applies and the chunk-by-chunk form would
 * take more than 16 + passes * m / 2^17 chunk steps, else 1.  Other values are
 * BGV_E_INVALID.
 */
typedef struct {
    int32_t threshold; /* D1 >= 0: threshold of the first pass                   */
    int32_t passes;    /* P >= 1                                                 */
    int32_t growth;    /* >= 1: threshold factor between passes                   */
    int32_t method;    /* 0 automatic, 1 chunk by chunk, 2 back-pointer resolution */
    int64_t chunk;     /* >= 1: edges per synchronous chunk                        */
    int32_t tie;       /* 0: equal counters do nothing (Algorithm 3's nested tests);
                          1: the edge's first endpoint joins the second's community  */
    int32_t rule;      /* 0: the degree rule above (the paper);
                          1: SCoDA's community-volume rule (see below)             */
} bgv_cd_params;

/* Workspace bytes for bgv_community (0 only on invalid arguments).  Up to 2^24 nodes:
 * 8 bytes per node and, per 2048-edge tile of a chunk, 32 KiB of grouped proposals and
 * endpoints plus two offset rows of 4 * (ceil(n / 4096) + 1) bytes.  Above: 16 bytes per
 * node and 4 per edge of a chunk.  With passes > 1 another 8 per edge (each edge's
 * pass-0 endpoint counters, from which later passes' counters follow without
 * increments), and up to 2^24 nodes with passes > 2 one more byte per edge (passes 2-5
 * decided once the degrees are known).  Method 2: 48 bytes per edge, 8 per node and at most 48 per (pass, edge)
 * proposal, plus radix-sort scratch. */
size_t bgv_community_workspace(int32_t n, int64_t m, const bgv_cd_params *p);

/*
 * n in [1, 2^31-1]; m in [0, 2^31-1]; edges: dev int32 (m,2), ids in [0,n).
 * Outputs (dev): labels int32[n] (community label = id of a node, the node's own id
 * if it never joined), degree int32[n] (true degree: occurrences as an endpoint of a
 * non-loop edge), volume int64[n] or NULL (volume[c] = sum of degree over nodes with
 * label c; the exact weight the sketch estimates).  Ids outside [0, n) are undefined
 * behaviour unless BGV_CHECK=1 (then BGV_E_RANGE, see the conventions above).
 */
bgv_status bgv_community(int32_t n, int64_t m, const int32_t *edges, const bgv_cd_params *p,
                         int32_t *labels, int32_t *degree, int64_t *volume,
                         void *ws, size_t ws_bytes, bgv_stream_t stream);

/*
 * Paper: Section 3.2.1 (the passes of Algorithm 3, read as hierarchical community
 * detection), Sections 5.3.3 and 5.3.5 (each pass's communities are kept as one level
 * of the hierarchy, through which a supernode's members are reached).  Same arguments,
 * workspace and outputs as bgv_community, plus pass_labels: dev int32[passes][n], row p = the labels after pass
 * p (0-based), equal to the labels of bgv_community run with passes = p + 1; the last
 * row equals `labels`.  pass_labels NULL is BGV_E_INVALID.  With m = 0 every row holds
 * each node's own id.
 */
bgv_status bgv_community_passes(int32_t n, int64_t m, const int32_t *edges, const bgv_cd_params *p,
                                int32_t *labels, int32_t *degree, int64_t *volume,
                                int32_t *pass_labels, void *ws, size_t ws_bytes,
                                bgv_stream_t stream);

/*
 * Paper: Section 3.2.1 and Algorithm 3 (the rounds share one state: each node's label
 * and degree counter, initialised once before the first round).  Continues a run of
 * bgv_community that stopped after `done` passes, 1 <= done < p->passes: same n, m,
 * edges and parameters; labels_in (dev int32[n], ids in [0, n)) holds that run's labels
 * after its `done` passes (e.g. row done-1 of bgv_community_passes, or the labels of
 * bgv_community with passes = done).  Runs passes done .. passes-1 and returns exactly
 * what bgv_community with p->passes returns (labels, degree, volume).  The counters at
 * that point are done * d(v) and d(v) follows from the stream, so labels and `done`
 * are the whole state; the degrees are recounted from the edges (one counting sweep).
 * labels_in must not overlap labels.  Workspace: bgv_community_workspace(n, m, p).
 * Invalid done, a null or aliased labels_in: BGV_E_INVALID.  With BGV_CHECK=1,
 * labels_in is range-checked too (BGV_E_RANGE).
 */
bgv_status bgv_community_resume(int32_t n, int64_t m, const int32_t *edges, const bgv_cd_params *p,
                                int32_t done, const int32_t *labels_in, int32_t *labels, int32_t *degree,
                                int64_t *volume, void *ws, size_t ws_bytes, bgv_stream_t stream);

/* ---------------------------------------------------------------------------- */
/* Count-min-sketch supergraph                                                  */
/* ---------------------------------------------------------------------------- */
/*
 * Paper: Section 3.3 and Algorithm 2 (count-min sketch: r rows of c counters, one
 * pairwise-independent hash per row, estimate = minimum over the rows),
 * Section 4.1 (supernode weight: each node v adds its degree to row i at column
 * hash_i(com(v))), Algorithm 3 (the supergraph handed to ForceAtlas2).
 *
 * Supernodes are the distinct labels, numbered by ascending label (sid).  Sketch 1
 * estimates each supernode's weight (sum of its nodes' degrees).  Sketch 2 counts
 * inter-community edges: every non-loop edge with labels a != b adds 1 at the key
 * (min(a,b), max(a,b)).  Superedges are the distinct such keys as (sid_lo, sid_hi)
 * pairs, sid_lo < sid_hi, sorted ascending; their weight is the sketch-2 estimate.
 *
 * Hash of row r with coefficients (A, B, C) (64-bit, arithmetic mod 2^64):
 *   key x:        t = A*x + B;          column = ((t >> 32) * cols) >> 32
 *   pair (a < b): t = A*a + C*b + B;    column = ((t >> 32) * cols) >> 32
 * The coefficients are the random draws of the hash family and are inputs.
 */
typedef struct {
    int32_t rows;          /* 1..8                                                  */
    int32_t cols;          /* 1..2^31-1                                             */
    const uint64_t *coef1; /* host, rows*3 values (A,B,C per row) for sketch 1      */
    const uint64_t *coef2; /* host, rows*3 values for sketch 2                      */
} bgv_sketch_params;

size_t bgv_supergraph_workspace(int32_t n, int64_t m, const bgv_sketch_params *s);

/*
 * Inputs (dev): edges (m,2), labels int32[n] and degree int32[n] from bgv_community.
 * Outputs: K (host int32) supernodes and E_S (host int64) superedges;
 *   super_label  dev int32[cap n]    label of supernode sid (ascending)
 *   super_size   dev uint32[cap n]   sketch-1 estimate of the supernode weight
 *   node_super   dev int32[n] or NULL   sid of each node's community
 *   superedges   dev int32[cap m][2] (sid_lo, sid_hi), sorted
 *   se_weight    dev uint32[cap m]   sketch-2 estimate of the superedge multiplicity
 *   se_count     dev uint32[cap m] or NULL   exact multiplicity (number of edges)
 *   M1, M2       dev uint32[rows][cols] the two sketches (required)
 * Synchronises `stream` (K and E_S are returned on the host): twice, each time by
 * polling an event with the calling thread (which stays busy until the work queued
 * before it has run) rather than sleeping on it.
 */
bgv_status bgv_supergraph(int32_t n, int64_t m, const int32_t *edges, const int32_t *labels,
                          const int32_t *degree, const bgv_sketch_params *s,
                          int32_t *K, int64_t *E_S, int32_t *super_label, uint32_t *super_size,
                          int32_t *node_super, int32_t *superedges, uint32_t *se_weight,
                          uint32_t *se_count, uint32_t *M1, uint32_t *M2,
                          void *ws, size_t ws_bytes, bgv_stream_t stream);

/* ---------------------------------------------------------------------------- */
/* ForceAtlas2 layout                                                            */
/* ---------------------------------------------------------------------------- */
/*
 * Paper: Section 3.1 and Algorithm 1 (gravity, Barnes-Hut repulsion, attraction,
 * swing-based speeds, displacement), in the force and speed laws of the cited
 * ForceAtlas2 publication.  For node i with mass m_i:
 *   repulsion  kr m_i m_j (x_i - x_j) / |x_i - x_j|^2   from every j != i (0 if coincident)
 *   attraction a_e (x_j - x_i)                          along every edge e = (i, j)
 *   gravity    -kg m_i x_i / |x_i|                      (0 at the origin)
 * Per iteration, with F' the previous force (zero initially) and s the global speed
 * (1 initially): swing_i = |F_i - F'_i|, traction_i = |F_i + F'_i| / 2;
 * s = min(tau * sum m_i traction_i / sum m_i swing_i, 1.5 s) when the swing sum is
 * positive; s_i = ks s / (1 + s sqrt(swing_i)), at most ksmax / |F_i|;
 * x_i += s_i F_i; F' = F.
 * Barnes-Hut (exact = 0), Section 3.1's hierarchical partition: bodies are quantised
 * in FP32 to a 2^16 x 2^16 grid over their bounding square (side s0 = the larger
 * extent, 1 if zero); the tree is the compressed quadtree of the grid points: each
 * node is the smallest cell (side s0 / 2^depth) that holds its bodies, whose bodies
 * occupy at least two of its quadrants; bodies on one grid point form one leaf.  A
 * node not containing i is replaced by its centre of mass when
 * size^2 < theta^2 * dist^2, else opened; leaves are summed body by body.
 */
typedef struct {
    int32_t iters; /* >= 0                                                        */
    int32_t exact; /* 1: all-pairs repulsion; 0: Barnes-Hut                        */
    float theta;   /* Barnes-Hut opening parameter (>= 0)                          */
    float kr;      /* repulsion constant                                           */
    float kg;      /* gravity constant                                             */
    float tau;     /* swing tolerance of the global speed                          */
    float ks;      /* local speed constant                                         */
    float ksmax;   /* cap of the displacement length                               */
} bgv_fa2_params;

size_t bgv_fa2_workspace(int32_t K, int64_t E, const bgv_fa2_params *p);

/*
 * K >= 1 nodes, E >= 0 undirected edges (dev int32 (E,2), ids in [0,K), no self-loops;
 * repeated pairs count repeatedly).  attr_w dev float[E] (a_e) or NULL (a_e = 1);
 * mass dev float[K] or NULL (m_i = number of incident edges + 1).
 * In/out (dev): pos float (K,2); fprev float (K,2) (zeros for a fresh start);
 * speed float[1] (1.0 for a fresh start).  Passing the state back in continues the
 * run exactly where it stopped.
 */
bgv_status bgv_fa2_layout(int32_t K, int64_t E, const int32_t *edges, const float *attr_w,
                          const float *mass, float *pos, float *fprev, float *speed,
                          const bgv_fa2_params *p, void *ws, size_t ws_bytes, bgv_stream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, hosts that forbid hipMalloc): bgv_fa2_layout with the same arguments
 * (less the workspace), kernels and results.  Scratch comes from a device array of
 * BGV_FA2_STATIC_SCRATCH_BYTES (64 MiB) inside the library, one copy per GPU, held
 * until the process ends; the call itself allocates nothing.  A call whose
 * bgv_fa2_workspace(K, E, p) exceeds that size returns BGV_E_INVALID and touches no
 * device memory (Barnes-Hut: K = 16,384 fits up to about 980,000 edges, K = 65,536 up
 * to about 720,000, K = 131,072 up to about 280,000; exact: K = 16,384 up to about
 * 960,000 edges, K = 65,536 never).
 * Every call on one GPU shares that GPU's array: calls that overlap in time on one GPU
 * (different streams, or host threads without an order between them) race and give
 * undefined results; calls queued on one stream are ordered.  The array keeps the last
 * call's contents; each call initialises what it reads.  The first call on each device
 * looks up the array's address (hipGetSymbolAddress, not a stream operation).
 */
#define BGV_FA2_STATIC_SCRATCH_BYTES (64u << 20)
bgv_status bgv_fa2_layout_static(int32_t K, int64_t E, const int32_t *edges, const float *attr_w,
                                 const float *mass, float *pos, float *fprev, float *speed,
                                 const bgv_fa2_params *p, bgv_stream_t stream);

/*
 * ForceAtlas2 energy, whose negative gradient is the force field above (exact
 * repulsion):  E = sum_e a_e |x_i - x_j|^2 / 2 - kr sum_{i<j} m_i m_j ln|x_i - x_j|
 *                  + kg sum_i m_i |x_i|    (coincident pairs contribute 0).
 * energy: dev double[1].  Pair terms in FP32, partial sums combined in FP64 in a
 * fixed order.
 */
size_t bgv_fa2_energy_workspace(int32_t K, int64_t E);
bgv_status bgv_fa2_energy(int32_t K, int64_t E, const int32_t *edges, const float *attr_w,
                          const float *mass, const float *pos, float kr, float kg, double *energy,
                          void *ws, size_t ws_bytes, bgv_stream_t stream);

/*
 * Gradient of that energy: grad = -F(pos) * g, with g = *grad_out (dev float[1]) or
 * 1 when grad_out is NULL.  grad: dev float (K,2).  Same workspace as the energy.
 */
bgv_status bgv_fa2_grad(int32_t K, int64_t E, const int32_t *edges, const float *attr_w,
                        const float *mass, const float *pos, float kr, float kg,
                        const float *grad_out, float *grad,
                        void *ws, size_t ws_bytes, bgv_stream_t stream);

/* ---------------------------------------------------------------------------- */
/* Batched form: many independent graphs in one persistent launch                 */
/* ---------------------------------------------------------------------------- */
/*
 * The whole path above (community passes, count-min supergraph, exact ForceAtlas2) for
 * G graphs at once; graph g is processed by one workgroup from start to end (but see
 * big_k), graphs are taken from a queue in `order` (e.g. largest first; NULL = 0..G-1).  Per graph the
 * results equal those of bgv_community + bgv_supergraph + bgv_fa2_layout (exact
 * repulsion, attraction weights 1, masses = degree + 1), with the same parameters.
 *
 * Graph g owns nodes [node_off[g], node_off[g+1]) and edges [edge_off[g], edge_off[g+1])
 * of the concatenated arrays (node_off, edge_off: dev int64[G+1], non-decreasing,
 * node_off[G] = n_total, edge_off[G] = m_total); its edges use local ids in
 * [0, n_g).  Sketch shape: rows * cols <= 8192 (each graph's sketches live in LDS).
 * cd: the degree rule only (cd->rule 0; cd->tie 0 or 1), cd->method 0 (each workgroup
 * runs its graph chunk by chunk).  fa->exact must be 1.  wg_threads: 256, 512 or 1024 (0 = 512), a launch parameter that
 * does not change any result.  big_k >= 0, another such parameter: a graph whose
 * supergraph has more than big_k nodes (and at most 4096) is laid out after the
 * persistent launch by kernels that spread each graph's tiles and repulsion segments
 * over many workgroups (a fixed sequence of three launches per iteration, sizes read on
 * the device), so that
 * a few large graphs do not each hold one compute unit for the whole layout; 0 keeps
 * every layout in the persistent launch.
 * Outputs (dev; per-node arrays indexed from node_off[g], per-edge arrays from
 * edge_off[g]): labels, degree int32[n_total]; K, E_S int32[G]; super_label int32 and
 * super_size uint32 [n_total] (first K[g] entries of each graph); superedges int32
 * (m_total, 2) and se_weight uint32[m_total] (first E_S[g] of each graph).
 * In/out: pos, fprev float (n_total, 2) -- each graph's first K[g] rows are the layout
 * (initial positions in, final out; fprev zeros for a fresh start); speed float[G]
 * (1.0 for a fresh start).
 */
size_t bgv_batched_workspace(int32_t G, int64_t n_total, int64_t m_total);
bgv_status bgv_batched(int32_t G, int64_t n_total, int64_t m_total, const int64_t *node_off,
                       const int64_t *edge_off, const int32_t *order, const int32_t *edges,
                       const bgv_cd_params *cd, const bgv_sketch_params *sk, const bgv_fa2_params *fa,
                       int32_t wg_threads, int32_t big_k, int32_t *labels, int32_t *degree, int32_t *K, int32_t *E_S,
                       int32_t *super_label, uint32_t *super_size, int32_t *superedges,
                       uint32_t *se_weight, float *pos, float *fprev, float *speed,
                       void *ws, size_t ws_bytes, bgv_stream_t stream);

/* ---------------------------------------------------------------------------- */
/* Drawing attributes of the supernodes                                          */
/* ---------------------------------------------------------------------------- */
/*
 * Paper: Section 4.1 (a supernode is drawn with a radius proportional to the square
 * root of its size) and Section 4.3 (eleven colour groups by community size).
 * alpha = sum of the sizes; supernodes are ranked by size, small first (equal sizes by
 * supernode id); one whose running total P (itself included) has 2P <= alpha is in
 * group 0 (the smallest communities holding at most half of alpha), any other in group
 * ceil(10 * (2P - alpha) / alpha), 1..10 (the remaining half cut into ten equal
 * shares: the paper leaves the cut open).  All integer arithmetic.
 * Inputs (dev): super_size uint32[K], e.g. the sketch-1 estimates from bgv_supergraph.
 * Outputs (dev): group int32[K] in 0..10; radius float[K] = sqrt(size), correctly
 * rounded (the caller scales it).  K >= 1; asynchronous on `stream`.
 */
size_t bgv_draw_workspace(int32_t K);
bgv_status bgv_draw_supernodes(int32_t K, const uint32_t *super_size, int32_t *group, float *radius,
                               void *ws, size_t ws_bytes, bgv_stream_t stream);

/* ---------------------------------------------------------------------------- */
/* Checks and diagnostics                                                        */
/* ---------------------------------------------------------------------------- */
/*
 * The id range check of the conventions above, on request: scans the m edges (dev
 * int32 (m,2)) for an id outside [0, n), with flag (dev int32[1], caller-owned) as
 * its device result (1 if any, else 0).  Synchronises `stream`; returns BGV_E_RANGE
 * if an id is out of range, BGV_OK if none, BGV_E_INVALID for n < 1, m < 0 or
 * m >= 2^31 or a null pointer.  Reads the edges only.
 */
bgv_status bgv_validate_edges(int32_t n, int64_t m, const int32_t *edges, int32_t *flag, bgv_stream_t stream);

/*
 * The Barnes-Hut tree that one ForceAtlas2 iteration builds for positions pos
 * (dev float (K,2)) and masses mass (dev float[K]), copied out for inspection.  The
 * device form is the binary radix tree of the sorted codes, which refines the
 * compressed quadtree above: its internal node j (0 <= j < K-1) covers sorted bodies
 * [first, last]; a node whose codes share a 2d-bit prefix (and differ in the next bit)
 * is the quadtree node of depth d; a node with a (2d+1)-bit prefix is one too unless
 * its parent has the 2d-bit prefix, in which case it is half of the parent's cell and
 * is always opened.  Outputs (dev): codes uint32[K] (Morton codes in sorted order: x
 * bits at even positions, ties by body index), body float (K,4) (x, y, mass, body
 * index as int32 bits, sorted), s0 float[1] (side of the root square), and for K > 1
 * nodeA float (K-1,4) (centre of mass x, y, mass, size^2; size^2 < 0 for a node whose
 * codes are all equal, a leaf summed body by body; +inf for a half cell) and nodeB
 * int32 (K-1,4) (left, right, first, last; a child c < 0 is the single body at sorted
 * position ~c).  Workspace from bgv_bh_tree_workspace(K).  K >= 1; asynchronous.
 */
size_t bgv_bh_tree_workspace(int32_t K);
bgv_status bgv_bh_tree(int32_t K, const float *pos, const float *mass, uint32_t *codes, float *body,
                       float *nodeA, int32_t *nodeB, float *s0, void *ws, size_t ws_bytes,
                       bgv_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* BGV_H */
