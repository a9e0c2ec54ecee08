/*
 * vr.h -- C ABI of the MI355X (gfx950) Vietoris-Rips filtration front end.
 *
 * One call builds the filtered Vietoris-Rips complex of a point cloud up to
 * dimension 2 on the GPU: exact squared distances of all pairs, the integer
 * rank of every edge, the threshold, every solid triangle valued at its
 * largest edge rank, and all simplices in filtration order.
 *
 * The problem statement follows arXiv:1809.04424:
 *   - Section 3 (the eirene call): a point cloud whose rows are points (or a
 *     symmetric dissimilarity matrix, dtype VR_DIST) plus an upper distance
 *     limit in,
 *     an integer rank matrix ("symmat") and integer filtration values out;
 *   - Section 2.1: an edge joins two points closer than the threshold, a
 *     solid triangle exists once its three edges exist;
 *   - Section 4.5: edge ranks are the sortperm of the distances;
 *   - Section 4.4: the library is reached through plain extern "C" host
 *     functions taking pointers and lengths.
 *
 * Conventions
 *   - Every index is 0-based (the paper's Julia is 1-based).
 *   - Squared distance q_ij = sum_c (x_ic - x_jc)^2, exact in integers; it
 *     orders edges exactly as the distance does.
 *   - Edge order: ascending (q, i, j) with i < j.  The rank r of an edge is
 *     its 0-based position in that order; ranks are unique, so every output
 *     is unique and bit-exact comparison is well defined.
 *   - Kept edges are the ranks r < K.  Vertices have filtration value -1 (they
 *     precede every edge); edge r has value r; a triangle has the value of its
 *     largest edge.  The whole filtration is ordered by (value, dimension,
 *     vertex tuple), so faces precede cofaces.
 *   - Device pointers are HIP device memory of the current device.
 *
 * Thread safety: calls on different streams (and different results) may run
 * concurrently from different host threads.
 */
#ifndef VR_H
#define VR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define VR_API __attribute__((visibility("default")))
#else
#define VR_API
#endif

/* Status codes.  Every entry point that can fail returns one of these. */
typedef enum {
    VR_OK = 0,
    VR_EINVAL = -1, /* bad argument: null pointer, d < 1, unknown dtype/kind, bad threshold */
    VR_ENOMEM = -2, /* a device allocation failed (nothing is leaked) */
    VR_E2BIG = -3,  /* n > VR_MAX_POINTS or K > VR_MAX_EDGES: outside the key packing */
    VR_EHIP = -4,   /* a HIP runtime call failed */
    VR_ERANGE = -5  /* some squared distance does not fit in 32 bits unsigned (or a VR_DIST entry is negative) */
} vr_status;

/* Coordinate types (signed integers).  VR_DIST: `points` is instead an
 * n x n row-major int32 matrix of non-negative dissimilarities (d = n, or 1
 * when n = 0); entry [i][j], i < j, is the pair's squared distance q (the
 * paper accepts a symmetric distance matrix in place of points, Section 3);
 * entries on and below the diagonal are not read, and a negative entry
 * fails the build with VR_ERANGE. */
enum { VR_I8 = 1, VR_I16 = 2, VR_I32 = 3, VR_DIST = 4 };

/* Threshold kinds (the paper's upper limit, Section 3; infinite by default,
 * Section 5).  E = n(n-1)/2 is the number of vertex pairs.
 *   VR_THR_FULL     : K = E (every pair is an edge)
 *   VR_THR_COUNT    : K = thr_num, 0 <= thr_num <= E
 *   VR_THR_FRACTION : K = floor(thr_num * E / thr_den), 0 <= thr_num <= thr_den, thr_den > 0
 *                     (the p-th percentile of edge ranks is thr_num/thr_den = p/100)
 *   VR_THR_SQDIST   : keep q < thr_num (strict: "closer than"), K = #{q < thr_num} */
enum { VR_THR_FULL = 0, VR_THR_COUNT = 1, VR_THR_FRACTION = 2, VR_THR_SQDIST = 3 };

/* Request flags. */
enum {
    VR_COUNT_ONLY = 1u,  /* compute (n, K, T) and the edges; do not write triangles */
    VR_TIMING = 2u,      /* record HIP events between all stages (see vr_query_stage_ms) */
    VR_TIMING_WRITE = 4u, /* record HIP events around the triangle write only */
    VR_GRAPH = 8u         /* capture the first phase into a hipGraph and replay it (see vr_build) */
};

/* Limits of the packed triangle key: 13 bits per vertex, 24 bits of value. */
#define VR_MAX_POINTS 8192
#define VR_MAX_EDGES (1 << 24)

/* Optional device allocator, e.g. a framework's caching allocator.
 * alloc returns device memory usable on `stream` (NULL on failure); free
 * releases it in stream order.  With no allocator the library uses its own
 * stream-ordered cache (see vr_trim). */
typedef struct vr_allocator {
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void (*free)(void *ptr, size_t bytes, void *stream, void *ctx);
    void *ctx;
} vr_allocator;

/* One build request.  `points` is borrowed for the duration of vr_build only. */
typedef struct vr_request {
    const void *points; /* device pointer, row-major n x d, dtype coordinates (rows are points) */
    int64_t n, d;       /* 0 <= n <= VR_MAX_POINTS, d >= 1 */
    int32_t dtype;      /* VR_I8, VR_I16, VR_I32, or VR_DIST (a dissimilarity matrix) */
    int32_t thr_kind;   /* VR_THR_* */
    int64_t thr_num, thr_den;
    int32_t maxdim;     /* 0: vertices only, 1: up to edges, 2: up to triangles,
                           3: also tetrahedra (vr_build only) */
    uint32_t flags;     /* VR_COUNT_ONLY | VR_TIMING | VR_TIMING_WRITE */
    const vr_allocator *alloc; /* NULL: the library's stream-ordered cache */
} vr_request;

/* Result handle, owned by the library until vr_free.  Fields are read-only. */
typedef struct vr_result {
    int64_t n_vertices;  /* n */
    int64_t n_edges;     /* K */
    int64_t n_triangles; /* T */
    /* device, 2*K: edge r joins edge_ij[2r] < edge_ij[2r+1]; rank order */
    const uint32_t *edge_ij;
    /* device, K: squared length of edge r (non-decreasing in r) */
    const int64_t *edge_q;
    /* device, T: triangle keys v<<39 | i<<26 | j<<13 | k, i<j<k, v = largest
     * edge rank; ascending, which is filtration order (NULL with VR_COUNT_ONLY) */
    const uint64_t *tri_key;
    /* maxdim 3 only (else 0 and NULL): the tetrahedra, T3 of them, in
     * filtration order (by value, the largest edge rank, then by vertices).
     * tet_off: device, K + 1: tet_off[r] = the first tetrahedron of value r,
     * tet_off[K] = T3.  tet_key: device, 2 T3: tetrahedron t has value
     * tet_key[2t] and vertices tet_key[2t+1] = a<<39 | b<<26 | c<<13 | d,
     * a<b<c<d (NULL with VR_COUNT_ONLY). */
    int64_t n_tetrahedra;
    const int64_t *tet_off;
    const uint64_t *tet_key;
} vr_result;

/*
 * Build the filtration of one point cloud (Section 3: the eirene call takes
 * the points and an upper limit and returns the integer rank matrix and the
 * filtered simplices; Section 2.1: edges below the threshold, triangles once
 * their three edges exist, each valued at its largest edge rank; Section
 * 4.5: ranks are the sortperm of the distances).
 * req:    the request; its points are read during the call only.
 * stream: a hipStream_t (NULL = the null stream).
 * out:    receives a new handle, owned by the caller until vr_free.
 * Errors: VR_EINVAL (bad argument), VR_E2BIG (n or K beyond the key
 * packing), VR_ERANGE (a squared distance of 2^32 or more, or a negative
 * VR_DIST entry), VR_ENOMEM, VR_EHIP.
 * Enqueues all work on `stream` (a hipStream_t; NULL = the null stream) and
 * waits once for the first phase (distances up to triangle counts) to reach
 * the host through host-pinned memory, to size the outputs.  When a build
 * of the same shape (vertices, pairs, kept-edge bound, threshold kind) ran
 * before in the process, the triangle write is enqueued before that wait,
 * into outputs of the earlier build's sizes; it writes nothing if the counts
 * do not fit them, and the outputs are then sized from the counts.  The
 * handle's output block may so be larger than its arrays (up to the earlier
 * build's).  With VR_GRAPH, the first build of a request (same points
 * pointer, size, threshold, flags and schedule) on a host thread captures
 * the first phase's launches into a hipGraph, and later builds of that
 * request on the thread replay it with one launch; the points may change
 * in place between builds.  Each captured graph keeps its own workspace
 * (at most 4 per thread, least recently used dropped first; vr_trim drops
 * the calling thread's).  Not combined with VR_TIMING.  On VR_OK, *out
 * receives a new handle whose device arrays are complete once `stream`
 * reaches the end of this call's work (stream order).  On error *out is
 * not written and nothing is leaked.
 * maxdim 3 (dimension 3 of Section 3's bettimax = 2: tetrahedra, so that
 * classes of dimension 2 can die): after the triangles the tetrahedra are
 * counted per value, their offsets scanned and read back (a second wait),
 * and listed into a second output block, as by vr_tetra_offsets and
 * vr_tetra_write (not combined with VR_GRAPH).
 */
VR_API int vr_build(const vr_request *req, void *stream, vr_result **out);

/* Triangles of a result (or of a batch view) unpacked into T rows of four
 * int32 (i, j, k, v), i < j < k, v = the value (largest edge rank), in the
 * filtration order of tri_key.  `rows` is caller-owned device memory of
 * 16*T bytes; enqueued on `stream` after the build's work.  VR_EINVAL for a
 * null argument or a count-only result with triangles. */
VR_API int vr_unpack_triangles(const vr_result *res, int32_t *rows, void *stream);

/* counts[0..2] = (n, K, T): the vertices, kept edges and triangles of the
 * filtration, whose sum is the size of the complex the paper tabulates per
 * data set (Table 5).  Host only: no device call, no synchronisation.
 * VR_EINVAL for a null argument. */
VR_API int vr_query_counts(const vr_result *res, int64_t counts[3]);

/*
 * Per-stage GPU times (milliseconds) of a build made with VR_TIMING, in the
 * order of vr_stage_name(0..); with VR_TIMING_WRITE only the triangle write
 * stage is timed (the others read 0).  Waits for the build's last event.
 * Returns the number of stages written (<= cap), or a negative vr_status.
 */
VR_API int vr_query_stage_ms(const vr_result *res, float *ms, int cap);

/* Name of stage s (static string), or NULL past the last stage. */
VR_API const char *vr_stage_name(int s);

/* Releases the handle's device memory (the filtration of Section 3's output:
 * edges and triangles) in stream order on `stream`, then the handle; device
 * arrays read through the handle must be used before, in stream order.
 * NULL-safe; no error. */
VR_API void vr_free(vr_result *res, void *stream);

/* Device bytes a build of this shape needs at most, besides its outputs
 * (edges 16 B each, triangles 8 B each).  For admission by HBM footprint.
 * Returns -1 for shapes vr_build would reject. */
VR_API int64_t vr_workspace_bytes(int64_t n, int64_t d, int32_t dtype, int32_t thr_kind);

/*
 * Batched builds: many independent clouds in one launch sequence instead of
 * one sequence per cloud.  Like the column partition of Section 4.6, the
 * parts are computed independently and their output offsets are fixed up
 * afterwards; here a part is a cloud.
 *
 * A batch is `count` requests that share dtype, d, thr_kind, maxdim and flags
 * (VR_EINVAL otherwise) and take their allocator from reqs[0]; n, points and
 * the threshold values are per request.  Every kernel runs once over all
 * clouds: vertices, pairs and distance tiles are numbered across the batch,
 * and the edge sort key carries the cloud index above the squared distance,
 * so each cloud's result is bit-identical to its own vr_build.  The key must
 * fit 32 bits: bits(255^2 d) + bits(count-1) <= 32 for VR_I8, so VR_I16 and
 * VR_I32 batches hold one cloud each (VR_E2BIG otherwise; split the batch).
 * Other limits of the whole batch: fewer than 2^24 vertices, fewer than 2^30
 * pairs and 2^31 kept edges (VR_E2BIG).  Each request keeps the per-cloud
 * limits of vr_build.  Same stream semantics and error behaviour as vr_build.
 * maxdim 3 is vr_build's alone (VR_EINVAL here).
 */
typedef struct vr_batch vr_batch;

VR_API int vr_build_batch(const vr_request *reqs, int64_t count, void *stream, vr_batch **out);

/* View of request `index`: counts and device pointers into the batch's
 * output block (valid until vr_batch_free).  Host only.  VR_EINVAL for an
 * index outside [0, count). */
VR_API int vr_batch_result(const vr_batch *batch, int64_t index, vr_result *view);

/* Exact device workspace bytes vr_build_batch would allocate for these
 * requests (count = 1: vr_build), besides the outputs (edges 16 B each,
 * triangles 8 B each, each array 256-byte aligned).  Host only.  0 when no
 * request needs the device; a negative vr_status for requests the build
 * would reject. */
VR_API int64_t vr_batch_workspace_bytes(const vr_request *reqs, int64_t count);

/* As vr_query_stage_ms, for the whole batch. */
VR_API int vr_batch_stage_ms(const vr_batch *batch, float *ms, int cap);

/* Releases the batch's device memory in stream order on `stream`, then the
 * handle; every view dies with it.  NULL-safe. */
VR_API void vr_batch_free(vr_batch *batch, void *stream);

/*
 * Autotuning of the triangle kernels' schedule (work-group size 128, 256 or 512,
 * work-groups per vertex 1, 2, 4, 8 or 16, and candidate pieces of 64 loaded
 * at a time: 2, 4 or 8 for the count, 4 or 8 for the write; the write also
 * takes 0 work-groups per vertex: one wave per vertex and eighth of its
 * partners, each die of the chip taking one eighth, with the work-group
 * size halved while its waves' LDS, 2 maxn + 2048 bytes each, would pass
 * 64 KiB) for the size
 * class of these requests (bits of their total vertex count and of their
 * mean degree).  Runs one build of the requests (as vr_build_batch), then
 * times the count and the write kernel at every schedule, keeps the fastest
 * of each in a process-wide table that later builds of the class use, and
 * frees the build.  Schedules change no output.  Synchronises `stream`.
 * sched[0..5] receive (count work-group size, count work-groups per vertex,
 * count pieces, write work-group size, write work-groups per vertex, write
 * pieces); all 0 when the requests have no triangles.  Same error behaviour
 * as vr_build_batch.
 */
VR_API int vr_autotune(const vr_request *reqs, int64_t count, void *stream, int32_t sched[6]);

/* Sets the schedule of these requests' size class, as vr_autotune would
 * have chosen it: sched[0..5] as vr_autotune reports them, each one of that
 * function's candidates (else VR_EINVAL).  For reusing a schedule tuned
 * earlier (e.g. in another process) without tuning again.  Host only. */
VR_API int vr_set_schedule(const vr_request *reqs, int64_t count, const int32_t sched[6]);

/* Per-column stable order of a compressed-sparse-column array (Section 4.3,
 * the ordering of the integers of every column; the paper's counting sort
 * prefix-sums each column's value range).
 * colptr: device, ncols + 1 int64 entries, colptr[0] = 0, non-decreasing,
 *         colptr[ncols] = nnz; column c holds entries colptr[c] ..
 *         colptr[c+1] - 1.
 * v:      device, nnz int32 values (any sign).
 * z:      device, nnz int64, caller-owned output: z[e] = colptr[c] + the
 *         entries of e's column with a smaller value + the entries before e
 *         in its column with the same value, i.e. the slot of entry e when
 *         its column is sorted stably by value.
 * Enqueued on `stream`; scratch of 4 bytes per entry comes from the
 * library's cache.  VR_EINVAL for negative sizes, a null pointer, or
 * entries without columns; VR_E2BIG for nnz >= 2^43; nnz = 0 does nothing.  A colptr that breaks the
 * rules above gives unspecified z but no access outside the arrays. */
VR_API int vr_column_order(const int64_t *colptr, int64_t ncols, const int32_t *v, int64_t nnz, int64_t *z,
                           void *stream);

/* vr_column_order for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, result and errors, but the scratch lives in
 * an array of VR_COLORDER_NOALLOC_BYTES that the library holds on every GPU
 * it runs on until the process ends, so the call allocates nothing (its
 * device address is looked up on the first call on each GPU).  Limit: the
 * scratch of one call, 8 ceil(nnz / 4096) bytes rounded up to 256, plus 4
 * nnz bytes (about 8.3 million entries), must fit, else VR_E2BIG and
 * nothing is enqueued.  `stream` must belong to the calling thread's
 * current device.  Every call on one GPU uses the same array: calls that
 * overlap on one GPU (different streams or threads without ordering
 * between them) race, and the caller must order them.  VR_EHIP if the
 * array's address cannot be found. */
#define VR_COLORDER_NOALLOC_BYTES (32u << 20)
VR_API int vr_column_order_noalloc(const int64_t *colptr, int64_t ncols, const int32_t *v, int64_t nnz,
                                   int64_t *z, void *stream);

/* Persistence pairs in dimension 0 of a build's filtration (Section 2.2.1:
 * Alg. 1 on the edge columns of the boundary matrix; vertices share one
 * value and are ordered by index).  Edge r is paired with the vertex that
 * is the smallest of its component just before r joins that component to
 * one holding a smaller vertex; every other edge is unpaired (it creates a
 * cycle).
 * res:    a single build's result (edges on the device, rank order).
 * e_low:  device, K int32, caller-owned: the vertex paired with edge r, or -1.
 * death:  device, n int32, caller-owned: the edge rank that pairs vertex v,
 *         or -1 for the smallest vertex of each final component (an
 *         infinite bar).
 * Enqueued on `stream`.  Up to 512 points the pairs come from the (min, max)
 * closure of the rank matrix, with scratch of 4 (64 ceil(n / 64))^2 bytes
 * from the library's cache; larger clouds use a spanning forest in rank
 * order (K finds and at most n - 1 unions, no scratch).  VR_EINVAL for a
 * null argument or n > VR_MAX_POINTS. */
VR_API int vr_pairs_dim0(const vr_result *res, int32_t *e_low, int32_t *death, void *stream);

/* Apparent persistence pairs in dimension 1 (Section 2.2.1, Alg. 1 on the
 * triangle columns).  The triangles of value r are the cofacets of edge r
 * whose other edges are older; the first of them in filtration order is
 * the oldest cofacet of edge r and has edge r as its youngest facet, and
 * the column algorithm pairs the two (edge r becomes a cycle that this
 * triangle fills at once: a bar of length zero).  The other pairs of
 * dimension 1, the bars of positive length among them, need column
 * additions and are not computed here.
 * res:          a single build's result with triangle keys (not count-only).
 * tri_of_edge:  device, K int32, caller-owned: the index in tri_key of the
 *               triangle paired with edge r, or -1.
 * Enqueued on `stream`; allocates nothing.  VR_EINVAL for a null argument,
 * a result without keys, or T >= 2^31. */
VR_API int vr_pairs_dim1_apparent(const vr_result *res, int32_t *tri_of_edge, void *stream);

/* All persistence pairs in dimension 1 (Section 2.2.1, Alg. 1, run as in
 * Section 2.2.2 on the anti-transpose of the boundary matrix with
 * clearing): the edge columns go from the youngest edge to the oldest, and
 * the pivot of an edge's column is its oldest cofacet (the smallest
 * triangle key).  Edges paired with a vertex are cleared (their columns
 * reduce to zero); an edge with triangles of its own value pairs with the
 * first of them (as in vr_pairs_dim1_apparent); the other edge columns are
 * reduced in rounds: every unsettled column at once (one work-group each)
 * adds the apparent coboundaries and the stored columns of owners before it
 * that its pivots meet, then each pivot goes to its first claimant in the
 * order, displacing a later owner; every round settles at least one column.
 * The pairs equal those of the column algorithm on the whole boundary
 * matrix (Section 2.2.2), whose pairs do not depend on the column
 * operations that reached them.
 * res:          a single build's result with its triangle keys (maxdim 2,
 *               not count-only).
 * e_low:        device, K int32: vr_pairs_dim0's e_low for this result.
 * tri_of_edge:  device, K int32, caller-owned output: the index in tri_key
 *               of the triangle paired with edge r (bar [r, its value); of
 *               length zero when its value is r), or -1: edge r is paired
 *               with a vertex (e_low[r] >= 0), or else starts a class of
 *               dimension 1 that never dies.
 * The working column is a base list in device memory plus a short sorted
 * delta in LDS that takes the additions and is folded into the base when
 * full.  Synchronises `stream` once per round (the number of unsettled
 * columns and a status word are read back).  Scratch from the library's
 * cache: 4 n^2 + 48 K + 32 H bytes (H = 2K rounded up to a power of two)
 * plus 1 GiB (the stored columns and rewritten bases, 2^27 keys), and when
 * 3 T <= 2^25 another 8 K + 24 T bytes: the apparent edges' coboundaries,
 * generated once, all at once, so that a long chain of additions copies
 * them instead of generating each.  VR_ENOMEM when the columns outgrow
 * that.
 * VR_EINVAL for a null argument, n > VR_MAX_POINTS or T >= 2^31.  With no
 * triangles (T = 0) no edge dies. */
VR_API int vr_pairs_dim1(const vr_result *res, const int32_t *e_low, int32_t *tri_of_edge, void *stream);

/* The barcode of dimensions 0 and 1 from the pairs (Section 2.2.1: a pair
 * (sigma, tau) is the bar [value of sigma, value of tau); a simplex paired
 * with nothing that kills nothing starts a bar that never ends).  Values:
 * -1 for vertices, the rank for edges, the value for triangles; a bar that
 * never ends has death INT64_MAX.  Bars of length zero are left out.
 * e_low, tri_of_edge: vr_pairs_dim0's and vr_pairs_dim1's outputs.
 * bars:    device, 3 (n + K) int64, caller-owned: (dimension, birth, death)
 *          triples.  bars[0, n): dimension 0, first [-1, r) for every edge
 *          r paired with a vertex, in edge order, then [-1, inf) for each
 *          vertex no edge pairs; from bars[n]: dimension 1 in edge order,
 *          [r, value) for edge r paired with a later triangle, [r, inf) for
 *          an edge paired with nothing.
 * counts:  host, 3 int64: n, the bars of dimension 1 written, and the
 *          triangles paired with nothing (bars [value, inf) of dimension 2,
 *          not listed).
 * Synchronises `stream`.  VR_EINVAL for a null argument, n > VR_MAX_POINTS
 * or T >= 2^31. */
VR_API int vr_barcode(const vr_result *res, const int32_t *e_low, const int32_t *tri_of_edge, int64_t *bars,
                      int64_t counts[3], void *stream);

/* Tetrahedra (dimension 3) of a build's filtration, counted per largest
 * edge: a tetrahedron exists once its six edges are kept, and its value is
 * its largest edge rank (Section 2.1's rule one dimension up).  The
 * tetrahedra themselves are not listed.
 * res:     a single build's result (edges on the device, rank order).
 * counts:  device, K int64, caller-owned: the tetrahedra whose largest
 *          edge is edge r.
 * Work: two rank rows per edge (K n reads), then, per edge, the pairs of
 * its m common older neighbours (m^2 / 2): milliseconds for a thousand
 * points, far longer near the largest n and K.
 * Enqueued on `stream`; scratch of 4 n^2 bytes from the library's cache.
 * VR_EINVAL for a null argument or n > VR_MAX_POINTS. */
VR_API int vr_tetra_counts(const vr_result *res, int64_t *counts, void *stream);

/* The tetrahedra themselves, in filtration order: by value, then by their
 * sorted vertices.  Two calls:
 *   vr_tetra_offsets writes offsets (K + 1 int64, caller-owned device
 *     memory): offsets[r] = the first tetrahedron of value r, offsets[K] =
 *     their number T3;
 *   vr_tetra_write writes keys (2 T3 uint64, caller-owned, 16-byte
 *     aligned): for the t-th
 *     tetrahedron keys[2t] = its value and keys[2t+1] = a<<39 | b<<26 |
 *     c<<13 | d with a < b < c < d.  `total` is offsets[K] as read back by
 *     the caller (nothing is written past it).
 * Both enqueued on `stream`, with scratch of 4 n^2 bytes from the library's
 * cache; the work is that of vr_tetra_counts, twice for the write.
 * VR_EINVAL for a null argument, total < 0, misaligned keys, or
 * n > VR_MAX_POINTS. */
VR_API int vr_tetra_offsets(const vr_result *res, int64_t *offsets, void *stream);
VR_API int vr_tetra_write(const vr_result *res, const int64_t *offsets, int64_t total, uint64_t *keys, void *stream);

/* Persistence pairs of dimension 2: triangles with tetrahedra (Section
 * 2.2.1, Alg. 1, run as in Section 2.2.2 on the anti-transpose with
 * clearing, one dimension above vr_pairs_dim1; Section 3's bettimax = 2).
 * The triangle columns go from the youngest triangle to the oldest, and a
 * column's pivot is its oldest cofacet.  Triangles paired with an edge are
 * cleared; a triangle whose oldest cofacet has it as its youngest facet
 * pairs with it at once (an apparent pair: per edge the vertices joined to
 * both ends are listed once, and one wave per triangle of that value finds
 * its oldest cofacet among them); the other columns are reduced in rounds
 * as by vr_pairs_dim1.  The pairs equal those of the column algorithm on
 * the tetrahedra's boundary block.
 * res:          a maxdim-3 build's result with its triangle and tetrahedron
 *               keys (not count-only).
 * tri_of_edge:  device, K int32: vr_pairs_dim1's output for this result.
 * tri_tet:      device, T int64, caller-owned output: the index (in
 *               tet_key's order) of the tetrahedron paired with triangle t,
 *               or -1: t is paired with an edge, or else starts a class of
 *               dimension 2 that never dies.
 * Synchronises `stream` once per round.  Scratch from the library's cache:
 * 4 n^2 + 8 K + 60 T + 32 H bytes (H = 2T rounded up to a power of two)
 * plus 1 GiB, as vr_pairs_dim1.  VR_ENOMEM when the columns outgrow it; VR_EINVAL for a
 * null argument, a result without tetrahedron keys, n > VR_MAX_POINTS or
 * T >= 2^31.  With no triangles nothing is written. */
VR_API int vr_pairs_dim2(const vr_result *res, const int32_t *tri_of_edge, int64_t *tri_tet, void *stream);

/* The barcode of dimension 2 (and the classes of dimension 3) from the
 * pairs (Section 2.2.1: a pair (sigma, tau) is the bar [value of sigma,
 * value of tau)), as vr_barcode one dimension up.  Values are largest edge
 * ranks; a bar that never ends has death INT64_MAX; bars of length zero are
 * left out.
 * res:          a maxdim-3 build's result with its triangle and tetrahedron
 *               keys.
 * tri_of_edge, tri_tet: vr_pairs_dim1's and vr_pairs_dim2's outputs.
 * bars:    device, 3 T int64, caller-owned: (2, birth, death) triples in
 *          triangle order: triangle t paired with a tetrahedron of larger
 *          value w gives [value of t, w); a triangle paired with neither an
 *          edge nor a tetrahedron gives [value of t, inf).
 * counts:  host: counts[0] = the bars written, counts[1] = the tetrahedra
 *          no triangle pairs with (classes of dimension 3 that never die;
 *          counted, not listed).
 * Synchronises `stream`.  VR_EINVAL for a null argument, a result without
 * tetrahedron keys, n > VR_MAX_POINTS or T >= 2^31. */
VR_API int vr_barcode_dim2(const vr_result *res, const int32_t *tri_of_edge, const int64_t *tri_tet, int64_t *bars,
                           int64_t counts[2], void *stream);

/* The F2 sparse product and sum of the Schur complement step (Section 4.6):
 * S = D + C E mod 2, where C is m x k, E is k x n and D is m x n, all in
 * compressed sparse columns on the device: colptr (ncols + 1 int64, from 0,
 * non-decreasing, ending at the entry count) and rows (int32 row indices;
 * NULL only for a matrix without entries).  Rows within a column may come
 * in any order, and a row listed twice in a column cancels.  Two calls:
 *   vr_blockprodsum_count writes S's column pointers into s_colptr (n + 1
 *     int64, caller-owned device memory);
 *   vr_blockprodsum_write then writes S's rows into s_rows (s_colptr[n]
 *     int32, caller-owned), ascending within each column; it takes the
 *     s_colptr of a count call on the same inputs.
 * Both are enqueued on `stream` and allocate nothing.  VR_EINVAL for
 * negative sizes or missing column pointers, VR_E2BIG for m > 262144 (the
 * rows of one column of S are gathered in a bitmap in LDS).  Malformed
 * column pointers or row indices give an unspecified S but no access
 * outside the arrays they describe. */
VR_API int vr_blockprodsum_count(int64_t m, int64_t k, int64_t n, const int64_t *c_colptr, const int32_t *c_rows,
                                 const int64_t *e_colptr, const int32_t *e_rows, const int64_t *d_colptr,
                                 const int32_t *d_rows, int64_t *s_colptr, void *stream);
VR_API int vr_blockprodsum_write(int64_t m, int64_t k, int64_t n, const int64_t *c_colptr, const int32_t *c_rows,
                                 const int64_t *e_colptr, const int32_t *e_rows, const int64_t *d_colptr,
                                 const int32_t *d_rows, const int64_t *s_colptr, int32_t *s_rows, void *stream);

/* Device memory.  Without a caller allocator, workspaces and output blocks
 * come from a stream-ordered cache inside the library: blocks are taken from
 * the driver once and reused by later builds of any stream (a reuse on
 * another stream first waits, on the device, for the block's last use), so
 * a stream of requests of changing sizes does not return to the driver.
 * vr_trim drops the calling thread's captured graphs (VR_GRAPH), then
 * releases the cached blocks of the current device that no result holds
 * (it synchronises the device) and returns the bytes released. */
VR_API int64_t vr_trim(void);

/* Static description of a status code. */
VR_API const char *vr_status_string(int status);

/* Library version, e.g. 130 for 0.1.3. */
VR_API int vr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VR_H */
