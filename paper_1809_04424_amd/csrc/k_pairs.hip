// k_pairs.hip -- persistence pairs in dimension 0 (Section 2.2.1, Alg. 1 on
// the edge columns of the boundary matrix) on the device.
//
// With every vertex at the same value and vertices ordered by index, the
// column algorithm pairs edge r with vertex v exactly when v is the smallest
// vertex of its component just before r joins it to a component holding a
// smaller vertex (the younger component dies).  So vertex v dies at
//     death(v) = min over u < v of  minimax(v, u),
// where minimax(v, u) is the least, over the paths from v to u, of the
// largest edge rank on the path (+inf when no path exists); v with no
// finite death is the oldest vertex of its component and never dies.
//
// minimax over all pairs is the closure of the rank matrix in the (min, max)
// semiring: a blocked Floyd-Warshall in 64 x 64 tiles.
//   k_pd_fill     D = +inf off the diagonal, -1 on it
//   k_pd_edges    D[i][j] = D[j][i] = r per kept edge
//   k_pd_diag     phase 1: the diagonal tile, pivots in order
//   k_pd_cross    phase 2: the tiles in the pivot's row and column, each a
//                 (min, max) product with the closed diagonal tile
//   k_pd_rest     phase 3: every other tile, the product of a column tile
//                 and a row tile
//   k_pd_death    death(v): a wave takes the minimum of row v left of v
//   k_pd_clear, k_pd_emit   e_low[r] = v for death(v) = r, else -1
// D is (nb * 64)^2 with the padding vertices isolated, so the tile kernels
// need no bounds tests.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vr.h"
#include "vr_cache.h"

#define PD_T 64      // tile edge
#define PD_BLOCK 256  // 16 x 16 threads, 4 x 4 entries each
#define PD_INF 0x7FFFFFFF
// Largest point count whose dimension-0 pairs come from the (min, max)
// closure; larger clouds use the spanning forest.
#define PD_CLOSURE_MAX 512

__global__ void __launch_bounds__(PD_BLOCK) k_pd_fill(int32_t *D, int64_t m) {
    const int64_t ld = m;
    for (int64_t x = blockIdx.x * (int64_t)PD_BLOCK + threadIdx.x; x < ld * ld; x += (int64_t)gridDim.x * PD_BLOCK)
        D[x] = (x / ld == x % ld) ? -1 : PD_INF;
}

__global__ void __launch_bounds__(PD_BLOCK) k_pd_edges(int32_t *D, int64_t ld, const int32_t *ij, int64_t K,
                                                      int64_t n) {
    for (int64_t r = blockIdx.x * (int64_t)PD_BLOCK + threadIdx.x; r < K; r += (int64_t)gridDim.x * PD_BLOCK) {
        const int64_t i = ij[2 * r], j = ij[2 * r + 1];
        if (i < 0 || j < 0 || i >= n || j >= n) continue;  // never for a library result
        D[i * ld + j] = (int32_t)r;
        D[j * ld + i] = (int32_t)r;
    }
}

// In the tile kernels thread (ty, tx) owns rows 4ty..4ty+3 and columns
// 4tx..4tx+3 of a tile.

// phase 1: D_kk closed over its own 64 pivots, in order, by 1024 threads of
// 2 x 2 entries each (thread (ty, tx) of 32 x 32: rows 2ty, 2ty+1, columns
// 2tx, 2tx+1), which keeps the work between two pivots short.  The entries
// stay in registers; after pivot k the owners of row k+1 and column k+1
// publish them to LDS for the next pivot.  Row k and column k do not change
// at pivot k (D[k][k] = -1), and the entries written after pivot k are not
// the ones read at pivot k, so one barrier per pivot suffices.
#define PD_DIAG_BLOCK 1024
__global__ void __launch_bounds__(PD_DIAG_BLOCK) k_pd_diag(int32_t *D, int64_t ld, int64_t kb) {
    __shared__ __align__(16) int32_t s[PD_T][PD_T + 4];
    const int ty = threadIdx.x >> 5, tx = threadIdx.x & 31;
    int32_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++) {
        const int2 v = *(const int2 *)(D + (kb * PD_T + 2 * ty + a) * ld + kb * PD_T + 2 * tx);
        acc[a][0] = v.x;
        acc[a][1] = v.y;
        *(int2 *)&s[2 * ty + a][2 * tx] = v;
    }
    __syncthreads();
    for (int k = 0; k < PD_T; k++) {
        const int32_t c0 = s[2 * ty][k], c1 = s[2 * ty + 1][k];
        const int2 r = *(const int2 *)&s[k][2 * tx];
        acc[0][0] = min(acc[0][0], max(c0, r.x));
        acc[0][1] = min(acc[0][1], max(c0, r.y));
        acc[1][0] = min(acc[1][0], max(c1, r.x));
        acc[1][1] = min(acc[1][1], max(c1, r.y));
        const int k1 = k + 1;
#pragma unroll
        for (int a = 0; a < 2; a++)
            if (2 * ty + a == k1) *(int2 *)&s[k1][2 * tx] = make_int2(acc[a][0], acc[a][1]);
#pragma unroll
        for (int b = 0; b < 2; b++)
            if (2 * tx + b == k1) {
                s[2 * ty][k1] = acc[0][b];
                s[2 * ty + 1][k1] = acc[1][b];
            }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; a++)
        *(int2 *)(D + (kb * PD_T + 2 * ty + a) * ld + kb * PD_T + 2 * tx) = make_int2(acc[a][0], acc[a][1]);
}

// out = min(out, A (min,max) B) for 64 x 64 tiles A = (ai, aj), B = (bi, bj),
// out = (oi, oj); out may be A or B (all reads precede the writes)
static __device__ __forceinline__ void pd_product(int32_t *D, int64_t ld, int64_t ai, int64_t aj, int64_t bi,
                                                  int64_t bj, int64_t oi, int64_t oj) {
    __shared__ __align__(16) int32_t at[PD_T][PD_T + 4];  // A transposed: at[m][i]
    __shared__ __align__(16) int32_t bt[PD_T][PD_T + 4];  // B: bt[m][j]
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
#pragma unroll
    for (int a = 0; a < 4; a++) {
        const int4 v = *(const int4 *)(D + (ai * PD_T + 4 * ty + a) * ld + aj * PD_T + 4 * tx);
        at[4 * tx + 0][4 * ty + a] = v.x;
        at[4 * tx + 1][4 * ty + a] = v.y;
        at[4 * tx + 2][4 * ty + a] = v.z;
        at[4 * tx + 3][4 * ty + a] = v.w;
        *(int4 *)&bt[4 * ty + a][4 * tx] = *(const int4 *)(D + (bi * PD_T + 4 * ty + a) * ld + bj * PD_T + 4 * tx);
    }
    int32_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; a++) {
        const int4 v = *(const int4 *)(D + (oi * PD_T + 4 * ty + a) * ld + oj * PD_T + 4 * tx);
        acc[a][0] = v.x;
        acc[a][1] = v.y;
        acc[a][2] = v.z;
        acc[a][3] = v.w;
    }
    __syncthreads();
#pragma unroll 8
    for (int m = 0; m < PD_T; m++) {
        const int4 c = *(const int4 *)&at[m][4 * ty];
        const int4 r = *(const int4 *)&bt[m][4 * tx];
        const int32_t cv[4] = {c.x, c.y, c.z, c.w}, rv[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 4; b++) acc[a][b] = min(acc[a][b], max(cv[a], rv[b]));
    }
#pragma unroll
    for (int a = 0; a < 4; a++)
        *(int4 *)(D + (oi * PD_T + 4 * ty + a) * ld + oj * PD_T + 4 * tx) =
            make_int4(acc[a][0], acc[a][1], acc[a][2], acc[a][3]);
}

// phase 2: with D_kk closed, the tiles of the pivot's row and column need
// one product each: row tile (kb, o) = D_kk (min,max) itself, column tile
// (o, kb) = itself (min,max) D_kk.  Work-group g < nb: row tile (kb, g);
// nb <= g < 2 nb: column tile (g - nb, kb).
__global__ void __launch_bounds__(PD_BLOCK) k_pd_cross(int32_t *D, int64_t ld, int64_t kb, int64_t nb) {
    const int64_t g = blockIdx.x;
    const bool row = g < nb;
    const int64_t o = row ? g : g - nb;
    if (o == kb) return;
    if (row) pd_product(D, ld, kb, kb, kb, o, kb, o);
    else pd_product(D, ld, o, kb, kb, kb, o, kb);
}

// phase 3: tile (bi, bj) off the pivot's row and column takes the product
// of column tile (bi, kb) and row tile (kb, bj)
__global__ void __launch_bounds__(PD_BLOCK) k_pd_rest(int32_t *D, int64_t ld, int64_t kb, int64_t nb) {
    const int64_t bi = blockIdx.y, bj = blockIdx.x;
    if (bi == kb || bj == kb) return;
    pd_product(D, ld, bi, kb, kb, bj, bi, bj);
}

// death(v) = min over u < v of D[v][u]; -1 when none is finite
__global__ void __launch_bounds__(PD_BLOCK) k_pd_death(const int32_t *D, int64_t ld, int64_t n, int32_t *death) {
    const int lane = threadIdx.x & 63;
    const int64_t v = blockIdx.x * (int64_t)(PD_BLOCK / 64) + (threadIdx.x >> 6);
    if (v >= n) return;
    int32_t m = PD_INF;
    for (int64_t u = lane; u < v; u += 64) m = min(m, D[v * ld + u]);
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) m = min(m, __shfl_xor(m, d, 64));
    if (lane == 0) death[v] = m == PD_INF ? -1 : m;
}

__global__ void __launch_bounds__(PD_BLOCK) k_pd_clear(int32_t *e_low, int64_t K) {
    for (int64_t r = blockIdx.x * (int64_t)PD_BLOCK + threadIdx.x; r < K; r += (int64_t)gridDim.x * PD_BLOCK)
        e_low[r] = -1;
}

__global__ void __launch_bounds__(PD_BLOCK) k_pd_emit(const int32_t *death, int64_t n, int32_t *e_low, int64_t K) {
    const int64_t v = blockIdx.x * (int64_t)PD_BLOCK + threadIdx.x;
    if (v >= n) return;
    const int32_t r = death[v];
    if (r >= 0 && r < K) e_low[r] = (int32_t)v;
}

// Dimension 0 by a spanning forest (Kruskal's order): the edges in rank
// order, a union-find whose roots are the smallest vertex of each component
// (the larger root is linked under the smaller), so the column algorithm's
// pair for an edge joining two components is the larger of the two roots.
// One work-group takes the edges 1024 at a time: every thread finds the
// roots of its edge's ends without writing, and only the edges whose ends
// lie in different components (the candidates) go, in rank order, through
// the serial union by one thread, which finds again (an earlier candidate
// of the chunk may have joined the two).  Work: K reads and finds, plus the
// serial step for at most n - 1 unions and the candidates that lost to an
// earlier one; it stops once n - 1 unions are made.
#define PF_BLOCK 1024
__global__ void __launch_bounds__(PF_BLOCK) k_pd_forest(const int32_t *ij, int64_t K, int64_t n, int32_t *e_low,
                                                       int32_t *death) {
    __shared__ int32_t par[VR_MAX_POINTS];
    __shared__ int32_t cand[PF_BLOCK], ca[PF_BLOCK], cb[PF_BLOCK];
    __shared__ uint32_t wc[PF_BLOCK / 64];
    __shared__ int32_t s_unions;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int64_t v = t; v < n; v += PF_BLOCK) par[v] = (int32_t)v;
    if (t == 0) s_unions = 0;
    __syncthreads();
    for (int64_t e0 = 0; e0 < K && s_unions < n - 1; e0 += PF_BLOCK) {
        const int64_t e = e0 + t;
        bool c = false;
        int32_t ea = 0, eb = 0;
        if (e < K) {
            ea = ij[2 * e];
            eb = ij[2 * e + 1];
            if (ea >= 0 && eb >= 0 && ea < n && eb < n) {  // always for a library result
                int32_t a = ea, b = eb;
                while (par[a] != a) a = par[a];
                while (par[b] != b) b = par[b];
                c = a != b;
            }
        }
        const unsigned long long m = __ballot(c);
        if (lane == 0) wc[wv] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = 0, tot = 0;
        for (int w = 0; w < PF_BLOCK / 64; w++) {
            if (w < wv) before += wc[w];
            tot += wc[w];
        }
        if (c) {
            const uint32_t at = before + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
            cand[at] = (int32_t)(e - e0);
            ca[at] = ea;
            cb[at] = eb;
        }
        __syncthreads();
        if (t == 0) {
            int32_t u = s_unions;
            for (uint32_t i = 0; i < tot; i++) {
                const int64_t f = e0 + cand[i];
                int32_t a = ca[i], b = cb[i];
                while (par[a] != a) {
                    par[a] = par[par[a]];
                    a = par[a];
                }
                while (par[b] != b) {
                    par[b] = par[par[b]];
                    b = par[b];
                }
                if (a != b) {
                    const int32_t lo = min(a, b), hi = max(a, b);
                    par[hi] = lo;
                    e_low[f] = hi;
                    death[hi] = (int32_t)f;
                    u++;
                }
            }
            s_unions = u;
        }
        __syncthreads();
    }
}

// Dimension 1, apparent pairs.  Triangles of value r are the cofacets of
// edge r whose other two edges are older, and the writer emits them
// together in lexicographic order, so the first of them is the oldest
// cofacet of edge r, and edge r (the largest edge) is its youngest facet:
// the two form an apparent pair, which the column algorithm always pairs.
// The first triangle of each value is where the value changes along the
// keys.
__global__ void __launch_bounds__(PD_BLOCK) k_pd_apparent(const unsigned long long *key, int64_t T, int32_t *first,
                                                         int64_t K) {
    for (int64_t t = blockIdx.x * (int64_t)PD_BLOCK + threadIdx.x; t < T; t += (int64_t)gridDim.x * PD_BLOCK) {
        const unsigned long long v = key[t] >> 39;
        const unsigned long long u = t > 0 ? key[t - 1] >> 39 : ~0ull;
        if (v != u && (int64_t)v < K) first[v] = (int32_t)t;
    }
}

static unsigned grid_for(int64_t items) {
    const int64_t g = (items + PD_BLOCK - 1) / PD_BLOCK;
    return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

extern "C" VR_API int vr_pairs_dim0(const vr_result *res, int32_t *e_low, int32_t *death, void *stream) {
    if (!res) return VR_EINVAL;
    const int64_t n = res->n_vertices, K = res->n_edges;
    if (n < 0 || K < 0 || n > VR_MAX_POINTS) return VR_EINVAL;
    if ((K > 0 && (!e_low || !res->edge_ij)) || (n > 0 && !death)) return VR_EINVAL;
    if (n == 0) return VR_OK;
    const hipStream_t s = (hipStream_t)stream;
    if (n > PD_CLOSURE_MAX) {
        // the spanning forest: K finds and at most n - 1 serial unions
        hipLaunchKernelGGL(k_pd_clear, dim3(grid_for(n)), dim3(PD_BLOCK), 0, s, death, n);
        if (K > 0) {
            hipLaunchKernelGGL(k_pd_clear, dim3(grid_for(K)), dim3(PD_BLOCK), 0, s, e_low, K);
            hipLaunchKernelGGL(k_pd_forest, dim3(1), dim3(PF_BLOCK), 0, s, (const int32_t *)res->edge_ij, K, n, e_low,
                               death);
        }
        return hipGetLastError() == hipSuccess ? VR_OK : VR_EHIP;
    }
    const int64_t nb = (n + PD_T - 1) / PD_T, ld = nb * PD_T;
    int32_t *D = (int32_t *)cache_get((size_t)ld * (size_t)ld * 4, s);
    if (!D) return VR_ENOMEM;
    hipLaunchKernelGGL(k_pd_fill, dim3(grid_for(ld * ld)), dim3(PD_BLOCK), 0, s, D, ld);
    if (K > 0)
        hipLaunchKernelGGL(k_pd_edges, dim3(grid_for(K)), dim3(PD_BLOCK), 0, s, D, ld,
                           (const int32_t *)res->edge_ij, K, n);
    if (K > 0)
        for (int64_t kb = 0; kb < nb; kb++) {
            hipLaunchKernelGGL(k_pd_diag, dim3(1), dim3(PD_DIAG_BLOCK), 0, s, D, ld, kb);
            if (nb > 1) {
                hipLaunchKernelGGL(k_pd_cross, dim3((unsigned)(2 * nb)), dim3(PD_BLOCK), 0, s, D, ld, kb, nb);
                hipLaunchKernelGGL(k_pd_rest, dim3((unsigned)nb, (unsigned)nb), dim3(PD_BLOCK), 0, s, D, ld, kb, nb);
            }
        }
    hipLaunchKernelGGL(k_pd_death, dim3((unsigned)((n + PD_BLOCK / 64 - 1) / (PD_BLOCK / 64))), dim3(PD_BLOCK), 0, s,
                       (const int32_t *)D, ld, n, death);
    if (K > 0) {
        hipLaunchKernelGGL(k_pd_clear, dim3(grid_for(K)), dim3(PD_BLOCK), 0, s, e_low, K);
        hipLaunchKernelGGL(k_pd_emit, dim3(grid_for(n)), dim3(PD_BLOCK), 0, s, (const int32_t *)death, n, e_low, K);
    }
    const hipError_t e = hipGetLastError();
    cache_put(D, s);
    return e == hipSuccess ? VR_OK : VR_EHIP;
}

extern "C" VR_API int vr_pairs_dim1_apparent(const vr_result *res, int32_t *tri_of_edge, void *stream) {
    if (!res) return VR_EINVAL;
    const int64_t K = res->n_edges, T = res->n_triangles;
    if (K < 0 || T < 0 || T > 0x7FFFFFFF) return VR_EINVAL;
    if (K == 0) return VR_OK;
    if (!tri_of_edge || (T > 0 && !res->tri_key)) return VR_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_pd_clear, dim3(grid_for(K)), dim3(PD_BLOCK), 0, s, tri_of_edge, K);
    if (T > 0)
        hipLaunchKernelGGL(k_pd_apparent, dim3(grid_for(T)), dim3(PD_BLOCK), 0, s, (const unsigned long long *)res->tri_key,
                           T, tri_of_edge, K);
    return hipGetLastError() == hipSuccess ? VR_OK : VR_EHIP;
}

// Index pairs (a, b), a < b < m, numbered row-major: p = S(a) + b - a - 1,
// S(a) = a (2m - a - 1) / 2 the pairs of the rows before a.
static __device__ __forceinline__ long long tet_row_start(long long a, long long m) { return a * (2 * m - a - 1) / 2; }

// Index pair of pair number p among the pairs of m entries: a from the
// closed form in single precision, then corrected with exact integers.
static __device__ __forceinline__ void tet_pair(long long p, long long m, uint32_t &a, uint32_t &b) {
    const float c = (float)(2 * m - 1);
    float disc = c * c - 8.0f * (float)p;
    disc = disc > 0.0f ? disc : 0.0f;
    long long x = (long long)((c - sqrtf(disc)) * 0.5f);
    x = x < 0 ? 0 : (x > m - 2 ? m - 2 : x);
    while (x > 0 && tet_row_start(x, m) > p) x--;
    while (x < m - 2 && tet_row_start(x + 1, m) <= p) x++;
    a = (uint32_t)x;
    b = (uint32_t)(p - tet_row_start(x, m) + x + 1);
}

// Move pair (a, b) d places on in row-major order (row a holds b = a+1 ..
// m-1): b grows by d, and each time it leaves its row it continues in the
// next, shorter one.  Past the last pair it stops at a = m - 1 (no pair).
static __device__ __forceinline__ void tet_advance(uint32_t &a, uint32_t &b, uint32_t d, uint32_t m) {
    b += d;
    while (b >= m && a + 2 < m) {
        a++;
        b = b - m + a + 1;
    }
    if (b >= m) a = m - 1;
}

// Tetrahedra (dimension 3) per largest edge.  Work-group g takes edge r:
// the vertices x joined to both ends by older edges (D[i][x] < r and
// D[j][x] < r; the ends themselves fail one test, D[i][j] = r), compacted
// into LDS in ascending order, then the pairs of them joined by an older
// edge, a wave per row of the pairs (rows are long, so lanes stay busy; the
// writer, which must also order its stores, numbers the pairs instead).  D
// as for the pairs of dimension 0 (ranks, +inf off the edges, -1 on the
// diagonal).
__global__ void __launch_bounds__(PD_BLOCK) k_tet_count(const int32_t *D, int64_t ld, int64_t n, const int32_t *ij,
                                                       int64_t K, long long *counts) {
    __shared__ uint16_t L[VR_MAX_POINTS];
    __shared__ uint32_t wc[PD_BLOCK / 64];
    __shared__ unsigned long long tot[PD_BLOCK / 64];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int64_t r = blockIdx.x; r < K; r += gridDim.x) {
        const int64_t i = ij[2 * r], j = ij[2 * r + 1];
        const bool ok = i >= 0 && j >= 0 && i < n && j < n;  // always for a library result
        uint32_t m = 0;
        for (int64_t x0 = 0; x0 < n; x0 += PD_BLOCK) {
            const int64_t x = x0 + t;
            const bool in = ok && x < n && D[i * ld + x] < r && D[j * ld + x] < r;
            const unsigned long long b = __ballot(in);
            if (lane == 0) wc[wv] = (uint32_t)__popcll(b);
            __syncthreads();
            uint32_t base = m, chunk = 0;
#pragma unroll
            for (int w = 0; w < PD_BLOCK / 64; w++) {
                if (w < wv) base += wc[w];
                chunk += wc[w];
            }
            if (in) L[base + __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0))] =
                (uint16_t)x;
            m += chunk;
            __syncthreads();  // wc is rewritten by the next chunk
        }
        // the pairs of the common neighbours joined by an older edge: wave w
        // takes the rows a = w, w + 4, ..., its lanes the later entries b of
        // row a together (ascending, so nearby addresses)
        unsigned long long c = 0;
        for (uint32_t a = wv; a + 1 < m; a += PD_BLOCK / 64) {
            const int32_t *row = D + (int64_t)L[a] * ld;
            for (uint32_t b2 = a + 1 + lane; b2 < m; b2 += 64) c += row[L[b2]] < r ? 1ull : 0ull;
        }
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d, 64);
        if (lane == 0) tot[wv] = c;
        __syncthreads();
        if (t == 0) {
            unsigned long long s2 = 0;
            for (int w = 0; w < PD_BLOCK / 64; w++) s2 += tot[w];
            counts[r] = (long long)s2;
        }
        __syncthreads();  // L and tot are reused by the next edge
    }
}

extern "C" VR_API int vr_tetra_counts(const vr_result *res, int64_t *counts, void *stream);

// Tetrahedra written in filtration order.  The group of edge r starts at
// off[r] (an exclusive scan of the counts).  Within it the tetrahedra
// {i, j, k, l} run in lexicographic order of their sorted vertices, which
// for a fixed pair i < j is the lexicographic order of (k, l), k < l.  With
// the common neighbours L ascending, that is the row-major order of the
// index pairs (a, b), a < b, numbered p = S(a) + b - a - 1 with
// S(a) = a (2m - a - 1) / 2 the pairs of the rows before a.  Each wave
// takes a contiguous quarter of the m (m - 1) / 2 pairs, 64 at a time (one
// pair per lane, so no lane idles on short rows): it counts its hits, the
// four counts are scanned, and it walks its pairs again, writing each hit
// through a ballot at its place.  Key of a tetrahedron: two words, its value
// r and a<<39 | b<<26 | c<<13 | d.
__global__ void __launch_bounds__(PD_BLOCK) k_tet_write(const int32_t *D, int64_t ld, int64_t n, const int32_t *ij,
                                                       int64_t K, const long long *off, long long total,
                                                       unsigned long long *keys) {
    __shared__ uint16_t L[VR_MAX_POINTS];
    __shared__ uint32_t wc[PD_BLOCK / 64];
    __shared__ unsigned long long wh[PD_BLOCK / 64];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int64_t r = blockIdx.x; r < K; r += gridDim.x) {
        const int64_t i = ij[2 * r], j = ij[2 * r + 1];
        const bool ok = i >= 0 && j >= 0 && i < n && j < n;
        uint32_t m = 0;
        for (int64_t x0 = 0; x0 < n; x0 += PD_BLOCK) {
            const int64_t x = x0 + t;
            const bool in = ok && x < n && D[i * ld + x] < r && D[j * ld + x] < r;
            const unsigned long long b = __ballot(in);
            if (lane == 0) wc[wv] = (uint32_t)__popcll(b);
            __syncthreads();
            uint32_t base = m, chunk = 0;
#pragma unroll
            for (int w = 0; w < PD_BLOCK / 64; w++) {
                if (w < wv) base += wc[w];
                chunk += wc[w];
            }
            if (in) L[base + __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0))] =
                (uint16_t)x;
            m += chunk;
            __syncthreads();
        }
        // this wave's pairs [p0, p1)
        const long long P = (long long)m * (m - 1) / 2;
        const long long p0 = P * wv / (PD_BLOCK / 64), p1 = P * (wv + 1) / (PD_BLOCK / 64);
        unsigned long long c = 0;
        uint32_t a0 = 0, b0 = 1;
        if (p0 + lane < p1) tet_pair(p0 + lane, m, a0, b0);  // once; then 64 places per step
        uint32_t a = a0, b = b0;
        for (long long q0 = p0; q0 < p1; q0 += 64) {
            const bool in = q0 + lane < p1 && D[(int64_t)L[a] * ld + L[b]] < r;
            c += (unsigned long long)__popcll(__ballot(in));
            tet_advance(a, b, 64, m);
        }
        if (lane == 0) wh[wv] = c;
        __syncthreads();
        unsigned long long pos = 0;
#pragma unroll
        for (int w = 0; w < PD_BLOCK / 64; w++)
            if (w < wv) pos += wh[w];
        const long long g0 = off[r];
        const uint32_t vi = (uint32_t)i, vj = (uint32_t)j;
        a = a0;
        b = b0;
        for (long long q0 = p0; q0 < p1; q0 += 64) {
            const bool live = q0 + lane < p1;  // a < b < m exactly then
            const uint32_t k = live ? L[a] : 0u, l = live ? L[b] : 0u;
            const bool in = live && D[(int64_t)k * ld + l] < r;
            tet_advance(a, b, 64, m);
            const unsigned long long bm = __ballot(in);
            if (in) {
                // sorted {i < j} and {k < l}: ends by min and max, the middle
                // two sorted between themselves
                const uint32_t lo = min(vi, k), hi = max(vj, l), u = max(vi, k), v = min(vj, l);
                const unsigned long long packed = ((unsigned long long)lo << 39) | ((unsigned long long)min(u, v) << 26) |
                                                  ((unsigned long long)max(u, v) << 13) | hi;
                const long long at = g0 + (long long)pos +
                    __builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0));
                if (at < total)  // one 16-byte store per tetrahedron
                    *(ulonglong2 *)(keys + 2 * at) = make_ulonglong2((unsigned long long)r, packed);
            }
            pos += (unsigned long long)__popcll(bm);
        }
        __syncthreads();  // L and wh are reused by the next edge
    }
}

__global__ void __launch_bounds__(1024) k_tet_scan(long long *v, int64_t K) {
    // exclusive scan of v[0..K) into v[0..K], v[K] = total; one work-group
    __shared__ long long wt[16];
    __shared__ long long carry;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < K; base += 4096) {  // 4 consecutive values per thread
        long long e[4], own = 0;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int64_t x = base + 4 * t + u;
            e[u] = x < K ? v[x] : 0;
            own += e[u];
        }
        long long incl = own;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const long long y = __shfl_up(incl, d, 64);
            if (lane >= d) incl += y;
        }
        if (lane == 63) wt[wv] = incl;
        __syncthreads();
        long long pre = carry + incl - own, tot = 0;
        for (int w = 0; w < 16; w++) {
            if (w < wv) pre += wt[w];
            tot += wt[w];
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int64_t x = base + 4 * t + u;
            if (x < K) v[x] = pre;
            pre += e[u];
        }
        __syncthreads();
        if (t == 0) carry += tot;
        __syncthreads();
    }
    if (t == 0) v[K] = carry;
}

// offsets[0..K]: the first tetrahedron of each edge's group, offsets[K] = the
// number of tetrahedra
extern "C" VR_API int vr_tetra_offsets(const vr_result *res, int64_t *offsets, void *stream) {
    if (!res || !offsets) return VR_EINVAL;
    const int64_t n = res->n_vertices, K = res->n_edges;
    if (n < 0 || K < 0 || n > VR_MAX_POINTS) return VR_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    if (K > 0) {
        const int st = vr_tetra_counts(res, offsets, stream);
        if (st != VR_OK) return st;
    }
    hipLaunchKernelGGL(k_tet_scan, dim3(1), dim3(1024), 0, s, (long long *)offsets, K);
    return hipGetLastError() == hipSuccess ? VR_OK : VR_EHIP;
}

extern "C" VR_API int vr_tetra_write(const vr_result *res, const int64_t *offsets, int64_t total, uint64_t *keys,
                                     void *stream) {
    if (!res || !offsets || total < 0 || (total > 0 && !keys)) return VR_EINVAL;
    if ((uintptr_t)keys % 16) return VR_EINVAL;  // keys are stored 16 bytes at a time
    const int64_t n = res->n_vertices, K = res->n_edges;
    if (n < 0 || K < 0 || n > VR_MAX_POINTS) return VR_EINVAL;
    if (K == 0 || total == 0) return VR_OK;
    if (!res->edge_ij) return VR_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    int32_t *D = (int32_t *)cache_get((size_t)n * (size_t)n * 4, s);
    if (!D) return VR_ENOMEM;
    hipLaunchKernelGGL(k_pd_fill, dim3(grid_for(n * n)), dim3(PD_BLOCK), 0, s, D, n);
    hipLaunchKernelGGL(k_pd_edges, dim3(grid_for(K)), dim3(PD_BLOCK), 0, s, D, n, (const int32_t *)res->edge_ij, K, n);
    hipLaunchKernelGGL(k_tet_write, dim3((unsigned)(K < 65536 ? K : 65536)), dim3(PD_BLOCK), 0, s, (const int32_t *)D,
                       n, n, (const int32_t *)res->edge_ij, K, (const long long *)offsets, (long long)total,
                       (unsigned long long *)keys);
    const hipError_t e = hipGetLastError();
    cache_put(D, s);
    return e == hipSuccess ? VR_OK : VR_EHIP;
}

extern "C" VR_API int vr_tetra_counts(const vr_result *res, int64_t *counts, void *stream) {
    if (!res) return VR_EINVAL;
    const int64_t n = res->n_vertices, K = res->n_edges;
    if (n < 0 || K < 0 || n > VR_MAX_POINTS) return VR_EINVAL;
    if (K == 0) return VR_OK;
    if (!counts || !res->edge_ij) return VR_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    int32_t *D = (int32_t *)cache_get((size_t)n * (size_t)n * 4, s);
    if (!D) return VR_ENOMEM;
    hipLaunchKernelGGL(k_pd_fill, dim3(grid_for(n * n)), dim3(PD_BLOCK), 0, s, D, n);
    hipLaunchKernelGGL(k_pd_edges, dim3(grid_for(K)), dim3(PD_BLOCK), 0, s, D, n, (const int32_t *)res->edge_ij, K, n);
    hipLaunchKernelGGL(k_tet_count, dim3((unsigned)(K < 65536 ? K : 65536)), dim3(PD_BLOCK), 0, s, (const int32_t *)D,
                       n, n, (const int32_t *)res->edge_ij, K, (long long *)counts);
    const hipError_t e = hipGetLastError();
    cache_put(D, s);
    return e == hipSuccess ? VR_OK : VR_EHIP;
}

// ------------------------------------------------ dimension 1, reduction ----
// Persistence pairs of dimension 1: Algorithm 1 (Section 2.2.1) on the
// anti-transpose of the boundary matrix, with clearing (Section 2.2.2), the
// edge columns taken from the youngest edge to the oldest.  In
// anti-transposed coordinates the column of edge r holds its cofacets (the
// triangles containing it) and its pivot is its oldest cofacet: the
// smallest key, since triangle keys (value << 39 | i << 26 | j << 13 | k)
// sort in filtration order.  Three kinds of column:
//   - cleared: an edge paired with a vertex (dimension 0) reduces to zero;
//   - apparent: an edge with triangles of its own value keeps its
//     coboundary, whose pivot is the first of them (a younger column holds
//     only triangles of larger values), so the two pair at once;
//   - the rest, reduced youngest first: while the working column (sorted
//     keys) is not empty, its pivot p is looked up; an apparent pivot adds
//     that edge's coboundary, the pivot of a column reduced before adds
//     that column, and a new pivot pairs the edge with p (a bar [r, value
//     of p)) and stores the column under p.  A column that empties is a
//     class born at r that never dies.  The columns are reduced in rounds,
//     all unsettled columns at once (k_rd_round, below).
// Additions are over F2: the symmetric difference of two sorted lists, a
// merge that drops the keys present in both.  Every addition removes the
// pivot and adds only larger keys, so the pivot grows and the loop ends.
#define RD_BLOCK 1024
#define RD_WAVES (RD_BLOCK / 64)
#define RD_GEN_MAX 8192                    // coboundary of one edge: at most n - 2 triangles
#define RD_POOL_ENTRIES (1ll << 27)        // stored columns and rewritten bases (keys)
#define RD_ACACHE_KEYS (1ll << 25)         // largest cache of apparent coboundaries (keys)
#define RD_WORK_ENTRIES (1ll << 22)        // one column (keys)
#define RD_EMPTY 0ull                      // no triangle key is 0 (its largest vertex is >= 2)

struct RdCtl {
    int32_t m;        // columns to reduce
    int32_t err;      // 1: stored columns outgrew the pool, 2: a working column outgrew its buffer
    long long ptop;   // pool entries taken
    int32_t next;     // a round's next unsettled column
    int32_t nh;       // columns left unsettled by a round
};

// A slot of the table of pivots: the key (RD_EMPTY: a free slot), its
// owner (column + 1; 0: none) and where the owner's stored version lies in
// the pool, and a round's first claimant (m - column; 0: none).
struct __attribute__((aligned(32))) RdSlot {
    unsigned long long key;
    uint32_t start, len;
    int32_t owner, claim;
    unsigned long long pad;
};
#define RD_SLOT_WORDS ((int64_t)(sizeof(RdSlot) / 8))  // 64-bit words a slot takes (the table is zeroed by words)
static_assert(sizeof(RdSlot) == 32, "a table slot is 32 bytes");

struct RdBufs {
    const int32_t *R;               // n x n ranks (+inf off the edges, -1 on the diagonal)
    const int32_t *ij;              // K edges (i, j)
    const unsigned long long *app;  // K: the key of edge r's apparent pivot, or RD_EMPTY
    const int32_t *rem;             // the columns to reduce, youngest first
    RdSlot *tab;                    // table of pivots
    long long hmask;                // table slots - 1 (a power of two, at least twice the columns)
    unsigned long long *pool;       // reduced columns, back to back
    long long *cstart;              // column ci: its keys start here in the pool
    int32_t *clen;                  //   and number this many
    unsigned long long *rkey;       // per column: its pivot, or RD_EMPTY for a class that never dies
    long long *cslot;               // per column: the slot of its claim in a round (-1: none)
    RdCtl *ctl;
    int64_t n, K;
    const unsigned long long *tri;  // dimension 2: the T triangle keys (the columns' simplices)
    int64_t T;
    // dimension 1, when the coboundaries are few enough: every apparent
    // edge's sorted coboundary, generated once (acache + astart[v], up to
    // astart[v + 1]); null otherwise
    const unsigned long long *acache;
    const long long *astart;
    // dimension 1: every vertex's kept edges as (rank << 16 | neighbour)
    // words, in neighbour order (nv) and in rank order (sr), from soff[v] to
    // soff[v + 1]; epos[2r + s] = the place of edge r in the rank order of
    // its lower (s = 0) or upper (s = 1) endpoint
    const unsigned long long *nv, *sr;
    const uint32_t *epos;
    const long long *soff;
};

// A table slot of dimension 2 whose length is RD_APP holds an apparent pair:
// its start is the triangle whose coboundary has that pivot.
#define RD_APP 0xFFFFFFFFu

// Columns to reduce: edges with neither a vertex (e_low) nor an apparent
// triangle (first), from the youngest down.  One work-group.
__global__ void __launch_bounds__(RD_BLOCK) k_rd_list(const int32_t *first, const int32_t *e_low, int64_t K,
                                                     int32_t *rem, RdCtl *ctl) {
    __shared__ uint32_t wc[RD_WAVES];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    uint32_t run = 0;
    for (int64_t base = K - 1; base >= 0; base -= RD_BLOCK) {
        const int64_t r = base - t;
        const bool keep = r >= 0 && first[r] < 0 && e_low[r] < 0;
        const unsigned long long b = __ballot(keep);
        if (lane == 0) wc[wv] = (uint32_t)__popcll(b);
        __syncthreads();
        uint32_t before = 0, tot = 0;
        for (int w = 0; w < RD_WAVES; w++) {
            if (w < wv) before += wc[w];
            tot += wc[w];
        }
        if (keep) rem[run + before + __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0))] = (int32_t)r;
        run += tot;
        __syncthreads();
    }
    if (t == 0) {
        ctl->m = (int32_t)run;
        ctl->err = 0;
        ctl->ptop = 0;
        ctl->next = 0;
        ctl->nh = 0;
    }
}

// app[r] = the key of the first triangle of value r when it pairs with edge
// r (an apparent pair), else RD_EMPTY: one load tells whether a pivot is
// apparent.
__global__ void __launch_bounds__(PD_BLOCK) k_rd_app(const int32_t *first, const unsigned long long *key, int64_t K,
                                                    unsigned long long *app) {
    for (int64_t r = blockIdx.x * (int64_t)PD_BLOCK + threadIdx.x; r < K; r += (int64_t)gridDim.x * PD_BLOCK) {
        const int32_t f = first[r];
        app[r] = f >= 0 ? key[f] : RD_EMPTY;
    }
}

__global__ void __launch_bounds__(PD_BLOCK) k_rd_zero(unsigned long long *p, int64_t m) {
    for (int64_t x = blockIdx.x * (int64_t)PD_BLOCK + threadIdx.x; x < m; x += (int64_t)gridDim.x * PD_BLOCK) p[x] = 0ull;
}

// Exclusive scan of one value per thread over the work-group; *total gets the sum.
static __device__ __forceinline__ uint32_t rd_scan(uint32_t x, uint32_t *sh, uint32_t *total) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) sh[wv] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int w = 0; w < RD_WAVES; w++) {
        const uint32_t v = sh[w];
        if (w < wv) before += v;
        tot += v;
    }
    __syncthreads();
    *total = tot;
    return before + inc - x;
}

static __device__ __forceinline__ unsigned long long rd_tri_key(uint32_t v, uint32_t a, uint32_t b, uint32_t c) {
    const uint32_t lo = min(a, min(b, c)), hi = max(a, max(b, c)), mid = a + b + c - lo - hi;
    return ((unsigned long long)v << 39) | ((unsigned long long)lo << 26) | ((unsigned long long)mid << 13) | hi;
}

// Order the LDS accesses of one wave (a bitonic stage whose partners lie
// within the wave's own elements needs no work-group barrier).
static __device__ __forceinline__ void rd_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

#define RD_SEG (VR_MAX_POINTS / RD_BLOCK)  // vertices per thread in rd_gen

static __device__ uint32_t rd_sort(unsigned long long *g, uint32_t run);

static __device__ __forceinline__ uint32_t rd_lower_bound(const unsigned long long *a, uint32_t n, unsigned long long x) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}


// The coboundary of edge e, sorted, into g (LDS); returns its length.  Each
// thread takes a run of at most RD_SEG consecutive vertices k (its loads
// all in flight at once), one scan places the keys, rd_sort sorts them.
// The keys of one stream of n0 items compacted in order into dst (LDS):
// key(x) is item x's key, or ~0 for none.  Each thread takes a run of at
// most RD_SEG consecutive items (n0 < VR_MAX_POINTS), so one scan places
// them.  Returns the count.
template <typename F>
static __device__ uint32_t rd_compact(uint32_t n0, unsigned long long *dst, uint32_t *sh, F key) {
    const uint32_t S = (n0 + RD_BLOCK - 1) / RD_BLOCK;
    const uint32_t x0 = (uint32_t)threadIdx.x * S;
    unsigned long long kv[RD_SEG];
    uint32_t c = 0;
#pragma unroll
    for (uint32_t u = 0; u < RD_SEG; u++) {
        kv[u] = ~0ull;
        if (u < S && x0 + u < n0) kv[u] = key(x0 + u);
        c += kv[u] != ~0ull ? 1u : 0u;
    }
    uint32_t tot;
    uint32_t at = rd_scan(c, sh, &tot);
#pragma unroll
    for (uint32_t u = 0; u < RD_SEG; u++)
        if (kv[u] != ~0ull) dst[at++] = kv[u];
    return tot;
}

// The coboundary of edge e = {a, b}, sorted, into g (LDS); returns its
// length.  No sort: the cofacets {a, b, k} of value e (both other edges
// older) come from a's edges in neighbour order, which is their order; a
// cofacet of larger value takes the value of its youngest edge, ak or bk,
// so the cofacets whose youngest edge is ak follow a's edges after e in
// rank order, those whose youngest edge is bk follow b's, and the two
// sorted runs are merged (each key placed by a binary search in the other
// run).
static __device__ uint32_t rd_gen_ab(const RdBufs &B, int64_t e, int32_t a, int32_t b, unsigned long long *g,
                                     uint32_t *sh) {
    const int t = threadIdx.x;
    const int32_t *Ra = B.R + (int64_t)a * B.n, *Rb = B.R + (int64_t)b * B.n;
    const long long oa = B.soff[a], ob = B.soff[b];
    const uint32_t da = (uint32_t)(B.soff[a + 1] - oa), db = (uint32_t)(B.soff[b + 1] - ob);
    const bool alo = a < b;
    const uint32_t pa = B.epos[2 * e + (alo ? 0 : 1)], pb = B.epos[2 * e + (alo ? 1 : 0)];
    const unsigned long long *nva = B.nv + oa, *sra = B.sr + oa + pa + 1, *srb = B.sr + ob + pb + 1;
    const int32_t E = (int32_t)e;
    // value e: ak and bk both older than e, in neighbour order
    const uint32_t c1 = rd_compact(da, g, sh, [&](uint32_t x) -> unsigned long long {
        const unsigned long long w = nva[x];
        const uint32_t k = (uint32_t)w & 0xFFFFu;
        if ((int32_t)(w >> 16) >= E) return ~0ull;
        return Rb[k] < E ? rd_tri_key((uint32_t)E, (uint32_t)a, (uint32_t)b, k) : ~0ull;
    });
    // youngest edge ak (after e in a's rank order), then youngest edge bk
    const uint32_t ca = rd_compact(da - pa - 1, g + c1, sh, [&](uint32_t x) -> unsigned long long {
        const unsigned long long w = sra[x];
        const uint32_t k = (uint32_t)w & 0xFFFFu;
        const int32_t r = (int32_t)(w >> 16), y = Rb[k];
        return (y != PD_INF && y < r) ? rd_tri_key((uint32_t)r, (uint32_t)a, (uint32_t)b, k) : ~0ull;
    });
    const uint32_t cb = rd_compact(db - pb - 1, g + c1 + ca, sh, [&](uint32_t x) -> unsigned long long {
        const unsigned long long w = srb[x];
        const uint32_t k = (uint32_t)w & 0xFFFFu;
        const int32_t r = (int32_t)(w >> 16), y = Ra[k];
        return (y != PD_INF && y < r) ? rd_tri_key((uint32_t)r, (uint32_t)a, (uint32_t)b, k) : ~0ull;
    });
    // merge the runs g[c1, c1 + ca) and g[c1 + ca, c1 + ca + cb) in place:
    // every key is read before any is written
    __syncthreads();
    const unsigned long long *A = g + c1, *Bq = g + c1 + ca;
    unsigned long long mv[RD_SEG];
    uint32_t md[RD_SEG];
    const uint32_t nm = ca + cb;
#pragma unroll
    for (uint32_t u = 0; u < RD_SEG; u++) {
        const uint32_t x = (uint32_t)t + u * RD_BLOCK;
        md[u] = ~0u;
        mv[u] = 0;
        if (x < nm) {
            const unsigned long long v = g[c1 + x];
            mv[u] = v;
            md[u] = x < ca ? x + rd_lower_bound(Bq, cb, v) : (x - ca) + rd_lower_bound(A, ca, v);
        }
    }
    __syncthreads();
#pragma unroll
    for (uint32_t u = 0; u < RD_SEG; u++)
        if (md[u] != ~0u) g[c1 + md[u]] = mv[u];
    __syncthreads();
    return c1 + nm;
}

// Sort the first run keys of g (LDS) in place; returns run.  Bitonic: in a
// stage of partner distance j <= 64 every wave reads and writes only its
// own 128-element blocks, so consecutive such stages need only the wave's
// own ordering.
static __device__ uint32_t rd_sort(unsigned long long *g, uint32_t run) {
    const int t = threadIdx.x;
    // padded to a power of two with the largest key
    uint32_t P = 1;
    while (P < run) P <<= 1;
    for (uint32_t x = run + t; x < P; x += RD_BLOCK) g[x] = ~0ull;
    __syncthreads();
    for (uint32_t kk = 2; kk <= P; kk <<= 1)
        for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
            for (uint32_t i = t; i < P / 2; i += RD_BLOCK) {
                const uint32_t lo = 2 * i - (i & (j - 1)), hi = lo + j;
                const unsigned long long x0 = g[lo], x1 = g[hi];
                if ((x0 > x1) == ((lo & kk) == 0)) {
                    g[lo] = x1;
                    g[hi] = x0;
                }
            }
            const uint32_t jn = j > 1 ? j >> 1 : kk;  // the next stage's distance
            if (j > 64 || jn > 64 || (j == 1 && kk == P)) __syncthreads();
            else rd_wave_sync();
        }
    return run;
}

static __device__ uint32_t rd_gen(const RdBufs &B, int64_t e, unsigned long long *g, uint32_t *sh) {
    return rd_gen_ab(B, e, B.ij[2 * e], B.ij[2 * e + 1], g, sh);
}

// Dimension 2.  A tetrahedron as a key of the reduction: w << 26 | c << 13
// | d, w its value (largest edge rank) and c < d its two vertices off edge
// w.  The tetrahedra of one value share that edge, and two 4-sets with two
// common vertices compare (sorted, lexicographically) as their other two
// vertices do, so these keys sort in filtration order.
static __device__ __forceinline__ unsigned long long rd_tet_key(int32_t w, uint32_t c, uint32_t d) {
    return ((unsigned long long)(uint32_t)w << 26) | ((unsigned long long)c << 13) | d;
}

// The cofacet t + {l} of triangle t = {i, j, k} (value v, m its vertex off
// its largest edge), given the ranks x, y, z of the edges il, jl, kl.
static __device__ __forceinline__ unsigned long long rd_cofacet(int32_t v, uint32_t i, uint32_t j, uint32_t k,
                                                                uint32_t m, uint32_t l, int32_t x, int32_t y,
                                                                int32_t z) {
    const int32_t w = max(v, max(x, max(y, z)));
    if (w == v) return rd_tet_key(w, min(m, l), max(m, l));  // the triangle's own largest edge
    if (w == x) return rd_tet_key(w, j, k);                  // edge il
    if (w == y) return rd_tet_key(w, i, k);                  // edge jl
    return rd_tet_key(w, i, j);                              // edge kl
}

// The coboundary of triangle tix (its cofacets t + {l}), sorted, into g.
static __device__ uint32_t rd_gen_tri(const RdBufs &B, int64_t tix, unsigned long long *g, uint32_t *sh) {
    const int t = threadIdx.x;
    const unsigned long long key = B.tri[tix];
    const int32_t v = (int32_t)(key >> 39);
    const uint32_t i = (uint32_t)(key >> 26) & 0x1FFFu, j = (uint32_t)(key >> 13) & 0x1FFFu, k = (uint32_t)key & 0x1FFFu;
    const int32_t *Ri = B.R + (int64_t)i * B.n, *Rj = B.R + (int64_t)j * B.n, *Rk = B.R + (int64_t)k * B.n;
    const uint32_t m = Ri[j] == v ? k : (Ri[k] == v ? j : i);
    const int S = (int)((B.n + RD_BLOCK - 1) / RD_BLOCK);
    const int l0 = t * S;
    unsigned long long kv[RD_SEG];
    bool ok[RD_SEG];
    uint32_t c = 0;
#pragma unroll
    for (int u = 0; u < RD_SEG; u++) {
        const int l = l0 + u;
        ok[u] = false;
        kv[u] = 0;
        if (u < S && l < B.n) {
            const int32_t x = Ri[l], y = Rj[l], z = Rk[l];
            if ((uint32_t)l != i && (uint32_t)l != j && (uint32_t)l != k && x != PD_INF && y != PD_INF &&
                z != PD_INF) {
                kv[u] = rd_cofacet(v, i, j, k, m, (uint32_t)l, x, y, z);
                ok[u] = true;
                c++;
            }
        }
    }
    uint32_t run;
    uint32_t at = rd_scan(c, sh, &run);
#pragma unroll
    for (int u = 0; u < RD_SEG; u++)
        if (ok[u]) g[at++] = kv[u];
    return rd_sort(g, run);
}

// dst = a + b over F2 (a, b sorted, without repeats); returns dst's length,
// or ~0u when it would not fit.  mrg holds the plain merge.
static __device__ uint32_t rd_add(const unsigned long long *a, uint32_t na, const unsigned long long *b, uint32_t nb,
                                  unsigned long long *mrg, unsigned long long *dst, uint32_t *sh) {
    const int t = threadIdx.x;
    const uint32_t L = na + nb;
    if ((long long)L > RD_WORK_ENTRIES) return ~0u;
    const uint32_t S = (L + RD_BLOCK - 1) / RD_BLOCK;
    const uint32_t d0 = min(L, (uint32_t)t * S), d1 = min(L, d0 + S);
    // merge path: a[i] goes before b[d - i] when a[i] <= b[d - i]
    uint32_t lo = d0 > nb ? d0 - nb : 0u, hi = min(d0, na);
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] <= b[d0 - 1 - mid]) lo = mid + 1;
        else hi = mid;
    }
    uint32_t i = lo, j = d0 - lo;
    for (uint32_t d = d0; d < d1; d++) {
        const bool take_a = j >= nb || (i < na && a[i] <= b[j]);
        mrg[d] = take_a ? a[i++] : b[j++];
    }
    __threadfence_block();
    __syncthreads();
    // a key in both lists sits twice in a row: drop both
    uint32_t c = 0;
    for (uint32_t d = d0; d < d1; d++) {
        const unsigned long long x = mrg[d];
        c += ((d == 0 || mrg[d - 1] != x) && (d + 1 == L || mrg[d + 1] != x)) ? 1u : 0u;
    }
    uint32_t tot;
    uint32_t o = rd_scan(c, sh, &tot);
    for (uint32_t d = d0; d < d1; d++) {
        const unsigned long long x = mrg[d];
        if ((d == 0 || mrg[d - 1] != x) && (d + 1 == L || mrg[d + 1] != x)) dst[o++] = x;
    }
    __threadfence_block();
    __syncthreads();
    return tot;
}

static __device__ __forceinline__ long long rd_slot(unsigned long long p, long long hmask) {
    return (long long)((p * 0x9E3779B97F4A7C15ull) >> 20) & hmask;
}

// The working column is kept in two parts whose sum (over F2) it is: a base
// list in global memory, of which the entries before a head index are gone,
// and a short delta list in LDS (at most RD_DCAP keys), also with a head.
// Additions go into the delta by a merge in LDS; only when the delta would
// overflow is it folded into the base, one pass over the base.  The pivot
// is the smallest key of the sum: the two heads, skipping keys present in
// both (they cancel).  A column of the essential class of the noisy circle
// takes 3537 additions and grows to 90 thousand keys, so re-merging the
// whole column at every addition would dominate.
#define RD_DCAP 4096


#define RD_SMP 2048  // keys of the base's sample in LDS

// dst = a + b over F2 for a sorted base a (global, na keys) and a sorted
// delta b (LDS, nb <= RD_DCAP keys); sc: LDS scratch of 2 RD_DCAP uint32,
// smp: LDS for RD_SMP keys.  Returns the length.  A delta key is matched
// when the base holds it (both vanish); an unmatched delta key b_j lands at
// pos_j + j - 2 M_j (pos_j: base keys below it, M_j: matched delta keys
// before it), an unmatched base key a_i at i + r - 2 M_r (r: delta keys
// below it).  The base's every 2^sh-th key is staged in LDS first (the
// whole base when it fits), so a delta key's place takes a search in LDS
// and at most sh steps in device memory.
#define RD_FOLD_U 4  // base keys per thread in flight in a fold
static __device__ uint32_t rd_fold(const unsigned long long *a, uint32_t na, const unsigned long long *b, uint32_t nb,
                                   unsigned long long *dst, uint32_t *sc, unsigned long long *smp, uint32_t *sh) {
    const int t = threadIdx.x;
    uint32_t *pos = sc, *minc = sc + RD_DCAP;  // minc[j]: matched delta keys in [0, j]
    uint32_t lg = 0;
    while (((size_t)RD_SMP << lg) < na) lg++;
    const uint32_t ns = (na + (1u << lg) - 1) >> lg;  // <= RD_SMP
    for (uint32_t q = t; q < ns; q += RD_BLOCK) smp[q] = a[(size_t)q << lg];
    __syncthreads();
    uint32_t mloc[RD_DCAP / RD_BLOCK], cnt = 0;
#pragma unroll
    for (int u = 0; u < RD_DCAP / RD_BLOCK; u++) {
        const uint32_t j = (uint32_t)t * (RD_DCAP / RD_BLOCK) + u;
        mloc[u] = 0;
        if (j < nb) {
            const unsigned long long x = b[j];
            // first sample >= x, then the keys between it and the sample before
            const uint32_t qs = rd_lower_bound(smp, ns, x);
            uint32_t lo = qs ? ((qs - 1) << lg) + 1 : 0u, hi = qs < ns ? qs << lg : na;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (a[mid] < x) lo = mid + 1;
                else hi = mid;
            }
            pos[j] = lo;
            const bool on = lo < na && ((lo & ((1u << lg) - 1)) ? a[lo] : smp[lo >> lg]) == x;
            mloc[u] = on ? 1u : 0u;
        }
        cnt += mloc[u];
    }
    uint32_t tot;
    uint32_t run = rd_scan(cnt, sh, &tot);
#pragma unroll
    for (int u = 0; u < RD_DCAP / RD_BLOCK; u++) {
        const uint32_t j = (uint32_t)t * (RD_DCAP / RD_BLOCK) + u;
        run += mloc[u];
        if (j < nb) minc[j] = run;
    }
    __syncthreads();
    for (uint32_t j = t; j < nb; j += RD_BLOCK) {
        const uint32_t mex = j ? minc[j - 1] : 0u;
        if (minc[j] == mex) dst[pos[j] + j - 2 * mex] = b[j];
    }
    // the base's keys, RD_FOLD_U per thread at a time: their loads issued
    // together, then their places in the delta found in lockstep (a
    // fixed-step lower bound, the U searches' LDS reads interleaved)
    uint32_t pw = 1;
    while (pw <= nb) pw <<= 1;
    for (uint32_t i0 = t; i0 < na; i0 += RD_BLOCK * RD_FOLD_U) {
        unsigned long long y[RD_FOLD_U];
        uint32_t lo[RD_FOLD_U];
#pragma unroll
        for (int u = 0; u < RD_FOLD_U; u++) {
            const uint32_t i = i0 + (uint32_t)u * RD_BLOCK;
            y[u] = i < na ? (lg ? a[i] : smp[i]) : 0ull;
            lo[u] = 0;
        }
        for (uint32_t step = pw >> 1; step > 0; step >>= 1) {
#pragma unroll
            for (int u = 0; u < RD_FOLD_U; u++) {
                const uint32_t c = lo[u] + step;  // lo[u] = keys of b below y[u] so far
                if (c <= nb && b[c - 1] < y[u]) lo[u] = c;
            }
        }
#pragma unroll
        for (int u = 0; u < RD_FOLD_U; u++) {
            const uint32_t i = i0 + (uint32_t)u * RD_BLOCK;
            if (i >= na || (lo[u] < nb && b[lo[u]] == y[u])) continue;
            const uint32_t mex = lo[u] ? minc[lo[u] - 1] : 0u;
            dst[i + lo[u] - 2 * mex] = y[u];
        }
    }
    __threadfence_block();
    __syncthreads();
    return na + nb - 2 * tot;
}

// o = d + x over F2 in LDS (d: nd keys in LDS, x: nx keys, LDS or global;
// nd + nx <= RD_DCAP); returns the length.  Merge path, then the keys in
// both lists (adjacent after the merge) are dropped in place.
static __device__ uint32_t rd_delta_add(const unsigned long long *d, uint32_t nd, const unsigned long long *x, uint32_t nx,
                                        unsigned long long *o, uint32_t *sh) {
    const int t = threadIdx.x;
    constexpr uint32_t S = RD_DCAP / RD_BLOCK;
    const uint32_t L = nd + nx;
    const uint32_t d0 = min(L, (uint32_t)t * S), d1 = min(L, d0 + S);
    uint32_t lo = d0 > nx ? d0 - nx : 0u, hi = min(d0, nd);
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (d[mid] <= x[d0 - 1 - mid]) lo = mid + 1;
        else hi = mid;
    }
    uint32_t i = lo, j = d0 - lo;
    for (uint32_t q = d0; q < d1; q++) {
        const bool take_d = j >= nx || (i < nd && d[i] <= x[j]);
        o[q] = take_d ? d[i++] : x[j++];
    }
    __syncthreads();
    unsigned long long v[S];
    bool keep[S];
    uint32_t c = 0;
#pragma unroll
    for (uint32_t u = 0; u < S; u++) {
        const uint32_t q = d0 + u;
        keep[u] = false;
        v[u] = 0;
        if (q < d1) {
            v[u] = o[q];
            keep[u] = (q == 0 || o[q - 1] != v[u]) && (q + 1 == L || o[q + 1] != v[u]);
        }
        c += keep[u] ? 1u : 0u;
    }
    uint32_t tot;
    uint32_t at = rd_scan(c, sh, &tot);  // its barriers also end every read of o above
#pragma unroll
    for (uint32_t u = 0; u < S; u++)
        if (keep[u]) o[at++] = v[u];
    __syncthreads();
    return tot;
}

// The coboundary of column simplex id: an edge (DIM 1) or a triangle (DIM 2).
template <int DIM>
static __device__ __forceinline__ uint32_t rd_gen_col(const RdBufs &B, int64_t id, unsigned long long *g,
                                                      uint32_t *sh) {
    if constexpr (DIM == 1) return rd_gen(B, id, g, sh);
    else return rd_gen_tri(B, id, g, sh);
}

// Dimension 2: the apparent partner of pivot p, from 64 table slots read at
// once by the calling wave (every lane gets it); -1 when p is no apparent
// pivot.
static __device__ __forceinline__ int32_t rd_app2(const RdBufs &B, unsigned long long p) {
    const int lane = threadIdx.x & 63;
    long long sl = rd_slot(p, B.hmask);
    for (;;) {
        const RdSlot q = B.tab[(sl + lane) & B.hmask];
        const unsigned long long stop = __ballot(q.key == p || q.key == RD_EMPTY);
        if (!stop) {
            sl += 64;
            continue;
        }
        const int f = __builtin_ctzll(stop);
        const bool hit = __shfl(q.key, f, 64) == p && __shfl(q.len, f, 64) == RD_APP;
        return hit ? (int32_t)__shfl(q.start, f, 64) : -1;
    }
}

// The reduction in rounds.  A column may add any stored version of a column
// before it (a younger simplex, reduced earlier in the order): that is a
// column operation of Algorithm 1, and the pairs of a reduced matrix do not
// depend on which operations reached it.  So every unsettled column is
// reduced at once against a table that does not change during the round:
// while its pivot is apparent (that coboundary is added) or owned by a
// column before it (that column's stored version is added); it stops at a
// pivot owned by nobody or by a column after it.  Then each pivot's
// claimants are settled: the first column claiming it owns it (a later
// former owner is displaced), the others stay unsettled.  The first
// unsettled column meets only settled owners before it, so it reduces as
// in the serial algorithm and wins: every round settles at least one
// column, and in practice nearly all (3 to 5 rounds on 300- to 1000-point
// clouds).  Round 0 is the pass over every column's coboundary.
//
// Column c's state: its stored version (cstart, clen; clen -1: not yet
// generated) and pivot (rkey; RD_EMPTY once it reduced to zero).  Stored
// versions are immutable: every new version, and every rewritten base,
// goes to a fresh stretch of the pool.  Table slot of pivot p: the owner
// (column + 1, 0: none) with its stored version (start, len), and this
// round's first claimant (m - column, 0: none).

// n keys from the pool for the work-group; -1 (and the error flagged) when
// the pool is full.
static __device__ long long rd_alloc(const RdBufs &B, uint32_t n, long long *s_off) {
    if (threadIdx.x == 0) {
        long long off = (long long)atomicAdd((unsigned long long *)&B.ctl->ptop, (unsigned long long)n);
        if (off + (long long)n > RD_POOL_ENTRIES) {
            off = -1;
            B.ctl->err = 1;
        }
        *s_off = off;
    }
    __syncthreads();
    const long long off = *s_off;
    __syncthreads();
    return off;
}

template <int DIM>
__global__ void __launch_bounds__(RD_BLOCK) k_rd_round(RdBufs B, const int32_t *H, int32_t nH) {
    __shared__ unsigned long long g[RD_GEN_MAX];
    __shared__ unsigned long long dl[2][RD_DCAP];
    __shared__ unsigned long long smp[RD_SMP];
    __shared__ uint32_t sh[RD_WAVES];
    __shared__ int32_t s_act, s_hx;
    __shared__ uint32_t s_h, s_dh, s_a0, s_a1, s_a2;
    __shared__ unsigned long long s_piv;
    __shared__ long long s_off;
    const int t = threadIdx.x;
    for (;;) {
        if (t == 0) s_hx = atomicAdd(&B.ctl->next, 1);
        __syncthreads();
        const int32_t hx = s_hx;
        __syncthreads();
        if (hx >= nH) break;
        const int32_t c = H[hx];
        // the base (global, entries before h gone) and the delta (LDS)
        const unsigned long long *bp = B.pool;
        int dc = 0;
        uint32_t nw = 0, h = 0, nd = 0, dh = 0;
        bool dirty = false, fail = false;
        const int32_t cl = B.clen[c];
        if (cl >= 0) {
            bp = B.pool + B.cstart[c];
            nw = (uint32_t)cl;
        } else {
            dirty = true;
            const uint32_t len = rd_gen_col<DIM>(B, B.rem[c], g, sh);
            if (len <= RD_DCAP) {
                for (uint32_t x = t; x < len; x += RD_BLOCK) dl[0][x] = g[x];
                nd = len;
            } else {
                const long long off = rd_alloc(B, len, &s_off);
                if (off < 0) {
                    fail = true;
                } else {
                    for (uint32_t x = t; x < len; x += RD_BLOCK) B.pool[off + x] = g[x];
                    bp = B.pool + off;
                    nw = len;
                }
            }
            __threadfence_block();
            __syncthreads();
        }
        while (!fail) {
            if (t < 64) {
                // the pivot: the smaller head, keys in both heads cancelling
                // (64 head pairs compared at a time)
                const int lane = t;
                unsigned long long p = 0;
                bool any = false;
                for (;;) {
                    const bool ha = h + lane < nw, hb = dh + lane < nd;
                    const unsigned long long ya = ha ? bp[h + lane] : ~0ull, yb = hb ? dl[dc][dh + lane] : ~0ull;
                    const unsigned long long diff = __ballot(!(ha && hb && ya == yb));
                    if (!diff) {
                        h += 64;
                        dh += 64;
                        continue;
                    }
                    const int f = __builtin_ctzll(diff);
                    h += f;
                    dh += f;
                    p = min(__shfl(ya, f, 64), __shfl(yb, f, 64));
                    any = h < nw || dh < nd;
                    break;
                }
                // 0: reduced to zero; 1: add the coboundary of simplex a0
                // (an edge {a1, a2} in dimension 1); 2: add the stored column
                // of a1 keys at a0; 3: stop at pivot p.  The apparent key,
                // the edge's endpoints and 64 table slots load at once.
                int32_t act = 0;
                uint32_t a0 = 0, a1 = 0, a2 = 0;
                if (any) {
                    const int64_t v = (int64_t)(p >> 39);
                    unsigned long long ap = RD_EMPTY;
                    int32_t ea = 0, eb = 0;
                    if (DIM == 1 && lane == 0 && v < B.K) {
                        ap = B.app[v];
                        ea = B.ij[2 * v];
                        eb = B.ij[2 * v + 1];
                    }
                    long long sl = rd_slot(p, B.hmask);
                    act = 3;
                    for (;;) {
                        const RdSlot q = B.tab[(sl + lane) & B.hmask];
                        const unsigned long long stop = __ballot(q.key == p || q.key == RD_EMPTY);
                        if (!stop) {
                            sl += 64;
                            continue;
                        }
                        const int f = __builtin_ctzll(stop);
                        if (__shfl(q.key, f, 64) == p) {
                            const uint32_t qs = __shfl(q.start, f, 64), ql = __shfl(q.len, f, 64);
                            const int32_t owner = __shfl(q.owner, f, 64) - 1;
                            if (DIM == 2 && ql == RD_APP) {
                                act = 1;  // an apparent pair's triangle
                                a0 = qs;
                            } else if (owner >= 0 && owner < c) {
                                act = 2;
                                a0 = qs;
                                a1 = ql;
                            }
                        }
                        break;
                    }
                    if (DIM == 1 && __shfl(ap, 0, 64) == p) {
                        act = 1;
                        a0 = (uint32_t)v;
                        a1 = (uint32_t)__shfl(ea, 0, 64);
                        a2 = (uint32_t)__shfl(eb, 0, 64);
                    }
                }
                if (lane == 0) {
                    s_act = act;
                    s_a0 = a0;
                    s_a1 = a1;
                    s_a2 = a2;
                    s_piv = p;
                    s_h = h;
                    s_dh = dh;
                }
            }
            __syncthreads();
            const int32_t act = s_act;
            const uint32_t a0 = s_a0, a1 = s_a1, a2 = s_a2;
            const unsigned long long p = s_piv;
            h = s_h;
            dh = s_dh;
            __syncthreads();
            if (act == 0) {
                if (t == 0) {
                    B.rkey[c] = RD_EMPTY;
                    B.clen[c] = 0;
                }
                break;
            }
            if (act == 3) {
                if (dirty) {
                    // store the new version (base + delta) in the pool
                    const long long off = rd_alloc(B, (nw - h) + (nd - dh), &s_off);
                    if (off < 0) break;
                    const uint32_t len =
                        rd_fold(bp + h, nw - h, dl[dc] + dh, nd - dh, B.pool + off, (uint32_t *)dl[dc ^ 1], smp, sh);
                    if (t == 0) {
                        B.cstart[c] = off;
                        B.clen[c] = (int32_t)len;
                    }
                }
                if (t == 0) B.rkey[c] = p;
                break;
            }
            dirty = true;
            // the column to add: a coboundary or a stored column, in g
            const unsigned long long *x = g;
            uint32_t nx;
            if (act == 1 && (DIM == 2 || !B.acache)) {
                if constexpr (DIM == 1) nx = rd_gen_ab(B, a0, (int32_t)a1, (int32_t)a2, g, sh);
                else nx = rd_gen_tri(B, a0, g, sh);
            } else {
                // a stored column, or an apparent edge's cached coboundary
                const unsigned long long *src = B.pool + a0;
                nx = a1;
                if (act == 1) {
                    const long long o = B.astart[a0];
                    src = B.acache + o;
                    nx = (uint32_t)(B.astart[a0 + 1] - o);
                }
                if (nx <= RD_DCAP) {
                    for (uint32_t y = t; y < nx; y += RD_BLOCK) g[y] = src[y];
                    __syncthreads();
                } else {
                    x = src;
                }
            }
            if ((nd - dh) + nx > RD_DCAP) {
                // fold the delta into a new base first
                const long long off = rd_alloc(B, (nw - h) + (nd - dh), &s_off);
                if (off < 0) break;
                nw = rd_fold(bp + h, nw - h, dl[dc] + dh, nd - dh, B.pool + off, (uint32_t *)dl[dc ^ 1], smp, sh);
                bp = B.pool + off;
                h = 0;
                nd = dh = 0;
            }
            if (nx <= RD_DCAP) {
                nd = rd_delta_add(dl[dc] + dh, nd - dh, x, nx, dl[dc ^ 1], sh);
                dc ^= 1;
                dh = 0;
            } else {
                // a column longer than the delta goes straight into the base
                const uint32_t L = (nw - h) + nx;
                const long long off = rd_alloc(B, 2 * L, &s_off);  // the merge, then the sum
                if (off < 0) break;
                const uint32_t nl = rd_add(bp + h, nw - h, x, nx, B.pool + off, B.pool + off + L, sh);
                if (nl == ~0u) {
                    if (t == 0) B.ctl->err = 2;
                    break;
                }
                bp = B.pool + off + L;
                nw = nl;
                h = 0;
            }
        }
        __syncthreads();  // LDS is reused by the next column
    }
}

// Dimension 1: each vertex's kept edges from its row of the rank matrix,
// in neighbour order (nv) and, sorted, in rank order (sr), with every
// edge's places in its endpoints' rank orders (epos).  soff[v] = the
// vertex's degree first (k_st_deg), then its start (after a scan).
__global__ void __launch_bounds__(PD_BLOCK) k_st_deg(const int32_t *R, int64_t n, long long *soff) {
    __shared__ uint32_t sw[PD_BLOCK / 64];
    const int t = threadIdx.x;
    const int32_t *row = R + (int64_t)blockIdx.x * n;
    uint32_t c = 0;
    for (int64_t k = t; k < n; k += PD_BLOCK) c += (k != (int64_t)blockIdx.x && row[k] != PD_INF) ? 1u : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((t & 63) == 0) sw[t >> 6] = c;
    __syncthreads();
    if (t == 0) {
        uint32_t d = 0;
        for (int w = 0; w < PD_BLOCK / 64; w++) d += sw[w];
        soff[blockIdx.x] = d;
    }
}

__global__ void __launch_bounds__(RD_BLOCK) k_st_fill(RdBufs B, unsigned long long *nv, unsigned long long *sr,
                                                     uint32_t *epos) {
    __shared__ unsigned long long g[RD_GEN_MAX];
    __shared__ uint32_t sh[RD_WAVES];
    const int64_t v = blockIdx.x;
    const int32_t *row = B.R + v * B.n;
    const long long o = B.soff[v];
    const uint32_t deg = rd_compact((uint32_t)B.n, g, sh, [&](uint32_t k) -> unsigned long long {
        const int32_t r = row[k];
        return ((int64_t)k != v && r != PD_INF) ? (((unsigned long long)(uint32_t)r << 16) | k) : ~0ull;
    });
    __syncthreads();
    for (uint32_t x = threadIdx.x; x < deg; x += RD_BLOCK) nv[o + x] = g[x];
    rd_sort(g, deg);  // its first barrier ends the reads above
    for (uint32_t x = threadIdx.x; x < deg; x += RD_BLOCK) {
        const unsigned long long w = g[x];
        const uint32_t k = (uint32_t)w & 0xFFFFu;
        sr[o + x] = w;
        epos[2 * (w >> 16) + ((int64_t)k > v ? 0 : 1)] = x;
    }
}

// Dimension 1, coboundaries of the apparent edges generated ahead, all at
// once: a chain of additions (the essential class of a noisy circle takes
// thousands, one after the other) then copies each from device memory
// instead of generating and sorting it.  alen[v] = the size of apparent edge
// v's coboundary (its common neighbours), 0 for the other edges; one wave
// per edge.
__global__ void __launch_bounds__(PD_BLOCK) k_rd_acount(RdBufs B, long long *alen) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t v = blockIdx.x * (int64_t)(PD_BLOCK / 64) + wv; v < B.K; v += (int64_t)gridDim.x * (PD_BLOCK / 64)) {
        if (B.app[v] == RD_EMPTY) {
            if (lane == 0) alen[v] = 0;
            continue;
        }
        const int32_t a = B.ij[2 * v], b = B.ij[2 * v + 1];
        const int32_t *Ra = B.R + (int64_t)a * B.n, *Rb = B.R + (int64_t)b * B.n;
        uint32_t cnt = 0;
        for (int64_t k0 = 0; k0 < B.n; k0 += 64) {
            const int64_t k = k0 + lane;
            const bool ok = k < B.n && k != a && k != b && Ra[k] != PD_INF && Rb[k] != PD_INF;
            cnt += (uint32_t)__popcll(__ballot(ok));
        }
        if (lane == 0) alen[v] = cnt;
    }
}

// The apparent edges' coboundaries into the cache (astart: the scanned
// sizes), one work-group per edge at a time.
__global__ void __launch_bounds__(RD_BLOCK) k_rd_agen(RdBufs B, unsigned long long *cache) {
    __shared__ unsigned long long g[RD_GEN_MAX];
    __shared__ uint32_t sh[RD_WAVES];
    for (int64_t v = blockIdx.x; v < B.K; v += gridDim.x) {
        const long long o = B.astart[v], len = B.astart[v + 1] - o;
        if (len == 0) continue;
        const uint32_t nx = rd_gen(B, v, g, sh);
        for (uint32_t x = threadIdx.x; x < nx; x += RD_BLOCK) cache[o + x] = g[x];
        __syncthreads();  // g is rewritten by the next edge
    }
}

// First round's input: every column unsettled, none generated.
__global__ void __launch_bounds__(PD_BLOCK) k_rd_init(RdBufs B, int32_t *H) {
    const int32_t m = B.ctl->m;
    for (int64_t x = blockIdx.x * (int64_t)PD_BLOCK + threadIdx.x; x < m; x += (int64_t)gridDim.x * PD_BLOCK) {
        H[x] = (int32_t)x;
        B.clen[x] = -1;
    }
}

__global__ void k_rd_reset(RdCtl *ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->next = 0;
        ctl->nh = 0;
    }
}

// Claims: each unsettled column with a pivot finds (or inserts) its slot
// and records itself as a claimant; the first column keeps the largest m - c.
__global__ void __launch_bounds__(PD_BLOCK) k_rd_claim(RdBufs B, const int32_t *H, int32_t nH) {
    const int32_t m = B.ctl->m;
    for (int64_t x = blockIdx.x * (int64_t)PD_BLOCK + threadIdx.x; x < nH; x += (int64_t)gridDim.x * PD_BLOCK) {
        const int32_t c = H[x];
        const unsigned long long p = B.rkey[c];
        if (p == RD_EMPTY) {
            B.cslot[c] = -1;
            continue;
        }
        long long sl = rd_slot(p, B.hmask);
        for (;; sl = (sl + 1) & B.hmask) {
            const unsigned long long q = atomicCAS((unsigned long long *)&B.tab[sl].key, RD_EMPTY, p);
            if (q == RD_EMPTY || q == p) break;
        }
        atomicMax(&B.tab[sl].claim, m - c);
        B.cslot[c] = sl;
    }
}

// The first claimant of each pivot owns it (with its stored version); a
// former owner, after it in the order, is displaced; the other claimants
// and the displaced owners form the next round's unsettled columns.
__global__ void __launch_bounds__(PD_BLOCK) k_rd_win(RdBufs B, const int32_t *H, int32_t nH, int32_t *Hn) {
    const int32_t m = B.ctl->m;
    for (int64_t x = blockIdx.x * (int64_t)PD_BLOCK + threadIdx.x; x < nH; x += (int64_t)gridDim.x * PD_BLOCK) {
        const int32_t c = H[x];
        const long long sl = B.cslot[c];
        if (sl < 0) continue;  // reduced to zero: settled
        RdSlot &q = B.tab[sl];
        if (q.claim == m - c) {
            const int32_t o = q.owner - 1;
            if (o >= 0) Hn[atomicAdd(&B.ctl->nh, 1)] = o;
            q.owner = c + 1;
            q.start = (uint32_t)B.cstart[c];
            q.len = (uint32_t)B.clen[c];
        } else {
            Hn[atomicAdd(&B.ctl->nh, 1)] = c;
        }
    }
}

__global__ void __launch_bounds__(PD_BLOCK) k_rd_unclaim(RdBufs B, const int32_t *H, int32_t nH) {
    for (int64_t x = blockIdx.x * (int64_t)PD_BLOCK + threadIdx.x; x < nH; x += (int64_t)gridDim.x * PD_BLOCK) {
        const long long sl = B.cslot[H[x]];
        if (sl >= 0) B.tab[sl].claim = 0;
    }
}

// The rounds, from the host: reads m, then after each round the number of
// unsettled columns and the error word (one synchronisation per round).
// H0, H1: m entries each.  Returns VR_OK, VR_ENOMEM or VR_EHIP.
template <int DIM>
static int rd_run(RdBufs &B, int32_t *H0, int32_t *H1, hipStream_t s) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return VR_EHIP;
    RdCtl hc{};
    if (hipMemcpyAsync(&hc, B.ctl, sizeof(hc), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return VR_EHIP;
    const int32_t m = hc.m;
    if (m == 0) return VR_OK;
    hipLaunchKernelGGL(k_rd_init, dim3(grid_for(m)), dim3(PD_BLOCK), 0, s, B, H0);
    int32_t *H = H0, *Hn = H1;
    int32_t nH = m;
    for (int32_t round = 0; nH > 0; round++) {
        if (round > m) return VR_EHIP;  // every round settles a column
        hipLaunchKernelGGL(k_rd_reset, dim3(1), dim3(64), 0, s, B.ctl);
        hipLaunchKernelGGL((k_rd_round<DIM>), dim3((unsigned)(nH < cus ? nH : cus)), dim3(RD_BLOCK), 0, s, B,
                           (const int32_t *)H, nH);
        hipLaunchKernelGGL(k_rd_claim, dim3(grid_for(nH)), dim3(PD_BLOCK), 0, s, B, (const int32_t *)H, nH);
        hipLaunchKernelGGL(k_rd_win, dim3(grid_for(nH)), dim3(PD_BLOCK), 0, s, B, (const int32_t *)H, nH, Hn);
        hipLaunchKernelGGL(k_rd_unclaim, dim3(grid_for(nH)), dim3(PD_BLOCK), 0, s, B, (const int32_t *)H, nH);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(&hc, B.ctl, sizeof(hc), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return VR_EHIP;
        if (hc.err) return VR_ENOMEM;
        nH = hc.nh;
        int32_t *tmp = H;
        H = Hn;
        Hn = tmp;
    }
    return VR_OK;
}

// tri_of_edge[rem[ci]] = the index of column ci's pivot among the keys
__global__ void __launch_bounds__(PD_BLOCK) k_rd_emit(const unsigned long long *key, int64_t T, const int32_t *rem,
                                                     const unsigned long long *rkey, const RdCtl *ctl,
                                                     int32_t *tri_of_edge) {
    const int32_t m = ctl->m;
    for (int64_t ci = blockIdx.x * (int64_t)PD_BLOCK + threadIdx.x; ci < m; ci += (int64_t)gridDim.x * PD_BLOCK) {
        const unsigned long long p = rkey[ci];
        if (p == RD_EMPTY) continue;
        int64_t lo = 0, hi = T;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (key[mid] < p) lo = mid + 1;
            else hi = mid;
        }
        if (lo < T && key[lo] == p) tri_of_edge[rem[ci]] = (int32_t)lo;
    }
}

extern "C" VR_API int vr_pairs_dim1(const vr_result *res, const int32_t *e_low, int32_t *tri_of_edge, void *stream) {
    if (!res) return VR_EINVAL;
    const int64_t n = res->n_vertices, K = res->n_edges, T = res->n_triangles;
    if (n < 0 || K < 0 || T < 0 || n > VR_MAX_POINTS || T > 0x7FFFFFFF) return VR_EINVAL;
    if (K == 0) return VR_OK;
    if (!tri_of_edge || !e_low || !res->edge_ij || (T > 0 && !res->tri_key)) return VR_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_pd_clear, dim3(grid_for(K)), dim3(PD_BLOCK), 0, s, tri_of_edge, K);
    if (T == 0) return hipGetLastError() == hipSuccess ? VR_OK : VR_EHIP;  // no triangles: nothing dies
    hipLaunchKernelGGL(k_pd_apparent, dim3(grid_for(T)), dim3(PD_BLOCK), 0, s, (const unsigned long long *)res->tri_key,
                       T, tri_of_edge, K);
    // scratch, from the library's cache
    long long H = 2;
    while (H < 2 * K) H <<= 1;
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t o = 0;
    const size_t o_R = o; o = up(o + 4 * (size_t)n * (size_t)n);
    const size_t o_rem = o; o = up(o + 4 * (size_t)K);
    const size_t o_tab = o; o = up(o + sizeof(RdSlot) * (size_t)H);
    const size_t o_app = o; o = up(o + 8 * (size_t)K);
    const size_t o_pool = o; o = up(o + 8 * (size_t)RD_POOL_ENTRIES);
    const size_t o_cst = o; o = up(o + 8 * (size_t)K);
    const size_t o_cln = o; o = up(o + 4 * (size_t)K);
    const size_t o_rkey = o; o = up(o + 8 * (size_t)K);
    const size_t o_cslot = o; o = up(o + 8 * (size_t)K);
    const size_t o_h0 = o; o = up(o + 4 * (size_t)K);
    const size_t o_h1 = o; o = up(o + 4 * (size_t)K);
    const size_t o_ctl = o; o = up(o + sizeof(RdCtl));
    // the apparent edges' coboundaries hold at most 3 T keys (a triangle
    // lies in three edges' coboundaries): generated ahead when that fits
    const bool acache = 3 * T <= RD_ACACHE_KEYS;
    const size_t o_alen = o; o = up(o + (acache ? 8 * (size_t)(K + 1) : 0));
    const size_t o_acache = o; o = up(o + (acache ? 8 * (size_t)(3 * T) : 0));
    // every vertex's edges in neighbour and in rank order, for the generator
    const size_t o_soff = o; o = up(o + 8 * (size_t)(n + 1));
    const size_t o_nv = o; o = up(o + 16 * (size_t)K);
    const size_t o_sr = o; o = up(o + 16 * (size_t)K);
    const size_t o_epos = o; o = up(o + 8 * (size_t)K);
    char *ws = (char *)cache_get(o, s);
    if (!ws) return VR_ENOMEM;
    RdBufs B{};
    B.R = (const int32_t *)(ws + o_R);
    B.ij = (const int32_t *)res->edge_ij;
    B.app = (const unsigned long long *)(ws + o_app);
    B.rem = (const int32_t *)(ws + o_rem);
    B.tab = (RdSlot *)(ws + o_tab);
    B.hmask = H - 1;
    B.pool = (unsigned long long *)(ws + o_pool);
    B.cstart = (long long *)(ws + o_cst);
    B.clen = (int32_t *)(ws + o_cln);
    B.rkey = (unsigned long long *)(ws + o_rkey);
    B.cslot = (long long *)(ws + o_cslot);
    B.ctl = (RdCtl *)(ws + o_ctl);
    B.n = n;
    B.K = K;
    hipLaunchKernelGGL(k_rd_list, dim3(1), dim3(RD_BLOCK), 0, s, (const int32_t *)tri_of_edge, e_low, K,
                       (int32_t *)(ws + o_rem), B.ctl);
    hipLaunchKernelGGL(k_pd_fill, dim3(grid_for(n * n)), dim3(PD_BLOCK), 0, s, (int32_t *)(ws + o_R), n);
    hipLaunchKernelGGL(k_pd_edges, dim3(grid_for(K)), dim3(PD_BLOCK), 0, s, (int32_t *)(ws + o_R), n,
                       (const int32_t *)res->edge_ij, K, n);
    hipLaunchKernelGGL(k_rd_zero, dim3(grid_for(RD_SLOT_WORDS * H)), dim3(PD_BLOCK), 0, s, (unsigned long long *)B.tab,
                       RD_SLOT_WORDS * H);
    hipLaunchKernelGGL(k_rd_app, dim3(grid_for(K)), dim3(PD_BLOCK), 0, s, (const int32_t *)tri_of_edge,
                       (const unsigned long long *)res->tri_key, K, (unsigned long long *)(ws + o_app));
    {
        long long *soff = (long long *)(ws + o_soff);
        hipLaunchKernelGGL(k_st_deg, dim3((unsigned)n), dim3(PD_BLOCK), 0, s, B.R, n, soff);
        hipLaunchKernelGGL(k_tet_scan, dim3(1), dim3(1024), 0, s, soff, n);  // degrees -> starts
        B.soff = soff;
        hipLaunchKernelGGL(k_st_fill, dim3((unsigned)n), dim3(RD_BLOCK), 0, s, B, (unsigned long long *)(ws + o_nv),
                           (unsigned long long *)(ws + o_sr), (uint32_t *)(ws + o_epos));
        B.nv = (const unsigned long long *)(ws + o_nv);
        B.sr = (const unsigned long long *)(ws + o_sr);
        B.epos = (const uint32_t *)(ws + o_epos);
    }
    if (acache) {
        long long *alen = (long long *)(ws + o_alen);
        const int64_t wblocks = (K + PD_BLOCK / 64 - 1) / (PD_BLOCK / 64);
        hipLaunchKernelGGL(k_rd_acount, dim3((unsigned)(wblocks < 65536 ? wblocks : 65536)), dim3(PD_BLOCK), 0, s, B,
                           alen);
        hipLaunchKernelGGL(k_tet_scan, dim3(1), dim3(1024), 0, s, alen, K);  // sizes -> starts, alen[K] = total
        B.astart = alen;
        B.acache = (const unsigned long long *)(ws + o_acache);
        hipLaunchKernelGGL(k_rd_agen, dim3((unsigned)(K < 2048 ? K : 2048)), dim3(RD_BLOCK), 0, s, B,
                           (unsigned long long *)(ws + o_acache));
    }
    const int st = rd_run<1>(B, (int32_t *)(ws + o_h0), (int32_t *)(ws + o_h1), s);
    if (st == VR_OK)
        hipLaunchKernelGGL(k_rd_emit, dim3(grid_for(K)), dim3(PD_BLOCK), 0, s, (const unsigned long long *)res->tri_key,
                           T, (const int32_t *)(ws + o_rem), (const unsigned long long *)B.rkey, (const RdCtl *)B.ctl,
                           tri_of_edge);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    cache_put(ws, s);
    if (st != VR_OK) return st;
    return e == hipSuccess ? VR_OK : VR_EHIP;
}

// ------------------------------------------------------------ barcode ----
// Bars of dimensions 0 and 1 from the pairs (birth, death in filtration
// values: -1 for vertices, the rank for edges, the value for triangles;
// death INT64_MAX for a class that never dies), as (dimension, birth,
// death) int64 triples: bars[0, n) = dimension 0 (an edge r paired with a
// vertex gives [-1, r), in edge order, then the vertices no edge pairs
// give [-1, inf)); from n, dimension 1 in edge order (edge r paired with a
// triangle of larger value t gives [r, t); an edge paired with nothing
// gives [r, inf); zero-length pairs give no bar).  Per 1024-edge chunk the
// two kinds are counted, the counts scanned, then the bars written.
#define BC_CHUNK 1024
__device__ __forceinline__ bool bc_dim0(const int32_t *e_low, int64_t r) { return e_low[r] >= 0; }
__device__ __forceinline__ bool bc_dim1(const int32_t *e_low, const int32_t *toe, const unsigned long long *key,
                                        int64_t r) {
    const int32_t t = toe[r];
    if (t >= 0) return (int64_t)(key[t] >> 39) > r;
    return e_low[r] < 0;
}

__global__ void __launch_bounds__(BC_CHUNK) k_bc_count(const int32_t *e_low, const int32_t *toe,
                                                      const unsigned long long *key, int64_t K, int32_t *cnt) {
    __shared__ uint32_t sh[BC_CHUNK / 64][2];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t r = (int64_t)blockIdx.x * BC_CHUNK + t;
    const bool d0 = r < K && bc_dim0(e_low, r), d1 = r < K && bc_dim1(e_low, toe, key, r);
    const unsigned long long b0 = __ballot(d0), b1 = __ballot(d1);
    if (lane == 0) {
        sh[wv][0] = (uint32_t)__popcll(b0);
        sh[wv][1] = (uint32_t)__popcll(b1);
    }
    __syncthreads();
    if (t < 2) {
        uint32_t s = 0;
        for (int w = 0; w < BC_CHUNK / 64; w++) s += sh[w][t];
        cnt[2 * (int64_t)blockIdx.x + t] = (int32_t)s;
    }
}

// exclusive scan of the per-chunk counts (two interleaved series) into off
// (int64); off[2 nch] / off[2 nch + 1] get the totals.  One work-group.
__global__ void __launch_bounds__(BC_CHUNK) k_bc_scan(const int32_t *cnt, int64_t nch, long long *off) {
    __shared__ long long sh[BC_CHUNK / 64][2];
    __shared__ long long carry[2];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (t < 2) carry[t] = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nch; c0 += BC_CHUNK) {
        const int64_t c = c0 + t;
        long long x[2];
        for (int s = 0; s < 2; s++) {
            x[s] = c < nch ? cnt[2 * c + s] : 0;
            long long inc = x[s];
            for (int o = 1; o < 64; o <<= 1) {
                const long long y = __shfl_up(inc, o, 64);
                if (lane >= o) inc += y;
            }
            if (lane == 63) sh[wv][s] = inc;
            x[s] = inc - x[s];
        }
        __syncthreads();
        long long tot[2] = {0, 0};
        for (int s = 0; s < 2; s++) {
            long long before = 0;
            for (int w = 0; w < BC_CHUNK / 64; w++) {
                if (w < wv) before += sh[w][s];
                tot[s] += sh[w][s];
            }
            if (c < nch) off[2 * c + s] = carry[s] + before + x[s];
        }
        __syncthreads();
        if (t < 2) carry[t] += tot[t];
        __syncthreads();
    }
    if (t < 2) off[2 * nch + t] = carry[t];
}

__global__ void __launch_bounds__(BC_CHUNK) k_bc_write(const int32_t *e_low, const int32_t *toe,
                                                      const unsigned long long *key, int64_t n, int64_t K,
                                                      const long long *off, long long *bars) {
    __shared__ uint32_t sh[BC_CHUNK / 64][2];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t r = (int64_t)blockIdx.x * BC_CHUNK + t;
    const bool d0 = r < K && bc_dim0(e_low, r), d1 = r < K && bc_dim1(e_low, toe, key, r);
    const unsigned long long b0 = __ballot(d0), b1 = __ballot(d1);
    if (lane == 0) {
        sh[wv][0] = (uint32_t)__popcll(b0);
        sh[wv][1] = (uint32_t)__popcll(b1);
    }
    __syncthreads();
    uint32_t before0 = 0, before1 = 0;
    for (int w = 0; w < wv; w++) {
        before0 += sh[w][0];
        before1 += sh[w][1];
    }
    const long long INF = 0x7FFFFFFFFFFFFFFFll;
    if (d0) {
        const long long at = off[2 * (int64_t)blockIdx.x] + before0 +
                             __builtin_amdgcn_mbcnt_hi((uint32_t)(b0 >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b0, 0));
        bars[3 * at] = 0;
        bars[3 * at + 1] = -1;
        bars[3 * at + 2] = r;
    }
    if (d1) {
        const long long at = n + off[2 * (int64_t)blockIdx.x + 1] + before1 +
                             __builtin_amdgcn_mbcnt_hi((uint32_t)(b1 >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b1, 0));
        const int32_t tt = toe[r];
        bars[3 * at] = 1;
        bars[3 * at + 1] = r;
        bars[3 * at + 2] = tt >= 0 ? (long long)(key[tt] >> 39) : INF;
    }
}

// the vertices no edge pairs: [-1, inf) at bars [f0, n), f0 = finite bars of dimension 0
__global__ void __launch_bounds__(PD_BLOCK) k_bc_ess0(const long long *f0p, int64_t n, long long *bars) {
    const long long f0 = *f0p;
    for (int64_t x = f0 + blockIdx.x * (int64_t)PD_BLOCK + threadIdx.x; x < n; x += (int64_t)gridDim.x * PD_BLOCK) {
        bars[3 * x] = 0;
        bars[3 * x + 1] = -1;
        bars[3 * x + 2] = 0x7FFFFFFFFFFFFFFFll;
    }
}

// paired triangles (for the essential classes of dimension 2)
__global__ void __launch_bounds__(PD_BLOCK) k_bc_paired(const int32_t *toe, int64_t K, unsigned long long *cnt) {
    __shared__ unsigned long long s;
    if (threadIdx.x == 0) s = 0;
    __syncthreads();
    unsigned long long c = 0;
    for (int64_t r = blockIdx.x * (int64_t)PD_BLOCK + threadIdx.x; r < K; r += (int64_t)gridDim.x * PD_BLOCK)
        c += toe[r] >= 0 ? 1ull : 0ull;
    atomicAdd(&s, c);
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(cnt, s);
}

extern "C" VR_API int vr_barcode(const vr_result *res, const int32_t *e_low, const int32_t *tri_of_edge,
                                 int64_t *bars, int64_t counts[3], void *stream) {
    if (!res || !counts) return VR_EINVAL;
    const int64_t n = res->n_vertices, K = res->n_edges, T = res->n_triangles;
    if (n < 0 || K < 0 || T < 0 || n > VR_MAX_POINTS || T > 0x7FFFFFFF) return VR_EINVAL;
    if ((n + K > 0 && !bars) || (K > 0 && (!e_low || !tri_of_edge)) || (T > 0 && !res->tri_key)) return VR_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    const int64_t nch = (K + BC_CHUNK - 1) / BC_CHUNK;
    // off: 2 nch + 2 int64 (chunk offsets, then the two totals), the paired
    // triangle count, then cnt: 2 nch int32
    char *ws = (char *)cache_get(8 * (size_t)(2 * nch + 3) + 4 * (size_t)(2 * nch + 2) + 64, s);
    if (!ws) return VR_ENOMEM;
    long long *off = (long long *)ws;
    unsigned long long *paired = (unsigned long long *)(off + 2 * nch + 2);
    int32_t *cnt = (int32_t *)(ws + 8 * (size_t)(2 * nch + 3));
    const unsigned long long *key = (const unsigned long long *)res->tri_key;
    if (nch > 0) {
        hipLaunchKernelGGL(k_bc_count, dim3((unsigned)nch), dim3(BC_CHUNK), 0, s, e_low, tri_of_edge, key, K, cnt);
    }
    hipLaunchKernelGGL(k_bc_scan, dim3(1), dim3(BC_CHUNK), 0, s, (const int32_t *)cnt, nch, off);
    if (nch > 0)
        hipLaunchKernelGGL(k_bc_write, dim3((unsigned)nch), dim3(BC_CHUNK), 0, s, e_low, tri_of_edge, key, n, K,
                           (const long long *)off, (long long *)bars);
    if (n > 0)
        hipLaunchKernelGGL(k_bc_ess0, dim3(grid_for(n)), dim3(PD_BLOCK), 0, s, (const long long *)(off + 2 * nch), n,
                           (long long *)bars);
    long long tot[2] = {0, 0};
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(tot, off + 2 * nch, sizeof(tot), hipMemcpyDeviceToHost, s);
    unsigned long long np = 0;
    if (K > 0 && e == hipSuccess) {
        hipLaunchKernelGGL(k_rd_zero, dim3(1), dim3(PD_BLOCK), 0, s, paired, (int64_t)1);
        hipLaunchKernelGGL(k_bc_paired, dim3(grid_for(K)), dim3(PD_BLOCK), 0, s, tri_of_edge, K, paired);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(&np, paired, sizeof(np), hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    cache_put(ws, s);
    if (e != hipSuccess) return VR_EHIP;
    counts[0] = n;
    counts[1] = tot[1];
    counts[2] = T - (int64_t)np;
    return VR_OK;
}

// ------------------------------------------------ dimension 2, reduction ----
// Pairs of triangles with tetrahedra (maxdim 3 builds): the same reduction
// one dimension up.  Columns are the triangles from the youngest to the
// oldest, a column holds the triangle's cofacets (keys rd_tet_key, in
// filtration order) and its pivot is its oldest cofacet.  Triangles paired
// with an edge (dimension 1) are cleared.  Apparent pairs: a triangle t
// whose oldest cofacet s has t as its youngest facet pairs with s at once
// (no younger triangle is a facet of s, so no column before holds s).  The
// youngest facet of s = {a, b, c, d} (value w, edge w = {a, b}, c < d) is
// {a, b, d}: of the two facets of value w, the one holding the larger of
// the two other vertices.  So t (value v, vertex m off its largest edge)
// is apparent exactly when its oldest cofacet has value v and m as its
// larger vertex off edge v.  The apparent pairs go into the pivot table
// (length RD_APP, start = the triangle) before the two passes of the
// reduction; a pivot found there adds that triangle's coboundary.

// The index of the tetrahedron of reduction key (w, c, d) in the listed
// tetrahedra (value w: tet_off[w] .. tet_off[w + 1], by vertex word), or -1.
static __device__ long long rd_tet_index(const int32_t *ij, const long long *toff, const unsigned long long *tkey,
                                         unsigned long long key) {
    const int64_t w = (int64_t)(key >> 26);
    const uint32_t c = (uint32_t)(key >> 13) & 0x1FFFu, d = (uint32_t)key & 0x1FFFu;
    const uint32_t a = (uint32_t)ij[2 * w], b = (uint32_t)ij[2 * w + 1];
    const uint32_t x0 = min(a, c), x3 = max(b, d), m1 = max(a, c), m2 = min(b, d);
    const unsigned long long vk = ((unsigned long long)x0 << 39) | ((unsigned long long)min(m1, m2) << 26) |
                                  ((unsigned long long)max(m1, m2) << 13) | x3;
    long long lo = toff[w], hi = toff[w + 1];
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if (tkey[2 * mid + 1] < vk) lo = mid + 1;
        else hi = mid;
    }
    return (lo < toff[w + 1] && tkey[2 * lo + 1] == vk) ? lo : -1;
}

// clr[t] = 1 for the triangles paired with an edge (clr zeroed before).
__global__ void __launch_bounds__(PD_BLOCK) k_d2_clear(const int32_t *toe, int64_t K, int32_t *clr) {
    for (int64_t r = blockIdx.x * (int64_t)PD_BLOCK + threadIdx.x; r < K; r += (int64_t)gridDim.x * PD_BLOCK) {
        const int32_t t = toe[r];
        if (t >= 0) clr[t] = 1;
    }
}

// Every triangle's oldest cofacet: a cleared triangle or one without
// cofacets has no partner (tri_tet -1, no column); an apparent one pairs at
// once (tri_tet, and its pivot into the table); the rest are columns to
// reduce (col 1).  One work-group per edge r = {a, b}: the triangles of
// value r are {a, b, m} for the vertices m older-joined to both, and all
// their cofacets {a, b, m, l} have l joined to both a and b.  The
// work-group lists those l once (with the larger of the ranks of al and
// bl, and which of the two it is), then one wave per triangle takes the
// least cofacet key over them, reading only row m of the rank matrix.
#define D2_BLOCK 256
#define D2_WAVES (D2_BLOCK / 64)

// rng[2r], rng[2r + 1] = the first and one past the last triangle of value r
// (both 0 when there is none; rng zeroed before).
__global__ void __launch_bounds__(PD_BLOCK) k_d2_range(const unsigned long long *tri, int64_t T, int32_t *rng) {
    for (int64_t t = blockIdx.x * (int64_t)PD_BLOCK + threadIdx.x; t < T; t += (int64_t)gridDim.x * PD_BLOCK) {
        const unsigned long long v = tri[t] >> 39;
        if (t == 0 || (tri[t - 1] >> 39) != v) rng[2 * v] = (int32_t)t;
        if (t == T - 1 || (tri[t + 1] >> 39) != v) rng[2 * v + 1] = (int32_t)(t + 1);
    }
}

__global__ void __launch_bounds__(D2_BLOCK) k_d2_first(RdBufs B, const int32_t *rng, const int32_t *clr,
                                                      unsigned long long *piv, int32_t *col) {
    __shared__ uint16_t Ll[VR_MAX_POINTS];  // the vertices joined to both a and b
    __shared__ uint32_t Lx[VR_MAX_POINTS];  // max(rank al, rank bl), bit 31 set when bl is the larger
    __shared__ uint32_t sh[D2_WAVES];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t n = B.n;
    for (int64_t r = blockIdx.x; r < B.K; r += gridDim.x) {
        const long long lo = rng[2 * r], hi = rng[2 * r + 1];  // the triangles of value r
        if (lo == hi) continue;
        const uint32_t a = (uint32_t)B.ij[2 * r], b = (uint32_t)B.ij[2 * r + 1];
        const int32_t *Ra = B.R + (int64_t)a * n, *Rb = B.R + (int64_t)b * n;
        // list the common neighbours of a and b, in vertex order
        uint32_t nl = 0;
        for (int64_t l0 = 0; l0 < n; l0 += D2_BLOCK) {
            const int64_t l = l0 + t;
            int32_t x = PD_INF, y = PD_INF;
            if (l < n) {
                x = Ra[l];
                y = Rb[l];
            }
            const bool ok = l < n && (uint32_t)l != a && (uint32_t)l != b && x != PD_INF && y != PD_INF;
            const unsigned long long bl = __ballot(ok);
            if (lane == 0) sh[wv] = (uint32_t)__popcll(bl);
            __syncthreads();
            uint32_t before = 0, tot = 0;
            for (int w = 0; w < D2_WAVES; w++) {
                if (w < wv) before += sh[w];
                tot += sh[w];
            }
            if (ok) {
                const uint32_t at = nl + before + __builtin_amdgcn_mbcnt_hi((uint32_t)(bl >> 32),
                                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)bl, 0));
                Ll[at] = (uint16_t)l;
                Lx[at] = y > x ? ((uint32_t)y | 0x80000000u) : (uint32_t)x;
            }
            nl += tot;
            __syncthreads();
        }
        const int32_t v = (int32_t)r;
        for (long long tix = lo + wv; tix < hi; tix += D2_WAVES) {
            if (clr[tix]) {
                if (lane == 0) {
                    col[tix] = 0;
                    piv[tix] = ~0ull;
                }
                continue;
            }
            const unsigned long long key = B.tri[tix];
            const uint32_t i = (uint32_t)(key >> 26) & 0x1FFFu, j = (uint32_t)(key >> 13) & 0x1FFFu,
                           k = (uint32_t)key & 0x1FFFu;
            const uint32_t m = (i != a && i != b) ? i : ((j != a && j != b) ? j : k);  // off edge r
            const int32_t *Rm = B.R + (int64_t)m * n;
            unsigned long long best = ~0ull;
            for (uint32_t p = lane; p < nl; p += 64) {
                const uint32_t l = Ll[p];
                if (l == m) continue;
                const int32_t z = Rm[l];
                if (z == PD_INF) continue;
                const uint32_t lx = Lx[p];
                const int32_t x = (int32_t)(lx & 0x7FFFFFFFu);
                const int32_t w = max(v, max(x, z));
                unsigned long long kk;
                if (w == v) kk = rd_tet_key(w, min(m, l), max(m, l));                // edge r itself
                else if (w == x) kk = (lx >> 31) ? rd_tet_key(w, min(a, m), max(a, m))  // edge bl
                                                 : rd_tet_key(w, min(b, m), max(b, m)); // edge al
                else kk = rd_tet_key(w, a, b);                                          // edge ml
                best = min(best, kk);
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) best = min(best, (unsigned long long)__shfl_xor(best, o, 64));
            if (lane == 0) {
                // apparent: the oldest cofacet has value v and m as its larger vertex off edge v
                const bool app = best != ~0ull && (int32_t)(best >> 26) == v && ((uint32_t)best & 0x1FFFu) == m;
                col[tix] = best != ~0ull && !app;
                piv[tix] = app ? best : ~0ull;
            }
        }
        __syncthreads();
    }
}

// The apparent pairs found by k_d2_first: into the pivot table (flagged,
// with their triangle) and tri_tet; every other triangle's tri_tet is -1
// (the reduction writes the pairs of its columns).  One thread per triangle.
__global__ void __launch_bounds__(PD_BLOCK) k_d2_app(RdBufs B, const unsigned long long *piv, const long long *toff,
                                                    const unsigned long long *tkey, long long *tri_tet) {
    for (int64_t tix = blockIdx.x * (int64_t)PD_BLOCK + threadIdx.x; tix < B.T;
         tix += (int64_t)gridDim.x * PD_BLOCK) {
        const unsigned long long p = piv[tix];
        long long q = -1;
        if (p != ~0ull) {
            q = rd_tet_index(B.ij, toff, tkey, p);
            long long sl = rd_slot(p, B.hmask);
            for (;; sl = (sl + 1) & B.hmask)
                if (atomicCAS((unsigned long long *)&B.tab[sl].key, RD_EMPTY, p) == RD_EMPTY) break;
            B.tab[sl].start = (uint32_t)tix;
            B.tab[sl].len = RD_APP;
        }
        tri_tet[tix] = q;
    }
}

// Columns to reduce per chunk of BC_CHUNK triangles (second series unused).
__global__ void __launch_bounds__(BC_CHUNK) k_d2_count(const int32_t *col, int64_t T, int32_t *cnt) {
    __shared__ uint32_t sh[BC_CHUNK / 64];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t x = (int64_t)blockIdx.x * BC_CHUNK + t;
    const unsigned long long b = __ballot(x < T && col[x]);
    if (lane == 0) sh[wv] = (uint32_t)__popcll(b);
    __syncthreads();
    if (t == 0) {
        uint32_t s = 0;
        for (int w = 0; w < BC_CHUNK / 64; w++) s += sh[w];
        cnt[2 * (int64_t)blockIdx.x] = (int32_t)s;
        cnt[2 * (int64_t)blockIdx.x + 1] = 0;
    }
}

__global__ void k_d2_ctl(const long long *off, int64_t nch, RdCtl *ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->m = (int32_t)off[2 * nch];
        ctl->err = 0;
        ctl->ptop = 0;
        ctl->next = 0;
        ctl->nh = 0;
    }
}

// rem: the columns youngest first (column x-th from the oldest at m - 1 - x).
__global__ void __launch_bounds__(BC_CHUNK) k_d2_list(const int32_t *col, int64_t T, const long long *off,
                                                     int64_t nch, int32_t *rem) {
    __shared__ uint32_t sh[BC_CHUNK / 64];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t x = (int64_t)blockIdx.x * BC_CHUNK + t;
    const bool keep = x < T && col[x];
    const unsigned long long b = __ballot(keep);
    if (lane == 0) sh[wv] = (uint32_t)__popcll(b);
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wv; w++) before += sh[w];
    if (keep) {
        const long long at = off[2 * (int64_t)blockIdx.x] + before +
                             __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0));
        rem[off[2 * nch] - 1 - at] = (int32_t)x;
    }
}

// tri_tet[rem[ci]] = the index of column ci's pivot among the tetrahedra
__global__ void __launch_bounds__(PD_BLOCK) k_d2_emit(const int32_t *ij, const long long *toff,
                                                     const unsigned long long *tkey, const int32_t *rem,
                                                     const unsigned long long *rkey, const RdCtl *ctl,
                                                     long long *tri_tet) {
    const int32_t m = ctl->m;
    for (int64_t ci = blockIdx.x * (int64_t)PD_BLOCK + threadIdx.x; ci < m; ci += (int64_t)gridDim.x * PD_BLOCK) {
        const unsigned long long p = rkey[ci];
        if (p != RD_EMPTY) tri_tet[rem[ci]] = rd_tet_index(ij, toff, tkey, p);
    }
}

extern "C" VR_API int vr_pairs_dim2(const vr_result *res, const int32_t *tri_of_edge, int64_t *tri_tet, void *stream) {
    if (!res) return VR_EINVAL;
    const int64_t n = res->n_vertices, K = res->n_edges, T = res->n_triangles, T3 = res->n_tetrahedra;
    if (n < 0 || K < 0 || T < 0 || T3 < 0 || n > VR_MAX_POINTS || T > 0x7FFFFFFF) return VR_EINVAL;
    if (T == 0) return VR_OK;
    if (!tri_tet || !tri_of_edge || !res->edge_ij || !res->tri_key || !res->tet_off || (T3 > 0 && !res->tet_key))
        return VR_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    long long H = 2;
    while (H < 2 * T) H <<= 1;
    const int64_t nch = (T + BC_CHUNK - 1) / BC_CHUNK;
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t o = 0;
    const size_t o_R = o; o = up(o + 4 * (size_t)n * (size_t)n);
    const size_t o_clr = o; o = up(o + 8 * (size_t)((T + 1) / 2));
    const size_t o_col = o; o = up(o + 4 * (size_t)T);
    const size_t o_piv = o; o = up(o + 8 * (size_t)T);
    const size_t o_rng = o; o = up(o + 8 * (size_t)K);
    const size_t o_cnt = o; o = up(o + 8 * (size_t)nch);
    const size_t o_off = o; o = up(o + 8 * (size_t)(2 * nch + 2));
    const size_t o_rem = o; o = up(o + 4 * (size_t)T);
    const size_t o_tab = o; o = up(o + sizeof(RdSlot) * (size_t)H);
    const size_t o_pool = o; o = up(o + 8 * (size_t)RD_POOL_ENTRIES);
    const size_t o_cst = o; o = up(o + 8 * (size_t)T);
    const size_t o_cln = o; o = up(o + 4 * (size_t)T);
    const size_t o_rkey = o; o = up(o + 8 * (size_t)T);
    const size_t o_cslot = o; o = up(o + 8 * (size_t)T);
    const size_t o_h0 = o; o = up(o + 4 * (size_t)T);
    const size_t o_h1 = o; o = up(o + 4 * (size_t)T);
    const size_t o_ctl = o; o = up(o + sizeof(RdCtl));
    char *ws = (char *)cache_get(o, s);
    if (!ws) return VR_ENOMEM;
    RdBufs B{};
    B.R = (const int32_t *)(ws + o_R);
    B.ij = (const int32_t *)res->edge_ij;
    B.app = nullptr;
    B.rem = (const int32_t *)(ws + o_rem);
    B.tab = (RdSlot *)(ws + o_tab);
    B.hmask = H - 1;
    B.pool = (unsigned long long *)(ws + o_pool);
    B.cstart = (long long *)(ws + o_cst);
    B.clen = (int32_t *)(ws + o_cln);
    B.rkey = (unsigned long long *)(ws + o_rkey);
    B.cslot = (long long *)(ws + o_cslot);
    B.ctl = (RdCtl *)(ws + o_ctl);
    B.n = n;
    B.K = K;
    B.tri = (const unsigned long long *)res->tri_key;
    B.T = T;
    const long long *toff = (const long long *)res->tet_off;
    const unsigned long long *tkey = (const unsigned long long *)res->tet_key;
    int32_t *clr = (int32_t *)(ws + o_clr), *col = (int32_t *)(ws + o_col), *cnt = (int32_t *)(ws + o_cnt);
    long long *off = (long long *)(ws + o_off);
    hipLaunchKernelGGL(k_pd_fill, dim3(grid_for(n * n)), dim3(PD_BLOCK), 0, s, (int32_t *)(ws + o_R), n);
    hipLaunchKernelGGL(k_pd_edges, dim3(grid_for(K)), dim3(PD_BLOCK), 0, s, (int32_t *)(ws + o_R), n,
                       (const int32_t *)res->edge_ij, K, n);
    hipLaunchKernelGGL(k_rd_zero, dim3(grid_for((T + 1) / 2)), dim3(PD_BLOCK), 0, s, (unsigned long long *)clr,
                       (T + 1) / 2);
    hipLaunchKernelGGL(k_rd_zero, dim3(grid_for(RD_SLOT_WORDS * H)), dim3(PD_BLOCK), 0, s, (unsigned long long *)B.tab,
                       RD_SLOT_WORDS * H);
    hipLaunchKernelGGL(k_d2_clear, dim3(grid_for(K)), dim3(PD_BLOCK), 0, s, tri_of_edge, K, clr);
    int32_t *rng = (int32_t *)(ws + o_rng);
    hipLaunchKernelGGL(k_rd_zero, dim3(grid_for(K)), dim3(PD_BLOCK), 0, s, (unsigned long long *)rng, K);
    hipLaunchKernelGGL(k_d2_range, dim3(grid_for(T)), dim3(PD_BLOCK), 0, s, B.tri, T, rng);
    unsigned long long *piv = (unsigned long long *)(ws + o_piv);
    hipLaunchKernelGGL(k_d2_first, dim3((unsigned)(K < 65536 ? K : 65536)), dim3(D2_BLOCK), 0, s, B,
                       (const int32_t *)rng, (const int32_t *)clr, piv, col);
    hipLaunchKernelGGL(k_d2_app, dim3(grid_for(T)), dim3(PD_BLOCK), 0, s, B, (const unsigned long long *)piv, toff,
                       tkey, (long long *)tri_tet);
    hipLaunchKernelGGL(k_d2_count, dim3((unsigned)nch), dim3(BC_CHUNK), 0, s, (const int32_t *)col, T, cnt);
    hipLaunchKernelGGL(k_bc_scan, dim3(1), dim3(BC_CHUNK), 0, s, (const int32_t *)cnt, nch, off);
    hipLaunchKernelGGL(k_d2_ctl, dim3(1), dim3(64), 0, s, (const long long *)off, nch, B.ctl);
    hipLaunchKernelGGL(k_d2_list, dim3((unsigned)nch), dim3(BC_CHUNK), 0, s, (const int32_t *)col, T,
                       (const long long *)off, nch, (int32_t *)(ws + o_rem));
    const int st = rd_run<2>(B, (int32_t *)(ws + o_h0), (int32_t *)(ws + o_h1), s);
    if (st == VR_OK)
        hipLaunchKernelGGL(k_d2_emit, dim3(grid_for(T)), dim3(PD_BLOCK), 0, s, (const int32_t *)res->edge_ij, toff,
                           tkey, (const int32_t *)(ws + o_rem), (const unsigned long long *)B.rkey, (const RdCtl *)B.ctl,
                           (long long *)tri_tet);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    cache_put(ws, s);
    if (st != VR_OK) return st;
    return e == hipSuccess ? VR_OK : VR_EHIP;
}

// ------------------------------------------------- barcode, dimension 2 ----
// Bars of dimension 2 from the pairs of dimensions 1 and 2, in triangle
// order: triangle t paired with a tetrahedron of larger value w gives
// [value of t, w); a triangle paired with neither an edge nor a tetrahedron
// gives [value of t, inf).  The tetrahedra no triangle pairs with are the
// classes of dimension 3 (counted).  Per chunk of BC_CHUNK triangles the
// bars and the pairs are counted, the counts scanned, the bars written.
__device__ __forceinline__ bool b2_bar(const int32_t *clr, const long long *tt, const unsigned long long *tri,
                                       const unsigned long long *tkey, int64_t t) {
    const long long q = tt[t];
    if (q >= 0) return (long long)tkey[2 * q] > (long long)(tri[t] >> 39);
    return !clr[t];
}

__global__ void __launch_bounds__(BC_CHUNK) k_b2_count(const int32_t *clr, const long long *tt,
                                                      const unsigned long long *tri, const unsigned long long *tkey,
                                                      int64_t T, int32_t *cnt) {
    __shared__ uint32_t sh[BC_CHUNK / 64][2];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t x = (int64_t)blockIdx.x * BC_CHUNK + t;
    const bool bar = x < T && b2_bar(clr, tt, tri, tkey, x), paired = x < T && tt[x] >= 0;
    const unsigned long long b0 = __ballot(bar), b1 = __ballot(paired);
    if (lane == 0) {
        sh[wv][0] = (uint32_t)__popcll(b0);
        sh[wv][1] = (uint32_t)__popcll(b1);
    }
    __syncthreads();
    if (t < 2) {
        uint32_t s = 0;
        for (int w = 0; w < BC_CHUNK / 64; w++) s += sh[w][t];
        cnt[2 * (int64_t)blockIdx.x + t] = (int32_t)s;
    }
}

__global__ void __launch_bounds__(BC_CHUNK) k_b2_write(const int32_t *clr, const long long *tt,
                                                      const unsigned long long *tri, const unsigned long long *tkey,
                                                      int64_t T, const long long *off, long long *bars) {
    __shared__ uint32_t sh[BC_CHUNK / 64];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t x = (int64_t)blockIdx.x * BC_CHUNK + t;
    const bool bar = x < T && b2_bar(clr, tt, tri, tkey, x);
    const unsigned long long b = __ballot(bar);
    if (lane == 0) sh[wv] = (uint32_t)__popcll(b);
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wv; w++) before += sh[w];
    if (bar) {
        const long long at = off[2 * (int64_t)blockIdx.x] + before +
                             __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0));
        const long long q = tt[x];
        bars[3 * at] = 2;
        bars[3 * at + 1] = (long long)(tri[x] >> 39);
        bars[3 * at + 2] = q >= 0 ? (long long)tkey[2 * q] : 0x7FFFFFFFFFFFFFFFll;
    }
}

extern "C" VR_API int vr_barcode_dim2(const vr_result *res, const int32_t *tri_of_edge, const int64_t *tri_tet,
                                      int64_t *bars, int64_t counts[2], void *stream) {
    if (!res || !counts) return VR_EINVAL;
    const int64_t n = res->n_vertices, K = res->n_edges, T = res->n_triangles, T3 = res->n_tetrahedra;
    if (n < 0 || K < 0 || T < 0 || T3 < 0 || n > VR_MAX_POINTS || T > 0x7FFFFFFF) return VR_EINVAL;
    counts[0] = 0;
    counts[1] = T3;
    if (T == 0) return VR_OK;
    if (!tri_of_edge || !tri_tet || !bars || !res->tri_key || !res->tet_off || (T3 > 0 && !res->tet_key))
        return VR_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    const int64_t nch = (T + BC_CHUNK - 1) / BC_CHUNK;
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t o = 0;
    const size_t o_clr = o; o = up(o + 8 * (size_t)((T + 1) / 2));
    const size_t o_cnt = o; o = up(o + 8 * (size_t)nch);
    const size_t o_off = o; o = up(o + 8 * (size_t)(2 * nch + 2));
    char *ws = (char *)cache_get(o, s);
    if (!ws) return VR_ENOMEM;
    int32_t *clr = (int32_t *)(ws + o_clr), *cnt = (int32_t *)(ws + o_cnt);
    long long *off = (long long *)(ws + o_off);
    const unsigned long long *tri = (const unsigned long long *)res->tri_key;
    const unsigned long long *tkey = (const unsigned long long *)res->tet_key;
    hipLaunchKernelGGL(k_rd_zero, dim3(grid_for((T + 1) / 2)), dim3(PD_BLOCK), 0, s, (unsigned long long *)clr,
                       (T + 1) / 2);
    hipLaunchKernelGGL(k_d2_clear, dim3(grid_for(K)), dim3(PD_BLOCK), 0, s, tri_of_edge, K, clr);
    hipLaunchKernelGGL(k_b2_count, dim3((unsigned)nch), dim3(BC_CHUNK), 0, s, (const int32_t *)clr,
                       (const long long *)tri_tet, tri, tkey, T, cnt);
    hipLaunchKernelGGL(k_bc_scan, dim3(1), dim3(BC_CHUNK), 0, s, (const int32_t *)cnt, nch, off);
    hipLaunchKernelGGL(k_b2_write, dim3((unsigned)nch), dim3(BC_CHUNK), 0, s, (const int32_t *)clr,
                       (const long long *)tri_tet, tri, tkey, T, (const long long *)off, (long long *)bars);
    long long tot[2] = {0, 0};
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(tot, off + 2 * nch, sizeof(tot), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    cache_put(ws, s);
    if (e != hipSuccess) return VR_EHIP;
    counts[0] = tot[0];
    counts[1] = T3 - tot[1];
    return VR_OK;
}
