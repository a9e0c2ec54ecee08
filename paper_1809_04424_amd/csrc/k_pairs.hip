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

// Tetrahedra (dimension 3) per largest edge.  Work-group g takes edge r:
// the vertices x joined to both ends by older edges (D[i][x] < r and
// D[j][x] < r; the ends themselves fail one test, D[i][j] = r), compacted
// into LDS in ascending order, then the pairs of them joined by an older
// edge: wave w takes the vertices a = w, w+4, ... and its lanes read the
// entries of row L[a] for the later vertices together (ascending, so nearby
// addresses).  D as for the pairs of dimension 0 (ranks, +inf off the
// edges, -1 on the diagonal).
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
// for a fixed pair i < j is the lexicographic order of (k, l), k < l: row
// a of the common neighbours L (ascending) holds the pairs (L[a], L[b]),
// b > a, so the rows are counted, scanned in LDS, and each wave writes its
// rows' pairs in order through a ballot.  Key of a tetrahedron: two words,
// its value r and a<<39 | b<<26 | c<<13 | d.
__global__ void __launch_bounds__(PD_BLOCK) k_tet_write(const int32_t *D, int64_t ld, int64_t n, const int32_t *ij,
                                                       int64_t K, const long long *off, long long total,
                                                       unsigned long long *keys) {
    __shared__ uint16_t L[VR_MAX_POINTS];
    __shared__ uint32_t rowc[VR_MAX_POINTS];
    __shared__ uint32_t wc[PD_BLOCK / 64];
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
        // pairs per row a
        for (uint32_t a = wv; a < m; a += PD_BLOCK / 64) {
            uint32_t c = 0;
            const int32_t *row = D + (int64_t)L[a] * ld;
            for (uint32_t b2 = a + 1 + lane; b2 < m; b2 += 64) c += row[L[b2]] < r ? 1u : 0u;
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d, 64);
            if (lane == 0) rowc[a] = c;
        }
        __syncthreads();
        // exclusive scan of rowc[0..m) in place: thread t takes the rows
        // [t*per, t*per + per), the work-group scans the threads' sums
        {
            const uint32_t per = (m + PD_BLOCK - 1) / PD_BLOCK;
            const uint32_t a0 = min((uint32_t)t * per, m), a1 = min(a0 + per, m);
            uint32_t own = 0;
            for (uint32_t a = a0; a < a1; a++) own += rowc[a];
            uint32_t incl = own;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t y = __shfl_up(incl, d, 64);
                if (lane >= d) incl += y;
            }
            if (lane == 63) wc[wv] = incl;
            __syncthreads();
            uint32_t run = incl - own;
#pragma unroll
            for (int w = 0; w < PD_BLOCK / 64; w++)
                if (w < wv) run += wc[w];
            for (uint32_t a = a0; a < a1; a++) {
                const uint32_t c = rowc[a];
                rowc[a] = run;
                run += c;
            }
            __syncthreads();
        }
        const long long g0 = off[r];
        const uint32_t vi = (uint32_t)i, vj = (uint32_t)j;
        for (uint32_t a = wv; a < m; a += PD_BLOCK / 64) {
            const uint32_t k = L[a];
            const int32_t *row = D + (int64_t)k * ld;
            uint32_t pos = rowc[a];
            for (uint32_t b0 = a + 1; b0 < m; b0 += 64) {
                const uint32_t b2 = b0 + lane;
                const bool in = b2 < m && row[L[b2]] < r;
                const unsigned long long bm = __ballot(in);
                if (in) {
                    const uint32_t l = L[b2];
                    // sorted merge of {i < j} and {k < l}
                    uint32_t q[4];
                    uint32_t x = 0, y = 0;
                    const uint32_t s1[2] = {vi, vj}, s2[2] = {k, l};
#pragma unroll
                    for (int z = 0; z < 4; z++) {
                        const bool take1 = y >= 2 || (x < 2 && s1[x < 2 ? x : 1] < s2[y < 2 ? y : 1]);
                        q[z] = take1 ? s1[x < 2 ? x : 1] : s2[y < 2 ? y : 1];
                        x += take1 ? 1 : 0;
                        y += take1 ? 0 : 1;
                    }
                    const long long at = g0 + pos +
                        __builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0));
                    if (at < total)  // one 16-byte store per tetrahedron
                        *(ulonglong2 *)(keys + 2 * at) =
                            make_ulonglong2((unsigned long long)r, ((unsigned long long)q[0] << 39) |
                                                                       ((unsigned long long)q[1] << 26) |
                                                                       ((unsigned long long)q[2] << 13) | q[3]);
                }
                pos += (uint32_t)__popcll(bm);
            }
        }
        __syncthreads();  // L and rowc are reused by the next edge
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
