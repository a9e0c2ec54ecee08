// k_triangles.hip -- per-vertex stars, triangle counting, offsets and the
// ordered triangle write.
//
// Ownership: a triangle enters the filtration with its largest edge (Section
// 2.1), so the triangles of value r are exactly {a, b, k} with edge r = {a,b}
// and both {a,k} and {b,k} ranked below r.  For a fixed edge the sorted vertex
// triples are increasing in k, and edges are visited in rank order through the
// offsets, so the output comes out in (value, i, j, k) order with no sort.
//
//   k_star        per-vertex segmented sort of incident edge ranks (a stable
//                 per-column ordering, like the paper's
//                 integersinsameorderbycolumn, Section 4.3)
//   k_tri_count   one work-group per vertex a, its rank row staged in LDS;
//                 each edge is handled at the endpoint whose partner has the
//                 shorter earlier-neighbour prefix
//   k_scan        exclusive scan of the counts (decoupled look-back)
//   k_tri_write   the same enumeration; hits go to a per-wave LDS bitset and
//                 are compacted in k order with wave prefix sums (the paper's
//                 ballot/popc compaction of init_supp, Section 4.4, on wave64)
//   k_emit_edges  public edge arrays
#include "vr_device.h"

#define VR_MAXN 8192
#define VR_MAXW (VR_MAXN / 64)

// --------------------------------------------------------------- k_star ----
__global__ __launch_bounds__(VR_BLOCK) void k_star(VrDev D) {
    __shared__ uint32_t s[VR_MAXN];
    const int v = blockIdx.x, n = D.n, t = threadIdx.x;
    const uint32_t dg = D.deg[v];
    uint32_t N = 1;
    while (N < dg) N <<= 1;
    uint32_t *__restrict__ row = D.inc + (size_t)v * n;
    for (uint32_t x = t; x < N; x += VR_BLOCK) s[x] = (x < dg) ? row[x] : 0xFFFFFFFFu;
    __syncthreads();
    // bitonic sort of N keys (ranks are distinct)
    for (uint32_t k = 2; k <= N; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t x = t; x < N; x += VR_BLOCK) {
                const uint32_t l = x ^ j;
                if (l > x) {
                    const uint32_t a = s[x], b = s[l];
                    const bool up = (x & k) == 0;
                    if ((a > b) == up) { s[x] = b; s[l] = a; }
                }
            }
            __syncthreads();
        }
    }
    uint16_t *__restrict__ nrow = D.nbr + (size_t)v * n;
    for (uint32_t x = t; x < dg; x += VR_BLOCK) {
        const uint32_t r = s[x];
        const uint32_t ij = D.se_ij[r];
        const uint32_t i = ij >> 16, j = ij & 0xFFFFu;
        const bool small = (i == (uint32_t)v);
        row[x] = r;
        nrow[x] = (uint16_t)(small ? j : i);
        D.pos[2 * (size_t)r + (small ? 0 : 1)] = (uint16_t)x;
    }
}

void launch_star(const VrDev &D, hipStream_t s) {
    hipLaunchKernelGGL(k_star, dim3(D.n), dim3(VR_BLOCK), 0, s, D);
}

// ------------------------------------------------- shared enumeration core ----
// Stage the rank row of vertex a: Ra[k] = rank of edge {a,k}, or VR_NOT_KEPT.
__device__ __forceinline__ uint32_t stage_row(const VrDev &D, int a, uint32_t *Ra) {
    const int n = D.n;
    for (int k = threadIdx.x; k < n; k += VR_BLOCK) Ra[k] = VR_NOT_KEPT;
    __syncthreads();
    const uint32_t dg = D.deg[a];
    const uint32_t *__restrict__ row = D.inc + (size_t)a * n;
    const uint16_t *__restrict__ nrow = D.nbr + (size_t)a * n;
    for (uint32_t x = threadIdx.x; x < dg; x += VR_BLOCK) Ra[nrow[x]] = row[x];
    __syncthreads();
    return dg;
}

// Edge at position x of a's star: rank r, partner b, and the length of b's
// prefix of neighbours joined by lower-ranked edges.  Returns whether a owns
// the edge's enumeration (the partner's prefix is the shorter one).
__device__ __forceinline__ bool edge_at(const VrDev &D, int a, uint32_t x, uint32_t *r, uint32_t *b, uint32_t *pb) {
    const size_t o = (size_t)a * D.n + x;
    const uint32_t rr = D.inc[o];
    const uint32_t bb = D.nbr[o];
    const uint32_t p = D.pos[2 * (size_t)rr + (bb > (uint32_t)a ? 1 : 0)];
    *r = rr;
    *b = bb;
    *pb = p;
    return p < x || (p == x && (uint32_t)a < bb);
}

// ----------------------------------------------------------- k_tri_count ----
__global__ __launch_bounds__(VR_BLOCK) void k_tri_count(VrDev D) {
    __shared__ uint32_t Ra[VR_MAXN];
    const int a = blockIdx.x, n = D.n;
    const uint32_t dg = stage_row(D, a, Ra);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (uint32_t x = w; x < dg; x += VR_WAVES) {
        uint32_t r, b, pb;
        if (!edge_at(D, a, x, &r, &b, &pb)) continue;
        const uint16_t *__restrict__ pre = D.nbr + (size_t)b * n;
        uint32_t c = 0;
        for (uint32_t y = lane; y < pb; y += VR_WAVE) c += (Ra[pre[y]] < r) ? 1u : 0u;
        c = wave_sum(c);
        if (lane == 0) D.cnt[r] = c;
    }
}

void launch_tri_count(const VrDev &D, hipStream_t s) {
    hipLaunchKernelGGL(k_tri_count, dim3(D.n), dim3(VR_BLOCK), 0, s, D);
}

// ---------------------------------------------------------------- k_scan ----
__global__ __launch_bounds__(VR_BLOCK) void k_scan(VrDev D) {
    __shared__ unsigned long long sh_w[VR_WAVES];
    __shared__ unsigned long long sh_prefix;
    __shared__ int sh_tile;
    VrCtl *ctl = D.ctl;
    const int t = threadIdx.x;
    const long long K = (long long)ctl->n_kept;
    const int ntiles = (int)((K + VR_TILE - 1) / VR_TILE);
    for (;;) {
        const int tile = claim_tile(&ctl->ticket[5], &sh_tile);
        if (tile >= ntiles) break;
        const long long i0 = (long long)tile * VR_TILE + (long long)t * VR_ITEMS;
        uint32_t c[VR_ITEMS];
        unsigned long long loc = 0;
#pragma unroll
        for (int m = 0; m < VR_ITEMS; m++) {
            c[m] = (i0 + m < K) ? D.cnt[i0 + m] : 0u;
            loc += c[m];
        }
        unsigned long long tot;
        const unsigned long long ex = block_excl_scan<unsigned long long>(loc, sh_w, &tot);
        if (t == 0) {
            unsigned long long prefix = 0;
            if (tile == 0) {
                st_store64(D.st_scan, st_pack64(VR_ST_INC, tot));
            } else {
                st_store64(D.st_scan + tile, st_pack64(VR_ST_AGG, tot));
                prefix = lookback64(D.st_scan, tile);
                st_store64(D.st_scan + tile, st_pack64(VR_ST_INC, prefix + tot));
            }
            sh_prefix = prefix;
            if (tile == ntiles - 1) ctl->n_tri = prefix + tot;
        }
        __syncthreads();
        unsigned long long o = sh_prefix + ex;
#pragma unroll
        for (int m = 0; m < VR_ITEMS; m++) {
            if (i0 + m < K) D.off[i0 + m] = o;
            o += c[m];
        }
    }
}

void launch_scan(const VrDev &D, long long Kmax, hipStream_t s) {
    long long g = (Kmax + VR_TILE - 1) / VR_TILE;
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_scan, dim3((unsigned)g), dim3(VR_BLOCK), 0, s, D);
}

// ----------------------------------------------------------- k_tri_write ----
__global__ __launch_bounds__(VR_BLOCK) void k_tri_write(VrDev D, unsigned long long *__restrict__ out) {
    __shared__ uint32_t Ra[VR_MAXN];
    __shared__ unsigned long long Y[VR_WAVES][VR_MAXW];
    const int a = blockIdx.x, n = D.n;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int W = (n + 63) >> 6;
    for (int x = lane; x < W; x += VR_WAVE) Y[w][x] = 0ull;
    const uint32_t dg = stage_row(D, a, Ra);
    for (uint32_t x = w; x < dg; x += VR_WAVES) {
        uint32_t r, b, pb;
        if (!edge_at(D, a, x, &r, &b, &pb)) continue;
        const uint16_t *__restrict__ pre = D.nbr + (size_t)b * n;
        for (uint32_t y = lane; y < pb; y += VR_WAVE) {
            const uint32_t k = pre[y];
            if (Ra[k] < r) atomicOr(&Y[w][k >> 6], 1ull << (k & 63));
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
        unsigned long long o = D.off[r];
        for (int x0 = 0; x0 < W; x0 += VR_WAVE) {
            const int wi = x0 + lane;
            unsigned long long word = 0ull;
            if (wi < W) {
                word = Y[w][wi];
                Y[w][wi] = 0ull;
            }
            const uint32_t pc = (uint32_t)__popcll(word);
            const uint32_t inc = wave_incl_scan(pc);
            unsigned long long p = o + (inc - pc);
            while (word) {
                const int bit = __ffsll((long long)word) - 1;
                out[p++] = tri_key(r, (uint32_t)a, b, (uint32_t)(wi * 64 + bit));
                word &= word - 1ull;
            }
            o += __shfl(inc, VR_WAVE - 1, VR_WAVE);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
}

void launch_tri_write(const VrDev &D, unsigned long long *tri_out, hipStream_t s) {
    hipLaunchKernelGGL(k_tri_write, dim3(D.n), dim3(VR_BLOCK), 0, s, D, tri_out);
}

// ---------------------------------------------------------- k_emit_edges ----
__global__ __launch_bounds__(VR_BLOCK) void k_emit_edges(VrDev D, long long K, uint32_t *__restrict__ ij,
                                                         long long *__restrict__ q) {
    for (long long r = (long long)blockIdx.x * VR_BLOCK + threadIdx.x; r < K; r += (long long)gridDim.x * VR_BLOCK) {
        const uint32_t v = D.se_ij[r];
        ij[2 * r] = v >> 16;
        ij[2 * r + 1] = v & 0xFFFFu;
        q[r] = (long long)D.se_q[r];
    }
}

void launch_emit_edges(const VrDev &D, long long K, uint32_t *edge_ij, long long *edge_q, hipStream_t s) {
    long long g = (K + VR_BLOCK - 1) / VR_BLOCK;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_emit_edges, dim3((unsigned)g), dim3(VR_BLOCK), 0, s, D, K, edge_ij, edge_q);
}
