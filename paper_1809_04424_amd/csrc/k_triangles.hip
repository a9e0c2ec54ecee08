// k_triangles.hip -- vertex stars, triangle counting, offsets and the
// ordered triangle write.
//
// Ownership: a triangle enters the filtration with its largest edge (Section
// 2.1), so the triangles of value r are exactly {a, b, k} with edge r = {a,b}
// and both {a,k} and {b,k} ranked below r.  Those k are the neighbours of b
// that come before edge r in b's rank-ordered star (a prefix of that star)
// and whose edge to a also ranks below r.  For a fixed edge the sorted vertex
// triples increase with k, and the offsets follow rank order, so the output
// is written in (value, i, j, k) order with no sort.
//
//   k_star        CSR stars from the stably sorted incidences (a stable
//                 per-column ordering, like the paper's
//                 integersinsameorderbycolumn, Section 4.3)
//   k_star_pos    position of every edge in both of its stars
//   k_tri_count   one work-group per vertex a with a's ranks staged in LDS;
//                 each edge is handled at the endpoint whose partner has the
//                 shorter prefix; a wave takes a batch of edges and walks all
//                 their candidates as one flat stream (full lanes, independent
//                 loads)
//   k_scan        exclusive scan of the counts (decoupled look-back)
//   k_publish     counts to the host-pinned mailbox
//   k_tri_write   the same walk; hits set bits of a per-edge LDS bitset, which
//                 is then compacted in k order with popcounts and wave prefix
//                 sums (the ballot/popc compaction of the paper's init_supp,
//                 Section 4.4, on 64-wide waves)
//   k_emit_edges  public edge arrays
#include "vr_device.h"

#define VR_YBUDGET 512  // u64 bitset words per wave in the write kernel

__device__ __forceinline__ int star_parity(const VrCtl *ctl) {
    // number of active passes of the two-pass star sort, from its histograms
    __shared__ int sh_nz[2];
    if (threadIdx.x < 2) sh_nz[threadIdx.x] = 0;
    __syncthreads();
    for (int x = threadIdx.x; x < 2 * VR_RADIX; x += VR_BLOCK)
        if ((&ctl->hinc[0][0])[x]) atomicAdd(&sh_nz[x / VR_RADIX], 1);
    __syncthreads();
    const int a = (sh_nz[0] > 1 ? 1 : 0) + (sh_nz[1] > 1 ? 1 : 0);
    __syncthreads();
    return a & 1;
}

// --------------------------------------------------------------- k_star ----
__global__ __launch_bounds__(VR_BLOCK) void k_star(VrDev D) {
    const VrCtl *ctl = D.ctl;
    const int par = star_parity(ctl);
    const uint32_t *__restrict__ kf = D.ikey[par];
    const uint32_t *__restrict__ vf = D.ival[par];
    const long long m = (long long)ctl->n_inc;
    const int n = D.n;
    if (m == 0) {
        if (blockIdx.x == 0)
            for (int u = threadIdx.x; u <= n; u += VR_BLOCK) D.start[u] = 0u;
        return;
    }
    for (long long p = (long long)blockIdx.x * VR_BLOCK + threadIdx.x; p < m; p += (long long)gridDim.x * VR_BLOCK) {
        const uint32_t v = kf[p], x = vf[p];
        const uint32_t r = x >> 1;
        const uint32_t ij = D.se_ij[r];
        D.star_r[p] = r;
        D.star_nbr[p] = (uint16_t)((x & 1u) ? (ij >> 16) : (ij & 0xFFFFu));
        const int prev = (p == 0) ? -1 : (int)kf[p - 1];
        for (int u = prev + 1; u <= (int)v; u++) D.start[u] = (uint32_t)p;
        if (p == m - 1)
            for (int u = (int)v + 1; u <= n; u++) D.start[u] = (uint32_t)m;
    }
}

__global__ __launch_bounds__(VR_BLOCK) void k_star_pos(VrDev D) {
    const VrCtl *ctl = D.ctl;
    const int par = star_parity(ctl);
    const uint32_t *__restrict__ kf = D.ikey[par];
    const uint32_t *__restrict__ vf = D.ival[par];
    const long long m = (long long)ctl->n_inc;
    for (long long p = (long long)blockIdx.x * VR_BLOCK + threadIdx.x; p < m; p += (long long)gridDim.x * VR_BLOCK)
        D.pos[vf[p]] = (uint16_t)(p - D.start[kf[p]]);
}

void launch_star(const VrDev &D, hipStream_t s) {
    long long g = (2 * ((D.thr_kind == 3) ? D.E : D.K_host) + VR_BLOCK - 1) / VR_BLOCK;
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_star, dim3((unsigned)g), dim3(VR_BLOCK), 0, s, D);
    hipLaunchKernelGGL(k_star_pos, dim3((unsigned)g), dim3(VR_BLOCK), 0, s, D);
}

// ------------------------------------------------- shared enumeration core ----
// Stage the ranks of vertex a: Ra[k] = rank of edge {a,k}, or VR_NOT_KEPT.
__device__ __forceinline__ void stage_row(const VrDev &D, int a, uint32_t *Ra, uint32_t s0, uint32_t s1) {
    for (int k = threadIdx.x; k < D.n; k += VR_BLOCK) Ra[k] = VR_NOT_KEPT;
    __syncthreads();
    for (uint32_t p = s0 + threadIdx.x; p < s1; p += VR_BLOCK) Ra[D.star_nbr[p]] = D.star_r[p];
    __syncthreads();
}

// Per-wave batch descriptors in LDS.
struct Batch {
    uint32_t r[VR_WAVE];
    uint32_t sb[VR_WAVE];   // start of the partner's star
    uint32_t b[VR_WAVE];
    uint32_t beg[VR_WAVE];  // flat offset of the edge's candidates
    uint32_t end[VR_WAVE];
    uint32_t cnt[VR_WAVE];
    unsigned long long off[VR_WAVE];
};

// Load the metadata of star entries [p0, p0+nb) of vertex a, keep the edges a
// owns, compact them into the batch (in star order) and lay their candidate
// prefixes end to end.  Returns (owned count, total candidates).
template <bool WRITE>
__device__ __forceinline__ void load_batch(const VrDev &D, int a, uint32_t s0, uint32_t s1, uint32_t p0, int nb,
                                           Batch &B, int *m_out, uint32_t *S_out) {
    const int lane = threadIdx.x & 63;
    const uint32_t p = p0 + (uint32_t)lane;
    bool owned = false;
    uint32_t r = 0, b = 0, pb = 0;
    if (lane < nb && p < s1) {
        r = D.star_r[p];
        b = D.star_nbr[p];
        pb = D.pos[2 * (size_t)r + (b > (uint32_t)a ? 1 : 0)];
        const uint32_t x = p - s0;
        owned = pb < x || (pb == x && (uint32_t)a < b);
    }
    const unsigned long long mask = ballot64(owned);
    const uint32_t idx = (uint32_t)__popcll(mask & lanemask_lt());
    const uint32_t len = owned ? pb : 0u;
    const uint32_t incl = wave_incl_scan(len);
    if (owned) {
        B.r[idx] = r;
        B.b[idx] = b;
        B.sb[idx] = D.start[b];
        B.beg[idx] = incl - len;
        B.end[idx] = incl;
        B.cnt[idx] = 0u;
        if (WRITE) B.off[idx] = D.off[r];
    }
    *m_out = __popcll(mask);
    *S_out = __shfl(incl, VR_WAVE - 1, VR_WAVE);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// Walk the flat candidate stream of a batch: candidate f of edge e is the
// neighbour star_nbr[sb_e + f - beg_e] of the partner; it is a hit when its
// edge to a ranks below r_e.  Count hits per edge, and with WRITE set the
// hit's bit in the edge's bitset.  VR_UNROLL chunks of 64 candidates are in
// flight at once: all loads of a round are issued before any is consumed.
#define VR_UNROLL 8
template <bool WRITE>
__device__ __forceinline__ void walk_batch(const VrDev &D, const uint32_t *Ra, Batch &B, int m, uint32_t S,
                                           unsigned long long *Y, int W) {
    const int lane = threadIdx.x & 63;
    int seg = 0;
    for (uint32_t f0 = 0; f0 < S; f0 += VR_WAVE * VR_UNROLL) {
        uint32_t kk[VR_UNROLL];
        int sg[VR_UNROLL];
#pragma unroll
        for (int u = 0; u < VR_UNROLL; u++) {
            const uint32_t f = f0 + (uint32_t)(u * VR_WAVE + lane);
            sg[u] = -1;
            kk[u] = 0;
            if (f < S) {
                while (seg < m - 1 && B.end[seg] <= f) seg++;
                sg[u] = seg;
                kk[u] = D.star_nbr[B.sb[seg] + (f - B.beg[seg])];
            }
        }
#pragma unroll
        for (int u = 0; u < VR_UNROLL; u++) {
            const int g = sg[u];
            const bool hit = g >= 0 && Ra[kk[u]] < B.r[g];
            if (WRITE) {
                if (hit) atomicOr(&Y[g * W + (kk[u] >> 6)], 1ull << (kk[u] & 63));
            } else {
                // segments are contiguous lane ranges: one add per segment
                const unsigned long long hits = ballot64(hit);
                const int gp = __shfl_up(g, 1, VR_WAVE);
                const bool first = g >= 0 && (lane == 0 || gp != g);
                const unsigned long long starts = ballot64(first);
                if (first) {
                    const unsigned long long above = starts & ~((2ull << lane) - 1ull);
                    const unsigned long long upto = above ? (above & (~above + 1ull)) - 1ull : ~0ull;
                    const unsigned long long mine = upto & ~((1ull << lane) - 1ull);
                    const uint32_t c = (uint32_t)__popcll(hits & mine);
                    if (c) atomicAdd(&B.cnt[g], c);
                }
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// ----------------------------------------------------------- k_tri_count ----
__global__ __launch_bounds__(VR_BLOCK) void k_tri_count(VrDev D) {
    extern __shared__ uint32_t lds[];
    const int a = blockIdx.x, n = D.n;
    uint32_t *Ra = lds;
    Batch *Bs = (Batch *)(lds + ((n + 3) & ~3));
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    Batch &B = Bs[w];
    const uint32_t s0 = D.start[a], s1 = D.start[a + 1];
    stage_row(D, a, Ra, s0, s1);
    for (uint32_t p0 = s0 + (uint32_t)w * VR_WAVE; p0 < s1; p0 += VR_WAVES * VR_WAVE) {
        int m;
        uint32_t S;
        load_batch<false>(D, a, s0, s1, p0, VR_WAVE, B, &m, &S);
        if (m == 0) continue;
        walk_batch<false>(D, Ra, B, m, S, nullptr, 0);
        if (lane < m) D.cnt[B.r[lane]] = B.cnt[lane];
        __builtin_amdgcn_wave_barrier();
    }
}

size_t batch_lds(int n) { return 4 * (size_t)((n + 3) & ~3) + VR_WAVES * sizeof(Batch); }

void launch_tri_count(const VrDev &D, hipStream_t s) {
    hipLaunchKernelGGL(k_tri_count, dim3(D.n), dim3(VR_BLOCK), batch_lds(D.n), s, D);
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
        if (t < VR_WAVE) {
            unsigned long long prefix = 0;
            if (tile == 0) {
                if (t == 0) st_store64(D.st_scan, st_pack64(VR_ST_INC, tot));
            } else {
                if (t == 0) st_store64(D.st_scan + tile, st_pack64(VR_ST_AGG, tot));
                prefix = lookback64_wave(D.st_scan, tile);
                if (t == 0) st_store64(D.st_scan + tile, st_pack64(VR_ST_INC, prefix + tot));
            }
            if (t == 0) {
                sh_prefix = prefix;
                if (tile == ntiles - 1) ctl->n_tri = prefix + tot;
            }
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

// ------------------------------------------------------------- k_publish ----
__global__ void k_publish(VrDev D) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const VrCtl *ctl = D.ctl;
    VrMailbox *mb = D.mailbox;
    __hip_atomic_store(&mb->flags, ctl->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&mb->n_cand, ctl->n_cand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&mb->n_kept, ctl->n_kept, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&mb->n_tri, D.tri ? ctl->n_tri : 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&mb->seq, D.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

void launch_publish(const VrDev &D, hipStream_t s) {
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, s, D);
}

// ----------------------------------------------------------- k_tri_write ----
__device__ __forceinline__ int write_batch_cap(int W) {
    int c = VR_YBUDGET / W;
    return c < 1 ? 1 : (c > VR_WAVE ? VR_WAVE : c);
}

__global__ __launch_bounds__(VR_BLOCK) void k_tri_write(VrDev D, unsigned long long *__restrict__ out) {
    extern __shared__ uint32_t lds[];
    const int a = blockIdx.x, n = D.n;
    const int W = (n + 63) >> 6;
    const int cap = write_batch_cap(W);
    uint32_t *Ra = lds;
    Batch *Bs = (Batch *)(lds + ((n + 3) & ~3));
    unsigned long long *Yall = (unsigned long long *)(Bs + VR_WAVES);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    Batch &B = Bs[w];
    unsigned long long *Y = Yall + (size_t)w * cap * W;
    for (int x = lane; x < cap * W; x += VR_WAVE) Y[x] = 0ull;
    const uint32_t s0 = D.start[a], s1 = D.start[a + 1];
    stage_row(D, a, Ra, s0, s1);
    for (uint32_t p0 = s0 + (uint32_t)w * cap; p0 < s1; p0 += (uint32_t)(VR_WAVES * cap)) {
        int m;
        uint32_t S;
        load_batch<true>(D, a, s0, s1, p0, cap, B, &m, &S);
        if (m == 0) continue;
        walk_batch<true>(D, Ra, B, m, S, Y, W);
        for (int e = 0; e < m; e++) {
            const uint32_t r = B.r[e], bb = B.b[e];
            unsigned long long o = B.off[e];
            unsigned long long *Ye = Y + (size_t)e * W;
            for (int x0 = 0; x0 < W; x0 += VR_WAVE) {
                const int wi = x0 + lane;
                unsigned long long word = 0ull;
                if (wi < W) {
                    word = Ye[wi];
                    Ye[wi] = 0ull;
                }
                const uint32_t pc = (uint32_t)__popcll(word);
                const uint32_t inc = wave_incl_scan(pc);
                unsigned long long p = o + (inc - pc);
                while (word) {
                    const int bit = __ffsll((long long)word) - 1;
                    out[p++] = tri_key(r, (uint32_t)a, bb, (uint32_t)(wi * 64 + bit));
                    word &= word - 1ull;
                }
                o += __shfl(inc, VR_WAVE - 1, VR_WAVE);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
}

void launch_tri_write(const VrDev &D, unsigned long long *tri_out, hipStream_t s) {
    const int W = (D.n + 63) >> 6;
    int cap = 512 / W;
    cap = cap < 1 ? 1 : (cap > 64 ? 64 : cap);
    const size_t lds = batch_lds(D.n) + (size_t)VR_WAVES * cap * W * 8;
    hipLaunchKernelGGL(k_tri_write, dim3(D.n), dim3(VR_BLOCK), lds, s, D, tri_out);
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
