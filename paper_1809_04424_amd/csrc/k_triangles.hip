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

#define VR_MAXN 8192


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
// One work-group per vertex a, its ranks staged in LDS.  The star is taken in
// chunks of ENUM_BLOCK entries; the edges a owns in a chunk are compacted
// (star order = rank order).  Edge e's candidates (the first pb_e entries of
// its partner's star) are cut into ceil(pb_e / 64) wave-sized pieces.  Each
// wave takes a contiguous run of whole edges holding about 1/8 of the pieces
// and works through it on its own, with no work-group barrier: the metadata
// of up to 64 edges sits in lane registers (read back with readlane), so the
// loads of VR_UNROLL pieces issue back to back.
#define ENUM_BLOCK 512
#define ENUM_WAVES (ENUM_BLOCK / VR_WAVE)
#define VR_UNROLL 8
#define VR_YWAVE 256   // u64 bitset words per wave in the write kernel
#define VR_STAGE 192   // staged hits per wave in the write kernel

struct EnumLds {
    uint32_t r[ENUM_BLOCK];
    uint32_t b[ENUM_BLOCK];
    uint32_t sb[ENUM_BLOCK];      // start of the partner's star
    uint32_t pb[ENUM_BLOCK];      // candidates of the edge
    uint32_t cb[ENUM_BLOCK + 1];  // first piece of the edge
    uint32_t ew[ENUM_WAVES + 1];  // first edge of each wave
    uint32_t scan[ENUM_WAVES];
    uint32_t scan2[ENUM_WAVES];
};

__device__ __forceinline__ uint32_t enum_excl_scan(uint32_t x, uint32_t *sh, uint32_t *total) {
    const uint32_t inc = wave_incl_scan_dpp(x);
    const int w = threadIdx.x / VR_WAVE;
    if (lane_id() == VR_WAVE - 1) sh[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < ENUM_WAVES; i++) {
        const uint32_t v = sh[i];
        if (i < w) off += v;
        tot += v;
    }
    __syncthreads();
    *total = tot;
    return off + inc - x;
}

// Compact the owned edges of star entries [p0, p0+ENUM_BLOCK) into L and
// split them over the waves by piece count.
__device__ __forceinline__ int load_chunk(const VrDev &D, int a, uint32_t s0, uint32_t s1, uint32_t p0, EnumLds &L) {
    const uint32_t p = p0 + threadIdx.x;
    bool owned = false;
    uint32_t r = 0, b = 0, pb = 0;
    if (p < s1) {
        r = D.star_r[p];
        b = D.star_nbr[p];
        pb = D.pos[2 * (size_t)r + (b > (uint32_t)a ? 1 : 0)];
        const uint32_t x = p - s0;
        owned = pb < x || (pb == x && (uint32_t)a < b);
    }
    uint32_t m, C;
    const uint32_t idx = enum_excl_scan(owned ? 1u : 0u, L.scan, &m);
    const uint32_t pieces = owned ? (pb + VR_WAVE - 1) / VR_WAVE : 0u;
    const uint32_t cbeg = enum_excl_scan(pieces, L.scan2, &C);
    if (owned) {
        L.r[idx] = r;
        L.b[idx] = b;
        L.sb[idx] = D.start[b];
        L.pb[idx] = pb;
        L.cb[idx] = cbeg;
    }
    if (threadIdx.x == 0) L.cb[m] = C;
    __syncthreads();
    if ((int)threadIdx.x <= ENUM_WAVES) {
        // first edge whose first piece reaches the wave's share
        const uint32_t target = (uint32_t)(((unsigned long long)C * threadIdx.x) / ENUM_WAVES);
        int lo = 0, hi = (int)m;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (L.cb[mid] < target) lo = mid + 1;
            else hi = mid;
        }
        L.ew[threadIdx.x] = (threadIdx.x == ENUM_WAVES) ? m : (uint32_t)lo;
    }
    __syncthreads();
    return (int)m;
}

__device__ __forceinline__ uint32_t rl(uint32_t v, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// Walk the pieces of edges [e_lo, e_hi) of the window of ne edges starting at
// edge eb (lane l of the metadata registers describes edge eb + l; cb_end is
// the first piece after the window).  Piece c of edge e covers candidates
// 64(c - cb_e) + lane of the partner's star; candidate k is a hit when its
// rank to a is below r_e.  Counts go to the lane of the edge; with WRITE each
// hit sets bit k of bitset row (e - e_lo).
template <bool WRITE>
__device__ __forceinline__ void walk(const VrDev &D, const uint32_t *Ra, int eb, int ne, int e_lo, int e_hi,
                                     uint32_t vr, uint32_t vsb, uint32_t vpb, uint32_t vcb, uint32_t cb_end,
                                     uint32_t *mycnt, unsigned long long *Y, int W) {
    const int lane = threadIdx.x & 63;
    auto cb_of = [&](int e) { return (e - eb < ne) ? rl(vcb, e - eb) : cb_end; };
    const uint32_t c_lo = cb_of(e_lo), c_hi = cb_of(e_hi);
    int e = e_lo;
    uint32_t e_end = cb_of(e + 1);
    for (uint32_t c0 = c_lo; c0 < c_hi; c0 += VR_UNROLL) {
        uint32_t kk[VR_UNROLL], rr[VR_UNROLL];
        int eu[VR_UNROLL];
        bool ok[VR_UNROLL];
#pragma unroll
        for (int u = 0; u < VR_UNROLL; u++) {
            const uint32_t c = c0 + u;
            eu[u] = -1;
            ok[u] = false;
            kk[u] = 0;
            rr[u] = 0;
            if (c < c_hi) {
                while (c >= e_end) {
                    e++;
                    e_end = cb_of(e + 1);
                }
                const int el = e - eb;
                const uint32_t y = (c - rl(vcb, el)) * VR_WAVE + (uint32_t)lane;
                eu[u] = e;
                rr[u] = rl(vr, el);
                ok[u] = y < rl(vpb, el);
                if (ok[u]) kk[u] = D.star_nbr[rl(vsb, el) + y];
            }
        }
#pragma unroll
        for (int u = 0; u < VR_UNROLL; u++) {
            const bool hit = ok[u] && Ra[kk[u]] < rr[u];
            if (WRITE) {
                if (hit) atomicOr(&Y[(eu[u] - e_lo) * W + (kk[u] >> 6)], 1ull << (kk[u] & 63));
            } else if (eu[u] >= 0) {
                const uint32_t c = (uint32_t)__popcll(ballot64(hit));
                if (lane == eu[u] - eb) *mycnt += c;
            }
        }
    }
}

__device__ __forceinline__ void stage_row(const VrDev &D, uint32_t *Ra, uint32_t s0, uint32_t s1) {
    for (int k = threadIdx.x; k < D.n; k += ENUM_BLOCK) Ra[k] = VR_NOT_KEPT;
    __syncthreads();
    for (uint32_t p = s0 + threadIdx.x; p < s1; p += ENUM_BLOCK) Ra[D.star_nbr[p]] = D.star_r[p];
    __syncthreads();
}

size_t enum_lds(int n) { return 4 * (size_t)((n + 3) & ~3) + sizeof(EnumLds); }

// ----------------------------------------------------------- k_tri_count ----
__global__ __launch_bounds__(ENUM_BLOCK) void k_tri_count(VrDev D) {
    extern __shared__ uint32_t lds[];
    const int a = blockIdx.x, n = D.n;
    uint32_t *Ra = lds;
    EnumLds &L = *(EnumLds *)(lds + ((n + 3) & ~3));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t s0 = D.start[a], s1 = D.start[a + 1];
    stage_row(D, Ra, s0, s1);
    for (uint32_t p0 = s0; p0 < s1; p0 += ENUM_BLOCK) {
        const int m = load_chunk(D, a, s0, s1, p0, L);
        const int w_lo = __builtin_amdgcn_readfirstlane((int)L.ew[w]);
        const int w_hi = __builtin_amdgcn_readfirstlane((int)L.ew[w + 1]);
        for (int eb = w_lo; eb < w_hi; eb += VR_WAVE) {
            const int ne = min(VR_WAVE, w_hi - eb);
            uint32_t vr = 0, vsb = 0, vpb = 0, vcb = 0;
            if (lane < ne) {
                vr = L.r[eb + lane];
                vsb = L.sb[eb + lane];
                vpb = L.pb[eb + lane];
                vcb = L.cb[eb + lane];
            }
            const uint32_t cb_end = (uint32_t)__builtin_amdgcn_readfirstlane((int)L.cb[eb + ne]);
            uint32_t mycnt = 0;
            walk<false>(D, Ra, eb, ne, eb, eb + ne, vr, vsb, vpb, vcb, cb_end, &mycnt, nullptr, 0);
            if (lane < ne) D.cnt[vr] = mycnt;
        }
        __syncthreads();
        (void)m;
    }
}

void launch_tri_count(const VrDev &D, hipStream_t s) {
    hipLaunchKernelGGL(k_tri_count, dim3(D.n), dim3(ENUM_BLOCK), enum_lds(D.n), s, D);
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
// Emit edge r = {a, b}'s triangles from its bitset row Ye in k order.  The
// sorted vertex triple is (k, lo, hi), (lo, k, hi) or (lo, hi, k) as k falls
// below, between or above the edge's endpoints, so each key is a per-edge base
// plus k shifted into place.  Hits are staged in LDS in k order and written
// with all 64 lanes, each store covering 512 contiguous bytes.
__device__ __forceinline__ void emit_edge(unsigned long long *Ye, int W, uint32_t r, uint32_t a, uint32_t b,
                                          unsigned long long o, uint16_t *stage,
                                          unsigned long long *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const uint32_t lo = min(a, b), hi = max(a, b);
    const unsigned long long R = (unsigned long long)r << 39;
    const unsigned long long k_below = R | ((unsigned long long)lo << 13) | hi;           // | k << 26
    const unsigned long long k_mid = R | ((unsigned long long)lo << 26) | hi;            // | k << 13
    const unsigned long long k_above = R | ((unsigned long long)lo << 26) | ((unsigned long long)hi << 13);  // | k
    for (int x0 = 0; x0 < W; x0 += VR_WAVE) {
        const int wi = x0 + lane;
        unsigned long long word = 0ull;
        if (wi < W) {
            word = Ye[wi];
            Ye[wi] = 0ull;
        }
        const uint32_t pc = (uint32_t)__popcll(word);
        const uint32_t inc = wave_incl_scan_dpp(pc);
        const uint32_t tot = wave_last(inc);
        if (tot == 0) continue;
        if (tot <= VR_STAGE) {
            uint32_t q = inc - pc;
            while (word) {
                const int bit = __ffsll((long long)word) - 1;
                stage[q++] = (uint16_t)(wi * 64 + bit);
                word &= word - 1ull;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            for (uint32_t t = (uint32_t)lane; t < tot; t += VR_WAVE) {
                const unsigned long long k = stage[t];
                out[o + t] = (k < lo) ? (k_below | (k << 26)) : (k < hi) ? (k_mid | (k << 13)) : (k_above | k);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
        } else {
            unsigned long long q = o + (inc - pc);
            while (word) {
                const unsigned long long k = (unsigned long long)(wi * 64 + __ffsll((long long)word) - 1);
                out[q++] = (k < lo) ? (k_below | (k << 26)) : (k < hi) ? (k_mid | (k << 13)) : (k_above | k);
                word &= word - 1ull;
            }
        }
        o += tot;
    }
}

__device__ __forceinline__ int write_batch_cap(int W) {
    const int c = VR_YWAVE / W;
    return c < 1 ? 1 : (c > VR_WAVE ? VR_WAVE : c);
}

__global__ __launch_bounds__(ENUM_BLOCK) void k_tri_write(VrDev D, unsigned long long *__restrict__ out) {
    extern __shared__ uint32_t lds[];
    const int a = blockIdx.x, n = D.n;
    const int W = (n + 63) >> 6;
    const int cap = write_batch_cap(W);
    uint32_t *Ra = lds;
    EnumLds &L = *(EnumLds *)(lds + ((n + 3) & ~3));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    unsigned long long *Y = (unsigned long long *)(&L + 1) + (size_t)w * cap * W;
    uint16_t *stage = (uint16_t *)((unsigned long long *)(&L + 1) + (size_t)ENUM_WAVES * cap * W) + (size_t)w * VR_STAGE;
    for (int x = lane; x < cap * W; x += VR_WAVE) Y[x] = 0ull;
    const uint32_t s0 = D.start[a], s1 = D.start[a + 1];
    stage_row(D, Ra, s0, s1);
    for (uint32_t p0 = s0; p0 < s1; p0 += ENUM_BLOCK) {
        load_chunk(D, a, s0, s1, p0, L);
        const int w_lo = __builtin_amdgcn_readfirstlane((int)L.ew[w]);
        const int w_hi = __builtin_amdgcn_readfirstlane((int)L.ew[w + 1]);
        for (int eb = w_lo; eb < w_hi; eb += VR_WAVE) {
            const int ne = min(VR_WAVE, w_hi - eb);
            uint32_t vr = 0, vsb = 0, vpb = 0, vcb = 0, vb = 0;
            unsigned long long voff = 0;
            if (lane < ne) {
                vr = L.r[eb + lane];
                vsb = L.sb[eb + lane];
                vpb = L.pb[eb + lane];
                vcb = L.cb[eb + lane];
                vb = L.b[eb + lane];
                voff = D.off[vr];
            }
            const uint32_t cb_end = (uint32_t)__builtin_amdgcn_readfirstlane((int)L.cb[eb + ne]);
            for (int e0 = eb; e0 < eb + ne; e0 += cap) {
                const int e1 = min(eb + ne, e0 + cap);
                walk<true>(D, Ra, eb, ne, e0, e1, vr, vsb, vpb, vcb, cb_end, nullptr, Y, W);
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                __builtin_amdgcn_wave_barrier();
                for (int e = e0; e < e1; e++) {
                    const int el = e - eb;
                    const unsigned long long o = ((unsigned long long)rl((uint32_t)(voff >> 32), el) << 32) |
                                                 rl((uint32_t)voff, el);
                    emit_edge(Y + (size_t)(e - e0) * W, W, rl(vr, el), (uint32_t)a, rl(vb, el), o, stage, out);
                }
            }
        }
        __syncthreads();
    }
}

void launch_tri_write(const VrDev &D, unsigned long long *tri_out, hipStream_t s) {
    const int W = (D.n + 63) >> 6;
    int cap = VR_YWAVE / W;
    cap = cap < 1 ? 1 : (cap > VR_WAVE ? VR_WAVE : cap);
    const size_t lds = enum_lds(D.n) + (size_t)ENUM_WAVES * cap * W * 8 + (size_t)ENUM_WAVES * VR_STAGE * 2;
    static_assert(4 * VR_MAXN + sizeof(EnumLds) + ENUM_WAVES * VR_YWAVE * 8 + ENUM_WAVES * VR_STAGE * 2 <= 65536,
                  "write kernel LDS above 64 KiB at the largest n");
    hipLaunchKernelGGL(k_tri_write, dim3(D.n), dim3(ENUM_BLOCK), lds, s, D, tri_out);
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
