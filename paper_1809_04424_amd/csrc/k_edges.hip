// k_edges.hip -- squared distances, threshold selection and the edge-rank
// radix sort (the paper's sortperm step, Section 4.5, rebuilt as a stable
// LSD radix sort over the kept edges only).
//
//   k_init       zero the control block, degrees and select statuses
//   k_dist       exact integer squared distance of every pair i<j (VALU),
//                plus a log-linear histogram used to find the threshold
//   k_select     compact the candidate edges in pair order (decoupled
//                look-back) and histogram their radix digits
//   k_sort_pass  one stable 8-bit LSD pass (Onesweep: Adinets and Merrill,
//                2022), skipped when every key shares the digit
//   k_edges      write the K kept edges in rank order and bin them by vertex
#include "vr_device.h"

// --------------------------------------------------------------- k_init ----
__global__ __launch_bounds__(VR_BLOCK) void k_init(uint32_t *__restrict__ w, size_t words) {
    for (size_t x = (size_t)blockIdx.x * VR_BLOCK + threadIdx.x; x < words; x += (size_t)gridDim.x * VR_BLOCK)
        w[x] = 0u;
}

void launch_init(const VrDev &D, size_t zero_words, hipStream_t s) {
    size_t blocks = (zero_words + VR_BLOCK - 1) / VR_BLOCK;
    if (blocks > 1024) blocks = 1024;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_init, dim3((unsigned)blocks), dim3(VR_BLOCK), 0, s, (uint32_t *)D.ctl, zero_words);
}

// --------------------------------------------------------------- k_dist ----
// One work-group computes the 64 x 64 pairs (i in block bi, j in block bj),
// bi <= bj.  Lane l of every wave owns column j = 64*bj + l; wave w owns rows
// i = 64*bi + w + 4m (m < 16).  Coordinates are staged through LDS 64 at a
// time; the column operand is padded to avoid bank conflicts.  Writes of a
// row are contiguous in pair order, so every wave stores 256 contiguous bytes.
#define DIST_TB 64
#define DIST_CC 64

template <typename T>
__global__ __launch_bounds__(VR_BLOCK) void k_dist(const T *__restrict__ pts, int n, int d, int need_hist,
                                                   uint32_t *__restrict__ q, VrCtl *__restrict__ ctl) {
    const int bi = blockIdx.y, bj = blockIdx.x;
    if (bi > bj) return;
    __shared__ int32_t xi[DIST_TB][DIST_CC];
    __shared__ int32_t xj[DIST_TB][DIST_CC + 1];
    __shared__ uint32_t hist[VR_NBUCKET];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int j = bj * DIST_TB + lane;
    unsigned long long acc[16];
#pragma unroll
    for (int m = 0; m < 16; m++) acc[m] = 0ull;
    uint32_t over = 0;
    if (need_hist)
        for (int b = threadIdx.x; b < VR_NBUCKET; b += VR_BLOCK) hist[b] = 0u;
    for (int c0 = 0; c0 < d; c0 += DIST_CC) {
        const int cc = min(DIST_CC, d - c0);
        __syncthreads();
        for (int x = threadIdx.x; x < DIST_TB * DIST_CC; x += VR_BLOCK) {
            int r = x / DIST_CC, c = x % DIST_CC;
            int gi = bi * DIST_TB + r, gj = bj * DIST_TB + r;
            xi[r][c] = (gi < n && c < cc) ? (int32_t)pts[(size_t)gi * d + c0 + c] : 0;
            xj[r][c] = (gj < n && c < cc) ? (int32_t)pts[(size_t)gj * d + c0 + c] : 0;
        }
        __syncthreads();
        for (int c = 0; c < cc; c++) {
            const long long y = xj[lane][c];
#pragma unroll
            for (int m = 0; m < 16; m++) {
                long long df = (long long)xi[w + 4 * m][c] - y;
                if (sizeof(T) == 4) {
                    // |df| >= 2^16 makes df^2 >= 2^32 on its own
                    over |= (df >= 65536 || df <= -65536) ? 1u : 0u;
                    df = (df >= 65536 || df <= -65536) ? 0 : df;
                }
                acc[m] += (unsigned long long)(df * df);
            }
        }
    }
#pragma unroll
    for (int m = 0; m < 16; m++) {
        const int i = bi * DIST_TB + w + 4 * m;
        const bool ok = i < j && j < n;
        uint32_t qq = 0;
        if (ok) {
            unsigned long long v = acc[m];
            if (v > 0xFFFFFFFFull) { over = 1u; v = 0xFFFFFFFFull; }
            qq = (uint32_t)v;
            q[row_start(i, n) + (j - i - 1)] = qq;
        }
        if (need_hist) match_add<11>(hist, bucket_of(qq), ok);
    }
    if (over) atomicOr(&ctl->flags, 1u);
    if (need_hist) {
        __syncthreads();
        for (int b = threadIdx.x; b < VR_NBUCKET; b += VR_BLOCK)
            if (hist[b]) atomicAdd(&ctl->bucket[b], hist[b]);
    }
}

void launch_dist(const VrDev &D, const void *points, hipStream_t s) {
    const int nb = (D.n + DIST_TB - 1) / DIST_TB;
    dim3 grid(nb, nb);
    if (D.dtype == 1)
        hipLaunchKernelGGL(k_dist<int8_t>, grid, dim3(VR_BLOCK), 0, s, (const int8_t *)points, D.n, D.d,
                           D.need_hist, D.q, D.ctl);
    else if (D.dtype == 2)
        hipLaunchKernelGGL(k_dist<int16_t>, grid, dim3(VR_BLOCK), 0, s, (const int16_t *)points, D.n, D.d,
                           D.need_hist, D.q, D.ctl);
    else
        hipLaunchKernelGGL(k_dist<int32_t>, grid, dim3(VR_BLOCK), 0, s, (const int32_t *)points, D.n, D.d,
                           D.need_hist, D.q, D.ctl);
}

// ------------------------------------------------------------- k_select ----
// Select modes: which edges become sort candidates.
#define SEL_ALL 0     // every pair (infinite threshold)
#define SEL_BUCKET 1  // bucket(q) <= pivot bucket: a superset of the K smallest
#define SEL_LESS 2    // q < tau (distance threshold)
#define SEL_NONE 3    // K = 0

__global__ __launch_bounds__(VR_BLOCK) void k_select(VrDev D) {
    __shared__ uint32_t sh_w[VR_WAVES];
    __shared__ unsigned long long sh_w64[VR_WAVES];
    __shared__ int sh_tile;
    __shared__ uint32_t sh_pivot, sh_prefix;
    __shared__ uint32_t h8[VR_MAX_PASSES][VR_RADIX];
    VrCtl *ctl = D.ctl;
    const int t = threadIdx.x;

    int mode;
    if (D.thr_kind == 0) mode = SEL_ALL;
    else if (D.thr_kind == 3) mode = SEL_LESS;
    else mode = (D.K_host == 0) ? SEL_NONE : SEL_BUCKET;

    if (mode == SEL_BUCKET) {
        // pivot bucket: the smallest b whose cumulative count reaches K
        const int per = (VR_NBUCKET + VR_BLOCK - 1) / VR_BLOCK;  // 7
        unsigned long long loc = 0;
        for (int b = t * per; b < min(VR_NBUCKET, (t + 1) * per); b++) loc += ctl->bucket[b];
        unsigned long long tot;
        unsigned long long ex = block_excl_scan<unsigned long long>(loc, sh_w64, &tot);
        const unsigned long long K = (unsigned long long)D.K_host;
        if (ex < K && K <= ex + loc) {
            unsigned long long c = ex;
            for (int b = t * per; b < min(VR_NBUCKET, (t + 1) * per); b++) {
                c += ctl->bucket[b];
                if (c >= K) { sh_pivot = (uint32_t)b; break; }
            }
        }
        __syncthreads();
    }
    const uint32_t pivot = (mode == SEL_BUCKET) ? sh_pivot : 0u;
    const uint32_t tau = (mode == SEL_LESS) ? (uint32_t)min((long long)D.thr_num, 0xFFFFFFFFll) : 0u;
    const bool tau_all = (mode == SEL_LESS) && D.thr_num > 0xFFFFFFFFll;

    for (int x = t; x < VR_MAX_PASSES * VR_RADIX; x += VR_BLOCK) (&h8[0][0])[x] = 0u;

    const long long E = D.E;
    const int ntiles = (int)D.ntile_E;
    for (;;) {
        const int tile = claim_tile(&ctl->ticket[0], &sh_tile);
        if (tile >= ntiles) break;
        const long long e0 = (long long)tile * VR_TILE + (long long)t * VR_ITEMS;
        uint32_t qv[VR_ITEMS];
        bool keep[VR_ITEMS];
        uint32_t c = 0;
        int pi = 0, pj = 0;
        if (e0 < E) pair_of(e0, D.n, &pi, &pj);
#pragma unroll
        for (int m = 0; m < VR_ITEMS; m++) {
            const long long e = e0 + m;
            bool k = false;
            uint32_t v = 0;
            if (e < E) {
                v = D.q[e];
                if (mode == SEL_ALL) k = true;
                else if (mode == SEL_BUCKET) k = bucket_of(v) <= pivot;
                else if (mode == SEL_LESS) k = tau_all || v < tau;
            }
            qv[m] = v;
            keep[m] = k;
            c += k ? 1u : 0u;
        }
        uint32_t tot;
        const uint32_t ex = block_excl_scan<uint32_t>(c, sh_w, &tot);
        if (t < VR_WAVE) {
            uint32_t prefix = 0;
            if (tile == 0) {
                if (t == 0) st_store32(D.st_sel, st_pack32(VR_ST_INC, tot));
            } else {
                if (t == 0) st_store32(D.st_sel + tile, st_pack32(VR_ST_AGG, tot));
                prefix = lookback32_wave(D.st_sel, tile);
                if (t == 0) st_store32(D.st_sel + tile, st_pack32(VR_ST_INC, prefix + tot));
            }
            if (t == 0) {
                sh_prefix = prefix;
                if (tile == ntiles - 1) ctl->n_cand = prefix + tot;
            }
        }
        // clear this tile's statuses for the first active radix pass
        D.st_sort[0][(size_t)tile * VR_RADIX + t] = 0u;
        __syncthreads();
        uint32_t p = sh_prefix + ex;
#pragma unroll
        for (int m = 0; m < VR_ITEMS; m++) {
            if (keep[m]) {
                D.key[0][p] = qv[m];
                D.val[0][p] = ((uint32_t)pi << 16) | (uint32_t)pj;
                p++;
            }
            if (++pj == D.n) { pi++; pj = pi + 1; }
        }
        for (int ps = 0; ps < D.passes; ps++)
#pragma unroll
            for (int m = 0; m < VR_ITEMS; m++) match_add<8>(h8[ps], (qv[m] >> (8 * ps)) & 255u, keep[m]);
    }
    __syncthreads();
    for (int x = t; x < D.passes * VR_RADIX; x += VR_BLOCK) {
        uint32_t v = (&h8[0][0])[x];
        if (v) atomicAdd(&(&ctl->hist8[0][0])[x], v);
    }
}

void launch_select(const VrDev &D, hipStream_t s) {
    long long g = D.ntile_E;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_select, dim3((unsigned)g), dim3(VR_BLOCK), 0, s, D);
}

// Active radix passes: a pass whose digit is the same for every key is the
// identity and is skipped.  Returns the number of active passes before
// `upto` and sets *active for pass `upto` (when upto < passes).
__device__ __forceinline__ int active_before(const uint32_t *hist, int passes, int upto, bool *active) {
    __shared__ int sh_nz[VR_MAX_PASSES];
    if (threadIdx.x < VR_MAX_PASSES) sh_nz[threadIdx.x] = 0;
    __syncthreads();
    for (int x = threadIdx.x; x < passes * VR_RADIX; x += VR_BLOCK)
        if (hist[x]) atomicAdd(&sh_nz[x / VR_RADIX], 1);
    __syncthreads();
    int a = 0;
    for (int p = 0; p < upto && p < passes; p++) a += (sh_nz[p] > 1) ? 1 : 0;
    if (active) *active = (upto < passes) && (sh_nz[upto] > 1);
    __syncthreads();
    return a;
}

SortJob edge_sort_job(const VrDev &D) {
    SortJob J;
    J.key[0] = D.key[0]; J.key[1] = D.key[1];
    J.val[0] = D.val[0]; J.val[1] = D.val[1];
    J.hist = &D.ctl->hist8[0][0];
    J.ticket = &D.ctl->ticket[1];
    J.st[0] = D.st_sort[0]; J.st[1] = D.st_sort[1];
    J.count = &D.ctl->n_cand;
    J.passes = D.passes;
    return J;
}

SortJob star_sort_job(const VrDev &D) {
    SortJob J;
    J.key[0] = D.ikey[0]; J.key[1] = D.ikey[1];
    J.val[0] = D.ival[0]; J.val[1] = D.ival[1];
    J.hist = &D.ctl->hinc[0][0];
    J.ticket = &D.ctl->ticket[6];
    J.st[0] = D.ist[0]; J.st[1] = D.ist[1];
    J.count = &D.ctl->n_inc;
    J.passes = 2;
    return J;
}

// ---------------------------------------------------------- k_sort_pass ----
// Tiles of 2048 keys; each wave ranks its 512 keys among equal digits in
// order (8 ballots per 64 keys), the work-group combines the waves, one
// look-back per digit gives the tile's global offsets, and the tile is
// scattered through LDS so equal digits leave as contiguous runs.
__global__ __launch_bounds__(VR_BLOCK) void k_sort_pass(SortJob J, int pass) {
    __shared__ uint32_t s_whist[VR_WAVES][VR_RADIX];
    __shared__ uint32_t s_tstart[VR_RADIX];
    __shared__ uint32_t s_gpre[VR_RADIX];
    __shared__ uint32_t s_key[VR_TILE];
    __shared__ uint32_t s_val[VR_TILE];
    __shared__ uint32_t sh_w[VR_WAVES];
    __shared__ int sh_tile;
    bool active = false;
    const int a = active_before(J.hist, J.passes, pass, &active);
    if (!active) return;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const uint32_t Kc = *J.count;
    const int ntiles = (int)((Kc + VR_TILE - 1) / VR_TILE);
    const uint32_t *__restrict__ ksrc = J.key[a & 1];
    const uint32_t *__restrict__ vsrc = J.val[a & 1];
    uint32_t *__restrict__ kdst = J.key[(a + 1) & 1];
    uint32_t *__restrict__ vdst = J.val[(a + 1) & 1];
    uint32_t *st = J.st[a & 1];
    uint32_t *st_next = J.st[(a + 1) & 1];
    const int shift = VR_RADIX_BITS * pass;

    // global start of digit t
    uint32_t tot;
    const uint32_t gstart = block_excl_scan<uint32_t>(J.hist[pass * VR_RADIX + t], sh_w, &tot);

    for (;;) {
        const int tile = claim_tile(&J.ticket[pass], &sh_tile);
        if (tile >= ntiles) break;
        for (int x = 0; x < VR_WAVES; x++) s_whist[x][t] = 0u;
        __syncthreads();
        uint32_t kk[VR_ITEMS], vv[VR_ITEMS], rk[VR_ITEMS];
        const long long base = (long long)tile * VR_TILE + (long long)w * (VR_TILE / VR_WAVES);
#pragma unroll
        for (int it = 0; it < VR_ITEMS; it++) {
            const long long idx = base + (long long)it * VR_WAVE + lane;
            const bool valid = idx < (long long)Kc;
            const uint32_t k = valid ? ksrc[idx] : 0u;
            kk[it] = k;
            vv[it] = valid ? vsrc[idx] : 0u;
            const uint32_t dg = (k >> shift) & 255u;
            unsigned long long peers = ballot64(valid);
#pragma unroll
            for (int b = 0; b < VR_RADIX_BITS; b++) {
                const unsigned long long m = ballot64((dg >> b) & 1u);
                peers &= ((dg >> b) & 1u) ? m : ~m;
            }
            uint32_t before = 0;
            if (valid) before = s_whist[w][dg];
            const uint32_t r = before + (uint32_t)__popcll(peers & lanemask_lt());
            rk[it] = r;
            if (valid && (peers & lanemask_lt()) == 0ull) s_whist[w][dg] = before + (uint32_t)__popcll(peers);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        uint32_t wpre[VR_WAVES];
        uint32_t tc = 0;
#pragma unroll
        for (int x = 0; x < VR_WAVES; x++) { wpre[x] = tc; tc += s_whist[x][t]; }
        uint32_t ttot;
        const uint32_t tstart = block_excl_scan<uint32_t>(tc, sh_w, &ttot);
        s_tstart[t] = tstart;
        uint32_t prev = 0;
        if (tile == 0) {
            st_store32(st + t, st_pack32(VR_ST_INC, tc));
        } else {
            st_store32(st + (size_t)tile * VR_RADIX + t, st_pack32(VR_ST_AGG, tc));
            prev = lookback32(st + t, tile, VR_RADIX);
            st_store32(st + (size_t)tile * VR_RADIX + t, st_pack32(VR_ST_INC, prev + tc));
        }
        s_gpre[t] = gstart + prev;
        st_next[(size_t)tile * VR_RADIX + t] = 0u;
        __syncthreads();
#pragma unroll
        for (int x = 0; x < VR_WAVES; x++) s_whist[x][t] = wpre[x];
        __syncthreads();
#pragma unroll
        for (int it = 0; it < VR_ITEMS; it++) {
            const long long idx = base + (long long)it * VR_WAVE + lane;
            if (idx < (long long)Kc) {
                const uint32_t dg = (kk[it] >> shift) & 255u;
                const uint32_t lp = s_tstart[dg] + s_whist[w][dg] + rk[it];
                s_key[lp] = kk[it];
                s_val[lp] = vv[it];
            }
        }
        __syncthreads();
        const uint32_t valid_n = (uint32_t)min((long long)VR_TILE, (long long)Kc - (long long)tile * VR_TILE);
#pragma unroll
        for (int m = 0; m < VR_ITEMS; m++) {
            const uint32_t lp = (uint32_t)t + (uint32_t)m * VR_BLOCK;
            if (lp < valid_n) {
                const uint32_t k = s_key[lp];
                const uint32_t dg = (k >> shift) & 255u;
                const uint32_t gp = s_gpre[dg] + (lp - s_tstart[dg]);
                kdst[gp] = k;
                vdst[gp] = s_val[lp];
            }
        }
    }
}

void launch_sort_pass(const SortJob &J, long long max_tiles, int pass, hipStream_t s) {
    long long g = max_tiles;
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_sort_pass, dim3((unsigned)g), dim3(VR_BLOCK), 0, s, J, pass);
}

// -------------------------------------------------------------- k_edges ----
// Kept edges in rank order.  With triangles wanted, also the list of vertex
// incidences (vertex, 2r+s) in rank order plus the digit histograms of the
// vertices, input of the stable star sort, and clear its first statuses.
__global__ __launch_bounds__(VR_BLOCK) void k_edges(VrDev D) {
    __shared__ uint32_t h[2][VR_RADIX];
    VrCtl *ctl = D.ctl;
    const int a = active_before(&ctl->hist8[0][0], D.passes, VR_MAX_PASSES, nullptr);
    const uint32_t *__restrict__ kf = D.key[a & 1];
    const uint32_t *__restrict__ vf = D.val[a & 1];
    const long long K = (D.thr_kind == 3) ? (long long)ctl->n_cand : D.K_host;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->n_kept = (uint32_t)K;
        ctl->n_inc = (uint32_t)(2 * K);
        // without triangles this is the last phase-1 kernel: publish now
        if (!D.tri) publish_counts(D.mailbox, D.seq, ctl->flags, ctl->n_cand, (uint32_t)K, 0ull);
    }
    if (D.tri) {
        for (int x = threadIdx.x; x < 2 * VR_RADIX; x += VR_BLOCK) (&h[0][0])[x] = 0u;
        __syncthreads();
        const long long words = (2 * K + VR_TILE - 1) / VR_TILE * VR_RADIX;
        for (long long x = (long long)blockIdx.x * VR_BLOCK + threadIdx.x; x < words; x += (long long)gridDim.x * VR_BLOCK)
            D.ist[0][x] = 0u;
    }
    const long long Kr = (K + VR_BLOCK - 1) / VR_BLOCK * VR_BLOCK;  // whole waves take part in match_add
    for (long long r = (long long)blockIdx.x * VR_BLOCK + threadIdx.x; r < Kr; r += (long long)gridDim.x * VR_BLOCK) {
        const bool ok = r < K;
        uint32_t i = 0, j = 0;
        if (ok) {
            const uint32_t k = kf[r], v = vf[r];
            D.se_q[r] = k;
            D.se_ij[r] = v;
            i = v >> 16;
            j = v & 0xFFFFu;
            if (D.tri) {
                D.ikey[0][2 * r] = i;
                D.ikey[0][2 * r + 1] = j;
                D.ival[0][2 * r] = (uint32_t)(2 * r);
                D.ival[0][2 * r + 1] = (uint32_t)(2 * r + 1);
            }
        }
        if (D.tri) {
            match_add<8>(h[0], i & 255u, ok);
            match_add<5>(h[1], i >> 8, ok);
            match_add<8>(h[0], j & 255u, ok);
            match_add<5>(h[1], j >> 8, ok);
        }
    }
    if (D.tri) {
        __syncthreads();
        for (int x = threadIdx.x; x < 2 * VR_RADIX; x += VR_BLOCK) {
            const uint32_t c = (&h[0][0])[x];
            if (c) atomicAdd(&(&ctl->hinc[0][0])[x], c);
        }
    }
}

void launch_edges(const VrDev &D, hipStream_t s) {
    long long K = (D.thr_kind == 3) ? D.E : D.K_host;
    long long g = (K + VR_BLOCK - 1) / VR_BLOCK;
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_edges, dim3((unsigned)g), dim3(VR_BLOCK), 0, s, D);
}
