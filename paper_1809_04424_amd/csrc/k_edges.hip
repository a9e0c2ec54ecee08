// k_edges.hip -- squared distances, threshold selection and the edge-rank
// radix sort (the paper's sortperm step, Section 4.5, rebuilt as a stable
// LSD radix sort over the kept edges only), for one cloud or a batch.
//
//   k_init       zero the control block, histograms and statuses
//   k_dist       exact integer squared distance of every pair i<j of every
//                cloud (VALU), plus a per-cloud log-linear histogram used to
//                find percentile thresholds
//   k_pivot      per cloud, the histogram bucket holding the K-th distance
//   k_sel_count, k_sel_scan, k_sel_write
//                compact the candidate edges in (cloud, pair) order (count
//                per tile, scan, write) and histogram their radix digits
//   k_sort_pass  one stable 8-bit LSD pass (Onesweep: Adinets and Merrill,
//                2022), skipped when every key shares the digit; keys are
//                (cloud << qbits) | q, so clouds stay apart
//   k_edges      the kept edges of every cloud in rank order, and their
//                ranks scattered into each cloud's rank matrix
#include "vr_device.h"

// --------------------------------------------------------------- k_init ----
__global__ __launch_bounds__(VR_BLOCK) void k_init(uint32_t *__restrict__ w, size_t words, VrCloud one,
                                                    VrCloud *__restrict__ dst) {
    if (dst && blockIdx.x == 0 && threadIdx.x == 0) *dst = one;
    for (size_t x = (size_t)blockIdx.x * VR_BLOCK + threadIdx.x; x < words; x += (size_t)gridDim.x * VR_BLOCK)
        w[x] = 0u;
}

// dst != null: also store the single cloud's descriptor (no host copy).
void launch_init(const VrDev &D, size_t zero_words, const VrCloud *one, VrCloud *dst, hipStream_t s) {
    size_t blocks = (zero_words + VR_BLOCK - 1) / VR_BLOCK;
    if (blocks > 1024) blocks = 1024;
    if (blocks == 0) blocks = 1;
    VrCloud c{};
    if (one) c = *one;
    hipLaunchKernelGGL(k_init, dim3((unsigned)blocks), dim3(VR_BLOCK), 0, s, (uint32_t *)D.ctl, zero_words, c,
                       one ? dst : nullptr);
}

// ------------------------------------------------------- k_cloud_maps ----
// Work-group c writes cloud c into the batch's maps: its vertices, its
// distance tiles, the select tiles and kept blocks whose first element it
// holds (kept blocks only when the kept counts are known on the host).
__global__ __launch_bounds__(VR_BLOCK) void k_cloud_maps(VrDev D) {
    const int c = blockIdx.x, t = threadIdx.x;
    const VrCloud cl = D.cl[c];
    const long long n = cl.n, E = n * (n - 1) / 2, nb = (n + 63) / 64;
    for (long long v = t; v < n; v += VR_BLOCK) D.vcloud[cl.vbase + v] = (uint32_t)c;
    for (long long x = t; x < nb * (nb + 1) / 2; x += VR_BLOCK) D.tcloud[cl.tbase + x] = (uint32_t)c;
    const long long s0 = (cl.pbase + VR_TILE - 1) / VR_TILE, s1 = (cl.pbase + E + VR_TILE - 1) / VR_TILE;
    for (long long x = s0 + t; x < s1; x += VR_BLOCK) D.scloud[x] = (uint32_t)c;
    if (D.thr_kind != 3) {
        const long long k0 = (cl.kbase + VR_BLOCK - 1) / VR_BLOCK, k1 = (cl.kbase + cl.K + VR_BLOCK - 1) / VR_BLOCK;
        for (long long x = k0 + t; x < k1; x += VR_BLOCK) D.kcloud[x] = (uint32_t)c;
    }
}

void launch_cloud_maps(const VrDev &D, hipStream_t s) {
    if (D.C > 1) hipLaunchKernelGGL(k_cloud_maps, dim3((unsigned)D.C), dim3(VR_BLOCK), 0, s, D);
}

// Distance tile t of a cloud with nb 64-point blocks: tiles are the blocks
// (bi, bj), bi <= bj, in row order.
__device__ __forceinline__ long long tile_row_start(long long bi, long long nb) { return bi * nb - bi * (bi - 1) / 2; }

__device__ __forceinline__ void tile_of(long long t, long long nb, int *bi, int *bj) {
    double b = 2.0 * (double)nb + 1.0;
    double disc = b * b - 8.0 * (double)t;
    long long i = (long long)((b - sqrt(disc > 0 ? disc : 0.0)) * 0.5);
    if (i < 0) i = 0;
    if (i > nb - 1) i = nb - 1;
    while (i > 0 && tile_row_start(i, nb) > t) i--;
    while (i < nb - 1 && tile_row_start(i + 1, nb) <= t) i++;
    *bi = (int)i;
    *bj = (int)(t - tile_row_start(i, nb) + i);
}

// --------------------------------------------------------------- k_dist ----
// One work-group computes the 64 x 64 pairs (i in block bi, j in block bj) of
// one cloud.  Lane l of every wave owns column j = 64*bj + l; wave w owns rows
// i = 64*bi + w + 4m (m < 16).  Coordinates are staged through LDS 64 at a
// time; the column operand is padded to avoid bank conflicts.  Writes of a
// row are contiguous in pair order, so every wave stores 256 contiguous bytes.
#define DIST_TB 64
#define DIST_CC 64

template <typename T>
__global__ __launch_bounds__(VR_BLOCK) void k_dist(VrDev D) {
    const long long tg = blockIdx.x;
    const int c = (D.C == 1) ? 0 : (int)D.tcloud[tg];
    const VrCloud cl = D.cl[c];
    const int n = cl.n, d = D.d;
    int bi, bj;
    tile_of(tg - cl.tbase, (n + DIST_TB - 1) / DIST_TB, &bi, &bj);
    const T *__restrict__ pts = (const T *)cl.points;
    uint32_t *__restrict__ q = D.q + cl.pbase;
    __shared__ int32_t xi[DIST_TB][DIST_CC];
    __shared__ int32_t xj[DIST_TB][DIST_CC + 1];
    __shared__ uint32_t hist[VR_NBUCKET];
    const int need_hist = D.need_hist;
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
        if (cc == DIST_CC) {
            for (int x = threadIdx.x; x < DIST_TB * DIST_CC; x += VR_BLOCK) {
                const int r = x / DIST_CC, cx = x % DIST_CC;
                const int gi = bi * DIST_TB + r, gj = bj * DIST_TB + r;
                xi[r][cx] = gi < n ? (int32_t)pts[(size_t)gi * d + c0 + cx] : 0;
                xj[r][cx] = gj < n ? (int32_t)pts[(size_t)gj * d + c0 + cx] : 0;
            }
        } else {
            // a partial chunk (every chunk when d < 64): stage only the cc
            // coordinates the loop below reads
            for (int x = threadIdx.x; x < DIST_TB * cc; x += VR_BLOCK) {
                const int r = x / cc, cx = x - r * cc;
                const int gi = bi * DIST_TB + r, gj = bj * DIST_TB + r;
                xi[r][cx] = gi < n ? (int32_t)pts[(size_t)gi * d + c0 + cx] : 0;
                xj[r][cx] = gj < n ? (int32_t)pts[(size_t)gj * d + c0 + cx] : 0;
            }
        }
        __syncthreads();
        for (int cx = 0; cx < cc; cx++) {
            const long long y = xj[lane][cx];
#pragma unroll
            for (int m = 0; m < 16; m++) {
                long long df = (long long)xi[w + 4 * m][cx] - y;
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
        if (i < j && j < n) {
            unsigned long long v = acc[m];
            if (v > 0xFFFFFFFFull) { over = 1u; v = 0xFFFFFFFFull; }
            const uint32_t qq = (uint32_t)v;
            q[row_start(i, n) + (j - i - 1)] = qq;
            if (need_hist) atomicAdd(&hist[bucket_of(qq)], 1u);
        }
    }
    if (over) atomicOr(&D.ctl->flags, 1u);
    if (need_hist) {
        __syncthreads();
        uint32_t *gh = D.hist + ((size_t)c * D.hcopies + blockIdx.x % D.hcopies) * VR_NBUCKET;
        for (int b = threadIdx.x; b < VR_NBUCKET; b += VR_BLOCK)
            if (hist[b]) atomicAdd(&gh[b], hist[b]);
    }
}

// ---------------------------------------------------------- k_dist_mat ----
// Dissimilarity-matrix input (the paper's Section 3 accepts a symmetric
// distance matrix in place of points): q of pair i<j is entry [i][j] of the
// cloud's n x n int32 matrix; the entries below the diagonal are not read.
// Same tiles, pair order and histogram as k_dist; a negative entry raises
// the overflow flag (VR_ERANGE).  Lane l of every wave reads column
// j = 64 bj + l of rows i = 64 bi + w + 4m, so each wave reads 256
// contiguous bytes of a row.
__global__ __launch_bounds__(VR_BLOCK) void k_dist_mat(VrDev D) {
    const long long tg = blockIdx.x;
    const int c = (D.C == 1) ? 0 : (int)D.tcloud[tg];
    const VrCloud cl = D.cl[c];
    const int n = cl.n;
    int bi, bj;
    tile_of(tg - cl.tbase, (n + DIST_TB - 1) / DIST_TB, &bi, &bj);
    const int32_t *__restrict__ M = (const int32_t *)cl.points;
    uint32_t *__restrict__ q = D.q + cl.pbase;
    __shared__ uint32_t hist[VR_NBUCKET];
    const int need_hist = D.need_hist;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int j = bj * DIST_TB + lane;
    if (need_hist) {
        for (int b = threadIdx.x; b < VR_NBUCKET; b += VR_BLOCK) hist[b] = 0u;
        __syncthreads();
    }
    uint32_t over = 0;
    int32_t v[16];
#pragma unroll
    for (int m = 0; m < 16; m++) {  // clamped addresses: every load is issued at once
        const int i = min(bi * DIST_TB + w + 4 * m, n - 1);
        v[m] = M[(size_t)i * n + min(j, n - 1)];
    }
#pragma unroll
    for (int m = 0; m < 16; m++) {
        const int i = bi * DIST_TB + w + 4 * m;
        if (i < j && j < n) {
            if (v[m] < 0) over = 1u;
            const uint32_t qq = v[m] < 0 ? 0u : (uint32_t)v[m];
            q[row_start(i, n) + (j - i - 1)] = qq;
            if (need_hist) atomicAdd(&hist[bucket_of(qq)], 1u);
        }
    }
    if (over) atomicOr(&D.ctl->flags, 1u);
    if (need_hist) {
        __syncthreads();
        uint32_t *gh = D.hist + ((size_t)c * D.hcopies + blockIdx.x % D.hcopies) * VR_NBUCKET;
        for (int b = threadIdx.x; b < VR_NBUCKET; b += VR_BLOCK)
            if (hist[b]) atomicAdd(&gh[b], hist[b]);
    }
}

void launch_dist(const VrDev &D, const void *points, hipStream_t s) {
    (void)points;
    const dim3 grid((unsigned)D.tiles);
    if (D.dtype == 1) hipLaunchKernelGGL(k_dist<int8_t>, grid, dim3(VR_BLOCK), 0, s, D);
    else if (D.dtype == 2) hipLaunchKernelGGL(k_dist<int16_t>, grid, dim3(VR_BLOCK), 0, s, D);
    else if (D.dtype == 3) hipLaunchKernelGGL(k_dist<int32_t>, grid, dim3(VR_BLOCK), 0, s, D);
    else hipLaunchKernelGGL(k_dist_mat, grid, dim3(VR_BLOCK), 0, s, D);  // VR_DIST
}

// -------------------------------------------------------------- k_pivot ----
// Work-group c: the smallest bucket of cloud c whose cumulative count reaches
// K_c; the candidates are then every pair below the end of that bucket (a
// superset of the K_c smallest, as buckets are monotone in q).
#define PIVOT_BLOCK 1024
__global__ __launch_bounds__(PIVOT_BLOCK) void k_pivot(VrDev D) {
    __shared__ uint32_t hb[VR_NBUCKET];
    __shared__ unsigned long long sh_w[PIVOT_BLOCK / VR_WAVE];
    __shared__ uint32_t sh_pivot;
    const int c = blockIdx.x, t = threadIdx.x;
    const uint32_t *h = D.hist + (size_t)c * D.hcopies * VR_NBUCKET;
    const unsigned long long K = (unsigned long long)D.cl[c].K;
    for (int b = t; b < VR_NBUCKET; b += PIVOT_BLOCK) hb[b] = hist_sum(h, VR_NBUCKET, D.hcopies, b);
    if (t == 0) sh_pivot = 0u;
    __syncthreads();
    // two buckets per thread, in order
    const int b0 = 2 * t;
    const uint32_t h0 = (b0 < VR_NBUCKET) ? hb[b0] : 0u, h1 = (b0 + 1 < VR_NBUCKET) ? hb[b0 + 1] : 0u;
    const unsigned long long loc = (unsigned long long)h0 + h1;
    unsigned long long inc = loc;
#pragma unroll
    for (int o = 1; o < VR_WAVE; o <<= 1) {
        const unsigned long long y = __shfl_up(inc, o, VR_WAVE);
        if ((t & 63) >= o) inc += y;
    }
    const int w = t / VR_WAVE;
    if ((t & 63) == 63) sh_w[w] = inc;
    __syncthreads();
    unsigned long long ex = inc - loc;
    for (int x = 0; x < w; x++) ex += sh_w[x];
    if (K > 0 && ex < K && K <= ex + loc) sh_pivot = (ex + h0 >= K) ? (uint32_t)b0 : (uint32_t)(b0 + 1);
    __syncthreads();
    // candidates: every q below the end of the pivot bucket (none when K = 0)
    if (t == 0) D.cs[c].qend = (K > 0) ? bucket_start(sh_pivot + 1u) : 0ull;
}

void launch_pivot(const VrDev &D, hipStream_t s) {
    hipLaunchKernelGGL(k_pivot, dim3((unsigned)D.C), dim3(PIVOT_BLOCK), 0, s, D);
}

// -------------------------------------------------------------- select ----
// A pair of cloud c is a candidate when q < qend(c): every pair (full
// threshold), q < tau (distance threshold), or q below the end of the
// cloud's pivot bucket (count / fraction threshold; a superset of the K_c
// smallest, as buckets are monotone in q).  Candidates keep (cloud, pair)
// order; the first pair of each cloud records where its candidates begin.
__device__ __forceinline__ unsigned long long cloud_qend(const VrDev &D, int c) {
    if (D.thr_kind == 0) return 1ull << 32;
    if (D.thr_kind == 3) {
        const long long tau = D.cl[c].thr_num;
        return tau > (1ll << 32) ? (1ull << 32) : (unsigned long long)tau;
    }
    return D.cs[c].qend;
}

// The 8 pairs of thread t in 2048-pair tile `tile`: candidate flags, sort
// keys (cloud << qbits | q), values (i << 16 | j), and the pairs that start
// a cloud.  Returns the thread's candidate count.
struct SelItems {
    uint32_t kv[VR_ITEMS], vv[VR_ITEMS];
    bool keep[VR_ITEMS], first[VR_ITEMS];
    int cc[VR_ITEMS];
};

__device__ __forceinline__ uint32_t select_items(const VrDev &D, int tile, SelItems &I) {
    const long long E = D.E;
    const long long e0 = (long long)tile * VR_TILE + (long long)threadIdx.x * VR_ITEMS;
    uint32_t q[VR_ITEMS];
    if (e0 + VR_ITEMS <= E) {  // 8 aligned words: two 16-byte loads
        const uint4 a = *(const uint4 *)(D.q + e0), b = *(const uint4 *)(D.q + e0 + 4);
        q[0] = a.x; q[1] = a.y; q[2] = a.z; q[3] = a.w;
        q[4] = b.x; q[5] = b.y; q[6] = b.z; q[7] = b.w;
    } else {
#pragma unroll
        for (int m = 0; m < VR_ITEMS; m++) q[m] = (e0 + m < E) ? D.q[e0 + m] : 0u;
    }
    int c = 0, pi = 0, pj = 0, n = 2;
    long long cstart = -1, cend = 0;
    unsigned long long qend = 0;
    if (e0 < E) {
        c = cloud_from_map(D, D.scloud, e0, VR_TILE, [&](int k) { return D.cl[k].pbase; });
        n = D.cl[c].n;
        cstart = D.cl[c].pbase;
        cend = cstart + (long long)n * (n - 1) / 2;
        qend = cloud_qend(D, c);
        pair_of(e0 - cstart, n, &pi, &pj);
    }
    const uint32_t qb = (uint32_t)D.qbits;
    uint32_t cnt = 0;
#pragma unroll
    for (int m = 0; m < VR_ITEMS; m++) {
        const long long e = e0 + m;
        const bool valid = e < E;
        bool f = valid && e == cstart;
        if (valid && e == cend) {  // next cloud (rare: every cloud of a batch has a pair)
            c++;
            n = D.cl[c].n;
            cend += (long long)n * (n - 1) / 2;
            qend = cloud_qend(D, c);
            pi = 0;
            pj = 1;
            f = true;
        }
        const bool k = valid && (unsigned long long)q[m] < qend;
        I.kv[m] = (qb >= 32) ? q[m] : (((uint32_t)c << qb) | q[m]);  // one cloud when q takes 32 bits
        I.vv[m] = ((uint32_t)pi << 16) | (uint32_t)pj;
        I.keep[m] = k;
        I.first[m] = f;
        I.cc[m] = c;
        cnt += k ? 1u : 0u;
        if (++pj == n) { pi++; pj = pi + 1; }
    }
    return cnt;
}

// Three launches, none of which waits on another work-group: the candidates
// of every tile are counted, the counts are scanned by one work-group into
// tile offsets, and every tile writes its candidates (reading q again).
// Cross-XCD status polling and a shared tile ticket cost more than the
// second read of q.
__global__ __launch_bounds__(VR_BLOCK) void k_sel_count(VrDev D) {
    __shared__ uint32_t sh_w[VR_WAVES];
    SelItems I;
    const uint32_t c = select_items(D, (int)blockIdx.x, I);
    uint32_t tot;
    (void)block_excl_scan<uint32_t>(c, sh_w, &tot);
    if (threadIdx.x == 0) D.st_sel[blockIdx.x] = tot;
}

// One work-group: exclusive scan of the tile counts in place; the total is
// the candidate count.
#define SCAN_BLOCK 1024
__global__ __launch_bounds__(SCAN_BLOCK) void k_sel_scan(VrDev D) {
    __shared__ uint32_t sh_w[SCAN_BLOCK / VR_WAVE];
    __shared__ uint32_t sh_carry;
    const int ntiles = (int)D.ntile_E, t = threadIdx.x;
    if (t == 0) sh_carry = 0u;
    __syncthreads();
    for (int base = 0; base < ntiles; base += SCAN_BLOCK) {
        const int i = base + t;
        const uint32_t v = (i < ntiles) ? D.st_sel[i] : 0u;
        const uint32_t inc = wave_incl_scan_dpp(v);
        const int w = t / VR_WAVE;
        if ((t & 63) == 63) sh_w[w] = inc;
        __syncthreads();
        uint32_t off = sh_carry, tot = 0;
        for (int x = 0; x < SCAN_BLOCK / VR_WAVE; x++) {
            const uint32_t y = sh_w[x];
            if (x < w) off += y;
            tot += y;
        }
        if (i < ntiles) D.st_sel[i] = off + inc - v;
        __syncthreads();
        if (t == 0) sh_carry += tot;
        __syncthreads();
    }
    if (t == 0) D.ctl->n_cand = sh_carry;
}

__global__ __launch_bounds__(VR_BLOCK) void k_sel_write(VrDev D) {
    __shared__ uint32_t sh_w[VR_WAVES];
    __shared__ uint32_t h8[VR_MAX_PASSES][VR_RADIX];
    VrCtl *ctl = D.ctl;
    const int t = threadIdx.x, tile = (int)blockIdx.x;
    for (int x = t; x < VR_MAX_PASSES * VR_RADIX; x += VR_BLOCK) (&h8[0][0])[x] = 0u;
    // clear this tile's statuses for the first active radix pass
    D.st_sort[0][(size_t)tile * VR_RADIX + t] = 0u;
    SelItems I;
    const uint32_t c = select_items(D, tile, I);
    uint32_t tt;
    const uint32_t ex = block_excl_scan<uint32_t>(c, sh_w, &tt);  // also orders the h8 clear
    uint32_t p = D.st_sel[tile] + ex;
#pragma unroll
    for (int m = 0; m < VR_ITEMS; m++) {
        if (I.first[m]) D.cs[I.cc[m]].cand_base = p;
        if (I.keep[m]) {
            D.key[0][p] = I.kv[m];
            D.val[0][p] = I.vv[m];
            p++;
        }
    }
    if (tt == 0) return;  // nothing to histogram (uniform over the work-group)
    // digit histograms: low digits are spread, the top one (cloud and high
    // bits of q) takes few values
    for (int ps = 0; ps < D.passes - 1; ps++)
#pragma unroll
        for (int m = 0; m < VR_ITEMS; m++) spread_add(h8[ps], (I.kv[m] >> (8 * ps)) & 255u, I.keep[m]);
#pragma unroll
    for (int m = 0; m < VR_ITEMS; m++)
        narrow_add<8>(h8[D.passes - 1], (I.kv[m] >> (8 * (D.passes - 1))) & 255u, I.keep[m]);
    __syncthreads();
    uint32_t *gh = hist_copy(&ctl->hist8[0][0][0], VR_HIST8_STRIDE);
    for (int x = t; x < D.passes * VR_RADIX; x += VR_BLOCK) {
        const uint32_t v = (&h8[0][0])[x];
        if (v) atomicAdd(&gh[x], v);
    }
}

void launch_select(const VrDev &D, hipStream_t s) {
    const dim3 grid((unsigned)(D.ntile_E > 0 ? D.ntile_E : 1));
    hipLaunchKernelGGL(k_sel_count, grid, dim3(VR_BLOCK), 0, s, D);
    hipLaunchKernelGGL(k_sel_scan, dim3(1), dim3(SCAN_BLOCK), 0, s, D);
    hipLaunchKernelGGL(k_sel_write, grid, dim3(VR_BLOCK), 0, s, D);
}

// Sum the VR_HCOPY copies of a histogram set into copy 0, which is all its
// readers then read (one work-group).
#define FOLD_BLOCK 1024
__global__ __launch_bounds__(FOLD_BLOCK) void k_hist_fold(uint32_t *h0, int stride, int bins) {
    for (int x = threadIdx.x; x < bins; x += FOLD_BLOCK) h0[x] = hist_sum(h0, stride, VR_HCOPY, x);
}

void launch_hist_fold(uint32_t *h0, int stride, int bins, hipStream_t s) {
    hipLaunchKernelGGL(k_hist_fold, dim3(1), dim3(FOLD_BLOCK), 0, s, h0, stride, bins);
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
    J.hist = &D.ctl->hist8[0][0][0];  // copy 0, folded
    J.ticket = &D.ctl->ticket[1];
    J.st[0] = D.st_sort[0]; J.st[1] = D.st_sort[1];
    J.count = &D.ctl->n_cand;
    J.cap = D.E > 0 ? D.E : 1;
    J.passes = D.passes;
    return J;
}

// ---------------------------------------------------------- k_sort_pass ----
// Tiles of 2048 keys; each wave ranks its 512 keys among equal digits in
// order (8 ballots per 64 keys), the work-group combines the waves, one
// look-back per digit gives the tile's global offsets, and the tile is
// scattered through LDS so equal digits leave as contiguous runs.
__global__ __launch_bounds__(VR_BLOCK) void k_sort_pass(SortJob J, int pass, int S) {
    __shared__ uint32_t s_whist[VR_WAVES][VR_RADIX];
    __shared__ uint32_t s_tstart[VR_RADIX];
    __shared__ uint32_t s_gpre[VR_RADIX];
    __shared__ uint32_t s_key[VR_TILE];
    __shared__ uint32_t s_val[VR_TILE];
    __shared__ uint32_t sh_w[VR_WAVES];
    __shared__ uint32_t sh_nz[VR_MAX_PASSES][VR_WAVES];
    __shared__ int sh_tile;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    // S == 0: tile = blockIdx.x, one per work-group, with every tile's
    // work-group launched; else tiles are claimed S at a time from the pass's
    // ticket.  Everything needed first is loaded at once: the item count,
    // this thread's digit in every pass's histogram and, with direct tiles,
    // the tile's keys from both buffers (which one holds the input depends on
    // the passes skipped so far, known only from the histograms).  Loads
    // are clamped to the buffers; items past the count are never used.
    const bool direct = S == 0;
    const uint32_t Kc = *J.count;
    uint32_t hv[VR_MAX_PASSES];
#pragma unroll
    for (int p = 0; p < VR_MAX_PASSES; p++) hv[p] = J.hist[p * VR_RADIX + t];
    uint32_t kA[VR_ITEMS], kB[VR_ITEMS];
    {
        const long long base = (long long)blockIdx.x * VR_TILE + (long long)w * (VR_TILE / VR_WAVES);
#pragma unroll
        for (int it = 0; it < VR_ITEMS; it++) {
            const long long idx = min(base + (long long)it * VR_WAVE + lane, J.cap - 1);
            kA[it] = direct ? J.key[0][idx] : 0u;
            kB[it] = direct ? J.key[1][idx] : 0u;
        }
    }
    // passes whose digit takes more than one value are active; the others
    // are skipped and do not flip the buffers
#pragma unroll
    for (int p = 0; p < VR_MAX_PASSES; p++) {
        const uint32_t nz = (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(hv[p] != 0u));
        if (lane == 0) sh_nz[p][w] = nz;
    }
    __syncthreads();
    int a = 0;
    bool active = false;
    uint32_t hp = 0;
#pragma unroll
    for (int p = 0; p < VR_MAX_PASSES; p++) {
        uint32_t nz = 0;
#pragma unroll
        for (int x = 0; x < VR_WAVES; x++) nz += sh_nz[p][x];
        if (p < pass && p < J.passes) a += (nz > 1) ? 1 : 0;
        if (p == pass) {
            active = nz > 1;
            hp = hv[p];
        }
    }
    const int ntiles = (int)((Kc + VR_TILE - 1) / VR_TILE);
    if (!active || (int)blockIdx.x >= ntiles) return;  // surplus work-groups never touch the ticket
    const uint32_t *__restrict__ vsrc = J.val[a & 1];
    const uint32_t *__restrict__ ksrc = J.key[a & 1];
    uint32_t *__restrict__ kdst = J.key[(a + 1) & 1];
    uint32_t *__restrict__ vdst = J.val[(a + 1) & 1];
    uint32_t *st = J.st[a & 1];
    uint32_t *st_next = J.st[(a + 1) & 1];
    const int shift = VR_RADIX_BITS * pass;

    // global start of digit t
    uint32_t tot;
    const uint32_t gstart = block_excl_scan<uint32_t>(hp, sh_w, &tot);

    auto do_tile = [&](int tile, const uint32_t (&kk)[VR_ITEMS]) {
        for (int x = 0; x < VR_WAVES; x++) s_whist[x][t] = 0u;
        __syncthreads();
        uint32_t vv[VR_ITEMS], rk[VR_ITEMS];
        const long long base = (long long)tile * VR_TILE + (long long)w * (VR_TILE / VR_WAVES);
        // values at clamped addresses, issued before the ranking (items
        // past the count are never used)
#pragma unroll
        for (int it = 0; it < VR_ITEMS; it++) vv[it] = vsrc[min(base + (long long)it * VR_WAVE + lane, J.cap - 1)];
#pragma unroll
        for (int it = 0; it < VR_ITEMS; it++) {
            const long long idx = base + (long long)it * VR_WAVE + lane;
            const bool valid = idx < (long long)Kc;
            const uint32_t k = kk[it];
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
            // the wave's LDS operations run in order; keep the compiler
            // from moving the next item's read above this write
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
    };
    if (direct) {
        uint32_t kk[VR_ITEMS];
#pragma unroll
        for (int it = 0; it < VR_ITEMS; it++) kk[it] = (a & 1) ? kB[it] : kA[it];
        do_tile((int)blockIdx.x, kk);
        return;
    }
    for (;;) {
        const int t0 = claim_tiles(&J.ticket[pass], S, &sh_tile);
        if (t0 >= ntiles) break;
        for (int tile = t0; tile < min(t0 + S, ntiles); tile++) {
            if (tile > t0) __syncthreads();  // LDS of the previous tile is reused
            uint32_t kk[VR_ITEMS];
            const long long base = (long long)tile * VR_TILE + (long long)w * (VR_TILE / VR_WAVES);
#pragma unroll
            for (int it = 0; it < VR_ITEMS; it++) kk[it] = ksrc[min(base + (long long)it * VR_WAVE + lane, J.cap - 1)];
            do_tile(tile, kk);
        }
        if ((int)gridDim.x >= ntiles) break;  // every tile went out in the first round of claims
    }
}

// ---------------------------------------------------- k_sort_pass_multi ----
// The same stable pass for large key counts, where one ticket per tile would
// serialise on the ticket: a work-group claims S consecutive tiles, first
// counts the digits of all S (publishing every tile's aggregate at once, so
// that later claims never wait for this one's scatter), then looks back once
// for its first tile, publishes the inclusive prefixes of all S, and finally
// re-reads, ranks and scatters each tile as the single-tile pass does.
#define SORT_MULTI_MAX 16
__global__ __launch_bounds__(VR_BLOCK) void k_sort_pass_multi(SortJob J, int pass) {
    __shared__ uint32_t s_whist[VR_WAVES][VR_RADIX];
    __shared__ uint32_t s_tstart[VR_RADIX];
    __shared__ uint32_t s_gpre[VR_RADIX];
    __shared__ uint32_t s_key[VR_TILE];
    __shared__ uint32_t s_val[VR_TILE];
    __shared__ uint32_t s_cnt[SORT_MULTI_MAX][VR_RADIX];  // digit counts of the claimed tiles
    __shared__ uint32_t sh_w[VR_WAVES];
    __shared__ int sh_tile;
    bool active = false;
    const uint32_t Kc = *J.count;
    const int ntiles = (int)((Kc + VR_TILE - 1) / VR_TILE);
    // tiles per claim from the device-side count: about a thousand claims
    const int S = max(1, min(SORT_MULTI_MAX, ntiles / 1024));
    const int nclaims = (ntiles + S - 1) / S;
    if ((int)blockIdx.x >= nclaims) return;  // surplus work-groups never touch the ticket
    const int a = active_before(J.hist, J.passes, pass, &active);
    if (!active) return;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const uint32_t *__restrict__ ksrc = J.key[a & 1];
    const uint32_t *__restrict__ vsrc = J.val[a & 1];
    uint32_t *__restrict__ kdst = J.key[(a + 1) & 1];
    uint32_t *__restrict__ vdst = J.val[(a + 1) & 1];
    uint32_t *st = J.st[a & 1];
    uint32_t *st_next = J.st[(a + 1) & 1];
    const int shift = VR_RADIX_BITS * pass;
    uint32_t tot;
    const uint32_t gstart = block_excl_scan<uint32_t>(J.hist[pass * VR_RADIX + t], sh_w, &tot);

    for (;;) {
        const int t0 = claim_tiles(&J.ticket[pass], S, &sh_tile);
        if (t0 >= ntiles) break;
        const int nt = min(S, ntiles - t0);
        // counts of every claimed tile, then all their aggregates
        for (int j = 0; j < SORT_MULTI_MAX; j++) s_cnt[j][t] = 0u;
        __syncthreads();
        const bool top = pass == J.passes - 1;  // the top digit takes few values
        for (int j = 0; j < nt; j++) {
            const long long base = (long long)(t0 + j) * VR_TILE + (long long)t * VR_ITEMS;
            uint32_t kk[VR_ITEMS];
#pragma unroll
            for (int it = 0; it < VR_ITEMS; it++) kk[it] = (base + it < (long long)Kc) ? ksrc[base + it] : 0u;
#pragma unroll
            for (int it = 0; it < VR_ITEMS; it++) {
                const bool valid = base + it < (long long)Kc;
                const uint32_t dg = (kk[it] >> shift) & 255u;
                if (top) narrow_add<8>(s_cnt[j], dg, valid);
                else spread_add(s_cnt[j], dg, valid);
            }
        }
        __syncthreads();
        for (int j = 0; j < nt; j++) {
            const int tile = t0 + j;
            if (tile == 0) st_store32(st + t, st_pack32(VR_ST_INC, s_cnt[0][t]));
            else st_store32(st + (size_t)tile * VR_RADIX + t, st_pack32(VR_ST_AGG, s_cnt[j][t]));
        }
        // one look-back for the first tile; the others follow from the
        // counts.  s_cnt[j][t] becomes tile j's prefix of digit t.
        uint32_t run = (t0 == 0) ? 0u : lookback32(st + t, t0, VR_RADIX);
        for (int j = 0; j < nt; j++) {
            const int tile = t0 + j;
            const uint32_t c = s_cnt[j][t];
            if (tile > 0) st_store32(st + (size_t)tile * VR_RADIX + t, st_pack32(VR_ST_INC, run + c));
            st_next[(size_t)tile * VR_RADIX + t] = 0u;
            s_cnt[j][t] = run;
            run += c;
        }
        for (int j = 0; j < nt; j++) {
            const int tile = t0 + j;
            __syncthreads();  // LDS of the previous tile is reused
            for (int x = 0; x < VR_WAVES; x++) s_whist[x][t] = 0u;
            __syncthreads();
            uint32_t kk[VR_ITEMS], vv[VR_ITEMS], rk[VR_ITEMS];
            const long long base = (long long)tile * VR_TILE + (long long)w * (VR_TILE / VR_WAVES);
#pragma unroll
            for (int it = 0; it < VR_ITEMS; it++) {
                const long long idx = base + (long long)it * VR_WAVE + lane;
                const bool valid = idx < (long long)Kc;
                kk[it] = valid ? ksrc[idx] : 0u;
                vv[it] = valid ? vsrc[idx] : 0u;
            }
#pragma unroll
            for (int it = 0; it < VR_ITEMS; it++) {
                const long long idx = base + (long long)it * VR_WAVE + lane;
                const bool valid = idx < (long long)Kc;
                const uint32_t dg = (kk[it] >> shift) & 255u;
                unsigned long long peers = ballot64(valid);
#pragma unroll
                for (int b = 0; b < VR_RADIX_BITS; b++) {
                    const unsigned long long m = ballot64((dg >> b) & 1u);
                    peers &= ((dg >> b) & 1u) ? m : ~m;
                }
                uint32_t before = 0;
                if (valid) before = s_whist[w][dg];
                rk[it] = before + (uint32_t)__popcll(peers & lanemask_lt());
                if (valid && (peers & lanemask_lt()) == 0ull) s_whist[w][dg] = before + (uint32_t)__popcll(peers);
                __builtin_amdgcn_wave_barrier();
            }
            __syncthreads();
            uint32_t wpre[VR_WAVES];
            uint32_t tc = 0;
#pragma unroll
            for (int x = 0; x < VR_WAVES; x++) { wpre[x] = tc; tc += s_whist[x][t]; }
            uint32_t ttot;
            s_tstart[t] = block_excl_scan<uint32_t>(tc, sh_w, &ttot);
            s_gpre[t] = gstart + s_cnt[j][t];
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
                    kdst[s_gpre[dg] + (lp - s_tstart[dg])] = k;
                    vdst[s_gpre[dg] + (lp - s_tstart[dg])] = s_val[lp];
                }
            }
        }
        __syncthreads();  // s_cnt is reused by the next claim
    }
}

void launch_sort_pass(const SortJob &J, long long max_tiles, int pass, hipStream_t s) {
    long long g = max_tiles;
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    if (max_tiles > 2048) {  // possibly many tiles: several per claim
        hipLaunchKernelGGL(k_sort_pass_multi, dim3((unsigned)g), dim3(VR_BLOCK), 0, s, J, pass);
        return;
    }
    // one tile per work-group (every tile's work-group is launched and all
    // fit on the device at once), else one tile per claim: a tile's
    // aggregate is published as soon as it is ranked
    hipLaunchKernelGGL(k_sort_pass, dim3((unsigned)g), dim3(VR_BLOCK), 0, s, J, pass, max_tiles <= 1024 ? 0 : 1);
}

// -------------------------------------------------------------- k_edges ----
// Kept edge g of cloud c is the (g - kbase_c)-th candidate of the cloud in
// sorted order.  With triangles wanted, its rank within the cloud, tagged
// with the build's tag in the top byte, also goes to entries [i][j] and
// [j][i] of the cloud's rank matrix, which k_rows turns into stars.
__global__ __launch_bounds__(VR_BLOCK) void k_edges(VrDev D) {
    VrCtl *ctl = D.ctl;
    const int a = active_before(&ctl->hist8[0][0][0], D.passes, VR_MAX_PASSES, nullptr);
    const uint32_t *__restrict__ kf = D.key[a & 1];
    const uint32_t *__restrict__ vf = D.val[a & 1];
    const long long K = (D.thr_kind == 3) ? (long long)ctl->n_cand : D.K_host;
    const uint32_t qmask = (D.qbits >= 32) ? 0xFFFFFFFFu : ((1u << D.qbits) - 1u);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->n_kept = (uint32_t)K;
        // without triangles this is the last phase-1 kernel of a single build
        if (!D.tri && D.C == 1) publish_counts(D.mailbox, D.seq, ctl->flags, ctl->n_cand, (uint32_t)K, 0ull);
    }
    // Work-groups go to the 8 XCDs in turn (b -> XCD b % 8).  Each XCD takes
    // one contiguous eighth of the edges and its work-groups stride through
    // it together, so the rank-matrix stores of one XCD fall into the
    // matrices of few clouds at a time and gather in that XCD's L2.
    const uint32_t G = gridDim.x, x8 = blockIdx.x % 8, i8 = blockIdx.x / 8;
    const long long nb8 = (long long)(G / 8) + (x8 < G % 8 ? 1 : 0), span8 = (K + 7) / 8;
    const long long gend = min(K, (long long)(x8 + 1) * span8);
    for (long long g = (long long)x8 * span8 + (long long)i8 * VR_BLOCK + threadIdx.x; g < gend;
         g += nb8 * VR_BLOCK) {
        const int c = (D.thr_kind == 3)  // kept bases known only on the device: search
                          ? cloud_of(g, D.C, [&](int k) { return kept_base(D, k); })
                          : cloud_from_map(D, D.kcloud, g, VR_BLOCK, [&](int k) { return D.cl[k].kbase; });
        const long long lr = g - kept_base(D, c);  // rank within the cloud
        const long long sp = (long long)D.cs[c].cand_base + lr;
        const uint32_t k = kf[sp], v = vf[sp];
        D.se_q[g] = k & qmask;
        D.se_ij[g] = v;
        if (D.tri) {
            // rank matrix: (tag, rank) at [i][j] and [j][i] of the cloud's star slots
            const uint32_t mb = (uint32_t)D.cl[c].mbase, n = (uint32_t)D.cl[c].n;
            const uint32_t i = v >> 16, j = v & 0xFFFFu, e = (D.tag << 24) | (uint32_t)lr;
            D.star_r[mb + i * n + j] = e;
            D.star_r[mb + j * n + i] = e;
        }
    }
}

void launch_edges(const VrDev &D, hipStream_t s) {
    long long K = (D.thr_kind == 3) ? D.E : D.K_host;
    long long g = (K + VR_BLOCK - 1) / VR_BLOCK;
    if (g > 1024) g = 1024;
    if (g < 8) g = 8;  // every XCD's eighth of the edges needs a work-group
    hipLaunchKernelGGL(k_edges, dim3((unsigned)g), dim3(VR_BLOCK), 0, s, D);
}
