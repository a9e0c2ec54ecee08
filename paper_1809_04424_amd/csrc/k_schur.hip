// k_schur.hip -- the F2 sparse product and sum S = D + C E of the Schur
// complement step (Section 4.6), for matrices in compressed sparse columns.
//
// Column j of S is column j of D plus the columns of C that column j of E
// selects, added mod 2.  A work-group takes one column at a time and XORs
// every row of those columns into a bitmap of the m rows in LDS (a row
// reached an even number of times cancels); the set bits, read in order,
// are column j of S with its rows ascending.  Columns are independent, as
// in the paper's column partition among workers; their offsets in S are an
// exclusive scan of the per-column counts (the paper's master adjusts the
// column pointers the same way).
//   k_bp_column<false>  count the rows of every column of S
//   k_bp_scan           the counts into column pointers
//   k_bp_column<true>   write the rows of every column of S
// (k_bp_column_wave: the same with one column per wave, for m <= 32768)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vr.h"

#define BP_BLOCK 256
#define BP_WAVE 64
#define BP_MAX_WORDS 8192  // bitmap words: m <= 262144 rows (32 KB of LDS)
#define BP_SCAN_BLOCK 1024
#define BP_SCAN_ITEMS 4

static __device__ __forceinline__ int64_t bp_clamp(int64_t x, int64_t lo, int64_t hi) {
    return x < lo ? lo : (x > hi ? hi : x);
}

struct BpArgs {
    int64_t m, k, n;
    const int64_t *cp_c, *cp_e, *cp_d;
    const int32_t *r_c, *r_e, *r_d;
};

// Column ranges are clamped into [0, nnz] of their matrix and rows outside
// the matrix are skipped, so malformed input cannot reach outside the
// arrays; it only gives an unspecified S.
template <bool WRITE>
__global__ void __launch_bounds__(BP_BLOCK) k_bp_column(BpArgs A, int64_t *s_colptr, int32_t *s_rows) {
    __shared__ uint32_t bm[BP_MAX_WORDS];
    __shared__ uint32_t wsum[BP_BLOCK / BP_WAVE];
    const int t = threadIdx.x, lane = t % BP_WAVE, wv = t / BP_WAVE;
    const int W = (int)((A.m + 31) / 32);
    const int64_t nnz_c = A.cp_c[A.k], nnz_e = A.cp_e[A.n], nnz_d = A.cp_d[A.n];
    const int64_t s_total = WRITE ? s_colptr[A.n] : 0;
    // thread t reads words [w0, w1) in order when collecting the column
    const int per = (W + BP_BLOCK - 1) / BP_BLOCK;
    const int w0 = min(t * per, W), w1 = min(w0 + per, W);
    for (int64_t j = blockIdx.x; j < A.n; j += gridDim.x) {
        for (int x = t; x < W; x += BP_BLOCK) bm[x] = 0u;
        __syncthreads();
        const int64_t d0 = bp_clamp(A.cp_d[j], 0, nnz_d), d1 = bp_clamp(A.cp_d[j + 1], d0, nnz_d);
        for (int64_t x = d0 + t; x < d1; x += BP_BLOCK) {
            const int32_t r = A.r_d[x];
            if (r >= 0 && r < A.m) atomicXor(&bm[r >> 5], 1u << (r & 31));
        }
        // wave wv takes the selected columns of C in turn; its lanes walk one
        const int64_t e0 = bp_clamp(A.cp_e[j], 0, nnz_e), e1 = bp_clamp(A.cp_e[j + 1], e0, nnz_e);
        for (int64_t e = e0 + wv; e < e1; e += BP_BLOCK / BP_WAVE) {
            const int32_t kk = A.r_e[e];
            if (kk < 0 || kk >= A.k) continue;
            const int64_t c0 = bp_clamp(A.cp_c[kk], 0, nnz_c), c1 = bp_clamp(A.cp_c[kk + 1], c0, nnz_c);
            for (int64_t x = c0 + lane; x < c1; x += BP_WAVE) {
                const int32_t r = A.r_c[x];
                if (r >= 0 && r < A.m) atomicXor(&bm[r >> 5], 1u << (r & 31));
            }
        }
        __syncthreads();
        uint32_t own = 0;
        for (int x = w0; x < w1; x++) own += (uint32_t)__popc(bm[x]);
        uint32_t incl = own;
#pragma unroll
        for (int d = 1; d < BP_WAVE; d <<= 1) {
            const uint32_t y = __shfl_up(incl, d, BP_WAVE);
            if (lane >= d) incl += y;
        }
        if (lane == BP_WAVE - 1) wsum[wv] = incl;
        __syncthreads();
        uint32_t before = incl - own, total = 0;
#pragma unroll
        for (int i = 0; i < BP_BLOCK / BP_WAVE; i++) {
            if (i < wv) before += wsum[i];
            total += wsum[i];
        }
        if (!WRITE) {
            if (t == 0) s_colptr[j + 1] = total;
        } else {
            int64_t pos = s_colptr[j] + before;
            for (int x = w0; x < w1; x++) {
                uint32_t b = bm[x];
                while (b) {
                    const int bit = __ffs(b) - 1;
                    b &= b - 1;
                    if (pos < s_total) s_rows[pos] = x * 32 + bit;
                    pos++;
                }
            }
        }
        __syncthreads();  // the bitmap and the totals are reused by the next column
    }
}

// The same per column, one column per wave, for m <= 32 * BP_WAVE_WORDS:
// each wave owns a bitmap of its own, so a work-group keeps four columns in
// flight and no column waits on a work-group barrier (a wave's LDS accesses
// stay in order; the fences keep the compiler from moving them).
#define BP_WAVE_WORDS 1024  // m <= 32768 rows
template <bool WRITE>
__global__ void __launch_bounds__(BP_BLOCK) k_bp_column_wave(BpArgs A, int64_t *s_colptr, int32_t *s_rows) {
    __shared__ uint32_t bms[BP_BLOCK / BP_WAVE][BP_WAVE_WORDS];
    const int t = threadIdx.x, lane = t % BP_WAVE, wv = t / BP_WAVE;
    uint32_t *bm = bms[wv];
    const int W = (int)((A.m + 31) / 32);
    const int64_t nnz_c = A.cp_c[A.k], nnz_e = A.cp_e[A.n], nnz_d = A.cp_d[A.n];
    const int64_t s_total = WRITE ? s_colptr[A.n] : 0;
    const int per = (W + BP_WAVE - 1) / BP_WAVE;
    const int w0 = min(lane * per, W), w1 = min(w0 + per, W);
    const int64_t waves = (int64_t)gridDim.x * (BP_BLOCK / BP_WAVE);
    for (int64_t j = (int64_t)blockIdx.x * (BP_BLOCK / BP_WAVE) + wv; j < A.n; j += waves) {
        for (int x = lane; x < W; x += BP_WAVE) bm[x] = 0u;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int64_t d0 = bp_clamp(A.cp_d[j], 0, nnz_d), d1 = bp_clamp(A.cp_d[j + 1], d0, nnz_d);
        for (int64_t x = d0 + lane; x < d1; x += BP_WAVE) {
            const int32_t r = A.r_d[x];
            if (r >= 0 && r < A.m) atomicXor(&bm[r >> 5], 1u << (r & 31));
        }
        // the lanes load the ranges of up to 64 selected columns of C at
        // once, then the wave walks them one by one (their row loads do not
        // depend on each other)
        const int64_t e0 = bp_clamp(A.cp_e[j], 0, nnz_e), e1 = bp_clamp(A.cp_e[j + 1], e0, nnz_e);
        for (int64_t base = e0; base < e1; base += BP_WAVE) {
            const int64_t e = base + lane;
            const int32_t kk = e < e1 ? A.r_e[e] : -1;
            const bool ok = kk >= 0 && kk < A.k;
            const int64_t c0 = ok ? bp_clamp(A.cp_c[kk], 0, nnz_c) : 0;
            const int64_t c1 = ok ? bp_clamp(A.cp_c[kk + 1], c0, nnz_c) : 0;
            const int cnt = (int)min((int64_t)BP_WAVE, e1 - base);
#pragma unroll 4
            for (int i = 0; i < cnt; i++) {
                const int64_t a = __shfl(c0, i, BP_WAVE), b = __shfl(c1, i, BP_WAVE);
                for (int64_t x = a + lane; x < b; x += BP_WAVE) {
                    const int32_t r = A.r_c[x];
                    if (r >= 0 && r < A.m) atomicXor(&bm[r >> 5], 1u << (r & 31));
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        uint32_t own = 0;
        for (int x = w0; x < w1; x++) own += (uint32_t)__popc(bm[x]);
        uint32_t incl = own;
#pragma unroll
        for (int d = 1; d < BP_WAVE; d <<= 1) {
            const uint32_t y = __shfl_up(incl, d, BP_WAVE);
            if (lane >= d) incl += y;
        }
        const uint32_t total = __shfl(incl, BP_WAVE - 1, BP_WAVE);
        if (!WRITE) {
            if (lane == 0) s_colptr[j + 1] = total;
        } else {
            int64_t pos = s_colptr[j] + (incl - own);
            for (int x = w0; x < w1; x++) {
                uint32_t b = bm[x];
                while (b) {
                    const int bit = __ffs(b) - 1;
                    b &= b - 1;
                    if (pos < s_total) s_rows[pos] = x * 32 + bit;
                    pos++;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();  // the bitmap is cleared for the next column
    }
}

// s_colptr[0] = 0 and s_colptr[1..n] hold the counts: an inclusive scan in
// place, one work-group, chunk after chunk
__global__ void __launch_bounds__(BP_SCAN_BLOCK) k_bp_scan(int64_t *s_colptr, int64_t n) {
    __shared__ int64_t wtot[BP_SCAN_BLOCK / BP_WAVE];
    __shared__ int64_t carry_s;
    const int t = threadIdx.x, lane = t % BP_WAVE, wv = t / BP_WAVE;
    if (t == 0) {
        s_colptr[0] = 0;
        carry_s = 0;
    }
    __syncthreads();
    constexpr int CH = BP_SCAN_BLOCK * BP_SCAN_ITEMS;
    for (int64_t base = 1; base <= n; base += CH) {
        int64_t v[BP_SCAN_ITEMS], own = 0;
#pragma unroll
        for (int i = 0; i < BP_SCAN_ITEMS; i++) {
            const int64_t x = base + (int64_t)t * BP_SCAN_ITEMS + i;
            v[i] = x <= n ? s_colptr[x] : 0;
            own += v[i];
        }
        int64_t incl = own;
#pragma unroll
        for (int d = 1; d < BP_WAVE; d <<= 1) {
            const int64_t y = __shfl_up(incl, d, BP_WAVE);
            if (lane >= d) incl += y;
        }
        if (lane == BP_WAVE - 1) wtot[wv] = incl;
        __syncthreads();
        int64_t run = carry_s + incl - own, total = 0;
        for (int i = 0; i < BP_SCAN_BLOCK / BP_WAVE; i++) {
            if (i < wv) run += wtot[i];
            total += wtot[i];
        }
#pragma unroll
        for (int i = 0; i < BP_SCAN_ITEMS; i++) {
            const int64_t x = base + (int64_t)t * BP_SCAN_ITEMS + i;
            run += v[i];
            if (x <= n) s_colptr[x] = run;
        }
        __syncthreads();  // every thread has read carry_s and wtot
        if (t == 0) carry_s += total;
        __syncthreads();
    }
}

static int bp_check(int64_t m, int64_t k, int64_t n, const int64_t *cp_c, const int32_t *r_c, const int64_t *cp_e,
                    const int32_t *r_e, const int64_t *cp_d, const int32_t *r_d, const int64_t *s_colptr) {
    (void)r_c;
    (void)r_e;
    (void)r_d;  // NULL only for a matrix without entries: never read then
    if (m < 0 || k < 0 || n < 0) return VR_EINVAL;
    if (!cp_c || !cp_e || !cp_d || !s_colptr) return VR_EINVAL;
    if ((m + 31) / 32 > BP_MAX_WORDS) return VR_E2BIG;
    return VR_OK;
}

static unsigned bp_grid(int64_t n) { return (unsigned)(n < 4096 ? (n > 0 ? n : 1) : 4096); }

extern "C" VR_API int vr_blockprodsum_count(int64_t m, int64_t k, int64_t n, const int64_t *c_colptr,
                                            const int32_t *c_rows, const int64_t *e_colptr, const int32_t *e_rows,
                                            const int64_t *d_colptr, const int32_t *d_rows, int64_t *s_colptr,
                                            void *stream) {
    const int st = bp_check(m, k, n, c_colptr, c_rows, e_colptr, e_rows, d_colptr, d_rows, s_colptr);
    if (st != VR_OK) return st;
    const hipStream_t s = (hipStream_t)stream;
    const BpArgs A{m, k, n, c_colptr, e_colptr, d_colptr, c_rows, e_rows, d_rows};
    if (n > 0 && m <= 32 * BP_WAVE_WORDS)
        hipLaunchKernelGGL(k_bp_column_wave<false>, dim3(bp_grid((n + 3) / 4)), dim3(BP_BLOCK), 0, s, A, s_colptr,
                           (int32_t *)nullptr);
    else if (n > 0)
        hipLaunchKernelGGL(k_bp_column<false>, dim3(bp_grid(n)), dim3(BP_BLOCK), 0, s, A, s_colptr, (int32_t *)nullptr);
    hipLaunchKernelGGL(k_bp_scan, dim3(1), dim3(BP_SCAN_BLOCK), 0, s, s_colptr, n);
    return hipGetLastError() == hipSuccess ? VR_OK : VR_EHIP;
}

extern "C" VR_API int vr_blockprodsum_write(int64_t m, int64_t k, int64_t n, const int64_t *c_colptr,
                                            const int32_t *c_rows, const int64_t *e_colptr, const int32_t *e_rows,
                                            const int64_t *d_colptr, const int32_t *d_rows, const int64_t *s_colptr,
                                            int32_t *s_rows, void *stream) {
    const int st = bp_check(m, k, n, c_colptr, c_rows, e_colptr, e_rows, d_colptr, d_rows, s_colptr);
    if (st != VR_OK) return st;
    if (n == 0) return VR_OK;
    if (!s_rows) return VR_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    const BpArgs A{m, k, n, c_colptr, e_colptr, d_colptr, c_rows, e_rows, d_rows};
    if (m <= 32 * BP_WAVE_WORDS)
        hipLaunchKernelGGL(k_bp_column_wave<true>, dim3(bp_grid((n + 3) / 4)), dim3(BP_BLOCK), 0, s, A,
                           (int64_t *)s_colptr, s_rows);
    else
        hipLaunchKernelGGL(k_bp_column<true>, dim3(bp_grid(n)), dim3(BP_BLOCK), 0, s, A, (int64_t *)s_colptr, s_rows);
    return hipGetLastError() == hipSuccess ? VR_OK : VR_EHIP;
}
