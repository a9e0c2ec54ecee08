// k_gram.hip -- squared distances of int8 points through the Gram identity
// q_ij = |x_i|^2 + |x_j|^2 - 2 <x_i, x_j>, with the inner products on the
// matrix cores (v_mfma_i32_16x16x64_i8: 16x16 output tile, 64-deep int8
// products, exact int32 accumulation).  Exact: |<x,y>| <= 16384 d and
// q <= 65025 d, both in int32 / uint32 for the dimensions routed here.
//
// A work-group owns a 64 x 64 tile of pairs (row block bi <= column block
// bj) of one cloud of the batch.  Both blocks of points are staged in LDS, zero-padded to a multiple
// of 64 coordinates (zeros change neither norms nor products).  Wave w
// computes rows 16w..16w+15 against the four 16-column blocks.  Each lane
// feeds the same 16-byte slice of coordinates to the A and B operands, so
// the products pair coordinates consistently for any lane-to-k assignment of
// the instruction.
#include "vr_device.h"

typedef int v4i __attribute__((ext_vector_type(4)));

#define GRAM_TB 64
#define GRAM_KC 64  // coordinates per MFMA step

__device__ __forceinline__ long long gram_tile_row_start(long long bi, long long nb) {
    return bi * nb - bi * (bi - 1) / 2;
}

// DPAD: d rounded up to a multiple of 64 (64, 128, 192 or 256), a
// compile-time constant so that staging indexes rows without divisions.
template <int DPAD>
__global__ __launch_bounds__(VR_BLOCK) void k_gram_i8(VrDev D) {
    constexpr int dpad = DPAD;
    const long long tg = blockIdx.x;
    const int c = (D.C == 1) ? 0 : (int)D.tcloud[tg];
    const VrCloud cl = D.cl[c];
    const int n = cl.n, d = D.d, need_hist = D.need_hist;
    const long long nb = (n + GRAM_TB - 1) / GRAM_TB, tl = tg - cl.tbase;
    // tile (bi, bj), bi <= bj, in row order
    long long ib = (long long)(((2.0 * nb + 1.0) - sqrt((2.0 * nb + 1.0) * (2.0 * nb + 1.0) - 8.0 * (double)tl)) * 0.5);
    if (ib < 0) ib = 0;
    if (ib > nb - 1) ib = nb - 1;
    while (ib > 0 && gram_tile_row_start(ib, nb) > tl) ib--;
    while (ib < nb - 1 && gram_tile_row_start(ib + 1, nb) <= tl) ib++;
    const int bi = (int)ib, bj = (int)(tl - gram_tile_row_start(ib, nb) + ib);
    const int8_t *__restrict__ pts = (const int8_t *)cl.points;
    uint32_t *__restrict__ q = D.q + cl.pbase;
    VrCtl *__restrict__ ctl = D.ctl;
    (void)ctl;
    extern __shared__ int4 lds4[];
    int8_t *xi = (int8_t *)lds4;                  // GRAM_TB * dpad
    int8_t *xj = xi + GRAM_TB * dpad;             // GRAM_TB * dpad
    int32_t *ni = (int32_t *)(xj + GRAM_TB * dpad);
    int32_t *nj = ni + GRAM_TB;
    uint32_t *hist = (uint32_t *)(nj + GRAM_TB);  // VR_NBUCKET
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;

    // stage both blocks (zero rows past n and coordinates past d): 16 bytes
    // at a time when every row starts on a 16-byte boundary, else bytewise
    if ((d & 15) == 0 && ((uintptr_t)pts & 15) == 0) {
        constexpr int CPR = DPAD / 16;  // 16-byte chunks per staged row
        const int cd = d / 16;          // chunks holding coordinates
        for (int x = t; x < GRAM_TB * CPR; x += VR_BLOCK) {
            const int r = x / CPR, ch = x % CPR;
            const int gi = bi * GRAM_TB + r, gj = bj * GRAM_TB + r;
            int4 vi = make_int4(0, 0, 0, 0), vj = make_int4(0, 0, 0, 0);
            if (ch < cd) {
                if (gi < n) vi = *(const int4 *)(pts + (size_t)gi * d + 16 * ch);
                if (gj < n) vj = *(const int4 *)(pts + (size_t)gj * d + 16 * ch);
            }
            ((int4 *)xi)[x] = vi;
            ((int4 *)xj)[x] = vj;
        }
    } else {
        for (int x = t; x < GRAM_TB * dpad; x += VR_BLOCK) {
            const int r = x / dpad, c = x % dpad;
            const int gi = bi * GRAM_TB + r, gj = bj * GRAM_TB + r;
            xi[x] = (gi < n && c < d) ? pts[(size_t)gi * d + c] : (int8_t)0;
            xj[x] = (gj < n && c < d) ? pts[(size_t)gj * d + c] : (int8_t)0;
        }
    }
    if (need_hist)
        for (int b = t; b < VR_NBUCKET; b += VR_BLOCK) hist[b] = 0u;
    __syncthreads();
    if (t < 2 * GRAM_TB) {
        // squared norm of one staged row, 4 coordinates per 32-bit word
        const int *row = (const int *)((t < GRAM_TB) ? xi + t * dpad : xj + (t - GRAM_TB) * dpad);
        int32_t s = 0;
#pragma unroll 4
        for (int c = 0; c < dpad / 4; c++) {
            const int v = row[c];
#pragma unroll
            for (int b = 0; b < 4; b++) {
                const int x = (int)(int8_t)(v >> (8 * b));  // signed byte b
                s += x * x;
            }
        }
        if (t < GRAM_TB) ni[t] = s;
        else nj[t - GRAM_TB] = s;
    }
    __syncthreads();

    v4i acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; cb++) acc[cb] = (v4i){0, 0, 0, 0};
    const int r16 = lane & 15, g = lane >> 4;
    for (int k0 = 0; k0 < dpad; k0 += GRAM_KC) {
        const v4i a = *(const v4i *)(xi + (w * 16 + r16) * dpad + k0 + g * 16);
#pragma unroll
        for (int cb = 0; cb < 4; cb++) {
            const v4i b = *(const v4i *)(xj + (cb * 16 + r16) * dpad + k0 + g * 16);
            acc[cb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc[cb], 0, 0, 0);
        }
    }

#pragma unroll
    for (int cb = 0; cb < 4; cb++) {
        const int jl = cb * 16 + r16;
        const int j = bj * GRAM_TB + jl;
#pragma unroll
        for (int ii = 0; ii < 4; ii++) {
            const int il = w * 16 + g * 4 + ii;
            const int i = bi * GRAM_TB + il;
            const bool ok = i < j && j < n;
            uint32_t qq = 0;
            if (ok) {
                qq = (uint32_t)(ni[il] + nj[jl] - 2 * acc[cb][ii]);
                q[row_start(i, n) + (j - i - 1)] = qq;
            }
            if (need_hist) spread_add(hist, bucket_of(qq), ok);
        }
    }
    if (need_hist) {
        __syncthreads();
        uint32_t *gh = D.hist + ((size_t)c * D.hcopies + blockIdx.x % D.hcopies) * VR_NBUCKET;
        for (int b = t; b < VR_NBUCKET; b += VR_BLOCK)
            if (hist[b]) atomicAdd(&gh[b], hist[b]);
    }
}

size_t gram_lds(int dpad) { return 2 * (size_t)GRAM_TB * dpad + 2 * GRAM_TB * 4 + VR_NBUCKET * 4; }

// Route int8 clouds with enough coordinates to the matrix cores.
bool gram_applies(const VrDev &D) { return D.dtype == 1 && D.d >= 16 && D.d <= 256; }

void launch_gram(const VrDev &D, const void *points, hipStream_t s) {
    (void)points;
    const int dpad = (D.d + GRAM_KC - 1) / GRAM_KC * GRAM_KC;  // gram_applies: 64 .. 256
    const dim3 grid((unsigned)D.tiles), block(VR_BLOCK);
    switch (dpad) {
    case 64: hipLaunchKernelGGL(k_gram_i8<64>, grid, block, gram_lds(64), s, D); break;
    case 128: hipLaunchKernelGGL(k_gram_i8<128>, grid, block, gram_lds(128), s, D); break;
    case 192: hipLaunchKernelGGL(k_gram_i8<192>, grid, block, gram_lds(192), s, D); break;
    default: hipLaunchKernelGGL(k_gram_i8<256>, grid, block, gram_lds(256), s, D); break;
    }
}
