// k_colsort.hip -- per-column stable ordering of a compressed-sparse-column
// array (Section 4.3: the slot every entry takes when its column is sorted by
// value, equal values keeping their order).
//
// The entries are cut into windows of CO_WIN consecutive entries, whatever
// the columns.  A window's entries fall into segments, one per column that
// meets the window.
//   k_co_first  per column: the windows whose first entry lies in it.
//   k_co_local  per window: each entry's rank inside its segment (counting
//               against the segment in LDS when every segment is short, an
//               LDS bitonic sort otherwise), plus the column's first slot;
//               the sorted values of segments whose column leaves the window
//               are kept for the next kernel.
//   k_co_merge  per window, only for the (at most two) columns that leave
//               it: adds, for every other window the column meets, the
//               entries there that come first (binary search in that
//               window's sorted run: values <= x before, < x after).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "vr.h"
#include "vr_cache.h"

#define CO_BLOCK 256
#define CO_WIN 4096
#define CO_PER (CO_WIN / CO_BLOCK)
#define CO_COUNT_MAX 256  // longest segment ranked by counting
#define CO_WAVE 64

static __device__ __forceinline__ int64_t clampi(int64_t x, int64_t lo, int64_t hi) {
    return x < lo ? lo : (x > hi ? hi : x);
}

// first[w] = the column holding entry w*CO_WIN (the non-empty column c with
// colptr[c] <= w*CO_WIN < colptr[c+1]).
__global__ void __launch_bounds__(CO_BLOCK) k_co_first(const int64_t *colptr, int64_t ncols, int64_t nnz,
                                                      int64_t *first) {
    for (int64_t c = blockIdx.x * (int64_t)CO_BLOCK + threadIdx.x; c < ncols;
         c += (int64_t)gridDim.x * CO_BLOCK) {
        const int64_t s = clampi(colptr[c], 0, nnz), e = clampi(colptr[c + 1], s, nnz);
        if (e == s) continue;
        for (int64_t w = (s + CO_WIN - 1) / CO_WIN; w <= (e - 1) / CO_WIN; w++) first[w] = c;
    }
}

struct CoWindow {
    int64_t a;    // first entry
    int cnt;      // entries
    int64_t c0;   // column of the first entry
    int64_t cs0;  // first slot of that column
    int64_t cl;   // column of entry a + CO_WIN (next window), or -1
};

static __device__ __forceinline__ CoWindow co_window(const int64_t *colptr, int64_t ncols, int64_t nnz,
                                                     const int64_t *first, int64_t nwin, int64_t w) {
    CoWindow W;
    W.a = w * CO_WIN;
    W.cnt = (int)min((int64_t)CO_WIN, nnz - W.a);
    W.c0 = clampi(first[w], 0, ncols - 1);
    W.cs0 = clampi(colptr[W.c0], 0, W.a);
    W.cl = w + 1 < nwin ? clampi(first[w + 1], W.c0, ncols - 1) : -1;
    return W;
}

// LDS index of key position p: one pad slot per 16 keys, so that the lanes
// of layout C (16 keys apart) spread over the banks
static __device__ __forceinline__ int co_phys(int p) { return p + (p >> 4); }

// position of register g of thread t in layout LAY (0: C, 1: S, 2: L)
template <int LAY>
static __device__ __forceinline__ int co_pos(int t, int g) {
    return LAY == 0 ? CO_PER * t + g : (LAY == 1 ? 256 * (t >> 4) + 16 * g + (t & 15) : 256 * g + t);
}

template <int LAY>
static __device__ __forceinline__ void co_put(const unsigned long long (&r)[CO_PER], int t, unsigned long long *keys) {
#pragma unroll
    for (int g = 0; g < CO_PER; g++) keys[co_phys(co_pos<LAY>(t, g))] = r[g];
}

// move the keys from layout cur to layout TO through LDS
template <int TO>
static __device__ __forceinline__ void co_to(unsigned long long (&r)[CO_PER], int &cur, int t,
                                             unsigned long long *keys) {
    if (cur == TO) return;  // uniform over the work-group
    __syncthreads();        // earlier reads of the buffer are done
    if (cur == 0) co_put<0>(r, t, keys);
    else if (cur == 1) co_put<1>(r, t, keys);
    else co_put<2>(r, t, keys);
    __syncthreads();
#pragma unroll
    for (int g = 0; g < CO_PER; g++) r[g] = keys[co_phys(co_pos<TO>(t, g))];
    cur = TO;
}

// the stages of one merge width kk on the position bits that layout LAY
// holds in registers (bits 4*LAY .. 4*LAY+3, at most bhi), highest first
template <int LAY>
static __device__ __forceinline__ void co_stages(unsigned long long (&r)[CO_PER], int t, int kk, int bhi) {
#pragma unroll
    for (int gb = 3; gb >= 0; gb--) {
        if (4 * LAY + gb > bhi) continue;
        const int j = 1 << gb;
#pragma unroll
        for (int g = 0; g < CO_PER; g++) {
            if (g & j) continue;
            const int h = g | j;
            const bool up = (co_pos<LAY>(t, g) & kk) == 0;
            const unsigned long long k0 = r[g], k1 = r[h];
            const bool sw = (k0 > k1) == up;
            r[g] = sw ? k1 : k0;
            r[h] = sw ? k0 : k1;
        }
    }
}

__global__ void __launch_bounds__(CO_BLOCK) k_co_local(const int64_t *colptr, int64_t ncols, const int32_t *v,
                                                      int64_t nnz, const int64_t *first, int64_t nwin, int64_t *z,
                                                      uint32_t *vs) {
    // keys: counting path, the values with the sign bit flipped (unsigned
    // order); sorting path, the keys between layouts, then the slots
    __shared__ unsigned long long keys[CO_WIN + CO_WIN / 16];
    uint32_t *kv = (uint32_t *)keys;
    __shared__ uint16_t segid[CO_WIN];  // first the segment-start flags
    __shared__ uint16_t segstart[CO_WIN + 2];
    __shared__ uint32_t wsum[CO_BLOCK / CO_WAVE];
    __shared__ uint32_t maxlen;

    const int t = threadIdx.x, lane = t % CO_WAVE, wv = t / CO_WAVE;
    const CoWindow W = co_window(colptr, ncols, nnz, first, nwin, blockIdx.x);
    const int cnt = W.cnt;
    const int64_t a = W.a;

    // values (clamped loads past the end, never stored) and cleared flags
    int32_t x[CO_PER];
#pragma unroll
    for (int m = 0; m < CO_PER; m++) x[m] = v[a + min(t + m * CO_BLOCK, cnt - 1)];
#pragma unroll
    for (int m = 0; m < CO_PER; m++) {
        kv[t + m * CO_BLOCK] = (uint32_t)x[m] ^ 0x80000000u;
        segid[t + m * CO_BLOCK] = 0;
    }
    if (t == 0) maxlen = 0;
    __syncthreads();
    // segment starts: every column that begins strictly inside the window
    const int64_t cend = W.cl >= 0 ? W.cl : ncols - 1;
    for (int64_t c = W.c0 + 1 + t; c <= cend; c += CO_BLOCK) {
        const int64_t p = colptr[c] - a;
        if (p > 0 && p < cnt) segid[p] = 1;
    }
    __syncthreads();
    // segment of every position: inclusive count of the starts up to it
    // (thread t scans positions CO_PER*t .. CO_PER*t + CO_PER-1)
    uint32_t f[CO_PER], own = 0;
#pragma unroll
    for (int m = 0; m < CO_PER; m++) {
        f[m] = segid[CO_PER * t + m];
        own += f[m];
    }
    uint32_t incl = own;
#pragma unroll
    for (int d = 1; d < CO_WAVE; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d, CO_WAVE);
        if (lane >= d) incl += y;
    }
    if (lane == CO_WAVE - 1) wsum[wv] = incl;
    __syncthreads();
    uint32_t run = incl - own, total = 0;
#pragma unroll
    for (int i = 0; i < CO_BLOCK / CO_WAVE; i++) {
        if (i < wv) run += wsum[i];
        total += wsum[i];
    }
#pragma unroll
    for (int m = 0; m < CO_PER; m++) {
        const int p = CO_PER * t + m;
        run += f[m];
        segid[p] = (uint16_t)run;
        if (f[m]) segstart[run] = (uint16_t)p;
    }
    const int nseg = (int)total + 1;
    if (t == 0) {
        segstart[0] = 0;
        segstart[nseg] = (uint16_t)cnt;
    }
    __syncthreads();
    for (int s = t; s < nseg; s += CO_BLOCK) atomicMax(&maxlen, (uint32_t)(segstart[s + 1] - segstart[s]));
    __syncthreads();

    // the first segment leaves the window on the left if its column began
    // earlier, the last on the right if the next window's first column
    // began in this one
    const bool spans_l = W.cs0 < a;
    const bool spans_r = W.cl >= 0 && colptr[W.cl] < a + cnt;
    auto base_of = [&](int s) -> int64_t { return s == 0 ? W.cs0 : a + segstart[s]; };
    auto spans = [&](int s) -> bool { return (s == 0 && spans_l) || (s == nseg - 1 && spans_r); };

    if (maxlen <= CO_COUNT_MAX) {
        // rank = entries of the segment with a smaller value or an equal
        // value earlier; lanes of a wave mostly share a segment, so LDS
        // broadcasts the compared values
#pragma unroll 1
        for (int m = 0; m < CO_PER; m++) {
            const int p = t + m * CO_BLOCK;
            if (p >= cnt) break;
            const uint32_t xv = kv[p];
            const int s = segid[p], st = segstart[s], en = segstart[s + 1];
            uint32_t r = 0;
            for (int q = st; q < en; q++) {
                const uint32_t u = kv[q];
                r += (uint32_t)(u < xv) | ((uint32_t)(u == xv) & (uint32_t)(q < p));
            }
            z[a + p] = base_of(s) + r;
            if (spans(s)) vs[a + st + r] = xv;
        }
        return;
    }

    // Bitonic sort of the keys (segment, value, position); pads sort last.
    // Every compare-exchange happens in registers: a thread holds 16 keys in
    // one of three layouts, each owning four bits of the position (C: bits
    // 0-3, position 16t + g; S: bits 4-7, 256(t/16) + 16g + t%16; L: bits
    // 8-11, 256g + t), and the keys move between layouts through LDS.  The
    // keys start in layout L, which is how the values were loaded.
    unsigned long long r[CO_PER];
#pragma unroll
    for (int g = 0; g < CO_PER; g++) {
        const int p = t + g * CO_BLOCK;
        const unsigned long long u = (uint32_t)x[g] ^ 0x80000000u;
        r[g] = p < cnt ? ((unsigned long long)segid[p] << 44) | (u << 12) | (unsigned)p : ~0ull;
    }
    int cur = 2;
    for (int lk = 1; lk <= 12; lk++) {  // merge width 2^lk: stages on bits lk-1 .. 0
        const int kk = 1 << lk;
        if (lk - 1 >= 8) {
            co_to<2>(r, cur, t, keys);
            co_stages<2>(r, t, kk, lk - 1);
        }
        if (lk - 1 >= 4) {
            co_to<1>(r, cur, t, keys);
            co_stages<1>(r, t, kk, lk - 1);
        }
        co_to<0>(r, cur, t, keys);
        co_stages<0>(r, t, kk, lk - 1);
    }
    __syncthreads();  // every thread's last layout read is done
#pragma unroll
    for (int g = 0; g < CO_PER; g++) {
        const int y = CO_PER * t + g;  // sorted position
        if (y < cnt) {
            const int s = (int)(r[g] >> 44), idx = (int)(r[g] & 0xFFFu);
            keys[co_phys(idx)] = (unsigned long long)(base_of(s) + (y - segstart[s]));
            if (spans(s)) vs[a + y] = (uint32_t)(r[g] >> 12);
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < CO_PER; m++) {
        const int p = t + m * CO_BLOCK;
        if (p < cnt) z[a + p] = (int64_t)keys[co_phys(p)];
    }
}

// Per window, for the (at most two) columns that leave it: every other
// window u the column meets holds a sorted run of the column's values; its
// entries come first when their value is smaller, or equal and u < w.  The
// run is staged in LDS, then each entry of this window binary-searches it.
__global__ void __launch_bounds__(CO_BLOCK) k_co_merge(const int64_t *colptr, int64_t ncols, const int32_t *v,
                                                      int64_t nnz, const int64_t *first, int64_t nwin, int64_t *z,
                                                      const uint32_t *vs) {
    __shared__ uint32_t run[CO_WIN];
    const int t = threadIdx.x;
    const int64_t w = blockIdx.x;
    const CoWindow W = co_window(colptr, ncols, nnz, first, nwin, w);
    const int64_t a = W.a, b = a + W.cnt;
    // the window's first column, and the column running into the next window
    const int64_t ce0 = clampi(colptr[W.c0 + 1], W.cs0, nnz);
    const bool l = W.cs0 < a || ce0 > b;
    const bool r = W.cl >= 0 && W.cl != W.c0 && colptr[W.cl] < b;
    if (!l && !r) return;
    for (int side = 0; side < 2; side++) {
        if (side == 0 ? !l : !r) continue;  // uniform over the work-group
        const int64_t c = side == 0 ? W.c0 : W.cl;
        const int64_t cs = side == 0 ? W.cs0 : clampi(colptr[c], a, b);
        const int64_t ce = side == 0 ? ce0 : clampi(colptr[c + 1], b, nnz);
        const int64_t ps = max(cs, a), pe = min(ce, b);
        if (pe <= ps) continue;  // only for a colptr that breaks the rules
        uint32_t xv[CO_PER];
        int64_t add[CO_PER];
#pragma unroll
        for (int m = 0; m < CO_PER; m++) {
            const int64_t p = ps + t + m * CO_BLOCK;
            xv[m] = (uint32_t)v[min(p, pe - 1)] ^ 0x80000000u;
            add[m] = 0;
        }
        const int nm = (int)((pe - ps + CO_BLOCK - 1) / CO_BLOCK);  // entries per thread, at most
        const int64_t w0 = cs / CO_WIN, w1 = (ce - 1) / CO_WIN;
        for (int64_t u = w0; u <= w1; u++) {
            if (u == w) continue;
            const int64_t rs = max(cs, u * CO_WIN);
            const int len = (int)(min(ce, (u + 1) * CO_WIN) - rs);
            if (len <= 0) continue;  // only for a colptr that breaks the rules
            __syncthreads();
            for (int i = t; i < len; i += CO_BLOCK) run[i] = vs[rs + i];
            __syncthreads();
            const bool before = u < w;
            // branchless search, steps outermost so that the entries' LDS
            // reads of one step are in flight together: pos = the run's
            // entries that come first (a prefix, since the run is sorted)
            int pos[CO_PER];
#pragma unroll
            for (int m = 0; m < CO_PER; m++) pos[m] = 0;
            for (int step = CO_WIN; step > 0; step >>= 1) {
#pragma unroll
                for (int m = 0; m < CO_PER; m++) {
                    if (m >= nm) break;
                    const int at = pos[m] + step;
                    const uint32_t y = run[min(at, len) - 1];
                    const bool first_ = y < xv[m] || (before && y == xv[m]);
                    pos[m] += (at <= len && first_) ? step : 0;
                }
            }
#pragma unroll
            for (int m = 0; m < CO_PER; m++) add[m] += pos[m];
        }
#pragma unroll
        for (int m = 0; m < CO_PER; m++) {
            const int64_t p = ps + t + m * CO_BLOCK;
            if (p < pe) z[p] += add[m];
        }
        __syncthreads();  // the next side reuses the run buffer
    }
}

// Scratch of one call: the first column of every window (nwin int64), then
// the sorted runs of the windows (nnz uint32) at off_vs.
static size_t co_scratch_off(int64_t nwin) { return ((size_t)nwin * 8 + 255) & ~(size_t)255; }

static int co_launch(const int64_t *colptr, int64_t ncols, const int32_t *v, int64_t nnz, int64_t *z, char *ws,
                     int64_t nwin, hipStream_t s) {
    int64_t *first = (int64_t *)ws;
    uint32_t *vs = (uint32_t *)(ws + co_scratch_off(nwin));
    const int64_t gb = (ncols + CO_BLOCK - 1) / CO_BLOCK;
    hipLaunchKernelGGL(k_co_first, dim3((unsigned)(gb < 8192 ? gb : 8192)), dim3(CO_BLOCK), 0, s, colptr, ncols,
                       nnz, first);
    hipLaunchKernelGGL(k_co_local, dim3((unsigned)nwin), dim3(CO_BLOCK), 0, s, colptr, ncols, v, nnz,
                       (const int64_t *)first, nwin, z, vs);
    hipLaunchKernelGGL(k_co_merge, dim3((unsigned)nwin), dim3(CO_BLOCK), 0, s, colptr, ncols, v, nnz,
                       (const int64_t *)first, nwin, z, (const uint32_t *)vs);
    return hipGetLastError() == hipSuccess ? VR_OK : VR_EHIP;
}

// Checks shared by both entry points; *nwin = the windows of nnz entries.
static int co_check(const int64_t *colptr, int64_t ncols, const int32_t *v, int64_t nnz, const int64_t *z,
                    int64_t *nwin) {
    if (ncols < 0 || nnz < 0 || (ncols > 0 && !colptr)) return VR_EINVAL;
    *nwin = (nnz + CO_WIN - 1) / CO_WIN;
    if (nnz == 0) return VR_OK;
    if (ncols == 0 || !v || !z) return VR_EINVAL;
    if (*nwin > 0x7FFFFFFF) return VR_E2BIG;
    return VR_OK;
}

extern "C" VR_API int vr_column_order(const int64_t *colptr, int64_t ncols, const int32_t *v, int64_t nnz,
                                      int64_t *z, void *stream) {
    int64_t nwin = 0;
    const int st = co_check(colptr, ncols, v, nnz, z, &nwin);
    if (st != VR_OK || nnz == 0) return st;
    const hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)cache_get(co_scratch_off(nwin) + (size_t)nnz * 4, s);
    if (!ws) return VR_ENOMEM;
    const int rc = co_launch(colptr, ncols, v, nnz, z, ws, nwin, s);
    cache_put(ws, s);
    return rc;
}

// ------------------------------------------------- without allocation ----
// The scratch of vr_column_order_noalloc: one array per GPU, loaded with the
// code object and held until the process ends.  In host code its name only
// stands in for the array, so each GPU's device address is looked up once
// (hipGetSymbolAddress, with that GPU current) and used from then on.
static __device__ __align__(256) unsigned char scratch[VR_COLORDER_NOALLOC_BYTES];

namespace {
constexpr int CO_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch[CO_MAX_DEVICES];

// Device address of the current GPU's scratch array; nullptr when the
// lookup fails.
char *scratch_here() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= CO_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch[dev] = (char *)p;
    }
    return g_scratch[dev];
}
}  // namespace

extern "C" VR_API int vr_column_order_noalloc(const int64_t *colptr, int64_t ncols, const int32_t *v, int64_t nnz,
                                              int64_t *z, void *stream) {
    int64_t nwin = 0;
    const int st = co_check(colptr, ncols, v, nnz, z, &nwin);
    if (st != VR_OK || nnz == 0) return st;
    if (co_scratch_off(nwin) + (size_t)nnz * 4 > (size_t)VR_COLORDER_NOALLOC_BYTES) return VR_E2BIG;
    char *ws = scratch_here();
    if (!ws) return VR_EHIP;
    return co_launch(colptr, ncols, v, nnz, z, ws, nwin, (hipStream_t)stream);
}
