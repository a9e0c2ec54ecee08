// vr_device.h -- device-side building blocks shared by the gfx950 kernels:
// wave64 ballots and scans, work-group scans, decoupled look-back status
// words, and the workspace layout the kernels agree on.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define VR_WAVE 64
#define VR_BLOCK 256                 // threads per work-group in every kernel
#define VR_WAVES (VR_BLOCK / VR_WAVE)
#define VR_ITEMS 8                   // items per thread in tiled passes
#define VR_TILE (VR_BLOCK * VR_ITEMS) // 2048 items per tile
#define VR_RADIX_BITS 8
#define VR_RADIX (1 << VR_RADIX_BITS)
#define VR_MAX_PASSES 4
#define VR_NBUCKET 1728              // log-linear buckets of a 32-bit key
#define VR_NOT_KEPT 0xFFFFFFFFu
// Prefix lists of the triangle writer: each star in neighbour order, whole
// and cut at every (1 / VR_PLISTS)-th of its rank order; VR_PLIST_PER n +
// 65 VR_PLISTS entries per vertex hold them with their sentinels.
#define VR_PLISTS 4
#define VR_PLIST_PER ((VR_PLISTS + 2) / 2)

// Look-back status words: 2-bit state in the top bits, value below.
#define VR_ST_NONE 0u
#define VR_ST_AGG 1u
#define VR_ST_INC 2u

// Global histograms that every work-group adds to are kept in VR_HCOPY
// copies, a work-group adding to copy blockIdx % VR_HCOPY, and summed by
// their readers: device-scope atomics on one address serialise across the
// XCDs, and a histogram flushed by thousands of work-groups would wait on
// them.
#define VR_HCOPY 32

// Control block in device memory, zeroed at the start of every build.
struct VrCtl {
    uint32_t ticket[16];            // tile tickets: 1..4 edge sort, 5 scan
    uint32_t done;                  // finished work-groups of the per-cloud publisher
    uint32_t flags;                 // bit 0: a squared distance overflowed 32 bits
    uint32_t n_cand;                // candidates kept by the select pass
    uint32_t n_kept;                // K
    unsigned long long n_tri;       // T
    uint32_t hist8[VR_HCOPY][VR_MAX_PASSES][VR_RADIX];  // digit histograms of the edge candidates
};
#define VR_HIST8_STRIDE (VR_MAX_PASSES * VR_RADIX)

// Host-pinned mailbox: the end of phase 1 publishes the counts here; the
// host polls `seq` instead of synchronising the stream.
struct VrMailbox {
    uint32_t seq;
    uint32_t flags;
    uint32_t n_cand;
    uint32_t n_kept;
    unsigned long long n_tri;
    unsigned long long pad[5];
};

// ---------------------------------------------------------------- lanes ----
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ unsigned long long lanemask_lt() {
    uint32_t l = lane_id();
    return (l == 0) ? 0ull : ((~0ull) >> (64 - l));
}

__device__ __forceinline__ unsigned long long ballot64(int p) { return __ballot(p); }

// Inclusive scan across the 64 lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
#pragma unroll
    for (int o = 1; o < VR_WAVE; o <<= 1) {
        T y = __shfl_up(x, o, VR_WAVE);
        if ((int)lane_id() >= o) x += y;
    }
    return x;
}

// Inclusive scan of a 32-bit value across the 64 lanes with DPP moves (row
// shifts within 16-lane rows, then row broadcasts 15 and 31): VALU only.
__device__ __forceinline__ uint32_t wave_incl_scan_dpp(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);  // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, true);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, true);  // row_bcast:31
    return x;
}

__device__ __forceinline__ uint32_t wave_last(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, VR_WAVE - 1);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int o = VR_WAVE / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, VR_WAVE);
    return x;
}

// Exclusive scan across a 256-thread work-group; returns the exclusive value
// and writes the group total.  `sh` holds VR_WAVES entries of LDS.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T x, T *sh, T *total) {
    T inc = wave_incl_scan(x);
    const int w = threadIdx.x / VR_WAVE;
    if (lane_id() == VR_WAVE - 1) sh[w] = inc;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < VR_WAVES; i++) {
        T s = sh[i];
        if (i < w) off += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + inc - x;
}

// Add 1 to hist[bin] for every lane with `valid`, one LDS add per distinct
// bin: lanes holding the same bin find each other with one ballot per bin
// bit, and the lowest of them adds the group's size.
template <int BITS>
__device__ __forceinline__ void match_add(uint32_t *hist, uint32_t bin, bool valid) {
    unsigned long long peers = ballot64(valid);
#pragma unroll
    for (int b = 0; b < BITS; b++) {
        const unsigned long long m = ballot64((bin >> b) & 1u);
        peers &= ((bin >> b) & 1u) ? m : ~m;
    }
    if (valid && (peers & lanemask_lt()) == 0ull) atomicAdd(&hist[bin], (uint32_t)__popcll(peers));
}

// Add 1 to hist[bin] for every lane with `valid` when bins are spread, so
// that few lanes of a wave share one: a plain LDS atomic per lane.
__device__ __forceinline__ void spread_add(uint32_t *hist, uint32_t bin, bool valid) {
    if (valid) atomicAdd(&hist[bin], 1u);
}

// The same for bins that a few values cover, often one per wave (the top
// digit of a key): one add when every valid lane holds the same bin, else
// match_add.  Called by the whole wave.
template <int BITS>
__device__ __forceinline__ void narrow_add(uint32_t *hist, uint32_t bin, bool valid) {
    const unsigned long long act = ballot64(valid);
    if (act == 0ull) return;
    const int first = __ffsll((long long)act) - 1;
    const uint32_t b0 = (uint32_t)__builtin_amdgcn_readlane((int)bin, first);
    if (ballot64(valid && bin == b0) == act) {
        if ((int)lane_id() == first) atomicAdd(&hist[b0], (uint32_t)__popcll(act));
        return;
    }
    match_add<BITS>(hist, bin, valid);
}

// ---------------------------------------------------- look-back statuses ----
__device__ __forceinline__ uint32_t st_load32(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_store32(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long st_load64(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_store64(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t st_pack32(uint32_t state, uint32_t v) { return (state << 30) | v; }
__device__ __forceinline__ unsigned long long st_pack64(uint32_t state, unsigned long long v) {
    return ((unsigned long long)state << 62) | v;
}

// Decoupled look-back (Merrill and Garland, "Single-pass Parallel Prefix Scan
// with Decoupled Look-back", 2016): sum the predecessors' aggregates back to
// the nearest inclusive prefix.  Every predecessor tile was claimed earlier by
// a running work-group through the ticket counter, so every wait ends.
//
// Status words live in memory shared by all XCDs, so each poll is a round
// trip of a microsecond or more: the rounds are made wide, with many
// independent loads in flight, so that a tile far from the nearest inclusive
// prefix needs few of them.
//
// A poll that finds a predecessor unpublished sleeps before polling again,
// longer each time (nap x 128 cycles, up to about 1 us): thousands of waves
// polling the same few lines back to back would slow every poll down.
__device__ __forceinline__ void backoff(int nap) {
    for (int i = 0; i < nap; i++) __builtin_amdgcn_s_sleep(2);
}

// Per-digit form (one thread per digit): R predecessors per round.
template <int R = 16>
__device__ __forceinline__ uint32_t lookback32(const uint32_t *st, int tile, int stride) {
    uint32_t acc = 0;
    for (int t = tile - 1; t >= 0; t -= R) {
        uint32_t s[R];
#pragma unroll
        for (int j = 0; j < R; j++) s[j] = (t - j >= 0) ? st_load32(st + (size_t)(t - j) * stride) : (VR_ST_INC << 30);
#pragma unroll
        for (int j = 0; j < R; j++) {
            for (int nap = 1; (s[j] >> 30) == VR_ST_NONE; nap = nap < 16 ? 2 * nap : 16) {
                backoff(nap);
                s[j] = st_load32(st + (size_t)(t - j) * stride);
            }
            acc += s[j] & 0x3FFFFFFFu;
            if ((s[j] >> 30) == VR_ST_INC) return acc;
        }
    }
    return acc;
}

// Wave form (all 64 lanes of one wave, same `tile`): 64 R predecessors per
// round, predecessor tile - 1 - (lane + 64 j) in slot j of a lane; returns
// the exclusive prefix in every lane.  T is the status word (u32 with 30
// value bits, or u64 with 62).
template <typename T, int R = 4>
__device__ __forceinline__ T lookback_wave(const T *st, int tile) {
    constexpr int SH = 8 * (int)sizeof(T) - 2;
    constexpr T VMASK = ((T)1 << SH) - 1;
    const int lane = (int)lane_id();
    T acc = 0;
    for (int base = tile - 1; base >= 0; base -= VR_WAVE * R) {
        T s[R];
#pragma unroll
        for (int j = 0; j < R; j++) {
            const int i = base - lane - VR_WAVE * j;
            s[j] = (i >= 0) ? (sizeof(T) == 4 ? (T)st_load32((const uint32_t *)st + i)
                                              : (T)st_load64((const unsigned long long *)st + i))
                            : ((T)VR_ST_INC << SH);
        }
        for (int nap = 1;; nap = nap < 16 ? 2 * nap : 16) {
            // nearest inclusive prefix: the smallest distance d = lane + 64 j
            int dmin = VR_WAVE * R;
#pragma unroll
            for (int j = R - 1; j >= 0; j--) {
                const unsigned long long inc = ballot64((s[j] >> SH) == VR_ST_INC);
                if (inc) dmin = VR_WAVE * j + __ffsll((long long)inc) - 1;
            }
            bool wait = false;
#pragma unroll
            for (int j = 0; j < R; j++) {
                const bool need = VR_WAVE * j + lane <= dmin;
                wait |= ballot64(need && (s[j] >> SH) == VR_ST_NONE) != 0ull;
            }
            if (wait) {
                backoff(nap);
#pragma unroll
                for (int j = 0; j < R; j++) {
                    const int i = base - lane - VR_WAVE * j;
                    if (i >= 0 && (s[j] >> SH) == VR_ST_NONE)
                        s[j] = sizeof(T) == 4 ? (T)st_load32((const uint32_t *)st + i)
                                              : (T)st_load64((const unsigned long long *)st + i);
                }
                continue;
            }
            T v = 0;
#pragma unroll
            for (int j = 0; j < R; j++)
                if (VR_WAVE * j + lane <= dmin) v += s[j] & VMASK;
            acc += wave_sum<T>(v);
            if (dmin < VR_WAVE * R) return acc;
            break;
        }
    }
    return acc;
}

__device__ __forceinline__ uint32_t lookback32_wave(const uint32_t *st, int tile) {
    return lookback_wave<uint32_t>(st, tile);
}

__device__ __forceinline__ unsigned long long lookback64_wave(const unsigned long long *st, int tile) {
    return lookback_wave<unsigned long long>(st, tile);
}

// Claim the next S consecutive tiles of a persistent loop with one atomic;
// broadcast through LDS.  A tile looking back at the last tile of the
// previous claim waits until that claim's work-group reaches it, so kernels
// that publish a tile's aggregate only when they process it claim one tile
// at a time.
__device__ __forceinline__ int claim_tiles(uint32_t *ticket, int S, int *sh) {
    __syncthreads();
    if (threadIdx.x == 0) *sh = (int)atomicAdd(ticket, (uint32_t)S);
    __syncthreads();
    return *sh;
}

// Copy of a global histogram that this work-group adds to, and the sum of
// bin `idx` over all copies (copies `stride` words apart).
__device__ __forceinline__ uint32_t *hist_copy(uint32_t *h0, int stride) {
    return h0 + (size_t)(blockIdx.x % VR_HCOPY) * stride;
}
__device__ __forceinline__ uint32_t hist_sum(const uint32_t *h0, int stride, int copies, int idx) {
    uint32_t v = 0;
    if (copies == VR_HCOPY) {  // all loads in flight at once
        uint32_t x[VR_HCOPY];
#pragma unroll
        for (int c = 0; c < VR_HCOPY; c++) x[c] = h0[(size_t)c * stride + idx];
#pragma unroll
        for (int c = 0; c < VR_HCOPY; c++) v += x[c];
        return v;
    }
    for (int c = 0; c < copies; c++) v += h0[(size_t)c * stride + idx];
    return v;
}



// ------------------------------------------------------ key conventions ----
// Log-linear bucket of a 32-bit key: exact below 128, then 64 buckets per
// power of two.  Monotone non-decreasing in q; 1728 buckets.
__device__ __forceinline__ uint32_t bucket_of(uint32_t q) {
    if (q < 128u) return q;
    uint32_t m = 31u - (uint32_t)__clz(q);
    return 128u + ((m - 7u) << 6) + ((q >> (m - 6u)) & 63u);
}

// Smallest key of bucket b (2^32 for b = VR_NBUCKET): the inverse of
// bucket_of on bucket starts.
__host__ __device__ __forceinline__ unsigned long long bucket_start(uint32_t b) {
    if (b < 128u) return b;
    const uint32_t r = b - 128u, m = 7u + r / 64u, f = r % 64u;
    return (1ull << m) | ((unsigned long long)f << (m - 6u));
}

// Packed triangle key: value (24 bits) | i | j | k (13 bits each), i<j<k.
__device__ __forceinline__ unsigned long long tri_key(uint32_t v, uint32_t a, uint32_t b, uint32_t c) {
    uint32_t lo = min(a, min(b, c)), hi = max(a, max(b, c));
    uint32_t mid = a + b + c - lo - hi;
    return ((unsigned long long)v << 39) | ((unsigned long long)lo << 26) |
           ((unsigned long long)mid << 13) | (unsigned long long)hi;
}

// First pair index of row i in the lexicographic list of pairs (i<j).
__host__ __device__ __forceinline__ long long row_start(long long i, long long n) {
    return i * (2 * n - i - 1) / 2;
}

// Pair index -> (i, j): solve row_start(i) <= e < row_start(i+1) with a
// floating-point guess corrected by exact integer comparisons.
__device__ __forceinline__ void pair_of(long long e, long long n, int *pi, int *pj) {
    double b = 2.0 * (double)n - 1.0;
    double disc = b * b - 8.0 * (double)e;
    long long i = (long long)((b - sqrt(disc > 0 ? disc : 0.0)) * 0.5);
    if (i < 0) i = 0;
    if (i > n - 2) i = n - 2;
    while (i > 0 && row_start(i, n) > e) i--;
    while (i < n - 2 && row_start(i + 1, n) <= e) i++;
    *pi = (int)i;
    *pj = (int)(e - row_start(i, n) + i + 1);
}

// Store the phase-1 results into the host-pinned mailbox (system scope; the
// sequence number last, so the host sees complete counts once it matches).
__device__ __forceinline__ void publish_counts(VrMailbox *mb, uint32_t seq, uint32_t flags, uint32_t n_cand,
                                               uint32_t n_kept, unsigned long long n_tri) {
    __hip_atomic_store(&mb->flags, flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&mb->n_cand, n_cand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&mb->n_kept, n_kept, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&mb->n_tri, n_tri, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&mb->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ------------------------------------------------------- launch wrappers ----
// One stable LSD radix sort (keys with values) over a device-side count.
struct SortJob {
    uint32_t *key[2];
    uint32_t *val[2];
    const uint32_t *hist;     // [passes][VR_RADIX] digit histograms (copy 0 after folding)
    uint32_t *ticket;         // one tile ticket per pass
    uint32_t *st[2];          // look-back statuses, by parity of the active pass
    const uint32_t *count;    // number of items
    long long cap;            // capacity of key[] and val[] (items)
    int passes;
};

// One cloud of a batch (written by the host).  Vertices, pairs and distance
// tiles of all clouds are numbered globally; every output of a cloud uses its
// own local vertex indices and local edge ranks.
struct VrCloud {
    const void *points;   // device, n x d row-major
    int n, d;
    long long vbase;      // first global vertex
    long long pbase;      // first global pair
    long long tbase;      // first distance tile
    long long kbase;      // first global kept edge (unless distance threshold)
    long long K;          // kept edges (unless distance threshold)
    long long thr_num;    // distance threshold (strict)
    long long mbase;      // first entry of the cloud's star slots (n x n per cloud)
};

// Per-cloud results written on the device.
struct VrCloudState {
    unsigned long long qend;  // candidates of a count/fraction threshold: q < qend (end of the pivot bucket)
    uint32_t cand_base;       // first candidate of the cloud in the candidate list
    uint32_t pad;
};

struct VrDev {
    // shape (dtype and d shared by every cloud of a batch)
    int C;                  // clouds
    int dtype, d;
    int maxn;               // largest cloud
    long long V, E;         // vertices, pairs over all clouds
    long long tiles;        // 64x64 distance tiles over all clouds
    int thr_kind;
    long long K_host;       // kept edges over all clouds when known on the host (else -1)
    int qbits;              // bits of a squared distance in the sort key; cloud id above
    int passes;             // radix passes launched for the edge keys
    int need_hist;          // histogram select needed (COUNT / FRACTION)
    int tri;                // triangles wanted
    int parts_count, parts_write;  // work-groups per vertex in the enumeration kernels
    int eb_count, eb_write;        // their work-group sizes (256 or 512)
    int pieces_count, pieces_write;  // candidate pieces of 64 loaded at a time (count 2/4/8, write 4/8)
    // workspace
    VrCtl *ctl;
    VrMailbox *mailbox;     // host-pinned
    uint32_t seq;
    uint32_t tag;           // 1..255: top byte of this build's rank-matrix entries
    const VrCloud *cl;      // C clouds
    VrCloudState *cs;       // C per-cloud results
    uint32_t *hist;         // C x hcopies x VR_NBUCKET log-linear histograms
    int hcopies;            // copies of each cloud's histogram
    unsigned long long *host_cloud;  // host-pinned: per cloud (kbase, K, tri_base, T)
    // cloud maps of a batch (null for one cloud): vertex, distance tile,
    // 2048-pair select tile and 256-edge kept block -> the cloud holding it
    // (a tile or block: the cloud of its first element)
    uint32_t *vcloud, *tcloud, *scloud, *kcloud;
    uint32_t *q;            // E squared distances
    uint32_t *key[2];       // E each, ping-pong (edge sort)
    uint32_t *val[2];       // E each (i<<16 | j, local)
    uint32_t *st_sel;       // ceil(E/TILE) candidates per pair tile, then their offsets
    uint32_t *st_sort[2];   // ceil(E/TILE)*RADIX edge-sort statuses
    uint32_t *se_ij;        // K sorted kept edges (i<<16|j, local)
    uint32_t *se_q;         // K
    // Star slots: vertex v of a cloud with n points owns entries
    // [mbase + v n, mbase + v n + n) of star_r, star_nbr and pos, and
    // P n + 65 VR_PLISTS entries of star_k from P mbase + 65 VR_PLISTS vbase +
    // v (P n + 65 VR_PLISTS), P = VR_PLIST_PER.
    uint32_t *star_r;       // sum n^2: first the rank matrix (tag << 24 | local rank at [v][k]),
                            // then each row's star in rank order (local rank, tag 0)
    uint16_t *star_nbr;     // sum n^2: the other endpoint (local), rank order
    uint32_t *star_k;       // VR_PLIST_PER sum n^2 + 65 VR_PLISTS V: per vertex, its prefix lists (the
                            // star in neighbour order, entries neighbour | rank-order position << 16,
                            // whole and cut at each 1/VR_PLISTS of the rank order), each followed by
                            // 64 sentinels
    uint32_t *deg;          // V: star sizes
    uint16_t *epos;         // 2 Kmax: entry 2r + s = position of kept edge r in the rank-ordered star of its
                            // lower (s = 0) or upper (s = 1) endpoint
                            // in v's rank-ordered star (set for v's neighbours only)
    uint16_t *ppos;         // sum n^2, in the star slots: entry x of v's star = the position of that
                            // edge in the partner's star (written by the count, read by the write)
    uint32_t *cnt;          // K triangles per kept edge
    unsigned long long *off;     // K exclusive offsets
    unsigned long long *st_scan; // ceil(K/TILE)
    long long ntile_E;
};

// Cloud of a global index, by the cloud's first index (upper bound - 1).
template <typename F>
__device__ __forceinline__ int cloud_of(long long x, int C, F first) {
    int lo = 0, hi = C - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first(mid) <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Cloud of element x from a map over blocks of B elements (the cloud of
// each block's first element), walking forward over the rare cloud starts
// inside the block.  first(c) is the first element of cloud c.
template <typename F>
__device__ __forceinline__ int cloud_from_map(const VrDev &D, const uint32_t *map, long long x, int B, F first) {
    if (D.C == 1) return 0;
    int c = (int)map[x / B];
    while (c + 1 < D.C && first(c + 1) <= x) c++;
    return c;
}

// Kept edges of cloud c and its first global kept edge.  With a distance
// threshold every candidate is kept, so both come from the candidate bases.
__device__ __forceinline__ long long kept_base(const VrDev &D, int c) {
    return (D.thr_kind == 3) ? (long long)D.cs[c].cand_base : D.cl[c].kbase;
}
__device__ __forceinline__ long long kept_count(const VrDev &D, int c) {
    if (D.thr_kind != 3) return D.cl[c].K;
    const long long nb = (c + 1 < D.C) ? (long long)D.cs[c + 1].cand_base : (long long)D.ctl->n_cand;
    return nb - (long long)D.cs[c].cand_base;
}

SortJob edge_sort_job(const VrDev &D);

void launch_init(const VrDev &D, size_t zero_words, const VrCloud *one, VrCloud *dst, hipStream_t s);
void launch_pivot(const VrDev &D, hipStream_t s);
void launch_cloud_maps(const VrDev &D, hipStream_t s);
void launch_cloud_publish(const VrDev &D, hipStream_t s);
void launch_dist(const VrDev &D, const void *points, hipStream_t s);
bool gram_applies(const VrDev &D);
void launch_gram(const VrDev &D, const void *points, hipStream_t s);
void launch_select(const VrDev &D, hipStream_t s);
void launch_sort_pass(const SortJob &J, long long max_tiles, int pass, hipStream_t s);
void launch_hist_fold(uint32_t *h0, int stride, int bins, hipStream_t s);
void launch_edges(const VrDev &D, hipStream_t s);
void launch_rows(const VrDev &D, hipStream_t s);
int enum_parts(long long V);
int enum_block(long long V);
int enum_pieces_count(long long V);
int enum_pieces_write(long long V);
void launch_tri_count(const VrDev &D, hipStream_t s);
void launch_scan(const VrDev &D, long long Kmax, hipStream_t s);
void launch_tri_write(const VrDev &D, unsigned long long *tri_out, long long cap_k, unsigned long long cap_t,
                      uint32_t *edge_ij, long long *edge_q, hipStream_t s, hipEvent_t ev0 = nullptr,
                      hipEvent_t ev1 = nullptr);
void launch_emit_edges(const VrDev &D, long long K, uint32_t *edge_ij, long long *edge_q, hipStream_t s);
void launch_unpack(const unsigned long long *keys, long long T, int *rows, hipStream_t s);
