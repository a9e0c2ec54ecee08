// k_triangles.hip -- vertex stars, triangle counting, offsets and the
// ordered triangle write.
//
// Ownership: a triangle enters the filtration with its largest edge (Section
// 2.1), so the triangles of value r are exactly {a, b, k} with edge r = {a,b}
// and both {a,k} and {b,k} ranked below r.  In rank-ordered stars, "ranked
// below r" is "before edge r": k lies in the first pb entries of b's star
// (pb = position of edge r in b's star) and in the first xa entries of a's
// star (xa = its position in a's star).  For a fixed edge the sorted vertex
// triples increase with k, and the offsets follow rank order, so the output
// is written in (value, i, j, k) order with no sort.
//
//   k_rows        per vertex: its row of the rank matrix, sorted by rank in
//                 LDS (the paper's per-column ordering, Section 4.3), gives
//                 the rank-ordered star, the position of each of its edges
//                 there, and the star again in neighbour order, each entry
//                 packing (neighbour | position in the rank-ordered star << 16)
//   k_tri_count   per vertex a: for each edge a owns, count the neighbours in
//                 the partner's rank prefix that precede the edge in a's star
//   k_scan        exclusive scan of the counts (decoupled look-back); the
//                 last tile stores (flags, K, T) into the host-pinned mailbox
//   k_tri_write   per vertex a: for each edge a owns, walk the partner's
//                 shortest neighbour-ordered prefix list that holds the
//                 partner's entries before the edge; hits are compacted with ballot and
//                 mbcnt (the ballot/popc compaction of the paper's init_supp,
//                 Section 4.4, on 64-wide waves) and stored contiguously
//   k_tri_write_x the same writes, one wave per (vertex, eighth of its
//                 partners), each die of the chip reading one eighth of the
//                 prefix lists (a schedule the tuner may pick)
//   k_emit_edges  public edge arrays
#include "vr_device.h"

#include <hip/hip_ext.h>

#include <type_traits>

// Cloud of global vertex v, and v's local index.
__device__ __forceinline__ int vertex_cloud(const VrDev &D, long long v) {
    return (D.C == 1) ? 0 : (int)D.vcloud[v];
}

// --------------------------------------------------------------- k_rows ----
// Star slots: vertex v of a cloud with n points owns n entries of star_r
// and star_nbr at star_slot(mbase, n, v).
#define STAR_SENTINEL 0xFFFF0000u  // neighbour 0, position 0xFFFF
__device__ __forceinline__ uint32_t star_slot(uint32_t mbase, int n, int v) { return mbase + (uint32_t)v * (uint32_t)n; }

// Prefix lists: for a star of deg entries, list j (j = 1..VR_PLISTS) holds
// the entries whose position in the rank-ordered star is below
// plist_len(j) = ceil(j deg / VR_PLISTS), in neighbour order, each packing
// (neighbour | position << 16), and is followed by 64 sentinels; the last
// list is the whole star.  An edge's triangles lie among its partner's
// first pb entries, which the partner's list plist_pick(pb) holds: walking
// that list instead of the whole star leaves the walk in neighbour order
// (so hits still come out in k order) while cutting the candidates to about
// half on average (cutting at each eighth instead left the writer's time
// unchanged and slowed the star stage).  Vertex v of a cloud owns
// VR_PLIST_PER n + 65 VR_PLISTS entries of star_k from plist_region (sum
// over the lists: at most (VR_PLISTS + 1) deg / 2 + VR_PLISTS + 64 VR_PLISTS).
__device__ __forceinline__ uint32_t plist_len(uint32_t j, uint32_t deg) { return (j * deg + VR_PLISTS - 1) / VR_PLISTS; }
__device__ __forceinline__ uint32_t plist_off(uint32_t j, uint32_t deg) {
    uint32_t o = 0;
    for (uint32_t i = 1; i < j; i++) o += plist_len(i, deg) + VR_WAVE;
    return o;
}
// smallest j with plist_len(j) >= p; 0 for p = 0 (no candidates)
__device__ __forceinline__ uint32_t plist_pick(uint32_t p, uint32_t deg) {
    return p == 0 ? 0u : (p * VR_PLISTS + deg - 1) / deg;
}
__device__ __forceinline__ uint32_t plist_region(uint32_t mbase, uint32_t vbase, int n, int v) {
    const uint32_t per = VR_PLIST_PER * (uint32_t)n + (VR_WAVE + 1) * VR_PLISTS;
    return VR_PLIST_PER * mbase + (uint32_t)(VR_WAVE + 1) * VR_PLISTS * vbase + (uint32_t)v * per;
}

// One work-group per vertex v reads row v of the rank matrix that k_edges
// scattered into v's star_r slot (entry k = this build's tag << 24 | rank
// of edge {v,k} within the cloud).  Entries of pairs that are not kept are
// left from earlier use of the memory: an entry counts only when it carries
// the tag and names a kept edge of this cloud whose endpoints are {v, k} in
// the sorted edge list, so the matrix is never cleared (the paper avoids
// re-initialising its per-column work array the same way, Section 4.3); the
// tag only spares most stale entries the look-up (the stars written over
// the rows carry tag 0, and tags repeat only every 255 builds).  The kept entries, in neighbour order, are sorted
// by rank in LDS (bitonic), which orders v's edges the way the paper's
// per-column ordering of the distance matrix does (Section 4.3).  Outputs:
// v's star in rank order (rank within the cloud, written over the row, and
// the neighbour), each edge's position in it (pos), the prefix lists (the
// star in neighbour order with those positions, whole and cut at each
// 1/VR_PLISTS of the rank order) and its size.
//
// Wave w reads the row's entries [64 S w, 64 S (w+1)) in S steps of 64, so
// the neighbour order is the order of (wave, step, lane); S * 256 >= n.
#define VR_ROWS_COUNT_MAX 512  // largest star ranked by counting (two keys per thread)

// Counting rank of a star of 1 <= deg <= NK * 256 entries: keys[x] = rank of the
// x-th neighbour (padded to a multiple of 4 with ~0), nbr[x] = that
// neighbour.  Writes the star in rank order over the row, its neighbours,
// the edges' positions, and the neighbour-ordered star (sk, and keys[x]
// once every key is read).
template <int NK>
__device__ __forceinline__ void rows_count_rank(const VrDev &D, uint32_t *keys, const uint16_t *nbr, uint32_t deg,
                                                uint32_t *__restrict__ row, uint32_t s0, uint32_t *__restrict__ sk,
                                                int v, long long kb) {
    uint32_t own[NK], y[NK];
#pragma unroll
    for (int i = 0; i < NK; i++) {
        const uint32_t x = threadIdx.x + VR_BLOCK * i;
        own[i] = keys[min(x, deg - 1)];
        y[i] = 0;
    }
    const uint4 *k4 = (const uint4 *)keys;
    for (uint32_t q = 0; q < (deg + 3) / 4; q++) {
        const uint4 e = k4[q];
#pragma unroll
        for (int i = 0; i < NK; i++)
            y[i] += (uint32_t)(e.x < own[i]) + (uint32_t)(e.y < own[i]) + (uint32_t)(e.z < own[i]) + (uint32_t)(e.w < own[i]);
    }
    uint32_t kx[NK];
#pragma unroll
    for (int i = 0; i < NK; i++) kx[i] = nbr[min(threadIdx.x + VR_BLOCK * i, deg - 1)];
    __syncthreads();  // every key is read: keys[] takes the packed entries
#pragma unroll
    for (int i = 0; i < NK; i++) {
        const uint32_t x = threadIdx.x + VR_BLOCK * i;
        if (x < deg) {
            const uint32_t k = kx[i], lr = own[i];
            row[y[i]] = lr;
            D.star_nbr[s0 + y[i]] = (uint16_t)k;
            D.epos[2 * (kb + lr) + ((uint32_t)v < k ? 0 : 1)] = (uint16_t)y[i];
            sk[x] = k | (y[i] << 16);
            keys[x] = k | (y[i] << 16);
        }
    }
}

template <int S>
__global__ __launch_bounds__(VR_BLOCK) void k_rows(VrDev D) {
    extern __shared__ uint32_t lds[];  // P sort keys, then the position of each neighbour (u16)
    __shared__ uint32_t sh_w[VR_WAVES];
    __shared__ uint32_t sh_l[VR_PLISTS - 1][VR_WAVES];
    const long long vg = blockIdx.x;
    const int c = vertex_cloud(D, vg);
    const int v = (int)(vg - D.cl[c].vbase), n = D.cl[c].n;
    const long long kb = kept_base(D, c), Kc = kept_count(D, c);
    const uint32_t s0 = star_slot((uint32_t)D.cl[c].mbase, n, v);
    uint32_t *__restrict__ row = D.star_r + s0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int per = (n + VR_BLOCK - 1) / VR_BLOCK;  // steps this launch needs (<= S)
    // Loads are issued unconditionally at clamped addresses: a guarded load
    // makes the compiler wait for it before the next one is issued.
    uint32_t rr[S];
#pragma unroll
    for (int s = 0; s < S; s++) rr[s] = row[min((w * per + s) * VR_WAVE + lane, n - 1)];
    // keep an entry when it names a kept edge {v, k} of this cloud; rr = rank within the cloud
    unsigned long long mk[S];  // kept entries of each step (wave-uniform)
    uint32_t cw = 0;
#pragma unroll
    for (int s = 0; s < S; s++) {
        const int k = (w * per + s) * VR_WAVE + lane;
        const uint32_t lr = rr[s] & 0xFFFFFFu;
        const bool in = s < per && k < n && k != v && (rr[s] >> 24) == D.tag && (long long)lr < Kc;
        const uint32_t ij = D.se_ij[kb + (in ? lr : 0u)];  // kept base itself when not in (se_ij has room)
        const uint32_t want = (k < v) ? (((uint32_t)k << 16) | (uint32_t)v) : (((uint32_t)v << 16) | (uint32_t)k);
        const bool kept = in && ij == want;
        rr[s] = lr;
        mk[s] = __builtin_amdgcn_ballot_w64(kept);
        cw += (uint32_t)__popcll(mk[s]);
    }
    if (lane == 0) sh_w[w] = cw;
    __syncthreads();
    uint32_t run = 0, deg = 0;
#pragma unroll
    for (int i = 0; i < VR_WAVES; i++) {
        const uint32_t t = sh_w[i];
        if (i < w) run += t;
        deg += t;
    }
    // sort keys: local ranks in neighbour order (entry x = x-th kept
    // neighbour), padded; small stars are ranked by counting, larger ones
    // sorted (bitonic)
    uint32_t P = VR_WAVE;
    while (P < deg) P <<= 1;
    const bool by_count = deg <= VR_ROWS_COUNT_MAX;
    // counting: the neighbour of entry x; bitonic: the position of neighbour k
    uint16_t *pk = (uint16_t *)(lds + P);
    for (uint32_t y = deg + threadIdx.x; y < P; y += VR_BLOCK) lds[y] = 0xFFFFFFFFu;
    {
        uint32_t x = run;
#pragma unroll
        for (int s = 0; s < S; s++) {
            const uint32_t at = __builtin_amdgcn_mbcnt_hi((uint32_t)(mk[s] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk[s], x));
            if ((mk[s] >> lane) & 1ull) {
                lds[at] = rr[s];
                if (by_count) pk[at] = (uint16_t)((w * per + s) * VR_WAVE + lane);
            }
            x += (uint32_t)__popcll(mk[s]);
        }
    }
    __syncthreads();
    uint32_t *lb = D.star_k + plist_region((uint32_t)D.cl[c].mbase, (uint32_t)D.cl[c].vbase, n, v);
    uint32_t *sk = lb + plist_off(VR_PLISTS, deg);  // the last list: the whole star
    if (by_count) {
        // rank-order position of entry x = number of smaller keys (ranks
        // are distinct); every lane reads the same keys, which LDS
        // broadcasts
        if (deg == 0) {
        } else if (deg <= VR_BLOCK) {
            rows_count_rank<1>(D, lds, pk, deg, row, s0, sk, v, kb);
        } else {
            rows_count_rank<2>(D, lds, pk, deg, row, s0, sk, v, kb);
        }
    } else {
        // Bitonic sort.  Wave w's pairs in a stage with distance j <= 64 lie
        // in its own 128-key blocks, so only stages with j >= 128 exchange
        // keys between waves and need the work-group barrier; the others
        // need the wave's LDS accesses in order, which a wave's LDS
        // instructions are.
        for (uint32_t kk = 2; kk <= P; kk <<= 1) {
            for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
                if (j >= 2 * VR_WAVE) __syncthreads();
                for (uint32_t i = threadIdx.x; i < P / 2; i += VR_BLOCK) {
                    const uint32_t lo = 2 * i - (i & (j - 1)), hi = lo + j;
                    const uint32_t x0 = lds[lo], x1 = lds[hi];
                    if ((x0 > x1) == ((lo & kk) == 0)) {
                        lds[lo] = x1;
                        lds[hi] = x0;
                    }
                }
                if (j >= 2 * VR_WAVE) __syncthreads();
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
        // rank order: entry y is the y-th smallest rank; its neighbour comes
        // from the edge list (lanes past the star repeat the last entry's
        // loads and store nothing)
        uint32_t ij[S];
#pragma unroll
        for (int i = 0; i < S; i++) ij[i] = D.se_ij[kb + lds[min(threadIdx.x + VR_BLOCK * i, deg - 1)]];
#pragma unroll
        for (int i = 0; i < S; i++) {
            const uint32_t y = threadIdx.x + VR_BLOCK * i;
            if (y < deg) {
                const uint32_t lr = lds[y];
                const uint32_t k = ((ij[i] >> 16) == (uint32_t)v) ? (ij[i] & 0xFFFFu) : (ij[i] >> 16);
                row[y] = lr;
                D.star_nbr[s0 + y] = (uint16_t)k;
                D.epos[2 * (kb + lr) + ((uint32_t)v < k ? 0 : 1)] = (uint16_t)y;
                pk[k] = (uint16_t)y;
            }
        }
        __syncthreads();
        uint32_t x = run;
#pragma unroll
        for (int s = 0; s < S; s++) {
            const uint32_t k = (uint32_t)((w * per + s) * VR_WAVE + lane);
            const uint32_t at = __builtin_amdgcn_mbcnt_hi((uint32_t)(mk[s] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk[s], x));
            if ((mk[s] >> lane) & 1ull) {
                const uint32_t e = k | ((uint32_t)pk[k] << 16);
                sk[at] = e;
                lds[at] = e;
            }
            x += (uint32_t)__popcll(mk[s]);
        }
    }
    // lds[0, deg) holds the star in neighbour order (packed); the shorter
    // lists are its entries below each cut, compacted in order
    __syncthreads();
    {
        uint32_t cut[VR_PLISTS - 1], off[VR_PLISTS - 1], run[VR_PLISTS - 1];
#pragma unroll
        for (int j = 0; j < VR_PLISTS - 1; j++) {
            cut[j] = plist_len((uint32_t)j + 1, deg);
            off[j] = plist_off((uint32_t)j + 1, deg);
            run[j] = 0;
        }
        for (uint32_t x0 = 0; x0 < deg; x0 += VR_BLOCK) {
            const uint32_t x = x0 + threadIdx.x;
            const uint32_t e = x < deg ? lds[x] : 0xFFFFFFFFu;
            unsigned long long m[VR_PLISTS - 1];
#pragma unroll
            for (int j = 0; j < VR_PLISTS - 1; j++) {
                m[j] = __builtin_amdgcn_ballot_w64((e >> 16) < cut[j]);
                if (lane == 0) sh_l[j][w] = (uint32_t)__popcll(m[j]);
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < VR_PLISTS - 1; j++) {
                uint32_t before = 0, tot = 0;
#pragma unroll
                for (int i = 0; i < VR_WAVES; i++) {
                    const uint32_t t = sh_l[j][i];
                    if (i < w) before += t;
                    tot += t;
                }
                if ((m[j] >> lane) & 1ull)
                    lb[off[j] + run[j] + __builtin_amdgcn_mbcnt_hi((uint32_t)(m[j] >> 32),
                                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m[j], before))] = e;
                run[j] += tot;
            }
            __syncthreads();  // sh_l is rewritten by the next chunk
        }
    }
    // 64 sentinels after each list: position 0xFFFF fails every prefix test,
    // so a piece may run past a list's end without a bounds test
    if (threadIdx.x < VR_WAVE)
        for (uint32_t j = 1; j <= VR_PLISTS; j++) lb[plist_off(j, deg) + plist_len(j, deg) + threadIdx.x] = STAR_SENTINEL;
    if (threadIdx.x == 0) D.deg[vg] = deg;
}

static uint32_t pow2_at_least(uint32_t x) {
    uint32_t p = VR_WAVE;
    while (p < x) p <<= 1;
    return p;
}

void launch_rows(const VrDev &D, hipStream_t s) {
    const int steps = (D.maxn + VR_BLOCK - 1) / VR_BLOCK;
    // sort keys (P <= pow2(maxn)) and the positions of the neighbours
    const size_t lds = 4 * (size_t)pow2_at_least((uint32_t)D.maxn) + 2 * (size_t)((D.maxn + 1) & ~1);
    const dim3 grid((unsigned)D.V);
    if (steps <= 4) hipLaunchKernelGGL(k_rows<4>, grid, dim3(VR_BLOCK), lds, s, D);
    else if (steps <= 8) hipLaunchKernelGGL(k_rows<8>, grid, dim3(VR_BLOCK), lds, s, D);
    else if (steps <= 16) hipLaunchKernelGGL(k_rows<16>, grid, dim3(VR_BLOCK), lds, s, D);
    else hipLaunchKernelGGL(k_rows<32>, grid, dim3(VR_BLOCK), lds, s, D);
}

// ------------------------------------------------- shared enumeration core ----
// One work-group per vertex a with Pa[k] = position of edge {a,k} in a's
// star (0xFFFF when k is no neighbour) staged in LDS.  The star is taken in
// chunks of EB entries (EB = the work-group size, 256 or 512, a schedule
// choice like the work-groups per vertex); the edges a owns in a chunk are compacted and
// cut into wave-sized pieces of candidates; each wave takes a contiguous run
// of whole edges holding about 1/8 of the pieces.  The metadata of up to 64
// edges sits in lane registers; the loads of the next edge are issued before
// the current edge is consumed.
// An edge's candidates are loaded NP pieces of 64 at a time (NP a schedule
// choice: 2, 4 or 8 for the count, 4 or 8 for the write); longer candidate
// lists finish piece by piece.

template <int EB>
struct EnumLds {
    static constexpr int W = EB / VR_WAVE;
    uint32_t r[EB];
    uint32_t b[EB];
    uint32_t sb[EB];      // start of the partner's star
    uint32_t len[EB];     // candidates of the edge
    uint32_t pb[EB];      // position of the edge in the partner's star
    uint32_t xa[EB];      // position of the edge in a's star
    uint32_t cb[EB + 1];  // first piece of the edge
    uint32_t ew[W + 1];   // first edge of each wave
    uint32_t scan[W];
    uint32_t scan2[W];
};

template <int EB>
__device__ __forceinline__ uint32_t enum_excl_scan(uint32_t x, uint32_t *sh, uint32_t *total) {
    constexpr int ENUM_WAVES = EB / VR_WAVE;
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

// Compact the edges a owns among star entries [p0, p0+EB) and split
// them by piece count: `parts` work-groups share a vertex (part = this one's
// index), each taking a contiguous slice, cut again into one run per wave.
// When `parts` is a multiple of 8, the work-groups of a vertex are split
// by the partner instead: work-group `part` takes only the edges whose
// partner lies in the (part mod 8)-th eighth of the cloud's vertices, and
// the parts / 8 work-groups of that eighth share them as above.  Work-groups
// are handed to the chip's 8 dies (XCDs, each with its own L2) in turn, so
// block index mod 8 names the die, and with parts a multiple of 8 it equals
// part mod 8: each die then reads the stars of one eighth of the vertices,
// which its L2 can hold, instead of all of them.  WRITE: an edge is written at the
// endpoint whose partner's prefix list (the shortest holding the partner's
// entries before the edge) is shorter; candidates = that list, in
// neighbour order.  Otherwise it is counted at the endpoint
// whose partner has the shorter rank prefix (candidates = that prefix).
// The first chunk's star entries come preloaded (r0, b0: see stage_pos).
// Which endpoint writes edge {a, b}: a walks b's shortest prefix list
// holding b's first pb entries, or b walks a's holding a's first xa; the
// shorter walk wins, the smaller vertex on a tie (so exactly one endpoint
// owns the edge).  xa, da: the edge's position in a's star and a's degree;
// pb: its position in b's star.  For a's side: len = the list's length and
// sb = where it starts in star_k.
__device__ __forceinline__ bool write_side(const VrDev &D, uint32_t a, uint32_t b, uint32_t xa, uint32_t da,
                                           uint32_t pb, uint32_t vb, uint32_t mb, int n, uint32_t &len,
                                           uint32_t &sb) {
    const uint32_t db = D.deg[vb + b];
    const uint32_t jb = plist_pick(pb, db), ja = plist_pick(xa, da);
    const uint32_t cb = jb ? plist_len(jb, db) : 0u, ca = ja ? plist_len(ja, da) : 0u;
    len = cb;
    sb = plist_region(mb, vb, n, (int)b) + plist_off(jb ? jb : 1u, db);
    return cb < ca || (cb == ca && a < b);
}

template <bool WRITE, int EB>
__device__ __forceinline__ int load_chunk(const VrDev &D, int a, uint32_t vb, uint32_t mb, int n, uint32_t kb,
                                          uint32_t s0, uint32_t s1, uint32_t p0, EnumLds<EB> &L, int part,
                                          int parts, uint32_t r0, uint32_t b0) {
    constexpr int ENUM_WAVES = EB / VR_WAVE;
    const uint32_t p = p0 + threadIdx.x;
    bool owned = false;
    uint32_t r = 0, b = 0, pb = 0, sb = 0, len = 0;
    const uint32_t x = p - s0;
    const bool by_partner = (parts & 7) == 0;
    const uint32_t eighth = (uint32_t)(part & 7);
    if (by_partner) {
        part >>= 3;
        parts >>= 3;
    }
    if (p < s1) {
        r = kb + (p0 == s0 ? r0 : D.star_r[p]);  // global kept-edge index
        b = p0 == s0 ? b0 : D.star_nbr[p];
        // edge {b,a} in b's star: the count reads it from the per-edge
        // positions (4 bytes per kept edge, written by the star stage) and
        // stores it beside the entry, where the write reads it in order
        if (WRITE) {
            pb = D.ppos[p];
        } else {
            pb = D.epos[2 * r + (b < (uint32_t)a ? 0u : 1u)];
            D.ppos[p] = (uint16_t)pb;
        }
        sb = star_slot(mb, n, (int)b);
        if (WRITE) {
            owned = write_side(D, (uint32_t)a, b, x, s1 - s0, pb, vb, mb, n, len, sb);
        } else {
            owned = pb < x || (pb == x && (uint32_t)a < b);
            len = pb;
        }
        if (by_partner) owned = owned && (b * 8u) / (uint32_t)n == eighth;
    }
    uint32_t m, C;
    const uint32_t idx = enum_excl_scan<EB>(owned ? 1u : 0u, L.scan, &m);
    const uint32_t pieces = owned ? (len + VR_WAVE - 1) / VR_WAVE : 0u;
    const uint32_t cbeg = enum_excl_scan<EB>(pieces, L.scan2, &C);
    if (owned) {
        L.r[idx] = r;
        L.b[idx] = b;
        L.sb[idx] = sb;
        L.len[idx] = len;
        L.pb[idx] = pb;
        L.xa[idx] = x;
        L.cb[idx] = cbeg;
    }
    if (threadIdx.x == 0) L.cb[m] = C;
    __syncthreads();
    if ((int)threadIdx.x <= ENUM_WAVES) {
        // this work-group's slice of the pieces, then one run per wave
        const unsigned long long gw = (unsigned long long)part * ENUM_WAVES + threadIdx.x;
        const uint32_t target = (uint32_t)(((unsigned long long)C * gw) / ((unsigned long long)parts * ENUM_WAVES));
        int lo = 0, hi = (int)m;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (L.cb[mid] < target) lo = mid + 1;
            else hi = mid;
        }
        L.ew[threadIdx.x] = (gw == (unsigned long long)parts * ENUM_WAVES) ? m : (uint32_t)lo;
    }
    __syncthreads();
    return (int)m;
}

__device__ __forceinline__ uint32_t rl(uint32_t v, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// Pa[k] = position of neighbour k in a's rank-ordered star (0xFFFF for
// non-neighbours).  The star's first EB entries (rank and neighbour) are
// loaded before the table is cleared and handed back for the first chunk,
// so neither waits on the other.
template <int EB>
__device__ __forceinline__ void stage_pos(const VrDev &D, int n, uint16_t *Pa, uint32_t s0, uint32_t s1,
                                          uint32_t &r0, uint32_t &b0) {
    r0 = b0 = 0;
    if (s1 > s0) {  // clamped loads: every lane issues them
        const uint32_t pc = min(s0 + (uint32_t)threadIdx.x, s1 - 1);
        r0 = D.star_r[pc];
        b0 = D.star_nbr[pc];
    }
    for (int k = threadIdx.x; k < n; k += EB) Pa[k] = 0xFFFF;
    __syncthreads();
    if (s0 + threadIdx.x < s1) Pa[b0] = (uint16_t)threadIdx.x;
    for (uint32_t p = s0 + threadIdx.x + EB; p < s1; p += EB) Pa[D.star_nbr[p]] = (uint16_t)(p - s0);
    __syncthreads();
}

template <int EB>
size_t enum_lds(int maxn) { return 2 * (size_t)((maxn + 7) & ~7) + sizeof(EnumLds<EB>); }

// Prefetch of one edge's candidates, NP pieces of 64.  Every load is
// issued unconditionally, with addresses clamped into valid memory, so that
// the compiler can count outstanding loads exactly: a conditional load makes
// it wait for every load in flight, the next edge's prefetch included.
// Pieces past the candidates are never consumed.
//
// Rank-prefix candidates (u16 neighbours; len may be 0): pieces past len
// re-read the last candidate, or the array's first entry when len is 0.
template <int NP>
__device__ __forceinline__ void issue_prefix(const uint16_t *__restrict__ base, uint32_t sb, uint32_t len,
                                             uint32_t (&kk)[NP]) {
    const uint32_t lane = threadIdx.x & 63;
    const uint16_t *src = base + (len ? sb : 0u);
    const uint32_t last = len ? len - 1u : 0u;
#pragma unroll
    for (int j = 0; j < NP; j++) {
        const uint32_t y = (uint32_t)(j * VR_WAVE) + lane;
        kk[j] = src[y < last ? y : last];
    }
}

// Padded neighbour-ordered star (len >= 1): pieces past len read the 64
// sentinels that follow the star.
template <int NP>
__device__ __forceinline__ void issue_padded(const uint32_t *__restrict__ src, uint32_t len,
                                             uint32_t (&kk)[NP]) {
    const uint32_t lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < NP; j++) kk[j] = src[min((uint32_t)(j * VR_WAVE), len) + lane];
}

// ----------------------------------------------------------- k_tri_count ----
template <int EB, int NP>
__global__ __launch_bounds__(EB) void k_tri_count(VrDev D, int parts) {
    extern __shared__ uint32_t lds[];
    const long long ag = blockIdx.x / parts;
    const int part = blockIdx.x % parts;
    const int c = vertex_cloud(D, ag);
    const uint32_t vb = (uint32_t)D.cl[c].vbase;
    const int a = (int)(ag - vb), n = D.cl[c].n;
    uint16_t *Pa = (uint16_t *)lds;
    EnumLds<EB> &L = *(EnumLds<EB> *)((char *)lds + 2 * ((D.maxn + 7) & ~7));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t mb = (uint32_t)D.cl[c].mbase, kb = (uint32_t)kept_base(D, c);
    const uint32_t s0 = star_slot(mb, n, a), s1 = s0 + D.deg[ag];
    uint32_t r0, b0;
    stage_pos<EB>(D, n, Pa, s0, s1, r0, b0);
    for (uint32_t p0 = s0; p0 < s1; p0 += EB) {
        load_chunk<false, EB>(D, a, vb, mb, n, kb, s0, s1, p0, L, part, parts, r0, b0);
        const int w_lo = __builtin_amdgcn_readfirstlane((int)L.ew[w]);
        const int w_hi = __builtin_amdgcn_readfirstlane((int)L.ew[w + 1]);
        for (int eb = w_lo; eb < w_hi; eb += VR_WAVE) {
            const int ne = min(VR_WAVE, w_hi - eb);
            uint32_t vr = 0, vsb = 0, vlen = 0, vxa = 0;
            if (lane < ne) {
                vr = L.r[eb + lane];
                vsb = L.sb[eb + lane];
                vlen = L.len[eb + lane];
                vxa = L.xa[eb + lane];
            }
            uint32_t mycnt = 0;
            // count of edge el from its prefetched pieces
            auto count_edge = [&](int el, const uint32_t (&kk)[NP]) {
                const uint32_t xa = rl(vxa, el), len = rl(vlen, el);
                uint32_t c = 0;
#pragma unroll
                for (int j = 0; j < NP; j++) {
                    if ((uint32_t)(j * VR_WAVE) < len) {  // whole pieces past len are skipped
                        const uint32_t y = (uint32_t)(j * VR_WAVE + lane);
                        // lane masks straight from the comparisons (unsigned less-than: 36)
                        c += (uint32_t)__popcll(__builtin_amdgcn_uicmp(y, len, 36) &
                                                __builtin_amdgcn_uicmp((uint32_t)Pa[kk[j]], xa, 36));
                    }
                }
                for (uint32_t y0 = NP * VR_WAVE; y0 < len; y0 += VR_WAVE) {
                    const uint32_t y = y0 + (uint32_t)lane;
                    const uint32_t k = D.star_nbr[rl(vsb, el) + (y < len ? y : len - 1u)];
                    c += (uint32_t)__popcll(__builtin_amdgcn_uicmp(y, len, 36) & __builtin_amdgcn_uicmp((uint32_t)Pa[k], xa, 36));
                }
                if (lane == el) mycnt = c;
            };
            // ping-pong prefetch one edge ahead; past the last edge the loads
            // repeat the last edge's (never consumed)
            uint32_t kA[NP], kB[NP];
            issue_prefix(D.star_nbr, rl(vsb, 0), rl(vlen, 0), kA);
            for (int el = 0; el < ne; el += 2) {
                const int e1 = min(el + 1, ne - 1), e2 = min(el + 2, ne - 1);
                issue_prefix(D.star_nbr, rl(vsb, e1), rl(vlen, e1), kB);
                count_edge(el, kA);
                issue_prefix(D.star_nbr, rl(vsb, e2), rl(vlen, e2), kA);
                if (el + 1 < ne) count_edge(el + 1, kB);
            }
            if (lane < ne) D.cnt[vr] = mycnt;
        }
        __syncthreads();
    }
}

// Work-groups per vertex, the default when no tuned value is known: enough
// groups to spread heavy vertices over many compute units when the cloud is
// small.
int enum_parts(long long V) {
    long long p = 4096 / (V > 0 ? V : 1);
    return p < 1 ? 1 : (p > 8 ? 8 : (int)p);
}

// Work-group size, the default: 256 threads for small clouds (more
// work-groups in flight), 512 for large ones (fewer chunk barriers).
int enum_block(long long V) { return V <= 2048 ? 256 : 512; }

// Pieces loaded at a time, the defaults: 4 for the count (its candidates are
// rank prefixes, often short), 8 for the write (whole stars).
int enum_pieces_count(long long) { return 4; }
int enum_pieces_write(long long) { return 8; }

template <int EB, int NP>
static void count_at(const VrDev &D, dim3 grid, hipStream_t s) {
    hipLaunchKernelGGL((k_tri_count<EB, NP>), grid, dim3(EB), enum_lds<EB>(D.maxn), s, D, D.parts_count);
}

template <int EB>
static void count_eb(const VrDev &D, dim3 grid, hipStream_t s) {
    switch (D.pieces_count) {
    case 2: count_at<EB, 2>(D, grid, s); break;
    case 8: count_at<EB, 8>(D, grid, s); break;
    default: count_at<EB, 4>(D, grid, s); break;
    }
}

void launch_tri_count(const VrDev &D, hipStream_t s) {
    const dim3 grid((unsigned)(D.V * D.parts_count));
    switch (D.eb_count) {
    case 128: count_eb<128>(D, grid, s); break;
    case 256: count_eb<256>(D, grid, s); break;
    default: count_eb<512>(D, grid, s); break;
    }
}

// ---------------------------------------------------------------- k_scan ----
// S == 0: tile = blockIdx.x (every tile's work-group is launched), with the
// tile's counts loaded together with K (clamped to the buffer; counts past
// K are never used); else tiles are claimed S at a time from a ticket.
__global__ __launch_bounds__(VR_BLOCK) void k_scan(VrDev D, int S) {
    __shared__ unsigned long long sh_w[VR_WAVES];
    __shared__ unsigned long long sh_prefix;
    __shared__ int sh_tile;
    VrCtl *ctl = D.ctl;
    const int t = threadIdx.x;
    const bool direct = S == 0;
    const long long cap = (D.K_host >= 0) ? D.K_host : D.E;  // entries of cnt and off
    uint32_t cd[VR_ITEMS];
    {
        const long long i0 = (long long)blockIdx.x * VR_TILE + (long long)t * VR_ITEMS;
#pragma unroll
        for (int m = 0; m < VR_ITEMS; m++) cd[m] = (direct && cap > 0) ? D.cnt[min(i0 + m, cap - 1)] : 0u;
    }
    const long long K = (long long)ctl->n_kept;
    const int ntiles = (int)((K + VR_TILE - 1) / VR_TILE);
    if (D.C == 1 && ntiles == 0 && blockIdx.x == 0 && t == 0)
        publish_counts(D.mailbox, D.seq, ctl->flags, ctl->n_cand, ctl->n_kept, 0ull);
    auto do_tile = [&](int tile, const uint32_t (&cin)[VR_ITEMS]) {
        const long long i0 = (long long)tile * VR_TILE + (long long)t * VR_ITEMS;
        uint32_t c[VR_ITEMS];
        unsigned long long loc = 0;
#pragma unroll
        for (int m = 0; m < VR_ITEMS; m++) {
            c[m] = (i0 + m < K) ? cin[m] : 0u;
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
                if (tile == ntiles - 1) {
                    ctl->n_tri = prefix + tot;
                    if (D.C == 1) publish_counts(D.mailbox, D.seq, ctl->flags, ctl->n_cand, ctl->n_kept, prefix + tot);
                }
            }
        }
        __syncthreads();
        unsigned long long o = sh_prefix + ex;
#pragma unroll
        for (int m = 0; m < VR_ITEMS; m++) {
            if (i0 + m < K) D.off[i0 + m] = o;
            o += c[m];
        }
    };
    if (direct) {
        if ((int)blockIdx.x < ntiles) do_tile((int)blockIdx.x, cd);
        return;
    }
    for (;;) {
        const int t0 = claim_tiles(&ctl->ticket[5], S, &sh_tile);
        if (t0 >= ntiles) break;
        for (int tile = t0; tile < min(t0 + S, ntiles); tile++) {
            if (tile > t0) __syncthreads();  // sh_prefix and sh_w are reused
            const long long i0 = (long long)tile * VR_TILE + (long long)t * VR_ITEMS;
            uint32_t c[VR_ITEMS];
#pragma unroll
            for (int m = 0; m < VR_ITEMS; m++) c[m] = D.cnt[min(i0 + m, cap - 1)];
            do_tile(tile, c);
        }
    }
}

void launch_scan(const VrDev &D, long long Kmax, hipStream_t s) {
    long long g = (Kmax + VR_TILE - 1) / VR_TILE;
    // every tile gets its own work-group when they all fit at once, else
    // 1024 work-groups claim one tile at a time
    const int S = (g <= 1024) ? 0 : 1;
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_scan, dim3((unsigned)g), dim3(VR_BLOCK), 0, s, D, S);
}

// ------------------------------------------------------ k_cloud_publish ----
// Batches: per cloud (kbase, K, first triangle, T) into host-pinned memory,
// then the counts into the mailbox from the last work-group to finish.
__global__ __launch_bounds__(VR_BLOCK) void k_cloud_publish(VrDev D) {
    __shared__ bool sh_last;
    const VrCtl *ctl = D.ctl;
    const int c = blockIdx.x * VR_BLOCK + threadIdx.x;
    if (c < D.C) {
        const long long kb = kept_base(D, c), K = kept_count(D, c);
        unsigned long long tb = 0, T = 0;
        if (D.tri && K > 0) {
            tb = D.off[kb];
            T = D.off[kb + K - 1] + D.cnt[kb + K - 1] - tb;
        } else if (D.tri) {
            tb = (kb < (long long)ctl->n_kept) ? D.off[kb] : ctl->n_tri;
        }
        unsigned long long *h = D.host_cloud + 4 * (size_t)c;
        __hip_atomic_store(&h[0], (unsigned long long)kb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&h[1], (unsigned long long)K, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&h[2], tb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&h[3], T, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    __syncthreads();
    if (threadIdx.x == 0)
        sh_last = atomicAdd(&((VrCtl *)ctl)->done, 1u) == gridDim.x - 1;
    __syncthreads();
    if (sh_last && threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        publish_counts(D.mailbox, D.seq, ctl->flags, ctl->n_cand, ctl->n_kept, D.tri ? ctl->n_tri : 0ull);
    }
}

void launch_cloud_publish(const VrDev &D, hipStream_t s) {
    hipLaunchKernelGGL(k_cloud_publish, dim3((unsigned)((D.C + VR_BLOCK - 1) / VR_BLOCK)), dim3(VR_BLOCK), 0, s, D);
}

// ----------------------------------------------------------- k_tri_write ----
// Edge r = {a, b}: walk b's prefix list; entry (k, position pk in b's
// rank-ordered star) is a triangle of value r when pk < pb and Pa[k] < xa.
// The sorted vertex triple is (k, lo, hi), (lo, k, hi) or (lo, hi, k) as k
// falls below, between or above the endpoints, so a key is a per-edge base
// plus k shifted into place.  Hits of a piece are compacted with ballot and
// mbcnt and stored contiguously, in k order.
__device__ __forceinline__ void emit_edges_range(const VrDev &D, long long K, uint32_t *__restrict__ ij,
                                                 long long *__restrict__ q, long long first, long long stride) {
    for (long long r = first; r < K; r += stride) {
        const uint32_t v = D.se_ij[r];
        __builtin_nontemporal_store(v >> 16, ij + 2 * r);
        __builtin_nontemporal_store(v & 0xFFFFu, ij + 2 * r + 1);
        __builtin_nontemporal_store((long long)D.se_q[r], q + r);
    }
}

// The triangles of up to 64 edges that vertex a (local index) writes, one
// edge's parameters per lane (lanes >= ne unused): global rank vr, start
// vsb and length vlen of the partner's prefix list in star_k, the edge's
// positions vxa in a's star and vpb in the partner's, the partner vb, and
// the edge's first output slot voff.  Pa = a's position table.  Each edge's
// list is walked in neighbour order, so its hits come out in k order.
template <int NP>
__device__ __forceinline__ void write_run(const VrDev &D, unsigned long long *__restrict__ out, uint32_t a,
                                          uint32_t kb, const uint16_t *Pa, int ne, uint32_t vr, uint32_t vsb,
                                          uint32_t vlen, uint32_t vxa, uint32_t vpb, uint32_t vb,
                                          unsigned long long voff) {
    const int lane = threadIdx.x & 63;
    // write the triangles of edge el from its prefetched pieces
    auto write_edge = [&](int el, const uint32_t (&kk)[NP]) {
        const uint32_t xa = rl(vxa, el), pb = rl(vpb, el), len = rl(vlen, el), b = rl(vb, el);
        const uint32_t r = rl(vr, el) - kb;  // local rank within the cloud
        unsigned long long *dst = out + (((unsigned long long)rl((uint32_t)(voff >> 32), el) << 32) |
                                         rl((uint32_t)voff, el));
        uint32_t run = 0;  // keys of this edge written so far
        // key = (r << 39) | (x0 << 26) | (x1 << 13) | x2 with x0 < x1 < x2 the
        // sorted triple {lo, hi, k}; k differs from both endpoints
        const uint32_t lo = min(a, b), hi = max(a, b);
        const uint32_t rh = r << 7;  // bits 39.. of the key, in the high word
        // one 64-entry piece of the partner's neighbour-ordered star, with
        // the position of each entry's neighbour in a's star (lanes past
        // the star read sentinels, which never hit)
        const unsigned long long kbase = (unsigned long long)rh << 32;
        auto piece = [&](uint32_t v, uint32_t pa) {
            const uint32_t k = v & 0xFFFFu, pk = v >> 16;
            // lane masks of the two tests straight from the comparisons
            // (unsigned less-than is predicate 36)
            const unsigned long long m = __builtin_amdgcn_uicmp(pk, pb, 36) & __builtin_amdgcn_uicmp(pa, xa, 36);
            if ((pk < pb) & (pa < xa)) {
                // x1 = k clamped to [lo, hi] is the median; x0 << 26 spans both
                // words, added to the edge's base with the low bits of x1, x2
                const uint32_t x0 = min(lo, k), x2 = max(hi, k), x1 = min(max(k, lo), hi);
                const unsigned long long key = (((unsigned long long)x0 << 26) + kbase) | ((x1 << 13) | x2);
                const uint32_t at = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, run));
                // streaming store: keeps the stars, not the output, in L2
                __builtin_nontemporal_store(key, dst + at);
            }
            run += (uint32_t)__popcll(m);
        };
        // pieces in groups of four: a group past len is skipped whole
        // (pieces past len inside a group read sentinels), and the four
        // position lookups of a group are issued together
#pragma unroll
        for (int g = 0; g < NP; g += 4) {
            if ((uint32_t)(g * VR_WAVE) < len) {
                uint32_t pa[4];
#pragma unroll
                for (int j = 0; j < 4; j++) pa[j] = Pa[kk[g + j] & 0xFFFFu];
#pragma unroll
                for (int j = 0; j < 4; j++) piece(kk[g + j], pa[j]);
            }
        }
        for (uint32_t y0 = NP * VR_WAVE; y0 < len; y0 += VR_WAVE) {
            const uint32_t v = D.star_k[rl(vsb, el) + y0 + (uint32_t)lane];
            piece(v, Pa[v & 0xFFFFu]);
        }
    };
    // ping-pong prefetch one edge ahead; past the last edge the loads
    // repeat the last edge's (never consumed)
    uint32_t kA[NP], kB[NP];
    issue_padded(D.star_k + rl(vsb, 0), rl(vlen, 0), kA);
    for (int el = 0; el < ne; el += 2) {
        const int e1 = min(el + 1, ne - 1), e2 = min(el + 2, ne - 1);
        issue_padded(D.star_k + rl(vsb, e1), rl(vlen, e1), kB);
        write_edge(el, kA);
        issue_padded(D.star_k + rl(vsb, e2), rl(vlen, e2), kA);
        if (el + 1 < ne) write_edge(el + 1, kB);
    }
}

// Blocks [0, n*parts) write triangles; the blocks after them write the
// public edge arrays.
template <int EB, int NP>
__global__ __launch_bounds__(EB) void k_tri_write(VrDev D, unsigned long long *__restrict__ out, int parts,
                                                          long long cap_k, unsigned long long cap_t,
                                                          uint32_t *__restrict__ edge_ij,
                                                          long long *__restrict__ edge_q) {
    extern __shared__ uint32_t lds[];
    // outputs sized before the counts were known: write nothing unless they fit
    const long long K = (long long)D.ctl->n_kept;
    if (K > cap_k || D.ctl->n_tri > cap_t) return;
    const long long nb = D.V * parts;
    if ((long long)blockIdx.x >= nb) {
        emit_edges_range(D, K, edge_ij, edge_q, (long long)(blockIdx.x - nb) * EB + threadIdx.x,
                         (long long)(gridDim.x - nb) * EB);
        return;
    }
    const long long ag = blockIdx.x / parts;
    const int part = blockIdx.x % parts;
    const int c = vertex_cloud(D, ag);
    const uint32_t vb = (uint32_t)D.cl[c].vbase;
    const uint32_t kb = (uint32_t)kept_base(D, c);  // the cloud's ranks start here
    const int a = (int)(ag - vb), n = D.cl[c].n;
    uint16_t *Pa = (uint16_t *)lds;
    EnumLds<EB> &L = *(EnumLds<EB> *)((char *)lds + 2 * ((D.maxn + 7) & ~7));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t mb = (uint32_t)D.cl[c].mbase;
    const uint32_t s0 = star_slot(mb, n, a), s1 = s0 + D.deg[ag];
    uint32_t r0, b0;
    stage_pos<EB>(D, n, Pa, s0, s1, r0, b0);
    for (uint32_t p0 = s0; p0 < s1; p0 += EB) {
        load_chunk<true, EB>(D, a, vb, mb, n, kb, s0, s1, p0, L, part, parts, r0, b0);
        const int w_lo = __builtin_amdgcn_readfirstlane((int)L.ew[w]);
        const int w_hi = __builtin_amdgcn_readfirstlane((int)L.ew[w + 1]);
        for (int eb = w_lo; eb < w_hi; eb += VR_WAVE) {
            const int ne = min(VR_WAVE, w_hi - eb);
            uint32_t vr = 0, vsb = 0, vlen = 0, vxa = 0, vpb = 0, vb = 0;
            unsigned long long voff = 0;
            if (lane < ne) {
                vr = L.r[eb + lane];
                vsb = L.sb[eb + lane];
                vlen = L.len[eb + lane];
                vxa = L.xa[eb + lane];
                vpb = L.pb[eb + lane];
                vb = L.b[eb + lane];
                voff = D.off[vr];
            }
            write_run<NP>(D, out, (uint32_t)a, kb, Pa, ne, vr, vsb, vlen, vxa, vpb, vb, voff);
        }
        __syncthreads();
    }
}

// LDS of one wave of k_tri_write_x: a's position table (maxn entries,
// rounded up to 8) and a ring of 128 staged edges.
#define VR_XRING 128
__host__ __device__ __forceinline__ uint32_t xwave_lds(int maxn) {
    return 2u * (((uint32_t)maxn + 7u) & ~7u) + VR_XRING * (uint32_t)sizeof(uint4);
}

// Orders a wave's LDS stores before its later LDS loads of other lanes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The write with 0 work-groups per vertex: one wave per (vertex a, eighth
// of its cloud's vertices), taking the edges a writes (write_side) whose
// partner lies in that eighth.  Work-group g holds the waves of vertices
// [W (g / 8), W (g / 8) + W) for eighth g mod 8.  Work-groups go to the
// chip's 8 dies (XCDs, each with its own L2) in turn, so block index mod 8
// names the die: each die reads the prefix lists of one eighth of the
// vertices, about an eighth of them all, which its L2 can hold.  Each wave
// runs on its own, with a's position table and a ring of staged edges in
// the wave's own LDS and no work-group barrier: the table is filled from
// a's rank-ordered star while counting a's neighbours below the eighth's
// bounds, which locates a's edges to the eighth as one run of its
// neighbour-ordered star; those a writes are staged in the ring and
// written 64 at a time (write_run).  Blocks past the vertices' write the
// public edge arrays.
template <int EB, int NP>
__global__ __launch_bounds__(EB) void k_tri_write_x(VrDev D, unsigned long long *__restrict__ out, long long cap_k,
                                                    unsigned long long cap_t, uint32_t *__restrict__ edge_ij,
                                                    long long *__restrict__ edge_q) {
    constexpr int W = EB / VR_WAVE;
    extern __shared__ uint32_t lds[];
    const long long K = (long long)D.ctl->n_kept;
    if (K > cap_k || D.ctl->n_tri > cap_t) return;
    const long long nb = (D.V + W - 1) / W * 8;
    if ((long long)blockIdx.x >= nb) {
        emit_edges_range(D, K, edge_ij, edge_q, (long long)(blockIdx.x - nb) * EB + threadIdx.x,
                         (long long)(gridDim.x - nb) * EB);
        return;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t x8 = blockIdx.x & 7u;
    const long long ag = (long long)(blockIdx.x >> 3) * W + w;
    if (ag >= D.V) return;  // the whole wave: nothing below waits on other waves
    const uint32_t deg = D.deg[ag];
    if (deg == 0) return;
    const int c = vertex_cloud(D, ag);
    const uint32_t vb = (uint32_t)D.cl[c].vbase;
    const uint32_t kb = (uint32_t)kept_base(D, c);
    const int n = D.cl[c].n;
    const uint32_t a = (uint32_t)(ag - vb);
    const uint32_t mb = (uint32_t)D.cl[c].mbase;
    const uint32_t pa_n = ((uint32_t)D.maxn + 7u) & ~7u;
    uint16_t *Pa = (uint16_t *)((char *)lds + (size_t)w * xwave_lds(D.maxn));
    uint4 *ring = (uint4 *)(Pa + pa_n);
    const uint32_t s0 = star_slot(mb, n, (int)a), s1 = s0 + deg;
    // partners b with (8 b) / n == x8
    const uint32_t blo = (x8 * (uint32_t)n + 7u) / 8u, bhi = ((x8 + 1u) * (uint32_t)n + 7u) / 8u;
    for (uint32_t i = (uint32_t)lane; i < pa_n / 8u; i += VR_WAVE) ((uint4 *)Pa)[i] = make_uint4(~0u, ~0u, ~0u, ~0u);
    wave_lds_sync();
    // position table; y0, y1 = a's neighbours below blo, below bhi
    uint32_t y0 = 0, y1 = 0;
    for (uint32_t base = s0; base < s1; base += 4 * VR_WAVE) {
        uint32_t k[4];
#pragma unroll
        for (int j = 0; j < 4; j++) k[j] = D.star_nbr[min(base + (uint32_t)(j * VR_WAVE + lane), s1 - 1u)];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint32_t p = base + (uint32_t)(j * VR_WAVE + lane);
            const bool in = p < s1;
            if (in) Pa[k[j]] = (uint16_t)(p - s0);
            y0 += (uint32_t)__popcll(ballot64(in && k[j] < blo));
            y1 += (uint32_t)__popcll(ballot64(in && k[j] < bhi));
        }
    }
    wave_lds_sync();
    // a's neighbour-ordered star (the last prefix list): entries [y0, y1)
    // are its edges to the eighth
    const uint32_t *sk = D.star_k + plist_region(mb, vb, n, (int)a) + plist_off(VR_PLISTS, deg);
    uint32_t head = 0, cnt = 0;  // staged edges: ring slots [head, head + cnt)
    auto flush = [&](int ne) {
        uint32_t vr = 0, vsb = 0, vlen = 0, vxa = 0, vpb = 0, vbp = 0;
        unsigned long long voff = 0;
        if (lane < ne) {
            const uint4 e = ring[(head + (uint32_t)lane) & (VR_XRING - 1)];
            vr = e.x;
            vsb = e.y;
            vbp = e.z & 0xFFFFu;
            vxa = e.z >> 16;
            vpb = e.w & 0xFFFFu;
            vlen = e.w >> 16;
            voff = D.off[vr];
        }
        write_run<NP>(D, out, a, kb, Pa, ne, vr, vsb, vlen, vxa, vpb, vbp, voff);
    };
    for (uint32_t y = y0; y < y1; y += VR_WAVE) {
        const uint32_t yy = y + (uint32_t)lane;
        const bool in = yy < y1;
        const uint32_t e = sk[in ? yy : y1 - 1u];
        const uint32_t b = e & 0xFFFFu, xa = e >> 16;
        const uint32_t r = kb + D.star_r[s0 + xa];
        const uint32_t pb = D.ppos[s0 + xa];
        uint32_t len = 0, sb = 0;
        const bool mine = write_side(D, a, b, xa, deg, pb, vb, mb, n, len, sb);
        const bool own = in && mine && len > 0;  // len 0: the edge has no triangles
        const unsigned long long m = ballot64(own);
        if (own) {
            const uint32_t at = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            ring[(head + cnt + at) & (VR_XRING - 1)] = make_uint4(r, sb, b | (xa << 16), pb | (len << 16));
        }
        cnt += (uint32_t)__popcll(m);
        if (cnt >= VR_WAVE) {  // cnt < 128: the ring never overflows
            wave_lds_sync();
            flush(VR_WAVE);
            head = (head + VR_WAVE) & (VR_XRING - 1);
            cnt -= VR_WAVE;
            wave_lds_sync();
        }
    }
    if (cnt > 0) {
        wave_lds_sync();
        flush((int)cnt);
    }
}

// The outputs hold cap_k edges and cap_t triangles; the kernel writes nothing
// when the build's counts (read on the device) exceed them.  With events,
// they take the dispatch's own start and end times (no separate markers).
void launch_tri_write(const VrDev &D, unsigned long long *tri_out, long long cap_k, unsigned long long cap_t,
                      uint32_t *edge_ij, long long *edge_q, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    const int parts = D.parts_write;
    int EB = D.eb_write;
    // one wave per (vertex, eighth): fewer waves per work-group while their
    // LDS would pass 64 KiB
    if (parts == 0)
        while (EB > 128 && (size_t)(EB / VR_WAVE) * xwave_lds(D.maxn) > 65536) EB /= 2;
    const long long K = cap_k;
    long long eb = (K + EB - 1) / EB;  // extra work-groups that write the edge arrays
    if (eb > 256) eb = 256;
    if (eb < 1) eb = 1;
    const long long W = EB / VR_WAVE;
    const dim3 grid((unsigned)((parts == 0 ? (D.V + W - 1) / W * 8 : D.V * parts) + eb));
    auto go = [&](auto eb_c, auto np_c) {
        constexpr int E = decltype(eb_c)::value, N = decltype(np_c)::value;
        if (parts == 0) {
            const size_t lb = (size_t)(E / VR_WAVE) * xwave_lds(D.maxn);
            if (ev0 && ev1)
                hipExtLaunchKernelGGL((k_tri_write_x<E, N>), grid, dim3(E), lb, s, ev0, ev1, 0u, D, tri_out, cap_k,
                                      cap_t, edge_ij, edge_q);
            else
                hipLaunchKernelGGL((k_tri_write_x<E, N>), grid, dim3(E), lb, s, D, tri_out, cap_k, cap_t, edge_ij,
                                   edge_q);
            return;
        }
        if (ev0 && ev1)
            hipExtLaunchKernelGGL((k_tri_write<E, N>), grid, dim3(E), enum_lds<E>(D.maxn), s, ev0, ev1, 0u, D, tri_out,
                                  parts, cap_k, cap_t, edge_ij, edge_q);
        else
            hipLaunchKernelGGL((k_tri_write<E, N>), grid, dim3(E), enum_lds<E>(D.maxn), s, D, tri_out, parts, cap_k,
                               cap_t, edge_ij, edge_q);
    };
    using I128 = std::integral_constant<int, 128>;
    using I256 = std::integral_constant<int, 256>;
    using I512 = std::integral_constant<int, 512>;
    using P4 = std::integral_constant<int, 4>;
    using P8 = std::integral_constant<int, 8>;
    const bool p4 = D.pieces_write == 4;
    if (EB == 128) p4 ? go(I128{}, P4{}) : go(I128{}, P8{});
    else if (EB == 256) p4 ? go(I256{}, P4{}) : go(I256{}, P8{});
    else p4 ? go(I512{}, P4{}) : go(I512{}, P8{});
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

// ----------------------------------------------------------- k_unpack ----
// Packed triangle keys -> rows (i, j, k, v) of int32, for callers that want
// the filtration's triangles unpacked.
__global__ __launch_bounds__(VR_BLOCK) void k_unpack(const unsigned long long *__restrict__ keys, long long T,
                                                     int4 *__restrict__ rows) {
    for (long long x = (long long)blockIdx.x * VR_BLOCK + threadIdx.x; x < T; x += (long long)gridDim.x * VR_BLOCK) {
        const unsigned long long k = keys[x];
        rows[x] = make_int4((int)((k >> 26) & 0x1FFFu), (int)((k >> 13) & 0x1FFFu), (int)(k & 0x1FFFu),
                            (int)(k >> 39));
    }
}

void launch_unpack(const unsigned long long *keys, long long T, int *rows, hipStream_t s) {
    long long g = (T + VR_BLOCK - 1) / VR_BLOCK;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_unpack, dim3((unsigned)g), dim3(VR_BLOCK), 0, s, keys, T, (int4 *)rows);
}
