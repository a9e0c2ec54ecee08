// vr_api.hip -- the C ABI (include/vr.h): request validation, workspace
// planning, the two-phase launch sequence and result ownership.
//
// Phase 1 (one stream, no host round trip): distances -> threshold select ->
// edge radix passes -> kept edges -> star radix passes -> stars -> triangle
// counts -> offsets -> publish.  The last kernel stores (flags, K, T) into a
// host-pinned mailbox; the host polls it (no stream synchronisation), sizes
// the outputs, and enqueues phase 2: the ordered triangle write and the
// public edge arrays.  The workspace is released in stream order.
#include <hip/hip_runtime.h>

#include <chrono>
#include <mutex>
#include <new>
#include <string.h>
#include <immintrin.h>

#include "vr.h"
#include "vr_device.h"

namespace {

enum Stage { ST_DIST, ST_SELECT, ST_SORT, ST_EDGES, ST_STAR, ST_COUNT, ST_SCAN, ST_SYNC, ST_WRITE, ST_EMIT, ST_N };
const char *kStageNames[ST_N] = {"dist", "select", "radix_sort", "kept_edges", "star_sort",
                                 "tri_count", "tri_scan", "count_readback", "tri_write", "emit_edges"};

struct Alloc {
    const vr_allocator *a;
    hipStream_t s;
    void *get(size_t bytes) {
        if (bytes == 0) bytes = 256;
        if (a && a->alloc) return a->alloc(bytes, (void *)s, a->ctx);
        void *p = nullptr;
        if (hipMallocAsync(&p, bytes, s) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }
    void put(void *p, size_t bytes) {
        if (!p) return;
        if (a && a->free) a->free(p, bytes, (void *)s, a->ctx);
        else (void)hipFreeAsync(p, s);
    }
};

struct Result : vr_result {
    void *block;
    size_t block_bytes;
    vr_allocator alloc;
    bool has_alloc;
    bool timing;
    hipEvent_t ev[ST_N + 1];
    bool ev_used[ST_N + 1];
};

// Keep freed pool memory cached in the device's default pool, so repeated
// builds do not return to the driver for every allocation.
std::once_flag g_pool_once[64];
void tune_pool(int dev) {
    if (dev < 0 || dev >= 64) return;
    std::call_once(g_pool_once[dev], [dev]() {
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t thr = ~0ull;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
        (void)hipGetLastError();
    });
}

// Host-pinned, device-visible mailbox per host thread for the count read-back.
struct Mailbox {
    VrMailbox *h = nullptr;
    VrMailbox *d = nullptr;
    uint32_t seq = 0;
    ~Mailbox() {
        if (h) (void)hipHostFree(h);
    }
};
thread_local Mailbox g_mb;

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Plan {
    size_t off_ctl, off_stscan, off_stsel, zero_bytes;
    size_t off_q, off_key0, off_key1, off_val0, off_val1, off_st0, off_st1;
    size_t off_seij, off_seq;
    size_t off_ikey0, off_ikey1, off_ival0, off_ival1, off_ist0, off_ist1;
    size_t off_star_r, off_star_nbr, off_star_k, off_start, off_pos, off_cnt, off_off;
    size_t total;
};

Plan plan(long long n, long long E, long long Kmax, bool tri) {
    Plan P{};
    const long long ntE = (E + VR_TILE - 1) / VR_TILE;
    const long long ntK = (Kmax + VR_TILE - 1) / VR_TILE;
    const long long ntI = (2 * Kmax + VR_TILE - 1) / VR_TILE;
    size_t o = 0;
    // zeroed region: control block, select and scan statuses
    P.off_ctl = o; o += sizeof(VrCtl);
    o = (o + 15) & ~(size_t)15;
    P.off_stscan = o; o += 8 * (size_t)(ntK > 0 ? ntK : 1);
    P.off_stsel = o; o += sizeof(uint32_t) * (size_t)(ntE > 0 ? ntE : 1);
    P.zero_bytes = (o + 3) & ~(size_t)3;
    o = align_up(o);
    P.off_q = o; o = align_up(o + 4 * (size_t)E);
    P.off_key0 = o; o = align_up(o + 4 * (size_t)E);
    P.off_key1 = o; o = align_up(o + 4 * (size_t)E);
    P.off_val0 = o; o = align_up(o + 4 * (size_t)E);
    P.off_val1 = o; o = align_up(o + 4 * (size_t)E);
    P.off_st0 = o; o = align_up(o + 4 * (size_t)VR_RADIX * (size_t)(ntE > 0 ? ntE : 1));
    P.off_st1 = o; o = align_up(o + 4 * (size_t)VR_RADIX * (size_t)(ntE > 0 ? ntE : 1));
    P.off_seij = o; o = align_up(o + 4 * (size_t)Kmax);
    P.off_seq = o; o = align_up(o + 4 * (size_t)Kmax);
    if (tri) {
        P.off_ikey0 = o; o = align_up(o + 8 * (size_t)Kmax);
        P.off_ikey1 = o; o = align_up(o + 8 * (size_t)Kmax);
        P.off_ival0 = o; o = align_up(o + 8 * (size_t)Kmax);
        P.off_ival1 = o; o = align_up(o + 8 * (size_t)Kmax);
        P.off_ist0 = o; o = align_up(o + 4 * (size_t)VR_RADIX * (size_t)(ntI > 0 ? ntI : 1));
        P.off_ist1 = o; o = align_up(o + 4 * (size_t)VR_RADIX * (size_t)(ntI > 0 ? ntI : 1));
        P.off_star_r = o; o = align_up(o + 8 * (size_t)Kmax);
        P.off_star_nbr = o; o = align_up(o + 4 * (size_t)Kmax);
        P.off_star_k = o; o = align_up(o + 8 * (size_t)Kmax);
        P.off_start = o; o = align_up(o + 4 * (size_t)(n + 1));
        P.off_pos = o; o = align_up(o + 4 * (size_t)Kmax);
        P.off_cnt = o; o = align_up(o + 4 * (size_t)Kmax);
        P.off_off = o; o = align_up(o + 8 * (size_t)Kmax);
    }
    P.total = o;
    return P;
}

int key_bits(int dtype, long long d) {
    if (dtype == VR_I8) {
        unsigned long long m = 65025ull * (unsigned long long)d;  // 255^2 per coordinate
        int b = 0;
        while (b < 32 && (m >> b)) b++;
        return b;
    }
    return 32;
}

int check_request(const vr_request *req, long long *E_out, long long *K_out) {
    if (!req) return VR_EINVAL;
    if (req->n < 0 || req->d < 1) return VR_EINVAL;
    if (req->dtype != VR_I8 && req->dtype != VR_I16 && req->dtype != VR_I32) return VR_EINVAL;
    if (req->maxdim < 0 || req->maxdim > 2) return VR_EINVAL;
    if (req->n > 0 && !req->points) return VR_EINVAL;
    if (req->n > VR_MAX_POINTS) return VR_E2BIG;
    const long long n = req->n;
    const long long E = n * (n - 1) / 2;
    long long K = -1;
    switch (req->thr_kind) {
    case VR_THR_FULL: K = E; break;
    case VR_THR_COUNT:
        if (req->thr_num < 0 || req->thr_num > E) return VR_EINVAL;
        K = req->thr_num;
        break;
    case VR_THR_FRACTION:
        if (req->thr_den <= 0 || req->thr_num < 0 || req->thr_num > req->thr_den) return VR_EINVAL;
        K = (long long)(((__int128)req->thr_num * E) / req->thr_den);
        break;
    case VR_THR_SQDIST:
        if (req->thr_num < 0) return VR_EINVAL;
        K = -1;
        break;
    default: return VR_EINVAL;
    }
    if (K > VR_MAX_EDGES) return VR_E2BIG;
    *E_out = E;
    *K_out = K;
    return VR_OK;
}

}  // namespace

extern "C" {

int vr_version(void) { return 100; }

const char *vr_status_string(int status) {
    switch (status) {
    case VR_OK: return "ok";
    case VR_EINVAL: return "invalid argument";
    case VR_ENOMEM: return "device allocation failed";
    case VR_E2BIG: return "too many points or edges for the packed keys";
    case VR_EHIP: return "HIP runtime error";
    case VR_ERANGE: return "a squared distance exceeds 32 bits";
    default: return "unknown status";
    }
}

const char *vr_stage_name(int s) { return (s >= 0 && s < ST_N) ? kStageNames[s] : nullptr; }

int64_t vr_workspace_bytes(int64_t n, int64_t d, int32_t dtype, int32_t thr_kind) {
    vr_request r{};
    r.n = n; r.d = d; r.dtype = dtype; r.thr_kind = thr_kind; r.thr_num = 0; r.thr_den = 1; r.maxdim = 2;
    r.points = (const void *)16;
    long long E, K;
    if (check_request(&r, &E, &K) != VR_OK) return -1;
    return (int64_t)plan(n, E, E, true).total;
}

int vr_query_counts(const vr_result *res, int64_t counts[3]) {
    if (!res || !counts) return VR_EINVAL;
    counts[0] = res->n_vertices;
    counts[1] = res->n_edges;
    counts[2] = res->n_triangles;
    return VR_OK;
}

int vr_query_stage_ms(const vr_result *res_, float *ms, int cap) {
    if (!res_ || (!ms && cap > 0)) return VR_EINVAL;
    const Result *res = static_cast<const Result *>(res_);
    if (!res->timing) return 0;
    int last = -1;
    for (int i = ST_N; i >= 0; i--)
        if (res->ev_used[i]) { last = i; break; }
    if (last < 0) return 0;
    if (hipEventSynchronize(res->ev[last]) != hipSuccess) return VR_EHIP;
    int w = 0;
    for (int s = 0; s < ST_N && w < cap; s++, w++) {
        ms[w] = 0.f;
        if (res->ev_used[s] && res->ev_used[s + 1]) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, res->ev[s], res->ev[s + 1]) == hipSuccess) ms[w] = t;
        }
    }
    return w;
}

void vr_free(vr_result *res_, void *stream) {
    if (!res_) return;
    Result *res = static_cast<Result *>(res_);
    Alloc A{res->has_alloc ? &res->alloc : nullptr, (hipStream_t)stream};
    A.put(res->block, res->block_bytes);
    if (res->timing)
        for (int i = 0; i <= ST_N; i++) (void)hipEventDestroy(res->ev[i]);
    delete res;
}

int vr_build(const vr_request *req, void *stream_, vr_result **out) {
    if (!out) return VR_EINVAL;
    long long E = 0, Khost = -1;
    int st = check_request(req, &E, &Khost);
    if (st != VR_OK) return st;
    hipStream_t s = (hipStream_t)stream_;
    const long long n = req->n;
    const bool want_edges = req->maxdim >= 1;
    const bool want_tri = req->maxdim >= 2 && n >= 3;
    const bool count_only = (req->flags & VR_COUNT_ONLY) != 0;
    const bool timing_all = (req->flags & VR_TIMING) != 0;
    const bool timing = timing_all || (req->flags & VR_TIMING_WRITE) != 0;

    Result *res = new (std::nothrow) Result();
    if (!res) return VR_ENOMEM;
    res->n_vertices = n;
    res->has_alloc = req->alloc != nullptr;
    if (res->has_alloc) res->alloc = *req->alloc;
    res->timing = timing;
    Alloc A{req->alloc, s};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { delete res; return VR_EHIP; }
    tune_pool(dev);

    auto fail = [&](int code, void *ws, size_t wsb) {
        if (ws) A.put(ws, wsb);
        if (res->timing)
            for (int i = 0; i <= ST_N; i++)
                if (res->ev[i]) (void)hipEventDestroy(res->ev[i]);
        delete res;
        (void)hipGetLastError();
        return code;
    };
    if (timing) {
        for (int i = 0; i <= ST_N; i++)
            if (hipEventCreate(&res->ev[i]) != hipSuccess) return fail(VR_EHIP, nullptr, 0);
    }
    auto mark = [&](int i) {
        if (timing_all || (timing && (i == ST_WRITE || i == ST_EMIT))) {
            (void)hipEventRecord(res->ev[i], s);
            res->ev_used[i] = true;
        }
    };

    // Nothing to compute on the device: no pairs, or no edges requested/kept.
    if (!want_edges || E == 0 || Khost == 0) {
        res->n_edges = 0;
        res->n_triangles = 0;
        *out = res;
        return VR_OK;
    }

    const long long Kmax = (Khost >= 0) ? Khost : E;
    const Plan P = plan(n, E, Kmax, want_tri);
    if (!g_mb.h) {
        void *h = nullptr;
        if (hipHostMalloc(&h, sizeof(VrMailbox), hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess)
            return fail(VR_ENOMEM, nullptr, 0);
        void *d = nullptr;
        if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
            (void)hipHostFree(h);
            return fail(VR_EHIP, nullptr, 0);
        }
        memset(h, 0, sizeof(VrMailbox));
        g_mb.h = (VrMailbox *)h;
        g_mb.d = (VrMailbox *)d;
    }
    char *ws = (char *)A.get(P.total);
    if (!ws) return fail(VR_ENOMEM, nullptr, 0);

    VrDev D{};
    D.n = (int)n;
    D.d = (int)req->d;
    D.dtype = req->dtype;
    D.E = E;
    D.thr_kind = req->thr_kind;
    D.thr_num = req->thr_num;
    D.K_host = Khost;
    D.passes = (key_bits(req->dtype, req->d) + VR_RADIX_BITS - 1) / VR_RADIX_BITS;
    if (D.passes < 1) D.passes = 1;
    D.need_hist = (req->thr_kind == VR_THR_COUNT || req->thr_kind == VR_THR_FRACTION) ? 1 : 0;
    D.tri = want_tri ? 1 : 0;
    D.mailbox = g_mb.d;
    D.seq = ++g_mb.seq;
    if (D.seq == 0) D.seq = ++g_mb.seq;
    D.ctl = (VrCtl *)(ws + P.off_ctl);
    D.st_scan = (unsigned long long *)(ws + P.off_stscan);
    D.st_sel = (uint32_t *)(ws + P.off_stsel);
    D.q = (uint32_t *)(ws + P.off_q);
    D.key[0] = (uint32_t *)(ws + P.off_key0);
    D.key[1] = (uint32_t *)(ws + P.off_key1);
    D.val[0] = (uint32_t *)(ws + P.off_val0);
    D.val[1] = (uint32_t *)(ws + P.off_val1);
    D.st_sort[0] = (uint32_t *)(ws + P.off_st0);
    D.st_sort[1] = (uint32_t *)(ws + P.off_st1);
    D.se_ij = (uint32_t *)(ws + P.off_seij);
    D.se_q = (uint32_t *)(ws + P.off_seq);
    if (want_tri) {
        D.ikey[0] = (uint32_t *)(ws + P.off_ikey0);
        D.ikey[1] = (uint32_t *)(ws + P.off_ikey1);
        D.ival[0] = (uint32_t *)(ws + P.off_ival0);
        D.ival[1] = (uint32_t *)(ws + P.off_ival1);
        D.ist[0] = (uint32_t *)(ws + P.off_ist0);
        D.ist[1] = (uint32_t *)(ws + P.off_ist1);
        D.star_r = (uint32_t *)(ws + P.off_star_r);
        D.star_nbr = (uint16_t *)(ws + P.off_star_nbr);
        D.star_k = (uint32_t *)(ws + P.off_star_k);
        D.start = (uint32_t *)(ws + P.off_start);
        D.pos = (uint16_t *)(ws + P.off_pos);
        D.cnt = (uint32_t *)(ws + P.off_cnt);
        D.off = (unsigned long long *)(ws + P.off_off);
    }
    D.ntile_E = (E + VR_TILE - 1) / VR_TILE;
    D.ntile_I = (2 * Kmax + VR_TILE - 1) / VR_TILE;

    // ---------------------------------------------------------- phase 1 ----
    mark(ST_DIST);
    launch_init(D, P.zero_bytes / 4, s);
    if (gram_applies(D)) launch_gram(D, req->points, s);
    else launch_dist(D, req->points, s);
    mark(ST_SELECT);
    launch_select(D, s);
    mark(ST_SORT);
    {
        const SortJob J = edge_sort_job(D);
        for (int p = 0; p < D.passes; p++) launch_sort_pass(J, D.ntile_E, p, s);
    }
    mark(ST_EDGES);
    launch_edges(D, s);
    mark(ST_STAR);
    if (want_tri) {
        const SortJob J = star_sort_job(D);
        launch_sort_pass(J, D.ntile_I, 0, s);
        launch_sort_pass(J, D.ntile_I, 1, s);
        launch_star(D, s);
    }
    mark(ST_COUNT);
    if (want_tri) launch_tri_count(D, s);
    mark(ST_SCAN);
    // the scan reads K from the device (unknown on the host for SQDIST)
    if (want_tri) launch_scan(D, Kmax, s);  // its last tile publishes the counts
    mark(ST_SYNC);
    if (hipGetLastError() != hipSuccess) {
        (void)hipStreamSynchronize(s);
        return fail(VR_EHIP, ws, P.total);
    }
    // Poll the mailbox; check the stream now and then so that a failed launch
    // cannot leave the host waiting.
    {
        volatile VrMailbox *mb = g_mb.h;
        unsigned long long spins = 0;
        while (__atomic_load_n(&g_mb.h->seq, __ATOMIC_ACQUIRE) != D.seq) {
            if ((++spins & 4095ull) == 0) {
                hipError_t q = hipStreamQuery(s);
                if (q == hipSuccess) {
                    if (__atomic_load_n(&g_mb.h->seq, __ATOMIC_ACQUIRE) == D.seq) break;
                    return fail(VR_EHIP, ws, P.total);
                }
                if (q != hipErrorNotReady) {
                    (void)hipGetLastError();
                    return fail(VR_EHIP, ws, P.total);
                }
            }
            _mm_pause();
        }
        (void)mb;
    }
    const uint32_t flags = g_mb.h->flags;
    const long long K = (long long)g_mb.h->n_kept;
    unsigned long long T = want_tri ? g_mb.h->n_tri : 0ull;
    if (flags & 1u) return fail(VR_ERANGE, ws, P.total);
    if (K > VR_MAX_EDGES) return fail(VR_E2BIG, ws, P.total);

    // ---------------------------------------------------------- phase 2 ----
    const bool write_tri = want_tri && !count_only && T > 0;
    const size_t eq_bytes = align_up(8 * (size_t)K), eij_bytes = align_up(8 * (size_t)K);
    const size_t tri_bytes = write_tri ? 8 * (size_t)T : 0;
    const size_t ob = eq_bytes + eij_bytes + tri_bytes;
    char *blk = (char *)A.get(ob);
    if (!blk) return fail(VR_ENOMEM, ws, P.total);
    res->block = blk;
    res->block_bytes = ob;
    res->edge_q = (const int64_t *)blk;
    res->edge_ij = (const uint32_t *)(blk + eq_bytes);
    res->tri_key = write_tri ? (const uint64_t *)(blk + eq_bytes + eij_bytes) : nullptr;
    res->n_edges = K;
    res->n_triangles = (int64_t)T;

    mark(ST_WRITE);
    if (write_tri) {
        // the triangle writer also writes the public edge arrays
        launch_tri_write(D, (unsigned long long *)res->tri_key, K, (uint32_t *)res->edge_ij,
                         (long long *)res->edge_q, s);
        mark(ST_EMIT);
    } else {
        mark(ST_EMIT);
        launch_emit_edges(D, K, (uint32_t *)res->edge_ij, (long long *)res->edge_q, s);
    }
    mark(ST_N);
    if (hipGetLastError() != hipSuccess) {
        (void)hipStreamSynchronize(s);
        A.put(blk, ob);
        res->block = nullptr;
        return fail(VR_EHIP, ws, P.total);
    }
    A.put(ws, P.total);
    *out = res;
    return VR_OK;
}

}  // extern "C"
