/*
 * vr_oracle.c -- plain CPU oracle for the Vietoris-Rips filtration front end
 * (simplices of dimension <= 2) and a standard F2 column reduction.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library.  The HIP library
 * never calls it and shares no code with it.
 *
 * Every routine follows a definition of the paper (arXiv:1809.04424) as
 * literally as possible: no blocking, no fusion, no reordering.  All
 * arithmetic is exact integer arithmetic.
 *
 *   Section 2.1 (Homological Persistence): an edge joins two points closer
 *     than the threshold; a solid triangle exists once its three edges exist;
 *     the threshold plays the role of time.
 *   Section 4.5 (Sortperm): the integer rank of every distance is the
 *     position of that distance in the sorted order (a sortperm); ties are
 *     broken by the position of the pair in the list.
 *   Section 2.2.1, Algorithm 1 (column algorithm): reduce the boundary matrix
 *     left to right until the lowest nonzeros are distinct; the pairs
 *     (low(j), j) are the persistence pairs.
 *   Section 2.2.2 (persistent cohomology; clear and compress): the same
 *     column algorithm run on the anti-transpose returns the same pivots;
 *     columns known to be zero may be skipped.
 *   One dimension up (Section 3's bettimax = 2): tetrahedra once their six
 *     edges exist, valued at their largest edge rank, and the pairs of
 *     triangles with tetrahedra by both reductions.
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_I8 1
#define OR_I16 2
#define OR_I32 3

#define OR_THR_FULL 0
#define OR_THR_COUNT 1
#define OR_THR_FRACTION 2
#define OR_THR_SQDIST 3

static int64_t coord(const void *pts, int dtype, int64_t idx) {
    if (dtype == OR_I8) return ((const int8_t *)pts)[idx];
    if (dtype == OR_I16) return ((const int16_t *)pts)[idx];
    return ((const int32_t *)pts)[idx];
}

int64_t or_num_pairs(int64_t n) { return n * (n - 1) / 2; }

/*
 * Squared Euclidean distance of every pair i < j, written in lexicographic
 * (i, j) order: q[0] = (0,1), q[1] = (0,2), ..., q[E-1] = (n-2,n-1).
 * Comparing squared distances orders edges exactly as comparing distances
 * (Section 2.1), and keeps everything in integers.
 * Returns the largest q, or -1 if some q does not fit in 63 bits.
 */
int64_t or_sqdist(const void *pts, int64_t n, int64_t d, int dtype, int64_t *q) {
    int64_t e = 0, qmax = 0;
    int bad = 0;
    for (int64_t i = 0; i < n; i++) {
        for (int64_t j = i + 1; j < n; j++) {
            __int128 s = 0;
            for (int64_t c = 0; c < d; c++) {
                __int128 diff = (__int128)coord(pts, dtype, i * d + c) - coord(pts, dtype, j * d + c);
                s += diff * diff;
            }
            if (s > (__int128)INT64_MAX) { bad = 1; s = INT64_MAX; }
            q[e++] = (int64_t)s;
            if ((int64_t)s > qmax) qmax = (int64_t)s;
        }
    }
    return bad ? -1 : qmax;
}

/* ---- sortperm (Section 4.5): order[r] = index of the r-th smallest key ---- */
static int cmp_key_then_index(const void *a, const void *b, void *ctx) {
    const int64_t *key = (const int64_t *)ctx;
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    if (key[x] < key[y]) return -1;
    if (key[x] > key[y]) return 1;
    return (x < y) ? -1 : (x > y);
}

/* 0-based sortperm of keys[0..m): ascending key, equal keys by index. */
void or_sortperm(const int64_t *keys, int64_t m, int64_t *order) {
    for (int64_t i = 0; i < m; i++) order[i] = i;
    qsort_r(order, (size_t)m, sizeof(int64_t), cmp_key_then_index, (void *)keys);
}

/*
 * Number of kept edges K for a threshold specification.
 *   FULL     -> every edge (the default infinite threshold, Section 5)
 *   COUNT    -> num edges (0 <= num <= E)
 *   FRACTION -> floor(num * E / den) edges
 *   SQDIST   -> edges with q strictly below num ("less than epsilon", 2.1)
 * Returns -1 for an invalid specification.
 */
int64_t or_num_kept(int kind, int64_t num, int64_t den, const int64_t *q, int64_t E) {
    if (kind == OR_THR_FULL) return E;
    if (kind == OR_THR_COUNT) return (num < 0 || num > E) ? -1 : num;
    if (kind == OR_THR_FRACTION) {
        if (den <= 0 || num < 0 || num > den) return -1;
        return (int64_t)(((__int128)num * E) / den);
    }
    if (kind == OR_THR_SQDIST) {
        int64_t k = 0;
        for (int64_t e = 0; e < E; e++) if (q[e] < num) k++;
        return k;
    }
    return -1;
}

/*
 * Dense symmetric rank matrix: R[i*n+j] = rank of edge {i,j} if that rank is
 * below K (the edge is in the complex), else -1.  The diagonal is -1.
 * order[] is the sortperm of the lexicographic pair list.
 */
void or_rank_matrix(int64_t n, const int64_t *order, int64_t K, int64_t *R) {
    for (int64_t x = 0; x < n * n; x++) R[x] = -1;
    int64_t E = n * (n - 1) / 2;
    /* pair index -> (i, j) by walking the lexicographic list once */
    int64_t *pi = (int64_t *)malloc(sizeof(int64_t) * (size_t)(E > 0 ? E : 1));
    int64_t *pj = (int64_t *)malloc(sizeof(int64_t) * (size_t)(E > 0 ? E : 1));
    int64_t e = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = i + 1; j < n; j++) { pi[e] = i; pj[e] = j; e++; }
    for (int64_t r = 0; r < K; r++) {
        int64_t p = order[r];
        R[pi[p] * n + pj[p]] = r;
        R[pj[p] * n + pi[p]] = r;
    }
    free(pi);
    free(pj);
}

/* kept edges in rank order: ei[r] < ej[r] */
void or_kept_edges(int64_t n, const int64_t *order, int64_t K, int64_t *ei, int64_t *ej) {
    int64_t E = n * (n - 1) / 2;
    int64_t *pi = (int64_t *)malloc(sizeof(int64_t) * (size_t)(E > 0 ? E : 1));
    int64_t *pj = (int64_t *)malloc(sizeof(int64_t) * (size_t)(E > 0 ? E : 1));
    int64_t e = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = i + 1; j < n; j++) { pi[e] = i; pj[e] = j; e++; }
    for (int64_t r = 0; r < K; r++) { ei[r] = pi[order[r]]; ej[r] = pj[order[r]]; }
    free(pi);
    free(pj);
}

static int64_t max3(int64_t a, int64_t b, int64_t c) {
    int64_t m = a > b ? a : b;
    return m > c ? m : c;
}

/* Number of solid triangles: all i<j<k whose three edges are in the complex. */
int64_t or_count_triangles(int64_t n, const int64_t *R) {
    int64_t t = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = i + 1; j < n; j++) {
            if (R[i * n + j] < 0) continue;
            for (int64_t k = j + 1; k < n; k++)
                if (R[i * n + k] >= 0 && R[j * n + k] >= 0) t++;
        }
    return t;
}

typedef struct { int64_t v, i, j, k; } tri_t;

static int cmp_tri(const void *a, const void *b) {
    const tri_t *x = (const tri_t *)a, *y = (const tri_t *)b;
    if (x->v != y->v) return x->v < y->v ? -1 : 1;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    if (x->j != y->j) return x->j < y->j ? -1 : 1;
    if (x->k != y->k) return x->k < y->k ? -1 : 1;
    return 0;
}

/*
 * All solid triangles, each valued at its largest edge rank (the time it
 * enters the filtration), sorted by (value, i, j, k).  Writes up to cap rows
 * of (v, i, j, k) into out[4*t ...]; returns the total number of triangles.
 */
int64_t or_triangles(int64_t n, const int64_t *R, int64_t cap, int64_t *out) {
    int64_t t = 0;
    tri_t *buf = (tri_t *)out; /* rows of 4 int64 have the layout of tri_t */
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = i + 1; j < n; j++) {
            int64_t a = R[i * n + j];
            if (a < 0) continue;
            for (int64_t k = j + 1; k < n; k++) {
                int64_t b = R[i * n + k], c = R[j * n + k];
                if (b < 0 || c < 0) continue;
                if (t < cap) { buf[t].v = max3(a, b, c); buf[t].i = i; buf[t].j = j; buf[t].k = k; }
                t++;
            }
        }
    if (t <= cap) qsort(buf, (size_t)t, sizeof(tri_t), cmp_tri);
    return t;
}

/*
 * For every kept edge r = (ei[r], ej[r]): the number of triangles whose
 * value (largest edge rank) is r, i.e. whose two other edges rank below r.
 */
void or_triangles_per_value(int64_t n, const int64_t *R, int64_t K, const int64_t *ei,
                            const int64_t *ej, int64_t *count) {
    for (int64_t r = 0; r < K; r++) {
        int64_t a = ei[r], b = ej[r], c = 0;
        for (int64_t k = 0; k < n; k++) {
            if (k == a || k == b) continue;
            int64_t x = R[a * n + k], y = R[b * n + k];
            if (x >= 0 && y >= 0 && x < r && y < r) c++;
        }
        count[r] = c;
    }
}

/* The triangles of value r (edge r = {a,b}), as sorted triples in (i,j,k)
 * order; returns how many. */
int64_t or_triangles_of_value(int64_t n, const int64_t *R, int64_t a, int64_t b, int64_t r,
                              int64_t cap, int64_t *out) {
    int64_t t = 0;
    tri_t *buf = (tri_t *)out;
    for (int64_t k = 0; k < n; k++) {
        if (k == a || k == b) continue;
        int64_t x = R[a * n + k], y = R[b * n + k];
        if (x < 0 || y < 0 || x >= r || y >= r) continue;
        int64_t s0 = a, s1 = b, s2 = k, tmp;
        if (s0 > s1) { tmp = s0; s0 = s1; s1 = tmp; }
        if (s1 > s2) { tmp = s1; s1 = s2; s2 = tmp; }
        if (s0 > s1) { tmp = s0; s0 = s1; s1 = tmp; }
        if (t < cap) { buf[t].v = r; buf[t].i = s0; buf[t].j = s1; buf[t].k = s2; }
        t++;
    }
    if (t <= cap) qsort(buf, (size_t)t, sizeof(tri_t), cmp_tri);
    return t;
}

static void sort3(int64_t *a, int64_t *b, int64_t *c) {
    int64_t t;
    if (*a > *b) { t = *a; *a = *b; *b = t; }
    if (*b > *c) { t = *b; *b = *c; *c = t; }
    if (*a > *b) { t = *a; *a = *b; *b = t; }
}

/* ================= the same steps on several host threads ================= */
/*
 * Threads here only split independent units of work whose results have a
 * fixed place in the output (a row of pairs, the triangles of one value), so
 * every output is byte-identical to the single-threaded routine above.  Work
 * is handed out in blocks from a shared counter, so threads that draw cheap
 * blocks take more of them.
 */
typedef struct {
    int64_t next;          /* next unclaimed unit */
    pthread_mutex_t lock;
} or_queue_t;

static int64_t queue_take(or_queue_t *qu, int64_t block, int64_t end, int64_t *stop) {
    pthread_mutex_lock(&qu->lock);
    int64_t a = qu->next;
    qu->next = a + block < end ? a + block : end;
    *stop = qu->next;
    pthread_mutex_unlock(&qu->lock);
    return a;
}

static void run_threads(int nthreads, void *(*fn)(void *), void *arg) {
    if (nthreads < 1) nthreads = 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int t = 1; t < nthreads; t++) pthread_create(&th[t], NULL, fn, arg);
    fn(arg);
    for (int t = 1; t < nthreads; t++) pthread_join(th[t], NULL);
    free(th);
}

/* Squared distances of all pairs, as or_sqdist, rows i split over threads:
 * the pairs (i, j > i) of row i start at i n - i (i + 1) / 2. */
typedef struct {
    or_queue_t qu;
    const void *pts;
    int64_t n, d;
    int dtype;
    int64_t *q;
    int bad;
} sqdist_job_t;

static void *sqdist_worker(void *arg) {
    sqdist_job_t *J = (sqdist_job_t *)arg;
    int bad = 0;
    for (;;) {
        int64_t stop, i0 = queue_take(&J->qu, 8, J->n, &stop);
        if (i0 >= J->n) break;
        for (int64_t i = i0; i < stop; i++) {
            int64_t e = i * J->n - i * (i + 1) / 2;
            for (int64_t j = i + 1; j < J->n; j++) {
                __int128 s = 0;
                for (int64_t c = 0; c < J->d; c++) {
                    __int128 diff = (__int128)coord(J->pts, J->dtype, i * J->d + c) -
                                    coord(J->pts, J->dtype, j * J->d + c);
                    s += diff * diff;
                }
                if (s > (__int128)INT64_MAX) { bad = 1; s = INT64_MAX; }
                J->q[e++] = (int64_t)s;
            }
        }
    }
    if (bad) {
        pthread_mutex_lock(&J->qu.lock);
        J->bad = 1;
        pthread_mutex_unlock(&J->qu.lock);
    }
    return NULL;
}

/* Returns 0, or -1 if some q does not fit in 63 bits (as or_sqdist). */
int or_sqdist_mt(const void *pts, int64_t n, int64_t d, int dtype, int64_t *q, int nthreads) {
    sqdist_job_t J = {{0, PTHREAD_MUTEX_INITIALIZER}, pts, n, d, dtype, q, 0};
    run_threads(nthreads, sqdist_worker, &J);
    return J.bad ? -1 : 0;
}

/*
 * Triangles by value (Section 2.1: a triangle enters with its largest edge).
 * The triangles of value r are the {a, b, k} with edge r = {a, b} and both
 * {a, k} and {b, k} kept with ranks below r.  For the values r0 <= r < r1:
 * count[r - r0] = how many (pass 1), then, at the offsets the caller derives
 * from those counts, the rows (r, i, j, k), i < j < k, of each value sorted
 * by (i, j, k) with qsort (pass 2).  Concatenated over the values in order,
 * this is the whole triangle list sorted by (value, i, j, k).
 */
typedef struct {
    or_queue_t qu;
    int64_t n;
    const int64_t *R, *ei, *ej;
    int64_t r0, r1;
    int64_t *count;        /* pass 1 output, or pass 2 input (offsets) */
    const int64_t *offset; /* NULL in pass 1 */
    int64_t *out;
} byvalue_job_t;

static void *byvalue_worker(void *arg) {
    byvalue_job_t *J = (byvalue_job_t *)arg;
    const int64_t n = J->n, *R = J->R;
    for (;;) {
        int64_t stop, v0 = queue_take(&J->qu, 256, J->r1, &stop);
        if (v0 >= J->r1) break;
        for (int64_t r = v0; r < stop; r++) {
            const int64_t a = J->ei[r], b = J->ej[r];
            const int64_t *Ra = R + a * n, *Rb = R + b * n;
            if (!J->offset) {
                int64_t c = 0;
                for (int64_t k = 0; k < n; k++)
                    if (k != a && k != b && Ra[k] >= 0 && Ra[k] < r && Rb[k] >= 0 && Rb[k] < r) c++;
                J->count[r - J->r0] = c;
                continue;
            }
            tri_t *dst = (tri_t *)J->out + J->offset[r - J->r0];
            int64_t m = 0;
            for (int64_t k = 0; k < n; k++) {
                if (k == a || k == b || Ra[k] < 0 || Ra[k] >= r || Rb[k] < 0 || Rb[k] >= r) continue;
                int64_t s0 = a, s1 = b, s2 = k;
                sort3(&s0, &s1, &s2);
                dst[m].v = r; dst[m].i = s0; dst[m].j = s1; dst[m].k = s2;
                m++;
            }
            qsort(dst, (size_t)m, sizeof(tri_t), cmp_tri);
        }
    }
    return NULL;
}

/* Pass 1: count[r - r0] for r0 <= r < r1.  Returns their sum. */
int64_t or_triangles_by_value_count(int64_t n, const int64_t *R, const int64_t *ei, const int64_t *ej, int64_t r0,
                                    int64_t r1, int64_t *count, int nthreads) {
    byvalue_job_t J = {{r0, PTHREAD_MUTEX_INITIALIZER}, n, R, ei, ej, r0, r1, count, NULL, NULL};
    run_threads(nthreads, byvalue_worker, &J);
    int64_t t = 0;
    for (int64_t r = r0; r < r1; r++) t += count[r - r0];
    return t;
}

/* Pass 2: rows (v, i, j, k) into out, value r's at out row offset[r - r0]
 * (offset = exclusive prefix sums of pass 1's counts). */
void or_triangles_by_value_write(int64_t n, const int64_t *R, const int64_t *ei, const int64_t *ej, int64_t r0,
                                 int64_t r1, const int64_t *offset, int64_t *out, int nthreads) {
    byvalue_job_t J = {{r0, PTHREAD_MUTEX_INITIALIZER}, n, R, ei, ej, r0, r1, NULL, offset, out};
    run_threads(nthreads, byvalue_worker, &J);
}

/* ======================= F2 column reduction ======================= */

/* A sparse F2 column: strictly increasing row indices. */
typedef struct { int64_t *x; int64_t len, cap; } col_t;

static void col_set(col_t *c, const int64_t *x, int64_t len) {
    if (c->cap < len) {
        c->cap = len + 4;
        c->x = (int64_t *)realloc(c->x, sizeof(int64_t) * (size_t)c->cap);
    }
    if (len) memcpy(c->x, x, sizeof(int64_t) * (size_t)len);
    c->len = len;
}

/* c <- c + d over F2 (symmetric difference of sorted lists); tmp is scratch */
static void col_add(col_t *c, const col_t *d, col_t *tmp) {
    int64_t need = c->len + d->len;
    if (tmp->cap < need) {
        tmp->cap = need + 4;
        tmp->x = (int64_t *)realloc(tmp->x, sizeof(int64_t) * (size_t)tmp->cap);
    }
    int64_t a = 0, b = 0, o = 0;
    while (a < c->len && b < d->len) {
        if (c->x[a] < d->x[b]) tmp->x[o++] = c->x[a++];
        else if (c->x[a] > d->x[b]) tmp->x[o++] = d->x[b++];
        else { a++; b++; }
    }
    while (a < c->len) tmp->x[o++] = c->x[a++];
    while (b < d->len) tmp->x[o++] = d->x[b++];
    tmp->len = o;
    col_t s = *c; *c = *tmp; *tmp = s;
}

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/*
 * Algorithm 1 over F2 (c = 1) on one block of the boundary matrix.  Column j
 * has rows colrows[colptr[j] .. colptr[j+1]) (any order).  For every column
 * that does not reduce to zero, pivot_row[j] = low(j); otherwise -1.
 * The lowest nonzero of the working column is compared against the lows of
 * the reduced earlier columns and cleared until it is new.
 * skip[j] != 0 marks a column known to reduce to zero (clearing).
 */
static void reduce_block(int64_t ncols, const int64_t *colptr, const int64_t *colrows,
                         int64_t nrows, const unsigned char *skip, int64_t *pivot_row) {
    int64_t *col_of_low = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nrows > 0 ? nrows : 1));
    for (int64_t r = 0; r < nrows; r++) col_of_low[r] = -1;
    col_t *red = (col_t *)calloc((size_t)(ncols > 0 ? ncols : 1), sizeof(col_t));
    col_t w = {0, 0, 0}, tmp = {0, 0, 0};
    for (int64_t j = 0; j < ncols; j++) {
        pivot_row[j] = -1;
        if (skip && skip[j]) continue;
        int64_t len = colptr[j + 1] - colptr[j];
        col_set(&w, colrows + colptr[j], len);
        qsort(w.x, (size_t)w.len, sizeof(int64_t), cmp_i64);
        while (w.len > 0) {
            int64_t low = w.x[w.len - 1];
            int64_t p = col_of_low[low];
            if (p < 0) break;
            col_add(&w, &red[p], &tmp);
        }
        if (w.len > 0) {
            pivot_row[j] = w.x[w.len - 1];
            col_of_low[w.x[w.len - 1]] = j;
            col_set(&red[j], w.x, w.len);
        }
    }
    for (int64_t j = 0; j < ncols; j++) free(red[j].x);
    free(red);
    free(w.x);
    free(tmp.x);
    free(col_of_low);
}

/* index of a triangle (v,i,j,k) in the sorted triangle list, or -1 */
static int64_t tri_index(const tri_t *tris, int64_t T, int64_t v, int64_t i, int64_t j, int64_t k) {
    tri_t key = {v, i, j, k};
    int64_t lo = 0, hi = T;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int c = cmp_tri(&tris[mid], &key);
        if (c == 0) return mid;
        if (c < 0) lo = mid + 1; else hi = mid;
    }
    return -1;
}

/*
 * Persistence pairs of the filtration by Algorithm 1 on the boundary matrix
 * (homology).  Simplices are ordered by (value, dimension, lexicographic):
 * vertices (value -1) by index, edges by rank, triangles as listed (sorted).
 * Because the boundary maps dimension k to k-1 only, and column additions
 * only combine columns of one dimension, reducing the edge block and the
 * triangle block separately gives exactly the pivots of the whole matrix.
 *
 * Outputs: e_low[r]  = vertex paired with edge r (its low), or -1;
 *          t_low[t]  = edge rank paired with triangle t (its low), or -1.
 * clear != 0 skips edge columns that are lows of triangle columns (they
 * reduce to zero; clear and compress, Section 2.2.2).
 */
void or_reduce_homology(int64_t n, int64_t K, const int64_t *ei, const int64_t *ej, int64_t T,
                        const int64_t *tris4, int clear, int64_t *e_low, int64_t *t_low) {
    const tri_t *tris = (const tri_t *)tris4;
    /* triangle block: rows are edge ranks */
    int64_t *R = NULL;
    int64_t *cp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(T + 1));
    int64_t *cr = (int64_t *)calloc((size_t)(3 * T + 1), sizeof(int64_t));
    R = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n * n > 0 ? n * n : 1));
    for (int64_t x = 0; x < n * n; x++) R[x] = -1;
    for (int64_t r = 0; r < K; r++) { R[ei[r] * n + ej[r]] = r; R[ej[r] * n + ei[r]] = r; }
    for (int64_t t = 0; t < T; t++) {
        cp[t] = 3 * t;
        cr[3 * t + 0] = R[tris[t].i * n + tris[t].j];
        cr[3 * t + 1] = R[tris[t].i * n + tris[t].k];
        cr[3 * t + 2] = R[tris[t].j * n + tris[t].k];
    }
    cp[T] = 3 * T;
    reduce_block(T, cp, cr, K, NULL, t_low);
    unsigned char *skip = (unsigned char *)calloc((size_t)(K > 0 ? K : 1), 1);
    if (clear)
        for (int64_t t = 0; t < T; t++) if (t_low[t] >= 0) skip[t_low[t]] = 1;
    /* edge block: rows are vertices */
    int64_t *ep = (int64_t *)malloc(sizeof(int64_t) * (size_t)(K + 1));
    int64_t *er = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * K + 1));
    for (int64_t r = 0; r < K; r++) { ep[r] = 2 * r; er[2 * r] = ei[r]; er[2 * r + 1] = ej[r]; }
    ep[K] = 2 * K;
    reduce_block(K, ep, er, n, skip, e_low);
    free(skip); free(ep); free(er); free(cp); free(cr); free(R);
}

/*
 * Persistence pairs by the same column algorithm applied to the
 * anti-transpose of the boundary matrix (persistent cohomology), dimension by
 * dimension from the bottom, with clearing: an edge that is the partner of a
 * vertex has a zero coboundary column after reduction and is skipped.
 * In anti-transposed coordinates the columns are the simplices from last to
 * first and the rows their cofaces from last to first, so the lowest nonzero
 * of a column is its earliest coface.
 *
 * Outputs use the same convention as or_reduce_homology:
 *   e_low[r] = vertex paired with edge r, or -1;  t_low[t] = edge paired with
 *   triangle t, or -1.
 */
void or_reduce_cohomology(int64_t n, int64_t K, const int64_t *ei, const int64_t *ej, int64_t T,
                          const int64_t *tris4, int64_t *e_low, int64_t *t_low) {
    const tri_t *tris = (const tri_t *)tris4;
    for (int64_t r = 0; r < K; r++) e_low[r] = -1;
    for (int64_t t = 0; t < T; t++) t_low[t] = -1;

    /* dimension 0: columns = vertices n-1..0, rows = edges in reversed order
       (anti-transposed row index of edge r is K-1-r). */
    {
        int64_t *deg = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
        for (int64_t r = 0; r < K; r++) { deg[ei[r]]++; deg[ej[r]]++; }
        int64_t *cp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
        int64_t *cr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * K + 1));
        int64_t *fill = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
        cp[0] = 0;
        for (int64_t c = 0; c < n; c++) cp[c + 1] = cp[c] + deg[n - 1 - c];
        for (int64_t r = 0; r < K; r++) {
            int64_t ca = n - 1 - ei[r], cb = n - 1 - ej[r];
            cr[cp[ca] + fill[ca]++] = K - 1 - r;
            cr[cp[cb] + fill[cb]++] = K - 1 - r;
        }
        int64_t *piv = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        reduce_block(n, cp, cr, K, NULL, piv);
        for (int64_t c = 0; c < n; c++)
            if (piv[c] >= 0) e_low[K - 1 - piv[c]] = n - 1 - c;
        free(piv); free(fill); free(cp); free(cr); free(deg);
    }

    /* dimension 1: columns = edges K-1..0 (cleared when already paired with a
       vertex), rows = triangles in reversed order (row of triangle t is T-1-t).
       A filtration without triangles (built up to dimension 1) has empty
       coboundaries here: nothing to reduce. */
    if (T > 0) {
        int64_t *R = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n * n > 0 ? n * n : 1));
        for (int64_t x = 0; x < n * n; x++) R[x] = -1;
        for (int64_t r = 0; r < K; r++) { R[ei[r] * n + ej[r]] = r; R[ej[r] * n + ei[r]] = r; }
        /* cofaces of each edge */
        int64_t *cnt = (int64_t *)calloc((size_t)(K > 0 ? K : 1), sizeof(int64_t));
        for (int64_t r = 0; r < K; r++) {
            int64_t a = ei[r], b = ej[r];
            for (int64_t k = 0; k < n; k++)
                if (k != a && k != b && R[a * n + k] >= 0 && R[b * n + k] >= 0) cnt[r]++;
        }
        int64_t *cp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(K + 1));
        cp[0] = 0;
        for (int64_t c = 0; c < K; c++) cp[c + 1] = cp[c] + cnt[K - 1 - c];
        int64_t *cr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cp[K] + 1));
        unsigned char *skip = (unsigned char *)calloc((size_t)(K > 0 ? K : 1), 1);
        for (int64_t c = 0; c < K; c++) {
            int64_t r = K - 1 - c, a = ei[r], b = ej[r], o = cp[c];
            if (e_low[r] >= 0) skip[c] = 1;
            for (int64_t k = 0; k < n; k++) {
                if (k == a || k == b) continue;
                int64_t x = R[a * n + k], y = R[b * n + k];
                if (x < 0 || y < 0) continue;
                int64_t v = max3(r, x, y), s0 = a, s1 = b, s2 = k;
                sort3(&s0, &s1, &s2);
                int64_t t = tri_index(tris, T, v, s0, s1, s2);
                cr[o++] = T - 1 - t;
            }
        }
        int64_t *piv = (int64_t *)malloc(sizeof(int64_t) * (size_t)(K > 0 ? K : 1));
        reduce_block(K, cp, cr, T, skip, piv);
        for (int64_t c = 0; c < K; c++)
            if (piv[c] >= 0) t_low[T - 1 - piv[c]] = K - 1 - c;
        free(piv); free(skip); free(cr); free(cp); free(cnt); free(R);
    }
}

/* ================= dimension 2: triangles and tetrahedra ================= */

/* A tetrahedron (value, a, b, c, d), a < b < c < d; rows of five int64. */
typedef struct { int64_t v, a, b, c, d; } tet_t;

static int cmp_tet(const tet_t *x, const tet_t *y) {
    const int64_t p[5] = {x->v, x->a, x->b, x->c, x->d}, q[5] = {y->v, y->a, y->b, y->c, y->d};
    for (int u = 0; u < 5; u++)
        if (p[u] != q[u]) return p[u] < q[u] ? -1 : 1;
    return 0;
}

/* index of a tetrahedron in the sorted list, or -1 */
static int64_t tet_index(const tet_t *tets, int64_t T3, const tet_t *key) {
    int64_t lo = 0, hi = T3;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int c = cmp_tet(&tets[mid], key);
        if (c == 0) return mid;
        if (c < 0) lo = mid + 1; else hi = mid;
    }
    return -1;
}

static int64_t *rank_matrix_of(int64_t n, int64_t K, const int64_t *ei, const int64_t *ej) {
    int64_t *R = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n * n > 0 ? n * n : 1));
    for (int64_t x = 0; x < n * n; x++) R[x] = -1;
    for (int64_t r = 0; r < K; r++) { R[ei[r] * n + ej[r]] = r; R[ej[r] * n + ei[r]] = r; }
    return R;
}

/* index of the triangle {x<y<z} (valued at its largest edge rank), or -1 */
static int64_t facet_index(const tri_t *tris, int64_t T, const int64_t *R, int64_t n, int64_t x, int64_t y, int64_t z) {
    int64_t v = max3(R[x * n + y], R[x * n + z], R[y * n + z]);
    return tri_index(tris, T, v, x, y, z);
}

/*
 * Persistence pairs of dimension 2 by Algorithm 1 on the boundary block of
 * the tetrahedra (homology): columns are the tetrahedra in filtration order
 * (value, then vertices), rows the indices of their four facets in the
 * triangle list.  As for the lower blocks, column additions stay within the
 * block, so its pivots are those of the whole boundary matrix.
 * q_low[s] = the triangle paired with tetrahedron s (its low), or -1.
 */
void or_reduce_dim2_homology(int64_t n, int64_t K, const int64_t *ei, const int64_t *ej, int64_t T,
                             const int64_t *tris4, int64_t T3, const int64_t *tets5, int64_t *q_low) {
    const tri_t *tris = (const tri_t *)tris4;
    const tet_t *tets = (const tet_t *)tets5;
    int64_t *R = rank_matrix_of(n, K, ei, ej);
    int64_t *cp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(T3 + 1));
    int64_t *cr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(4 * T3 + 1));
    for (int64_t s = 0; s < T3; s++) {
        const tet_t *q = &tets[s];
        cp[s] = 4 * s;
        cr[4 * s + 0] = facet_index(tris, T, R, n, q->a, q->b, q->c);
        cr[4 * s + 1] = facet_index(tris, T, R, n, q->a, q->b, q->d);
        cr[4 * s + 2] = facet_index(tris, T, R, n, q->a, q->c, q->d);
        cr[4 * s + 3] = facet_index(tris, T, R, n, q->b, q->c, q->d);
    }
    cp[T3] = 4 * T3;
    reduce_block(T3, cp, cr, T, NULL, q_low);
    free(cp); free(cr); free(R);
}

/*
 * The same pairs from the anti-transpose (persistent cohomology) with
 * clearing (Section 2.2.2): columns are the triangles from last to first,
 * rows the tetrahedra from last to first, so a column's low is its earliest
 * cofacet.  A triangle paired with an edge (t_low[t] >= 0, the dimension-1
 * pairs) has a coboundary that reduces to zero and is skipped.
 * Output in the convention of or_reduce_dim2_homology.
 */
void or_reduce_dim2_cohomology(int64_t n, int64_t K, const int64_t *ei, const int64_t *ej, int64_t T,
                               const int64_t *tris4, const int64_t *t_low, int64_t T3, const int64_t *tets5,
                               int64_t *q_low) {
    const tri_t *tris = (const tri_t *)tris4;
    const tet_t *tets = (const tet_t *)tets5;
    for (int64_t s = 0; s < T3; s++) q_low[s] = -1;
    if (T == 0 || T3 == 0) return;
    int64_t *R = rank_matrix_of(n, K, ei, ej);
    /* cofacets of each triangle: the vertices l joined to all three */
    int64_t *cp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(T + 1));
    cp[0] = 0;
    for (int64_t c = 0; c < T; c++) {
        const tri_t *t = &tris[T - 1 - c];
        int64_t m = 0;
        for (int64_t l = 0; l < n; l++)
            if (l != t->i && l != t->j && l != t->k && R[t->i * n + l] >= 0 && R[t->j * n + l] >= 0 &&
                R[t->k * n + l] >= 0)
                m++;
        cp[c + 1] = cp[c] + m;
    }
    int64_t *cr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cp[T] + 1));
    unsigned char *skip = (unsigned char *)calloc((size_t)T, 1);
    for (int64_t c = 0; c < T; c++) {
        const int64_t ti = T - 1 - c;
        const tri_t *t = &tris[ti];
        if (t_low[ti] >= 0) skip[c] = 1;
        int64_t o = cp[c];
        for (int64_t l = 0; l < n; l++) {
            if (l == t->i || l == t->j || l == t->k) continue;
            const int64_t x = R[t->i * n + l], y = R[t->j * n + l], z = R[t->k * n + l];
            if (x < 0 || y < 0 || z < 0) continue;
            int64_t w = max3(x, y, z);
            if (t->v > w) w = t->v;
            int64_t u[4] = {t->i, t->j, t->k, l};
            for (int p = 3; p > 0 && u[p] < u[p - 1]; p--) { int64_t h = u[p]; u[p] = u[p - 1]; u[p - 1] = h; }
            const tet_t key = {w, u[0], u[1], u[2], u[3]};
            cr[o++] = T3 - 1 - tet_index(tets, T3, &key);
        }
    }
    int64_t *piv = (int64_t *)malloc(sizeof(int64_t) * (size_t)T);
    reduce_block(T, cp, cr, T3, skip, piv);
    for (int64_t c = 0; c < T; c++)
        if (piv[c] >= 0) q_low[T3 - 1 - piv[c]] = T - 1 - c;
    free(piv); free(skip); free(cr); free(cp); free(R);
}

/*
 * Section 4.3 (redundant calculations): the per-column ordering of the
 * integers of a compressed-sparse-column array.  Column c holds the entries
 * colptr[c] .. colptr[c+1]-1.  By definition entry e of column c goes to
 * slot colptr[c] + (the entries of c with a smaller value) + (the entries of
 * c before e with the same value): its place once the column is sorted by
 * value with equal values kept in entry order.
 *
 * Computed as exactly that sort: the column's (value, entry index) pairs
 * are sorted with the C library's qsort under the order value first, entry
 * index second (no two pairs compare equal, so qsort's lack of stability
 * does not matter), and the pair sorted to position t gives its entry the
 * slot colptr[c] + t.  Any integer values are accepted.
 */
typedef struct { int64_t value, entry; } ventry_t;

static int cmp_value_then_entry(const void *a, const void *b) {
    const ventry_t *x = (const ventry_t *)a, *y = (const ventry_t *)b;
    if (x->value != y->value) return x->value < y->value ? -1 : 1;
    return (x->entry > y->entry) - (x->entry < y->entry);
}

void or_column_order(int64_t ncols, const int64_t *colptr, const int64_t *v, int64_t *z) {
    int64_t longest = 0;
    for (int64_t c = 0; c < ncols; c++)
        if (colptr[c + 1] - colptr[c] > longest) longest = colptr[c + 1] - colptr[c];
    ventry_t *col = (ventry_t *)malloc(sizeof(ventry_t) * (size_t)(longest > 0 ? longest : 1));
    for (int64_t c = 0; c < ncols; c++) {
        const int64_t start = colptr[c], len = colptr[c + 1] - colptr[c];
        for (int64_t t = 0; t < len; t++) {
            col[t].value = v[start + t];
            col[t].entry = start + t;
        }
        qsort(col, (size_t)len, sizeof(ventry_t), cmp_value_then_entry);
        for (int64_t t = 0; t < len; t++) z[col[t].entry] = start + t;
    }
    free(col);
}
