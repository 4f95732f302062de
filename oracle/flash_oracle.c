/*
 * Plain CPU oracle for the FLASH hot path (Wang, Shrivastava, Wang & Ryu,
 * "FLASH: Randomized Algorithms Accelerated over CPU-GPU for Ultra-High
 * Dimensional Similarity Search", arXiv 1709.01190).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this file.  It shares no code, header,
 * table or constant generator with the HIP library; it is written to be
 * slow and obviously correct, in the paper's order of steps.
 *
 * Functions and what pins them (see tests/test_oracle_pins.py):
 *   orc_seeds, orc_mix64, orc_fmix32   bit-level building blocks; pinned by
 *                                      bijectivity, a published splitmix64
 *                                      output sequence and the Eq. 2 rate.
 *   orc_doph                           Sec. 2.3 DOPH + Sec. 2.2 key mapping;
 *                                      pinned by Eq. 1 (K = L = 1 is plain
 *                                      minhash), Eq. 2 (collision = Jaccard),
 *                                      b-bit collision rate, no empty bins.
 *   orc_build                          Alg. 1/2 reservoirs (bottom-R reading);
 *                                      pinned by brute-force histograms,
 *                                      min(count, R) occupancy, uniform
 *                                      inclusion, order independence.
 *   orc_query                          Alg. 3 KSELECT; pinned by a brute-force
 *                                      recount, an independent dynamic-bucket
 *                                      LSH when R covers every bucket, and
 *                                      App. B's retrieval probability.
 *   orc_jaccard_knn                    exact Jaccard neighbours (Eq. 2's right
 *                                      side) for recall; pinned by direct set
 *                                      intersection on tiny inputs.
 *   orc_pool_size, orc_reservoir       Sec. 3.5 reservoir sharing; pinned by
 *                                      F = 1 giving the plain index, the
 *                                      pool of ceil(F * L * M) reservoirs
 *                                      (exact rational arithmetic), a uniform
 *                                      map, brute-force shared tables and
 *                                      queries.
 *   orc_rerank                         Sec. 4.3 exact cosine (Eq. 3) / Jaccard
 *                                      ordering; pinned by Python sets and
 *                                      fractions and a hand-worked case.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_EMPTY 0xFFFFFFFFu

typedef struct {
    int32_t K;                /* minhashes per meta-hash (Sec. 2.2) */
    int32_t L;                /* tables */
    int32_t bits_per_hash;    /* b: low bits of each minhash kept in the key */
    int32_t R;                /* reservoir size (Sec. 2.4, Alg. 2) */
    uint64_t seed;            /* user seed */
    int32_t densify_attempts; /* random probes per empty bin before rotation */
    int32_t share_permille;   /* reservoir sharing F in thousandths (Sec. 3.5); 0 or 1000: none */
} orc_params;

/* ---- bit-level building blocks ------------------------------------------ */

/* splitmix64 output function (Steele, Lea & Flood 2014). */
uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* MurmurHash3 32-bit finaliser (Appleby); a bijection on 32-bit words. */
uint32_t orc_fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

/* One user seed expanded by the splitmix64 sequence into the hash seed s_h,
 * the densification seed s_d and the reservoir priority seed s_p.  The
 * paper says DOPH needs only a handful of random numbers (Sec. 2.3). */
void orc_seeds(uint64_t seed, uint32_t *s_h, uint32_t *s_d, uint64_t *s_p)
{
    uint64_t state = seed;
    state += 0x9E3779B97F4A7C15ULL;
    *s_h = (uint32_t)orc_mix64(state);
    state += 0x9E3779B97F4A7C15ULL;
    *s_d = (uint32_t)orc_mix64(state);
    state += 0x9E3779B97F4A7C15ULL;
    *s_p = orc_mix64(state);
}

/* The fourth output of the same splitmix64 sequence: the seed of the
 * bucket-to-reservoir map used when reservoirs are shared (Sec. 3.5). */
uint32_t orc_share_seed(uint64_t seed)
{
    return (uint32_t)orc_mix64(seed + 4 * 0x9E3779B97F4A7C15ULL);
}

/* Position of 32-bit value h in a range of n equal slices (multiply-shift). */
static uint32_t slice_of(uint32_t h, uint32_t n)
{
    return (uint32_t)(((uint64_t)h * (uint64_t)n) >> 32);
}

/* ---- Sec. 2.3: densified one-permutation hashing of one row ------------- */

/*
 * One permutation pi(i) = fmix32(i ^ s_h) of the column space; the permuted
 * range is cut into B = K*L equal bins and code[j] is the smallest pi(i) of
 * the row's columns that fall in bin j (Eq. 1 restricted to one bin).
 * Empty bins are then filled from originally non-empty ones: bin j tries the
 * bins chosen by a hash of (j, attempt) for attempt = 1..A, and if none of
 * them is occupied takes the nearest occupied bin to its right (cyclically).
 * Returns 0 for an empty row (all codes ORC_EMPTY), 1 otherwise.
 */
static int doph_codes(const int32_t *cols, int64_t n, int B, uint32_t s_h, uint32_t s_d,
                      int A, uint32_t *code, unsigned char *occ, uint32_t *out)
{
    int j;
    int64_t e;
    for (j = 0; j < B; j++) {
        occ[j] = 0;
        code[j] = 0;
    }
    for (e = 0; e < n; e++) {
        uint32_t h = orc_fmix32((uint32_t)cols[e] ^ s_h);
        uint32_t bin = slice_of(h, (uint32_t)B);
        if (!occ[bin] || h < code[bin]) {
            code[bin] = h;
            occ[bin] = 1;
        }
    }
    if (n == 0) {
        for (j = 0; j < B; j++) out[j] = ORC_EMPTY;
        return 0;
    }
    for (j = 0; j < B; j++) {
        int a, r, done = 0;
        if (occ[j]) {
            out[j] = code[j];
            continue;
        }
        for (a = 1; a <= A && !done; a++) {
            uint32_t p = slice_of(orc_fmix32((((uint32_t)j << 16) | (uint32_t)a) ^ s_d), (uint32_t)B);
            if (occ[p]) {
                out[j] = code[p];
                done = 1;
            }
        }
        for (r = 1; r < B && !done; r++) {
            int p = (j + r) % B;
            if (occ[p]) {
                out[j] = code[p];
                done = 1;
            }
        }
    }
    return 1;
}

/* Sec. 2.2 "MapKHashesToAddress": table t's key concatenates the low b bits
 * of minhashes t*K .. t*K+K-1, the first in the lowest bits. */
static uint32_t table_key(const uint32_t *codes, int t, int K, int b)
{
    uint32_t key = 0, mask = (b >= 32) ? 0xFFFFFFFFu : ((1u << b) - 1u);
    int j;
    for (j = 0; j < K; j++) key |= (codes[t * K + j] & mask) << (b * j);
    return key;
}

/* Hash every row: keys[i][t] (ORC_EMPTY for an empty row) and, if codes is
 * not NULL, the B densified minhashes codes[i][j]. */
void orc_doph(const orc_params *p, int64_t n_rows, const int64_t *row_ptr,
              const int32_t *col_idx, uint32_t *keys, uint32_t *codes)
{
    const int B = p->K * p->L;
    uint32_t s_h, s_d;
    uint64_t s_p;
    int64_t i;
    orc_seeds(p->seed, &s_h, &s_d, &s_p);
#pragma omp parallel
    {
        uint32_t *code = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)B);
        uint32_t *dense = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)B);
        unsigned char *occ = (unsigned char *)malloc((size_t)B);
#pragma omp for schedule(dynamic, 64)
        for (i = 0; i < n_rows; i++) {
            int t, nonempty;
            int64_t beg = row_ptr[i], len = row_ptr[i + 1] - row_ptr[i];
            nonempty = doph_codes(col_idx + beg, len, B, s_h, s_d, p->densify_attempts,
                                  code, occ, dense);
            for (t = 0; t < p->L; t++)
                keys[i * p->L + t] = nonempty ? table_key(dense, t, p->K, p->bits_per_hash) : ORC_EMPTY;
            if (codes) memcpy(codes + i * B, dense, sizeof(uint32_t) * (size_t)B);
        }
        free(code);
        free(dense);
        free(occ);
    }
}

/* ---- Alg. 1/2: reservoirs of size R, read as bottom-R priority sampling - */

/* Priority of id in table t: a 32-bit pseudo-random value from
 * (s_p, t, id), with the id itself below it so that priorities are
 * distinct.  The R smallest priorities among a bucket's arrivals are a
 * uniform R-subset, which is what Vitter's reservoir keeps (Sec. 2.4). */
uint64_t orc_priority(uint64_t s_p, int t, int32_t id)
{
    uint64_t x = orc_mix64(s_p ^ (((uint64_t)(uint32_t)t << 32) | (uint64_t)(uint32_t)id));
    return ((x >> 32) << 32) | (uint64_t)(uint32_t)id;
}

typedef struct {
    uint32_t key;
    uint64_t pri;
} arrival;

static int cmp_arrival(const void *a, const void *b)
{
    const arrival *x = (const arrival *)a, *y = (const arrival *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->pri != y->pri) return x->pri < y->pri ? -1 : 1;
    return 0;
}

/* ---- Sec. 3.5: reservoir sharing ----------------------------------------- */

static int shared(const orc_params *p)
{
    return p->share_permille > 0 && p->share_permille < 1000;
}

/*
 * Number of reservoirs.  Without sharing, one per bucket: L * M.  With
 * sharing, Sec. 3.5 defines F as the ratio of the reservoirs allocated to
 * the range they serve; the pool serves all L tables of M buckets, so it
 * holds ceil(F * L * M) reservoirs (at least one), F = share_permille / 1000.
 */
uint64_t orc_pool_size(const orc_params *p)
{
    const uint64_t M = 1ULL << (p->K * p->bits_per_hash);
    const uint64_t LM = (uint64_t)p->L * M;
    uint64_t P;
    if (!shared(p)) return LM;
    P = (LM * (uint64_t)p->share_permille + 999) / 1000;
    return P < 1 ? 1 : P;
}

/*
 * Reservoir of bucket m of table t.  Without sharing: t * M + m.  With
 * sharing, every bucket is given one reservoir of the pool at random (a
 * seeded hash of its index), so buckets of any tables may share one.
 */
uint64_t orc_reservoir(const orc_params *p, uint64_t t, uint64_t m)
{
    const uint64_t M = 1ULL << (p->K * p->bits_per_hash);
    if (!shared(p)) return t * M + m;
    return slice_of(orc_fmix32((uint32_t)(t * M + m) ^ orc_share_seed(p->seed)),
                    (uint32_t)orc_pool_size(p));
}

/*
 * counts[t][m] = number of rows whose key in table t is m (Alg. 2's
 * ReservoirCounter after all additions); ids[t][m][0 .. min(count, R)) hold
 * the ids of the smallest priorities in ascending priority order; the other
 * slots are -1.  Rows whose key is ORC_EMPTY or >= 2^(K*b) are not added.
 */
static void build_shared(const orc_params *p, int64_t n_rows, const uint32_t *keys,
                         uint32_t *counts, int32_t *ids);

void orc_build(const orc_params *p, int64_t n_rows, const uint32_t *keys,
               uint32_t *counts, int32_t *ids)
{
    const int L = p->L, R = p->R;
    const uint64_t M = 1ULL << (p->K * p->bits_per_hash);
    uint32_t s_h, s_d;
    uint64_t s_p;
    int t;
    if (shared(p)) {
        build_shared(p, n_rows, keys, counts, ids);
        return;
    }
    orc_seeds(p->seed, &s_h, &s_d, &s_p);
#pragma omp parallel for schedule(dynamic, 1)
    for (t = 0; t < L; t++) {
        arrival *arr = (arrival *)malloc(sizeof(arrival) * (size_t)(n_rows > 0 ? n_rows : 1));
        int64_t n = 0, i, g;
        uint32_t *cnt = counts + (uint64_t)t * M;
        int32_t *tab = ids + (uint64_t)t * M * (uint64_t)R;
        memset(cnt, 0, sizeof(uint32_t) * M);
        for (i = 0; i < (int64_t)(M * (uint64_t)R); i++) tab[i] = -1;
        for (i = 0; i < n_rows; i++) {
            uint32_t k = keys[i * L + t];
            if (k == ORC_EMPTY || (uint64_t)k >= M) continue;
            arr[n].key = k;
            arr[n].pri = orc_priority(s_p, t, (int32_t)i);
            n++;
        }
        qsort(arr, (size_t)n, sizeof(arrival), cmp_arrival);
        for (g = 0; g < n;) {
            int64_t e = g;
            uint32_t k = arr[g].key;
            while (e < n && arr[e].key == k) e++;
            cnt[k] = (uint32_t)(e - g);
            for (i = g; i < e && i - g < R; i++)
                tab[(uint64_t)k * R + (uint64_t)(i - g)] = (int32_t)(uint32_t)(arr[i].pri & 0xFFFFFFFFu);
            g = e;
        }
        free(arr);
    }
}

/*
 * The same bottom-R reading over a shared pool: every (table, row) arrival
 * goes to the reservoir of its bucket; a reservoir counts its arrivals and
 * keeps the R with the smallest priority, where the priority of id i in
 * reservoir r is orc_priority(s_p, r, i) (the reservoir takes the place of
 * the table).  A row whose buckets in several tables map to one reservoir
 * arrives there once (from its first such table), so a reservoir holds
 * distinct ids and a query's count stays at most L.
 */
static void build_shared(const orc_params *p, int64_t n_rows, const uint32_t *keys,
                         uint32_t *counts, int32_t *ids)
{
    const int L = p->L, R = p->R;
    const uint64_t M = 1ULL << (p->K * p->bits_per_hash);
    const uint64_t P = orc_pool_size(p);
    uint32_t s_h, s_d;
    uint64_t s_p;
    arrival *arr = (arrival *)malloc(sizeof(arrival) * (size_t)(n_rows * L + 1));
    uint64_t *res = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n_rows * L + 1));
    int64_t n = 0, i, g;
    uint64_t r;
    orc_seeds(p->seed, &s_h, &s_d, &s_p);
    memset(counts, 0, sizeof(uint32_t) * P);
    for (r = 0; r < P * (uint64_t)R; r++) ids[r] = -1;
    /* arrivals keyed by (reservoir, priority); the reservoir index fits in
     * the 32-bit key field because P < 2^32 */
    for (i = 0; i < n_rows; i++) {
        int t, u;
        int64_t first = n;
        for (t = 0; t < L; t++) {
            uint32_t k = keys[i * L + t];
            uint64_t r;
            int seen = 0;
            if (k == ORC_EMPTY || (uint64_t)k >= M) continue;
            r = orc_reservoir(p, (uint64_t)t, k);
            for (u = (int)first; u < (int)n; u++)
                if (res[u] == r) seen = 1;
            if (seen) continue;
            res[n] = r;
            arr[n].key = (uint32_t)r;
            arr[n].pri = orc_priority(s_p, (int)r, (int32_t)i);
            n++;
        }
    }
    qsort(arr, (size_t)n, sizeof(arrival), cmp_arrival);
    for (g = 0; g < n;) {
        int64_t e = g;
        uint32_t k = arr[g].key;
        while (e < n && arr[e].key == k) e++;
        counts[k] = (uint32_t)(e - g);
        for (i = g; i < e && i - g < R; i++)
            ids[(uint64_t)k * R + (uint64_t)(i - g)] = (int32_t)(uint32_t)(arr[i].pri & 0xFFFFFFFFu);
        g = e;
    }
    free(arr);
    free(res);
}

/* ---- Alg. 3: gather L reservoirs, count, rank --------------------------- */

typedef struct {
    int32_t id;
    int32_t cnt;
} idcount;

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static int cmp_rank(const void *a, const void *b)
{
    const idcount *x = (const idcount *)a, *y = (const idcount *)b;
    if (x->cnt != y->cnt) return x->cnt > y->cnt ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

/*
 * For query q with keys qkeys[q][0..L): A is the concatenation of the
 * occupied slots of bucket qkeys[q][t] of every table t (self_ids[q], if
 * given and >= 0, is left out); KSELECT sorts A, counts each run of equal
 * ids, sorts the (id, count) pairs by count descending then id ascending
 * and returns the first k.  Missing entries are (-1, 0).
 */
void orc_query(const orc_params *p, const uint32_t *counts, const int32_t *ids,
               int64_t n_queries, const uint32_t *qkeys, const int32_t *self_ids,
               int32_t k, int32_t *out_ids, int32_t *out_counts)
{
    const int L = p->L, R = p->R;
    const uint64_t M = 1ULL << (p->K * p->bits_per_hash);
    int64_t q;
#pragma omp parallel
    {
        int32_t *A = (int32_t *)malloc(sizeof(int32_t) * (size_t)L * (size_t)R + 1);
        idcount *kv = (idcount *)malloc(sizeof(idcount) * (size_t)L * (size_t)R + 1);
#pragma omp for schedule(dynamic, 16)
        for (q = 0; q < n_queries; q++) {
            int64_t na = 0, nkv = 0, e;
            int t, j;
            int32_t self = self_ids ? self_ids[q] : -1;
            for (t = 0; t < L; t++) {
                uint32_t key = qkeys[q * L + t];
                uint64_t occ;
                uint64_t res;
                if (key == ORC_EMPTY || (uint64_t)key >= M) continue;
                res = orc_reservoir(p, (uint64_t)t, key);
                occ = counts[res];
                if (occ > (uint64_t)R) occ = (uint64_t)R;
                for (j = 0; j < (int)occ; j++) {
                    int32_t x = ids[res * (uint64_t)R + (uint64_t)j];
                    if (self >= 0 && x == self) continue;
                    A[na++] = x;
                }
            }
            qsort(A, (size_t)na, sizeof(int32_t), cmp_i32);
            for (e = 0; e < na; e++) {
                if (e == 0 || A[e] != A[e - 1]) {
                    kv[nkv].id = A[e];
                    kv[nkv].cnt = 0;
                    nkv++;
                }
                kv[nkv - 1].cnt++;
            }
            qsort(kv, (size_t)nkv, sizeof(idcount), cmp_rank);
            for (j = 0; j < k; j++) {
                out_ids[q * k + j] = j < nkv ? kv[j].id : -1;
                out_counts[q * k + j] = j < nkv ? kv[j].cnt : 0;
            }
        }
        free(A);
        free(kv);
    }
}

/* ---- exact Jaccard neighbours for recall (Eq. 2's right-hand side) ----- */

static int64_t dedup_sorted(int32_t *v, int64_t n)
{
    int64_t i, m = 0;
    qsort(v, (size_t)n, sizeof(int32_t), cmp_i32);
    for (i = 0; i < n; i++)
        if (m == 0 || v[i] != v[m - 1]) v[m++] = v[i];
    return m;
}

/* |x ∩ y| and |x ∪ y| of two rows read as sets of column ids. */
void orc_jaccard_pairs(const int64_t *row_ptr, const int32_t *col_idx, int64_t n_pairs,
                       const int64_t *xs, const int64_t *ys, int64_t *inter, int64_t *uni)
{
    int64_t pi;
#pragma omp parallel for schedule(dynamic, 64)
    for (pi = 0; pi < n_pairs; pi++) {
        int64_t x = xs[pi], y = ys[pi];
        int64_t nx = row_ptr[x + 1] - row_ptr[x], ny = row_ptr[y + 1] - row_ptr[y];
        int32_t *a = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nx + 1));
        int32_t *b = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ny + 1));
        int64_t i = 0, j = 0, c = 0;
        memcpy(a, col_idx + row_ptr[x], sizeof(int32_t) * (size_t)nx);
        memcpy(b, col_idx + row_ptr[y], sizeof(int32_t) * (size_t)ny);
        nx = dedup_sorted(a, nx);
        ny = dedup_sorted(b, ny);
        while (i < nx && j < ny) {
            if (a[i] == b[j]) {
                c++;
                i++;
                j++;
            } else if (a[i] < b[j]) {
                i++;
            } else {
                j++;
            }
        }
        inter[pi] = c;
        uni[pi] = nx + ny - c;
        free(a);
        free(b);
    }
}

/* J(q,x) > J(q,y) for J = i/u, compared exactly. */
static int jac_greater(int64_t i1, int64_t u1, int64_t i2, int64_t u2)
{
    return (__int128)i1 * u2 > (__int128)i2 * u1;
}

/*
 * Exact Jaccard top-k of each query row q (a row of the same CSR) over all
 * rows x != q, ranked by J descending then id ascending; rows with no
 * common column are never listed (pad -1, J = 0/1).  Rows are read as sets
 * (duplicates ignored); they are expected sorted and distinct for speed
 * but correctness does not depend on it except through the inverted index
 * (built from distinct (column,row) pairs below).
 */
void orc_jaccard_knn(const int64_t *row_ptr, const int32_t *col_idx, int64_t n_rows,
                     int64_t n_cols, int64_t n_queries, const int64_t *queries, int32_t k,
                     int32_t *out_ids, int64_t *out_inter, int64_t *out_union)
{
    int64_t nnz = row_ptr[n_rows], i, q;
    int64_t *post_ptr = (int64_t *)calloc((size_t)n_cols + 1, sizeof(int64_t));
    int64_t *post_fill = (int64_t *)calloc((size_t)n_cols + 1, sizeof(int64_t));
    int32_t *post = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz + 1));
    int64_t *rowlen = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_rows + 1));
    for (i = 0; i < n_rows; i++) {
        int64_t e;
        rowlen[i] = 0;
        for (e = row_ptr[i]; e < row_ptr[i + 1]; e++) {
            if (e > row_ptr[i] && col_idx[e] == col_idx[e - 1]) continue;
            post_ptr[col_idx[e] + 1]++;
            rowlen[i]++;
        }
    }
    for (i = 0; i < n_cols; i++) post_ptr[i + 1] += post_ptr[i];
    for (i = 0; i < n_rows; i++) {
        int64_t e;
        for (e = row_ptr[i]; e < row_ptr[i + 1]; e++) {
            if (e > row_ptr[i] && col_idx[e] == col_idx[e - 1]) continue;
            post[post_ptr[col_idx[e]] + post_fill[col_idx[e]]++] = (int32_t)i;
        }
    }
#pragma omp parallel
    {
        int32_t *inter = (int32_t *)calloc((size_t)n_rows + 1, sizeof(int32_t));
        int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_rows + 1));
        int32_t *best = (int32_t *)malloc(sizeof(int32_t) * (size_t)(k + 1));
#pragma omp for schedule(dynamic, 4)
        for (q = 0; q < n_queries; q++) {
            int64_t qr = queries[q], nt = 0, e, c;
            int nb = 0, j;
            for (e = row_ptr[qr]; e < row_ptr[qr + 1]; e++) {
                int32_t col = col_idx[e];
                int64_t pp;
                if (e > row_ptr[qr] && col == col_idx[e - 1]) continue;
                for (pp = post_ptr[col]; pp < post_ptr[col + 1]; pp++) {
                    int32_t x = post[pp];
                    if (x == qr) continue;
                    if (inter[x] == 0) touched[nt++] = x;
                    inter[x]++;
                }
            }
            /* insertion into a sorted top-k list */
            for (c = 0; c < nt; c++) {
                int32_t x = touched[c];
                int64_t ix = inter[x], ux = rowlen[qr] + rowlen[x] - inter[x];
                int pos = nb;
                while (pos > 0) {
                    int32_t y = best[pos - 1];
                    int64_t iy = inter[y], uy = rowlen[qr] + rowlen[y] - inter[y];
                    if (jac_greater(ix, ux, iy, uy) || (!jac_greater(iy, uy, ix, ux) && x < y)) pos--;
                    else break;
                }
                if (pos >= k) continue;
                if (nb < k) nb++;
                for (j = nb - 1; j > pos; j--) best[j] = best[j - 1];
                best[pos] = x;
            }
            for (j = 0; j < k; j++) {
                if (j < nb) {
                    int32_t y = best[j];
                    out_ids[q * k + j] = y;
                    out_inter[q * k + j] = inter[y];
                    out_union[q * k + j] = rowlen[qr] + rowlen[y] - inter[y];
                } else {
                    out_ids[q * k + j] = -1;
                    out_inter[q * k + j] = 0;
                    out_union[q * k + j] = 1;
                }
            }
            for (c = 0; c < nt; c++) inter[touched[c]] = 0;
        }
        free(inter);
        free(touched);
        free(best);
    }
    free(post_ptr);
    free(post_fill);
    free(post);
    free(rowlen);
}

/* ---- exact re-rank of candidate lists (Sec. 4.3's gold standard) ------- */

#define ORC_SIM_COSINE 0
#define ORC_SIM_JACCARD 1

/*
 * sim1 > sim2 for candidates with intersections i1, i2 and sizes x1, x2
 * against a query of size nq, exactly.  Jaccard (Eq. 2's right-hand side)
 * is i / (nq + x - i); cosine for binary vectors (Eq. 3) is i / sqrt(nq x),
 * compared through its square i^2 / (nq x), which orders the same way; nq
 * cancels.  A candidate with no common column has similarity 0.
 */
static int sim_greater(int measure, int64_t nq, int64_t i1, int64_t x1, int64_t i2, int64_t x2)
{
    __int128 a, b;
    if (i1 == 0) return 0;
    if (i2 == 0) return 1;
    if (measure == ORC_SIM_JACCARD) {
        a = (__int128)i1 * (nq + x2 - i2);
        b = (__int128)i2 * (nq + x1 - i1);
    } else {
        a = (__int128)i1 * i1 * x2;
        b = (__int128)i2 * i2 * x1;
    }
    return a > b;
}

/*
 * For each query row q (q_row_ptr / q_col_idx) and its candidate ids
 * cand[q][0..nc) (rows of row_ptr / col_idx; negative = no candidate):
 * inter = |q ∩ x| over distinct columns, then the candidates ordered by
 * similarity descending, ties by smaller id (insertion sort), and the first
 * k written to out_ids / out_inter, padded with (-1, 0).
 */
void orc_rerank(int measure, const int64_t *row_ptr, const int32_t *col_idx, int64_t n_queries,
                const int64_t *q_row_ptr, const int32_t *q_col_idx, const int32_t *cand, int32_t nc,
                int32_t k, int32_t *out_ids, int64_t *out_inter)
{
    int64_t q;
#pragma omp parallel for schedule(dynamic, 8)
    for (q = 0; q < n_queries; q++) {
        int64_t nq = q_row_ptr[q + 1] - q_row_ptr[q];
        int32_t *qa = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nq + 1));
        int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nc + 1));
        int64_t *in = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nc + 1));
        int64_t *sz = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nc + 1));
        int m = 0, c, j;
        memcpy(qa, q_col_idx + q_row_ptr[q], sizeof(int32_t) * (size_t)nq);
        nq = dedup_sorted(qa, nq);
        for (c = 0; c < nc; c++) {
            int32_t x = cand[q * nc + c];
            int64_t nx, i = 0, jj = 0, cnt = 0;
            int32_t *xa;
            int pos;
            if (x < 0) continue;
            nx = row_ptr[x + 1] - row_ptr[x];
            xa = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nx + 1));
            memcpy(xa, col_idx + row_ptr[x], sizeof(int32_t) * (size_t)nx);
            nx = dedup_sorted(xa, nx);
            while (i < nq && jj < nx) {
                if (qa[i] == xa[jj]) {
                    cnt++;
                    i++;
                    jj++;
                } else if (qa[i] < xa[jj]) {
                    i++;
                } else {
                    jj++;
                }
            }
            free(xa);
            /* insert (x, cnt, nx) into the ordered list */
            pos = m;
            while (pos > 0) {
                int better = sim_greater(measure, nq, cnt, nx, in[pos - 1], sz[pos - 1]);
                int worse = sim_greater(measure, nq, in[pos - 1], sz[pos - 1], cnt, nx);
                if (better || (!worse && x < ids[pos - 1])) pos--;
                else break;
            }
            for (j = m; j > pos; j--) {
                ids[j] = ids[j - 1];
                in[j] = in[j - 1];
                sz[j] = sz[j - 1];
            }
            ids[pos] = x;
            in[pos] = cnt;
            sz[pos] = nx;
            m++;
        }
        for (j = 0; j < k; j++) {
            out_ids[q * k + j] = j < m ? ids[j] : -1;
            out_inter[q * k + j] = j < m ? in[j] : 0;
        }
        free(qa);
        free(ids);
        free(in);
        free(sz);
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads the parallel loops use from now on (n >= 1); for timing only. */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
