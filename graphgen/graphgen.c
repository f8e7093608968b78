/*
 * graphgen.c - seeded synthetic graph generators (host side).
 *
 * Inputs only: nothing here computes any part of the community-detection
 * method.  Every random number comes from a counter-based generator, the
 * SplitMix64 output function (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) applied to
 * (stream key + (counter + 1) * golden gamma), so any draw can be recomputed
 * from (seed, stream, counter) alone and the GPU generator in
 * graphgen_gpu.hip reproduces the R-MAT graphs bit for bit.
 *
 * Output convention (the CSR the library and the oracle both take):
 *   off[n+1] int64, col[nnz] int32, rows strictly ascending, symmetric,
 *   no self-loops, no duplicates; w[nnz] int32 or NULL for unit weights.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GG_GOLDEN 0x9E3779B97F4A7C15ULL

typedef struct {
    int64_t n, nnz;
    int64_t *off;
    int32_t *col;
    int32_t *w; /* NULL = unit weights */
} gg_csr;

static inline uint64_t gg_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
/* key of stream `stream` under `seed` */
static inline uint64_t gg_stream_key(uint64_t seed, uint64_t stream) {
    return gg_mix(seed + (stream + 1) * GG_GOLDEN);
}
/* counter-th 64-bit draw of a stream */
static inline uint64_t gg_draw(uint64_t key, uint64_t counter) {
    return gg_mix(key + (counter + 1) * GG_GOLDEN);
}
/* uniform in [0,1): top 53 bits */
static inline double gg_unit(uint64_t d) { return (double)(d >> 11) * 0x1.0p-53; }
/* uniform in (0,1] */
static inline double gg_unit_pos(uint64_t d) { return (double)((d >> 11) + 1) * 0x1.0p-53; }

uint64_t gg_draw_export(uint64_t seed, uint64_t stream, uint64_t counter) {
    return gg_draw(gg_stream_key(seed, stream), counter);
}

void gg_free(gg_csr *g) {
    if (!g) return;
    free(g->off); free(g->col); free(g->w);
    g->off = NULL; g->col = NULL; g->w = NULL;
}

/* ---- LSD radix sort of uint64 keys (8-bit digits over the low `bits` bits) ---- */
static int gg_sort_u64(uint64_t *a, int64_t n, int bits) {
    if (n <= 1) return 0;
    uint64_t *tmp = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    if (!tmp) return -1;
    uint64_t *src = a, *dst = tmp;
    for (int shift = 0; shift < bits; shift += 8) {
        int64_t cnt[257];
        memset(cnt, 0, sizeof(cnt));
        for (int64_t i = 0; i < n; ++i) cnt[((src[i] >> shift) & 255) + 1]++;
        for (int d = 0; d < 256; ++d) cnt[d + 1] += cnt[d];
        for (int64_t i = 0; i < n; ++i) dst[cnt[(src[i] >> shift) & 255]++] = src[i];
        uint64_t *t = src; src = dst; dst = t;
    }
    if (src != a) memcpy(a, src, (size_t)n * sizeof(uint64_t));
    free(tmp);
    return 0;
}

/* Build a symmetric CSR from sorted, unique undirected pairs key = (lo << sh) | hi,
 * lo < hi.  Rows come out strictly ascending without a per-row sort: the first
 * pass appends every lo to row hi (lo ascending over the sorted pairs), the
 * second appends every hi to row lo (hi ascending), and all lo < row < hi. */
static int gg_pairs_to_csr(const uint64_t *pairs, int64_t m, int sh, int64_t n,
                           int weighted, uint64_t wkey, gg_csr *out) {
    uint64_t mask = (sh == 64) ? ~0ULL : ((1ULL << sh) - 1);
    memset(out, 0, sizeof(*out));
    out->n = n;
    out->nnz = 2 * m;
    out->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    out->col = (int32_t *)malloc((size_t)(2 * m > 0 ? 2 * m : 1) * sizeof(int32_t));
    if (weighted) out->w = (int32_t *)malloc((size_t)(2 * m > 0 ? 2 * m : 1) * sizeof(int32_t));
    int64_t *fill = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!out->off || !out->col || (weighted && !out->w) || !fill) { free(fill); gg_free(out); return -1; }
    for (int64_t i = 0; i < m; ++i) {
        out->off[(pairs[i] >> sh) + 1]++;
        out->off[(pairs[i] & mask) + 1]++;
    }
    for (int64_t v = 0; v < n; ++v) out->off[v + 1] += out->off[v];
    memcpy(fill, out->off, ((size_t)n + 1) * sizeof(int64_t));
    for (int pass = 0; pass < 2; ++pass) {
        for (int64_t i = 0; i < m; ++i) {
            int64_t lo = (int64_t)(pairs[i] >> sh), hi = (int64_t)(pairs[i] & mask);
            int64_t row = pass == 0 ? hi : lo, other = pass == 0 ? lo : hi;
            int64_t p = fill[row]++;
            out->col[p] = (int32_t)other;
            if (weighted) {
                uint64_t h = gg_draw(wkey, ((uint64_t)lo << 32) | (uint64_t)hi);
                out->w[p] = (int32_t)(1 + h % 100);
            }
        }
    }
    free(fill);
    return 0;
}

/* ---- stochastic block model with contiguous near-equal blocks ----
 * block b covers [floor(b*n/k), floor((b+1)*n/k)).  Each pair {i<j} is an edge
 * independently with p_in (same block) or p_out; sampled block pair by block
 * pair with geometric skipping (Batagelj & Brandes, Phys. Rev. E 71, 2005),
 * stream of block pair (a<=b) = a*k + b. */
int gg_sbm(int64_t n, int64_t k, double p_in, double p_out, uint64_t seed, gg_csr *out) {
    memset(out, 0, sizeof(*out));
    if (n < 0 || k < 1 || n >= (1LL << 31)) return -1;
    int64_t cap = 1024, m = 0;
    uint64_t *pairs = (uint64_t *)malloc((size_t)cap * sizeof(uint64_t));
    if (!pairs) return -1;
    for (int64_t a = 0; a < k; ++a) {
        int64_t a0 = a * n / k, a1 = (a + 1) * n / k;
        for (int64_t b = a; b < k; ++b) {
            int64_t b0 = b * n / k, b1 = (b + 1) * n / k;
            double p = (a == b) ? p_in : p_out;
            if (p <= 0.0 || a1 <= a0 || b1 <= b0) continue;
            int64_t L = (a == b) ? (a1 - a0) * (a1 - a0 - 1) / 2 : (a1 - a0) * (b1 - b0);
            if (L <= 0) continue;
            uint64_t key = gg_stream_key(seed, (uint64_t)(a * k + b));
            uint64_t ctr = 0;
            double lq = (p < 1.0) ? log1p(-p) : 0.0;
            /* row walker for the triangle case */
            int64_t ri = a0, rstart = 0, rlen = a1 - a0 - 1;
            int64_t t = -1;
            for (;;) {
                if (p >= 1.0) t += 1;
                else {
                    double u = gg_unit_pos(gg_draw(key, ctr++));
                    double s = floor(log(u) / lq);
                    if (s >= (double)L) break;
                    t += 1 + (int64_t)s;
                }
                if (t >= L) break;
                int64_t i, j;
                if (a == b) {
                    while (t >= rstart + rlen) { rstart += rlen; ri++; rlen--; }
                    i = ri; j = ri + 1 + (t - rstart);
                } else {
                    i = a0 + t / (b1 - b0); j = b0 + t % (b1 - b0);
                }
                if (m == cap) {
                    cap *= 2;
                    uint64_t *np = (uint64_t *)realloc(pairs, (size_t)cap * sizeof(uint64_t));
                    if (!np) { free(pairs); return -1; }
                    pairs = np;
                }
                pairs[m++] = ((uint64_t)i << 32) | (uint64_t)j;
            }
        }
    }
    int rc = gg_sort_u64(pairs, m, 64);
    if (rc == 0) rc = gg_pairs_to_csr(pairs, m, 32, n, 0, 0, out);
    free(pairs);
    return rc;
}

/* ---- R-MAT ----
 * scale s, edge factor ef: ef*2^s directed draws.  Draw e picks its quadrant at
 * depth d (d = 0 is the most significant bit) from uniform number e*s + d of
 * stream 1: [0,a) -> (0,0), [a,a+b) -> (0,1), [a+b,a+b+c) -> (1,0), else (1,1).
 * Endpoints are then relabelled by the bijection gg_rmat_perm, self-loops are
 * dropped and {u,v} duplicates are merged.  Weighted graphs take
 * w = 1 + (draw(stream 2, (lo << 32) | hi) mod 100), a function of the pair. */
uint64_t gg_rmat_perm(uint64_t x, int s, uint64_t seed) {
    uint64_t mask = (s >= 64) ? ~0ULL : ((1ULL << s) - 1);
    uint64_t key = gg_stream_key(seed, 3);
    int sh = (s + 1) / 2;
    for (int r = 0; r < 3; ++r) {
        uint64_t mul = gg_draw(key, 2 * r) | 1ULL;
        uint64_t add = gg_draw(key, 2 * r + 1);
        x = (x * mul) & mask;
        if (s > 1) x ^= x >> sh;
        x = (x + add) & mask;
    }
    return x;
}

static inline uint64_t gg_rmat_edge(uint64_t key, int64_t e, int s, double a, double ab, double abc) {
    uint64_t r = 0, c = 0;
    for (int d = 0; d < s; ++d) {
        double u = gg_unit(gg_draw(key, (uint64_t)e * (uint64_t)s + (uint64_t)d));
        uint64_t rb = (u >= ab), cb = (u >= a && u < ab) || (u >= abc);
        r = (r << 1) | rb;
        c = (c << 1) | cb;
    }
    return (r << 32) | c;
}

int gg_rmat(int s, int64_t ef, double a, double b, double c, uint64_t seed, int weighted, gg_csr *out) {
    memset(out, 0, sizeof(*out));
    if (s < 1 || s > 30 || ef < 0) return -1;
    int64_t n = 1LL << s, E = ef * n;
    uint64_t *pairs = (uint64_t *)malloc((size_t)(E > 0 ? E : 1) * sizeof(uint64_t));
    if (!pairs) return -1;
    uint64_t key = gg_stream_key(seed, 1);
    double ab = a + b, abc = a + b + c;
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        uint64_t rc = gg_rmat_edge(key, e, s, a, ab, abc);
        uint64_t u = gg_rmat_perm(rc >> 32, s, seed), v = gg_rmat_perm(rc & 0xffffffffULL, s, seed);
        if (u == v) pairs[e] = ~0ULL;
        else {
            uint64_t lo = u < v ? u : v, hi = u < v ? v : u;
            pairs[e] = (lo << s) | hi;
        }
    }
    int rc = gg_sort_u64(pairs, E, 2 * s + (2 * s < 64 ? 1 : 0));
    if (rc) { free(pairs); return rc; }
    /* sentinels (self-loops) have bit 2s set and sort last; unique the rest */
    int64_t m = 0;
    uint64_t lim = 1ULL << (2 * s);
    for (int64_t i = 0; i < E; ++i) {
        if (pairs[i] >= lim) break;
        if (m == 0 || pairs[i] != pairs[m - 1]) pairs[m++] = pairs[i];
    }
    rc = gg_pairs_to_csr(pairs, m, s, n, weighted, gg_stream_key(seed, 2), out);
    free(pairs);
    return rc;
}

/* ---- parameters of the batch of SBM graphs ----
 * graph i: n_i = floor(exp(U(ln n_lo, ln n_hi))) with U drawn from stream 5,
 * counter i; k_i = max(2, floor(n_i / 100)); p_in = 20 / (n_i / k_i) (capped at 1);
 * p_out = 1 / n_i; graph seed = draw(stream 6, counter i). */
void gg_batch_params(uint64_t seed, int64_t count, double n_lo, double n_hi, int64_t *n_out,
                     int64_t *k_out, double *pin_out, double *pout_out, uint64_t *seed_out) {
    uint64_t kn = gg_stream_key(seed, 5), ks = gg_stream_key(seed, 6);
    double l0 = log(n_lo), l1 = log(n_hi);
    for (int64_t i = 0; i < count; ++i) {
        double u = gg_unit(gg_draw(kn, (uint64_t)i));
        int64_t ni = (int64_t)floor(exp(l0 + u * (l1 - l0)));
        if (ni < 2) ni = 2;
        int64_t ki = ni / 100;
        if (ki < 2) ki = 2;
        double bs = (double)ni / (double)ki;
        double pin = 20.0 / bs;
        if (pin > 1.0) pin = 1.0;
        n_out[i] = ni; k_out[i] = ki; pin_out[i] = pin; pout_out[i] = 1.0 / (double)ni;
        seed_out[i] = gg_draw(ks, (uint64_t)i);
    }
}
