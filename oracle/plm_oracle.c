/*
 * plm_oracle.c - plain, slow, single-threaded reference of the Parallel Louvain
 * Method (PLM) under a deterministic colour-class schedule.
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the CPU
 * baseline of the benchmark call it to check the GPU library; the library never
 * links, loads or calls it, and the two share no code.
 *
 * What is computed (Staudt & Meyerhenke, "Engineering Parallel Algorithms for
 * Community Detection in Massive Networks", section III-B):
 *   - the graph is undirected with positive weights; node volume vol(u) is the
 *     sum of incident weights with a self-loop counted twice (section III-B,
 *     definition of vol).  Internally every self-loop entry therefore carries
 *     twice its weight ("doubled diagonal"), so vol(u) is a plain row sum and
 *     S = sum of all volumes = 2 w(E).
 *   - modularity, Equation (3.1), written with integers:
 *       mod = (S * I2 - sum_C vol(C)^2) / S^2,
 *     I2 = sum of doubled-diagonal entries inside communities = 2 sum_C w(C).
 *   - the gain of moving u from D = zeta(u) to a neighbouring community X is the
 *     paper's Delta-mod (section III-B, the formula after Equation (3.1)) times
 *     2 w(E)^2:
 *       gain = S (w(u,X) - w(u,D\u)) - vol(u) (vol(X) - vol(D\u)),
 *     computed exactly in 128-bit integers.
 *   - move (Algorithm 2): u takes the best neighbouring community if the gain is
 *     strictly positive; ties go to the lowest community id.
 *   - PLM (Algorithm 3): singletons, move until stable, coarsen if the
 *     partition changed, recurse on the coarse graph, prolong.
 *   - coarsen (section III-B, implementation): one coarse node per community,
 *     inter-community weights summed, intra-community weight kept as a
 *     self-loop; prolongation composes the fine-to-coarse maps.
 *
 * Where the paper leaves the order of moves to asynchronous threads, this
 * oracle fixes it: nodes are coloured greedily in descending priority
 * (H(seed, level, u), u) with H = SplitMix64, which equals the Jones-Plassmann
 * colouring; a sweep visits the colour classes in ascending order, and all nodes
 * of one class decide against the community volumes at the start of the class
 * (they are pairwise non-adjacent, so no decision sees another's move), then
 * all their moves are applied.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

#ifdef _OPENMP
#include <omp.h>
static int orc_thread(void) { return omp_get_thread_num(); }
#else
static int orc_thread(void) { return 0; }
#endif

/* ------------------------------------------------------------------ hashing */
/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): one step from state x. */
uint64_t orc_splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Priority hash of node u at a level. */
uint64_t orc_priority(uint64_t seed, int32_t level, int64_t u) {
    return orc_splitmix64(seed ^ ((uint64_t)(uint32_t)level << 40) ^ (uint64_t)u);
}

/* ------------------------------------------------------------------ graph prep */
/* w2[e] = w[e], doubled on the diagonal; w == NULL means unit weights. */
void orc_double_diagonal(int64_t n, const int64_t *off, const int32_t *col, const int64_t *w, int64_t *w2) {
    for (int64_t u = 0; u < n; ++u)
        for (int64_t e = off[u]; e < off[u + 1]; ++e) {
            int64_t x = w ? w[e] : 1;
            w2[e] = (col[e] == u) ? 2 * x : x;
        }
}

/* vol[u] = row sum of the doubled-diagonal weights; returns S = sum vol. */
int64_t orc_volumes(int64_t n, const int64_t *off, const int64_t *w2, int64_t *vol) {
    int64_t S = 0;
    for (int64_t u = 0; u < n; ++u) {
        int64_t s = 0;
        for (int64_t e = off[u]; e < off[u + 1]; ++e) s += w2[e];
        vol[u] = s;
        S += s;
    }
    return S;
}

/* ------------------------------------------------------------------ colouring */
typedef struct { uint64_t h; int64_t u; } orc_key;

/* descending priority: larger hash first, equal hashes -> larger id first */
static int orc_key_cmp(const void *a, const void *b) {
    const orc_key *x = (const orc_key *)a, *y = (const orc_key *)b;
    if (x->h != y->h) return x->h > y->h ? -1 : 1;
    if (x->u != y->u) return x->u > y->u ? -1 : 1;
    return 0;
}

/* Nodes in descending priority order. */
void orc_priority_order(int64_t n, uint64_t seed, int32_t level, int32_t *order) {
    orc_key *k = (orc_key *)malloc((size_t)(n > 0 ? n : 1) * sizeof(orc_key));
    for (int64_t u = 0; u < n; ++u) { k[u].h = orc_priority(seed, level, u); k[u].u = u; }
    qsort(k, (size_t)n, sizeof(orc_key), orc_key_cmp);
    for (int64_t i = 0; i < n; ++i) order[i] = (int32_t)k[i].u;
    free(k);
}

/* schedule 0: greedy first-fit colouring in descending priority order; the
 *             colour of u is the smallest one not taken by an already coloured
 *             (that is: higher-priority) neighbour; self-loops are ignored.
 * schedule 1: one class per node, class = position in the priority order
 *             (sequential local moving).
 * Returns the number of classes. */
int64_t orc_colour(int64_t n, const int64_t *off, const int32_t *col, uint64_t seed, int32_t level,
                   int32_t schedule, int32_t *colour) {
    if (n == 0) return 0;
    int32_t *order = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    orc_priority_order(n, seed, level, order);
    if (schedule == 1) {
        for (int64_t i = 0; i < n; ++i) colour[order[i]] = (int32_t)i;
        free(order);
        return n;
    }
    int64_t maxdeg = 0;
    for (int64_t u = 0; u < n; ++u)
        if (off[u + 1] - off[u] > maxdeg) maxdeg = off[u + 1] - off[u];
    int64_t *stamp = (int64_t *)malloc((size_t)(maxdeg + 2) * sizeof(int64_t));
    for (int64_t c = 0; c < maxdeg + 2; ++c) stamp[c] = -1;
    for (int64_t u = 0; u < n; ++u) colour[u] = -1;
    int64_t ncol = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t u = order[i];
        for (int64_t e = off[u]; e < off[u + 1]; ++e) {
            int64_t v = col[e];
            if (v != u && colour[v] >= 0 && colour[v] <= maxdeg) stamp[colour[v]] = u;
        }
        int64_t c = 0;
        while (stamp[c] == u) ++c;
        colour[u] = (int32_t)c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    free(stamp);
    free(order);
    return ncol;
}

/* ------------------------------------------------------------------ move */
/* Scratch for the per-node map community -> summed weight (a dense array with
 * a list of touched keys, as the paper's per-thread vector). */
typedef struct {
    int64_t n;
    int64_t *acc;
    uint8_t *seen;
    int32_t *touched;
} orc_map;

static void orc_map_init(orc_map *m, int64_t n) {
    m->n = n;
    m->acc = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    m->seen = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    m->touched = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
}
static void orc_map_free(orc_map *m) { free(m->acc); free(m->seen); free(m->touched); }

static int orc_i32_cmp(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Best move of u: the target community, or -1 to stay.  *gain_out gets the
 * winning gain (0 when staying).  Resolution gamma = gp / gq (section III-B
 * names the parameter; gamma = 1 is plain modularity): the gain is scaled by
 * gq > 0, gq S (w(u,X) - w(u,D\u)) - gp vol(u) (vol(X) - vol(D\u)), which keeps
 * every comparison exact; callers keep S vol(u) max(gp, gq) below 2^126. */
static int32_t orc_decide_m(int64_t u, const int64_t *off, const int32_t *col, const int64_t *w2,
                            const int32_t *zeta, const int64_t *volC, const int64_t *vol, int64_t S,
                            int64_t gp, int64_t gq, orc_map *m, i128 *gain_out) {
    int64_t nt = 0;
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
        int64_t v = col[e];
        if (v == u) continue;          /* w(u, X) excludes the self-loop */
        int32_t X = zeta[v];
        if (!m->seen[X]) { m->seen[X] = 1; m->acc[X] = 0; m->touched[nt++] = X; }
        m->acc[X] += w2[e];
    }
    int32_t D = zeta[u];
    int32_t best = -1;
    i128 best_gain = 0;
    if (nt > 0) {
        qsort(m->touched, (size_t)nt, sizeof(int32_t), orc_i32_cmp);
        int64_t wD = m->seen[D] ? m->acc[D] : 0;
        int64_t base = volC[D] - vol[u];           /* vol(D \ u) */
        for (int64_t i = 0; i < nt; ++i) {
            int32_t X = m->touched[i];
            if (X == D) continue;
            i128 g = (i128)gq * (i128)S * (i128)(m->acc[X] - wD) - (i128)gp * (i128)vol[u] * (i128)(volC[X] - base);
            if (g > best_gain) { best_gain = g; best = X; }  /* ascending X: ties keep the lowest id */
        }
    }
    for (int64_t i = 0; i < nt; ++i) m->seen[m->touched[i]] = 0;
    *gain_out = best_gain;
    return best;
}

/* Single-node decision (exported for sampled checks).  gain_hi/gain_lo receive
 * the 128-bit winning gain. */
int32_t orc_decide(int64_t n, int64_t u, const int64_t *off, const int32_t *col, const int64_t *w2,
                   const int32_t *zeta, const int64_t *volC, const int64_t *vol, int64_t S, int64_t gp, int64_t gq,
                   int64_t *gain_hi, uint64_t *gain_lo) {
    orc_map m;
    orc_map_init(&m, n);
    i128 g;
    int32_t x = orc_decide_m(u, off, col, w2, zeta, volC, vol, S, gp, gq, &m, &g);
    orc_map_free(&m);
    if (gain_hi) *gain_hi = (int64_t)(g >> 64);
    if (gain_lo) *gain_lo = (uint64_t)g;
    return x;
}

/* Sampled decisions: for each listed node, its decision against (zeta, volC). */
void orc_decide_many(int64_t n, int64_t count, const int32_t *nodes, const int64_t *off, const int32_t *col,
                     const int64_t *w2, const int32_t *zeta, const int64_t *volC, const int64_t *vol, int64_t S,
                     int64_t gp, int64_t gq, int32_t *out) {
    orc_map m;
    orc_map_init(&m, n);
    for (int64_t i = 0; i < count; ++i) {
        i128 g;
        out[i] = orc_decide_m(nodes[i], off, col, w2, zeta, volC, vol, S, gp, gq, &m, &g);
    }
    orc_map_free(&m);
}

/* One class step: every node of class c decides against the volumes at the
 * start of the class, then all moves are applied.  Returns the move count.
 * `members`/`count` list the class; decisions[] is scratch of size count. */
static int64_t orc_apply_class(const int32_t *members, int64_t count, const int32_t *decisions, const int64_t *vol,
                               int32_t *zeta, int64_t *volC);

static int64_t orc_class_step_m(const int32_t *members, int64_t count, const int64_t *off, const int32_t *col,
                                const int64_t *w2, const int64_t *vol, int64_t S, int64_t gp, int64_t gq,
                                int32_t *zeta, int64_t *volC, int32_t *decisions, orc_map *m) {
    for (int64_t i = 0; i < count; ++i) {
        i128 g;
        decisions[i] = orc_decide_m(members[i], off, col, w2, zeta, volC, vol, S, gp, gq, m, &g);
    }
    return orc_apply_class(members, count, decisions, vol, zeta, volC);
}

/* The moves of a class, applied after all its decisions were taken. */
static int64_t orc_apply_class(const int32_t *members, int64_t count, const int32_t *decisions, const int64_t *vol,
                               int32_t *zeta, int64_t *volC) {
    int64_t moves = 0;
    for (int64_t i = 0; i < count; ++i) {
        int32_t X = decisions[i];
        if (X < 0) continue;
        int32_t u = members[i], D = zeta[u];
        zeta[u] = X;
        volC[D] -= vol[u];
        volC[X] += vol[u];
        ++moves;
    }
    return moves;
}

/* Class lists: members of class c are cls_nodes[cls_off[c] .. cls_off[c+1]),
 * ascending node ids.  cls_off has ncol+1 entries. */
static void orc_classes(int64_t n, const int32_t *colour, int64_t ncol, int64_t *cls_off, int32_t *cls_nodes) {
    memset(cls_off, 0, (size_t)(ncol + 1) * sizeof(int64_t));
    for (int64_t u = 0; u < n; ++u) cls_off[colour[u] + 1]++;
    for (int64_t c = 0; c < ncol; ++c) cls_off[c + 1] += cls_off[c];
    int64_t *fill = (int64_t *)malloc((size_t)(ncol + 1) * sizeof(int64_t));
    memcpy(fill, cls_off, (size_t)(ncol + 1) * sizeof(int64_t));
    for (int64_t u = 0; u < n; ++u) cls_nodes[fill[colour[u]]++] = (int32_t)u;
    free(fill);
}

/* One class step by class index (exported). */
int64_t orc_class_step(int64_t n, const int64_t *off, const int32_t *col, const int64_t *w2, const int64_t *vol,
                       int64_t S, int64_t gp, int64_t gq, const int32_t *colour, int32_t c, int32_t *zeta,
                       int64_t *volC) {
    int64_t count = 0;
    for (int64_t u = 0; u < n; ++u) count += (colour[u] == c);
    int32_t *members = (int32_t *)malloc((size_t)(count > 0 ? count : 1) * sizeof(int32_t));
    int32_t *dec = (int32_t *)malloc((size_t)(count > 0 ? count : 1) * sizeof(int32_t));
    int64_t k = 0;
    for (int64_t u = 0; u < n; ++u)
        if (colour[u] == c) members[k++] = (int32_t)u;
    orc_map m;
    orc_map_init(&m, n);
    int64_t moves = orc_class_step_m(members, count, off, col, w2, vol, S, gp, gq, zeta, volC, dec, &m);
    orc_map_free(&m);
    free(members);
    free(dec);
    return moves;
}

/* One sweep: all classes in ascending colour order.  Returns the move count. */
int64_t orc_sweep(int64_t n, const int64_t *off, const int32_t *col, const int64_t *w2, const int64_t *vol,
                  int64_t S, int64_t gp, int64_t gq, const int32_t *colour, int64_t ncol, int32_t *zeta,
                  int64_t *volC) {
    int64_t *cls_off = (int64_t *)malloc((size_t)(ncol + 1) * sizeof(int64_t));
    int32_t *cls_nodes = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *dec = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    orc_classes(n, colour, ncol, cls_off, cls_nodes);
    orc_map m;
    orc_map_init(&m, n);
    int64_t moves = 0;
    for (int64_t c = 0; c < ncol; ++c)
        moves += orc_class_step_m(cls_nodes + cls_off[c], cls_off[c + 1] - cls_off[c], off, col, w2, vol, S, gp, gq,
                                  zeta, volC, dec, &m);
    orc_map_free(&m);
    free(cls_off); free(cls_nodes); free(dec);
    return moves;
}

/* One sweep whose class decisions are spread over `threads` threads (for
 * writing stored expected values of very large graphs in reasonable time).
 * The members of a class are pairwise non-adjacent and every one of them
 * decides against the state at the class start, so the decisions do not
 * depend on each other or on the order in which they are taken; they are then
 * applied exactly as in orc_sweep.  The result equals orc_sweep's for any
 * thread count.  Returns the move count, or -1 if threads < 1. */
int64_t orc_sweep_mt(int64_t n, const int64_t *off, const int32_t *col, const int64_t *w2, const int64_t *vol,
                     int64_t S, int64_t gp, int64_t gq, const int32_t *colour, int64_t ncol, int32_t *zeta,
                     int64_t *volC, int32_t threads) {
    if (threads < 1) return -1;
    int64_t *cls_off = (int64_t *)malloc((size_t)(ncol + 1) * sizeof(int64_t));
    int32_t *cls_nodes = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *dec = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    orc_classes(n, colour, ncol, cls_off, cls_nodes);
    orc_map *maps = (orc_map *)malloc((size_t)threads * sizeof(orc_map));
    for (int32_t t = 0; t < threads; ++t) orc_map_init(&maps[t], n);
    int64_t moves = 0;
    for (int64_t c = 0; c < ncol; ++c) {
        const int32_t *mem = cls_nodes + cls_off[c];
        const int64_t count = cls_off[c + 1] - cls_off[c];
#pragma omp parallel for num_threads(threads) schedule(dynamic, 64) if (threads > 1 && count >= 1024)
        for (int64_t i = 0; i < count; ++i) {
            i128 g;
            dec[i] = orc_decide_m(mem[i], off, col, w2, zeta, volC, vol, S, gp, gq, &maps[orc_thread()], &g);
        }
        moves += orc_apply_class(mem, count, dec, vol, zeta, volC);
    }
    for (int32_t t = 0; t < threads; ++t) orc_map_free(&maps[t]);
    free(maps); free(cls_off); free(cls_nodes); free(dec);
    return moves;
}

/* ------------------------------------------------------------------ coarsen */
/* pi[u] = rank of zeta[u] among the non-empty community ids (ascending).
 * Returns the number of communities. */
int64_t orc_relabel(int64_t n, const int32_t *zeta, int32_t *pi) {
    int32_t *newid = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    for (int64_t x = 0; x < n; ++x) newid[x] = 0;
    for (int64_t u = 0; u < n; ++u) newid[zeta[u]] = 1;
    int64_t k = 0;
    for (int64_t x = 0; x < n; ++x) {
        int32_t present = newid[x];
        newid[x] = (int32_t)k;
        k += present;
    }
    for (int64_t u = 0; u < n; ++u) pi[u] = newid[zeta[u]];
    free(newid);
    return k;
}

/* Coarse graph: W'[pi(u)][pi(v)] = sum of w2 over entries (u, v).  The fine
 * graph's diagonal is doubled and every intra-community edge appears in both
 * directions, so the coarse diagonal is again doubled.  Rows ascending.
 * coff[k+1], ccol[], cw[] must hold up to nnz entries.  Returns nnz'. */
int64_t orc_contract(int64_t n, const int64_t *off, const int32_t *col, const int64_t *w2, const int32_t *pi,
                     int64_t k, int64_t *coff, int32_t *ccol, int64_t *cw) {
    /* members of each coarse node, ascending fine id */
    int64_t *moff = (int64_t *)calloc((size_t)k + 1, sizeof(int64_t));
    int32_t *mem = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    for (int64_t u = 0; u < n; ++u) moff[pi[u] + 1]++;
    for (int64_t c = 0; c < k; ++c) moff[c + 1] += moff[c];
    int64_t *fill = (int64_t *)malloc(((size_t)k + 1) * sizeof(int64_t));
    memcpy(fill, moff, ((size_t)k + 1) * sizeof(int64_t));
    for (int64_t u = 0; u < n; ++u) mem[fill[pi[u]]++] = (int32_t)u;
    free(fill);
    orc_map m;
    orc_map_init(&m, k);
    int64_t p = 0;
    coff[0] = 0;
    for (int64_t c = 0; c < k; ++c) {
        int64_t nt = 0;
        for (int64_t i = moff[c]; i < moff[c + 1]; ++i) {
            int64_t u = mem[i];
            for (int64_t e = off[u]; e < off[u + 1]; ++e) {
                int32_t t = pi[col[e]];
                if (!m.seen[t]) { m.seen[t] = 1; m.acc[t] = 0; m.touched[nt++] = t; }
                m.acc[t] += w2[e];
            }
        }
        qsort(m.touched, (size_t)nt, sizeof(int32_t), orc_i32_cmp);
        for (int64_t i = 0; i < nt; ++i) {
            int32_t t = m.touched[i];
            ccol[p] = t;
            cw[p] = m.acc[t];
            ++p;
            m.seen[t] = 0;
        }
        coff[c + 1] = p;
    }
    orc_map_free(&m);
    free(moff); free(mem);
    return p;
}

/* ------------------------------------------------------------------ modularity */
/* Equation (3.1) with integers: N = S*I2 - sum_C vol(C)^2 and D = S^2 (both
 * 128-bit), Q = (double)N / (double)D.  labels in [0, n). */
double orc_modularity(int64_t n, const int64_t *off, const int32_t *col, const int64_t *w2, const int32_t *labels,
                      int64_t *num_hi, uint64_t *num_lo, int64_t *den_hi, uint64_t *den_lo) {
    int64_t *vC = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    int64_t S = 0, I2 = 0;
    for (int64_t u = 0; u < n; ++u)
        for (int64_t e = off[u]; e < off[u + 1]; ++e) {
            S += w2[e];
            vC[labels[u]] += w2[e];
            if (labels[col[e]] == labels[u]) I2 += w2[e];
        }
    i128 sq = 0;
    for (int64_t x = 0; x < n; ++x) sq += (i128)vC[x] * (i128)vC[x];
    free(vC);
    i128 N = (i128)S * (i128)I2 - sq, D = (i128)S * (i128)S;
    if (num_hi) *num_hi = (int64_t)(N >> 64);
    if (num_lo) *num_lo = (uint64_t)N;
    if (den_hi) *den_hi = (int64_t)(D >> 64);
    if (den_lo) *den_lo = (uint64_t)D;
    if (S == 0) return 0.0;
    return (double)N / (double)D;
}

/* ------------------------------------------------------------------ full run */
typedef struct {
    int32_t max_sweeps;   /* per level, >= 1 */
    int32_t max_levels;   /* 0 = unlimited */
    int32_t schedule;     /* 0 colour classes, 1 sequential */
    int32_t refine;       /* 1: PLMR (Algorithm 4), a move phase after every prolongation */
    uint64_t seed;
    int64_t gamma_num;    /* resolution gamma = gamma_num / gamma_den (0/0 = 1) */
    int64_t gamma_den;
} orc_options;

#define ORC_MAX_LEVELS 64
#define ORC_MAX_SWEEPS 64
typedef struct {
    int32_t levels;
    int32_t pad;
    int64_t n[ORC_MAX_LEVELS], nnz[ORC_MAX_LEVELS], colours[ORC_MAX_LEVELS], sweeps[ORC_MAX_LEVELS];
    int64_t communities[ORC_MAX_LEVELS];
    int64_t moves[ORC_MAX_LEVELS][ORC_MAX_SWEEPS];
    int64_t ref_sweeps[ORC_MAX_LEVELS];   /* refinement (PLMR): sweeps of the move after prolongation */
    int64_t ref_moves[ORC_MAX_LEVELS];    /* and the nodes moved by it */
    int64_t S;
} orc_trace;

/* Canonical labels: renumber by first occurrence in node order. */
void orc_canonical(int64_t n, const int32_t *lab, int32_t *out) {
    int32_t *map = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    for (int64_t x = 0; x < n; ++x) map[x] = -1;
    int32_t next = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (map[lab[v]] < 0) map[lab[v]] = next++;
        out[v] = map[lab[v]];
    }
    free(map);
}

/* Algorithm 3 under the colour-class schedule.  w: input weights (self-loops
 * given once) or NULL for unit weights.  labels[n] receives canonical labels.
 * Returns 0 on success, -1 on bad options or allocation failure. */
/* PLMR, Algorithm 4, on the graph (n, off, col, w2) (doubled diagonal) at the
 * given level: move from singletons; if communities merged (and the level cap
 * allows), coarsen, recurse, prolong the coarse result (the community of u is
 * that of its coarse node, named by its coarse id) and move again from it.
 * Leaves the communities in zeta_out[n]; returns the number of levels below
 * and including this one. */
static int32_t orc_plmr(int64_t n, const int64_t *off, const int32_t *col, const int64_t *w2, int32_t level,
                        int32_t first, const orc_options *opt, int32_t *zeta_out, orc_trace *tr) {
    const int32_t t = level - first;   /* trace slot and level count relative to the first level */
    int64_t nnz = off[n];
    int64_t *vol = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *volC = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int32_t *colour = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t S = orc_volumes(n, off, w2, vol);
    int64_t ncol = orc_colour(n, off, col, opt->seed, level, opt->schedule, colour);
    /* move from singletons */
    for (int64_t u = 0; u < n; ++u) { zeta_out[u] = (int32_t)u; volC[u] = vol[u]; }
    int64_t sweeps = 0;
    if (t < ORC_MAX_LEVELS) { tr->n[t] = n; tr->nnz[t] = nnz; tr->colours[t] = ncol; }
    for (int32_t s = 0; s < opt->max_sweeps; ++s) {
        int64_t mv = orc_sweep(n, off, col, w2, vol, S, opt->gamma_num, opt->gamma_den, colour, ncol, zeta_out,
                               volC);
        if (t < ORC_MAX_LEVELS) tr->moves[t][s] = mv;
        ++sweeps;
        if (mv == 0) break;
    }
    int32_t *pi = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t k = orc_relabel(n, zeta_out, pi);
    if (t < ORC_MAX_LEVELS) { tr->sweeps[t] = sweeps; tr->communities[t] = k; }
    int32_t depth = 1;
    if (k < n && !(opt->max_levels > 0 && t + 1 >= opt->max_levels)) {
        /* coarsen, recurse, prolong */
        int64_t *coff = (int64_t *)malloc(((size_t)k + 1) * sizeof(int64_t));
        int32_t *ccol = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
        int64_t *cw = (int64_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int64_t));
        orc_contract(n, off, col, w2, pi, k, coff, ccol, cw);
        int32_t *zc = (int32_t *)malloc((size_t)(k > 0 ? k : 1) * sizeof(int32_t));
        depth += orc_plmr(k, coff, ccol, cw, level + 1, first, opt, zc, tr);
        for (int64_t u = 0; u < n; ++u) zeta_out[u] = zc[pi[u]];
        free(zc); free(coff); free(ccol); free(cw);
        /* move again, from the prolonged communities */
        for (int64_t u = 0; u < n; ++u) volC[u] = 0;
        for (int64_t u = 0; u < n; ++u) volC[zeta_out[u]] += vol[u];
        int64_t rs = 0, rm = 0;
        for (int32_t s = 0; s < opt->max_sweeps; ++s) {
            int64_t mv = orc_sweep(n, off, col, w2, vol, S, opt->gamma_num, opt->gamma_den, colour, ncol, zeta_out,
                                   volC);
            ++rs;
            rm += mv;
            if (mv == 0) break;
        }
        if (t < ORC_MAX_LEVELS) { tr->ref_sweeps[t] = rs; tr->ref_moves[t] = rm; }
    }
    free(pi); free(vol); free(volC); free(colour);
    return depth;
}

int orc_run(int64_t n, const int64_t *off, const int32_t *col, const int64_t *w, const orc_options *opt_in,
            int32_t *labels, double *q_out, orc_trace *tr) {
    if (opt_in->max_sweeps < 1 || opt_in->max_sweeps > ORC_MAX_SWEEPS) return -1;
    /* resolution: 0/0 means 1; 0 <= gamma_num, 1 <= gamma_den, both below 2^16 */
    orc_options o = *opt_in;
    const orc_options *opt = &o;
    if (o.gamma_num == 0 && o.gamma_den == 0) o.gamma_num = o.gamma_den = 1;
    if (o.gamma_num < 0 || o.gamma_den < 1 || o.gamma_num >= 65536 || o.gamma_den >= 65536) return -1;
    memset(tr, 0, sizeof(*tr));
    int64_t nnz = off[n];
    int64_t *w2_0 = (int64_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int64_t));
    orc_double_diagonal(n, off, col, w, w2_0);
    if (o.gamma_num != o.gamma_den) {
        /* every gain stays below 2^126: S^2 max(gamma_num, gamma_den) < 2^126 */
        int64_t S0 = 0;
        for (int64_t e = 0; e < nnz; ++e) S0 += w2_0[e];
        unsigned __int128 b = (unsigned __int128)S0 * (unsigned __int128)S0 *
                              (unsigned __int128)(o.gamma_num > o.gamma_den ? o.gamma_num : o.gamma_den);
        if (b >> 126) { free(w2_0); return -1; }
    }
    if (opt->refine) {
        int32_t *zeta = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
        tr->levels = orc_plmr(n, off, col, w2_0, 0, 0, opt, zeta, tr);
        tr->S = 0;
        for (int64_t e = 0; e < nnz; ++e) tr->S += w2_0[e];
        orc_canonical(n, zeta, labels);
        *q_out = orc_modularity(n, off, col, w2_0, labels, NULL, NULL, NULL, NULL);
        free(zeta); free(w2_0);
        return 0;
    }
    /* current level graph (level 0 aliases the input) */
    int64_t ln = n, lnnz = nnz;
    const int64_t *loff = off;
    const int32_t *lcol = col;
    const int64_t *lw = w2_0;
    int64_t *own_off = NULL; int32_t *own_col = NULL; int64_t *own_w = NULL;
    int32_t *lab = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    for (int64_t v = 0; v < n; ++v) lab[v] = (int32_t)v;   /* fine node -> current level node */
    int64_t S = 0;
    int32_t level = 0;
    for (;;) {
        int64_t *vol = (int64_t *)malloc((size_t)(ln > 0 ? ln : 1) * sizeof(int64_t));
        int64_t *volC = (int64_t *)malloc((size_t)(ln > 0 ? ln : 1) * sizeof(int64_t));
        int32_t *zeta = (int32_t *)malloc((size_t)(ln > 0 ? ln : 1) * sizeof(int32_t));
        int32_t *colour = (int32_t *)malloc((size_t)(ln > 0 ? ln : 1) * sizeof(int32_t));
        S = orc_volumes(ln, loff, lw, vol);
        for (int64_t u = 0; u < ln; ++u) { zeta[u] = (int32_t)u; volC[u] = vol[u]; }
        int64_t ncol = orc_colour(ln, loff, lcol, opt->seed, level, opt->schedule, colour);
        int64_t sweeps = 0;
        if (level < ORC_MAX_LEVELS) { tr->n[level] = ln; tr->nnz[level] = lnnz; tr->colours[level] = ncol; }
        for (int32_t s = 0; s < opt->max_sweeps; ++s) {
            int64_t mv = orc_sweep(ln, loff, lcol, lw, vol, S, opt->gamma_num, opt->gamma_den, colour, ncol, zeta,
                                   volC);
            if (level < ORC_MAX_LEVELS) tr->moves[level][s] = mv;
            ++sweeps;
            if (mv == 0) break;
        }
        int32_t *pi = (int32_t *)malloc((size_t)(ln > 0 ? ln : 1) * sizeof(int32_t));
        int64_t k = orc_relabel(ln, zeta, pi);
        if (level < ORC_MAX_LEVELS) { tr->sweeps[level] = sweeps; tr->communities[level] = k; }
        ++level;
        int stop = (k == ln) || (opt->max_levels > 0 && level >= opt->max_levels);
        if (stop) {
            for (int64_t v = 0; v < n; ++v) lab[v] = zeta[lab[v]];
            free(pi); free(vol); free(volC); free(zeta); free(colour);
            break;
        }
        /* coarsen and descend: fine node -> coarse node */
        int64_t *coff = (int64_t *)malloc(((size_t)k + 1) * sizeof(int64_t));
        int32_t *ccol = (int32_t *)malloc((size_t)(lnnz > 0 ? lnnz : 1) * sizeof(int32_t));
        int64_t *cw = (int64_t *)malloc((size_t)(lnnz > 0 ? lnnz : 1) * sizeof(int64_t));
        int64_t cnnz = orc_contract(ln, loff, lcol, lw, pi, k, coff, ccol, cw);
        for (int64_t v = 0; v < n; ++v) lab[v] = pi[lab[v]];
        free(own_off); free(own_col); free(own_w);
        own_off = coff; own_col = ccol; own_w = cw;
        loff = coff; lcol = ccol; lw = cw; ln = k; lnnz = cnnz;
        free(pi); free(vol); free(volC); free(zeta); free(colour);
    }
    tr->levels = level;
    tr->S = S;
    orc_canonical(n, lab, labels);
    *q_out = orc_modularity(n, off, col, w2_0, labels, NULL, NULL, NULL, NULL);
    free(lab); free(w2_0);
    free(own_off); free(own_col); free(own_w);
    return 0;
}

/* ------------------------------------------------------------------ PLP (Algorithm 1)
 * Label propagation with the deterministic schedule of this library: the
 * colour classes of the level (ascending), each class deciding against the
 * labels at its start and then applying (classes are independent sets).  A node
 * is visited while active (Algorithm 1: it turns inactive when it keeps its
 * label, and active again when a neighbour changes label).  The dominant label
 * of v maximises the weight sum of its non-loop neighbours carrying it; v keeps
 * its label when that label attains the maximum, else takes, among the labels
 * l that do, the one with the largest tie key t(v, l) = upper 32 bits of
 * SplitMix64(H(seed, level, v) ^ l), then the lowest label.  The paper breaks
 * ties arbitrarily; a key drawn per (node, label) stands in for an independent
 * random choice at every node (a fixed order of labels would let one label win
 * every tie and flood the graph).  Iterations (passes over all classes) continue while the number
 * of updated nodes exceeds theta = n * 10^-5, at most max_iters times.
 * zeta[n] receives the labels (node ids); returns the number of iterations. */
static int32_t orc_dominant_label(int64_t v, const int64_t *off, const int32_t *col, const int64_t *w2,
                                  const int32_t *zeta, uint64_t seed, int32_t level, orc_map *m) {
    int64_t nt = 0;
    for (int64_t e = off[v]; e < off[v + 1]; ++e) {
        int64_t u = col[e];
        if (u == v) continue;
        int32_t l = zeta[u];
        if (!m->seen[l]) { m->seen[l] = 1; m->acc[l] = 0; m->touched[nt++] = l; }
        m->acc[l] += w2[e];
    }
    const int32_t own = zeta[v];
    const int64_t wown = m->seen[own] ? m->acc[own] : 0;
    const uint64_t hv = orc_priority(seed, level, v);   /* tie keys differ from node to node */
    int32_t best = -1;
    int64_t bw = 0;
    uint32_t bt = 0;
    if (nt > 0) {
        qsort(m->touched, (size_t)nt, sizeof(int32_t), orc_i32_cmp);
        for (int64_t i = 0; i < nt; ++i) {        /* ascending labels: strict comparisons keep the lowest */
            int32_t l = m->touched[i];
            if (l == own) continue;
            uint32_t t = (uint32_t)(orc_splitmix64(hv ^ (uint64_t)(uint32_t)l) >> 32);
            if (best < 0 || m->acc[l] > bw || (m->acc[l] == bw && t > bt)) { best = l; bw = m->acc[l]; bt = t; }
        }
    }
    for (int64_t i = 0; i < nt; ++i) m->seen[m->touched[i]] = 0;
    return (best >= 0 && bw > wown) ? best : own;
}

int32_t orc_plp(int64_t n, const int64_t *off, const int32_t *col, const int64_t *w2, uint64_t seed, int32_t level,
                int32_t max_iters, int32_t *zeta, int64_t *updates_out) {
    int32_t *colour = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t ncol = orc_colour(n, off, col, seed, level, 0, colour);
    int64_t *cls_off = (int64_t *)malloc((size_t)(ncol + 1) * sizeof(int64_t));
    int32_t *cls_nodes = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *dec = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    uint8_t *active = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    orc_classes(n, colour, ncol, cls_off, cls_nodes);
    orc_map m;
    orc_map_init(&m, n);
    for (int64_t v = 0; v < n; ++v) {
        zeta[v] = (int32_t)v;
        int deg = 0;   /* degree without the self-loop */
        for (int64_t e = off[v]; e < off[v + 1]; ++e) deg += (col[e] != v);
        active[v] = deg > 0;
    }
    int64_t updated = n;
    int32_t it = 0;
    while (updated * 100000 > n && it < max_iters) {    /* updated > theta = n * 10^-5 */
        updated = 0;
        for (int64_t c = 0; c < ncol; ++c) {
            const int32_t *mem = cls_nodes + cls_off[c];
            int64_t cnt = cls_off[c + 1] - cls_off[c];
            for (int64_t i = 0; i < cnt; ++i)
                dec[i] = active[mem[i]] ? orc_dominant_label(mem[i], off, col, w2, zeta, seed, level, &m)
                                        : zeta[mem[i]];
            for (int64_t i = 0; i < cnt; ++i) {
                int32_t v = mem[i];
                if (!active[v]) continue;
                if (dec[i] != zeta[v]) {
                    zeta[v] = dec[i];
                    ++updated;
                    for (int64_t e = off[v]; e < off[v + 1]; ++e)
                        if (col[e] != v) active[col[e]] = 1;
                } else {
                    active[v] = 0;
                }
            }
        }
        if (updates_out && it < ORC_MAX_SWEEPS) updates_out[it] = updated;
        ++it;
    }
    orc_map_free(&m);
    free(colour); free(cls_off); free(cls_nodes); free(dec); free(active);
    return it;
}

/* PLP from the input CSR: canonical labels, modularity, iterations. */
int orc_plp_run(int64_t n, const int64_t *off, const int32_t *col, const int64_t *w, uint64_t seed, int32_t max_iters,
                int32_t *labels, double *q_out, int64_t *updates_out, int32_t *iters_out) {
    if (max_iters < 1 || max_iters > ORC_MAX_SWEEPS) return -1;
    int64_t nnz = off[n];
    int64_t *w2 = (int64_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int64_t));
    int32_t *zeta = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    orc_double_diagonal(n, off, col, w, w2);
    *iters_out = orc_plp(n, off, col, w2, seed, 0, max_iters, zeta, updates_out);
    orc_canonical(n, zeta, labels);
    *q_out = orc_modularity(n, off, col, w2, labels, NULL, NULL, NULL, NULL);
    free(w2); free(zeta);
    return 0;
}

/* ------------------------------------------------------------------ EPP (Algorithm 5)
 * EPP(b, PLP, PLMR): b PLP runs (colour seeds seed .. seed+b-1), core groups by
 * Equation (3.2) (same group iff every base solution agrees; exact tuple
 * comparison instead of a hash), coarsening by the core groups (coarse ids
 * ascending with the smallest member), PLMR on the coarse graph as level 1, and
 * prolongation.  Canonical labels and the modularity on the input graph. */
static const int32_t *orc_epp_base;   /* b base solutions, row-major [b][n], for the tuple sort */
static int64_t orc_epp_b, orc_epp_n;
static int orc_tuple_cmp(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    for (int64_t i = 0; i < orc_epp_b; ++i) {
        int32_t lx = orc_epp_base[i * orc_epp_n + x], ly = orc_epp_base[i * orc_epp_n + y];
        if (lx != ly) return lx < ly ? -1 : 1;
    }
    return x < y ? -1 : (x > y);
}

int orc_epp(int64_t n, const int64_t *off, const int32_t *col, const int64_t *w, int32_t b, int32_t plp_iters,
            const orc_options *opt, int32_t *labels, double *q_out, int64_t *cores_out, int32_t *core_groups,
            orc_trace *tr) {
    if (b < 1 || plp_iters < 1 || plp_iters > ORC_MAX_SWEEPS || opt->max_sweeps < 1 ||
        opt->max_sweeps > ORC_MAX_SWEEPS)
        return -1;
    memset(tr, 0, sizeof(*tr));
    orc_options o = *opt;
    if (o.gamma_num == 0 && o.gamma_den == 0) o.gamma_num = o.gamma_den = 1;
    o.refine = 1;
    int64_t nnz = off[n];
    int64_t *w2 = (int64_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int64_t));
    orc_double_diagonal(n, off, col, w, w2);
    int32_t *base = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * (size_t)b * sizeof(int32_t));
    for (int32_t i = 0; i < b; ++i)
        orc_plp(n, off, col, w2, o.seed + (uint64_t)i, 0, plp_iters, base + (size_t)i * (size_t)n, NULL);
    /* core groups: nodes sorted by their tuple of base labels; a group's id is its smallest member */
    int32_t *ord = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *core = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    for (int64_t v = 0; v < n; ++v) ord[v] = (int32_t)v;
    orc_epp_base = base; orc_epp_b = b; orc_epp_n = n;
    qsort(ord, (size_t)n, sizeof(int32_t), orc_tuple_cmp);
    for (int64_t i = 0; i < n;) {
        int64_t j = i;
        while (j < n) {
            int same = 1;
            for (int32_t t = 0; t < b && same; ++t)
                same = base[(size_t)t * n + ord[j]] == base[(size_t)t * n + ord[i]];
            if (!same) break;
            ++j;
        }
        for (int64_t k = i; k < j; ++k) core[ord[k]] = ord[i];   /* smallest member: the sort breaks ties by id */
        i = j;
    }
    int32_t *pi = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t k = orc_relabel(n, core, pi);
    *cores_out = k;
    if (core_groups) memcpy(core_groups, pi, (size_t)n * sizeof(int32_t));   /* coarse node of each node */
    int64_t *coff = (int64_t *)malloc(((size_t)k + 1) * sizeof(int64_t));
    int32_t *ccol = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    int64_t *cw = (int64_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int64_t));
    orc_contract(n, off, col, w2, pi, k, coff, ccol, cw);
    int32_t *zc = (int32_t *)malloc((size_t)(k > 0 ? k : 1) * sizeof(int32_t));
    tr->levels = orc_plmr(k, coff, ccol, cw, 1, 1, &o, zc, tr);
    int32_t *zeta = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    for (int64_t v = 0; v < n; ++v) zeta[v] = zc[pi[v]];
    orc_canonical(n, zeta, labels);
    *q_out = orc_modularity(n, off, col, w2, labels, NULL, NULL, NULL, NULL);
    free(w2); free(base); free(ord); free(core); free(pi); free(coff); free(ccol); free(cw); free(zc); free(zeta);
    return 0;
}
