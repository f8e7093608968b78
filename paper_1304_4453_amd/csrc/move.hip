// move.hip - the move-decide and apply kernels of one colour class
// (Algorithm 2 under the colour-class schedule).
//
// For node u in community D every neighbouring community X != D is scored by
//   gain(X) = S (w(u,X) - w(u,D\u)) - vol(u) (vol(X) - vol(D\u))
// (2 w(E)^2 times Delta-mod of section III-B).  The kernels rank candidates by
//   s(X) = S w(u,X) - vol(u) vol(X)
// which differs from gain(X) by the constant K = S w(u,D\u) - vol(u) vol(D\u),
// so the best candidate is the same and the move happens iff s_best > K.
// With a resolution gamma = p / q every S is scaled by q and every vol(u)
// multiplier by p (q times the gamma gain: same ranking, exact).
// |s|, |K| <= S vol(u) max(p, q): 64-bit arithmetic is exact below 2^62,
// otherwise the node takes the 128-bit path.  Ties go to the lowest X.
//
// Degree bins: rows up to 16 entries are handled one lane per node (register
// arrays), up to the wave limit one wavefront per node (LDS hash table; rows
// of at most kQuadRow entries 16 lanes per node), up to the block limit one
// workgroup per node (LDS hash table; 256 threads for rows of at most
// kBlockShortRow entries, 512 above), and longer rows
// ("hubs") by one 1024-thread workgroup with a 16384-slot LDS table when the
// row has at most kSingleMaxRow entries, else by several workgroups per node
// through hash-partitioned staging.  The LDS tables sum weights in 32 bits:
// the bucketing sends a node whose vol(u) (an upper bound of every w(u, X))
// does not fit to the partitioned hub path, whose sums are 64-bit.
//
// The same kernels (template flag LP) run label propagation (Algorithm 1):
// with S = 2^32, a zero vol(u) multiplier and K raised by 2^32 - 1, a label X
// scores (w(u,X) << 32) + t(u,X) against K = (w(u,D) << 32) + 2^32 - 1, so the
// best label has the largest weight, then the largest tie key t, then the
// lowest id, and u keeps its label iff that label's weight is the maximum.
// No community volumes are read.  w(u,X) <= vol(u) < 2^31 keeps the scores in
// 64 bits (wide_lim = 2^31 - 1 sends larger nodes to the 128-bit path).  Only
// active nodes are decided; a node that keeps its label turns inactive and a
// node that takes a new one activates its neighbours (neighbours are never in
// the same class, so this cannot disturb the class's own decisions).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "level.h"

namespace plm {

typedef __int128 i128;
constexpr int32_t kNone = 0x7fffffff;

__device__ __forceinline__ uint32_t slot_hash(int32_t x, int bits) {
    return ((uint32_t)x * 2654435769u) >> (32 - bits);
}

template <typename G>
__device__ __forceinline__ G neg_inf();
template <>
__device__ __forceinline__ int64_t neg_inf<int64_t>() { return INT64_MIN; }
template <>
__device__ __forceinline__ i128 neg_inf<i128>() { return -(((i128)1) << 126); }

template <typename G>
__device__ __forceinline__ G shfl_xor_g(G x, int d);
template <>
__device__ __forceinline__ int64_t shfl_xor_g<int64_t>(int64_t x, int d) { return __shfl_xor(x, d); }
template <>
__device__ __forceinline__ i128 shfl_xor_g<i128>(i128 x, int d) {
    int64_t hi = (int64_t)(x >> 64);
    uint64_t lo = (uint64_t)x;
    hi = __shfl_xor(hi, d);
    lo = __shfl_xor(lo, d);
    return (i128)(((unsigned __int128)(uint64_t)hi << 64) | lo);
}

// (s desc, X asc) argmax over the wavefront
template <typename G>
__device__ __forceinline__ void wave_argmax(G &s, int32_t &x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        G os = shfl_xor_g<G>(s, d);
        int32_t ox = __shfl_xor(x, d);
        if (os > s || (os == s && ox < x)) { s = os; x = ox; }
    }
}

__device__ __forceinline__ int64_t wave_sum(int64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

template <typename G>
__device__ __forceinline__ G wave_max(G x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        G o = shfl_xor_g<G>(x, d);
        if (o > x) x = o;
    }
    return x;
}

// ------------------------------------------------------------------ settled nodes
// Node u (community D) scores each candidate X by the gain
//   q S (w(u,X) - w(u,D\u)) - p vol(u) (vol(X) - vol(D\u)).
// Say u last stayed at clock t0 with every gain at most -slack, and with the
// score of staying K = q S w(u,D\u) - p vol(u) vol(D\u).  Since then:
//  - community volumes changed by at most V in total, V summing 2 vol(m)
//    over the moves m applied meanwhile (the moved-volume clock);
//  - neighbours of u of total edge weight dw moved (u itself did not), which
//    changed w(u,X) - w(u,D\u) by at most 2 dw for any X, and can have made
//    new communities candidates, whose score q S w(u,X) - p vol(u) vol(X) is
//    at most q S dw.
// So every gain of an old candidate is now at most -slack + 2 q S dw + p vol(u) V,
// and that of a new one at most -K + 2 q S dw + p vol(u) V.  When these bounds
// are <= 0, u stays without a scan of its row: exactly the decision a full
// scan would take.  kslack = min(slack, K) (-1 when K < 0) covers both cases.
constexpr uint64_t kStaleDw = 1ULL << 63;  // dw at or above: must be decided
struct Settle {
    bool on;
    uint64_t now;  // the moved-volume clock at the start of the class step
};
__device__ __forceinline__ Settle settle_state(const MoveState &ms) {
    Settle st{false, 0};
    if (ms.sctl) {  // the arming word and the clock share a line: one load
        const uint64_t a = ms.sctl[0], now = ms.sctl[1];
        st.on = a != 0;
        st.now = now;
    }
    return st;
}
// Every word the test reads is loaded up front and the test is evaluated
// without branches: the loads are then in flight together instead of each
// waiting for the branch on the one before (the test sits at the head of every
// decide kernel's chain of dependent loads).
__device__ __forceinline__ bool settled(const MoveState &ms, const Settle &st, int32_t u) {
    if (!st.on) return false;
    const uint64_t dw = ms.dw[u];
    const int64_t sl = ms.slack[u], ks = ms.kslack[u];
    const uint64_t ts = ms.tstamp[u];
    const uint64_t vu = (uint64_t)ms.vol[u];
    const uint64_t su = (uint64_t)node_S(ms, u);
    const int64_t room = dw == 0 ? sl : ks;
    bool ok = dw < kStaleDw && room >= 0;
    // p vol(u) V <= room (< 2^63), then 2 q S dw <= what is left; products
    // only (room < 2^63 bounds every factor that can pass)
    uint64_t rem = ok ? (uint64_t)room : 0;
    if (ms.gp > 0) {
        const unsigned __int128 vv = (unsigned __int128)vu * (st.now - ts);
        const unsigned __int128 need = (unsigned __int128)(uint64_t)ms.gp * (uint64_t)vv;
        ok = ok && !(vv >> 63) && need <= rem;
        rem = ok ? rem - (uint64_t)need : 0;
    }
    const unsigned __int128 per = (unsigned __int128)2u * (uint64_t)ms.gq * su;
    return ok && (dw == 0 || (!(per >> 63) && (unsigned __int128)dw * (uint64_t)per <= rem));
}
__device__ __forceinline__ void record_stay(const MoveState &ms, const Settle &st, int32_t u, int64_t slack,
                                            int64_t kslack) {
    ms.dw[u] = 0;
    ms.slack[u] = slack;
    ms.kslack[u] = kslack;
    ms.tstamp[u] = st.now;
}
template <typename G>
__device__ __forceinline__ int64_t clamp_i64(G x) {
    return x <= 0 ? 0 : (x >= (G)INT64_MAX ? INT64_MAX : (int64_t)x);
}
// slack = K - ub as int64, where ub bounds every candidate's score from above
// (neg_inf: no candidate), clamped to [0, INT64_MAX] (a lower bound of the
// true slack); kslack = min(slack, K), or -1 when K < 0
template <typename G>
__device__ __forceinline__ void slack_of(G K, G ub, int64_t &slack, int64_t &kslack) {
    slack = ub == neg_inf<G>() ? INT64_MAX : clamp_i64<G>(K - ub);
    kslack = K < 0 ? -1 : (clamp_i64<G>(K) < slack ? clamp_i64<G>(K) : slack);
}
// The same from the best evaluated score bs and the largest weight maxpa of a
// pruned candidate (-1: none), whose score is at most S maxpa: the bound ub is
// max(bs, S maxpa)
template <typename G>
__device__ __forceinline__ void slack_from(G K, G S, G bs, int64_t maxpa, int64_t &slack, int64_t &kslack) {
    G ub = bs;
    if (maxpa >= 0 && (G)S * (G)maxpa > ub) ub = (G)S * (G)maxpa;
    slack_of<G>(K, ub, slack, kslack);
}
// In the per-node kernels the 128-bit gains (vol(u) S >= 2^62, rare) record
// the lower bound 0 as slack, which keeps those kernels within their register
// budget: such a node is settled only while nothing moved at all.
template <typename G>
__device__ __forceinline__ void slack_lean(G K, G S, G bs, int64_t maxpa, int64_t &slack, int64_t &kslack) {
    if constexpr (sizeof(G) > 8) {
        slack = 0;
        kslack = K < 0 ? -1 : 0;
    } else {
        slack_from<G>(K, S, bs, maxpa, slack, kslack);
    }
}
__device__ __forceinline__ int64_t wave_max_i64(int64_t x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        int64_t o = __shfl_xor(x, d);
        if (o > x) x = o;
    }
    return x;
}

// tie key of label x for the node with priority hash hv: upper half of
// SplitMix64(hv ^ x), so that each node breaks ties in its own random order
__device__ __forceinline__ uint32_t lp_tie(uint64_t hv, int32_t x) {
    return (uint32_t)(splitmix64(hv ^ (uint64_t)(uint32_t)x) >> 32);
}

// The arrays the per-entry community gathers of a sweep go through: the
// level's sweep layout when it has one (see MoveState), else the graph's own
// ids.  Community indices of the layout are turned back into original ids
// (orig_id) wherever candidates are compared or reported.
struct GatherIds {
    const int32_t *col;   // neighbour index of each entry
    const int32_t *zeta;  // community index of each neighbour index
    const int64_t *volC;  // volume of each community index
    const int32_t *ord;   // original id of a community index (null: the index itself)
};
__device__ __forceinline__ GatherIds gather_ids(const GraphView &g, const MoveState &ms) {
    return ms.colp ? GatherIds{ms.colp, ms.zetap, ms.volCp, ms.ord} : GatherIds{g.col, ms.zeta, ms.volC, nullptr};
}
__device__ __forceinline__ int32_t orig_id(const int32_t *ord, int32_t x) { return ord ? ord[x] : x; }
constexpr uint32_t kLpTieMax = 0xFFFFFFFFu;

// label propagation: u moved, so its non-loop neighbours become active
__device__ __forceinline__ void lp_activate(const GraphView &g, uint8_t *active, int32_t u, int64_t e0, int64_t e1,
                                            int64_t first, int64_t step) {
    for (int64_t e = e0 + first; e < e1; e += step) {
        int32_t v = g.col[e];
        if (v != u) active[v] = 1;
    }
}

// settled nodes: u decided to move, so u must be decided again and each
// neighbour v gains w(u,v) of moved weight; threads first, first + step, ...
// of the row.  Neighbours are never in u's class, so no decision of the class
// reads these words.
template <int WK>
__device__ __forceinline__ void mark_moved(const GraphView &g, const MoveState &ms, int32_t u, int64_t e0, int64_t e1,
                                           int64_t first, int64_t step) {
    for (int64_t e = e0 + first; e < e1; e += step) {
        const int32_t v = g.col[e];
        if (v != u) atomicAdd((unsigned long long *)&ms.dw[v], (unsigned long long)wload<WK>(g.w, e));
    }
    if (first == 0) ms.dw[u] = kStaleDw;
}

__device__ __forceinline__ void count_candidates(unsigned long long *cand, int64_t c) {
    if (!cand) return;
    c = wave_sum(c);
    if (lane_id() == 0 && c) atomicAdd(cand, (unsigned long long)c);
}
// nodes decided (scanned) and their entries, into dec[i] and dec[i + 4 or 1]
__device__ __forceinline__ void count_decided(unsigned long long *dec, int i, int j, int64_t nodes, int64_t entries) {
    if (!dec) return;
    nodes = wave_sum(nodes);
    entries = wave_sum(entries);
    if (lane_id() == 0) {
        if (nodes) atomicAdd(dec + i, (unsigned long long)nodes);
        if (entries) atomicAdd(dec + j, (unsigned long long)entries);
    }
}

// ------------------------------------------------------------------ lane per node
constexpr int kLaneMax = 16;

// *slack: when u stays, a lower bound of minus its best gain (see slack_of)
template <int WK, bool LP, typename G>
__device__ __forceinline__ int32_t lane_pick(const int32_t (&X)[kLaneMax], const int64_t (&W)[kLaneMax], int32_t D,
                                             int64_t wD, G vu, int64_t base, G S, const int64_t *volC,
                                             const int32_t *ord, uint64_t hv, int64_t *slack, int64_t *kslack) {
    G bg = 0, mg = neg_inf<G>();
    int32_t bx = kNone;
    const G vb = (G)vu * (G)base;
#pragma unroll
    for (int j = 0; j < kLaneMax; ++j) {
        // vol(X) >= 0 bounds the gain by S (w(u,X) - w(u,D\u)) + vol(u) vol(D\u):
        // a candidate that cannot reach a positive gain is not gathered
        if (X[j] >= 0 && X[j] != D) {
            const G bound = (G)S * (G)(W[j] - wD) + vb;
            if (bound > 0) {
                const int32_t ox = orig_id(ord, X[j]);
                G g;
                if constexpr (LP)
                    g = (G)S * (G)(W[j] - wD) + (G)lp_tie(hv, ox) - (G)kLpTieMax;
                else
                    g = (G)S * (G)(W[j] - wD) - (G)vu * (G)(volC[X[j]] - base);
                if (g > mg) mg = g;
                if (g > 0 && (g > bg || (g == bg && ox < bx))) { bg = g; bx = ox; }
            } else if (bound > mg) {
                mg = bound;
            }
        }
    }
    // gains here are scores minus K = S w(u,D\u) - vol(u) vol(D\u)
    const G K = (G)S * (G)wD - vb;
    slack_of<G>(K, mg == neg_inf<G>() ? mg : mg + K, *slack, *kslack);
    return bx;
}

// (at most 128 VGPRs, four waves per SIMD, no spills: left alone the compiler
// hoists the loads of the unrolled row and takes ~250, one wave per SIMD)
template <int WK, bool LP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_decide_lane(GraphView g, MoveState ms,
                                                                                           int64_t begin, int64_t count,
                                                                                           int force_wide) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t ncand = 0, nd = 0, ne = 0;
    int32_t u = 0;
    const Settle st = LP ? Settle{false, 0} : settle_state(ms);
    int64_t e0 = 0, d = 0;
    int32_t su = 0;
    const GatherIds gi = gather_ids(g, ms);
    if (i < count) {
        const NodeRec r = ms.rec[(int64_t)begin + i];
        u = r.u;
        su = r.s;
        e0 = r.e0;
        d = r.len;
        if ((LP && !ms.active[u]) || settled(ms, st, u)) {
            ms.move_to[begin + i] = -1;
            i = count;  // inactive or settled: nothing to decide
        }
    }
    if (i < count) {
        int64_t pos = begin + i;
        int32_t X[kLaneMax];
        int64_t W[kLaneMax];
#pragma unroll
        for (int j = 0; j < kLaneMax; ++j) {
            X[j] = -1;
            W[j] = 0;
            if (j < d) {
                int32_t v = gi.col[e0 + j];
                if (v != su) {
                    X[j] = gi.zeta[v];
                    W[j] = wload<WK>(g.w, e0 + j);
                }
            }
        }
        // merge equal communities into their first occurrence
#pragma unroll
        for (int a = 0; a < kLaneMax; ++a)
#pragma unroll
            for (int b = a + 1; b < kLaneMax; ++b)
                if (X[b] >= 0 && X[b] == X[a]) { W[a] += W[b]; X[b] = -1; }
        int32_t D = gi.zeta[su];
        int64_t wD = 0;
#pragma unroll
        for (int j = 0; j < kLaneMax; ++j) {
            if (X[j] == D) wD = W[j];
            ncand += (X[j] >= 0 && X[j] != D);
        }
        int64_t vu = ms.vol[u];
        int64_t base = LP ? 0 : gi.volC[D] - vu;
        const int64_t S_u = node_S(ms, u);
        const uint64_t hv = LP ? prio_hash(ms.lp_seed, ms.lp_level, u) : 0;
        int64_t slack, kslack;
        int32_t bx = (force_wide || vu > node_wl(ms, u))
                         ? lane_pick<WK, LP, i128>(X, W, D, wD, (i128)vu * ms.gp, base, (i128)S_u * ms.gq, gi.volC,
                                                   gi.ord, hv, &slack, &kslack)
                         : lane_pick<WK, LP, int64_t>(X, W, D, wD, vu * ms.gp, base, S_u * ms.gq, gi.volC, gi.ord,
                                                      hv, &slack, &kslack);
        ms.move_to[pos] = (bx == kNone) ? -1 : bx;
        if (st.on) {
            if (bx == kNone) record_stay(ms, st, u, slack, kslack);
            else mark_moved<WK>(g, ms, u, e0, e0 + d, 0, 1);
        }
        nd = 1;
        ne = d;
        if (LP) {
            if (bx == kNone) ms.active[u] = 0;
            else lp_activate(g, ms.active, u, e0, e0 + d, 0, 1);
        }
    }
    count_candidates(ms.cand_dev ? ms.cand_dev + 0 : nullptr, ncand);
    count_decided(ms.dec_dev, 0, 4, nd, ne);
}

// ------------------------------------------------------------------ wavefront per node
// Entries whose neighbour is already in u's own community D are summed in
// registers (w(u, D\u) is needed on its own anyway) and never enter the hash
// table: on graphs where many neighbours have joined u, the table would
// otherwise serialise on that one key.
constexpr int kWaveCap = 1024;  // slots per wavefront (rows up to 512 entries)

// Scores the occupied slots of a table (and empties them).  Slots are taken
// kEvalBatch per thread at a time, so that their community-volume gathers are
// in flight together.  s(X) = S w(u,X) - vol(u) vol(X) <= S w(u,X) since
// vol(X) >= 0, so a slot with S w(u,X) <= K (the score of staying) can never
// be chosen and its volume is not gathered; the best of the remaining slots,
// and whether it beats K, are exactly those of a full scan.
constexpr int kEvalBatch = 8;

// maxpa: raised to the largest weight of a pruned slot (its score is at most
// S w(u,X)), from which, with bs, a node that stays gets its slack
template <typename G, typename V, bool LP>
__device__ __forceinline__ void eval_slots(int32_t *tk, V *tv, int tsize, int first, int step, G vu, G S, G K,
                                           const int64_t *volC, const int32_t *ord, bool clear, G &bs, int32_t &bx,
                                           int64_t &maxpa, int64_t &ncand, uint64_t hv) {
    for (int s0 = first; s0 < tsize; s0 += kEvalBatch * step) {
        int32_t X[kEvalBatch];
        int64_t a[kEvalBatch], vc[kEvalBatch];
        bool c[kEvalBatch];
#pragma unroll
        for (int j = 0; j < kEvalBatch; ++j) {
            int s = s0 + j * step;
            X[j] = s < tsize ? tk[s] : kEmpty;
            a[j] = 0;
            if (X[j] >= 0) {
                a[j] = (int64_t)tv[s];
                if (clear) { tk[s] = kEmpty; tv[s] = 0; }
            }
            c[j] = X[j] >= 0 && (G)S * (G)a[j] > K;
        }
        int32_t ox[kEvalBatch];
#pragma unroll
        for (int j = 0; j < kEvalBatch; ++j) {
            vc[j] = (!LP && c[j]) ? volC[X[j]] : 0;
            ox[j] = c[j] ? orig_id(ord, X[j]) : X[j];
        }
#pragma unroll
        for (int j = 0; j < kEvalBatch; ++j) {
            ncand += X[j] >= 0;
            if (X[j] < 0) continue;
            if (!c[j]) {
                if (a[j] > maxpa) maxpa = a[j];
                continue;
            }
            G sc = (G)S * (G)a[j] - (G)vu * (G)vc[j];
            if constexpr (LP) sc += (G)lp_tie(hv, ox[j]);
            if (sc > bs || (sc == bs && ox[j] < bx)) { bs = sc; bx = ox[j]; }
        }
    }
}

template <typename G, bool LP>
__device__ __forceinline__ void wave_eval(int32_t *tk, int32_t *tv, int tsize, int64_t wD, G vu, int64_t base, G S,
                                          const int64_t *volC, const int32_t *ord, int32_t &best_x, bool &move,
                                          int64_t &ncand, uint64_t hv, int64_t &slack, int64_t &kslack) {
    G bs = neg_inf<G>();
    int64_t maxpa = -1;
    int32_t bx = kNone;
    const G K = (G)S * (G)wD - (G)vu * (G)base + (LP ? (G)kLpTieMax : (G)0);
    eval_slots<G, int32_t, LP>(tk, tv, tsize, lane_id(), kWave, vu, S, K, volC, ord, true, bs, bx, maxpa, ncand, hv);
    wave_argmax<G>(bs, bx);
    best_x = bx;
    move = bx != kNone && bs > K;
    slack_lean<G>(K, S, bs, wave_max_i64(maxpa), slack, kslack);
}

// folds the (X, w) entries of u into a hash table (LDS) except X == D; returns
// this thread's share of w(u, D \ u).  Entries are taken B at a time: B column
// loads, then B community gathers, then B inserts, so that the memory
// latencies of a batch overlap.
__device__ __forceinline__ void lds_add(int32_t *p, int64_t x) { atomicAdd(p, (int32_t)x); }
__device__ __forceinline__ void lds_add(int64_t *p, int64_t x) {
    atomicAdd((unsigned long long *)p, (unsigned long long)x);
}

template <int WK, int B, typename V>
__device__ __forceinline__ int64_t fold_row(const GraphView &g, const GatherIds &gi, int32_t su, int32_t D, int64_t e0,
                                            int64_t e1, int64_t first, int64_t step, int32_t *tk, V *tv, int bits) {
    const uint32_t mask = (1u << bits) - 1;
    int64_t myD = 0;
    for (int64_t base = e0 + first; base < e1; base += step * B) {
        int32_t v[B], X[B];
        int64_t wt[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            int64_t e = base + b * step;
            bool ok = e < e1;
            v[b] = ok ? gi.col[e] : su;
            wt[b] = ok ? wload<WK>(g.w, e) : 0;
        }
#pragma unroll
        for (int b = 0; b < B; ++b) X[b] = v[b] != su ? gi.zeta[v[b]] : -1;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            if (X[b] < 0) continue;
            if (X[b] == D) {
                myD += wt[b];
                continue;
            }
            uint32_t h = slot_hash(X[b], bits);
            for (;;) {
                int32_t k = atomicCAS(&tk[h], kEmpty, X[b]);
                if (k == kEmpty || k == X[b]) {
                    lds_add(&tv[h], wt[b]);
                    break;
                }
                h = (h + 1) & mask;
            }
        }
    }
    return myD;
}

// (at most 128 VGPRs: four waves per SIMD)
template <int WK, bool LP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_decide_wave(GraphView g, MoveState ms,
                                                                                           int64_t begin, int64_t count,
                                                                                           int force_wide) {
    __shared__ int32_t tk[4][kWaveCap];
    __shared__ int32_t tv[4][kWaveCap];
    const int w = threadIdx.x / kWave, lane = lane_id();
    for (int s = lane; s < kWaveCap; s += kWave) { tk[w][s] = kEmpty; tv[w][s] = 0; }
    wave_sync();
    int64_t ncand = 0, nd = 0, ne = 0;
    const Settle st = LP ? Settle{false, 0} : settle_state(ms);
    const GatherIds gi = gather_ids(g, ms);
    for (int64_t i = (int64_t)blockIdx.x * 4 + w; i < count; i += (int64_t)gridDim.x * 4) {
        int64_t pos = begin + i;
        const NodeRec r = ms.rec[pos];
        const int32_t u = r.u;
        if ((LP && !ms.active[u]) || settled(ms, st, u)) {  // wave-uniform
            if (lane == 0) ms.move_to[pos] = -1;
            continue;
        }
        const int64_t e0 = r.e0, e1 = r.e0 + r.len;
        int bits = ceil_log2_dev(2 * (e1 - e0));
        bits = bits < 6 ? 6 : bits;
        int32_t D = gi.zeta[r.s];
        int64_t wD = fold_row<WK, 4, int32_t>(g, gi, r.s, D, e0, e1, lane, kWave, tk[w], tv[w], bits);
        wD = wave_sum(wD);
        wave_sync();
        int64_t vu = ms.vol[u];
        int64_t base = LP ? 0 : gi.volC[D] - vu;
        int32_t bx;
        bool mv;
        const int64_t S_u = node_S(ms, u);
        const uint64_t hv = LP ? prio_hash(ms.lp_seed, ms.lp_level, u) : 0;
        int64_t slack, kslack;
        if (force_wide || vu > node_wl(ms, u))
            wave_eval<i128, LP>(tk[w], tv[w], 1 << bits, wD, (i128)vu * ms.gp, base, (i128)S_u * ms.gq, gi.volC,
                                gi.ord, bx, mv, ncand, hv, slack, kslack);
        else
            wave_eval<int64_t, LP>(tk[w], tv[w], 1 << bits, wD, vu * ms.gp, base, S_u * ms.gq, gi.volC, gi.ord, bx, mv,
                                   ncand, hv, slack, kslack);
        if (lane == 0) {
            ms.move_to[pos] = mv ? bx : -1;
            if (st.on && !mv) record_stay(ms, st, u, slack, kslack);
            nd += 1;
            ne += e1 - e0;
        }
        if (LP) {
            if (mv) lp_activate(g, ms.active, u, e0, e1, lane, kWave);
            else if (lane == 0) ms.active[u] = 0;
        } else if (st.on && mv) {
            mark_moved<WK>(g, ms, u, e0, e1, lane, kWave);
        }
        wave_sync();
    }
    count_candidates(ms.cand_dev ? ms.cand_dev + 1 : nullptr, ncand);
    count_decided(ms.dec_dev, 1, 5, nd, ne);
}

// ------------------------------------------------------------------ 16 lanes per node
// Short rows of the wavefront bin (at most kQuadRow entries): four nodes per
// wavefront, each with 16 lanes and a table of at most 128 slots, so that a row
// of ~20 entries no longer leaves most of a wavefront idle.  The body is
// uniform over the wavefront: a group without a node (past the end, or
// inactive in label propagation) folds an empty row.
constexpr int kQuadLanes = 16;
constexpr int kQuadCap = 2 * (int)kQuadRow;

template <typename G>
__device__ __forceinline__ G quad_max(G x) {
#pragma unroll
    for (int d = kQuadLanes / 2; d >= 1; d >>= 1) {
        G o = shfl_xor_g<G>(x, d);
        if (o > x) x = o;
    }
    return x;
}
template <typename G>
__device__ __forceinline__ void quad_argmax(G &s, int32_t &x) {
#pragma unroll
    for (int d = kQuadLanes / 2; d >= 1; d >>= 1) {
        G os = shfl_xor_g<G>(s, d);
        int32_t ox = __shfl_xor(x, d);
        if (os > s || (os == s && ox < x)) { s = os; x = ox; }
    }
}
__device__ __forceinline__ int64_t quad_sum(int64_t v) {
#pragma unroll
    for (int d = kQuadLanes / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

template <typename G, bool LP>
__device__ __forceinline__ void quad_eval(int32_t *tk, int32_t *tv, int tsize, int64_t wD, G vu, int64_t base, G S,
                                          const int64_t *volC, const int32_t *ord, int32_t &best_x, bool &move,
                                          int64_t &ncand,
                                          uint64_t hv, int64_t &slack, int64_t &kslack) {
    G bs = neg_inf<G>();
    int64_t maxpa = -1;
    int32_t bx = kNone;
    const G K = (G)S * (G)wD - (G)vu * (G)base + (LP ? (G)kLpTieMax : (G)0);
    eval_slots<G, int32_t, LP>(tk, tv, tsize, (int)(threadIdx.x % kQuadLanes), kQuadLanes, vu, S, K, volC, ord, true,
                               bs, bx, maxpa, ncand, hv);
    quad_argmax<G>(bs, bx);
    best_x = bx;
    move = bx != kNone && bs > K;
    slack_lean<G>(K, S, bs, quad_max<int64_t>(maxpa), slack, kslack);
}

// (at most 128 VGPRs: four waves per SIMD)
template <int WK, bool LP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_decide_quad(GraphView g, MoveState ms,
                                                                                           int64_t begin, int64_t count,
                                                                                           int force_wide) {
    constexpr int kGroups = 256 / kQuadLanes;
    __shared__ int32_t tk[kGroups][kQuadCap];
    __shared__ int32_t tv[kGroups][kQuadCap];
    const int grp = threadIdx.x / kQuadLanes, l = threadIdx.x % kQuadLanes;
    for (int s = l; s < kQuadCap; s += kQuadLanes) { tk[grp][s] = kEmpty; tv[grp][s] = 0; }
    wave_sync();
    int64_t ncand = 0, nd = 0, ne = 0;
    const Settle st = LP ? Settle{false, 0} : settle_state(ms);
    const GatherIds gi = gather_ids(g, ms);
    for (int64_t b0 = (int64_t)blockIdx.x * kGroups; b0 < count; b0 += (int64_t)gridDim.x * kGroups) {
        const int64_t i = b0 + grp, pos = begin + i;
        const bool has = i < count;
        const NodeRec r = has ? ms.rec[pos] : NodeRec{0, 0, 0, 0, 0};
        const int32_t u = r.u;
        const bool act = has && (!LP || ms.active[u]) && !settled(ms, st, u);
        if (has && !act && l == 0) ms.move_to[pos] = -1;
        const int64_t e0 = act ? r.e0 : 0, e1 = act ? r.e0 + r.len : 0;
        int bits = ceil_log2_dev(2 * (e1 - e0));
        bits = bits < 6 ? 6 : bits;  // rows of at most kQuadRow entries: at most kQuadCap slots
        const int32_t D = act ? gi.zeta[r.s] : -1;
        int64_t wD = fold_row<WK, 4, int32_t>(g, gi, r.s, D, e0, e1, l, kQuadLanes, tk[grp], tv[grp], bits);
        wD = quad_sum(wD);
        wave_sync();
        const int64_t vu = act ? ms.vol[u] : 0;
        const int64_t base = (LP || !act) ? 0 : gi.volC[D] - vu;
        const int64_t S_u = act ? node_S(ms, u) : 0;
        const uint64_t hv = (LP && act) ? prio_hash(ms.lp_seed, ms.lp_level, u) : 0;
        int32_t bx;
        bool mv;
        int64_t slack, kslack;
        if (act && (force_wide || vu > node_wl(ms, u)))
            quad_eval<i128, LP>(tk[grp], tv[grp], 1 << bits, wD, (i128)vu * ms.gp, base, (i128)S_u * ms.gq, gi.volC,
                                gi.ord, bx, mv, ncand, hv, slack, kslack);
        else
            quad_eval<int64_t, LP>(tk[grp], tv[grp], 1 << bits, wD, vu * ms.gp, base, S_u * ms.gq, gi.volC, gi.ord, bx,
                                   mv, ncand, hv, slack, kslack);
        if (act && l == 0) {
            ms.move_to[pos] = mv ? bx : -1;
            if (st.on && !mv) record_stay(ms, st, u, slack, kslack);
            nd += 1;
            ne += e1 - e0;
        }
        if (LP && act) {
            if (mv) lp_activate(g, ms.active, u, e0, e1, l, kQuadLanes);
            else if (l == 0) ms.active[u] = 0;
        } else if (!LP && act && st.on && mv) {
            mark_moved<WK>(g, ms, u, e0, e1, l, kQuadLanes);
        }
        wave_sync();
    }
    count_candidates(ms.cand_dev ? ms.cand_dev + 1 : nullptr, ncand);
    count_decided(ms.dec_dev, 1, 5, nd, ne);
}

// ------------------------------------------------------------------ workgroup per node
// rows up to kBlockShortRow entries: 256 threads and a 4096-slot table (32 KB:
// four workgroups per CU); longer rows: 512 threads and 8192 slots (64 KB: two)
constexpr int kBlockThreads = 512;
constexpr int kBlockCap = 8192;  // rows up to 4096 entries
constexpr int kBlockShortThreads = 256;
constexpr int kBlockShortCap = 4096;
static_assert(2 * kBlockShortRow <= kBlockShortCap, "short workgroup-bin table too small");

// leaves the decision (community or -1) in *out and the slack of staying in
// *slack_out (LDS), written by thread 0
template <typename G, int NT, bool LP>
__device__ __forceinline__ void block_eval(int32_t *tk, int32_t *tv, int tsize, int64_t wD, G vu, int64_t base, G S,
                                           const int64_t *volC, const int32_t *ord, int32_t *out, int64_t *slack_out,
                                           int64_t &ncand, uint64_t hv) {
    // slack_out[0], slack_out[1]: slack and kslack
    __shared__ int64_t red_w[NT / kWave];
    __shared__ G red_s[NT / kWave];
    __shared__ int64_t red_u[NT / kWave];
    __shared__ int32_t red_x[NT / kWave];
    // w(u, D \ u) first (wD enters as this thread's share): the score of staying
    // bounds which slots need their community volume
    wD = wave_sum(wD);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) red_w[w] = wD;
    __syncthreads();
    wD = 0;
    for (int j = 0; j < NT / kWave; ++j) wD += red_w[j];
    const G K = (G)S * (G)wD - (G)vu * (G)base + (LP ? (G)kLpTieMax : (G)0);
    G bs = neg_inf<G>();
    int64_t maxpa = -1;
    int32_t bx = kNone;
    eval_slots<G, int32_t, LP>(tk, tv, tsize, threadIdx.x, NT, vu, S, K, volC, ord, true, bs, bx, maxpa, ncand, hv);
    wave_argmax<G>(bs, bx);
    maxpa = wave_max_i64(maxpa);
    if (lane_id() == 0) { red_s[w] = bs; red_x[w] = bx; red_u[w] = maxpa; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int j = 1; j < NT / kWave; ++j) {
            if (red_s[j] > bs || (red_s[j] == bs && red_x[j] < bx)) { bs = red_s[j]; bx = red_x[j]; }
            if (red_u[j] > maxpa) maxpa = red_u[j];
        }
        *out = (bx != kNone && bs > K) ? bx : -1;
        slack_lean<G>(K, S, bs, maxpa, slack_out[0], slack_out[1]);
    }
}

// (NT threads, a CAP-slot table; at most 128 VGPRs)
template <int WK, bool LP, int NT, int CAP>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_decide_block(GraphView g, MoveState ms,
                                                                                          int64_t begin, int64_t count,
                                                                                          int force_wide) {
    __shared__ int32_t tk[CAP];
    __shared__ int32_t tv[CAP];
    __shared__ int32_t dec;
    __shared__ int64_t slack[2];
    for (int s = threadIdx.x; s < CAP; s += NT) { tk[s] = kEmpty; tv[s] = 0; }
    __syncthreads();
    int64_t ncand = 0, nd = 0, ne = 0;
    const Settle st = LP ? Settle{false, 0} : settle_state(ms);
    const GatherIds gi = gather_ids(g, ms);
    for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
        int64_t pos = begin + i;
        const NodeRec r = ms.rec[pos];
        const int32_t u = r.u;
        if ((LP && !ms.active[u]) || settled(ms, st, u)) {  // workgroup-uniform
            if (threadIdx.x == 0) ms.move_to[pos] = -1;
            continue;
        }
        const int64_t e0 = r.e0, e1 = r.e0 + r.len;
        int bits = ceil_log2_dev(2 * (e1 - e0));
        bits = bits < 6 ? 6 : bits;
        int32_t D = gi.zeta[r.s];
        int64_t myD = fold_row<WK, 4, int32_t>(g, gi, r.s, D, e0, e1, threadIdx.x, NT, tk, tv, bits);
        __syncthreads();
        int64_t vu = ms.vol[u];
        int64_t base = LP ? 0 : gi.volC[D] - vu;
        const int64_t S_u = node_S(ms, u);
        const uint64_t hv = LP ? prio_hash(ms.lp_seed, ms.lp_level, u) : 0;
        if (force_wide || vu > node_wl(ms, u))
            block_eval<i128, NT, LP>(tk, tv, 1 << bits, myD, (i128)vu * ms.gp, base, (i128)S_u * ms.gq, gi.volC,
                                     gi.ord, &dec, slack, ncand, hv);
        else
            block_eval<int64_t, NT, LP>(tk, tv, 1 << bits, myD, vu * ms.gp, base, S_u * ms.gq, gi.volC, gi.ord, &dec,
                                        slack, ncand, hv);
        __syncthreads();
        const int32_t x = dec;
        if (threadIdx.x == 0) {
            ms.move_to[pos] = x;
            if (st.on && x < 0) record_stay(ms, st, u, slack[0], slack[1]);
            nd += 1;
            ne += e1 - e0;
        }
        if (LP) {
            if (x >= 0) lp_activate(g, ms.active, u, e0, e1, threadIdx.x, NT);
            else if (threadIdx.x == 0) ms.active[u] = 0;
        } else if (st.on && x >= 0) {
            mark_moved<WK>(g, ms, u, e0, e1, threadIdx.x, NT);
        }
    }
    count_candidates(ms.cand_dev ? ms.cand_dev + 2 : nullptr, ncand);
    count_decided(ms.dec_dev, 2, 6, nd, ne);
}

// ------------------------------------------------------------------ hubs: one large workgroup per node
constexpr int kSingleThreads = 1024;
constexpr int kSingleBits = 14;  // 16384 slots of int32 key + int32 sum: 128 KB of LDS

template <int WK, bool LP>
__global__ __launch_bounds__(kSingleThreads) void k_hub_single(GraphView g, MoveState ms, HubArrays ha, int64_t blk0,
                                                               int force_wide) {
    __shared__ int32_t tk[1 << kSingleBits];
    __shared__ int32_t tv[1 << kSingleBits];
    __shared__ int32_t dec;
    __shared__ int64_t slack[2];
    const HubSglPlan pl = ha.splan[blk0 + blockIdx.x];
    const int32_t u = pl.u;
    const int64_t pos = pl.pos;
    const Settle st = LP ? Settle{false, 0} : settle_state(ms);
    if ((LP && !ms.active[u]) || settled(ms, st, u)) {
        if (threadIdx.x == 0) ms.move_to[pos] = -1;
        return;
    }
    const int64_t e0 = pl.e0, e1 = pl.e1;
    // rows of at most kSingleMaxRow entries: load factor <= 0.75
    int bits = ceil_log2_dev(2 * (e1 - e0));
    bits = bits < 6 ? 6 : (bits > kSingleBits ? kSingleBits : bits);
    for (int s = threadIdx.x; s < (1 << bits); s += kSingleThreads) { tk[s] = kEmpty; tv[s] = 0; }
    __syncthreads();
    const GatherIds gi = gather_ids(g, ms);
    const int32_t D = gi.zeta[pl.s];
    int64_t myD = fold_row<WK, 4, int32_t>(g, gi, pl.s, D, e0, e1, threadIdx.x, kSingleThreads, tk, tv, bits);
    __syncthreads();
    const int64_t vu = ms.vol[u];
    const int64_t base = LP ? 0 : gi.volC[D] - vu;
    const int64_t S_u = node_S(ms, u);
    const uint64_t hv = LP ? prio_hash(ms.lp_seed, ms.lp_level, u) : 0;
    int64_t ncand = 0;
    if (force_wide || vu > node_wl(ms, u))
        block_eval<i128, kSingleThreads, LP>(tk, tv, 1 << bits, myD, (i128)vu * ms.gp, base, (i128)S_u * ms.gq,
                                             gi.volC, gi.ord, &dec, slack, ncand, hv);
    else
        block_eval<int64_t, kSingleThreads, LP>(tk, tv, 1 << bits, myD, vu * ms.gp, base, S_u * ms.gq, gi.volC,
                                                gi.ord, &dec, slack, ncand, hv);
    __syncthreads();
    const int32_t x = dec;
    if (threadIdx.x == 0) {
        ms.move_to[pos] = x;
        if (st.on && x < 0) record_stay(ms, st, u, slack[0], slack[1]);
        if (ms.dec_dev) {
            atomicAdd(ms.dec_dev + 3, 1ULL);
            atomicAdd(ms.dec_dev + 7, (unsigned long long)(e1 - e0));
            atomicAdd(ms.dec_dev + 8, 1ULL);
            atomicAdd(ms.dec_dev + 9, (unsigned long long)(e1 - e0));
        }
    }
    if (LP) {
        if (x >= 0) lp_activate(g, ms.active, u, e0, e1, threadIdx.x, kSingleThreads);
        else if (threadIdx.x == 0) ms.active[u] = 0;
    } else if (st.on && x >= 0) {
        mark_moved<WK>(g, ms, u, e0, e1, threadIdx.x, kSingleThreads);
    }
    count_candidates(ms.cand_dev ? ms.cand_dev + 3 : nullptr, ncand);
    count_candidates(ms.cand_sgl, ncand);
}

// ------------------------------------------------------------------ hubs: several workgroups per node
// Rows longer than the workgroup limit are aggregated without global atomics.
//  1. part: a workgroup per chunk of kHubInsChunk entries merges its entries
//     of equal X in LDS and counting-sorts the merged (X, w) pairs into
//     P = 2^pbits hash buckets of X (P ~ row length / 1024)
//     and writes them to a staging area, with a (start, count) word per
//     (bucket, chunk); entries of u's own community D only add to a per-chunk
//     share of w(u, D \ u).
//  2. agg: a workgroup per (node, bucket) gathers that bucket from all chunks
//     into an LDS hash table, scores its communities and leaves a partial best.
//     A bucket with more than kAggMaxKeys distinct communities (not expected
//     for hashed ids, but possible) is redone in 2, 4, ... passes, each over a
//     sub-partition of its keys, so any input stays exact.
//  3. reduce: a workgroup per node combines the partial bests and the w(u, D)
//     shares, decides the move and applies it, within the launch that applies
//     the class's other moves (k_reduce_apply).
constexpr int kHubThreads = 256;
constexpr int kHubPerThread = (int)(kHubInsChunk / kHubThreads);
constexpr int kAggBits = 11;
constexpr int kAggSlots = 1 << kAggBits;  // LDS table of a bucket workgroup (~1024 entries expected)
// new keys allowed per pass: each thread claims at most one slot past the
// limit before it stops, so at most kAggMaxKeys + kHubThreads < kAggSlots
// slots are ever taken and every probe ends
constexpr int kAggMaxKeys = 1536;
static_assert(kAggMaxKeys + 256 < kAggSlots, "agg table must never fill");
constexpr int kAggTile = 512;      // chunks whose segments are flattened at once (52 KB of LDS: 3 per CU)
constexpr int32_t kHubPending = -2;  // class position of a partitioned hub until its reduce
constexpr int kAggBatch = 4;       // staged entries per thread loaded together

__device__ __forceinline__ uint32_t hub_bucket(int32_t x, int pbits) {
    return pbits == 0 ? 0u : ((uint32_t)x * 2654435769u) >> (32 - pbits);
}
__device__ __forceinline__ uint32_t agg_slot(int32_t x) { return ((uint32_t)x * 0x85EBCA6Bu) >> (32 - kAggBits); }
__device__ __forceinline__ uint32_t agg_subpart(int32_t x, int qbits) {
    return qbits == 0 ? 0u : ((uint32_t)x * 0xC2B2AE35u) >> (32 - qbits);
}

constexpr int kMergeBits = 11;
constexpr int kMergeSlots = 1 << kMergeBits;  // a chunk's merge table: at most kHubInsChunk keys, load <= 1/2
static_assert(2 * kHubInsChunk <= kMergeSlots, "merge table must never fill");
__device__ __forceinline__ uint32_t merge_slot(int32_t x) {
    return ((uint32_t)x * 0x27D4EB2Fu) >> (32 - kMergeBits);
}

template <int WK, bool LP>
__global__ __launch_bounds__(kHubThreads) void k_hub_part(GraphView g, MoveState ms, HubArrays ha, int64_t blk0) {
    // the chunk's merge table, then (once the merged weights are in registers)
    // the bucket counts and fill cursors
    __shared__ union {
        struct {
            int32_t key[kMergeSlots];
            int64_t val[kMergeSlots];
        } m;
        struct {
            int32_t start[1 << kHubMaxPBits];
            int32_t fill[1 << kHubMaxPBits];
        } b;
    } lds;
    int32_t *const start = lds.b.start;
    int32_t *const fill = lds.b.fill;
    __shared__ int64_t wsum[kHubThreads / kWave];
    const HubPartPlan pl = ha.pplan[blk0 + blockIdx.x];
    const int32_t u = pl.u;
    const int64_t k = pl.k;
    // the apply launch leaves this position to the hub's own reduce
    if (k == 0 && threadIdx.x == 0) ms.move_to[pl.pos] = kHubPending;
    // the chunk's entries are loaded beside the hub's own words (community,
    // settled test), not after them
    const int64_t c0 = pl.c0;
    const GatherIds gi = gather_ids(g, ms);
    const int32_t su = pl.s;
    int32_t v[kHubPerThread], X[kHubPerThread], bk[kHubPerThread];
    int64_t W[kHubPerThread];
#pragma unroll
    for (int j = 0; j < kHubPerThread; ++j) {
        const int32_t i = j * kHubThreads + threadIdx.x;
        const bool ok = i < pl.len;
        v[j] = ok ? gi.col[c0 + i] : su;
        W[j] = ok ? wload<WK>(g.w, c0 + i) : 0;
    }
    const int32_t D = gi.zeta[su];
    if (LP && !ms.active[u]) return;  // label propagation: inactive hub, nothing staged
    if (!LP && settled(ms, settle_state(ms), u)) return;  // settled hub: nothing staged
    if (threadIdx.x == 0 && ms.dec_dev) {
        if (k == 0) atomicAdd(ms.dec_dev + 3, 1ULL);
        atomicAdd(ms.dec_dev + 7, (unsigned long long)pl.len);
    }
    const int pb = pl.pb;
    const int P = 1 << pb;
    for (int i = threadIdx.x; i < kMergeSlots; i += kHubThreads) { lds.m.key[i] = kEmpty; lds.m.val[i] = 0; }
#pragma unroll
    for (int j = 0; j < kHubPerThread; ++j) X[j] = v[j] != su ? gi.zeta[v[j]] : -1;
    int64_t myD = 0;
#pragma unroll
    for (int j = 0; j < kHubPerThread; ++j)
        if (X[j] == D) {
            myD += W[j];
            X[j] = -1;
        }
    __syncthreads();
    // merge equal communities of the chunk: the entry that claims a key's slot
    // carries the key's summed weight, the others drop out, so a bucket holds
    // at most one entry per (community, chunk) however large the community is
    int32_t slot[kHubPerThread];
#pragma unroll
    for (int j = 0; j < kHubPerThread; ++j) {
        slot[j] = -1;
        if (X[j] < 0) continue;
        uint32_t h = merge_slot(X[j]);
        for (;;) {
            int32_t kk = atomicCAS(&lds.m.key[h], kEmpty, X[j]);
            if (kk == kEmpty || kk == X[j]) {
                atomicAdd((unsigned long long *)&lds.m.val[h], (unsigned long long)W[j]);
                if (kk == kEmpty) slot[j] = (int32_t)h;
                else X[j] = -1;
                break;
            }
            h = (h + 1) & (kMergeSlots - 1);
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kHubPerThread; ++j)
        if (slot[j] >= 0) W[j] = lds.m.val[slot[j]];
    __syncthreads();
    for (int i = threadIdx.x; i < P; i += kHubThreads) { start[i] = 0; fill[i] = 0; }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kHubPerThread; ++j) {
        bk[j] = X[j] >= 0 ? (int32_t)hub_bucket(X[j], pb) : -1;
        if (bk[j] >= 0) atomicAdd(&start[bk[j]], 1);
    }
    __syncthreads();
    // exclusive scan of the P bucket counts: thread t owns buckets [t*per, (t+1)*per)
    const int per = (P + kHubThreads - 1) / kHubThreads;
    int32_t cnts[(1 << kHubMaxPBits) / kHubThreads];
    int32_t local = 0;
#pragma unroll
    for (int i = 0; i < (1 << kHubMaxPBits) / kHubThreads; ++i) {
        int b = threadIdx.x * per + i;
        cnts[i] = (i < per && b < P) ? start[b] : 0;
        local += cnts[i];
    }
    int32_t inc = local;
    for (int d = 1; d < kWave; d <<= 1) {
        int32_t y = __shfl_up(inc, d);
        if (lane_id() >= d) inc += y;
    }
    __shared__ int32_t wtot[kHubThreads / kWave];
    if (lane_id() == kWave - 1) wtot[threadIdx.x / kWave] = inc;
    __syncthreads();
    int32_t run = inc - local;
    for (int i = 0; i < threadIdx.x / kWave; ++i) run += wtot[i];
    const int32_t nch = pl.nch;
    uint32_t *bkt = ha.bkt + pl.bkt;
#pragma unroll
    for (int i = 0; i < (1 << kHubMaxPBits) / kHubThreads; ++i) {
        int b = threadIdx.x * per + i;
        if (i < per && b < P) {
            start[b] = run;
            bkt[(int64_t)b * nch + k] = ((uint32_t)run << 16) | (uint32_t)cnts[i];
            run += cnts[i];
        }
    }
    __syncthreads();
    int32_t *sx = ha.stg_x + pl.stg;
    int64_t *sw = ha.stg_w + pl.stg;
#pragma unroll
    for (int j = 0; j < kHubPerThread; ++j) {
        if (bk[j] < 0) continue;
        int32_t pos = start[bk[j]] + atomicAdd(&fill[bk[j]], 1);
        sx[pos] = X[j];
        sw[pos] = W[j];
    }
    myD = wave_sum(myD);
    if (lane_id() == 0) wsum[threadIdx.x / kWave] = myD;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int i = 0; i < kHubThreads / kWave; ++i) s += wsum[i];
        ha.wd_part[blockIdx.x] = s;
    }
}

// block-wide (s desc, X asc) argmax; result valid in thread 0
template <typename G>
__device__ __forceinline__ void block_argmax(G &bs, int32_t &bx) {
    __shared__ G red_s[kHubThreads / kWave];
    __shared__ int32_t red_x[kHubThreads / kWave];
    wave_argmax<G>(bs, bx);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if (lane_id() == 0) { red_s[w] = bs; red_x[w] = bx; }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int j = 0; j < kHubThreads / kWave; ++j)
            if (red_s[j] > bs || (red_s[j] == bs && red_x[j] < bx)) { bs = red_s[j]; bx = red_x[j]; }
}

// block-wide max; result valid in thread 0
template <typename G>
__device__ __forceinline__ G block_max(G x) {
    __shared__ G red[kHubThreads / kWave];
    x = wave_max<G>(x);
    __syncthreads();
    if (lane_id() == 0) red[threadIdx.x / kWave] = x;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int j = 0; j < kHubThreads / kWave; ++j)
            if (red[j] > x) x = red[j];
    return x;
}

// Entries of bucket p of a hub, over all its chunks, processed kAggTile chunks
// at a time: an LDS prefix sum over the chunks' segment lengths turns the
// bucket into one flat index space that every thread strides over (a binary
// search finds the chunk of an index).
constexpr int kAggPer = kAggTile / kHubThreads;  // chunk words per thread and tile
// pre: this thread's words of the first tile, loaded at the start of the
// kernel (tile 0 is read by every pass)
template <typename G, bool LP>
__device__ __forceinline__ void agg_bucket(const HubArrays &ha, const HubAggPlan &pl, const uint32_t (&pre)[kAggPer],
                                           G vu, G S, G K, const int64_t *volC, const int32_t *ord, int32_t *tk,
                                           int64_t *tv, int32_t *cpre, int32_t *cbase, int32_t *wtot, int32_t *nkeys,
                                           int32_t *overflow, G &bs, int32_t &bx, int64_t &maxpa, int64_t &ncand,
                                           uint64_t hv) {
    const int32_t nch = pl.nch;
    const uint32_t *bkt = ha.bkt + pl.bkt;
    const int32_t *sx = ha.stg_x + pl.stg;
    const int64_t *sw = ha.stg_w + pl.stg;
    constexpr int kPer = kAggPer;
    const int32_t max_keys = ha.agg_max_keys > 0 ? ha.agg_max_keys : kAggMaxKeys;
    const int32_t tile = ha.agg_tile > 0 ? ha.agg_tile : kAggTile;
    for (int qbits = 0;; ++qbits) {
        G pbs = neg_inf<G>();
        int64_t pmaxpa = -1;
        int32_t pbx = kNone;
        int64_t pc = 0;
        bool ok = true;
        for (int q = 0; q < (1 << qbits); ++q) {
            for (int s = threadIdx.x; s < kAggSlots; s += kHubThreads) { tk[s] = kEmpty; tv[s] = 0; }
            if (threadIdx.x == 0) { *nkeys = 0; *overflow = 0; }
            __syncthreads();
            bool stop = false;
            for (int32_t t0 = 0; t0 < nch; t0 += tile) {
                const int32_t tn = nch - t0 < tile ? nch - t0 : tile;
                // segment lengths of this tile's chunks, exclusive prefix into cpre
                int32_t cnt[kPer], loc = 0;
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    int32_t c = threadIdx.x * kPer + i;
                    uint32_t word = c < tn ? (t0 == 0 ? pre[i] : bkt[t0 + c]) : 0u;
                    cnt[i] = (int32_t)(word & 0xffffu);
                    if (c < tn) cbase[c] = (t0 + c) * (int32_t)kHubInsChunk + (int32_t)(word >> 16);
                    loc += cnt[i];
                }
                int32_t inc = loc;
                for (int d = 1; d < kWave; d <<= 1) {
                    int32_t y = __shfl_up(inc, d);
                    if (lane_id() >= d) inc += y;
                }
                if (lane_id() == kWave - 1) wtot[threadIdx.x / kWave] = inc;
                __syncthreads();
                int32_t run = inc - loc, total = 0;
                for (int i = 0; i < kHubThreads / kWave; ++i) {
                    if (i < (int)(threadIdx.x / kWave)) run += wtot[i];
                    total += wtot[i];
                }
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    cpre[threadIdx.x * kPer + i] = run;
                    run += cnt[i];
                }
                __syncthreads();
                // kAggBatch entries per thread at a time: staging loads in flight together
                for (int32_t i0 = threadIdx.x; i0 < total && !stop; i0 += kAggBatch * kHubThreads) {
                    int32_t X[kAggBatch];
                    int64_t w[kAggBatch];
#pragma unroll
                    for (int b = 0; b < kAggBatch; ++b) {
                        int32_t i = i0 + b * kHubThreads;
                        X[b] = kEmpty;
                        w[b] = 0;
                        if (i < total) {
                            int32_t lo = 0, hi = tn;  // last chunk c with cpre[c] <= i
                            while (hi - lo > 1) {
                                int32_t mid = (lo + hi) >> 1;
                                if (cpre[mid] <= i) lo = mid; else hi = mid;
                            }
                            int64_t idx = (int64_t)cbase[lo] + (i - cpre[lo]);
                            X[b] = sx[idx];
                            w[b] = sw[idx];
                        }
                    }
#pragma unroll
                    for (int b = 0; b < kAggBatch; ++b) {
                        if (stop || X[b] < 0 || agg_subpart(X[b], qbits) != (uint32_t)q) continue;
                        uint32_t h = agg_slot(X[b]);
                        for (;;) {
                            int32_t kk = atomicCAS(&tk[h], kEmpty, X[b]);
                            if (kk == kEmpty && atomicAdd(nkeys, 1) >= max_keys) {
                                *overflow = 1;
                                stop = true;
                                break;
                            }
                            if (kk == kEmpty || kk == X[b]) {
                                atomicAdd((unsigned long long *)&tv[h], (unsigned long long)w[b]);
                                break;
                            }
                            h = (h + 1) & (kAggSlots - 1);
                        }
                    }
                }
                __syncthreads();
            }
            if (*overflow) {
                ok = false;
                __syncthreads();
                break;
            }
            eval_slots<G, int64_t, LP>(tk, tv, kAggSlots, threadIdx.x, kHubThreads, vu, S, K, volC, ord, false, pbs,
                                       pbx, pmaxpa, pc, hv);
            __syncthreads();
        }
        if (ok) {
            bs = pbs;
            bx = pbx;
            maxpa = pmaxpa;
            ncand += pc;
            return;
        }
    }
}

// (WK only names the instantiation after the level's weight kind, so that
// profiles tell the input level from the coarse ones)
template <int WK, bool LP>
__global__ __launch_bounds__(kHubThreads) void k_hub_agg(MoveState ms, HubArrays ha, int64_t blk0, int force_wide) {
    __shared__ int32_t tk[kAggSlots];
    __shared__ int64_t tv[kAggSlots];
    __shared__ int32_t cpre[kAggTile], cbase[kAggTile], wtot[kHubThreads / kWave];
    __shared__ int32_t nkeys, overflow;
    __shared__ int64_t wred[kHubThreads / kWave];
    const HubAggPlan pl = ha.aplan[blk0 + blockIdx.x];
    const int64_t hg = pl.hg, p = pl.p;
    const int32_t u = pl.u;
    // words that depend only on the plan go out together: the first tile of
    // the bucket's chunk words, the chunk shares of w(u, D \ u), u's own words
    uint32_t pre[kAggPer];
    {
        const int32_t tile = ha.agg_tile > 0 ? ha.agg_tile : kAggTile;
        const int32_t tn = pl.nch < tile ? pl.nch : tile;
#pragma unroll
        for (int i = 0; i < kAggPer; ++i) {
            const int32_t c = threadIdx.x * kAggPer + i;
            pre[i] = c < tn ? ha.bkt[pl.bkt + c] : 0u;
        }
    }
    int64_t wD = 0;
    for (int64_t j = threadIdx.x; j < pl.nch; j += kHubThreads) wD += ha.wd_part[pl.wd + j];
    const int64_t vu = ms.vol[u];
    // community ids of the sweep layout when the level has one (see MoveState)
    const int64_t *vcs = ms.colp ? ms.volCp : ms.volC;
    const int32_t *ord = ms.colp ? ms.ord : nullptr;
    const int32_t D = ms.colp ? ms.zetap[pl.s] : ms.zeta[u];
    if (LP && !ms.active[u]) return;
    if (!LP) {
        // whether the hub is settled, and the clock its decision is taken at,
        // for the reduce (which runs while the class's moves advance the clock)
        const Settle st = settle_state(ms);
        const bool sk = settled(ms, st, u);
        if (p == 0 && threadIdx.x == 0) {
            ha.hub_skip[hg] = sk ? 1 : 0;
            ha.hub_clk[hg] = st.now;
        }
        if (sk) return;
    }
    // w(u, D \ u) from the chunk shares (written by the chunk launch) and the
    // score of staying, which bounds the slots worth a volume gather
    wD = wave_sum(wD);
    if (lane_id() == 0) wred[threadIdx.x / kWave] = wD;
    __syncthreads();
    wD = 0;
    for (int i = 0; i < kHubThreads / kWave; ++i) wD += wred[i];
    const int64_t base = LP ? 0 : vcs[D] - vu;
    // vol(D \ u) at the start of the class, for the reduce (which runs while the
    // class's other moves apply)
    if (p == 0 && threadIdx.x == 0) ha.hub_base[hg] = base;
    int64_t ncand = 0;
    i128 bs = neg_inf<i128>();
    int32_t bx = kNone;
    int64_t slack = 0;  // of this bucket's communities (thread 0)
    const int64_t S_u = node_S(ms, u);
    const uint64_t hv = LP ? prio_hash(ms.lp_seed, ms.lp_level, u) : 0;
    if (force_wide || vu > node_wl(ms, u)) {
        const i128 Sg = (i128)S_u * ms.gq, vg = (i128)vu * ms.gp;
        const i128 K = Sg * (i128)wD - vg * (i128)base + (LP ? (i128)kLpTieMax : (i128)0);
        int64_t maxpa = -1;
        agg_bucket<i128, LP>(ha, pl, pre, vg, Sg, K, vcs, ord, tk, tv, cpre, cbase, wtot, &nkeys, &overflow, bs,
                             bx, maxpa, ncand, hv);
        block_argmax<i128>(bs, bx);
        maxpa = block_max<int64_t>(maxpa);
        int64_t ks;
        slack_from<i128>(K, Sg, bs, maxpa, slack, ks);
    } else {
        const int64_t Sg = S_u * ms.gq, vg = vu * ms.gp;
        const int64_t K = Sg * wD - vg * base + (LP ? (int64_t)kLpTieMax : 0);
        int64_t b64 = neg_inf<int64_t>(), maxpa = -1;
        agg_bucket<int64_t, LP>(ha, pl, pre, vg, Sg, K, vcs, ord, tk, tv, cpre, cbase, wtot, &nkeys, &overflow, b64,
                                bx, maxpa, ncand, hv);
        block_argmax<int64_t>(b64, bx);
        maxpa = block_max<int64_t>(maxpa);
        int64_t ks;
        slack_from<int64_t>(K, Sg, b64, maxpa, slack, ks);
        bs = (i128)b64;
    }
    if (threadIdx.x == 0) {
        unsigned long long *part = ha.part + 4 * (size_t)blockIdx.x;
        part[0] = (unsigned long long)(uint64_t)(bs >> 64);
        part[1] = (unsigned long long)(uint64_t)bs;
        part[2] = (unsigned long long)(uint32_t)bx;
        part[3] = (unsigned long long)slack;
    }
    count_candidates(ms.cand_dev ? ms.cand_dev + 3 : nullptr, ncand);
}

// apply of one decided move (X >= 0) of node u; returns 1
__device__ __forceinline__ int64_t apply_move(const MoveState &ms, int32_t u, int32_t X) {
    int32_t D = ms.zeta[u];
    int64_t vu = ms.vol[u];
    ms.zeta[u] = X;
    if (ms.zetap) ms.zetap[ms.sig[u]] = ms.sig[X];  // the sweep layout's copy
    if (!ms.active) {  // label propagation keeps no community volumes
        atomicAdd((unsigned long long *)&ms.volC[D], (unsigned long long)(-vu));
        atomicAdd((unsigned long long *)&ms.volC[X], (unsigned long long)vu);
        if (ms.volCp) {
            atomicAdd((unsigned long long *)&ms.volCp[ms.sig[D]], (unsigned long long)(-vu));
            atomicAdd((unsigned long long *)&ms.volCp[ms.sig[X]], (unsigned long long)vu);
        }
    }
    if (ms.gmoved) ms.gmoved[ms.gid[u]] = 1;
    return 1;
}

// A partitioned hub's reduce: a workgroup per slice of the hub's row combines
// the bucket partials and the w(u, D) shares (written by earlier launches) and
// decides the move like any other node (every slice reaches the same decision
// from the same words); slice 0 applies it, and when the hub moves each slice
// marks (or, in label propagation, activates) the neighbours in its part of
// the row, so that a hub of millions of entries is not marked by one
// workgroup.  vol(D \ u) comes from the bucket launch, taken before any move of
// the class applied.
template <bool LP>
__device__ __forceinline__ void hub_reduce_apply(const GraphView &g, const MoveState &ms, const HubArrays &ha,
                                                 const HubRedPlan &pl) {
    __shared__ int64_t wsum[kHubThreads / kWave];
    __shared__ int32_t dec;
    const int32_t u = pl.u;
    const int64_t hg = pl.hg;
    if (LP && !ms.active[u]) return;  // nothing decided, nothing to apply
    // settled (decided by the bucket launch before any move of the class): stays
    const bool sk = !LP && ms.sctl && ms.sctl[0];
    if (sk && ha.hub_skip[hg]) return;
    const int64_t nagg = pl.nagg;
    const unsigned long long *p0 = ha.part + 4 * (size_t)pl.agg;
    i128 bs = neg_inf<i128>();
    int32_t bx = kNone;
    int64_t slack = INT64_MAX;
    for (int64_t j = threadIdx.x; j < nagg; j += kHubThreads) {
        int32_t x = (int32_t)p0[4 * j + 2];
        i128 s = (i128)(((unsigned __int128)p0[4 * j + 0] << 64) | p0[4 * j + 1]);
        if (x != kNone && (s > bs || (s == bs && x < bx))) { bs = s; bx = x; }
        const int64_t sl = (int64_t)p0[4 * j + 3];
        if (sl < slack) slack = sl;
    }
    if (sk) slack = -block_max<int64_t>(-slack);  // the smallest bucket slack, in thread 0
    int64_t wD = 0;
    for (int64_t j = threadIdx.x; j < pl.nch; j += kHubThreads) wD += ha.wd_part[pl.wd + j];
    wD = wave_sum(wD);
    if (lane_id() == 0) wsum[threadIdx.x / kWave] = wD;
    block_argmax<i128>(bs, bx);
    if (threadIdx.x == 0) {
        wD = 0;
        for (int i = 0; i < kHubThreads / kWave; ++i) wD += wsum[i];
        const int64_t vu = ms.vol[u];
        const int64_t base = ha.hub_base[hg];
        i128 K = (i128)node_S(ms, u) * ms.gq * (i128)wD - (i128)vu * ms.gp * (i128)base +
                 (LP ? (i128)kLpTieMax : (i128)0);
        dec = (bx != kNone && bs > K) ? bx : -1;
        if (pl.k == 0) {
            if (dec >= 0) atomicAdd(ms.moves_dev, (unsigned long long)apply_move(ms, u, dec));
            if (sk) {
                if (dec >= 0) {
                    atomicAdd(&ms.sctl[1], (unsigned long long)(2 * vu));
                } else {
                    int64_t s_, k_;
                    slack_of<i128>(K, K - (i128)slack, s_, k_);  // slack = the smallest bucket slack
                    record_stay(ms, Settle{true, ha.hub_clk[hg]}, u, s_, k_);
                }
            }
        }
    }
    if (LP) {
        __syncthreads();
        if (dec >= 0) lp_activate(g, ms.active, u, pl.s0, pl.s1, threadIdx.x, kHubThreads);
        else if (pl.k == 0 && threadIdx.x == 0) ms.active[u] = 0;
    } else if (sk) {
        __syncthreads();
        if (dec >= 0) {
            switch (g.wkind) {
                case 0: mark_moved<0>(g, ms, u, pl.s0, pl.s1, threadIdx.x, kHubThreads); break;
                case 1: mark_moved<1>(g, ms, u, pl.s0, pl.s1, threadIdx.x, kHubThreads); break;
                default: mark_moved<2>(g, ms, u, pl.s0, pl.s1, threadIdx.x, kHubThreads); break;
            }
        }
    }
}

// ------------------------------------------------------------------ apply
// The moves of class positions [begin, begin + count): workgroups [0, nred)
// reduce and apply the class's partitioned hubs (red_hub[red0 ..]), the rest
// (grid-stride) apply every other decided move and add their count with one
// atomic per workgroup.  Partitioned hubs' positions hold kHubPending and are
// skipped by the latter.
template <bool LP>
__global__ __launch_bounds__(kHubThreads) void k_reduce_apply(GraphView g, MoveState ms, HubArrays ha, int64_t red0,
                                                              int64_t nred, int64_t begin, int64_t count) {
    if ((int64_t)blockIdx.x < nred) {  // workgroup-uniform
        hub_reduce_apply<LP>(g, ms, ha, ha.rplan[red0 + blockIdx.x]);
        return;
    }
    __shared__ int64_t red[kHubThreads / kWave];
    const int64_t nblk = (int64_t)gridDim.x - nred;
    int64_t moved = 0, mvol = 0;
    if (LP) {
        for (int64_t i = ((int64_t)blockIdx.x - nred) * kHubThreads + threadIdx.x; i < count;
             i += nblk * kHubThreads) {
            int64_t pos = begin + i;
            int32_t X = ms.move_to[pos];
            if (X >= 0) moved += apply_move(ms, ms.class_nodes[pos], X);
        }
    } else {
        // wavefront-uniform trips: the volume updates of moves that leave or
        // join the same community are combined per wavefront
        const bool sk = ms.sctl && ms.sctl[0];
        for (int64_t i0 = ((int64_t)blockIdx.x - nred) * kHubThreads + (threadIdx.x & ~(kWave - 1)); i0 < count;
             i0 += nblk * kHubThreads) {
            const int64_t i = i0 + lane_id();
            const int32_t X = i < count ? ms.move_to[begin + i] : -1;
            const int32_t u = i < count ? ms.class_nodes[begin + i] : 0;  // beside the move, not after it
            const bool mv = X >= 0;
            int32_t D = 0;
            int64_t join = 0, leave = 0;
            if (mv) {
                D = ms.zeta[u];
                join = leave = ms.vol[u];
                ms.zeta[u] = X;
                if (ms.zetap) ms.zetap[ms.sig[u]] = ms.sig[X];  // the sweep layout's copy
                if (ms.gmoved) ms.gmoved[ms.gid[u]] = 1;
                ++moved;
                mvol += join;
            }
            if (wave_group_sum(X, mv, join)) {
                atomicAdd((unsigned long long *)&ms.volC[X], (unsigned long long)join);
                if (ms.volCp) atomicAdd((unsigned long long *)&ms.volCp[ms.sig[X]], (unsigned long long)join);
            }
            if (wave_group_sum(D, mv, leave)) {
                atomicAdd((unsigned long long *)&ms.volC[D], (unsigned long long)(-leave));
                if (ms.volCp) atomicAdd((unsigned long long *)&ms.volCp[ms.sig[D]], (unsigned long long)(-leave));
            }
        }
        if (sk) {
            mvol = wave_sum(mvol);
            if (lane_id() == 0 && mvol) atomicAdd(&ms.sctl[1], (unsigned long long)(2 * mvol));
        }
    }
    moved = wave_sum(moved);
    if (lane_id() == 0) red[threadIdx.x / kWave] = moved;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t m = 0;
        for (int w = 0; w < kHubThreads / kWave; ++w) m += red[w];
        if (m) atomicAdd(ms.moves_dev, (unsigned long long)m);
    }
}

__global__ void k_node_recs(GraphView g, const int32_t *class_nodes, int64_t count, NodeRec *rec, const int32_t *sig) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = class_nodes[i];
        const int64_t e0 = g.off[u];
        rec[i] = NodeRec{e0, (int32_t)(g.off[u + 1] - e0), u, sig ? sig[u] : u, 0};
    }
}

void launch_node_recs(const GraphView &g, const int32_t *class_nodes, int64_t count, NodeRec *rec, const int32_t *sig,
                      hipStream_t st) {
    if (count <= 0) return;
    const int64_t blocks = cdiv(count, 256);
    hipLaunchKernelGGL(k_node_recs, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(256), 0, st, g, class_nodes,
                       count, rec, sig);
    HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------------ sweep layout
__global__ void k_layout_keys(GraphView g, uint32_t *keys, int32_t *vals) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < g.n; u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = g.off[u + 1] - g.off[u];
        keys[u] = ~(uint32_t)(d < (int64_t)UINT32_MAX ? d : (int64_t)UINT32_MAX);  // descending degree
        vals[u] = (int32_t)u;
    }
}
__global__ void k_layout_inverse(int64_t n, const int32_t *ord, int32_t *sig) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        sig[ord[i]] = (int32_t)i;
}
__global__ void k_layout_col(const int32_t *col, int64_t nnz, const int32_t *sig, int32_t *colp) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
        colp[e] = sig[col[e]];
}
__global__ void k_layout_sync(int64_t n, const int32_t *zeta, const int64_t *volC, const int32_t *sig, int32_t *zetap,
                              int64_t *volCp) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const int32_t s = sig[u];
        zetap[s] = sig[zeta[u]];
        volCp[s] = volC[u];
    }
}

void build_layout(const GraphView &g, int32_t *sig, int32_t *ord, int32_t *colp, uint32_t *keys, int32_t *vals,
                  uint32_t *keys_alt, int32_t *vals_alt, void *rs, hipStream_t st) {
    const int64_t n = g.n;
    if (n <= 0) return;
    const unsigned nb = (unsigned)(cdiv(n, 256) < 8192 ? cdiv(n, 256) : 8192);
    hipLaunchKernelGGL(k_layout_keys, dim3(nb), dim3(256), 0, st, g, keys, vals);
    // a stable sort: equal degrees keep ascending ids
    radix_sort_u32_i32(&keys, &vals, &keys_alt, &vals_alt, n, 32, rs, st);
    HIPCHK(hipMemcpyAsync(ord, vals, n * 4, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_layout_inverse, dim3(nb), dim3(256), 0, st, n, (const int32_t *)ord, sig);
    if (g.nnz > 0) {
        const int64_t eb = cdiv(g.nnz, 256);
        hipLaunchKernelGGL(k_layout_col, dim3((unsigned)(eb < 16384 ? eb : 16384)), dim3(256), 0, st, g.col, g.nnz,
                           (const int32_t *)sig, colp);
    }
    HIPCHK(hipGetLastError());
}

void sync_layout(int64_t n, const int32_t *zeta, const int64_t *volC, const int32_t *sig, int32_t *zetap,
                 int64_t *volCp, hipStream_t st) {
    if (n <= 0) return;
    const unsigned nb = (unsigned)(cdiv(n, 256) < 8192 ? cdiv(n, 256) : 8192);
    hipLaunchKernelGGL(k_layout_sync, dim3(nb), dim3(256), 0, st, n, zeta, volC, sig, zetap, volCp);
    HIPCHK(hipGetLastError());
}

// launch plans of the level-wide hub lists: one thread per workgroup record
__global__ void k_hub_plans(GraphView g, HubArrays ha, const int32_t *sig, const int64_t *ins_abs,
                            const int64_t *agg_abs, const int64_t *red_abs, int64_t n_sgl, int64_t n_ins,
                            int64_t n_agg, int64_t n_red, HubSglPlan *sp, HubPartPlan *pp, HubAggPlan *ap,
                            HubRedPlan *rp) {
    const int64_t tot = n_sgl + n_ins + n_agg + n_red;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < n_sgl) {
            const int32_t hg = ha.sgl_hub[i], u = ha.hub_u[hg];
            sp[i] = HubSglPlan{g.off[u], g.off[u + 1], u, ha.hub_pos[hg], sig ? sig[u] : u, 0};
            continue;
        }
        int64_t j = i - n_sgl;
        if (j < n_ins) {
            const int32_t hg = ha.ins_hub[j], u = ha.hub_u[hg];
            const int64_t k = j - ins_abs[hg], e0 = g.off[u], e1 = g.off[u + 1];
            const int64_t c0 = e0 + k * kHubInsChunk, c1 = c0 + kHubInsChunk < e1 ? c0 + kHubInsChunk : e1;
            pp[j] = HubPartPlan{c0, ha.stg_off[hg] + k * kHubInsChunk, ha.bkt_off[hg], u, hg, (int32_t)k,
                                (int32_t)(c1 - c0), ha.nchunk[hg], ha.pbits[hg], ha.hub_pos[hg], sig ? sig[u] : u};
            continue;
        }
        j -= n_ins;
        if (j < n_agg) {
            const int32_t hg = ha.agg_hub[j], u = ha.hub_u[hg];
            const int64_t p = j - agg_abs[hg];
            const int32_t nch = ha.nchunk[hg];
            ap[j] = HubAggPlan{ha.bkt_off[hg] + p * nch, ha.stg_off[hg], ha.ins_first[hg], u, hg, (int32_t)p, nch,
                               sig ? sig[u] : u, 0};
            continue;
        }
        j -= n_agg;
        const int32_t hg = ha.red_hub[j], u = ha.hub_u[hg];
        const int64_t k = j - red_abs[hg], e1 = g.off[u + 1];
        const int64_t s0 = g.off[u] + k * kHubMarkSlice, s1 = s0 + kHubMarkSlice < e1 ? s0 + kHubMarkSlice : e1;
        rp[j] = HubRedPlan{ha.agg_first[hg], ha.ins_first[hg], s0, s1, u, hg, 1 << ha.pbits[hg], ha.nchunk[hg],
                           (int32_t)k, sig ? sig[u] : u};
    }
}

void launch_hub_plans(const GraphView &g, const HubArrays &ha, const int32_t *sig, const int64_t *ins_abs,
                      const int64_t *agg_abs, const int64_t *red_abs, int64_t n_sgl, int64_t n_ins, int64_t n_agg,
                      int64_t n_red, HubSglPlan *sp, HubPartPlan *pp, HubAggPlan *ap, HubRedPlan *rp,
                      hipStream_t st) {
    const int64_t tot = n_sgl + n_ins + n_agg + n_red;
    if (tot <= 0) return;
    const int64_t blocks = cdiv(tot, 256);
    hipLaunchKernelGGL(k_hub_plans, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, st, g, ha, sig,
                       ins_abs, agg_abs, red_abs, n_sgl, n_ins, n_agg, n_red, sp, pp, ap, rp);
    HIPCHK(hipGetLastError());
}

// row length of each hub, negated when vol(u) does not fit 32 bits
__global__ void k_hub_degrees(GraphView g, const int32_t *class_nodes, const int64_t *vol, int64_t begin,
                              int64_t count, int64_t *deg, int32_t *uo) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    int32_t u = class_nodes[begin + i];
    int64_t d = g.off[u + 1] - g.off[u];
    deg[i] = vol[u] > (int64_t)INT32_MAX ? -d : d;
    uo[i] = u;
}

// ------------------------------------------------------------------ launchers
// A dispatch with start/stop events attached when either is given, else a plain
// launch (the form stream capture records).
template <typename... Params, typename... Args>
static void dispatch(void (*kernel)(Params...), dim3 grid, dim3 block, hipStream_t st, hipEvent_t start,
                     hipEvent_t stop, Args... args) {
    if (start || stop)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, st, start, stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
}

template <int WK, bool LP>
static void class_step_wk(const GraphView &g, const MoveState &ms, const ClassRange &cr, const HubArrays &ha,
                          int fw, const hipEvent_t *ev, unsigned ev_mask, unsigned groups, hipStream_t st) {
    // start / stop events of kernel group i (taken by the dispatch itself)
    auto t0 = [&](int i) { return (ev && ((ev_mask >> i) & 1u)) ? ev[2 * i] : (hipEvent_t) nullptr; };
    auto t1 = [&](int i) { return (ev && ((ev_mask >> i) & 1u)) ? ev[2 * i + 1] : (hipEvent_t) nullptr; };
    if (cr.count[0] > 0 && (groups & 1u))
        dispatch(k_decide_lane<WK, LP>, dim3((unsigned)cdiv(cr.count[0], 256)), dim3(256), st, t0(0), t1(0), g, ms,
                 cr.begin[0], cr.count[0], fw);
    if (cr.count[1] > 0 && (groups & 2u)) {
        // short rows (16 lanes per node) first, then a wavefront per node; the
        // group's start event goes on its first launch, the stop on its last
        const int64_t nq = cr.quad, nw = cr.count[1] - cr.quad;
        if (nq > 0) {
            int64_t blocks = cdiv(nq, 256 / kQuadLanes);
            dispatch(k_decide_quad<WK, LP>, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(256), st, t0(1),
                     nw > 0 ? (hipEvent_t) nullptr : t1(1), g, ms, cr.begin[1], nq, fw);
        }
        if (nw > 0) {
            int64_t blocks = cdiv(nw, 4);
            dispatch(k_decide_wave<WK, LP>, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(256), st,
                     nq > 0 ? (hipEvent_t) nullptr : t0(1), t1(1), g, ms, cr.begin[1] + nq, nw, fw);
        }
    }
    if (cr.count[2] > 0 && (groups & 4u)) {
        // rows of at most kBlockShortRow entries first; the group's start event
        // goes on its first launch, the stop on its last
        const int64_t ns = cr.blk_short, nl = cr.count[2] - cr.blk_short;
        if (ns > 0)
            dispatch(k_decide_block<WK, LP, kBlockShortThreads, kBlockShortCap>,
                     dim3((unsigned)(ns < 4096 ? ns : 4096)), dim3(kBlockShortThreads), st, t0(2),
                     nl > 0 ? (hipEvent_t) nullptr : t1(2), g, ms, cr.begin[2], ns, fw);
        if (nl > 0)
            dispatch(k_decide_block<WK, LP, kBlockThreads, kBlockCap>, dim3((unsigned)(nl < 2048 ? nl : 2048)),
                     dim3(kBlockThreads), st, ns > 0 ? (hipEvent_t) nullptr : t0(2), t1(2), g, ms,
                     cr.begin[2] + ns, nl, fw);
    }
    if (cr.sgl_count > 0 && (groups & 8u))
        dispatch(k_hub_single<WK, LP>, dim3((unsigned)cr.sgl_count), dim3(kSingleThreads), st, t0(3), t1(3), g, ms,
                 ha, cr.sgl_base, fw);
    if (cr.red_count > 0 && (groups & 16u)) {
        // the partitioned group is timed per launch (events 8, 9 and 10, 11), so
        // that the gap between its two dependent launches is not counted
        const bool t4 = ev && ((ev_mask >> 4) & 1u);
        dispatch(k_hub_part<WK, LP>, dim3((unsigned)cr.ins_blocks), dim3(kHubThreads), st, t4 ? ev[8] : nullptr,
                 t4 ? ev[9] : nullptr, g, ms, ha, cr.ins_base);
        dispatch(k_hub_agg<WK, LP>, dim3((unsigned)cr.agg_blocks), dim3(kHubThreads), st, t4 ? ev[10] : nullptr,
                 t4 ? ev[11] : nullptr, ms, ha, cr.agg_base, fw);
    }
}

void launch_class_step(const GraphView &g, const MoveState &ms, const ClassRange &cr, const HubArrays &ha,
                       bool force_wide, const hipEvent_t *ev, unsigned ev_mask, hipStream_t st, unsigned groups) {
    int fw = force_wide ? 1 : 0;
    const bool lp = ms.active != nullptr;
    switch (g.wkind) {
        case 0:
            if (lp) class_step_wk<0, true>(g, ms, cr, ha, fw, ev, ev_mask, groups, st);
            else class_step_wk<0, false>(g, ms, cr, ha, fw, ev, ev_mask, groups, st);
            break;
        case 1:
            if (lp) class_step_wk<1, true>(g, ms, cr, ha, fw, ev, ev_mask, groups, st);
            else class_step_wk<1, false>(g, ms, cr, ha, fw, ev, ev_mask, groups, st);
            break;
        default:
            if (lp) class_step_wk<2, true>(g, ms, cr, ha, fw, ev, ev_mask, groups, st);
            else class_step_wk<2, false>(g, ms, cr, ha, fw, ev, ev_mask, groups, st);
            break;
    }
    HIPCHK(hipGetLastError());
}

void launch_apply(const GraphView &g, const MoveState &ms, const HubArrays &ha, const ClassRange &cr,
                  hipStream_t st) {
    const int64_t begin = cr.begin[0], count = cr.begin[3] + cr.count[3] - cr.begin[0];
    if (count <= 0) return;
    const int64_t ab = cdiv(count, kHubThreads);
    const int64_t blocks = cr.red_count + (ab < 2048 ? ab : 2048);
    if (ms.active)
        hipLaunchKernelGGL(k_reduce_apply<true>, dim3((unsigned)blocks), dim3(kHubThreads), 0, st, g, ms, ha,
                           cr.red_base, cr.red_count, begin, count);
    else
        hipLaunchKernelGGL(k_reduce_apply<false>, dim3((unsigned)blocks), dim3(kHubThreads), 0, st, g, ms, ha,
                           cr.red_base, cr.red_count, begin, count);
    HIPCHK(hipGetLastError());
}

void launch_hub_degrees(const GraphView &g, const int32_t *class_nodes, const int64_t *vol, int64_t begin,
                        int64_t count, int64_t *deg_out, int32_t *u_out, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_hub_degrees, dim3((unsigned)cdiv(count, 256)), dim3(256), 0, st, g, class_nodes, vol, begin,
                       count, deg_out, u_out);
    HIPCHK(hipGetLastError());
}

}  // namespace plm
