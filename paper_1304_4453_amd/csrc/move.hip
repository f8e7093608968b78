// move.hip - the move-decide and apply kernels of one colour class
// (Algorithm 2 under the colour-class schedule).
//
// For node u in community D every neighbouring community X != D is scored by
//   gain(X) = S (w(u,X) - w(u,D\u)) - vol(u) (vol(X) - vol(D\u))
// (2 w(E)^2 times Delta-mod of section III-B).  The kernels rank candidates by
//   s(X) = S w(u,X) - vol(u) vol(X)
// which differs from gain(X) by the constant K = S w(u,D\u) - vol(u) vol(D\u),
// so the best candidate is the same and the move happens iff s_best > K.
// |s|, |K| <= S vol(u): 64-bit arithmetic is exact while S vol(u) < 2^62,
// otherwise the node takes the 128-bit path.  Ties go to the lowest X.
//
// Degree bins: rows up to 16 entries are handled one lane per node (register
// arrays), up to the wave limit one wavefront per node (LDS hash table), up to
// the block limit one workgroup per node (LDS hash table), and longer rows
// ("hubs") by several workgroups per node through a global hash table.
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

__device__ __forceinline__ void count_candidates(unsigned long long *cand, int64_t c) {
    if (!cand) return;
    c = wave_sum(c);
    if (lane_id() == 0 && c) atomicAdd(cand, (unsigned long long)c);
}

// ------------------------------------------------------------------ lane per node
constexpr int kLaneMax = 16;

template <int WK, typename G>
__device__ __forceinline__ int32_t lane_pick(const int32_t (&X)[kLaneMax], const int64_t (&W)[kLaneMax], int32_t D,
                                             int64_t wD, int64_t vu, int64_t base, int64_t S, const int64_t *volC) {
    G bg = 0;
    int32_t bx = kNone;
#pragma unroll
    for (int j = 0; j < kLaneMax; ++j) {
        if (X[j] >= 0 && X[j] != D) {
            G g = (G)S * (G)(W[j] - wD) - (G)vu * (G)(volC[X[j]] - base);
            if (g > 0 && (g > bg || (g == bg && X[j] < bx))) { bg = g; bx = X[j]; }
        }
    }
    return bx;
}

template <int WK>
__global__ __launch_bounds__(256) void k_decide_lane(GraphView g, MoveState ms, int64_t begin, int64_t count,
                                                     int force_wide) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t ncand = 0;
    if (i < count) {
        int64_t pos = begin + i;
        int32_t u = ms.class_nodes[pos];
        int64_t e0 = g.off[u];
        int64_t d = g.off[u + 1] - e0;
        int32_t X[kLaneMax];
        int64_t W[kLaneMax];
#pragma unroll
        for (int j = 0; j < kLaneMax; ++j) {
            X[j] = -1;
            W[j] = 0;
            if (j < d) {
                int32_t v = g.col[e0 + j];
                if (v != u) {
                    X[j] = ms.zeta[v];
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
        int32_t D = ms.zeta[u];
        int64_t wD = 0;
#pragma unroll
        for (int j = 0; j < kLaneMax; ++j) {
            if (X[j] == D) wD = W[j];
            ncand += (X[j] >= 0 && X[j] != D);
        }
        int64_t vu = ms.vol[u];
        int64_t base = ms.volC[D] - vu;
        int32_t bx = (force_wide || vu > ms.wide_lim) ? lane_pick<WK, i128>(X, W, D, wD, vu, base, ms.S, ms.volC)
                                                      : lane_pick<WK, int64_t>(X, W, D, wD, vu, base, ms.S, ms.volC);
        ms.move_to[pos] = (bx == kNone) ? -1 : bx;
    }
    count_candidates(ms.cand_dev ? ms.cand_dev + 0 : nullptr, ncand);
}

// ------------------------------------------------------------------ wavefront per node
// Entries whose neighbour is already in u's own community D are summed in
// registers (w(u, D\u) is needed on its own anyway) and never enter the hash
// table: on graphs where many neighbours have joined u, the table would
// otherwise serialise on that one key.
constexpr int kWaveCap = 1024;  // slots per wavefront (rows up to 512 entries)

template <typename G>
__device__ __forceinline__ void wave_eval(int32_t *tk, int64_t *tv, int tsize, int64_t wD, int64_t vu, int64_t base,
                                          int64_t S, const int64_t *volC, int32_t &best_x, bool &move,
                                          int64_t &ncand) {
    G bs = neg_inf<G>();
    int32_t bx = kNone;
    for (int s = lane_id(); s < tsize; s += kWave) {
        int32_t X = tk[s];
        if (X >= 0) {
            int64_t a = tv[s];
            tk[s] = kEmpty;
            tv[s] = 0;
            ++ncand;
            G sc = (G)S * (G)a - (G)vu * (G)volC[X];
            if (sc > bs || (sc == bs && X < bx)) { bs = sc; bx = X; }
        }
    }
    wave_argmax<G>(bs, bx);
    G K = (G)S * (G)wD - (G)vu * (G)base;
    best_x = bx;
    move = bx != kNone && bs > K;
}

// folds the (X, w) entries of u into a hash table (LDS) except X == D; returns
// this thread's share of w(u, D \ u).  Entries are taken B at a time: B column
// loads, then B community gathers, then B inserts, so that the memory
// latencies of a batch overlap.
template <int WK, int B>
__device__ __forceinline__ int64_t fold_row(const GraphView &g, const int32_t *zeta, int32_t u, int32_t D, int64_t e0,
                                            int64_t e1, int64_t first, int64_t step, int32_t *tk, int64_t *tv,
                                            int bits) {
    const uint32_t mask = (1u << bits) - 1;
    int64_t myD = 0;
    for (int64_t base = e0 + first; base < e1; base += step * B) {
        int32_t v[B], X[B];
        int64_t wt[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            int64_t e = base + b * step;
            bool ok = e < e1;
            v[b] = ok ? g.col[e] : u;
            wt[b] = ok ? wload<WK>(g.w, e) : 0;
        }
#pragma unroll
        for (int b = 0; b < B; ++b) X[b] = v[b] != u ? zeta[v[b]] : -1;
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
                    atomicAdd((unsigned long long *)&tv[h], (unsigned long long)wt[b]);
                    break;
                }
                h = (h + 1) & mask;
            }
        }
    }
    return myD;
}

template <int WK>
__global__ __launch_bounds__(256) void k_decide_wave(GraphView g, MoveState ms, int64_t begin, int64_t count,
                                                     int force_wide) {
    __shared__ int32_t tk[4][kWaveCap];
    __shared__ int64_t tv[4][kWaveCap];
    const int w = threadIdx.x / kWave, lane = lane_id();
    for (int s = lane; s < kWaveCap; s += kWave) { tk[w][s] = kEmpty; tv[w][s] = 0; }
    wave_sync();
    int64_t ncand = 0;
    for (int64_t i = (int64_t)blockIdx.x * 4 + w; i < count; i += (int64_t)gridDim.x * 4) {
        int64_t pos = begin + i;
        int32_t u = ms.class_nodes[pos];
        int64_t e0 = g.off[u], e1 = g.off[u + 1];
        int bits = ceil_log2_dev(2 * (e1 - e0));
        bits = bits < 6 ? 6 : bits;
        int32_t D = ms.zeta[u];
        int64_t wD = fold_row<WK, 4>(g, ms.zeta, u, D, e0, e1, lane, kWave, tk[w], tv[w], bits);
        wD = wave_sum(wD);
        wave_sync();
        int64_t vu = ms.vol[u];
        int64_t base = ms.volC[D] - vu;
        int32_t bx;
        bool mv;
        if (force_wide || vu > ms.wide_lim)
            wave_eval<i128>(tk[w], tv[w], 1 << bits, wD, vu, base, ms.S, ms.volC, bx, mv, ncand);
        else
            wave_eval<int64_t>(tk[w], tv[w], 1 << bits, wD, vu, base, ms.S, ms.volC, bx, mv, ncand);
        if (lane == 0) ms.move_to[pos] = mv ? bx : -1;
        wave_sync();
    }
    count_candidates(ms.cand_dev ? ms.cand_dev + 1 : nullptr, ncand);
}

// ------------------------------------------------------------------ workgroup per node
constexpr int kBlockThreads = 512;
constexpr int kBlockCap = 8192;  // rows up to 4096 entries

template <typename G>
__device__ __forceinline__ void block_eval(int32_t *tk, int64_t *tv, int tsize, int64_t wD, int64_t vu, int64_t base,
                                           int64_t S, const int64_t *volC, int32_t *out, int64_t &ncand) {
    __shared__ int64_t red_w[kBlockThreads / kWave];
    __shared__ G red_s[kBlockThreads / kWave];
    __shared__ int32_t red_x[kBlockThreads / kWave];
    G bs = neg_inf<G>();
    int32_t bx = kNone;
    for (int s = threadIdx.x; s < tsize; s += kBlockThreads) {
        int32_t X = tk[s];
        if (X >= 0) {
            int64_t a = tv[s];
            tk[s] = kEmpty;
            tv[s] = 0;
            ++ncand;
            G sc = (G)S * (G)a - (G)vu * (G)volC[X];
            if (sc > bs || (sc == bs && X < bx)) { bs = sc; bx = X; }
        }
    }
    wD = wave_sum(wD);  // wD enters as this thread's share
    wave_argmax<G>(bs, bx);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) { red_w[w] = wD; red_s[w] = bs; red_x[w] = bx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int j = 1; j < kBlockThreads / kWave; ++j) {
            wD += red_w[j];
            if (red_s[j] > bs || (red_s[j] == bs && red_x[j] < bx)) { bs = red_s[j]; bx = red_x[j]; }
        }
        G K = (G)S * (G)wD - (G)vu * (G)base;
        *out = (bx != kNone && bs > K) ? bx : -1;
    }
}

template <int WK>
__global__ __launch_bounds__(kBlockThreads) void k_decide_block(GraphView g, MoveState ms, int64_t begin,
                                                                int64_t count, int force_wide) {
    __shared__ int32_t tk[kBlockCap];
    __shared__ int64_t tv[kBlockCap];
    for (int s = threadIdx.x; s < kBlockCap; s += kBlockThreads) { tk[s] = kEmpty; tv[s] = 0; }
    __syncthreads();
    int64_t ncand = 0;
    for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
        int64_t pos = begin + i;
        int32_t u = ms.class_nodes[pos];
        int64_t e0 = g.off[u], e1 = g.off[u + 1];
        int bits = ceil_log2_dev(2 * (e1 - e0));
        bits = bits < 6 ? 6 : bits;
        int32_t D = ms.zeta[u];
        int64_t myD = fold_row<WK, 4>(g, ms.zeta, u, D, e0, e1, threadIdx.x, kBlockThreads, tk, tv, bits);
        __syncthreads();
        int64_t vu = ms.vol[u];
        int64_t base = ms.volC[D] - vu;
        if (force_wide || vu > ms.wide_lim)
            block_eval<i128>(tk, tv, 1 << bits, myD, vu, base, ms.S, ms.volC, &ms.move_to[pos], ncand);
        else
            block_eval<int64_t>(tk, tv, 1 << bits, myD, vu, base, ms.S, ms.volC, &ms.move_to[pos], ncand);
        __syncthreads();
    }
    count_candidates(ms.cand_dev ? ms.cand_dev + 2 : nullptr, ncand);
}

// ------------------------------------------------------------------ hubs: several workgroups per node
// Rows longer than the workgroup limit accumulate w(u, X) in a per-node hash
// table in global memory.  Insert: each workgroup first folds a chunk of
// kHubInsChunk entries into an LDS table, then adds its distinct communities
// to the node's global table; a key that a workgroup creates is appended to the
// node's list of occupied slots.  Eval: workgroups walk the occupied list
// (clearing the slots), each leaves a partial best, and a third launch (one
// workgroup per node) combines them.  When every partial sum of the level fits 32 bits (max
// vol(u) < 2^32) a global slot is one 64-bit word (community << 32 | weight);
// otherwise keys and 64-bit values sit in two arrays.
constexpr int kHubThreads = 256;
constexpr int kHubLdsSlots = 4096;  // LDS table of an insert workgroup (2 x kHubInsChunk)
constexpr uint64_t kEmptyWord = 0xFFFFFFFF00000000ULL;

// hub h of a class owning class-relative block b: last h with first[h] <= b
__device__ __forceinline__ int64_t hub_of_block(const int64_t *first, int64_t nh, int64_t b) {
    int64_t lo = 0, hi = nh;
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (first[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// continues the linear probe for key X from slot s + 1 (slot s held another
// key); true if this call created the key; *slot_out = the key's slot
template <bool PACKED>
__device__ __noinline__ bool global_probe(const HubArrays &ha, int64_t hg, int32_t X, int64_t a, uint32_t mask,
                                          uint32_t s, uint32_t *slot_out) {
    for (;;) {
        s = (s + 1) & mask;
        if constexpr (PACKED) {
            unsigned long long *tw = (unsigned long long *)ha.tab_val + ha.tab_off[hg];
            const unsigned long long want = ((unsigned long long)(uint32_t)X << 32) | (unsigned long long)a;
            unsigned long long old = atomicCAS(&tw[s], kEmptyWord, want);
            if (old == kEmptyWord) { *slot_out = s; return true; }
            if ((uint32_t)(old >> 32) == (uint32_t)X) {
                atomicAdd(&tw[s], (unsigned long long)a);
                *slot_out = s;
                return false;
            }
        } else {
            int32_t *tk = ha.tab_key + ha.tab_off[hg];
            int64_t *tv = ha.tab_val + ha.tab_off[hg];
            int32_t k = atomicCAS(&tk[s], kEmpty, X);
            if (k == kEmpty || k == X) {
                atomicAdd((unsigned long long *)&tv[s], (unsigned long long)a);
                *slot_out = s;
                return k == kEmpty;
            }
        }
    }
}

template <int WK, bool PACKED>
__global__ __launch_bounds__(kHubThreads) void k_hub_insert(GraphView g, MoveState ms, HubArrays ha, int64_t hub0,
                                                            int64_t nh) {
    __shared__ int32_t lk[kHubLdsSlots];
    __shared__ int64_t lv[kHubLdsSlots];
    for (int s = threadIdx.x; s < kHubLdsSlots; s += kHubThreads) { lk[s] = kEmpty; lv[s] = 0; }
    int64_t h = hub_of_block(ha.ins_first + hub0, nh, blockIdx.x);
    int64_t hg = hub0 + h;
    int64_t chunk = blockIdx.x - ha.ins_first[hg];
    int32_t u = ms.class_nodes[ha.hub_pos[hg]];
    int64_t e0 = g.off[u], e1 = g.off[u + 1];
    int64_t c0 = e0 + chunk * kHubInsChunk, c1 = c0 + kHubInsChunk < e1 ? c0 + kHubInsChunk : e1;
    __syncthreads();
    constexpr int kLdsBits = 12;
    const int32_t D = ms.zeta[u];
    int64_t myD = fold_row<WK, 8>(g, ms.zeta, u, D, c0, c1, threadIdx.x, kHubThreads, lk, lv, kLdsBits);
    myD = wave_sum(myD);
    if (lane_id() == 0 && myD) atomicAdd((unsigned long long *)&ha.hub_wD[hg], (unsigned long long)myD);
    __syncthreads();
    // flush: every thread takes kFlush LDS slots, issues the CAS of each non-empty
    // one on its home slot at once, then resolves the (rare) collisions
    const int bits = ha.tab_bits[hg];
    const uint32_t mask = (1u << bits) - 1;
    int32_t *occ = ha.occ + (ha.tab_off[hg] >> 1);
    const int lane = lane_id();
    const uint64_t lt = (lane == 0) ? 0ULL : (~0ULL >> (64 - lane));
    constexpr int kFlush = kHubLdsSlots / kHubThreads;
    int32_t X[kFlush];
    int64_t a[kFlush];
    uint32_t slot[kFlush];
    bool created[kFlush];
#pragma unroll
    for (int j = 0; j < kFlush; ++j) {
        X[j] = lk[j * kHubThreads + threadIdx.x];
        a[j] = lv[j * kHubThreads + threadIdx.x];
        slot[j] = X[j] >= 0 ? slot_hash(X[j], bits) : 0;
        created[j] = false;
    }
    if constexpr (PACKED) {
        unsigned long long *tw = (unsigned long long *)ha.tab_val + ha.tab_off[hg];
        unsigned long long old[kFlush];
#pragma unroll
        for (int j = 0; j < kFlush; ++j)
            if (X[j] >= 0)
                old[j] = atomicCAS(&tw[slot[j]], kEmptyWord,
                                   ((unsigned long long)(uint32_t)X[j] << 32) | (unsigned long long)a[j]);
#pragma unroll
        for (int j = 0; j < kFlush; ++j) {
            if (X[j] < 0) continue;
            if (old[j] == kEmptyWord) created[j] = true;
            else if ((uint32_t)(old[j] >> 32) == (uint32_t)X[j]) atomicAdd(&tw[slot[j]], (unsigned long long)a[j]);
            else created[j] = global_probe<true>(ha, hg, X[j], a[j], mask, slot[j], &slot[j]);
        }
    } else {
        int32_t *tk = ha.tab_key + ha.tab_off[hg];
        int64_t *tv = ha.tab_val + ha.tab_off[hg];
        int32_t old[kFlush];
#pragma unroll
        for (int j = 0; j < kFlush; ++j)
            if (X[j] >= 0) old[j] = atomicCAS(&tk[slot[j]], kEmpty, X[j]);
#pragma unroll
        for (int j = 0; j < kFlush; ++j) {
            if (X[j] < 0) continue;
            if (old[j] == kEmpty || old[j] == X[j]) {
                atomicAdd((unsigned long long *)&tv[slot[j]], (unsigned long long)a[j]);
                created[j] = old[j] == kEmpty;
            } else {
                created[j] = global_probe<false>(ha, hg, X[j], a[j], mask, slot[j], &slot[j]);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kFlush; ++j) {
        uint64_t m = __ballot(created[j]);
        if (m) {
            int leader = __ffsll((unsigned long long)m) - 1;
            int32_t base = 0;
            if (lane == leader) base = atomicAdd(&ha.occ_cnt[hg], (int32_t)__popcll(m));
            base = __shfl(base, leader);
            if (created[j]) occ[base + (int32_t)__popcll(m & lt)] = (int32_t)slot[j];
        }
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

template <typename G, bool PACKED>
__device__ __forceinline__ void hub_slots_best(const HubArrays &ha, int64_t hg, const int32_t *occ, int64_t i0,
                                               int64_t i1, int32_t D, int64_t vu, int64_t S, const int64_t *volC,
                                               int64_t *wD_slot, G &bs, int32_t &bx, int64_t &ncand) {
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kHubThreads) {
        int32_t s = occ[i];
        int32_t X;
        int64_t a;
        if constexpr (PACKED) {
            unsigned long long *tw = (unsigned long long *)ha.tab_val + ha.tab_off[hg];
            unsigned long long word = tw[s];
            tw[s] = kEmptyWord;
            X = (int32_t)(word >> 32);
            a = (int64_t)(word & 0xffffffffULL);
        } else {
            int32_t *tk = ha.tab_key + ha.tab_off[hg];
            int64_t *tv = ha.tab_val + ha.tab_off[hg];
            X = tk[s];
            a = tv[s];
            tk[s] = kEmpty;
            tv[s] = 0;
        }
        ++ncand;  // the tables never hold D (summed into hub_wD by the insert launch)
        G sc = (G)S * (G)a - (G)vu * (G)volC[X];
        if (sc > bs || (sc == bs && X < bx)) { bs = sc; bx = X; }
    }
}

template <bool PACKED>
__global__ __launch_bounds__(kHubThreads) void k_hub_eval(GraphView g, MoveState ms, HubArrays ha, int64_t hub0,
                                                          int64_t nh, int force_wide) {
    int64_t h = hub_of_block(ha.eval_first + hub0, nh, blockIdx.x);
    int64_t hg = hub0 + h;
    int64_t chunk = blockIdx.x - ha.eval_first[hg];
    int64_t pos = ha.hub_pos[hg];
    int32_t u = ms.class_nodes[pos];
    int32_t D = ms.zeta[u];
    int64_t vu = ms.vol[u];
    bool wide = force_wide || vu > ms.wide_lim;
    const int32_t *occ = ha.occ + (ha.tab_off[hg] >> 1);
    int64_t nocc = ha.occ_cnt[hg];
    int64_t i0 = chunk * kHubEvalChunk, i1 = i0 + kHubEvalChunk < nocc ? i0 + kHubEvalChunk : nocc;
    int64_t ncand = 0;
    unsigned long long *part = ha.part + 4 * (size_t)blockIdx.x;
    i128 bs = neg_inf<i128>();
    int32_t bx = kNone;
    if (wide) {
        hub_slots_best<i128, PACKED>(ha, hg, occ, i0, i1, D, vu, ms.S, ms.volC, &ha.hub_wD[hg], bs, bx, ncand);
        block_argmax<i128>(bs, bx);
    } else {
        int64_t b64 = neg_inf<int64_t>();
        hub_slots_best<int64_t, PACKED>(ha, hg, occ, i0, i1, D, vu, ms.S, ms.volC, &ha.hub_wD[hg], b64, bx, ncand);
        block_argmax<int64_t>(b64, bx);
        bs = (i128)b64;
    }
    if (threadIdx.x == 0) {
        part[0] = (unsigned long long)(uint64_t)(bs >> 64);
        part[1] = (unsigned long long)(uint64_t)bs;
        part[2] = (unsigned long long)(uint32_t)bx;
    }
    count_candidates(ms.cand_dev ? ms.cand_dev + 3 : nullptr, ncand);
}

// One workgroup per hub of the class combines the eval partials (written by
// the previous launch, so no fence is needed) and decides the move.
__global__ __launch_bounds__(kHubThreads) void k_hub_reduce(MoveState ms, HubArrays ha, int64_t hub0) {
    int64_t hg = hub0 + blockIdx.x;
    int64_t nblk = ha.eval_cnt[hg];
    const unsigned long long *p0 = ha.part + 4 * (size_t)ha.eval_first[hg];
    i128 bs = neg_inf<i128>();
    int32_t bx = kNone;
    for (int64_t j = threadIdx.x; j < nblk; j += kHubThreads) {
        int32_t x = (int32_t)p0[4 * j + 2];
        i128 s = (i128)(((unsigned __int128)p0[4 * j + 0] << 64) | p0[4 * j + 1]);
        if (x != kNone && (s > bs || (s == bs && x < bx))) { bs = s; bx = x; }
    }
    block_argmax<i128>(bs, bx);
    if (threadIdx.x == 0) {
        int64_t pos = ha.hub_pos[hg];
        int32_t u = ms.class_nodes[pos];
        int32_t D = ms.zeta[u];
        int64_t vu = ms.vol[u];
        int64_t wD = ha.hub_wD[hg];
        int64_t base = ms.volC[D] - vu;
        i128 K = (i128)ms.S * (i128)wD - (i128)vu * (i128)base;
        ms.move_to[pos] = (bx != kNone && bs > K) ? bx : -1;
        ha.hub_wD[hg] = 0;
        ha.occ_cnt[hg] = 0;
    }
}

// ------------------------------------------------------------------ apply
__global__ __launch_bounds__(256) void k_apply(MoveState ms, int64_t begin, int64_t count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t moved = 0;
    if (i < count) {
        int64_t pos = begin + i;
        int32_t X = ms.move_to[pos];
        if (X >= 0) {
            int32_t u = ms.class_nodes[pos];
            int32_t D = ms.zeta[u];
            int64_t vu = ms.vol[u];
            ms.zeta[u] = X;
            atomicAdd((unsigned long long *)&ms.volC[D], (unsigned long long)(-vu));
            atomicAdd((unsigned long long *)&ms.volC[X], (unsigned long long)vu);
            moved = 1;
        }
    }
    moved = wave_sum(moved);
    if (lane_id() == 0 && moved) atomicAdd(ms.moves_dev, (unsigned long long)moved);
}

__global__ void k_hub_degrees(GraphView g, const int32_t *class_nodes, int64_t begin, int64_t count, int64_t *deg) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    int32_t u = class_nodes[begin + i];
    deg[i] = g.off[u + 1] - g.off[u];
}

// ------------------------------------------------------------------ launchers
template <int WK>
static void class_step_wk(const GraphView &g, const MoveState &ms, const ClassRange &cr, const HubArrays &ha,
                          int fw, const hipEvent_t *ev, hipStream_t st) {
    auto mark = [&](int i) {
        if (ev) HIPCHK(hipEventRecord(ev[i], st));
    };
    mark(0);
    if (cr.count[0] > 0)
        hipLaunchKernelGGL(k_decide_lane<WK>, dim3((unsigned)cdiv(cr.count[0], 256)), dim3(256), 0, st, g, ms,
                           cr.begin[0], cr.count[0], fw);
    mark(1);
    if (cr.count[1] > 0) {
        int64_t blocks = cdiv(cr.count[1], 4);
        hipLaunchKernelGGL(k_decide_wave<WK>, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(256), 0, st, g,
                           ms, cr.begin[1], cr.count[1], fw);
    }
    mark(2);
    if (cr.count[2] > 0) {
        int64_t blocks = cr.count[2];
        hipLaunchKernelGGL(k_decide_block<WK>, dim3((unsigned)(blocks < 2048 ? blocks : 2048)), dim3(kBlockThreads),
                           0, st, g, ms, cr.begin[2], cr.count[2], fw);
    }
    mark(3);
    if (cr.hub_count > 0) {
        if (ha.packed) {
            hipLaunchKernelGGL((k_hub_insert<WK, true>), dim3((unsigned)cr.ins_blocks), dim3(kHubThreads), 0, st, g,
                               ms, ha, cr.hub_first, cr.hub_count);
            hipLaunchKernelGGL(k_hub_eval<true>, dim3((unsigned)cr.eval_blocks), dim3(kHubThreads), 0, st, g, ms, ha,
                               cr.hub_first, cr.hub_count, fw);
            hipLaunchKernelGGL(k_hub_reduce, dim3((unsigned)cr.hub_count), dim3(kHubThreads), 0, st, ms, ha,
                               cr.hub_first);
        } else {
            hipLaunchKernelGGL((k_hub_insert<WK, false>), dim3((unsigned)cr.ins_blocks), dim3(kHubThreads), 0, st, g,
                               ms, ha, cr.hub_first, cr.hub_count);
            hipLaunchKernelGGL(k_hub_eval<false>, dim3((unsigned)cr.eval_blocks), dim3(kHubThreads), 0, st, g, ms,
                               ha, cr.hub_first, cr.hub_count, fw);
            hipLaunchKernelGGL(k_hub_reduce, dim3((unsigned)cr.hub_count), dim3(kHubThreads), 0, st, ms, ha,
                               cr.hub_first);
        }
    }
    mark(4);
}

void launch_class_step(const GraphView &g, const MoveState &ms, const ClassRange &cr, const HubArrays &ha,
                       bool force_wide, const hipEvent_t *ev, hipStream_t st) {
    int fw = force_wide ? 1 : 0;
    switch (g.wkind) {
        case 0: class_step_wk<0>(g, ms, cr, ha, fw, ev, st); break;
        case 1: class_step_wk<1>(g, ms, cr, ha, fw, ev, st); break;
        default: class_step_wk<2>(g, ms, cr, ha, fw, ev, st); break;
    }
    HIPCHK(hipGetLastError());
}

void launch_apply(const MoveState &ms, int64_t begin, int64_t count, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_apply, dim3((unsigned)cdiv(count, 256)), dim3(256), 0, st, ms, begin, count);
    HIPCHK(hipGetLastError());
}

void launch_hub_degrees(const GraphView &g, const int32_t *class_nodes, int64_t begin, int64_t count,
                        int64_t *deg_out, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_hub_degrees, dim3((unsigned)cdiv(count, 256)), dim3(256), 0, st, g, class_nodes, begin,
                       count, deg_out);
    HIPCHK(hipGetLastError());
}

}  // namespace plm
