// colour.hip - the priority colouring that fixes the move schedule.
//
// Colour of u = smallest colour not used by a higher-priority non-loop
// neighbour, priorities (H(seed, level, u), u).  Computed as Jones-Plassmann:
// pending(u) = number of higher-priority neighbours; a node whose count drops
// to 0 joins the next frontier; a frontier node takes the smallest free colour
// among its (all already coloured) higher-priority neighbours and decrements
// its lower-priority neighbours.  This is exactly the greedy colouring in
// descending priority order.
//
// Rounds run back to back on the device: each round is one launch over
// triple-buffered queues (round r reads set r%3, pushes into set (r+1)%3 and
// clears set (r+2)%3), so the host only checks for an empty frontier every few
// rounds.  Frontier nodes are split by row length: eight lanes per node (<= 32
// entries), one wavefront per node (<= 1024), and several workgroups per node
// above that; the latter OR the colours they see into a block-local LDS bitmap
// and merge it into a per-node global bitmap, from which the workgroup that
// finishes the row's last chunk picks the smallest free colour.  The three
// tiers of a round run on workgroups of their own.  Small frontiers run as
// back-to-back rounds inside one workgroup (the tail).  A round is bound by
// latency (its frontier is often small), so every lane loads a batch of
// entries before it gathers their colours, instead of walking a row one
// dependent load after another.
#include <hip/hip_runtime.h>

#include <cstring>

#include "level.h"

namespace plm {

constexpr int kCT = 256;                  // threads per workgroup
constexpr int64_t kLaneRow = 32;          // row length handled by eight lanes
constexpr int64_t kWaveRow = 1024;        // row length handled by one wavefront
constexpr int kWin = 4096;                // colour window of a bitmap (bits)
constexpr int kWinWords = kWin / 32;
constexpr int kRoundGrid = 2048;          // workgroups of a round launch
constexpr int kRoundsPerCheck = 16;       // rounds launched between host checks
constexpr int64_t kHubChunk = 4 * 256;    // entries of a long row per work item (4 per thread)

// counters, each on a 128-byte line of its own (the pushes of a round hit
// them from every XCD, and counters that share a line serialise each other):
// the four of set s (queue kinds 0..2, then chunks), then the number of
// colours, the uncoloured-node count (both written once, after the last
// round) and the round a tail launch reached
constexpr int kCntLine = 32;
__host__ __device__ __forceinline__ int cidx(int set, int kind) { return (set * 4 + kind) * kCntLine; }
constexpr int kCntNcol = 12 * kCntLine, kCntUncoloured = 13 * kCntLine, kCntTail = 14 * kCntLine;
constexpr int kCntWords = 15 * kCntLine;

// A work item of a long row: everything its workgroup indexes, so that the
// row's entries are its first dependent load
struct HubItem {
    int64_t c0, c1;           // entries of the chunk
    int32_t u, slot, nch, pad;  // node, queue slot (bitmap, chunk counter), chunks of the row
};

struct JpQ {
    int32_t *q[3][2];  // [set][kind]: 0 lane, 1 wavefront (long rows: cq)
    HubItem *cq[3];    // [set]: chunks of the multi-workgroup rows
    int32_t *cnt;      // kCntWords counters (above)
    uint32_t *bitmap;  // per multi-workgroup queue slot: kWinWords words
    int32_t *done;     // per multi-workgroup queue slot: chunks finished (0 between uses)
};

// pending(u) = number of higher-priority non-loop neighbours (low 32 bits;
// k_jp_seed adds u's row kind in bits 32-33, so that the release that takes
// the count to zero knows the queue without loading u's row offsets).  A workgroup
// takes kPendTile consecutive entries (read lane by lane), finds each entry's
// row through the tile's row offsets staged in LDS (a binary search; a global
// one when the tile spans a run of empty rows) and counts into the row's LDS
// counter; rows wholly inside the tile are stored, the edge rows added
// atomically (pending zeroed first).
constexpr int kPendTile = 2048;
constexpr int kPendPer = kPendTile / kCT;
__global__ __launch_bounds__(kCT) void k_jp_pending(GraphView g, uint64_t seed, int32_t level, uint64_t *pending) {
    __shared__ int64_t soff[kPendTile + 1];
    __shared__ int32_t acc[kPendTile];
    __shared__ int64_t rr[2];
    const int64_t E0 = (int64_t)blockIdx.x * kPendTile;
    const int64_t E1 = E0 + kPendTile < g.nnz ? E0 + kPendTile : g.nnz;
    if (threadIdx.x == 0) rr[0] = row_of(g.off, g.n, E0);
    if (threadIdx.x == kWave) rr[1] = row_of(g.off, g.n, E1 - 1);
    int32_t v[kPendPer];
#pragma unroll
    for (int q = 0; q < kPendPer; ++q) {
        const int64_t e = E0 + q * kCT + threadIdx.x;
        v[q] = e < E1 ? g.col[e] : 0;
    }
    __syncthreads();
    const int64_t r0 = rr[0], nr = rr[1] - r0 + 1;
    const bool staged = nr <= kPendTile;  // workgroup-uniform
    if (staged) {
        for (int64_t j = threadIdx.x; j <= nr; j += kCT) soff[j] = g.off[r0 + j];
        for (int64_t j = threadIdx.x; j < nr; j += kCT) acc[j] = 0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPendPer; ++q) {
        const int64_t e = E0 + q * kCT + threadIdx.x;
        if (e >= E1) continue;
        int64_t r;
        int lo = 0;
        if (staged) {
            int hi = (int)nr;  // soff[lo] <= e < soff[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (soff[mid] <= e) lo = mid; else hi = mid;
            }
            r = r0 + lo;
        } else {
            r = row_of(g.off, g.n, e);
        }
        const int64_t br = node_base(g, r);
        const int32_t lr = node_level(g, level, r);
        const int64_t x = v[q];
        if (x == r || !prio_greater(prio_hash(seed, lr, x - br), x, prio_hash(seed, lr, r - br), r)) continue;
        if (staged) atomicAdd(&acc[lo], 1);
        else atomicAdd((unsigned long long *)&pending[r], 1ULL);
    }
    if (!staged) return;  // workgroup-uniform
    __syncthreads();
    for (int64_t j = threadIdx.x; j < nr; j += kCT) {
        if (soff[j] >= E0 && soff[j + 1] <= E1) pending[r0 + j] = (uint64_t)acc[j];
        else if (acc[j]) atomicAdd((unsigned long long *)&pending[r0 + j], (unsigned long long)acc[j]);
    }
}

__device__ __forceinline__ int row_kind(const int64_t *off, int32_t v) {
    int64_t d = off[v + 1] - off[v];
    return d <= kLaneRow ? 0 : (d <= kWaveRow ? 1 : 2);
}

// A long row (rare) enters the multi-workgroup queue: a slot, and one work
// item per kHubChunk entries, written by the active lanes of the wavefront
// (the short-row tier leaves the lanes of groups past the frontier's end
// inactive).  hv, e0 and e1 are uniform over the active lanes.
__device__ __forceinline__ void push_long(const JpQ &Q, int set, int32_t hv, int64_t e0, int64_t e1) {
    const int32_t nc = (int32_t)((e1 - e0 + kHubChunk - 1) / kHubChunk);
    const uint64_t act = __ballot(1);
    const int leader = __ffsll((unsigned long long)act) - 1;
    const int lane = lane_id();
    const int32_t rank = (int32_t)__popcll(act & ((lane == 0) ? 0ULL : (~0ULL >> (64 - lane))));
    const int32_t nact = (int32_t)__popcll(act);
    int32_t slot = 0, c0 = 0;
    if (lane == leader) {
        slot = atomicAdd(&Q.cnt[cidx(set, 2)], 1);
        c0 = atomicAdd(&Q.cnt[cidx(set, 3)], nc);
    }
    slot = __shfl(slot, leader);
    c0 = __shfl(c0, leader);
    for (int32_t c = rank; c < nc; c += nact) {
        const int64_t a = e0 + (int64_t)c * kHubChunk;
        Q.cq[set][c0 + c] = HubItem{a, a + kHubChunk < e1 ? a + kHubChunk : e1, hv, slot, nc, 0};
    }
}

// Queue pushes of a wavefront: each lane offers v[j] to queue kind[j] (3: no
// push).  All of the wavefront's pushes of one short-row queue kind are ranked
// by ballots and take their slots with a single counter atomic (the early
// rounds push millions of nodes, and per-push atomics on the two counters would
// serialise); long rows are pushed one at a time by all active lanes.  Order
// within a frontier does not matter: it is an independent set.  Call with
// every lane of the loop iteration active (lanes that left the loop may be
// inactive).
template <int NV>
__device__ __forceinline__ void wave_push(const JpQ &Q, int set, const int32_t (&v)[NV], const int (&kind)[NV],
                                          const int64_t *off) {
    const int lane = lane_id();
    const uint64_t lt = (lane == 0) ? 0ULL : (~0ULL >> (64 - lane));
    int32_t rank[NV];
    int32_t tot0 = 0, tot1 = 0;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const uint64_t m0 = __ballot(kind[j] == 0), m1 = __ballot(kind[j] == 1);
        uint64_t m2 = __ballot(kind[j] == 2);
        rank[j] = kind[j] == 0 ? tot0 + (int32_t)__popcll(m0 & lt) : tot1 + (int32_t)__popcll(m1 & lt);
        tot0 += (int32_t)__popcll(m0);
        tot1 += (int32_t)__popcll(m1);
        while (m2) {
            const int l = __ffsll((unsigned long long)m2) - 1;
            m2 &= m2 - 1;
            const int32_t hv = __shfl(v[j], l);
            push_long(Q, set, hv, off[hv], off[hv + 1]);
        }
    }
    const int leader = __ffsll((unsigned long long)__ballot(1)) - 1;
    int32_t b0 = 0, b1 = 0;
    if (lane == leader) {
        if (tot0) b0 = atomicAdd(&Q.cnt[cidx(set, 0)], tot0);
        if (tot1) b1 = atomicAdd(&Q.cnt[cidx(set, 1)], tot1);
    }
    b0 = __shfl(b0, leader);
    b1 = __shfl(b1, leader);
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        if (kind[j] == 0) Q.q[set][0][b0 + rank[j]] = v[j];
        else if (kind[j] == 1) Q.q[set][1][b1 + rank[j]] = v[j];
    }
}

// Releases v (a lower-priority neighbour of a node coloured this round): the
// queue kind it joins when its count reaches zero, else 3
__device__ __forceinline__ int release(uint64_t *pending, int32_t v) {
    const uint64_t old = atomicSub((unsigned long long *)&pending[v], 1ULL);
    return (uint32_t)old == 1u ? (int)(old >> 32) : 3;
}

__global__ void k_jp_seed(GraphView g, uint64_t *pending, int32_t *colour, JpQ Q) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int kind[1] = {3};
    if (u < g.n) {
        colour[u] = -1;
        const int kd = row_kind(g.off, (int32_t)u);
        const uint64_t p = pending[u];
        if (p == 0) kind[0] = kd;
        else pending[u] = p | ((uint64_t)kd << 32);
    }
    const int32_t v[1] = {(int32_t)(u < g.n ? u : 0)};
    wave_push<1>(Q, 0, v, kind, g.off);
}

// smallest colour >= base not set in an LDS window bitmap, or -1 (wave-wide)
__device__ __forceinline__ int32_t wave_first_free(const uint32_t *bm, int32_t base) {
    int32_t best = 0x7fffffff;
    for (int j = lane_id(); j < kWinWords; j += kWave) {
        uint32_t f = ~bm[j];
        if (f) {
            int32_t c = j * 32 + __builtin_ctz(f);
            best = c < best ? c : best;
        }
    }
    for (int d = 32; d >= 1; d >>= 1) {
        int32_t o = __shfl_xor(best, d);
        best = o < best ? o : best;
    }
    return best == 0x7fffffff ? -1 : base + best;
}

// Wavefront colours node u by scanning its row in colour windows (used for
// rows up to kWaveRow, and as the rare fallback when a hub's first window is
// full).
__device__ __forceinline__ int32_t wave_colour_scan(const GraphView &g, uint64_t seed, int32_t level, int32_t u,
                                                    uint64_t hu, const int32_t *colour, uint32_t *bm,
                                                    int32_t base0) {
    int64_t e0 = g.off[u], e1 = g.off[u + 1];
    const int64_t bu = node_base(g, u);
    const int32_t lu = node_level(g, level, u);
    for (int32_t base = base0;; base += kWin) {
        for (int j = lane_id(); j < kWinWords; j += kWave) bm[j] = 0;
        wave_sync();
        // four entries per lane at a time: the column loads, then the colour
        // gathers of a batch are in flight together
        for (int64_t e = e0 + lane_id(); e < e1; e += 4 * kWave) {
            int32_t v[4], c[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = e + j * kWave < e1 ? g.col[e + j * kWave] : u;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                c[j] = (v[j] != u && prio_greater(prio_hash(seed, lu, v[j] - bu), v[j], hu, u)) ? colour[v[j]] : -1;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                int32_t x = c[j] - base;
                if (c[j] >= 0 && x >= 0 && x < kWin) atomicOr(&bm[x >> 5], 1u << (x & 31));
            }
        }
        wave_sync();
        int32_t f = wave_first_free(bm, base);
        wave_sync();
        if (f >= 0) return f;
    }
}

// Workgroups of a grid round per tier.  The three tiers of a frontier are
// independent (the frontier is an independent set and its nodes only read
// colours of earlier rounds), so each tier gets workgroups of its own and a
// round lasts as long as its slowest tier's chain of dependent loads and
// atomics, not the sum of the three.  A tier gets the workgroups it can use in
// one pass when they fit in the grid, else a share of the grid in proportion
// to its passes (at least one workgroup when it has work); three workgroups
// are held back so that the shares, each rounded down and raised to at least
// one, never exceed the grid.
struct TierSplit {
    int64_t first[3], count[3];
};
__device__ __forceinline__ TierSplit tier_split(int64_t ns, int64_t nm, int64_t nc, int64_t per_s, int64_t per_m,
                                                int64_t nblk) {
    const int64_t need[3] = {(ns + per_s - 1) / per_s, (nm + per_m - 1) / per_m, nc};
    const int64_t tot = need[0] + need[1] + need[2];
    TierSplit t;
    int64_t at = 0;
    for (int k = 0; k < 3; ++k) {
        int64_t c = need[k];
        if (tot > nblk && c > 0) {
            c = need[k] * (nblk - 3) / tot;
            c = c > 0 ? c : 1;
        }
        t.first[k] = at;
        t.count[k] = c;
        at += c;
    }
    return t;
}

// One round, run by workgroups [bid, bid + nblk) of NT threads: the grid
// launch passes its own block index and size (the tiers split the grid), the
// single-workgroup tail 0, 1 (its workgroup runs the three tiers in turn).
template <int NT>
__device__ __forceinline__ void jp_round_body(const GraphView &g, uint64_t seed, int32_t level, int32_t r,
                                              int32_t *colour, uint64_t *pending, const JpQ &Q, int64_t bid,
                                              int64_t nblk) {
    __shared__ uint32_t wbm[NT / kWave][kWinWords];
    __shared__ uint32_t bbm[kWinWords];
    const int set = r % 3, nxt = (r + 1) % 3, old = (r + 2) % 3;
    if (bid == 0 && threadIdx.x < 4) Q.cnt[cidx(old, (int)threadIdx.x)] = 0;
    const int32_t ns = Q.cnt[cidx(set, 0)], nm = Q.cnt[cidx(set, 1)], nc = Q.cnt[cidx(set, 3)];
    TierSplit ts;
    for (int k = 0; k < 3; ++k) { ts.first[k] = 0; ts.count[k] = 1; }
    if (nblk > 1) ts = tier_split(ns, nm, nc, NT / 8, NT / kWave, nblk);
    // eight lanes per node (rows of at most 32 entries: four per lane, loaded
    // together); the colours seen are OR-ed over the eight lanes
    const int sub = (int)(threadIdx.x & 7);
    const int64_t b0 = bid - ts.first[0];
    const bool in0 = b0 >= 0 && b0 < ts.count[0];
    for (int64_t i = in0 ? (b0 * NT + threadIdx.x) >> 3 : ns; i < ns; i += (ts.count[0] * NT) >> 3) {
        int32_t u = Q.q[set][0][i];
        const int64_t bu = node_base(g, u);
        const int32_t lu = node_level(g, level, u);
        uint64_t hu = prio_hash(seed, lu, u - bu);
        int64_t e0 = g.off[u], e1 = g.off[u + 1];
        int32_t v[4];
        bool hi[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int64_t e = e0 + sub + 8 * j;
            v[j] = e < e1 ? g.col[e] : u;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) hi[j] = v[j] != u && prio_greater(prio_hash(seed, lu, v[j] - bu), v[j], hu, u);
        int32_t c[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) c[j] = hi[j] ? colour[v[j]] : 64;
        uint64_t used = 0;  // at most 32 higher neighbours: the answer is below 33
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (c[j] < 64) used |= 1ULL << c[j];
#pragma unroll
        for (int d = 1; d < 8; d <<= 1) used |= __shfl_xor(used, d);
        int32_t cu = __builtin_ctzll(~used);
        if (sub == 0) colour[u] = cu;
        int kd[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) kd[j] = (v[j] != u && !hi[j]) ? release(pending, v[j]) : 3;
        wave_push<4>(Q, nxt, v, kd, g.off);
    }
    // one wavefront per node: a row of up to kWaveRow entries is held in
    // registers (kWaveRow / 64 per lane), its colours gathered in one batch and
    // its lower-priority neighbours released from the same registers
    const int w = threadIdx.x / kWave;
    const int64_t b1 = bid - ts.first[1];
    const bool in1 = b1 >= 0 && b1 < ts.count[1];
    for (int64_t i = in1 ? b1 * (NT / kWave) + w : nm; i < nm; i += ts.count[1] * (NT / kWave)) {
        int32_t u = Q.q[set][1][i];
        const int64_t bu = node_base(g, u);
        const int32_t lu = node_level(g, level, u);
        uint64_t hu = prio_hash(seed, lu, u - bu);
        const int64_t e0 = g.off[u], e1 = g.off[u + 1];
        constexpr int kPer = (int)(kWaveRow / kWave);
        int32_t v[kPer], c[kPer];
        uint32_t hi = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            int64_t e = e0 + lane_id() + (int64_t)j * kWave;
            v[j] = e < e1 ? g.col[e] : u;
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j)
            if (v[j] != u && prio_greater(prio_hash(seed, lu, v[j] - bu), v[j], hu, u)) hi |= 1u << j;
#pragma unroll
        for (int j = 0; j < kPer; ++j) c[j] = (hi >> j) & 1u ? colour[v[j]] : -1;
        int32_t f = -1;
        for (int32_t base = 0; f < 0; base += kWin) {
            for (int j = lane_id(); j < kWinWords; j += kWave) wbm[w][j] = 0;
            wave_sync();
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
                int32_t x = c[j] - base;
                if (c[j] >= 0 && x >= 0 && x < kWin) atomicOr(&wbm[w][x >> 5], 1u << (x & 31));
            }
            wave_sync();
            f = wave_first_free(wbm[w], base);
            wave_sync();
        }
        if (lane_id() == 0) colour[u] = f;
        int kd[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) kd[j] = (v[j] != u && !((hi >> j) & 1u)) ? release(pending, v[j]) : 3;
        wave_push<kPer>(Q, nxt, v, kd, g.off);
    }
    // several workgroups per node: each work item is kHubChunk entries of one
    // long row; its colours go into an LDS bitmap that is OR-ed into the row's
    // global bitmap, and the workgroup that finishes the row's last chunk
    // (counted by a per-slot atomic that each workgroup increments after its
    // returning bitmap ORs, whose results it has consumed) picks the smallest
    // free colour from it.
    // The nodes this round releases read that colour only in the next round.
    __shared__ int32_t last_chunk;
    __shared__ uint32_t or_sink[NT];
    const int64_t b2 = bid - ts.first[2];
    const bool in2 = b2 >= 0 && b2 < ts.count[2];  // workgroup-uniform: the loop holds barriers
    for (int64_t it = in2 ? b2 : nc; it < nc; it += ts.count[2]) {
        const HubItem item = Q.cq[set][it];
        const int32_t j = item.slot, u = item.u;
        const int64_t bu = node_base(g, u);
        const int32_t lu = node_level(g, level, u);
        uint64_t hu = prio_hash(seed, lu, u - bu);
        const int64_t c0 = item.c0, c1 = item.c1;
        for (int i = threadIdx.x; i < kWinWords; i += NT) bbm[i] = 0;
        __syncthreads();
        constexpr int kQ = (int)(kHubChunk / NT) > 0 ? (int)(kHubChunk / NT) : 1;
        int32_t v[kQ], c[kQ];
        bool hi[kQ];
        int kd[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            int64_t e = c0 + q * NT + threadIdx.x;
            v[q] = e < c1 ? g.col[e] : u;
        }
#pragma unroll
        for (int q = 0; q < kQ; ++q)
            hi[q] = v[q] != u && prio_greater(prio_hash(seed, lu, v[q] - bu), v[q], hu, u);
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            c[q] = hi[q] ? colour[v[q]] : kWin;
            kd[q] = (v[q] != u && !hi[q]) ? release(pending, v[q]) : 3;
        }
#pragma unroll
        for (int q = 0; q < kQ; ++q)
            if (c[q] < kWin) atomicOr(&bbm[c[q] >> 5], 1u << (c[q] & 31));
        wave_push<kQ>(Q, nxt, v, kd, g.off);
        __syncthreads();
        // the bitmap words change only through device atomics, which every XCD
        // sees; each OR returns (and its result is consumed) before the barrier,
        // so it has been performed before thread 0 counts the chunk
        uint32_t *bm = Q.bitmap + (int64_t)j * kWinWords;
        uint32_t seen = 0;
        for (int i = threadIdx.x; i < kWinWords; i += NT)
            if (bbm[i]) seen |= atomicOr(&bm[i], bbm[i]);
        or_sink[threadIdx.x] = seen;
        __syncthreads();
        if (threadIdx.x == 0) {
            last_chunk = atomicAdd(&Q.done[j], 1) == item.nch - 1 ? 1 : 0;
        }
        __syncthreads();
        if (last_chunk && threadIdx.x < kWave) {  // workgroup-uniform flag; the first wavefront
            for (int i = lane_id(); i < kWinWords; i += kWave)
                bbm[i] = __hip_atomic_load(&bm[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            wave_sync();
            int32_t cu = wave_first_free(bbm, 0);
            wave_sync();
            for (int i = lane_id(); i < kWinWords; i += kWave) bm[i] = 0;
            if (cu < 0) cu = wave_colour_scan(g, seed, level, u, hu, colour, bbm, kWin);
            if (lane_id() == 0) {
                colour[u] = cu;
                Q.done[j] = 0;
            }
        }
        __syncthreads();  // bbm and last_chunk are reused by the next item
    }
}

__global__ __launch_bounds__(kCT) void k_jp_round(GraphView g, uint64_t seed, int32_t level, int32_t r,
                                                  int32_t *colour, uint64_t *pending, JpQ Q) {
    jp_round_body<kCT>(g, seed, level, r, colour, pending, Q, blockIdx.x, gridDim.x);
}

// Tail of the colouring: once frontiers are small, rounds [r0, r_end) run back
// to back in one workgroup (a grid launch per round would cost far more than
// the round's work), each round's writes made visible to the next by an agent
// fence around a workgroup barrier (counters, queues and bitmaps are updated
// by device atomics, which the CU's L1 does not see).  The workgroup stops at
// an empty frontier, at one whose work exceeds kTailExit passes of the
// workgroup (the grid takes it back), or at r_end, and leaves the round it
// reached in cnt[kCntTail].  Every loop is bounded by the counters of its round.
constexpr int kTailThreads = 1024;
constexpr int32_t kTailEnter = 8;   // frontier work (workgroup passes) at which the host starts the tail
constexpr int32_t kTailExit = 32;   // ... above which the tail hands the rounds back
constexpr int32_t kTailRounds = 1 << 16;  // rounds per tail launch at most
__host__ __device__ __forceinline__ int64_t tail_passes(int64_t ns, int64_t nm, int64_t nc) {
    return ns / (kTailThreads / 8) + nm / (kTailThreads / kWave) + nc + 1;
}
__device__ __forceinline__ void tail_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}
__global__ __launch_bounds__(kTailThreads) void k_jp_tail(GraphView g, uint64_t seed, int32_t level, int32_t r0,
                                                          int32_t r_end, int32_t *colour, uint64_t *pending, JpQ Q) {
    int32_t r = r0;
    tail_barrier();
    for (; r < r_end; ++r) {
        const int set = r % 3;
        const int32_t ns = Q.cnt[cidx(set, 0)], nm = Q.cnt[cidx(set, 1)], nh = Q.cnt[cidx(set, 2)],
                      nc = Q.cnt[cidx(set, 3)];
        // uniform: set r's counters do not change during round r
        if (ns + nm + nh == 0 || tail_passes(ns, nm, nc) > kTailExit) break;
        jp_round_body<kTailThreads>(g, seed, level, r, colour, pending, Q, 0, 1);
        tail_barrier();
    }
    if (threadIdx.x == 0) Q.cnt[kCntTail] = r;
}

// number of colours (1 + the largest) and uncoloured nodes, once at the end
__global__ __launch_bounds__(kCT) void k_colour_stats(const int32_t *colour, int64_t n, int32_t *cnt) {
    int32_t mx = -1, bad = 0;
    for (int64_t u = (int64_t)blockIdx.x * kCT + threadIdx.x; u < n; u += (int64_t)gridDim.x * kCT) {
        const int32_t c = colour[u];
        mx = c > mx ? c : mx;
        bad += c < 0;
    }
    for (int d = 32; d >= 1; d >>= 1) {
        const int32_t o = __shfl_xor(mx, d);
        mx = o > mx ? o : mx;
        bad += __shfl_xor(bad, d);
    }
    if (lane_id() == 0) {
        if (mx >= 0) atomicMax(&cnt[kCntNcol], mx + 1);
        if (bad) atomicAdd(&cnt[kCntUncoloured], bad);
    }
}

__global__ __launch_bounds__(kCT) void k_count_hubs(const int64_t *off, int64_t n, unsigned long long *cnt) {
    unsigned long long c = 0;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x)
        c += (off[u + 1] - off[u] > kWaveRow) ? 1 : 0;
    block_count_add(cnt, c);
}

// Sequential schedule: class = rank in descending priority.  Keys are the
// complemented hash; the value array starts in descending id order so that the
// stable sort puts the larger id first among equal hashes.
__global__ void k_seq_keys(int64_t n, uint64_t seed, int32_t level, uint64_t *keys, int32_t *vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t u = n - 1 - i;
    keys[i] = ~prio_hash(seed, level, u);
    vals[i] = (int32_t)u;
}
__global__ void k_seq_rank(int64_t n, const int32_t *order, int32_t *colour) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) colour[order[i]] = (int32_t)i;
}

int32_t build_colouring(const GraphView &g, uint64_t seed, int32_t level, int schedule, int32_t *colour,
                        Scratch &scr, int32_t *host_counters, int32_t *jp_rounds, hipStream_t st, bool use_tail) {
    int64_t n = g.n;
    *jp_rounds = 0;
    if (n == 0) return 0;
    if (schedule == 1) {
        scr.reserve(2 * align_up(n * 8) + 2 * align_up(n * 4) + radix_scratch_bytes(n));
        uint64_t *k = (uint64_t *)scr.get(n * 8), *ka = (uint64_t *)scr.get(n * 8);
        int32_t *v = (int32_t *)scr.get(n * 4), *va = (int32_t *)scr.get(n * 4);
        void *rs = scr.get(radix_scratch_bytes(n));
        hipLaunchKernelGGL(k_seq_keys, dim3((unsigned)cdiv(n, kCT)), dim3(kCT), 0, st, n, seed, level, k, v);
        radix_sort_u64_i32(&k, &v, &ka, &va, n, 64, rs, st);
        hipLaunchKernelGGL(k_seq_rank, dim3((unsigned)cdiv(n, kCT)), dim3(kCT), 0, st, n, v, colour);
        HIPCHK(hipGetLastError());
        return (int32_t)n;
    }
    // count rows longer than kWaveRow to size the hub bitmaps
    scr.reserve(4096);
    unsigned long long *hc = (unsigned long long *)scr.get(8);
    HIPCHK(hipMemsetAsync(hc, 0, 8, st));
    const int64_t hb = cdiv(n, kCT);
    hipLaunchKernelGGL(k_count_hubs, dim3((unsigned)(hb < kCountGrid ? hb : kCountGrid)), dim3(kCT), 0, st, g.off, n,
                       hc);
    HIPCHK(hipMemcpyAsync(host_counters, hc, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    uint64_t nhub_u = 0;
    std::memcpy(&nhub_u, host_counters, 8);
    int64_t nhub = (int64_t)nhub_u;
    // pending counts, 6 node queues, counters, hub bitmaps, 3 item queues
    // work items of long rows in one set: at most nnz / kHubChunk + nhub
    const int64_t ncap = g.nnz / kHubChunk + nhub + 1;
    const size_t nslot = (size_t)(nhub > 0 ? nhub : 1);
    scr.reserve(align_up(n * 8) + align_up(n * 4) * 6 + align_up(kCntWords * sizeof(int32_t)) +
                align_up(nslot * kWinWords * 4) + align_up(nslot * 4) + 3 * align_up(ncap * sizeof(HubItem)));
    uint64_t *pending = (uint64_t *)scr.get(n * 8);
    JpQ Q;
    for (int s = 0; s < 3; ++s)
        for (int k = 0; k < 2; ++k) Q.q[s][k] = (int32_t *)scr.get(n * 4);
    Q.cnt = (int32_t *)scr.get(kCntWords * sizeof(int32_t));
    Q.bitmap = (uint32_t *)scr.get(nslot * kWinWords * 4);
    Q.done = (int32_t *)scr.get(nslot * 4);
    for (int s = 0; s < 3; ++s) Q.cq[s] = (HubItem *)scr.get(ncap * sizeof(HubItem));
    HIPCHK(hipMemsetAsync(pending, 0, n * 8, st));
    HIPCHK(hipMemsetAsync(Q.cnt, 0, kCntWords * sizeof(int32_t), st));
    HIPCHK(hipMemsetAsync(Q.bitmap, 0, nslot * kWinWords * 4, st));
    HIPCHK(hipMemsetAsync(Q.done, 0, nslot * 4, st));
    if (g.nnz > 0)
        hipLaunchKernelGGL(k_jp_pending, dim3((unsigned)cdiv(g.nnz, kPendTile)), dim3(kCT), 0, st, g, seed, level,
                           pending);
    hipLaunchKernelGGL(k_jp_seed, dim3((unsigned)cdiv(n, kCT)), dim3(kCT), 0, st, g, pending, colour, Q);
    HIPCHK(hipGetLastError());
    // grid rounds while frontiers are large, the one-workgroup tail once the
    // frontier the host last saw is small (the seed frontier is known without
    // a copy only for its size, so the first check decides).  Grid batches are
    // pipelined: the counters after batch k (copied into one of two host
    // buffers) are examined while batch k + 1 runs, so the device does not
    // idle while the host decides; rounds launched past an empty frontier
    // find nothing to do.  A tail launch is waited for, since the launch after
    // it needs the round it reached.
    struct Events {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~Events() {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } ev;
    for (hipEvent_t &x : ev.e) HIPCHK(hipEventCreateWithFlags(&x, hipEventDisableTiming));
    int32_t *hcb[2] = {host_counters, host_counters + kCntWords};
    auto frontier = [&](const int32_t *c, int32_t rr, int32_t &ns, int32_t &nm, int32_t &nh, int32_t &nc) {
        const int s = rr % 3;
        ns = c[cidx(s, 0)]; nm = c[cidx(s, 1)]; nh = c[cidx(s, 2)]; nc = c[cidx(s, 3)];
        return ns == 0 && nm == 0 && nh == 0;
    };
    int32_t r = 0, r_done = 0, r_prev = 0;
    int prev = -1;  // host buffer of the grid batch not yet examined
    bool tail = false;
    for (;;) {
        int32_t ns = 0, nm = 0, nh = 0, nc = 0;
        if (tail) {
            const int32_t r_end = r < INT32_MAX - kTailRounds ? r + kTailRounds : INT32_MAX;
            hipLaunchKernelGGL(k_jp_tail, dim3(1), dim3(kTailThreads), 0, st, g, seed, level, r, r_end, colour,
                               pending, Q);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(hcb[0], Q.cnt, kCntWords * sizeof(int32_t), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            r = hcb[0][kCntTail];
            if (frontier(hcb[0], r, ns, nm, nh, nc)) { r_done = r; break; }
            tail = use_tail && tail_passes(ns, nm, nc) <= kTailEnter;
            continue;
        }
        for (int i = 0; i < kRoundsPerCheck; ++i, ++r) {
            hipLaunchKernelGGL(k_jp_round, dim3(kRoundGrid), dim3(kCT), 0, st, g, seed, level, r, colour,
                               pending, Q);
        }
        HIPCHK(hipGetLastError());
        const int cur = prev == 0 ? 1 : 0;
        HIPCHK(hipMemcpyAsync(hcb[cur], Q.cnt, kCntWords * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIPCHK(hipEventRecord(ev.e[cur], st));
        if (prev < 0) {  // nothing to examine yet: launch the next batch first
            prev = cur;
            r_prev = r;
            continue;
        }
        HIPCHK(hipEventSynchronize(ev.e[prev]));
        if (frontier(hcb[prev], r_prev, ns, nm, nh, nc)) {
            r_done = r_prev;
            HIPCHK(hipStreamSynchronize(st));
            break;
        }
        if (r_prev > n + 2 * kRoundsPerCheck) throw Error{-6, "internal: colouring did not converge"};
        if (use_tail && tail_passes(ns, nm, nc) <= kTailEnter) {
            // the batch just launched has run on: decide from its counters
            HIPCHK(hipEventSynchronize(ev.e[cur]));
            prev = -1;
            if (frontier(hcb[cur], r, ns, nm, nh, nc)) {
                r_done = r;
                break;
            }
            tail = tail_passes(ns, nm, nc) <= kTailEnter;
            continue;
        }
        prev = cur;
        r_prev = r;
    }
    hipLaunchKernelGGL(k_colour_stats, dim3((unsigned)(hb < kCountGrid ? hb : kCountGrid)), dim3(kCT), 0, st, colour,
                       n, Q.cnt);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(host_counters, Q.cnt, kCntWords * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (host_counters[kCntUncoloured] != 0) throw Error{-6, "internal: colouring did not reach every node"};
    *jp_rounds = r_done;
    return host_counters[kCntNcol];
}

}  // namespace plm
