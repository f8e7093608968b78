// level.hip - per-level set-up: node volumes, the priority colouring that fixes
// the move schedule, and the bucketing of nodes into (colour class, degree bin).
#include <hip/hip_runtime.h>

#include "level.h"

namespace plm {

constexpr int kThreads = 256;
constexpr int kChunk = 16;  // entries per thread in entry-parallel kernels

// ------------------------------------------------------------------ volumes
// vol(u) = row sum with self-loop entries multiplied by diag_mult (section
// III-B: a self-loop counts twice in vol).  Entry-parallel: each thread walks
// kChunk consecutive entries and flushes one partial sum per row segment
// (atomic when the row extends past the chunk).  Also accumulates S and the
// largest volume.
template <int WK>
__global__ __launch_bounds__(kThreads) void k_vol(GraphView g, int64_t *vol, unsigned long long *S,
                                                  unsigned long long *maxvol) {
    int64_t e0 = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * kChunk;
    int64_t tot = 0;
    if (e0 < g.nnz) {
        int64_t e1 = e0 + kChunk < g.nnz ? e0 + kChunk : g.nnz;
        int64_t r = row_of(g.off, g.n, e0);
        int64_t rend = g.off[r + 1];
        int64_t seg_start = e0, acc = 0;
        for (int64_t e = e0; e < e1; ++e) {
            while (e >= rend) {  // flush row r
                if (seg_start == g.off[r] && rend <= e1) vol[r] = acc;
                else if (acc) atomicAdd((unsigned long long *)&vol[r], (unsigned long long)acc);
                tot += acc;
                acc = 0;
                ++r;
                rend = g.off[r + 1];
                seg_start = e;
            }
            int64_t x = wload<WK>(g.w, e);
            if (g.col[e] == r) x *= g.diag_mult;
            acc += x;
        }
        if (seg_start == g.off[r] && rend <= e1) vol[r] = acc;
        else if (acc) atomicAdd((unsigned long long *)&vol[r], (unsigned long long)acc);
        tot += acc;
    }
    // block sum of tot -> S
    __shared__ int64_t red[kThreads / kWave];
    for (int d = 32; d >= 1; d >>= 1) tot += __shfl_xor(tot, d);
    if (lane_id() == 0) red[threadIdx.x / kWave] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int i = 0; i < kThreads / kWave; ++i) s += red[i];
        if (s) atomicAdd(S, (unsigned long long)s);
    }
}

__global__ void k_max_vol(const int64_t *vol, int64_t n, unsigned long long *maxvol) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t m = 0;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) m = vol[i] > m ? vol[i] : m;
    for (int d = 32; d >= 1; d >>= 1) {
        int64_t o = __shfl_xor(m, d);
        m = o > m ? o : m;
    }
    if (lane_id() == 0 && m) atomicMax(maxvol, (unsigned long long)m);
}

void launch_volumes(const GraphView &g, int64_t *vol, unsigned long long *S_dev, unsigned long long *maxvol_dev,
                    hipStream_t st) {
    HIPCHK(hipMemsetAsync(vol, 0, (size_t)(g.n > 0 ? g.n : 1) * sizeof(int64_t), st));
    HIPCHK(hipMemsetAsync(S_dev, 0, sizeof(unsigned long long), st));
    HIPCHK(hipMemsetAsync(maxvol_dev, 0, sizeof(unsigned long long), st));
    if (g.nnz > 0) {
        dim3 grid((unsigned)cdiv(cdiv(g.nnz, kChunk), kThreads));
        switch (g.wkind) {
            case 0: hipLaunchKernelGGL(k_vol<0>, grid, dim3(kThreads), 0, st, g, vol, S_dev, maxvol_dev); break;
            case 1: hipLaunchKernelGGL(k_vol<1>, grid, dim3(kThreads), 0, st, g, vol, S_dev, maxvol_dev); break;
            default: hipLaunchKernelGGL(k_vol<2>, grid, dim3(kThreads), 0, st, g, vol, S_dev, maxvol_dev); break;
        }
        int64_t nb = cdiv(g.n, kThreads);
        hipLaunchKernelGGL(k_max_vol, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(kThreads), 0, st, vol, g.n,
                           maxvol_dev);
    }
    HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------------ colouring
// Jones-Plassmann with a pending counter per node: pending(u) = number of
// non-loop neighbours of higher priority.  Nodes with pending 0 form the
// first frontier; a frontier node takes the smallest colour unused by its
// higher-priority neighbours (all coloured by then) and decrements its
// lower-priority neighbours, which join the next frontier when they reach 0.
// The result equals the greedy colouring in descending priority order.

__global__ __launch_bounds__(kThreads) void k_jp_pending(GraphView g, uint64_t seed, int32_t level,
                                                         int32_t *pending) {
    int64_t e0 = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * kChunk;
    if (e0 >= g.nnz) return;
    int64_t e1 = e0 + kChunk < g.nnz ? e0 + kChunk : g.nnz;
    int64_t r = row_of(g.off, g.n, e0);
    int64_t rend = g.off[r + 1];
    uint64_t hr = prio_hash(seed, level, r);
    int32_t cnt = 0;
    for (int64_t e = e0; e < e1; ++e) {
        while (e >= rend) {
            if (cnt) atomicAdd(&pending[r], cnt);
            cnt = 0;
            ++r;
            rend = g.off[r + 1];
            hr = prio_hash(seed, level, r);
        }
        int64_t v = g.col[e];
        if (v != r && prio_greater(prio_hash(seed, level, v), v, hr, r)) ++cnt;
    }
    if (cnt) atomicAdd(&pending[r], cnt);
}

// frontier queues: small (row length <= kJpSmall) handled one lane per node,
// large handled one wavefront per node
constexpr int64_t kJpSmall = 32;

__device__ __forceinline__ void jp_push(int32_t v, const int64_t *off, int32_t *qs, int32_t *qs_n, int32_t *ql,
                                        int32_t *ql_n) {
    int64_t d = off[v + 1] - off[v];
    if (d <= kJpSmall) qs[atomicAdd(qs_n, 1)] = v;
    else ql[atomicAdd(ql_n, 1)] = v;
}

__global__ void k_jp_seed(GraphView g, const int32_t *pending, int32_t *colour, int32_t *qs, int32_t *qs_n,
                          int32_t *ql, int32_t *ql_n) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= g.n) return;
    colour[u] = -1;
    if (pending[u] == 0) jp_push((int32_t)u, g.off, qs, qs_n, ql, ql_n);
}

__device__ __forceinline__ void jp_release(int32_t v, int32_t *pending, const int64_t *off, int32_t *qs,
                                           int32_t *qs_n, int32_t *ql, int32_t *ql_n) {
    if (atomicSub(&pending[v], 1) == 1) jp_push(v, off, qs, qs_n, ql, ql_n);
}

// one lane per small frontier node
__global__ __launch_bounds__(kThreads) void k_jp_small(GraphView g, uint64_t seed, int32_t level,
                                                       const int32_t *q, int32_t qn, int32_t *colour,
                                                       int32_t *pending, int32_t *ncol, int32_t *qs, int32_t *qs_n,
                                                       int32_t *ql, int32_t *ql_n) {
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= qn) return;
    int32_t u = q[i];
    uint64_t hu = prio_hash(seed, level, u);
    int64_t e0 = g.off[u], e1 = g.off[u + 1];
    uint64_t used = 0;  // colours < 64 of higher-priority neighbours (row length <= 32 bounds the answer)
    for (int64_t e = e0; e < e1; ++e) {
        int32_t v = g.col[e];
        if (v == u) continue;
        if (prio_greater(prio_hash(seed, level, v), v, hu, u)) {
            int32_t c = colour[v];
            if (c < 64) used |= 1ULL << c;
        }
    }
    int32_t c = __builtin_ctzll(~used);
    colour[u] = c;
    atomicMax(ncol, c + 1);
    for (int64_t e = e0; e < e1; ++e) {
        int32_t v = g.col[e];
        if (v == u) continue;
        if (!prio_greater(prio_hash(seed, level, v), v, hu, u)) jp_release(v, pending, g.off, qs, qs_n, ql, ql_n);
    }
}

// one wavefront per large frontier node; colours are searched in windows of
// kJpWin through an LDS bitmap
constexpr int kJpWin = 4096;
__global__ __launch_bounds__(kThreads) void k_jp_large(GraphView g, uint64_t seed, int32_t level,
                                                       const int32_t *q, int32_t qn, int32_t *colour,
                                                       int32_t *pending, int32_t *ncol, int32_t *qs, int32_t *qs_n,
                                                       int32_t *ql, int32_t *ql_n) {
    __shared__ uint32_t bm[kThreads / kWave][kJpWin / 32];
    const int w = threadIdx.x / kWave, lane = lane_id();
    for (int64_t i = (int64_t)blockIdx.x * (kThreads / kWave) + w; i < qn;
         i += (int64_t)gridDim.x * (kThreads / kWave)) {
        int32_t u = q[i];
        uint64_t hu = prio_hash(seed, level, u);
        int64_t e0 = g.off[u], e1 = g.off[u + 1];
        int32_t found = -1;
        for (int32_t base = 0; found < 0; base += kJpWin) {
            for (int j = lane; j < kJpWin / 32; j += kWave) bm[w][j] = 0;
            wave_sync();
            for (int64_t e = e0 + lane; e < e1; e += kWave) {
                int32_t v = g.col[e];
                if (v == u) continue;
                if (prio_greater(prio_hash(seed, level, v), v, hu, u)) {
                    int32_t c = colour[v] - base;
                    if (c >= 0 && c < kJpWin) atomicOr(&bm[w][c >> 5], 1u << (c & 31));
                }
            }
            wave_sync();
            int32_t best = 0x7fffffff;
            for (int j = lane; j < kJpWin / 32; j += kWave) {
                uint32_t free_bits = ~bm[w][j];
                if (free_bits) {
                    int32_t c = j * 32 + __builtin_ctz(free_bits);
                    best = c < best ? c : best;
                }
            }
            for (int d = 32; d >= 1; d >>= 1) {
                int32_t o = __shfl_xor(best, d);
                best = o < best ? o : best;
            }
            if (best != 0x7fffffff) found = base + best;
            wave_sync();
        }
        if (lane == 0) {
            colour[u] = found;
            atomicMax(ncol, found + 1);
        }
        for (int64_t e = e0 + lane; e < e1; e += kWave) {
            int32_t v = g.col[e];
            if (v == u) continue;
            if (!prio_greater(prio_hash(seed, level, v), v, hu, u)) jp_release(v, pending, g.off, qs, qs_n, ql, ql_n);
        }
    }
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
                        Scratch &scr, int32_t *host_counters, int32_t *jp_rounds, hipStream_t st) {
    int64_t n = g.n;
    *jp_rounds = 0;
    if (n == 0) return 0;
    if (schedule == 1) {
        scr.reserve(2 * align_up(n * 8) + 2 * align_up(n * 4) + radix_scratch_bytes(n));
        uint64_t *k = (uint64_t *)scr.get(n * 8), *ka = (uint64_t *)scr.get(n * 8);
        int32_t *v = (int32_t *)scr.get(n * 4), *va = (int32_t *)scr.get(n * 4);
        void *rs = scr.get(radix_scratch_bytes(n));
        hipLaunchKernelGGL(k_seq_keys, dim3((unsigned)cdiv(n, kThreads)), dim3(kThreads), 0, st, n, seed, level, k, v);
        radix_sort_u64_i32(&k, &v, &ka, &va, n, 64, rs, st);
        hipLaunchKernelGGL(k_seq_rank, dim3((unsigned)cdiv(n, kThreads)), dim3(kThreads), 0, st, n, v, colour);
        HIPCHK(hipGetLastError());
        return (int32_t)n;
    }
    // pending counts, 4 queues (2 current, 2 next), counters
    scr.reserve(align_up(n * 4) * 5 + 256);
    int32_t *pending = (int32_t *)scr.get(n * 4);
    int32_t *q[4];
    for (int i = 0; i < 4; ++i) q[i] = (int32_t *)scr.get(n * 4);
    int32_t *cnt = (int32_t *)scr.get(8 * sizeof(int32_t));  // [qs_n, ql_n, qs2_n, ql2_n, ncol]
    HIPCHK(hipMemsetAsync(pending, 0, n * 4, st));
    HIPCHK(hipMemsetAsync(cnt, 0, 8 * sizeof(int32_t), st));
    if (g.nnz > 0)
        hipLaunchKernelGGL(k_jp_pending, dim3((unsigned)cdiv(cdiv(g.nnz, kChunk), kThreads)), dim3(kThreads), 0, st,
                           g, seed, level, pending);
    hipLaunchKernelGGL(k_jp_seed, dim3((unsigned)cdiv(n, kThreads)), dim3(kThreads), 0, st, g, pending, colour, q[0],
                       cnt + 0, q[1], cnt + 1);
    HIPCHK(hipGetLastError());
    int cur = 0;  // current queues q[2cur], q[2cur+1], counters cnt[2cur], cnt[2cur+1]
    int64_t done = 0;
    for (;;) {
        HIPCHK(hipMemcpyAsync(host_counters, cnt, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        int32_t ns = host_counters[2 * cur], nl = host_counters[2 * cur + 1];
        if (ns == 0 && nl == 0) break;
        done += ns + nl;
        if (done > n) throw Error{-6, "internal: colouring frontier overflow"};
        int nx = 1 - cur;
        HIPCHK(hipMemsetAsync(cnt + 2 * nx, 0, 2 * sizeof(int32_t), st));
        if (ns > 0)
            hipLaunchKernelGGL(k_jp_small, dim3((unsigned)cdiv(ns, kThreads)), dim3(kThreads), 0, st, g, seed, level,
                               q[2 * cur], ns, colour, pending, cnt + 4, q[2 * nx], cnt + 2 * nx, q[2 * nx + 1],
                               cnt + 2 * nx + 1);
        if (nl > 0) {
            int64_t blocks = cdiv(nl, kThreads / kWave);
            hipLaunchKernelGGL(k_jp_large, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(kThreads), 0, st, g,
                               seed, level, q[2 * cur + 1], nl, colour, pending, cnt + 4, q[2 * nx], cnt + 2 * nx,
                               q[2 * nx + 1], cnt + 2 * nx + 1);
        }
        HIPCHK(hipGetLastError());
        cur = nx;
        ++*jp_rounds;
    }
    if (done != n) throw Error{-6, "internal: colouring did not reach every node"};
    return host_counters[4];
}

// ------------------------------------------------------------------ bucketing
// key(u) = colour(u) * 4 + bin(u); nodes without a non-loop neighbour get the
// sentinel key ncol * 4 (they can never move).
__global__ void k_bucket_keys(GraphView g, const int32_t *colour, int32_t ncol, int64_t b0, int64_t b1, int64_t b2,
                              uint32_t *keys, int32_t *vals, unsigned long long *bin_entries) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t cnt[4] = {0, 0, 0, 0};
    if (u < g.n) {
        int64_t e0 = g.off[u], d = g.off[u + 1] - e0;
        bool active = d > 1 || (d == 1 && g.col[e0] != u);
        uint32_t bin = d <= b0 ? 0u : (d <= b1 ? 1u : (d <= b2 ? 2u : 3u));
        keys[u] = active ? (uint32_t)colour[u] * 4u + bin : (uint32_t)ncol * 4u;
        vals[u] = (int32_t)u;
        if (active) cnt[bin] = d;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        int64_t c = cnt[b];
        for (int s = 32; s >= 1; s >>= 1) c += __shfl_xor(c, s);
        if (lane_id() == 0 && c) atomicAdd(&bin_entries[b], (unsigned long long)c);
    }
}

// bstart[k] = first position with key >= k, for k in [0, nkeys]
__global__ void k_bucket_bounds(const uint32_t *keys, int64_t n, int64_t nkeys, int64_t *bstart) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    int64_t prev = (i == 0) ? -1 : (int64_t)keys[i - 1];
    int64_t cur = (i == n) ? nkeys : (int64_t)keys[i];
    for (int64_t k = prev + 1; k <= cur && k <= nkeys; ++k) bstart[k] = i;
}

void build_buckets(const GraphView &g, const int32_t *colour, int32_t ncol, int64_t b0, int64_t b1, int64_t b2,
                   int32_t *class_nodes, int64_t *bstart_dev, unsigned long long *bin_entries, Scratch &scr,
                   hipStream_t st) {
    int64_t n = g.n;
    if (n == 0) return;
    scr.reserve(2 * align_up(n * 4) * 2 + radix_scratch_bytes(n));
    uint32_t *k = (uint32_t *)scr.get(n * 4), *ka = (uint32_t *)scr.get(n * 4);
    int32_t *v = (int32_t *)scr.get(n * 4), *va = (int32_t *)scr.get(n * 4);
    void *rs = scr.get(radix_scratch_bytes(n));
    hipLaunchKernelGGL(k_bucket_keys, dim3((unsigned)cdiv(n, kThreads)), dim3(kThreads), 0, st, g, colour, ncol, b0,
                       b1, b2, k, v, bin_entries);
    int64_t nkeys = (int64_t)ncol * 4 + 1;  // including the sentinel
    radix_sort_u32_i32(&k, &v, &ka, &va, n, ceil_log2((uint64_t)nkeys), rs, st);
    hipLaunchKernelGGL(k_bucket_bounds, dim3((unsigned)cdiv(n + 1, kThreads)), dim3(kThreads), 0, st, k, n, nkeys,
                       bstart_dev);
    HIPCHK(hipMemcpyAsync(class_nodes, v, n * 4, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipGetLastError());
}

}  // namespace plm
