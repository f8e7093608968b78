// level.hip - per-level set-up: node volumes and the bucketing of nodes into
// (colour class, degree bin).
#include <hip/hip_runtime.h>

#include "level.h"

namespace plm {

constexpr int kThreads = 256;

// ------------------------------------------------------------------ volumes
// vol(u) = row sum with self-loop entries multiplied by diag_mult (section
// III-B: a self-loop counts twice in vol); also accumulates S.  A workgroup
// takes kVolTile consecutive entries, stages the offsets of the rows they
// touch in LDS, and reads its entries lane by lane (coalesced, all of a
// thread's loads in flight together); each entry
// finds its row by a binary search in LDS and adds into that row's LDS sum.
// Rows wholly inside the tile are stored, the edge rows added atomically.  A
// tile touching more rows than fit (a run of empty rows) walks its entries
// instead, one thread per kVolPer consecutive entries, flushing a partial sum
// per row segment.
constexpr int kVolTile = 2048;
constexpr int kVolPer = kVolTile / kThreads;
template <int WK>
__global__ __launch_bounds__(kThreads) void k_vol_tile(GraphView g, int64_t *vol, unsigned long long *S) {
    __shared__ int64_t soff[kVolTile + 1];
    __shared__ int64_t acc[kVolTile];
    __shared__ int64_t rr[2];
    const int64_t E0 = (int64_t)blockIdx.x * kVolTile;
    const int64_t E1 = E0 + kVolTile < g.nnz ? E0 + kVolTile : g.nnz;
    if (threadIdx.x == 0) rr[0] = row_of(g.off, g.n, E0);
    if (threadIdx.x == kWave) rr[1] = row_of(g.off, g.n, E1 - 1);
    __syncthreads();
    const int64_t r0 = rr[0], nr = rr[1] - r0 + 1;
    int64_t tot = 0;
    if (nr <= kVolTile) {  // workgroup-uniform
        for (int64_t j = threadIdx.x; j <= nr; j += kThreads) soff[j] = g.off[r0 + j];
        for (int64_t j = threadIdx.x; j < nr; j += kThreads) acc[j] = 0;
        int32_t c[kVolPer];
        int64_t x[kVolPer];
#pragma unroll
        for (int q = 0; q < kVolPer; ++q) {
            const int64_t e = E0 + q * kThreads + threadIdx.x;
            c[q] = e < E1 ? g.col[e] : -1;
            x[q] = e < E1 ? wload<WK>(g.w, e) : 0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kVolPer; ++q) {
            const int64_t e = E0 + q * kThreads + threadIdx.x;
            if (e >= E1) continue;
            int lo = 0, hi = (int)nr;  // soff[lo] <= e < soff[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (soff[mid] <= e) lo = mid; else hi = mid;
            }
            int64_t v = x[q];
            if (c[q] == r0 + lo) v *= g.diag_mult;
            atomicAdd((unsigned long long *)&acc[lo], (unsigned long long)v);
            tot += v;
        }
        __syncthreads();
        for (int64_t j = threadIdx.x; j < nr; j += kThreads) {
            if (soff[j] >= E0 && soff[j + 1] <= E1) vol[r0 + j] = acc[j];
            else if (acc[j]) atomicAdd((unsigned long long *)&vol[r0 + j], (unsigned long long)acc[j]);
        }
    } else {
        const int64_t e0 = E0 + (int64_t)threadIdx.x * kVolPer;
        if (e0 < E1) {
            const int64_t e1 = e0 + kVolPer < E1 ? e0 + kVolPer : E1;
            int64_t r = row_of(g.off, g.n, e0);
            int64_t rend = g.off[r + 1];
            int64_t seg_start = e0, a = 0;
            for (int64_t e = e0; e < e1; ++e) {
                while (e >= rend) {
                    if (seg_start == g.off[r] && rend <= e1) vol[r] = a;
                    else if (a) atomicAdd((unsigned long long *)&vol[r], (unsigned long long)a);
                    tot += a;
                    a = 0;
                    r = next_row(g.off, g.n, r, e);
                    rend = g.off[r + 1];
                    seg_start = e;
                }
                int64_t v = wload<WK>(g.w, e);
                if (g.col[e] == r) v *= g.diag_mult;
                a += v;
            }
            if (seg_start == g.off[r] && rend <= e1) vol[r] = a;
            else if (a) atomicAdd((unsigned long long *)&vol[r], (unsigned long long)a);
            tot += a;
        }
    }
    block_count_add(S, (unsigned long long)tot);
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
        const dim3 tiles((unsigned)cdiv(g.nnz, kVolTile));
        switch (g.wkind) {
            case 0: hipLaunchKernelGGL(k_vol_tile<0>, tiles, dim3(kThreads), 0, st, g, vol, S_dev); break;
            case 1: hipLaunchKernelGGL(k_vol_tile<1>, tiles, dim3(kThreads), 0, st, g, vol, S_dev); break;
            default: hipLaunchKernelGGL(k_vol_tile<2>, tiles, dim3(kThreads), 0, st, g, vol, S_dev); break;
        }
        int64_t nb = cdiv(g.n, kThreads);
        hipLaunchKernelGGL(k_max_vol, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(kThreads), 0, st, vol, g.n,
                           maxvol_dev);
    }
    HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------------ bucketing
// key(u) = (colour(u) * 4 + bin(u)) * 2 + sub(u), sub = 1 for wavefront-bin
// rows longer than kQuadRow and workgroup-bin rows longer than kBlockShortRow
// (so that the short ones come first in their bucket); nodes without a non-loop neighbour get the sentinel key ncol * 8
// (they can never move).
// Grid-stride, with the per-bin entry counts summed per workgroup: one atomic
// per (workgroup, bin) instead of one per wavefront, on four counters.
__global__ __launch_bounds__(kThreads) void k_bucket_keys(GraphView g, const int64_t *vol, const int32_t *colour,
                                                          int32_t ncol, int64_t b0, int64_t b1, int64_t b2,
                                                          const uint8_t *keep, uint32_t *keys, int32_t *vals,
                                                          unsigned long long *bin_entries) {
    __shared__ unsigned long long red[kThreads / kWave][4];
    int64_t cnt[4] = {0, 0, 0, 0};
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < g.n; u += (int64_t)gridDim.x * blockDim.x) {
        int64_t e0 = g.off[u], d = g.off[u + 1] - e0;
        bool active = (d > 1 || (d == 1 && g.col[e0] != u)) && (!keep || keep[g.gid[u]]);
        uint32_t bin = d <= b0 ? 0u : (d <= b1 ? 1u : (d <= b2 ? 2u : 3u));
        if ((bin == 1u || bin == 2u) && vol[u] > (int64_t)INT32_MAX) bin = 3u;
        const uint32_t sub = ((bin == 1u && d > kQuadRow) || (bin == 2u && d > kBlockShortRow)) ? 1u : 0u;
        keys[u] = active ? ((uint32_t)colour[u] * 4u + bin) * 2u + sub : (uint32_t)ncol * 8u;
        vals[u] = (int32_t)u;
        if (active) cnt[bin] += d;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        int64_t c = cnt[b];
        for (int s = 32; s >= 1; s >>= 1) c += __shfl_xor(c, s);
        if (lane_id() == 0) red[threadIdx.x / kWave][b] = (unsigned long long)c;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        unsigned long long c = 0;
        for (int w = 0; w < kThreads / kWave; ++w) c += red[w][threadIdx.x];
        if (c) atomicAdd(&bin_entries[threadIdx.x], c);
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

void build_buckets(const GraphView &g, const int64_t *vol, const int32_t *colour, int32_t ncol, int64_t b0,
                   int64_t b1, int64_t b2, int32_t *class_nodes, int64_t *bstart_dev,
                   unsigned long long *bin_entries, Scratch &scr, hipStream_t st, const uint8_t *keep) {
    int64_t n = g.n;
    if (n == 0) return;
    scr.reserve(2 * align_up(n * 4) * 2 + radix_scratch_bytes(n));
    uint32_t *k = (uint32_t *)scr.get(n * 4), *ka = (uint32_t *)scr.get(n * 4);
    int32_t *v = (int32_t *)scr.get(n * 4), *va = (int32_t *)scr.get(n * 4);
    void *rs = scr.get(radix_scratch_bytes(n));
    const int64_t kb = cdiv(n, kThreads);
    hipLaunchKernelGGL(k_bucket_keys, dim3((unsigned)(kb < 4096 ? kb : 4096)), dim3(kThreads), 0, st, g, vol, colour,
                       ncol, b0, b1, b2, keep, k, v, bin_entries);
    int64_t nkeys = (int64_t)ncol * 8 + 1;  // including the sentinel
    radix_sort_u32_i32(&k, &v, &ka, &va, n, ceil_log2((uint64_t)nkeys), rs, st);
    hipLaunchKernelGGL(k_bucket_bounds, dim3((unsigned)cdiv(n + 1, kThreads)), dim3(kThreads), 0, st, k, n, nkeys,
                       bstart_dev);
    HIPCHK(hipMemcpyAsync(class_nodes, v, n * 4, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipGetLastError());
}

}  // namespace plm
