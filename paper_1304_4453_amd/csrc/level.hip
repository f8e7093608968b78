// level.hip - per-level set-up: node volumes and the bucketing of nodes into
// (colour class, degree bin).
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
    int64_t tot = 0;
    const int64_t nchunks = cdiv_dev(g.nnz, kChunk);
    for (int64_t ch = (int64_t)blockIdx.x * kThreads + threadIdx.x; ch < nchunks;
         ch += (int64_t)gridDim.x * kThreads) {
        const int64_t e0 = ch * kChunk;
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
                r = next_row(g.off, g.n, r, e);
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
    block_count_add(S, (unsigned long long)tot);  // S: one atomic per workgroup
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
        const int64_t vb = cdiv(cdiv(g.nnz, kChunk), kThreads);
        dim3 grid((unsigned)(vb < 4 * kCountGrid ? vb : 4 * kCountGrid));
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

// ------------------------------------------------------------------ bucketing
// key(u) = (colour(u) * 4 + bin(u)) * 2 + sub(u), sub = 1 for wavefront-bin
// rows longer than kQuadRow (so that the short ones come first in their
// bucket); nodes without a non-loop neighbour get the sentinel key ncol * 8
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
        const uint32_t sub = (bin == 1u && d > kQuadRow) ? 1u : 0u;
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
