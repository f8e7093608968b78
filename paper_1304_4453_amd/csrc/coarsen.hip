// coarsen.hip - contraction of communities into a coarse graph (section III-B,
// implementation of coarsen), prolongation, canonical labels, modularity
// (Equation (3.1)) and input validation.
#include <hip/hip_runtime.h>

#include "level.h"

namespace plm {

constexpr int kT = 256;
constexpr int kChunk = 16;

// ------------------------------------------------------------------ relabel
__global__ void k_flag_present(const int32_t *zeta, int64_t n, int32_t *flag) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n) flag[zeta[u]] = 1;
}
__global__ void k_apply_map(const int32_t *zeta, const int64_t *newid, int64_t n, int32_t *pi) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n) pi[u] = (int32_t)newid[zeta[u]];
}

// Coarse ids ascend with the community ids: newid = exclusive prefix sum of
// the "community is non-empty" flags.
int64_t build_relabel(const int32_t *zeta, int64_t n, int32_t *pi, Scratch &scr, int64_t *host_i64,
                      hipStream_t st) {
    if (n == 0) return 0;
    scr.reserve(align_up(n * 4) + align_up(n * 8) + 256 + scan_scratch_bytes(n));
    int32_t *flag = (int32_t *)scr.get(n * 4);
    int64_t *newid = (int64_t *)scr.get(n * 8);
    int64_t *total = (int64_t *)scr.get(8);
    void *ss = scr.get(scan_scratch_bytes(n));
    HIPCHK(hipMemsetAsync(flag, 0, n * 4, st));
    hipLaunchKernelGGL(k_flag_present, dim3((unsigned)cdiv(n, kT)), dim3(kT), 0, st, zeta, n, flag);
    exclusive_scan_i32(flag, newid, n, total, ss, st);
    hipLaunchKernelGGL(k_apply_map, dim3((unsigned)cdiv(n, kT)), dim3(kT), 0, st, zeta, newid, n, pi);
    HIPCHK(hipMemcpyAsync(host_i64, total, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return host_i64[0];
}

int64_t count_communities(const int32_t *zeta, int64_t n, Scratch &scr, int64_t *host_i64, hipStream_t st) {
    if (n == 0) return 0;
    scr.reserve(align_up(n * 4) + align_up(n * 8) + 256 + scan_scratch_bytes(n));
    int32_t *flag = (int32_t *)scr.get(n * 4);
    int64_t *tmp = (int64_t *)scr.get(n * 8);
    int64_t *total = (int64_t *)scr.get(8);
    void *ss = scr.get(scan_scratch_bytes(n));
    HIPCHK(hipMemsetAsync(flag, 0, n * 4, st));
    hipLaunchKernelGGL(k_flag_present, dim3((unsigned)cdiv(n, kT)), dim3(kT), 0, st, zeta, n, flag);
    exclusive_scan_i32(flag, tmp, n, total, ss, st);
    HIPCHK(hipMemcpyAsync(host_i64, total, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return host_i64[0];
}

// ------------------------------------------------------------------ contraction
// key = (pi(u) << b) | pi(v), value = entry weight (self-loops times diag_mult,
// so the coarse diagonal is again "doubled").
//
// Packed items: when every entry's weight (times diag_mult) fits the wb =
// 64 - 2b bits below the key, an item is one word (key << wb) | w and the sort
// moves keys alone (half the bytes of key-value pairs).  A merged weight W
// above wmax = 2^wb - 1 is carried by ceil(W / wmax) items of the same key,
// which the reduction sums again; each of the c entries merged into W weighs
// at most wmax, so there are at most c of them and the item count stays within
// the entry count.
// Merged before the sort, per tile of kCTile consecutive entries: each entry
// (read lane by lane, coalesced) finds its row through the tile's row offsets
// staged in LDS (a binary search there; a global one when the tile spans a run
// of empty rows), and the tile's equal keys merge in an LDS hash table (within
// a row many neighbours fall into the same coarse node, and so do the rows of
// one community).  The workgroup appends its merged entries after a global
// cursor (one atomic).  Their order does not matter: the sort that follows
// orders them completely and equal keys' weights are summed.  Rows of graphs
// that are not kept (batched runs) are left out.
constexpr uint64_t kNoKey = ~0ULL;  // keys are below 2^(2b) <= 2^62
constexpr int kCTile = 1024;
constexpr int kCPer = kCTile / kT;
constexpr int kCBits = 11;
constexpr int kCSlots = 1 << kCBits;  // at most kCTile keys: load <= 1/2
static_assert(2 * kCTile <= kCSlots, "contraction merge table must never fill");
template <int WK, bool PK>
__global__ __launch_bounds__(kT) void k_contract_merge(GraphView g, const int32_t *pi, int b, int wb,
                                                       const uint8_t *keep, uint64_t *keys, int64_t *vals,
                                                       unsigned long long *cursor) {
    __shared__ int64_t soff[kCTile + 1];
    __shared__ uint64_t tk[kCSlots];
    __shared__ int64_t tv[kCSlots];
    __shared__ int64_t rr[2];
    __shared__ int32_t wsum[kT / kWave];
    __shared__ unsigned long long sbase;
    const int64_t E0 = (int64_t)blockIdx.x * kCTile;
    const int64_t E1 = E0 + kCTile < g.nnz ? E0 + kCTile : g.nnz;
    if (threadIdx.x == 0) rr[0] = row_of(g.off, g.n, E0);
    if (threadIdx.x == kWave) rr[1] = row_of(g.off, g.n, E1 - 1);
    for (int s = threadIdx.x; s < kCSlots; s += kT) { tk[s] = kNoKey; tv[s] = 0; }
    int32_t v[kCPer];
    int64_t x[kCPer];
#pragma unroll
    for (int q = 0; q < kCPer; ++q) {
        const int64_t e = E0 + q * kT + threadIdx.x;
        v[q] = e < E1 ? g.col[e] : 0;
        x[q] = e < E1 ? wload<WK>(g.w, e) : 0;
    }
    __syncthreads();
    const int64_t r0 = rr[0], nr = rr[1] - r0 + 1;
    const bool staged = nr <= kCTile;  // workgroup-uniform
    if (staged)
        for (int64_t j = threadIdx.x; j <= nr; j += kT) soff[j] = g.off[r0 + j];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kCPer; ++q) {
        const int64_t e = E0 + q * kT + threadIdx.x;
        if (e >= E1) continue;
        int64_t r;
        if (staged) {
            int lo = 0, hi = (int)nr;  // soff[lo] <= e < soff[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (soff[mid] <= e) lo = mid; else hi = mid;
            }
            r = r0 + lo;
        } else {
            r = row_of(g.off, g.n, e);
        }
        if (keep && !keep[g.gid[r]]) continue;
        int64_t w = x[q];
        if (v[q] == r) w *= g.diag_mult;
        const uint64_t key = ((uint64_t)pi[r] << b) | (uint64_t)pi[v[q]];
        uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ULL) >> (64 - kCBits));
        for (;;) {
            const uint64_t old = atomicCAS((unsigned long long *)&tk[h], (unsigned long long)kNoKey,
                                           (unsigned long long)key);
            if (old == kNoKey || old == key) {
                atomicAdd((unsigned long long *)&tv[h], (unsigned long long)w);
                break;
            }
            h = (h + 1) & (kCSlots - 1);
        }
    }
    __syncthreads();
    // each thread appends the keys of its kCSlots / kT slots (packed: a slot's
    // ceil(W / wmax) items, at least one)
    constexpr int kSP = kCSlots / kT;
    const uint64_t wmax = PK ? (1ULL << wb) - 1 : 0;
    int32_t cnt = 0;
#pragma unroll
    for (int j = 0; j < kSP; ++j) {
        const int s = threadIdx.x * kSP + j;
        if (tk[s] == kNoKey) continue;
        if (PK) {
            const uint64_t W = (uint64_t)tv[s];
            cnt += W > wmax ? (int32_t)((W + wmax - 1) / wmax) : 1;
        } else {
            ++cnt;
        }
    }
    int32_t inc = cnt;
    for (int d = 1; d < kWave; d <<= 1) {
        int32_t y = __shfl_up(inc, d);
        if (lane_id() >= d) inc += y;
    }
    if (lane_id() == kWave - 1) wsum[threadIdx.x / kWave] = inc;
    __syncthreads();
    int32_t before = 0, total = 0;
    for (int w = 0; w < kT / kWave; ++w) {
        if (w < (int)(threadIdx.x / kWave)) before += wsum[w];
        total += wsum[w];
    }
    if (threadIdx.x == 0) sbase = total ? atomicAdd(cursor, (unsigned long long)total) : 0ULL;
    __syncthreads();
    int64_t pos = (int64_t)sbase + before + (inc - cnt);
#pragma unroll
    for (int j = 0; j < kSP; ++j) {
        const int s = threadIdx.x * kSP + j;
        if (tk[s] == kNoKey) continue;
        if (PK) {
            const uint64_t k = tk[s] << wb;
            uint64_t W = (uint64_t)tv[s];
            do {
                const uint64_t part = W < wmax ? W : wmax;
                keys[pos++] = k | part;
                W -= part;
            } while (W > 0);
        } else {
            keys[pos] = tk[s];
            vals[pos] = tv[s];
            ++pos;
        }
    }
}

// the weight of every entry as uint32 (negative weights read as >= 2^31)
__global__ __launch_bounds__(kT) void k_weight_max(const int32_t *w, int64_t nnz, unsigned int *out) {
    uint32_t m = 0;
    const int64_t stride = (int64_t)gridDim.x * kT;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < nnz; i += 4 * stride) {
        uint32_t x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = i + q * stride < nnz ? (uint32_t)w[i + q * stride] : 0u;
#pragma unroll
        for (int q = 0; q < 4; ++q) m = x[q] > m ? x[q] : m;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)m, d);
        m = o > m ? o : m;
    }
    if (lane_id() == 0 && m) atomicMax(out, m);
}

// packed items (PK) compare their keys above bit wb
template <bool PK>
__global__ void k_head_flags(const uint64_t *keys, int64_t n, int wb, int32_t *head) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const uint64_t k = PK ? keys[i] >> wb : keys[i];
        head[i] = (i == 0 || k != (PK ? keys[i - 1] >> wb : keys[i - 1])) ? 1 : 0;
    }
}

// Reduce-by-key over sorted keys.  Run id of item i = incl_scan(head)[i] - 1 =
// excl[i] + head[i] - 1.  The items of a block are read lane by lane
// (coalesced, all loads of a thread in flight together) and added into their
// run's LDS slot; a run that lies wholly inside the block is stored, a run
// crossing a block edge is added atomically (out_w zeroed first).
constexpr int kRbkItems = kT * kChunk;
template <bool PK>
__global__ __launch_bounds__(kT) void k_reduce_by_key(const uint64_t *keys, const int64_t *vals, const int32_t *head,
                                                      const int64_t *excl, int64_t n, int wb, uint64_t *out_k,
                                                      int64_t *out_w) {
    __shared__ int64_t acc[kRbkItems];
    int64_t blk0 = (int64_t)blockIdx.x * kRbkItems;
    int64_t blk1 = blk0 + kRbkItems < n ? blk0 + kRbkItems : n;
    int64_t run0 = excl[blk0] + head[blk0] - 1;  // run id of the block's first item
    for (int i = threadIdx.x; i < kRbkItems; i += kT) acc[i] = 0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kChunk; ++q) {
        const int64_t i = blk0 + (int64_t)q * kT + threadIdx.x;
        if (i < blk1) {
            const int32_t h = head[i];
            const int64_t r = excl[i] + h - 1;
            const uint64_t k = keys[i];
            if (h) out_k[r] = PK ? k >> wb : k;
            const uint64_t w = PK ? k & ((1ULL << wb) - 1) : (uint64_t)vals[i];
            atomicAdd((unsigned long long *)&acc[r - run0], (unsigned long long)w);
        }
    }
    __syncthreads();
    int64_t last_run = excl[blk1 - 1] + head[blk1 - 1] - 1;
    int64_t nruns = last_run - run0 + 1;
    bool first_complete = head[blk0] != 0;
    bool last_complete = (blk1 == n) || head[blk1] != 0;
    for (int64_t j = threadIdx.x; j < nruns; j += kT) {
        bool whole = (j > 0 || first_complete) && (j < nruns - 1 || last_complete);
        if (whole) out_w[run0 + j] = acc[j];
        else atomicAdd((unsigned long long *)&out_w[run0 + j], (unsigned long long)acc[j]);
    }
}

// coarse columns: the low b bits of each unique key
__global__ void k_coarse_col(const uint64_t *ukeys, int64_t m, int b, int32_t *ccol) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) ccol[i] = (int32_t)(ukeys[i] & ((b >= 64) ? ~0ULL : ((1ULL << b) - 1)));
}
// coarse offsets: coff[r] = first unique entry with row >= r (a binary search
// per row, so runs of empty rows cost nothing extra)
__global__ void k_coarse_off(const uint64_t *ukeys, int64_t m, int b, int64_t k, int64_t *coff) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > k) return;
    int64_t lo = 0, hi = m;  // first i in [0, m] with (ukeys[i] >> b) >= r
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)(ukeys[mid] >> b) < r) lo = mid + 1;
        else hi = mid;
    }
    coff[r] = lo;
}

int64_t build_contraction(const GraphView &g, const int32_t *pi, int64_t k, int64_t **coff_out, int32_t **ccol_out,
                          int64_t **cw_out, Scratch &scr, int64_t *host_i64, hipStream_t st, const uint8_t *keep,
                          int pack_bits) {
    int64_t nnz = g.nnz;
    int b = ceil_log2((uint64_t)(k > 1 ? k : 2));
    int64_t nb = nnz > 0 ? nnz : 1;
    scr.reserve(4 * align_up(nb * 8) + align_up(nb * 4) + align_up(nb * 8) + 256 +
                (radix_scratch_bytes(nb) > scan_scratch_bytes(nb) ? radix_scratch_bytes(nb) : scan_scratch_bytes(nb)));
    uint64_t *ka = (uint64_t *)scr.get(nb * 8), *kb = (uint64_t *)scr.get(nb * 8);
    int64_t *va = (int64_t *)scr.get(nb * 8), *vb = (int64_t *)scr.get(nb * 8);
    int32_t *head = (int32_t *)scr.get(nb * 4);
    int64_t *excl = (int64_t *)scr.get(nb * 8);
    int64_t *total = (int64_t *)scr.get(8);
    size_t tmpb = radix_scratch_bytes(nb) > scan_scratch_bytes(nb) ? radix_scratch_bytes(nb) : scan_scratch_bytes(nb);
    void *tmp = scr.get(tmpb);
    int64_t *coff = nullptr;
    int32_t *ccol = nullptr;
    int64_t *cw = nullptr;
    auto fail = [&](hipError_t e) {
        if (coff) (void)hipFree(coff);
        if (ccol) (void)hipFree(ccol);
        if (cw) (void)hipFree(cw);
        (void)hipGetLastError();
        throw Error{-3, std::string("coarse graph allocation failed: ") + hipGetErrorString(e)};
    };
    hipError_t e = hipMalloc(&coff, (k + 1) * 8);
    if (e != hipSuccess) fail(e);
    if (nnz == 0) {
        HIPCHK(hipMemsetAsync(coff, 0, (k + 1) * 8, st));
        e = hipMalloc(&ccol, 4);
        if (e != hipSuccess) fail(e);
        e = hipMalloc(&cw, 8);
        if (e != hipSuccess) fail(e);
        *coff_out = coff; *ccol_out = ccol; *cw_out = cw;
        return 0;
    }
    const dim3 grid((unsigned)cdiv(nnz, kCTile));
    unsigned long long *cursor = (unsigned long long *)total;
    // packed items for 32-bit (or unit) weights whose largest entry, times
    // diag_mult, fits below the key (in at most pack_bits bits when that is set)
    const int wb = pack_bits > 0 && pack_bits < 64 - 2 * b ? pack_bits : 64 - 2 * b;
    bool pk = false;
    if (pack_bits >= 0 && g.wkind <= 1 && wb >= 2) {
        uint64_t wtop = 1;
        if (g.wkind == 1) {
            unsigned int *wm = (unsigned int *)cursor;
            HIPCHK(hipMemsetAsync(wm, 0, 8, st));
            const int64_t blocks = cdiv(nnz, 4 * kT);
            hipLaunchKernelGGL(k_weight_max, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(kT), 0, st,
                               (const int32_t *)g.w, nnz, wm);
            HIPCHK(hipMemcpyAsync(host_i64, wm, 8, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            wtop = (uint64_t)(uint32_t)host_i64[0];
        }
        pk = wtop <= (uint64_t)INT32_MAX && wtop * (uint64_t)(g.diag_mult > 1 ? g.diag_mult : 1) <= (1ULL << wb) - 1;
    }
    HIPCHK(hipMemsetAsync(cursor, 0, 8, st));
#define PLM_MERGE(WK, PK)                                                                                        \
    hipLaunchKernelGGL((k_contract_merge<WK, PK>), grid, dim3(kT), 0, st, g, pi, b, wb, keep, ka, va, cursor)
    switch (g.wkind) {
        case 0: if (pk) PLM_MERGE(0, true); else PLM_MERGE(0, false); break;
        case 1: if (pk) PLM_MERGE(1, true); else PLM_MERGE(1, false); break;
        default: PLM_MERGE(2, false); break;
    }
#undef PLM_MERGE
    HIPCHK(hipMemcpyAsync(host_i64, cursor, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    nnz = host_i64[0];  // merged entries (kept rows only)
    if (pk) radix_sort_u64_keys(&ka, &kb, nnz, wb, 2 * b, tmp, st);
    else radix_sort_u64_i64(&ka, &va, &kb, &vb, nnz, 2 * b, tmp, st);
    if (nnz == 0) {
        HIPCHK(hipMemsetAsync(coff, 0, (k + 1) * 8, st));
        e = hipMalloc(&ccol, 4);
        if (e != hipSuccess) fail(e);
        e = hipMalloc(&cw, 8);
        if (e != hipSuccess) fail(e);
        *coff_out = coff; *ccol_out = ccol; *cw_out = cw;
        return 0;
    }
    if (pk) hipLaunchKernelGGL(k_head_flags<true>, dim3((unsigned)cdiv(nnz, kT)), dim3(kT), 0, st, ka, nnz, wb, head);
    else hipLaunchKernelGGL(k_head_flags<false>, dim3((unsigned)cdiv(nnz, kT)), dim3(kT), 0, st, ka, nnz, wb, head);
    exclusive_scan_i32(head, excl, nnz, total, tmp, st);
    HIPCHK(hipMemcpyAsync(host_i64, total, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int64_t m = host_i64[0];
    e = hipMalloc(&ccol, (m > 0 ? m : 1) * 4);
    if (e != hipSuccess) fail(e);
    e = hipMalloc(&cw, (m > 0 ? m : 1) * 8);
    if (e != hipSuccess) fail(e);
    // unique keys go to kb (free after the sort), summed weights to cw
    HIPCHK(hipMemsetAsync(cw, 0, m * 8, st));
    if (pk)
        hipLaunchKernelGGL(k_reduce_by_key<true>, dim3((unsigned)cdiv(nnz, kRbkItems)), dim3(kT), 0, st, ka, va, head,
                           excl, nnz, wb, kb, cw);
    else
        hipLaunchKernelGGL(k_reduce_by_key<false>, dim3((unsigned)cdiv(nnz, kRbkItems)), dim3(kT), 0, st, ka, va,
                           head, excl, nnz, wb, kb, cw);
    hipLaunchKernelGGL(k_coarse_col, dim3((unsigned)cdiv(m, kT)), dim3(kT), 0, st, kb, m, b, ccol);
    hipLaunchKernelGGL(k_coarse_off, dim3((unsigned)cdiv(k + 1, kT)), dim3(kT), 0, st, kb, m, b, k, coff);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    *coff_out = coff; *ccol_out = ccol; *cw_out = cw;
    return m;
}

// ------------------------------------------------------------------ prolongation / labels
__global__ void k_compose(int32_t *lab, const int32_t *map, int64_t n) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) lab[v] = map[lab[v]];
}
void launch_compose(int32_t *lab, const int32_t *map, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_compose, dim3((unsigned)cdiv(n, kT)), dim3(kT), 0, st, lab, map, n);
    HIPCHK(hipGetLastError());
}
__global__ void k_iota(int32_t *a, int64_t n) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) a[v] = (int32_t)v;
}
// volC[x] = sum of vol[u] over the nodes u with zeta[u] = x (volC zeroed first)
__global__ void k_comm_vol(const int32_t *zeta, const int64_t *vol, int64_t n, int64_t *volC) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t x = u < n ? vol[u] : 0;
    int32_t c = x ? zeta[u] : 0;
    if (wave_group_sum(c, x != 0, x)) atomicAdd((unsigned long long *)&volC[c], (unsigned long long)x);
}
void launch_comm_vol(const int32_t *zeta, const int64_t *vol, int64_t n, int64_t *volC, hipStream_t st) {
    if (n <= 0) return;
    HIPCHK(hipMemsetAsync(volC, 0, n * 8, st));
    hipLaunchKernelGGL(k_comm_vol, dim3((unsigned)cdiv(n, kT)), dim3(kT), 0, st, zeta, vol, n, volC);
    HIPCHK(hipGetLastError());
}
// *flag = 1 if a and b differ anywhere in [0, n) (flag cleared by the caller)
__global__ void k_differ(const int32_t *a, const int32_t *b, int64_t n, int32_t *flag) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (a[i] != b[i]) {
            *flag = 1;
            return;
        }
}
void launch_differ(const int32_t *a, const int32_t *b, int64_t n, int32_t *flag, hipStream_t st) {
    if (n <= 0) return;
    int64_t blocks = cdiv(n, kT);
    hipLaunchKernelGGL(k_differ, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(kT), 0, st, a, b, n, flag);
    HIPCHK(hipGetLastError());
}
void launch_iota(int32_t *a, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_iota, dim3((unsigned)cdiv(n, kT)), dim3(kT), 0, st, a, n);
    HIPCHK(hipGetLastError());
}
void launch_copy_vol(int64_t *dst, const int64_t *src, int64_t n, hipStream_t st) {
    if (n > 0) HIPCHK(hipMemcpyAsync(dst, src, n * 8, hipMemcpyDeviceToDevice, st));
}

// canonical label of v = number of distinct labels whose first node precedes
// the first node of v's label
__global__ void k_first_min(const int32_t *lab, int64_t n, int32_t *first) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t l = v < n ? lab[v] : 0;
    int64_t unused = 0;
    // a group's leader is its lowest lane, which holds the group's smallest v
    if (wave_group_sum(l, v < n, unused)) atomicMin(&first[l], (int32_t)v);
}
__global__ void k_is_first(const int32_t *lab, const int32_t *first, int64_t n, int32_t *isf) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) isf[v] = first[lab[v]] == (int32_t)v ? 1 : 0;
}
__global__ void k_canon(const int32_t *lab, const int32_t *first, const int64_t *rank, int64_t n, int32_t *out) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) out[v] = (int32_t)rank[first[lab[v]]];
}
__global__ void k_fill_i32(int32_t *a, int64_t n, int32_t x) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) a[v] = x;
}

void build_canonical(const int32_t *lab, int64_t n, int32_t *out, Scratch &scr, hipStream_t st) {
    if (n == 0) return;
    scr.reserve(2 * align_up(n * 4) + align_up(n * 8) + scan_scratch_bytes(n));
    int32_t *first = (int32_t *)scr.get(n * 4);
    int32_t *isf = (int32_t *)scr.get(n * 4);
    int64_t *rank = (int64_t *)scr.get(n * 8);
    void *ss = scr.get(scan_scratch_bytes(n));
    dim3 grid((unsigned)cdiv(n, kT));
    hipLaunchKernelGGL(k_fill_i32, grid, dim3(kT), 0, st, first, n, (int32_t)0x7fffffff);
    hipLaunchKernelGGL(k_first_min, grid, dim3(kT), 0, st, lab, n, first);
    hipLaunchKernelGGL(k_is_first, grid, dim3(kT), 0, st, lab, first, n, isf);
    exclusive_scan_i32(isf, rank, n, nullptr, ss, st);
    hipLaunchKernelGGL(k_canon, grid, dim3(kT), 0, st, lab, first, rank, n, out);
    HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------------ modularity
__global__ void k_label_check(const int32_t *lab, int64_t n, int32_t *bad) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n && (lab[v] < 0 || lab[v] >= n)) atomicOr(bad, 1);
}
__global__ void k_label_vol(const int32_t *lab, const int64_t *vol, int64_t n, int64_t *volL) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t x = v < n ? vol[v] : 0;
    int32_t l = x ? lab[v] : 0;
    if (wave_group_sum(l, x != 0, x)) atomicAdd((unsigned long long *)&volL[l], (unsigned long long)x);
}
// I2 = sum of intra-label entries with self-loops times diag_mult.  A
// workgroup takes kITile consecutive entries (read lane by lane) and finds
// each entry's row through the tile's row offsets staged in LDS (a binary
// search; a global one when the tile spans a run of empty rows); one atomic
// per workgroup.
constexpr int kITile = 2048;
constexpr int kIPer = kITile / kT;
template <int WK>
__global__ __launch_bounds__(kT) void k_intra(GraphView g, const int32_t *lab, unsigned long long *I2) {
    __shared__ int64_t soff[kITile + 1];
    __shared__ int64_t rr[2];
    const int64_t E0 = (int64_t)blockIdx.x * kITile;
    const int64_t E1 = E0 + kITile < g.nnz ? E0 + kITile : g.nnz;
    if (threadIdx.x == 0) rr[0] = row_of(g.off, g.n, E0);
    if (threadIdx.x == kWave) rr[1] = row_of(g.off, g.n, E1 - 1);
    int32_t v[kIPer], lv[kIPer];
#pragma unroll
    for (int q = 0; q < kIPer; ++q) {
        const int64_t e = E0 + q * kT + threadIdx.x;
        v[q] = e < E1 ? g.col[e] : 0;
    }
#pragma unroll
    for (int q = 0; q < kIPer; ++q) lv[q] = lab[v[q]];
    __syncthreads();
    const int64_t r0 = rr[0], nr = rr[1] - r0 + 1;
    const bool staged = nr <= kITile;  // workgroup-uniform
    if (staged)
        for (int64_t j = threadIdx.x; j <= nr; j += kT) soff[j] = g.off[r0 + j];
    __syncthreads();
    int64_t s = 0;
#pragma unroll
    for (int q = 0; q < kIPer; ++q) {
        const int64_t e = E0 + q * kT + threadIdx.x;
        if (e >= E1) continue;
        int64_t r;
        if (staged) {
            int lo = 0, hi = (int)nr;  // soff[lo] <= e < soff[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (soff[mid] <= e) lo = mid; else hi = mid;
            }
            r = r0 + lo;
        } else {
            r = row_of(g.off, g.n, e);
        }
        if (lv[q] != lab[r]) continue;
        int64_t x = wload<WK>(g.w, e);
        if (v[q] == r) x *= g.diag_mult;
        s += x;
    }
    block_count_add(I2, (unsigned long long)s);
}
// sum of volL^2 as 128-bit: per-thread squares, wave sums, two-word atomic add
__global__ __launch_bounds__(kT) void k_sum_sq(const int64_t *volL, int64_t n, unsigned long long *acc2) {
    unsigned __int128 s = 0;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
        unsigned __int128 x = (unsigned __int128)(uint64_t)volL[i];
        s += x * x;
    }
    uint64_t lo = (uint64_t)s, hi = (uint64_t)(s >> 64);
    for (int d = 32; d >= 1; d >>= 1) {
        uint64_t olo = __shfl_xor(lo, d), ohi = __shfl_xor(hi, d);
        uint64_t nlo = lo + olo;
        hi = hi + ohi + (nlo < lo ? 1 : 0);
        lo = nlo;
    }
    if (lane_id() == 0 && (lo || hi)) {
        unsigned long long old = atomicAdd(&acc2[0], (unsigned long long)lo);
        uint64_t carry = (old + lo < old) ? 1 : 0;
        if (hi + carry) atomicAdd(&acc2[1], (unsigned long long)(hi + carry));
    }
}

// zero fill of n int64 words (a kernel rather than a memset node, so a caller
// may capture it)
__global__ void k_zero_i64(int64_t *a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) a[i] = 0;
}

size_t modularity_ws_bytes(int64_t n) { return align_up((size_t)(n > 0 ? n : 1) * 8) + 4 * 8; }

int modularity_parts_ws(const GraphView &g0, const int64_t *vol0, const int32_t *labels, int64_t S, void *ws,
                        int64_t *host_i64, __int128 *num, __int128 *den, hipStream_t st) {
    int64_t n = g0.n;
    *den = (__int128)S * (__int128)S;
    if (n == 0) { *num = 0; return 0; }
    int64_t *volL = (int64_t *)ws;
    unsigned long long *cnt = (unsigned long long *)((char *)ws + align_up((size_t)n * 8));  // [I2, sq lo, sq hi, bad]
    const int64_t nb = cdiv(n, kT);
    hipLaunchKernelGGL(k_zero_i64, dim3((unsigned)(nb < 2048 ? nb : 2048)), dim3(kT), 0, st, volL, n);
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(kT), 0, st, (int64_t *)cnt, (int64_t)4);
    dim3 grid((unsigned)nb);
    hipLaunchKernelGGL(k_label_check, grid, dim3(kT), 0, st, labels, n, (int32_t *)(cnt + 3));
    HIPCHK(hipMemcpyAsync(host_i64, cnt + 3, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (host_i64[0] != 0) return -1;
    hipLaunchKernelGGL(k_label_vol, grid, dim3(kT), 0, st, labels, vol0, n, volL);
    if (g0.nnz > 0) {
        dim3 eg((unsigned)cdiv(g0.nnz, kITile));
        switch (g0.wkind) {
            case 0: hipLaunchKernelGGL(k_intra<0>, eg, dim3(kT), 0, st, g0, labels, cnt); break;
            case 1: hipLaunchKernelGGL(k_intra<1>, eg, dim3(kT), 0, st, g0, labels, cnt); break;
            default: hipLaunchKernelGGL(k_intra<2>, eg, dim3(kT), 0, st, g0, labels, cnt); break;
        }
    }
    hipLaunchKernelGGL(k_sum_sq, dim3((unsigned)(nb < 2048 ? nb : 2048)), dim3(kT), 0, st, volL, n, cnt + 1);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(host_i64, cnt, 3 * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    unsigned __int128 sq = ((unsigned __int128)(uint64_t)host_i64[2] << 64) | (uint64_t)host_i64[1];
    *num = (__int128)S * (__int128)host_i64[0] - (__int128)sq;
    return 0;
}

int modularity_parts(const GraphView &g0, const int64_t *vol0, const int32_t *labels, int64_t S, Scratch &scr,
                     int64_t *host_i64, __int128 *num, __int128 *den, hipStream_t st) {
    if (g0.n == 0) return modularity_parts_ws(g0, vol0, labels, S, nullptr, host_i64, num, den, st);
    scr.reserve(modularity_ws_bytes(g0.n));
    void *ws = scr.get(modularity_ws_bytes(g0.n));
    return modularity_parts_ws(g0, vol0, labels, S, ws, host_i64, num, den, st);
}

// ------------------------------------------------------------------ validation
// bit 1: col out of range; 2: non-positive weight; 4: row not strictly
// ascending; 8: missing or unequal mirror entry; 16: offsets not monotone
template <int WK>
__global__ __launch_bounds__(kT) void k_validate(GraphView g, uint32_t *bad) {
    int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= g.nnz) return;
    int64_t r = row_of(g.off, g.n, e);
    int32_t v = g.col[e];
    uint32_t f = 0;
    if (v < 0 || v >= g.n) {
        atomicOr(bad, 1u);
        return;
    }
    int64_t x = wload<WK>(g.w, e);
    if (x <= 0) f |= 2u;
    if (e > g.off[r] && g.col[e - 1] >= v) f |= 4u;
    if (v != r) {
        // binary search for r in row v
        int64_t lo = g.off[v], hi = g.off[v + 1];
        bool found = false;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            int32_t c = g.col[mid];
            if (c == r) { found = true; lo = mid; break; }
            if (c < r) lo = mid + 1; else hi = mid;
        }
        if (!found || wload<WK>(g.w, lo) != x) f |= 8u;
    }
    if (f) atomicOr(bad, f);
}
__global__ void k_validate_off(const int64_t *off, int64_t n, int64_t nnz, uint32_t *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && off[i + 1] < off[i]) atomicOr(bad, 16u);
    if (i == 0 && (off[0] != 0 || off[n] != nnz)) atomicOr(bad, 16u);
}

uint32_t validate_graph(const GraphView &g, Scratch &scr, int64_t *host_i64, hipStream_t st) {
    scr.reserve(256);
    uint32_t *bad = (uint32_t *)scr.get(8);
    HIPCHK(hipMemsetAsync(bad, 0, 8, st));
    hipLaunchKernelGGL(k_validate_off, dim3((unsigned)cdiv(g.n + 1, kT)), dim3(kT), 0, st, g.off, g.n, g.nnz, bad);
    HIPCHK(hipMemcpyAsync(host_i64, bad, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (host_i64[0] & 0xffffffff) return (uint32_t)host_i64[0];
    if (g.nnz > 0) {
        dim3 grid((unsigned)cdiv(g.nnz, kT));
        switch (g.wkind) {
            case 0: hipLaunchKernelGGL(k_validate<0>, grid, dim3(kT), 0, st, g, bad); break;
            case 1: hipLaunchKernelGGL(k_validate<1>, grid, dim3(kT), 0, st, g, bad); break;
            default: hipLaunchKernelGGL(k_validate<2>, grid, dim3(kT), 0, st, g, bad); break;
        }
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(host_i64, bad, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return (uint32_t)(host_i64[0] & 0xffffffff);
}

}  // namespace plm
