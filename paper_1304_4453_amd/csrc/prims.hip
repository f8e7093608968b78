// prims.hip - device primitives of libplm: exclusive scan and a stable LSD
// radix sort of (key, value) pairs, written for wave64 (gfx950).
#include <hip/hip_runtime.h>

#include "plm_internal.h"

namespace plm {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ------------------------------------------------------------------ scan
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int64_t kScanTile = kScanThreads * kScanItems;

// inclusive scan of one int64 per thread across a 256-thread block; returns
// the exclusive prefix of this thread and the block total in *total
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t x, int64_t *total) {
    __shared__ int64_t wsum[kScanThreads / kWave];
    const int lane = lane_id(), w = threadIdx.x / kWave;
    int64_t inc = x;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int64_t y = __shfl_up(inc, d);
        if (lane >= d) inc += y;
    }
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kScanThreads / kWave; ++i) {
        if (i < w) before += wsum[i];
        all += wsum[i];
    }
    __syncthreads();
    *total = all;
    return before + inc - x;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_tile_reduce(const T *in, int64_t n, int64_t *sums) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j)
        if (base + j < n) s += (int64_t)in[base + j];
    int64_t total;
    (void)block_exclusive_scan(s, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// exclusive scan of each tile plus the tile's offset (tile_off may be null)
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_tile_scan(const T *in, int64_t *out, int64_t n,
                                                            const int64_t *tile_off, int64_t *total_dev) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = (base + j < n) ? (int64_t)in[base + j] : 0;
        s += v[j];
    }
    int64_t total;
    int64_t run = block_exclusive_scan(s, &total) + (tile_off ? tile_off[blockIdx.x] : 0);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
    if (total_dev && blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) *total_dev = run;
}

__global__ void k_set_i64(int64_t *p, int64_t v) { *p = v; }

size_t scan_scratch_bytes(int64_t n) {
    size_t b = 0;
    while (n > kScanTile) {
        int64_t t = cdiv(n, kScanTile);
        b += 2 * align_up((size_t)t * sizeof(int64_t));
        n = t;
    }
    return b + 256;
}

template <typename T>
static void scan_impl(const T *in, int64_t *out, int64_t n, int64_t *total_dev, char *scratch, hipStream_t st) {
    if (n <= 0) {
        if (total_dev) hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, st, total_dev, (int64_t)0);
        return;
    }
    int64_t tiles = cdiv(n, kScanTile);
    if (tiles == 1) {
        hipLaunchKernelGGL((k_tile_scan<T>), dim3(1), dim3(kScanThreads), 0, st, in, out, n, (const int64_t *)nullptr,
                           total_dev);
        return;
    }
    int64_t *sums = (int64_t *)scratch;
    int64_t *sums_scanned = (int64_t *)(scratch + align_up((size_t)tiles * sizeof(int64_t)));
    char *rest = scratch + 2 * align_up((size_t)tiles * sizeof(int64_t));
    hipLaunchKernelGGL((k_tile_reduce<T>), dim3(tiles), dim3(kScanThreads), 0, st, in, n, sums);
    scan_impl<int64_t>(sums, sums_scanned, tiles, nullptr, rest, st);
    hipLaunchKernelGGL((k_tile_scan<T>), dim3(tiles), dim3(kScanThreads), 0, st, in, out, n,
                       (const int64_t *)sums_scanned, total_dev);
}

void exclusive_scan_i32(const int32_t *in, int64_t *out, int64_t n, int64_t *total_dev, void *scratch,
                        hipStream_t st) {
    scan_impl<int32_t>(in, out, n, total_dev, (char *)scratch, st);
    HIPCHK(hipGetLastError());
}
void exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total_dev, void *scratch,
                        hipStream_t st) {
    scan_impl<int64_t>(in, out, n, total_dev, (char *)scratch, st);
    HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------------ radix sort
constexpr int kRadixThreads = 256;
constexpr int kRadixRounds = 16;
constexpr int64_t kRadixTile = (int64_t)kRadixThreads * kRadixRounds;
constexpr int kRadixWaves = kRadixThreads / kWave;

template <typename K>
__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(const K *keys, int64_t n, int shift, int32_t *counts,
                                                              int64_t ntiles) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll 4
    for (int r = 0; r < kRadixRounds; ++r) {
        int64_t i = base + (int64_t)r * kRadixThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = (int32_t)h[threadIdx.x];
}

// Items of a tile are taken 256 at a time in input order; within such a round
// a lane's rank among equal digits comes from 8 ballots (one per digit bit),
// so equal keys keep their input order (stability).  The tile is first sorted
// by digit in LDS (its digit starts are the exclusive scan of its histogram
// counts), then written out in LDS order: consecutive threads write
// consecutive positions of a digit's run, so the stores coalesce.  KV = false
// sorts keys alone (vin / vout unused): half the LDS and traffic of 8-byte
// key-value pairs.
template <typename K, typename V, bool KV>
__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(const K *kin, const V *vin, K *kout, V *vout,
                                                                 int64_t n, int shift, const int64_t *offsets,
                                                                 const int32_t *counts, int64_t ntiles) {
    __shared__ uint32_t running[256];
    __shared__ uint32_t wcnt[kRadixWaves][256];
    __shared__ uint32_t lstart[256];
    __shared__ uint32_t wsum[kRadixWaves];
    __shared__ int64_t gofs[256];
    __shared__ K sk[kRadixTile];
    __shared__ V sv[KV ? kRadixTile : 1];
    const int tid = threadIdx.x, w = tid / kWave, lane = lane_id();
    running[tid] = 0;
#pragma unroll
    for (int i = 0; i < kRadixWaves; ++i) wcnt[i][tid] = 0;
    gofs[tid] = offsets[(int64_t)tid * ntiles + blockIdx.x];
    // exclusive scan of the tile's 256 digit counts (thread t holds digit t)
    const uint32_t cnt = (uint32_t)counts[(int64_t)tid * ntiles + blockIdx.x];
    uint32_t inc = cnt;
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t y = __shfl_up(inc, d);
        if (lane >= d) inc += y;
    }
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int j = 0; j < w; ++j) before += wsum[j];
    lstart[tid] = before + inc - cnt;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ULL : (~0ULL >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    // the tile's items are loaded together (one memory latency per tile)
    K kr[kRadixRounds];
    V vr[KV ? kRadixRounds : 1];
#pragma unroll
    for (int r = 0; r < kRadixRounds; ++r) {
        const int64_t i = base + (int64_t)r * kRadixThreads + tid;
        kr[r] = i < n ? kin[i] : (K)0;
        if constexpr (KV) vr[r] = i < n ? vin[i] : (V)0;
    }
#pragma unroll
    for (int r = 0; r < kRadixRounds; ++r) {
        const bool valid = base + (int64_t)r * kRadixThreads + tid < n;
        const K k = kr[r];
        uint32_t d = (uint32_t)(k >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pre = running[d];
            for (int j = 0; j < w; ++j) pre += wcnt[j][d];
            const uint32_t lp = lstart[d] + pre + rank;
            sk[lp] = k;
            if constexpr (KV) sv[lp] = vr[r];
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int j = 0; j < kRadixWaves; ++j) {
            add += wcnt[j][tid];
            wcnt[j][tid] = 0;
        }
        running[tid] += add;
        __syncthreads();
    }
    const int64_t left = n - base;
    const int tn = left < kRadixTile ? (int)left : (int)kRadixTile;
    for (int j = tid; j < tn; j += kRadixThreads) {
        const K k = sk[j];
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        const int64_t pos = gofs[d] + (int64_t)(j - (int)lstart[d]);
        kout[pos] = k;
        if constexpr (KV) vout[pos] = sv[j];
    }
}

size_t radix_scratch_bytes(int64_t n) {
    int64_t ntiles = cdiv(n > 0 ? n : 1, kRadixTile);
    int64_t m = 256 * ntiles;
    return align_up((size_t)m * sizeof(int32_t)) + align_up((size_t)m * sizeof(int64_t)) + scan_scratch_bytes(m);
}

// LSD passes over key bits [lo, lo + bits), 8 at a time (lo + bits <= 8 *
// sizeof(K) + 7: bits above the key read as zero)
template <typename K, typename V, bool KV>
static void radix_impl(K **keys, V **vals, K **keys_alt, V **vals_alt, int64_t n, int lo, int bits, void *scratch,
                       hipStream_t st) {
    if (n <= 1 || bits <= 0) return;
    int64_t ntiles = cdiv(n, kRadixTile);
    int64_t m = 256 * ntiles;
    char *s = (char *)scratch;
    int32_t *counts = (int32_t *)s;
    int64_t *offsets = (int64_t *)(s + align_up((size_t)m * sizeof(int32_t)));
    char *scan_tmp = s + align_up((size_t)m * sizeof(int32_t)) + align_up((size_t)m * sizeof(int64_t));
    for (int shift = lo; shift < lo + bits; shift += 8) {
        hipLaunchKernelGGL((k_radix_hist<K>), dim3(ntiles), dim3(kRadixThreads), 0, st, *keys, n, shift, counts,
                           ntiles);
        exclusive_scan_i32(counts, offsets, m, nullptr, scan_tmp, st);
        hipLaunchKernelGGL((k_radix_scatter<K, V, KV>), dim3(ntiles), dim3(kRadixThreads), 0, st, *keys, *vals,
                           *keys_alt, *vals_alt, n, shift, (const int64_t *)offsets, (const int32_t *)counts, ntiles);
        K *tk = *keys; *keys = *keys_alt; *keys_alt = tk;
        V *tv = *vals; *vals = *vals_alt; *vals_alt = tv;
    }
    HIPCHK(hipGetLastError());
}

void radix_sort_u32_i32(uint32_t **k, int32_t **v, uint32_t **ka, int32_t **va, int64_t n, int bits, void *s,
                        hipStream_t st) {
    radix_impl<uint32_t, int32_t, true>(k, v, ka, va, n, 0, bits, s, st);
}
void radix_sort_u64_i32(uint64_t **k, int32_t **v, uint64_t **ka, int32_t **va, int64_t n, int bits, void *s,
                        hipStream_t st) {
    radix_impl<uint64_t, int32_t, true>(k, v, ka, va, n, 0, bits, s, st);
}
void radix_sort_u64_i64(uint64_t **k, int64_t **v, uint64_t **ka, int64_t **va, int64_t n, int bits, void *s,
                        hipStream_t st) {
    radix_impl<uint64_t, int64_t, true>(k, v, ka, va, n, 0, bits, s, st);
}
void radix_sort_u64_keys(uint64_t **k, uint64_t **ka, int64_t n, int lo, int bits, void *s, hipStream_t st) {
    int32_t *nv = nullptr, *nva = nullptr;  // no values
    radix_impl<uint64_t, int32_t, false>(k, &nv, ka, &nva, n, lo, bits, s, st);
}

// ------------------------------------------------------------------ host helpers
void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) throw Error{-4, std::string(what) + ": " + hipGetErrorString(e)};
}

Scratch::~Scratch() {
    if (base_) (void)hipFree(base_);
}

void Scratch::reserve(size_t bytes) {
    used_ = 0;
    if (bytes <= cap_) return;
    // work queued on the owner's stream may still use the old buffer
    if (base_) {
        HIPCHK(hipStreamSynchronize(stream_));
        HIPCHK(hipFree(base_));
    }
    base_ = nullptr;
    cap_ = 0;
    size_t want = align_up(bytes + bytes / 8 + 4096, 1 << 20);
    hipError_t e = hipMalloc(&base_, want);
    if (e != hipSuccess) {
        base_ = nullptr;
        (void)hipGetLastError();
        throw Error{-3, "device scratch allocation of " + std::to_string(want) + " bytes failed"};
    }
    cap_ = want;
}

void *Scratch::get(size_t bytes) {
    size_t b = align_up(bytes > 0 ? bytes : 1);
    if (used_ + b > cap_) throw Error{-6, "internal: scratch overflow"};
    void *p = base_ + used_;
    used_ += b;
    return p;
}

}  // namespace plm
