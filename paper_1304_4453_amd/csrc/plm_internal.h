// plm_internal.h - shared declarations of the libplm HIP sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

namespace plm {

constexpr int kWave = 64;
constexpr int32_t kEmpty = -1;  // empty hash slot / "stay" decision

// ------------------------------------------------------------------ device helpers
// SplitMix64 step (Steele, Lea & Flood 2014) from state x.
__device__ __host__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Hash part of the priority of node u at a level; full priority is (hash, u).
__device__ __host__ __forceinline__ uint64_t prio_hash(uint64_t seed, int32_t level, int64_t u) {
    return splitmix64(seed ^ ((uint64_t)(uint32_t)level << 40) ^ (uint64_t)u);
}

// true iff (ha, a) > (hb, b)
__device__ __host__ __forceinline__ bool prio_greater(uint64_t ha, int64_t a, uint64_t hb, int64_t b) {
    return ha > hb || (ha == hb && a > b);
}

// Entry weight: WK = 0 unit, 1 int32, 2 int64.
template <int WK>
__device__ __forceinline__ int64_t wload(const void *w, int64_t e) {
    if constexpr (WK == 0) {
        return 1;
    } else if constexpr (WK == 1) {
        return (int64_t)((const int32_t *)w)[e];
    } else {
        return ((const int64_t *)w)[e];
    }
}

// Last row r with off[r] <= e (rows may be empty): binary search on off[0..n].
__device__ __forceinline__ int64_t row_of(const int64_t *off, int64_t n, int64_t e) {
    int64_t lo = 0, hi = n;  // invariant off[lo] <= e < off[hi]
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (off[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// The row holding entry e, given that e lies past row r (e >= off[r + 1]):
// one step when the next row holds e, a binary search across a run of empty
// rows (coarse levels keep millions of isolated nodes)
__device__ __forceinline__ int64_t next_row(const int64_t *off, int64_t n, int64_t r, int64_t e) {
    ++r;
    return e < off[r + 1] ? r : row_of(off, n, e);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int64_t cdiv_dev(int64_t a, int64_t b) { return (a + b - 1) / b; }

// smallest b with 2^b >= x (x >= 1)
__device__ __forceinline__ int ceil_log2_dev(int64_t x) {
    return x <= 1 ? 0 : 64 - __clzll((unsigned long long)(x - 1));
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// Adds c of every thread of a 256-thread workgroup to *dst with one atomic
// (counters that every wavefront would otherwise hit one by one).  Call from
// every thread of the workgroup.
__device__ __forceinline__ void block_count_add(unsigned long long *dst, unsigned long long c) {
    __shared__ unsigned long long red[4];
    for (int s = 32; s >= 1; s >>= 1) c += __shfl_xor(c, s);
    if (lane_id() == 0) red[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = red[0] + red[1] + red[2] + red[3];
        if (t) atomicAdd(dst, t);
    }
}
constexpr int64_t kCountGrid = 2048;  // workgroups of the grid-stride counting kernels

// Combines the updates of wavefront lanes that target the same key before
// they reach memory (scatters onto a few large communities otherwise
// serialise on one address): up to kGroupRounds times, the remaining lanes
// whose key equals that of the lowest remaining lane form a group whose v sum
// lands in that lane, the group's leader.  Returns whether this lane still
// updates memory: a leader (v now its group's sum) or a lane left over after
// the last round (its own v).  The leader is the group's lowest lane.  live:
// the lane has an update.  Every lane of the wavefront must call.
constexpr int kGroupRounds = 4;
__device__ __forceinline__ bool wave_group_sum(int32_t key, bool live, int64_t &v) {
    unsigned long long rem = __ballot(live);
    bool act = live;
    const int lane = lane_id();
    for (int r = 0; r < kGroupRounds && rem; ++r) {
        const int lead = __ffsll(rem) - 1;
        const int32_t lk = __shfl(key, lead);
        const bool in = ((rem >> lane) & 1ull) && key == lk;
        int64_t x = in ? v : 0;
        for (int s = 32; s >= 1; s >>= 1) x += __shfl_xor(x, s);
        if (in) {
            if (lane == lead) v = x;
            else act = false;
        }
        rem &= ~__ballot(in);
    }
    return act;
}

// ------------------------------------------------------------------ graph of one level
struct GraphView {
    int64_t n = 0, nnz = 0;
    const int64_t *off = nullptr;
    const int32_t *col = nullptr;
    const void *w = nullptr;  // nullptr when wkind == 0
    int wkind = 0;            // 0 unit, 1 int32, 2 int64
    int diag_mult = 1;        // 2: self-loop entries hold w(u,u) (input level); 1: they hold 2 w(u,u)
    // several graphs side by side (batched runs): graph of each node and the
    // first node of each graph; null for a single graph
    const int32_t *gid = nullptr;
    const int64_t *gbase = nullptr;
    // batched runs in which graphs joined later: per graph of the level, the
    // level of the batch at which it joined (null when every graph started
    // together), so that its own level is the batch's minus that
    const int32_t *gshift = nullptr;
};

// A graph joining a running batch (request server): an input CSR as
// plm_create takes it, in host or device memory (mem_kind).
struct JoinGraph {
    int64_t n = 0, nnz = 0;
    const int64_t *off = nullptr;
    const int32_t *col = nullptr;
    const int32_t *w = nullptr;
    int mem_kind = 0;
};
// Callbacks of a batched run that takes graphs in at its level boundaries and
// reports each graph as soon as it finishes (continuous batching).
struct BatchHooks {
    // at a level boundary: graphs to add (may be none)
    std::function<std::vector<JoinGraph>()> join;
    // then, per offered graph in order: 0 (added as the next graph index) or an
    // error status with its message
    std::function<void(const std::vector<int> &codes, const std::vector<std::string> &msgs)> joined;
    // graph g finished: its canonical labels (device, n int32, valid during the
    // call, on the run's stream), Q and level count
    std::function<void(int64_t g, const int32_t *labels, int64_t n, double q, int32_t levels)> done;
};

// first node of u's graph (priorities hash the id local to the graph)
__device__ __forceinline__ int64_t node_base(const GraphView &g, int64_t u) { return g.gid ? g.gbase[g.gid[u]] : 0; }
// level of u's own graph when the batch is at `level` (priorities hash it)
__device__ __forceinline__ int32_t node_level(const GraphView &g, int32_t level, int64_t u) {
    return g.gshift ? level - g.gshift[g.gid[u]] : level;
}

// ------------------------------------------------------------------ error type
struct Error {
    int code;
    std::string msg;
};

// throws Error(PLM_E_DEVICE) on failure
void hip_check(hipError_t e, const char *what);
#define HIPCHK(x) ::plm::hip_check((x), #x)

// ------------------------------------------------------------------ scratch allocator
// Grow-only device scratch handed out as aligned slices; reset per use site.
// Only work on the owner's stream (set_stream) uses it.
class Scratch {
  public:
    ~Scratch();
    void set_stream(hipStream_t s) { stream_ = s; }
    void reserve(size_t bytes);
    void *get(size_t bytes);  // next aligned slice (reserve() first)
    void reset() { used_ = 0; }
    size_t capacity() const { return cap_; }

  private:
    char *base_ = nullptr;
    size_t cap_ = 0, used_ = 0;
    hipStream_t stream_ = nullptr;
};

size_t align_up(size_t x, size_t a = 256);

// ------------------------------------------------------------------ primitives (prims.hip)
// Exclusive scan of n values into out (int64); the total goes to *total_dev.
// Needs scan_scratch_bytes(n) of scratch.
size_t scan_scratch_bytes(int64_t n);
void exclusive_scan_i32(const int32_t *in, int64_t *out, int64_t n, int64_t *total_dev, void *scratch,
                        hipStream_t st);
void exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total_dev, void *scratch,
                        hipStream_t st);

// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of the key.
// Sorted data ends up in *keys / *vals (which may be swapped with the alt
// buffers).  Needs radix_scratch_bytes(n) of scratch.
size_t radix_scratch_bytes(int64_t n);
void radix_sort_u32_i32(uint32_t **keys, int32_t **vals, uint32_t **keys_alt, int32_t **vals_alt, int64_t n,
                        int bits, void *scratch, hipStream_t st);
void radix_sort_u64_i32(uint64_t **keys, int32_t **vals, uint64_t **keys_alt, int32_t **vals_alt, int64_t n,
                        int bits, void *scratch, hipStream_t st);
void radix_sort_u64_i64(uint64_t **keys, int64_t **vals, uint64_t **keys_alt, int64_t **vals_alt, int64_t n,
                        int bits, void *scratch, hipStream_t st);
// Keys alone, on key bits [lo, lo + bits) (the bits below lo are carried, not
// ordered).
void radix_sort_u64_keys(uint64_t **keys, uint64_t **keys_alt, int64_t n, int lo, int bits, void *scratch,
                         hipStream_t st);

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int ceil_log2(uint64_t x) {  // smallest b with 2^b >= x
    int b = 0;
    while (b < 64 && (1ULL << b) < x) ++b;
    return b;
}

}  // namespace plm
