// graphgen_gpu.hip - the R-MAT generator of graphgen.c, run on the GPU.
//
// Inputs only, no part of the community-detection method.  It reproduces
// gg_rmat() bit for bit (same counter-based draws, same relabelling bijection,
// same pair-hash weights) so that graphs too large to build quickly on the
// host can be made directly in device memory.  Sorting uses rocPRIM; the
// generator is not part of the library under test.
#include <cstring>
#include <hip/hip_runtime.h>
#include <rocprim/rocprim.hpp>
#include <stdint.h>
#include <stdio.h>

#define GG_GOLDEN 0x9E3779B97F4A7C15ULL

__host__ __device__ static inline uint64_t gg_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
__host__ __device__ static inline uint64_t gg_stream_key(uint64_t seed, uint64_t stream) {
    return gg_mix(seed + (stream + 1) * GG_GOLDEN);
}
__host__ __device__ static inline uint64_t gg_draw(uint64_t key, uint64_t counter) {
    return gg_mix(key + (counter + 1) * GG_GOLDEN);
}
__host__ __device__ static inline double gg_unit(uint64_t d) { return (double)(d >> 11) * 0x1.0p-53; }

struct PermKey { uint64_t mul[3], add[3]; };

__device__ static inline uint64_t perm(uint64_t x, uint64_t mask, int sh, int s, const PermKey &k) {
    for (int r = 0; r < 3; ++r) {
        x = (x * k.mul[r]) & mask;
        if (s > 1) x ^= x >> sh;
        x = (x + k.add[r]) & mask;
    }
    return x;
}

__global__ void k_rmat_keys(uint64_t *keys, int64_t E, int s, uint64_t key, double a, double ab, double abc,
                            PermKey pk) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    uint64_t r = 0, c = 0;
    for (int d = 0; d < s; ++d) {
        double u = gg_unit(gg_draw(key, (uint64_t)e * (uint64_t)s + (uint64_t)d));
        uint64_t rb = (u >= ab), cb = (u >= a && u < ab) || (u >= abc);
        r = (r << 1) | rb;
        c = (c << 1) | cb;
    }
    uint64_t mask = (1ULL << s) - 1;
    int sh = (s + 1) / 2;
    uint64_t pu = perm(r, mask, sh, s, pk), pv = perm(c, mask, sh, s, pk);
    if (pu == pv) { keys[e] = ~0ULL; return; }
    uint64_t lo = pu < pv ? pu : pv, hi = pu < pv ? pv : pu;
    keys[e] = (lo << s) | hi;
}

// flag[i] = 1 if keys[i] is the first copy of a valid (non-sentinel) pair
__global__ void k_unique_flags(const uint64_t *keys, int64_t E, uint64_t lim, uint64_t *flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= E) return;
    uint64_t k = keys[i];
    flags[i] = (k < lim && (i == 0 || keys[i - 1] != k)) ? 1 : 0;
}

// scatter each unique pair as both directed entries (row << s) | col
__global__ void k_expand(const uint64_t *keys, const uint64_t *flags, const uint64_t *pos, int64_t E, int s,
                         uint64_t *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= E || !flags[i]) return;
    uint64_t k = keys[i], mask = (1ULL << s) - 1;
    uint64_t lo = k >> s, hi = k & mask;
    int64_t p = (int64_t)pos[i];
    out[2 * p] = (lo << s) | hi;
    out[2 * p + 1] = (hi << s) | lo;
}

__global__ void k_to_csr(const uint64_t *dkeys, int64_t nnz, int s, int64_t n, int64_t *off, int32_t *col,
                         int32_t *w, uint64_t wkey) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nnz) return;
    uint64_t k = dkeys[i], mask = (1ULL << s) - 1;
    int64_t row = (int64_t)(k >> s), c = (int64_t)(k & mask);
    col[i] = (int32_t)c;
    if (w) {
        uint64_t lo = row < c ? row : c, hi = row < c ? c : row;
        w[i] = (int32_t)(1 + gg_draw(wkey, (lo << 32) | hi) % 100);
    }
    int64_t prev = (i == 0) ? -1 : (int64_t)(dkeys[i - 1] >> s);
    for (int64_t r = prev + 1; r <= row; ++r) off[r] = i;
    if (i == nnz - 1)
        for (int64_t r = row + 1; r <= n; ++r) off[r] = nnz;
}

__global__ void k_fill_off(int64_t *off, int64_t n) {  // empty graph
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) off[i] = 0;
}

static int64_t nblk(int64_t n, int b) { return (n + b - 1) / b; }

#define GCHK(x)                                                                          \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) {                                                          \
            fprintf(stderr, "graphgen_gpu: %s failed: %s\n", #x, hipGetErrorString(e_)); \
            return -1;                                                                   \
        }                                                                                \
    } while (0)

extern "C" {

// Build R-MAT(s, ef, a, b, c, seed) in device memory.  On success *off_out,
// *col_out and (if weighted) *w_out are hipMalloc'ed device arrays owned by the
// caller (release with ggpu_free); returns nnz, or -1 on error.
int64_t ggpu_rmat(int s, int64_t ef, double a, double b, double c, uint64_t seed, int weighted,
                  int64_t **off_out, int32_t **col_out, int32_t **w_out) {
    *off_out = nullptr; *col_out = nullptr; *w_out = nullptr;
    if (s < 1 || s > 30 || ef < 0) return -1;
    int64_t n = 1LL << s, E = ef * n;
    hipStream_t st = 0;
    uint64_t *ka = nullptr, *kb = nullptr, *flags = nullptr, *pos = nullptr;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    PermKey pk;
    uint64_t key3 = gg_stream_key(seed, 3);
    for (int r = 0; r < 3; ++r) { pk.mul[r] = gg_draw(key3, 2 * r) | 1ULL; pk.add[r] = gg_draw(key3, 2 * r + 1); }
    int64_t Eb = E > 0 ? E : 1;
    GCHK(hipMalloc(&ka, Eb * sizeof(uint64_t)));
    GCHK(hipMalloc(&kb, Eb * sizeof(uint64_t)));
    if (E > 0)
        hipLaunchKernelGGL(k_rmat_keys, dim3(nblk(E, 256)), dim3(256), 0, st, ka, E, s, gg_stream_key(seed, 1), a,
                           a + b, a + b + c, pk);
    rocprim::double_buffer<uint64_t> db(ka, kb);
    GCHK(rocprim::radix_sort_keys(nullptr, tmp_bytes, db, (size_t)E, 0, 2 * s + 1, st));
    GCHK(hipMalloc(&tmp, tmp_bytes > 0 ? tmp_bytes : 1));
    GCHK(rocprim::radix_sort_keys(tmp, tmp_bytes, db, (size_t)E, 0, 2 * s + 1, st));
    uint64_t *sorted = db.current(), *other = db.alternate();
    // unique
    GCHK(hipMalloc(&flags, Eb * sizeof(uint64_t)));
    GCHK(hipMalloc(&pos, Eb * sizeof(uint64_t)));
    if (E > 0)
        hipLaunchKernelGGL(k_unique_flags, dim3(nblk(E, 256)), dim3(256), 0, st, sorted, E, 1ULL << (2 * s), flags);
    size_t tb2 = 0;
    GCHK(rocprim::exclusive_scan(nullptr, tb2, flags, pos, (uint64_t)0, (size_t)E, rocprim::plus<uint64_t>(), st));
    if (tb2 > tmp_bytes) { GCHK(hipFree(tmp)); tmp_bytes = tb2; GCHK(hipMalloc(&tmp, tmp_bytes)); }
    GCHK(rocprim::exclusive_scan(tmp, tb2, flags, pos, (uint64_t)0, (size_t)E, rocprim::plus<uint64_t>(), st));
    uint64_t m = 0, lastf = 0;
    if (E > 0) {
        GCHK(hipMemcpyAsync(&m, pos + (E - 1), sizeof(uint64_t), hipMemcpyDeviceToHost, st));
        GCHK(hipMemcpyAsync(&lastf, flags + (E - 1), sizeof(uint64_t), hipMemcpyDeviceToHost, st));
        GCHK(hipStreamSynchronize(st));
        m += lastf;
    }
    int64_t nnz = 2 * (int64_t)m;
    // directed entries, sorted by (row, col); reuse `other` (E >= 2m? not always) -> new buffers
    uint64_t *da = nullptr, *dbuf = nullptr;
    int64_t nb = nnz > 0 ? nnz : 1;
    GCHK(hipMalloc(&da, nb * sizeof(uint64_t)));
    if (E > 0)
        hipLaunchKernelGGL(k_expand, dim3(nblk(E, 256)), dim3(256), 0, st, sorted, flags, pos, E, s, da);
    GCHK(hipStreamSynchronize(st));
    GCHK(hipFree(flags)); GCHK(hipFree(pos)); GCHK(hipFree(ka)); GCHK(hipFree(kb));
    flags = pos = ka = kb = nullptr;
    (void)other;
    GCHK(hipMalloc(&dbuf, nb * sizeof(uint64_t)));
    rocprim::double_buffer<uint64_t> d2(da, dbuf);
    size_t tb3 = 0;
    GCHK(rocprim::radix_sort_keys(nullptr, tb3, d2, (size_t)nnz, 0, 2 * s, st));
    if (tb3 > tmp_bytes) { GCHK(hipFree(tmp)); tmp_bytes = tb3; GCHK(hipMalloc(&tmp, tmp_bytes)); }
    GCHK(rocprim::radix_sort_keys(tmp, tb3, d2, (size_t)nnz, 0, 2 * s, st));
    int64_t *off = nullptr; int32_t *col = nullptr, *w = nullptr;
    GCHK(hipMalloc(&off, (n + 1) * sizeof(int64_t)));
    GCHK(hipMalloc(&col, nb * sizeof(int32_t)));
    if (weighted) GCHK(hipMalloc(&w, nb * sizeof(int32_t)));
    if (nnz > 0)
        hipLaunchKernelGGL(k_to_csr, dim3(nblk(nnz, 256)), dim3(256), 0, st, d2.current(), nnz, s, n, off, col, w,
                           gg_stream_key(seed, 2));
    else
        hipLaunchKernelGGL(k_fill_off, dim3(nblk(n + 1, 256)), dim3(256), 0, st, off, n);
    GCHK(hipStreamSynchronize(st));
    GCHK(hipGetLastError());
    GCHK(hipFree(da)); GCHK(hipFree(dbuf)); GCHK(hipFree(tmp));
    *off_out = off; *col_out = col; *w_out = w;
    return nnz;
}

void ggpu_free(void *p) {
    if (p) (void)hipFree(p);
}

int ggpu_copy_to_host(void *dst, const void *src, int64_t bytes) {
    return hipMemcpy(dst, src, (size_t)bytes, hipMemcpyDeviceToHost) == hipSuccess ? 0 : -1;
}

}  // extern "C"
