// batch.hip - kernels of batched runs: many independent graphs side by side in
// one level, each following Algorithm 3 on its own.
//
// The graphs of a level occupy contiguous node ranges.  Priorities hash ids
// local to each graph and gains use each graph's own S, so colour classes,
// decisions, coarse ids and levels are exactly those of separate runs.  A
// graph whose communities stop merging is finished: its input nodes receive
// their labels and it leaves the next level.
#include <hip/hip_runtime.h>

#include "level.h"

namespace plm {

constexpr int kBT = 256;

// out[i] = a[idx[i]]
__global__ void k_gather_i64(const int64_t *a, const int64_t *idx, int64_t count, int64_t *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = a[idx[i]];
}
void launch_gather_i64(const int64_t *a, const int64_t *idx, int64_t count, int64_t *out, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_gather_i64, dim3((unsigned)cdiv(count, kBT)), dim3(kBT), 0, st, a, idx, count, out);
    HIPCHK(hipGetLastError());
}

// flag[zeta[u]] = 1 for the nodes of kept graphs (keep == null: all nodes)
__global__ void k_flag_kept(const int32_t *zeta, int64_t n, const int32_t *gid, const uint8_t *keep, int32_t *flag) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n && (!keep || keep[gid[u]])) flag[zeta[u]] = 1;
}
__global__ void k_map_kept(const int32_t *zeta, const int64_t *newid, int64_t n, const int32_t *gid,
                           const uint8_t *keep, int32_t *pi) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n) pi[u] = (!keep || keep[gid[u]]) ? (int32_t)newid[zeta[u]] : -1;
}

// Community flags of the kept graphs' nodes, their exclusive prefix sum
// (newid[0..n], newid[n] = total) and, if pi is not null, the fine-to-coarse map.
void batch_relabel(const int32_t *zeta, int64_t n, const int32_t *gid, const uint8_t *keep, int32_t *flag,
                   int64_t *newid, int32_t *pi, void *scan_scratch, hipStream_t st) {
    if (n == 0) {
        HIPCHK(hipMemsetAsync(newid, 0, 8, st));
        return;
    }
    HIPCHK(hipMemsetAsync(flag, 0, n * 4, st));
    hipLaunchKernelGGL(k_flag_kept, dim3((unsigned)cdiv(n, kBT)), dim3(kBT), 0, st, zeta, n, gid, keep, flag);
    exclusive_scan_i32(flag, newid, n, newid + n, scan_scratch, st);
    if (pi) hipLaunchKernelGGL(k_map_kept, dim3((unsigned)cdiv(n, kBT)), dim3(kBT), 0, st, zeta, newid, n, gid, keep, pi);
    HIPCHK(hipGetLastError());
}

// gid[u] = last a with base[a] <= u
__global__ void k_fill_gid(const int64_t *base, int64_t A, int64_t n, int32_t *gid) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int64_t lo = 0, hi = A;
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (base[mid] <= u) lo = mid; else hi = mid;
    }
    gid[u] = (int32_t)lo;
}
void launch_fill_gid(const int64_t *base, int64_t A, int64_t n, int32_t *gid, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_gid, dim3((unsigned)cdiv(n, kBT)), dim3(kBT), 0, st, base, A, n, gid);
    HIPCHK(hipGetLastError());
}

// For every input node v of graph g = gid0[v], whose node at this level is
// x = lab[v] (of active graph gid[x], first node base[gid[x]]):
//   status[g] == 1 (finishing at this level): out[v] = zeta[x] - base[gid[x]]
//   status[g] == 0 (continuing):              lab[v] = pi[x]
__global__ void k_batch_step(int64_t n0, const int32_t *gid0, const uint8_t *status, const int32_t *gid,
                             const int64_t *base, const int32_t *zeta, const int32_t *pi, int32_t *lab, int32_t *out) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n0) return;
    uint8_t s = status[gid0[v]];
    if (s > 1) return;
    int32_t x = lab[v];
    if (s == 1) out[v] = (int32_t)((int64_t)zeta[x] - base[gid[x]]);
    else lab[v] = pi[x];
}
void launch_batch_step(int64_t n0, const int32_t *gid0, const uint8_t *status, const int32_t *gid,
                       const int64_t *base, const int32_t *zeta, const int32_t *pi, int32_t *lab, int32_t *out,
                       hipStream_t st) {
    if (n0 <= 0) return;
    hipLaunchKernelGGL(k_batch_step, dim3((unsigned)cdiv(n0, kBT)), dim3(kBT), 0, st, n0, gid0, status, gid, base,
                       zeta, pi, lab, out);
    HIPCHK(hipGetLastError());
}

// Per graph a: S[a] = sum of vol over its node range and the 64-bit limit
// wl[a] = (2^62 - 1) / (S[a] gmax) of the gain arithmetic (gmax = max of the
// resolution's numerator and denominator; no limit when S[a] = 0).
__global__ __launch_bounds__(kBT) void k_graph_S(const int64_t *vol, const int64_t *base, int64_t gmax, int64_t *S,
                                                 int64_t *wl) {
    __shared__ int64_t part[kBT / 64];
    int64_t a = blockIdx.x;
    int64_t lo = base[a], hi = base[a + 1];
    int64_t s = 0;
    for (int64_t u = lo + threadIdx.x; u < hi; u += kBT) s += vol[u];
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if (lane_id() == 0) part[threadIdx.x / 64] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int i = 0; i < kBT / 64; ++i) t += part[i];
        S[a] = t;
        unsigned __int128 sg = (unsigned __int128)(uint64_t)t * (unsigned __int128)(uint64_t)gmax;
        wl[a] = sg == 0 ? INT64_MAX : ((sg >> 62) ? 0 : (int64_t)(((1ULL << 62) - 1) / (uint64_t)sg));
    }
}
void launch_graph_S(const int64_t *vol, const int64_t *base, int64_t A, int64_t gmax, int64_t *S, int64_t *wl,
                    hipStream_t st) {
    if (A <= 0) return;
    hipLaunchKernelGGL(k_graph_S, dim3((unsigned)A), dim3(kBT), 0, st, vol, base, gmax, S, wl);
    HIPCHK(hipGetLastError());
}

// key[v] = first input node of v's graph + local label
__global__ void k_batch_keys(int64_t n0, const int32_t *gid0, const int64_t *gbase0, const int32_t *local,
                             int32_t *key) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n0) key[v] = (int32_t)(gbase0[gid0[v]] + local[v]);
}
// canonical label within the graph = global rank - rank of the graph's first node
__global__ void k_batch_canon(int64_t n0, const int32_t *gid0, const int64_t *gbase0, const int32_t *rank,
                              int32_t *out) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n0) out[v] = rank[v] - rank[gbase0[gid0[v]]];
}
void batch_canonical(int64_t n0, const int32_t *gid0, const int64_t *gbase0, const int32_t *local, int32_t *keys,
                     int32_t *rank, int32_t *out, Scratch &scr, hipStream_t st) {
    if (n0 <= 0) return;
    hipLaunchKernelGGL(k_batch_keys, dim3((unsigned)cdiv(n0, kBT)), dim3(kBT), 0, st, n0, gid0, gbase0, local, keys);
    build_canonical(keys, n0, rank, scr, st);
    hipLaunchKernelGGL(k_batch_canon, dim3((unsigned)cdiv(n0, kBT)), dim3(kBT), 0, st, n0, gid0, gbase0, rank, out);
    HIPCHK(hipGetLastError());
}

// Per-graph modularity parts on the input level: I2[g] and sum of vol(C)^2 of
// graph g (two words, carry handled), with labels given as global keys.
// A thread sums its kC entries per graph (rows of a graph are contiguous, so
// they rarely span two); a wavefront whose lanes all end in one graph adds its
// total with a single atomic, since a graph's counter would otherwise take an
// atomic per row of a graph with millions of entries.
template <int WK>
__global__ __launch_bounds__(kBT) void k_batch_intra(GraphView g, const int32_t *gid0, const int32_t *key,
                                                      unsigned long long *I2) {
    constexpr int kC = 16;
    const int64_t e0 = ((int64_t)blockIdx.x * kBT + threadIdx.x) * kC;
    int32_t gcur = -1;
    int64_t s = 0;
    if (e0 < g.nnz) {
        const int64_t e1 = e0 + kC < g.nnz ? e0 + kC : g.nnz;
        int64_t r = row_of(g.off, g.n, e0);
        int64_t rend = g.off[r + 1];
        int32_t kr = key[r];
        gcur = gid0[r];
        for (int64_t e = e0; e < e1; ++e) {
            while (e >= rend) {
                r = next_row(g.off, g.n, r, e);
                rend = g.off[r + 1];
                kr = key[r];
                const int32_t gr = gid0[r];
                if (gr != gcur) {
                    if (s) atomicAdd(&I2[gcur], (unsigned long long)s);
                    s = 0;
                    gcur = gr;
                }
            }
            int32_t v = g.col[e];
            if (key[v] == kr) {
                int64_t x = wload<WK>(g.w, e);
                if (v == r) x *= g.diag_mult;
                s += x;
            }
        }
    }
    const int32_t g0 = __shfl(gcur, 0);
    if (__all(gcur == g0)) {
        for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
        if (lane_id() == 0 && s) atomicAdd(&I2[g0], (unsigned long long)s);
    } else if (s) {
        atomicAdd(&I2[gcur], (unsigned long long)s);
    }
}
__global__ void k_batch_vol(int64_t n0, const int32_t *key, const int64_t *vol0, int64_t *volL) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t x = v < n0 ? vol0[v] : 0;
    int32_t l = x ? key[v] : 0;
    if (wave_group_sum(l, x != 0, x)) atomicAdd((unsigned long long *)&volL[l], (unsigned long long)x);
}
__global__ void k_batch_sq(int64_t n0, const int32_t *gid0, const int64_t *volL, unsigned long long *sq) {
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n0 || volL[x] == 0) return;
    unsigned __int128 q = (unsigned __int128)(uint64_t)volL[x] * (unsigned __int128)(uint64_t)volL[x];
    uint64_t lo = (uint64_t)q, hi = (uint64_t)(q >> 64);
    int32_t g = gid0[x];
    unsigned long long old = atomicAdd(&sq[2 * g], (unsigned long long)lo);
    uint64_t carry = (old + lo < old) ? 1 : 0;
    if (hi + carry) atomicAdd(&sq[2 * g + 1], (unsigned long long)(hi + carry));
}

void batch_modularity_parts(const GraphView &g0, const int32_t *gid0, const int32_t *key, const int64_t *vol0,
                            int64_t G, int64_t *volL, unsigned long long *I2, unsigned long long *sq,
                            hipStream_t st) {
    int64_t n0 = g0.n;
    HIPCHK(hipMemsetAsync(I2, 0, (size_t)(G > 0 ? G : 1) * 8, st));
    HIPCHK(hipMemsetAsync(sq, 0, (size_t)(G > 0 ? G : 1) * 16, st));
    if (n0 <= 0) return;
    HIPCHK(hipMemsetAsync(volL, 0, n0 * 8, st));
    if (g0.nnz > 0) {
        dim3 eg((unsigned)cdiv(cdiv(g0.nnz, 16), kBT));
        switch (g0.wkind) {
            case 0: hipLaunchKernelGGL(k_batch_intra<0>, eg, dim3(kBT), 0, st, g0, gid0, key, I2); break;
            case 1: hipLaunchKernelGGL(k_batch_intra<1>, eg, dim3(kBT), 0, st, g0, gid0, key, I2); break;
            default: hipLaunchKernelGGL(k_batch_intra<2>, eg, dim3(kBT), 0, st, g0, gid0, key, I2); break;
        }
    }
    hipLaunchKernelGGL(k_batch_vol, dim3((unsigned)cdiv(n0, kBT)), dim3(kBT), 0, st, n0, key, vol0, volL);
    hipLaunchKernelGGL(k_batch_sq, dim3((unsigned)cdiv(n0, kBT)), dim3(kBT), 0, st, n0, gid0, volL, sq);
    HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------------ one graph of a union
// Modularity parts of graph g of the input union (nodes [a, a + n), entries
// [ea, eb), columns global ids) for local labels lab[0..n): I2 and the
// 128-bit sum of the label volumes squared (volL: n words of scratch).
template <int WK>
__global__ __launch_bounds__(kBT) void k_range_intra(const int64_t *off, const int32_t *col, const void *w,
                                                     int diag_mult, int64_t a, int64_t n, int64_t ea, int64_t eb,
                                                     const int32_t *lab, unsigned long long *I2) {
    // kC consecutive entries per thread: one row search, then row by row
    constexpr int kC = 16;
    const int64_t e0 = ea + ((int64_t)blockIdx.x * kBT + threadIdx.x) * kC;
    int64_t s = 0;
    if (e0 < eb) {
        const int64_t *loff = off + a;  // local rows: loff[r] <= e < loff[r + 1]
        const int64_t e1 = e0 + kC < eb ? e0 + kC : eb;
        int64_t r = row_of(loff, n, e0);
        int64_t rend = loff[r + 1];
        int32_t lr = lab[r];
        for (int64_t e = e0; e < e1; ++e) {
            while (e >= rend) {
                r = next_row(loff, n, r, e);
                rend = loff[r + 1];
                lr = lab[r];
            }
            const int64_t v = (int64_t)col[e] - a;
            if (lab[v] == lr) {
                int64_t x = wload<WK>(w, e);
                if (v == r) x *= diag_mult;
                s += x;
            }
        }
    }
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
    if (lane_id() == 0 && s) atomicAdd(I2, (unsigned long long)s);
}
__global__ void k_range_vol(int64_t n, const int32_t *lab, const int64_t *vol, int64_t *volL) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t x = v < n ? vol[v] : 0;
    int32_t l = x ? lab[v] : 0;
    if (wave_group_sum(l, x != 0, x)) atomicAdd((unsigned long long *)&volL[l], (unsigned long long)x);
}
__global__ __launch_bounds__(kBT) void k_range_sq(const int64_t *volL, int64_t n, unsigned long long *acc2) {
    unsigned __int128 s = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBT) {
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
__global__ void k_zero_words(unsigned long long *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

void graph_modularity_parts(const GraphView &g0, int64_t a, int64_t n, const int32_t *lab, const int64_t *vol0,
                            int64_t *volL, unsigned long long *acc3, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, acc3, (int64_t)3);
    if (n <= 0) return;
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)cdiv(n, kBT)), dim3(kBT), 0, st, (unsigned long long *)volL, n);
    int64_t ea = 0, eb = 0;
    HIPCHK(hipMemcpyAsync(&ea, g0.off + a, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&eb, g0.off + a + n, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (eb > ea) {
        dim3 eg((unsigned)cdiv(cdiv(eb - ea, 16), kBT));
        switch (g0.wkind) {
            case 0: hipLaunchKernelGGL(k_range_intra<0>, eg, dim3(kBT), 0, st, g0.off, g0.col, g0.w, g0.diag_mult, a, n, ea, eb, lab, acc3); break;
            case 1: hipLaunchKernelGGL(k_range_intra<1>, eg, dim3(kBT), 0, st, g0.off, g0.col, g0.w, g0.diag_mult, a, n, ea, eb, lab, acc3); break;
            default: hipLaunchKernelGGL(k_range_intra<2>, eg, dim3(kBT), 0, st, g0.off, g0.col, g0.w, g0.diag_mult, a, n, ea, eb, lab, acc3); break;
        }
    }
    hipLaunchKernelGGL(k_range_vol, dim3((unsigned)cdiv(n, kBT)), dim3(kBT), 0, st, n, lab, vol0 + a, volL);
    const int64_t nb = cdiv(n, kBT);
    hipLaunchKernelGGL(k_range_sq, dim3((unsigned)(nb < 1024 ? nb : 1024)), dim3(kBT), 0, st, volL, n, acc3 + 1);
    HIPCHK(hipGetLastError());
}

// ------------------------------------------------------------------ joins
// Appending a graph (input CSR with local ids) to a union: offsets shifted by
// the union's entries before it, columns by its nodes before it.
__global__ void k_append_off(int64_t *dst, const int64_t *off, int64_t n, int64_t ebase) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) dst[i] = ebase + off[i];
}
// input level: columns shifted, weights copied (unit weights written out when
// the graph has none and the union has a weight array)
__global__ void k_append_input(int32_t *col, int32_t *w, const int32_t *jcol, const int32_t *jw, int64_t nnz,
                               int32_t nbase) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    col[e] = jcol[e] + nbase;
    if (w) w[e] = jw ? jw[e] : 1;
}
// coarse-level format: int64 weights with the self-loop doubled
__global__ void k_append_coarse(int32_t *col, int64_t *w, const int64_t *joff, int64_t n, const int32_t *jcol,
                                const int32_t *jw, int64_t nnz, int32_t nbase) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const int64_t r = row_of(joff, n, e);
    const int32_t v = jcol[e];
    col[e] = v + nbase;
    w[e] = (int64_t)(jw ? jw[e] : 1) * (v == r ? 2 : 1);
}
__global__ void k_iota_from(int32_t *a, int64_t n, int64_t first) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = (int32_t)(first + i);
}
__global__ void k_fill_i32v(int32_t *a, int64_t n, int32_t x) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = x;
}

void launch_append_off(int64_t *dst, const int64_t *off, int64_t n, int64_t ebase, hipStream_t st) {
    hipLaunchKernelGGL(k_append_off, dim3((unsigned)cdiv(n + 1, kBT)), dim3(kBT), 0, st, dst, off, n, ebase);
    HIPCHK(hipGetLastError());
}
void launch_append_input(int32_t *col, int32_t *w, const int32_t *jcol, const int32_t *jw, int64_t nnz, int64_t nbase,
                         hipStream_t st) {
    if (nnz <= 0) return;
    hipLaunchKernelGGL(k_append_input, dim3((unsigned)cdiv(nnz, kBT)), dim3(kBT), 0, st, col, w, jcol, jw, nnz,
                       (int32_t)nbase);
    HIPCHK(hipGetLastError());
}
void launch_append_coarse(int32_t *col, int64_t *w, const int64_t *joff, int64_t n, const int32_t *jcol,
                          const int32_t *jw, int64_t nnz, int64_t nbase, hipStream_t st) {
    if (nnz <= 0) return;
    hipLaunchKernelGGL(k_append_coarse, dim3((unsigned)cdiv(nnz, kBT)), dim3(kBT), 0, st, col, w, joff, n, jcol, jw,
                       nnz, (int32_t)nbase);
    HIPCHK(hipGetLastError());
}
void launch_iota_from(int32_t *a, int64_t n, int64_t first, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_iota_from, dim3((unsigned)cdiv(n, kBT)), dim3(kBT), 0, st, a, n, first);
    HIPCHK(hipGetLastError());
}
void launch_fill_i32(int32_t *a, int64_t n, int32_t x, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i32v, dim3((unsigned)cdiv(n, kBT)), dim3(kBT), 0, st, a, n, x);
    HIPCHK(hipGetLastError());
}

// batched validation: every column lies in its row's graph
__global__ void k_batch_validate(const int64_t *off, const int32_t *col, int64_t n, const int32_t *gid0,
                                 const int64_t *gbase0, uint32_t *bad) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int32_t g = gid0[u];
    int64_t lo = gbase0[g], hi = gbase0[g + 1];
    for (int64_t e = off[u]; e < off[u + 1]; ++e)
        if (col[e] < lo || col[e] >= hi) {
            atomicOr(bad, 32u);
            return;
        }
}
uint32_t batch_validate(const GraphView &g, const int32_t *gid0, const int64_t *gbase0, Scratch &scr,
                        int64_t *host_i64, hipStream_t st) {
    scr.reserve(256);
    uint32_t *bad = (uint32_t *)scr.get(8);
    HIPCHK(hipMemsetAsync(bad, 0, 8, st));
    if (g.n > 0)
        hipLaunchKernelGGL(k_batch_validate, dim3((unsigned)cdiv(g.n, kBT)), dim3(kBT), 0, st, g.off, g.col, g.n,
                           gid0, gbase0, bad);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(host_i64, bad, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return (uint32_t)(host_i64[0] & 0xffffffff);
}

}  // namespace plm
