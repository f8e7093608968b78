// ensemble.hip - core groups of an ensemble of base solutions (Equation (3.2)):
// two nodes share a core group iff every base solution puts them in the same
// community.
//
// The groups are refined one base solution at a time.  Node v gets the key
// (group of v so far, label of v in the next solution), the (key, v) pairs are
// radix-sorted (stable, so within a run of equal keys the nodes ascend), and
// every node of a run is given the run's first node: the group's smallest
// member.  Comparing whole keys, not hashes of the label tuples, keeps the
// groups exact.
#include <hip/hip_runtime.h>

#include "level.h"

namespace plm {

constexpr int kET = 256;

__global__ void k_pair_keys(const int32_t *grp, const int32_t *lab, int64_t n, int bits, uint64_t *keys,
                            int32_t *vals) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    uint64_t hi = grp ? (uint64_t)(uint32_t)grp[v] << bits : 0;
    keys[v] = hi | (uint64_t)(uint32_t)lab[v];
    vals[v] = (int32_t)v;
}

// head[i] = 1 where a run of equal keys starts
__global__ void k_run_heads(const uint64_t *keys, int64_t n, int32_t *head) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

// run r = ex[i] + head[i] - 1; first[r] = node at the run's head
__global__ void k_run_first(const int32_t *vals, const int32_t *head, const int64_t *ex, int64_t n, int32_t *first) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && head[i]) first[ex[i]] = vals[i];
}

__global__ void k_run_assign(const int32_t *vals, const int32_t *head, const int64_t *ex, const int32_t *first,
                             int64_t n, int32_t *grp) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) grp[vals[i]] = first[ex[i] + head[i] - 1];
}

size_t ensemble_scratch_bytes(int64_t n) {
    size_t r = radix_scratch_bytes(n), s = scan_scratch_bytes(n);
    return r > s ? r : s;
}

void ensemble_refine(int32_t *grp, const int32_t *lab, int64_t n, bool first_solution, EnsembleWork &wk,
                     hipStream_t st) {
    if (n <= 0) return;
    const int bits = ceil_log2((uint64_t)n) > 0 ? ceil_log2((uint64_t)n) : 1;  // node ids < 2^bits
    const unsigned blocks = (unsigned)cdiv(n, kET);
    uint64_t *keys = wk.keys, *keys_alt = wk.keys_alt;
    int32_t *vals = wk.vals, *vals_alt = wk.vals_alt;
    hipLaunchKernelGGL(k_pair_keys, dim3(blocks), dim3(kET), 0, st, first_solution ? nullptr : grp, lab, n, bits,
                       keys, vals);
    HIPCHK(hipGetLastError());
    radix_sort_u64_i32(&keys, &vals, &keys_alt, &vals_alt, n, first_solution ? bits : 2 * bits, wk.scratch, st);
    // the sort leaves its input in the alt buffers: the head flags and the
    // run index reuse them
    int32_t *head = vals_alt;
    int64_t *ex = (int64_t *)keys_alt;
    hipLaunchKernelGGL(k_run_heads, dim3(blocks), dim3(kET), 0, st, keys, n, head);
    exclusive_scan_i32(head, ex, n, nullptr, wk.scratch, st);
    hipLaunchKernelGGL(k_run_first, dim3(blocks), dim3(kET), 0, st, vals, head, ex, n, wk.first);
    hipLaunchKernelGGL(k_run_assign, dim3(blocks), dim3(kET), 0, st, vals, head, ex, wk.first, n, grp);
    HIPCHK(hipGetLastError());
}

}  // namespace plm
