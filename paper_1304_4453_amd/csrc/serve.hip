// serve.hip - request server over the batched engine (plm_server_* in
// include/plm.h).
//
// Requests (one graph each) wait in a first-in first-out queue.  A step admits
// queued requests in order while their resident footprint fits the HBM budget
// (and their entries fit the per-batch cap), lays their CSRs side by side in
// device memory as one disjoint union, runs Algorithm 3 on all of them at once
// (run_batch in api.hip: every graph gets exactly the result of its own run),
// and completes them.  Labels stay in device memory until the client fetches
// them.
#include <hip/hip_runtime.h>

#include <cstring>
#include <deque>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/plm.h"
#include "plm_internal.h"

plm_status plm_internal_batch_adopt(plm_ctx **out, int64_t G, const int64_t *node_base, int64_t nnz, int64_t *off,
                                    int32_t *col, int32_t *w, void *hip_stream, const plm_options *opt);

namespace {

using plm::cdiv;
using plm::Error;

// Resident bytes of one graph while it runs: the CSR, per-node state of the
// level engine and the batch bookkeeping, and the sort buffers of contraction.
int64_t footprint(int64_t n, int64_t nnz, bool weighted) {
    return 8 * (n + 1) + (weighted ? 8 : 4) * nnz + 128 * n + 64 * nnz;
}

// union fix-up of one request: rows shift by the entries before it, columns
// by the nodes before it; unit weights are written out when the union carries
// weights but this request does not
__global__ void k_union_fix(int64_t *off, int64_t n, int64_t ebase, int32_t *col, int64_t nnz, int32_t nbase,
                            int32_t *w, int fill_unit) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) off[i] += ebase;
    if (i < nnz) {
        col[i] += nbase;
        if (fill_unit) w[i] = 1;
    }
}
__global__ void k_set_i64(int64_t *p, int64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

}  // namespace

struct plm_server {
    struct Req {
        int64_t n = 0, nnz = 0;
        const int64_t *off = nullptr;
        const int32_t *col = nullptr;
        const int32_t *w = nullptr;
        int mem_kind = PLM_MEM_HOST;
        int state = 0;  // 0 queued, 1 done, 2 failed
        bool solo = false;  // runs in a batch of its own (its batch was refused as a whole)
        int32_t *labels = nullptr;  // device, when done
        double q = 0.0;
        int32_t levels = 0;
        int64_t bytes = 0;
        plm_status err = PLM_OK;
        std::string msg;
    };
    hipStream_t st = nullptr;
    plm_options opt;
    int64_t budget = 0, max_entries = 0;
    std::string err;
    std::deque<int64_t> queue;
    std::unordered_map<int64_t, Req> reqs;
    int64_t next_id = 0, completed = 0, batches = 0, resident = 0;

    ~plm_server() {
        for (auto &kv : reqs)
            if (kv.second.labels) (void)hipFree(kv.second.labels);
    }

    // one batch: admission, union, run, completion; returns requests completed
    int32_t step() {
        std::vector<int64_t> take;
        int64_t bytes = 0, entries = 0;
        while (!queue.empty()) {
            const Req &r = reqs[queue.front()];
            if (!take.empty() && (r.solo || bytes + r.bytes > budget || entries + r.nnz > max_entries)) break;
            bytes += r.bytes;
            entries += r.nnz;
            take.push_back(queue.front());
            queue.pop_front();
            if (r.solo) break;
        }
        if (take.empty()) return 0;
        const int64_t G = (int64_t)take.size();
        std::vector<int64_t> nbase(G + 1, 0), ebase(G + 1, 0);
        bool weighted = false;
        for (int64_t g = 0; g < G; ++g) {
            const Req &r = reqs[take[g]];
            nbase[g + 1] = nbase[g] + r.n;
            ebase[g + 1] = ebase[g] + r.nnz;
            weighted = weighted || r.w != nullptr;
        }
        const int64_t N = nbase[G], E = ebase[G];
        auto fail_all = [&](plm_status code, const std::string &m) {
            for (int64_t id : take) {
                Req &r = reqs[id];
                r.state = 2;
                r.err = code;
                r.msg = m;
            }
        };
        if (N >= (1LL << 31)) {
            fail_all(PLM_E_BUDGET, "admitted requests exceed 2^31 nodes");
            return 0;
        }
        int64_t *off = nullptr;
        int32_t *col = nullptr, *w = nullptr;
        bool ok = hipMalloc(&off, (size_t)(N + 1) * 8) == hipSuccess &&
                  hipMalloc(&col, (size_t)(E > 0 ? E : 1) * 4) == hipSuccess &&
                  (!weighted || hipMalloc(&w, (size_t)(E > 0 ? E : 1) * 4) == hipSuccess);
        if (!ok) {
            (void)hipGetLastError();
            if (off) (void)hipFree(off);
            if (col) (void)hipFree(col);
            if (w) (void)hipFree(w);
            fail_all(PLM_E_NOMEM, "device allocation of the batch failed");
            return 0;
        }
        resident = bytes;
        try {
            for (int64_t g = 0; g < G; ++g) {
                const Req &r = reqs[take[g]];
                hipMemcpyKind kind = r.mem_kind == PLM_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
                if (r.n > 0) HIPCHK(hipMemcpyAsync(off + nbase[g], r.off, (size_t)r.n * 8, kind, st));
                if (r.nnz > 0) HIPCHK(hipMemcpyAsync(col + ebase[g], r.col, (size_t)r.nnz * 4, kind, st));
                if (r.nnz > 0 && r.w) HIPCHK(hipMemcpyAsync(w + ebase[g], r.w, (size_t)r.nnz * 4, kind, st));
                int64_t m = r.n > r.nnz ? r.n : r.nnz;
                if (m > 0)
                    hipLaunchKernelGGL(k_union_fix, dim3((unsigned)cdiv(m, 256)), dim3(256), 0, st, off + nbase[g],
                                       r.n, ebase[g], col + ebase[g], r.nnz, (int32_t)nbase[g],
                                       weighted ? w + ebase[g] : nullptr, (weighted && !r.w) ? 1 : 0);
            }
            hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, st, off + N, E);
            HIPCHK(hipGetLastError());
            HIPCHK(hipStreamSynchronize(st));
        } catch (const Error &e) {
            (void)hipFree(off);
            (void)hipFree(col);
            if (w) (void)hipFree(w);
            fail_all(e.code, e.msg);
            resident = 0;
            return 0;
        }
        plm_ctx *ctx = nullptr;
        plm_status rc = plm_internal_batch_adopt(&ctx, G, nbase.data(), E, off, col, w, st, &opt);
        if (rc == PLM_E_GRAPH && G > 1) {
            // an invalid graph refuses the whole union: rerun these requests one
            // per batch, in their order, so that only the invalid ones fail
            for (int64_t g = G - 1; g >= 0; --g) {
                reqs[take[g]].solo = true;
                queue.push_front(take[g]);
            }
            resident = 0;
            return 0;
        }
        if (rc != PLM_OK) {
            fail_all(rc, plm_last_error(nullptr));
            resident = 0;
            return 0;
        }
        int32_t *canon = nullptr;
        if (hipMalloc(&canon, (size_t)(N > 0 ? N : 1) * 4) != hipSuccess) {
            (void)hipGetLastError();
            plm_destroy(ctx);
            fail_all(PLM_E_NOMEM, "device allocation of the labels failed");
            resident = 0;
            return 0;
        }
        std::vector<double> q(G);
        std::vector<int32_t> lv(G);
        rc = plm_batch_run(ctx, canon, q.data(), lv.data());
        if (rc != PLM_OK) {
            std::string m = plm_last_error(ctx);
            plm_destroy(ctx);
            (void)hipFree(canon);
            fail_all(rc, m);
            resident = 0;
            return 0;
        }
        plm_destroy(ctx);
        for (int64_t g = 0; g < G; ++g) {
            Req &r = reqs[take[g]];
            r.q = q[g];
            r.levels = lv[g];
            if (hipMalloc(&r.labels, (size_t)(r.n > 0 ? r.n : 1) * 4) != hipSuccess ||
                (r.n > 0 && hipMemcpyAsync(r.labels, canon + nbase[g], (size_t)r.n * 4, hipMemcpyDeviceToDevice, st) !=
                                hipSuccess)) {
                (void)hipGetLastError();
                if (r.labels) (void)hipFree(r.labels);
                r.labels = nullptr;
                r.state = 2;
                r.err = PLM_E_NOMEM;
                r.msg = "device allocation or copy of the result failed";
            }
        }
        (void)hipStreamSynchronize(st);
        (void)hipFree(canon);
        int32_t done = 0;
        for (int64_t id : take) {
            Req &r = reqs[id];
            if (r.state == 0) {
                r.state = 1;
                ++done;
            }
            r.off = nullptr;
            r.col = nullptr;
            r.w = nullptr;
        }
        completed += done;
        ++batches;
        resident = 0;
        return done;
    }
};

namespace {

template <typename F>
plm_status server_guard(plm_server *s, F f) {
    if (!s) return PLM_E_ARG;
    try {
        s->err.clear();
        f();
        return PLM_OK;
    } catch (const Error &e) {
        s->err = e.msg;
        return e.code;
    } catch (const std::exception &e) {
        s->err = e.what();
        return PLM_E_NOMEM;
    }
}

}  // namespace

extern "C" {

plm_status plm_server_create(plm_server **out, int64_t hbm_budget_bytes, int64_t max_batch_entries, void *hip_stream,
                             const plm_options *opt) {
    if (!out) return PLM_E_ARG;
    *out = nullptr;
    if (hbm_budget_bytes <= 0 || max_batch_entries <= 0) return PLM_E_ARG;
    plm_options o;
    plm_default_options(&o);
    if (opt) o = *opt;
    if (o.schedule != PLM_SCHEDULE_COLOUR || o.int_mode == PLM_INT_64 || o.refine) return PLM_E_ARG;
    plm_server *s = new (std::nothrow) plm_server();
    if (!s) return PLM_E_NOMEM;
    s->st = (hipStream_t)hip_stream;
    s->opt = o;
    s->budget = hbm_budget_bytes;
    s->max_entries = max_batch_entries;
    *out = s;
    return PLM_OK;
}

plm_status plm_server_submit(plm_server *s, int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *cols,
                             const int32_t *weights, int32_t mem_kind, int64_t *request_id) {
    return server_guard(s, [&] {
        if (n < 0 || n >= (1LL << 31) || nnz < 0 || !offsets || (nnz > 0 && !cols) || !request_id)
            throw Error{PLM_E_ARG, "bad request arguments"};
        if (mem_kind != PLM_MEM_HOST && mem_kind != PLM_MEM_DEVICE) throw Error{PLM_E_ARG, "bad mem_kind"};
        int64_t ends[2] = {0, 0};
        if (mem_kind == PLM_MEM_HOST) {
            ends[0] = offsets[0];
            ends[1] = offsets[n];
        } else {
            HIPCHK(hipMemcpy(&ends[0], offsets, 8, hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(&ends[1], offsets + n, 8, hipMemcpyDeviceToHost));
        }
        if (ends[0] != 0 || ends[1] != nnz) throw Error{PLM_E_GRAPH, "offsets[0] must be 0 and offsets[n] = nnz"};
        plm_server::Req r;
        r.n = n;
        r.nnz = nnz;
        r.off = offsets;
        r.col = cols;
        r.w = weights;
        r.mem_kind = mem_kind;
        r.bytes = footprint(n, nnz, weights != nullptr);
        if (r.bytes > s->budget) throw Error{PLM_E_BUDGET, "the request alone exceeds the HBM budget"};
        int64_t id = s->next_id++;
        s->reqs[id] = r;
        s->queue.push_back(id);
        *request_id = id;
    });
}

plm_status plm_server_step(plm_server *s, int32_t *completed_out) {
    return server_guard(s, [&] {
        int32_t c = s->step();
        if (completed_out) *completed_out = c;
    });
}

plm_status plm_server_result(plm_server *s, int64_t request_id, int32_t *labels, int32_t mem_kind, double *q_out,
                             int32_t *levels_out, int32_t *ready_out) {
    return server_guard(s, [&] {
        auto it = s->reqs.find(request_id);
        if (it == s->reqs.end()) throw Error{PLM_E_ARG, "unknown or already fetched request"};
        plm_server::Req &r = it->second;
        if (ready_out) *ready_out = r.state != 0 ? 1 : 0;
        if (r.state == 0) return;
        if (r.state == 2) {
            Error e{r.err, r.msg};
            s->reqs.erase(it);
            throw e;
        }
        if (mem_kind != PLM_MEM_HOST && mem_kind != PLM_MEM_DEVICE) throw Error{PLM_E_ARG, "bad mem_kind"};
        if (labels && r.n > 0)
            HIPCHK(hipMemcpyAsync(labels, r.labels, (size_t)r.n * 4,
                                  mem_kind == PLM_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s->st));
        HIPCHK(hipStreamSynchronize(s->st));
        if (q_out) *q_out = r.q;
        if (levels_out) *levels_out = r.levels;
        (void)hipFree(r.labels);
        s->reqs.erase(it);
    });
}

plm_status plm_server_info(plm_server *s, plm_server_info_t *out) {
    return server_guard(s, [&] {
        if (!out) throw Error{PLM_E_ARG, "out is NULL"};
        out->queued = (int64_t)s->queue.size();
        out->completed = s->completed;
        out->batches = s->batches;
        out->held_results = (int64_t)s->reqs.size() - (int64_t)s->queue.size();
        out->budget_bytes = s->budget;
    });
}

void plm_server_destroy(plm_server *s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->st);
    delete s;
}

const char *plm_server_last_error(const plm_server *s) { return s ? s->err.c_str() : ""; }

}  // extern "C"
