// serve.hip - request server over the batched engine (plm_server_* in
// include/plm.h).
//
// Requests (one graph each) wait in a first-in first-out queue.  A step admits
// queued requests in order while their resident footprint fits what the HBM
// budget leaves beside the batches still running (and their entries fit the
// per-batch cap), lays their CSRs side by side in device memory as one
// disjoint union, runs Algorithm 3 on all of them at once (run_batch in
// api.hip: every graph gets exactly the result of its own run), and completes
// them.  Labels stay in device memory until the client fetches them.
//
// With max_inflight = 1 the batch runs inside the step, on the server's
// stream.  With k >= 2, k worker threads of the server each own a stream; a
// step hands the admitted batch to a free worker and returns, so requests that
// arrive while batches run are admitted as soon as a worker and budget are
// free, and the batches' kernels share the device.
//
// With opt.join (continuous batching) batches always run on workers, and a
// running batch takes queued requests in at each of its level boundaries, as
// far as the budget and the entry cap allow: each joins at level 0 of its own
// run inside the batch's union (run_batch with hooks in api.hip), and every
// request completes as soon as its own run ends.
#include <hip/hip_runtime.h>

#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/plm.h"
#include "plm_internal.h"

plm_status plm_internal_batch_adopt(plm_ctx **out, int64_t G, const int64_t *node_base, int64_t nnz, int64_t *off,
                                    int32_t *col, int32_t *w, void *hip_stream, const plm_options *opt);
plm_status plm_internal_batch_serve(plm_ctx *ctx, plm::BatchHooks *hooks);

namespace {

using plm::cdiv;
using plm::Error;

// Resident bytes of one graph while it runs: the CSR (with a weight array:
// the union of a batch carries one, unit weights written out, as soon as any
// of its graphs is weighted), per-node state of the level engine and the
// batch bookkeeping, and the sort buffers of contraction.
int64_t footprint(int64_t n, int64_t nnz) { return 8 * (n + 1) + 8 * nnz + 128 * n + 64 * nnz; }

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
        int state = 0;  // 0 queued, 3 running, 1 done, 2 failed
        bool solo = false;  // runs in a batch of its own (its batch was refused as a whole)
        int32_t *labels = nullptr;  // device, when done
        double q = 0.0;
        int32_t levels = 0;
        int64_t bytes = 0;
        plm_status err = PLM_OK;
        std::string msg;
    };
    // one admitted batch: the requests (ids and copies of their descriptors)
    struct Job {
        std::vector<int64_t> ids;
        std::vector<Req> in;
        int64_t bytes = 0, entries = 0;
    };
    hipStream_t st = nullptr;
    bool own_st = false;          // st created here (none given): results never touch the legacy stream
    hipStream_t io_st = nullptr;  // reads of device requests at submission (created on first use)
    plm_options opt;
    int64_t budget = 0, max_entries = 0;
    int32_t max_inflight = 1;
    std::string err;
    // everything below is guarded by mu
    std::mutex mu;
    std::condition_variable cv_job, cv_idle;
    std::deque<int64_t> queue;
    std::unordered_map<int64_t, Req> reqs;
    std::deque<Job> jobs;  // admitted, waiting for a worker
    int64_t next_id = 0, completed = 0, batches = 0, resident = 0, inflight = 0, unreported = 0, joined = 0;
    bool stop = false;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> wstreams;

    ~plm_server() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv_job.notify_all();
        for (auto &t : workers) t.join();
        for (auto s : wstreams) (void)hipStreamDestroy(s);
        if (io_st) (void)hipStreamDestroy(io_st);
        if (own_st && st) (void)hipStreamDestroy(st);
        for (auto &kv : reqs)
            if (kv.second.labels) (void)hipFree(kv.second.labels);
    }

    // Admission (mu held): the longest queue prefix whose footprint fits the
    // budget beside the running batches and whose entries fit the cap; with
    // nothing running, at least one request.  False when none is admitted.
    bool admit(Job &job) {
        int64_t bytes = 0, entries = 0;
        const int64_t room = budget - resident;
        while (!queue.empty()) {
            const Req &r = reqs[queue.front()];
            if (!job.ids.empty() && (r.solo || bytes + r.bytes > room || entries + r.nnz > max_entries)) break;
            if (job.ids.empty() && inflight > 0 && r.bytes > room) break;  // waits for memory
            bytes += r.bytes;
            entries += r.nnz;
            job.ids.push_back(queue.front());
            queue.pop_front();
            if (r.solo) break;
        }
        if (job.ids.empty()) return false;
        for (int64_t id : job.ids) {
            Req &r = reqs[id];
            r.state = 3;
            job.in.push_back(r);
        }
        job.bytes = bytes;
        job.entries = entries;
        resident += bytes;
        ++inflight;
        return true;
    }

    // end of a batch (mu held): its memory goes back to the budget
    void retire(const Job &job) {
        resident -= job.bytes;
        --inflight;
        cv_idle.notify_all();
    }

    // every request of the job still running fails with (code, m) (mu held)
    void fail_job(const Job &job, plm_status code, const std::string &m) {
        for (int64_t id : job.ids) {
            Req &r = reqs[id];
            if (r.state != 3) continue;  // completed already (continuous batching)
            r.state = 2;
            r.err = code;
            r.msg = m;
            ++unreported;
        }
        retire(job);
    }

    // Continuous batching (mu held): the queue prefix that fits beside what
    // runs, joining job at a level boundary; those requests are marked
    // running and charged to the job.
    std::vector<int64_t> admit_joiners(Job &job) {
        std::vector<int64_t> ids;
        while (!queue.empty() && !stop) {
            Req &r = reqs[queue.front()];
            if (r.solo || resident + r.bytes > budget || job.entries + r.nnz > max_entries) break;
            ids.push_back(queue.front());
            queue.pop_front();
            r.state = 3;
            resident += r.bytes;
            job.bytes += r.bytes;
            job.entries += r.nnz;
        }
        return ids;
    }

    // Runs one admitted batch on stream s (mu not held).
    void run_job(Job &job, hipStream_t s) {
        const int64_t G = (int64_t)job.ids.size();
        std::vector<int64_t> nbase(G + 1, 0), ebase(G + 1, 0);
        bool weighted = false;
        for (int64_t g = 0; g < G; ++g) {
            const Req &r = job.in[g];
            nbase[g + 1] = nbase[g] + r.n;
            ebase[g + 1] = ebase[g] + r.nnz;
            weighted = weighted || r.w != nullptr;
        }
        const int64_t N = nbase[G], E = ebase[G];
        auto fail_all = [&](plm_status code, const std::string &m) {
            std::lock_guard<std::mutex> lk(mu);
            fail_job(job, code, m);
        };
        if (N >= (1LL << 31)) return fail_all(PLM_E_BUDGET, "admitted requests exceed 2^31 nodes");
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
            return fail_all(PLM_E_NOMEM, "device allocation of the batch failed");
        }
        try {
            for (int64_t g = 0; g < G; ++g) {
                const Req &r = job.in[g];
                hipMemcpyKind kind = r.mem_kind == PLM_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
                if (r.n > 0) HIPCHK(hipMemcpyAsync(off + nbase[g], r.off, (size_t)r.n * 8, kind, s));
                if (r.nnz > 0) HIPCHK(hipMemcpyAsync(col + ebase[g], r.col, (size_t)r.nnz * 4, kind, s));
                if (r.nnz > 0 && r.w) HIPCHK(hipMemcpyAsync(w + ebase[g], r.w, (size_t)r.nnz * 4, kind, s));
                int64_t m = r.n > r.nnz ? r.n : r.nnz;
                if (m > 0)
                    hipLaunchKernelGGL(k_union_fix, dim3((unsigned)cdiv(m, 256)), dim3(256), 0, s, off + nbase[g],
                                       r.n, ebase[g], col + ebase[g], r.nnz, (int32_t)nbase[g],
                                       weighted ? w + ebase[g] : nullptr, (weighted && !r.w) ? 1 : 0);
            }
            hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, s, off + N, E);
            HIPCHK(hipGetLastError());
            HIPCHK(hipStreamSynchronize(s));
        } catch (const Error &e) {
            (void)hipFree(off);
            (void)hipFree(col);
            if (w) (void)hipFree(w);
            return fail_all(e.code, e.msg);
        }
        plm_ctx *ctx = nullptr;
        plm_status rc = plm_internal_batch_adopt(&ctx, G, nbase.data(), E, off, col, w, s, &opt);
        if (rc == PLM_E_GRAPH && G > 1) {
            // an invalid graph refuses the whole union: these requests go back to
            // the front of the queue, in their order, to run one per batch, so
            // that only the invalid ones fail
            std::lock_guard<std::mutex> lk(mu);
            for (int64_t g = G - 1; g >= 0; --g) {
                Req &r = reqs[job.ids[g]];
                r.solo = true;
                r.state = 0;
                queue.push_front(job.ids[g]);
            }
            retire(job);
            return;
        }
        if (rc != PLM_OK) return fail_all(rc, plm_last_error(nullptr));
        int32_t *canon = nullptr;
        if (hipMalloc(&canon, (size_t)(N > 0 ? N : 1) * 4) != hipSuccess) {
            (void)hipGetLastError();
            plm_destroy(ctx);
            return fail_all(PLM_E_NOMEM, "device allocation of the labels failed");
        }
        if (opt.join) {
            (void)hipFree(canon);
            return serve_joining(job, ctx, s);
        }
        std::vector<double> q(G);
        std::vector<int32_t> lv(G);
        rc = plm_batch_run(ctx, canon, q.data(), lv.data());
        if (rc != PLM_OK) {
            std::string m = plm_last_error(ctx);
            plm_destroy(ctx);
            (void)hipFree(canon);
            return fail_all(rc, m);
        }
        plm_destroy(ctx);
        std::vector<int32_t *> lab(G, nullptr);
        for (int64_t g = 0; g < G; ++g) {
            const int64_t n = job.in[g].n;
            if (hipMalloc(&lab[g], (size_t)(n > 0 ? n : 1) * 4) != hipSuccess ||
                (n > 0 && hipMemcpyAsync(lab[g], canon + nbase[g], (size_t)n * 4, hipMemcpyDeviceToDevice, s) !=
                              hipSuccess)) {
                (void)hipGetLastError();
                if (lab[g]) (void)hipFree(lab[g]);
                lab[g] = nullptr;
            }
        }
        (void)hipStreamSynchronize(s);
        (void)hipFree(canon);
        std::lock_guard<std::mutex> lk(mu);
        for (int64_t g = 0; g < G; ++g) {
            Req &r = reqs[job.ids[g]];
            if (!lab[g]) {
                r.state = 2;
                r.err = PLM_E_NOMEM;
                r.msg = "device allocation or copy of the result failed";
                continue;
            }
            r.state = 1;
            r.labels = lab[g];
            r.q = q[g];
            r.levels = lv[g];
            ++completed;
        }
        unreported += G;
        ++batches;
        retire(job);
    }

    // Continuous batching: runs the batch of ctx (its first job.ids.size()
    // graphs) with hooks that take queued requests in at level boundaries and
    // complete every request when its run ends (mu not held).
    void serve_joining(Job &job, plm_ctx *ctx, hipStream_t s) {
        std::vector<int64_t> offered;
        plm::BatchHooks hooks;
        hooks.join = [&]() {
            std::vector<plm::JoinGraph> js;
            std::lock_guard<std::mutex> lk(mu);
            offered = admit_joiners(job);
            for (int64_t id : offered) {
                const Req &r = reqs[id];
                plm::JoinGraph j;
                j.n = r.n;
                j.nnz = r.nnz;
                j.off = r.off;
                j.col = r.col;
                j.w = r.w;
                j.mem_kind = r.mem_kind;
                js.push_back(j);
            }
            return js;
        };
        hooks.joined = [&](const std::vector<int> &codes, const std::vector<std::string> &msgs) {
            std::lock_guard<std::mutex> lk(mu);
            for (size_t i = 0; i < offered.size(); ++i) {
                Req &r = reqs[offered[i]];
                if (codes[i] == PLM_OK) {
                    job.ids.push_back(offered[i]);
                    job.in.push_back(r);
                    ++joined;
                    continue;
                }
                r.state = 2;
                r.err = codes[i];
                r.msg = msgs[i];
                ++unreported;
                resident -= r.bytes;
                job.bytes -= r.bytes;
                job.entries -= r.nnz;
            }
            offered.clear();
        };
        hooks.done = [&](int64_t g, const int32_t *labels, int64_t n, double q, int32_t levels) {
            int32_t *buf = nullptr;
            bool ok = hipMalloc(&buf, (size_t)(n > 0 ? n : 1) * 4) == hipSuccess &&
                      (n == 0 || hipMemcpyAsync(buf, labels, (size_t)n * 4, hipMemcpyDeviceToDevice, s) == hipSuccess) &&
                      hipStreamSynchronize(s) == hipSuccess;
            if (!ok) {
                (void)hipGetLastError();
                if (buf) (void)hipFree(buf);
                buf = nullptr;
            }
            std::lock_guard<std::mutex> lk(mu);
            Req &r = reqs[job.ids[g]];
            if (!buf) {
                r.state = 2;
                r.err = PLM_E_NOMEM;
                r.msg = "device allocation or copy of the result failed";
            } else {
                r.state = 1;
                r.labels = buf;
                r.q = q;
                r.levels = levels;
                ++completed;
            }
            ++unreported;
        };
        plm_status rc = plm_internal_batch_serve(ctx, &hooks);
        std::string m = rc != PLM_OK ? std::string(plm_last_error(ctx)) : std::string();
        plm_destroy(ctx);
        std::lock_guard<std::mutex> lk(mu);
        if (!offered.empty()) {  // taken from the queue but never handed over
            for (int64_t id : offered) {
                job.ids.push_back(id);
                job.in.push_back(reqs[id]);
            }
        }
        if (rc != PLM_OK) {
            fail_job(job, rc, m);
            return;
        }
        ++batches;
        fail_job(job, PLM_E_STATE, "internal: request not reported by its batch");  // none expected; retires
    }

    // run_job, with anything thrown outside its own error paths (host
    // allocation) failing the batch instead of escaping
    void run_job_safe(Job &job, hipStream_t s) {
        try {
            run_job(job, s);
        } catch (...) {
            std::lock_guard<std::mutex> lk(mu);
            fail_job(job, PLM_E_NOMEM, "host allocation failed while running the batch");
        }
    }

    void worker(hipStream_t s) {
        for (;;) {
            Job job;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_job.wait(lk, [&] { return stop || !jobs.empty(); });
                if (jobs.empty()) return;  // stopping, and nothing left to run
                job = std::move(jobs.front());
                jobs.pop_front();
            }
            run_job_safe(job, s);
        }
    }

    void start_workers() {
        for (int32_t i = 0; i < max_inflight; ++i) {
            hipStream_t s = nullptr;
            HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));  // default priority
            wstreams.push_back(s);
        }
        for (int32_t i = 0; i < max_inflight; ++i) {
            hipStream_t s = wstreams[i];
            workers.emplace_back([this, s] { worker(s); });
        }
    }

    // One step; *reported = requests completed or failed since the last report.
    void step(int32_t *reported) {
        if (max_inflight == 1 && !opt.join) {
            Job job;
            bool got;
            {
                std::lock_guard<std::mutex> lk(mu);
                got = admit(job);
            }
            if (got) run_job_safe(job, st);
        } else {
            std::lock_guard<std::mutex> lk(mu);
            Job job;
            if (inflight < max_inflight && admit(job)) {
                jobs.push_back(std::move(job));
                cv_job.notify_one();
            }
        }
        std::lock_guard<std::mutex> lk(mu);
        if (reported) *reported = (int32_t)unreported;
        unreported = 0;
    }

    void wait_idle(int32_t *reported) {
        std::unique_lock<std::mutex> lk(mu);
        cv_idle.wait(lk, [&] { return inflight == 0; });
        if (reported) *reported = (int32_t)unreported;
        unreported = 0;
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

plm_status plm_server_create(plm_server **out, int64_t hbm_budget_bytes, int64_t max_batch_entries,
                             int32_t max_inflight, void *hip_stream, const plm_options *opt) {
    if (!out) return PLM_E_ARG;
    *out = nullptr;
    if (hbm_budget_bytes <= 0 || max_batch_entries <= 0 || max_inflight < 1 || max_inflight > 16) return PLM_E_ARG;
    plm_options o;
    plm_default_options(&o);
    if (opt) o = *opt;
    if (o.schedule != PLM_SCHEDULE_COLOUR || o.int_mode == PLM_INT_64 || o.refine || o.join < 0) return PLM_E_ARG;
    plm_server *s = new (std::nothrow) plm_server();
    if (!s) return PLM_E_NOMEM;
    s->st = (hipStream_t)hip_stream;
    if (!s->st && (max_inflight > 1 || o.join)) {
        // the result copies of the client thread go to a stream of the server's
        // own, so that they never wait on the legacy stream while a worker
        // captures a sweep
        if (hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            delete s;
            return PLM_E_DEVICE;
        }
        s->own_st = true;
    }
    s->opt = o;
    s->budget = hbm_budget_bytes;
    s->max_entries = max_batch_entries;
    s->max_inflight = max_inflight;
    // with several workers, batches launch one by one (a capture in one worker
    // made other threads' synchronous copies on the legacy stream fail); a
    // single worker (continuous batching) replays its captured sweeps, and the
    // client's result copies then go to the server's own stream
    if (max_inflight > 1) s->opt.graph_sweeps = 0;
    if (max_inflight > 1 || o.join) {
        try {
            s->start_workers();
        } catch (...) {
            delete s;
            return PLM_E_DEVICE;
        }
    }
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
            // on a stream of the server's own, not the legacy default stream
            if (!s->io_st) HIPCHK(hipStreamCreateWithFlags(&s->io_st, hipStreamNonBlocking));
            HIPCHK(hipMemcpyAsync(&ends[0], offsets, 8, hipMemcpyDeviceToHost, s->io_st));
            HIPCHK(hipMemcpyAsync(&ends[1], offsets + n, 8, hipMemcpyDeviceToHost, s->io_st));
            HIPCHK(hipStreamSynchronize(s->io_st));
        }
        if (ends[0] != 0 || ends[1] != nnz) throw Error{PLM_E_GRAPH, "offsets[0] must be 0 and offsets[n] = nnz"};
        plm_server::Req r;
        r.n = n;
        r.nnz = nnz;
        r.off = offsets;
        r.col = cols;
        r.w = weights;
        r.mem_kind = mem_kind;
        r.bytes = footprint(n, nnz);
        if (r.bytes > s->budget) throw Error{PLM_E_BUDGET, "the request alone exceeds the HBM budget"};
        std::lock_guard<std::mutex> lk(s->mu);
        int64_t id = s->next_id++;
        s->reqs[id] = r;
        s->queue.push_back(id);
        *request_id = id;
    });
}

plm_status plm_server_step(plm_server *s, int32_t *completed_out) {
    return server_guard(s, [&] { s->step(completed_out); });
}

plm_status plm_server_wait(plm_server *s, int32_t *completed_out) {
    return server_guard(s, [&] { s->wait_idle(completed_out); });
}

plm_status plm_server_result(plm_server *s, int64_t request_id, int32_t *labels, int32_t mem_kind, double *q_out,
                             int32_t *levels_out, int32_t *ready_out) {
    return server_guard(s, [&] {
        plm_server::Req r;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            auto it = s->reqs.find(request_id);
            if (it == s->reqs.end()) throw Error{PLM_E_ARG, "unknown or already fetched request"};
            const int state = it->second.state;
            if (ready_out) *ready_out = (state == 1 || state == 2) ? 1 : 0;
            if (state == 0 || state == 3) return;
            if (state == 1 && mem_kind != PLM_MEM_HOST && mem_kind != PLM_MEM_DEVICE)
                throw Error{PLM_E_ARG, "bad mem_kind"};
            r = it->second;  // done or failed: no worker touches it any more
            s->reqs.erase(it);
        }
        if (r.state == 2) throw Error{r.err, r.msg};
        plm_status rc = PLM_OK;
        std::string m;
        try {
            if (labels && r.n > 0)
                HIPCHK(hipMemcpyAsync(labels, r.labels, (size_t)r.n * 4,
                                      mem_kind == PLM_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                      s->st));
            HIPCHK(hipStreamSynchronize(s->st));
        } catch (const Error &e) {
            rc = e.code;
            m = e.msg;
        }
        (void)hipFree(r.labels);
        if (rc != PLM_OK) throw Error{rc, m};
        if (q_out) *q_out = r.q;
        if (levels_out) *levels_out = r.levels;
    });
}

plm_status plm_server_info(plm_server *s, plm_server_info_t *out) {
    return server_guard(s, [&] {
        if (!out) throw Error{PLM_E_ARG, "out is NULL"};
        std::lock_guard<std::mutex> lk(s->mu);
        int64_t running = 0;
        for (const auto &kv : s->reqs) running += kv.second.state == 3 ? 1 : 0;
        out->queued = (int64_t)s->queue.size();
        out->completed = s->completed;
        out->batches = s->batches;
        out->held_results = (int64_t)s->reqs.size() - (int64_t)s->queue.size() - running;
        out->budget_bytes = s->budget;
        out->inflight = s->inflight;
        out->running = running;
        out->resident_bytes = s->resident;
        out->joined = s->joined;
    });
}

void plm_server_destroy(plm_server *s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->st);
    delete s;  // the workers finish the batches they hold, then join
}

const char *plm_server_last_error(const plm_server *s) { return s ? s->err.c_str() : ""; }

}  // extern "C"
