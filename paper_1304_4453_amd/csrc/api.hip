// api.hip - the C ABI of libplm (include/plm.h) and the level engine behind it:
// level set-up, schedule, sweeps, coarsening and the multilevel run of
// Algorithm 3 with prolongation.
#include <hip/hip_runtime.h>

#include <dlfcn.h>

#include <chrono>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <exception>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "../../include/plm.h"
#include "level.h"

using namespace plm;

namespace {

thread_local std::string g_create_error;

// Workspace of plm_modularity_noalloc: the volume of every label (int64) and
// four counters.  One copy per device, held until the process ends; host code
// reaches it only through the address hipGetSymbolAddress returns on that
// device (noalloc_workspace), never through the array's name.
constexpr int64_t kNoAllocMaxNodes = PLM_NOALLOC_MAX_NODES;
constexpr size_t kNoAllocBytes = (size_t)kNoAllocMaxNodes * 8 + 256;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
constexpr int kNoAllocDevices = 64;
void *g_noalloc_ptr[kNoAllocDevices] = {};
std::mutex g_noalloc_mu;

// batched runs: rebuild the class buckets when the graphs still sweeping hold
// less than this fraction of the planned entries
constexpr double kReplanFraction = 0.7;
// timing events per class step: start and stop of the 5 kernel groups (the
// partitioned group's part launch), then start and stop of the agg launch
constexpr size_t kEv = 12;
// settled nodes: a move phase arms after a sweep that moved at most n / this
// (input level, coarse levels); measured on R-MAT 26: arming at n / 64 on the
// input level costs 45 ms more sweep time, and the coarse level's sweeps take
// 1,675 / 1,625 / 1,601 / 1,575 ms arming at n / 16, 64, 256, 1024
constexpr int64_t kSettleDiv = 16;
constexpr int64_t kSettleDivCoarse = 1024;
// single graphs with more entries take the sweep layout by default (opt.layout = 0)
constexpr int64_t kLayoutMinEntries = (int64_t)1 << 27;
// pinned host scratch of a context, in int64 words (the colouring's counter
// read-back takes 480 int32)
constexpr size_t kHostWords = 512;

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

template <typename T>
T *dev_alloc(int64_t count) {
    T *p = nullptr;
    size_t bytes = (size_t)(count > 0 ? count : 1) * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{PLM_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
    }
    return p;
}

template <typename T>
void dev_free(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

struct LevelData {
    int64_t n = 0, nnz = 0;
    int64_t *off = nullptr;
    int32_t *col = nullptr;
    void *w = nullptr;
    int wkind = 0;
    int diag_mult = 1;
    int32_t *pi = nullptr;  // fine -> coarse map, set when this level is coarsened
    // batched runs: graph (index among this level's graphs) of each node, and
    // the first node of each graph (count + 1 entries)
    int32_t *gid = nullptr;
    int64_t *gbase = nullptr;
    int32_t *gshift = nullptr;  // batches with joined graphs: per graph, the batch level it joined at
    // colouring of this level kept by a descent that refines on its way back
    // up (the refinement's colouring is the same: same graph, seed and level)
    int32_t *colour_kept = nullptr;
    int32_t ncol_kept = 0;
    bool borrowed = false;  // off/col/w belong to another context (ensemble base runs)
    // sweep layout of this level (see MoveState), built with its first plan
    int32_t *sig = nullptr, *ord = nullptr, *colp = nullptr;

    GraphView view() const {
        GraphView g;
        g.n = n; g.nnz = nnz; g.off = off; g.col = col; g.w = w; g.wkind = wkind; g.diag_mult = diag_mult;
        g.gid = gid; g.gbase = gbase; g.gshift = gshift;
        return g;
    }
    void release() {
        if (borrowed) {
            off = nullptr; col = nullptr; w = nullptr;
        }
        dev_free(off); dev_free(col); dev_free(w); dev_free(pi); dev_free(gid); dev_free(gbase); dev_free(gshift);
        dev_free(colour_kept); dev_free(sig); dev_free(ord); dev_free(colp);
    }
};

__global__ void k_export_w(GraphView g, int64_t *out) {
    int64_t e0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 16;
    if (e0 >= g.nnz) return;
    int64_t e1 = e0 + 16 < g.nnz ? e0 + 16 : g.nnz;
    int64_t r = row_of(g.off, g.n, e0);
    int64_t rend = g.off[r + 1];
    for (int64_t e = e0; e < e1; ++e) {
        while (e >= rend) { r = next_row(g.off, g.n, r, e); rend = g.off[r + 1]; }
        int64_t x = g.wkind == 0 ? 1 : (g.wkind == 1 ? (int64_t)((const int32_t *)g.w)[e] : ((const int64_t *)g.w)[e]);
        if (g.col[e] == r) x *= g.diag_mult;
        out[e] = x;
    }
}

// rows holding a self-loop entry (rows are strictly ascending: binary search)
__global__ __launch_bounds__(256) void k_count_loops(GraphView g, unsigned long long *cnt) {
    unsigned long long c = 0;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < g.n; u += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = g.off[u], hi = g.off[u + 1];
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            int32_t x = g.col[mid];
            if (x == u) { ++c; break; }
            if (x < u) lo = mid + 1; else hi = mid;
        }
    }
    block_count_add(cnt, c);
}

__global__ __launch_bounds__(256) void k_count_loop_only(GraphView g, unsigned long long *cnt) {
    unsigned long long c = 0;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < g.n; u += (int64_t)gridDim.x * blockDim.x) {
        int64_t d = g.off[u + 1] - g.off[u];
        c += (d == 1 && g.col[g.off[u]] == u) ? 1 : 0;
    }
    block_count_add(cnt, c);
}

}  // namespace

struct plm_ctx {
    hipStream_t st = nullptr;
    plm_options opt;
    int mem_kind = PLM_MEM_HOST;
    std::string err;
    std::vector<LevelData> levels;  // [0] = private copy of the input
    int cur = 0;
    int64_t n0 = 0, S = 0;
    // state of the current level (capacity n0)
    int64_t *vol0 = nullptr, *vol = nullptr, *volC = nullptr;
    int32_t *zeta = nullptr, *colour = nullptr, *class_nodes = nullptr, *move_to = nullptr, *lab = nullptr;
    NodeRec *noderec = nullptr;  // per class position: node and row (with class_nodes)
    // the sweep layout's copies of zeta and volC (see MoveState), synchronised
    // from them before a sweep whenever they changed outside the apply
    int32_t *zetap = nullptr;
    int64_t *volCp = nullptr;
    bool layout_dirty = true;
    int64_t *bstart_dev = nullptr;
    int64_t max_vol = 0, wide_lim = 0;
    bool sched = false;
    int32_t ncol = 0, jp_rounds = 0;
    std::vector<int64_t> bstart;
    std::vector<ClassRange> classes;
    int64_t active_nodes = 0, active_entries = 0;
    // hub arrays of the current level (see the hub kernels in move.hip)
    int32_t *hub_pos = nullptr, *nchunk = nullptr, *pbits = nullptr, *stg_x = nullptr;
    int64_t *ins_first = nullptr, *agg_first = nullptr, *stg_off = nullptr, *bkt_off = nullptr, *stg_w = nullptr,
            *wd_part = nullptr, *hub_base = nullptr;
    uint32_t *bkt = nullptr;
    unsigned long long *part = nullptr;
    int32_t *hub_u = nullptr, *ins_hub = nullptr, *agg_hub = nullptr, *sgl_hub = nullptr, *red_hub = nullptr;
    int64_t cap_hubs = 0, cap_stg = 0, cap_bkt = 0, cap_ins = 0, cap_agg = 0, cap_hubu = 0, cap_ihub = 0,
            cap_ahub = 0, cap_shub = 0, cap_rhub = 0;
    int32_t sweeps = 0;
    // device counters: [0] moves, [1..4] candidates per bin, [5] S, [6] max vol,
    // [7] loop-only rows, [8..11] entries per bin, [12] self-loops, [13]
    // candidates of the one-workgroup hubs
    unsigned long long *dcnt = nullptr;
    int64_t bin_nodes[4] = {0, 0, 0, 0}, bin_entries[4] = {0, 0, 0, 0};
    int64_t sgl_nodes = 0, sgl_entries = 0;  // hubs of the one-workgroup path
    int64_t loops = 0;  // self-loop entries of the current level
    int64_t *hbuf = nullptr;             // pinned host scratch (kHostWords int64)
    void *noalloc_ws = nullptr;          // this device's plm_modularity_noalloc workspace
    Scratch scr;
    plm_stats_t stats;
    std::vector<hipEvent_t> events;

    // batched runs (plm_batch_create): G graphs side by side on node ranges
    // gbase0_h[g] .. gbase0_h[g+1]; levels[0].gid / .gbase hold the input ranges
    bool batch = false;
    int64_t G = 0;
    std::vector<int64_t> gbase0_h;
    int64_t *gS0 = nullptr, *gwl0 = nullptr;   // per input graph: S and 64-bit limit
    std::vector<int64_t> act_h;                // graphs of the current level (input ids)
    int64_t *act = nullptr, *gS = nullptr, *gwl = nullptr;  // the same, per current graph
    int32_t *bflag = nullptr, *bout = nullptr;
    int64_t *bnewid = nullptr, *bgath = nullptr;
    void *bscan = nullptr;
    uint8_t *bstatus = nullptr, *bkeep = nullptr, *bsweep = nullptr;
    int32_t *bgmoved = nullptr;  // per graph of the level: moved in the current sweep
    // continuous batching (request server): per input graph the batch level it
    // joined at, and the canonical labels of graphs reported as they finish
    std::vector<int32_t> bshift_h;
    int32_t *bcanon = nullptr;
    unsigned long long *bI2 = nullptr, *bsq = nullptr;

    // settled nodes (see move.hip): per node the moved neighbour weight since
    // its last decision, the slacks of its last stay and the moved-volume clock
    // it was taken at; sctl = [on, clock].  Armed for a move phase once its
    // sweeps move few nodes (opt.settle).
    uint64_t *dw = nullptr;
    int64_t *slack = nullptr, *kslack = nullptr;
    uint64_t *tstamp = nullptr;
    unsigned long long *sctl = nullptr;
    bool skip_armed = false;
    int64_t armed_sweeps = 0;
    int32_t *hub_skip = nullptr;
    uint64_t *hub_clk = nullptr;
    // launch plans of the hub kernels (one record per workgroup of the
    // level-wide lists) and each hub's first chunk / bucket list index
    HubSglPlan *splan = nullptr;
    HubPartPlan *pplan = nullptr;
    HubAggPlan *aplan = nullptr;
    HubRedPlan *rplan = nullptr;
    int64_t *ins_abs = nullptr, *agg_abs = nullptr, *red_abs = nullptr;

    // label propagation (Algorithm 1): active flag of each node; lp_mode turns
    // the class steps into label-propagation steps with tie keys of lp_seed
    uint8_t *active = nullptr;
    bool lp_mode = false;
    uint64_t lp_seed = 0;
    // device time and algorithmic bytes of the last timed run_classes
    double last_ms = 0, last_bytes = 0;
    // states after the last two sweeps of a move phase (cycle detection)
    int32_t *snap[2] = {nullptr, nullptr};
    // a whole sweep's launches captured once per plan (graph_sweeps), on a
    // private stream (capture cannot use the null stream), replayed on st
    hipStream_t cap_st = nullptr;
    hipGraphExec_t sweep_exec = nullptr;
    // capture stream of the partitioned-hub branch of a captured sweep
    // (hub_stream), and a ring of fork/join events
    static constexpr int kAux = 4;  // branches beside the capture stream
    // kernel groups per branch with hub_stream = 2 (bit i: group i = lane,
    // wavefront, workgroup, one-workgroup hub, partitioned hub); measured on
    // R-MAT 26 against one branch per group and two other groupings
    static constexpr unsigned kBranchGroups[3] = {1u | 2u | 8u, 4u, 16u};
    hipStream_t hub_cap_st[kAux] = {};
    static constexpr int kForkRing = 16;
    hipEvent_t fork_ev[kForkRing] = {}, join_ev[kAux][kForkRing] = {};

    ~plm_ctx() {
        for (auto &l : levels) l.release();
        dev_free(vol0); dev_free(vol); dev_free(volC); dev_free(zeta); dev_free(colour); dev_free(class_nodes);
        dev_free(noderec); dev_free(zetap); dev_free(volCp); dev_free(move_to); dev_free(lab); dev_free(bstart_dev); dev_free(dcnt);
        dev_free(gS0); dev_free(gwl0); dev_free(act); dev_free(gS); dev_free(gwl); dev_free(bflag); dev_free(bout);
        dev_free(bnewid); dev_free(bgath); dev_free(bscan); dev_free(bstatus); dev_free(bkeep); dev_free(bI2);
        dev_free(bsq); dev_free(bsweep); dev_free(bgmoved); dev_free(active); dev_free(snap[0]); dev_free(snap[1]);
        dev_free(bcanon);
        dev_free(dw); dev_free(slack); dev_free(kslack); dev_free(tstamp); dev_free(sctl);
        free_hubs();
        if (hbuf) (void)hipHostFree(hbuf);
        for (auto e : events) (void)hipEventDestroy(e);
        drop_graph();
        if (cap_st) (void)hipStreamDestroy(cap_st);
        for (int a = 0; a < kAux; ++a)
            if (hub_cap_st[a]) (void)hipStreamDestroy(hub_cap_st[a]);
        for (int i = 0; i < kForkRing; ++i) {
            if (fork_ev[i]) (void)hipEventDestroy(fork_ev[i]);
            for (int a = 0; a < kAux; ++a)
                if (join_ev[a][i]) (void)hipEventDestroy(join_ev[a][i]);
        }
    }
    void drop_graph() {
        if (sweep_exec) (void)hipGraphExecDestroy(sweep_exec);
        sweep_exec = nullptr;
    }
    void free_hubs() {
        dev_free(hub_pos); dev_free(nchunk); dev_free(pbits); dev_free(stg_x); dev_free(ins_first);
        dev_free(agg_first); dev_free(stg_off); dev_free(bkt_off); dev_free(stg_w); dev_free(wd_part); dev_free(hub_base);
        dev_free(bkt); dev_free(part); dev_free(hub_u); dev_free(ins_hub); dev_free(agg_hub); dev_free(sgl_hub);
        dev_free(red_hub); dev_free(hub_skip); dev_free(hub_clk);
        dev_free(splan); dev_free(pplan); dev_free(aplan); dev_free(rplan); dev_free(ins_abs); dev_free(agg_abs);
        dev_free(red_abs);
        cap_hubs = cap_stg = cap_bkt = cap_ins = cap_agg = cap_hubu = cap_ihub = cap_ahub = cap_shub = cap_rhub = 0;
    }

    LevelData &L() { return levels[cur]; }

    // resolution gamma = gp / gq (normalised at creation)
    int64_t gp() const { return opt.gamma_num; }
    int64_t gq() const { return opt.gamma_den; }
    int64_t gmax() const { return opt.gamma_num > opt.gamma_den ? opt.gamma_num : opt.gamma_den; }
    // largest vol(u) whose gains fit 64 bits: S vol(u) max(p, q) < 2^62
    int64_t wide_limit(int64_t s) const {
        unsigned __int128 sg = (unsigned __int128)(uint64_t)s * (unsigned __int128)(uint64_t)gmax();
        if (sg == 0) return INT64_MAX;
        if (sg >> 62) return 0;
        return (int64_t)(((1ULL << 62) - 1) / (uint64_t)sg);
    }

    int64_t bin_lane() const { return opt.bin_lane > 0 ? opt.bin_lane : 16; }
    int64_t bin_wave() const { return opt.bin_wave > 0 ? opt.bin_wave : 512; }
    int64_t bin_block() const { return opt.bin_block > 0 ? opt.bin_block : 4096; }
    int64_t single_max_row() const { return opt.hub_row_max > 0 ? opt.hub_row_max : kSingleMaxRow; }

    // ---------------------------------------------------------------- level set-up
    void init_level() {
        LevelData &l = L();
        GraphView g = l.view();
        launch_volumes(g, vol, dcnt + 5, dcnt + 6, st);
        HIPCHK(hipMemsetAsync(dcnt + 12, 0, 8, st));
        if (l.n > 0) {
            const int64_t nb = cdiv(l.n, 256);
            hipLaunchKernelGGL(k_count_loops, dim3((unsigned)(nb < kCountGrid ? nb : kCountGrid)), dim3(256), 0, st, g,
                               dcnt + 12);
        }
        HIPCHK(hipMemcpyAsync(hbuf, dcnt + 5, 16, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(hbuf + 2, dcnt + 12, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        loops = hbuf[2];
        uint64_t s = (uint64_t)hbuf[0];
        if (cur == 0) {
            if (s >= (1ULL << 62))
                throw Error{PLM_E_GRAPH, batch ? "total weight of the batch must be below 2^62"
                                               : "total weight S = 2 w(E) must be below 2^62"};
            S = (int64_t)s;
            if (gp() != gq()) {
                unsigned __int128 b = (unsigned __int128)s * (unsigned __int128)s * (unsigned __int128)gmax();
                if (b >> 126) throw Error{PLM_E_ARG, "gamma != 1 needs S^2 max(gamma_num, gamma_den) < 2^126"};
            }
            HIPCHK(hipMemcpyAsync(vol0, vol, l.n * 8, hipMemcpyDeviceToDevice, st));
            if (batch) {
                launch_graph_S(vol, l.gbase, G, gmax(), gS0, gwl0, st);
                HIPCHK(hipMemcpyAsync(gS, gS0, G * 8, hipMemcpyDeviceToDevice, st));
                HIPCHK(hipMemcpyAsync(gwl, gwl0, G * 8, hipMemcpyDeviceToDevice, st));
            }
        } else if (batch) {
            // the graphs of this level keep their input S (contraction preserves it)
            launch_gather_i64(gS0, act, (int64_t)act_h.size(), gS, st);
            launch_gather_i64(gwl0, act, (int64_t)act_h.size(), gwl, st);
        } else if ((int64_t)s != S) {
            throw Error{PLM_E_STATE, "internal: coarse graph changed the total weight"};
        }
        max_vol = hbuf[1];
        wide_lim = wide_limit(S);
        if (!batch && opt.int_mode == PLM_INT_64 && max_vol > wide_lim)
            throw Error{PLM_E_STATE, "int_mode PLM_INT_64: S * vol(u) reaches 2^62 at this level"};
        launch_iota(zeta, l.n, st);
        launch_copy_vol(volC, vol, l.n, st);
        layout_dirty = true;
        sched = false;
        ncol = 0;
        sweeps = 0;
        disarm();
    }

    // ---------------------------------------------------------------- settled nodes
    // Armed: every node's moved weight at 0x8080... >= 2^63 (so the next class
    // steps decide them all and record their slacks; what moves add before
    // then stays below 2^64), clock at 0.  The kernels of a captured sweep
    // read sctl, so the same graph serves armed and unarmed sweeps.
    bool settle_usable() { return sctl != nullptr && opt.settle >= 0 && L().n > 0; }
    void arm() {
        HIPCHK(hipMemsetAsync(dw, 0x80, (size_t)L().n * 8, st));
        const unsigned long long on[2] = {1ULL, 0ULL};
        HIPCHK(hipMemcpyAsync(sctl, on, sizeof(on), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        skip_armed = true;
        armed_sweeps = 0;
    }
    void disarm() {
        if (!sctl || !skip_armed) return;
        HIPCHK(hipMemsetAsync(sctl, 0, 8, st));
        skip_armed = false;
    }

    // grow-only device arrays of the hub plan
    void ensure_hub_nodes(int64_t hubs) {
        if (hubs > cap_hubu) { dev_free(hub_u); hub_u = dev_alloc<int32_t>(hubs); cap_hubu = hubs; }
    }
    void ensure_hub_capacity(int64_t hubs, int64_t stg, int64_t bk, int64_t ins, int64_t agg, int64_t ins_tot,
                             int64_t agg_tot, int64_t sgl_tot, int64_t red_tot) {
        if (hubs > cap_hubs) {
            dev_free(hub_pos); dev_free(nchunk); dev_free(pbits); dev_free(ins_first); dev_free(agg_first);
            dev_free(stg_off); dev_free(bkt_off); dev_free(hub_base); dev_free(hub_skip); dev_free(hub_clk);
            dev_free(ins_abs); dev_free(agg_abs); dev_free(red_abs);
            ins_abs = dev_alloc<int64_t>(hubs);
            agg_abs = dev_alloc<int64_t>(hubs);
            red_abs = dev_alloc<int64_t>(hubs);
            hub_base = dev_alloc<int64_t>(hubs);
            hub_skip = dev_alloc<int32_t>(hubs);
            hub_clk = dev_alloc<uint64_t>(hubs);
            hub_pos = dev_alloc<int32_t>(hubs); nchunk = dev_alloc<int32_t>(hubs); pbits = dev_alloc<int32_t>(hubs);
            ins_first = dev_alloc<int64_t>(hubs); agg_first = dev_alloc<int64_t>(hubs);
            stg_off = dev_alloc<int64_t>(hubs); bkt_off = dev_alloc<int64_t>(hubs);
            cap_hubs = hubs;
        }
        if (stg > cap_stg) {
            dev_free(stg_x); dev_free(stg_w);
            stg_x = dev_alloc<int32_t>(stg); stg_w = dev_alloc<int64_t>(stg);
            cap_stg = stg;
        }
        if (bk > cap_bkt) { dev_free(bkt); bkt = dev_alloc<uint32_t>(bk); cap_bkt = bk; }
        if (ins > cap_ins) { dev_free(wd_part); wd_part = dev_alloc<int64_t>(ins); cap_ins = ins; }
        if (agg > cap_agg) { dev_free(part); part = dev_alloc<unsigned long long>(4 * agg); cap_agg = agg; }
        if (ins_tot > cap_ihub) {
            dev_free(ins_hub); dev_free(pplan);
            ins_hub = dev_alloc<int32_t>(ins_tot); pplan = dev_alloc<HubPartPlan>(ins_tot);
            cap_ihub = ins_tot;
        }
        if (agg_tot > cap_ahub) {
            dev_free(agg_hub); dev_free(aplan);
            agg_hub = dev_alloc<int32_t>(agg_tot); aplan = dev_alloc<HubAggPlan>(agg_tot);
            cap_ahub = agg_tot;
        }
        if (sgl_tot > cap_shub) {
            dev_free(sgl_hub); dev_free(splan);
            sgl_hub = dev_alloc<int32_t>(sgl_tot); splan = dev_alloc<HubSglPlan>(sgl_tot);
            cap_shub = sgl_tot;
        }
        if (red_tot > cap_rhub) {
            dev_free(red_hub); dev_free(rplan);
            red_hub = dev_alloc<int32_t>(red_tot); rplan = dev_alloc<HubRedPlan>(red_tot);
            cap_rhub = red_tot;
        }
    }

    void build_schedule() { build_schedule(opt.colour_seed, opt.schedule); }
    void build_schedule(uint64_t seed, int schedule) {
        LevelData &l = L();
        GraphView g = l.view();
        double t0 = now_ms();
        ncol = build_colouring(g, seed, cur, schedule, colour, scr, (int32_t *)hbuf, &jp_rounds, st,
                               opt.colour_tail != 0);
        if (cur < PLM_MAX_LEVELS) {
            stats.colour_ms[cur] = now_ms() - t0;
            stats.schedule_rounds[cur] = jp_rounds;
        }
        build_plan(nullptr);
    }

    // Class buckets and hub plan of the current colouring.  keep (batched runs,
    // device, one flag per graph of the level, else null): only the nodes of
    // kept graphs enter the buckets.
    // the sweep layout (see MoveState): large single graphs (opt.layout 0), all
    // single graphs (1) or none (-1); batches keep their graphs' own ids
    bool layout_wanted() const {
        const LevelData &l = levels[cur];
        return !batch && opt.layout >= 0 && l.n > 0 && (opt.layout == 1 || l.nnz > kLayoutMinEntries);
    }
    void ensure_layout() {
        LevelData &l = L();
        if (l.sig || !layout_wanted()) return;
        const GraphView g = l.view();
        l.sig = dev_alloc<int32_t>(l.n);
        l.ord = dev_alloc<int32_t>(l.n);
        l.colp = dev_alloc<int32_t>(l.nnz > 0 ? l.nnz : 1);
        if (!zetap) {
            zetap = dev_alloc<int32_t>(n0);
            volCp = dev_alloc<int64_t>(n0);
        }
        scr.reserve(4 * align_up(l.n * 4) + radix_scratch_bytes(l.n));
        uint32_t *k = (uint32_t *)scr.get(l.n * 4), *ka = (uint32_t *)scr.get(l.n * 4);
        int32_t *v = (int32_t *)scr.get(l.n * 4), *va = (int32_t *)scr.get(l.n * 4);
        void *rs = scr.get(radix_scratch_bytes(l.n));
        build_layout(g, l.sig, l.ord, l.colp, k, v, ka, va, rs, st);
        HIPCHK(hipStreamSynchronize(st));
        layout_dirty = true;
    }

    void build_plan(const uint8_t *keep) {
        drop_graph();  // the captured sweep belongs to the previous plan
        ensure_layout();
        LevelData &l = L();
        GraphView g = l.view();
        int64_t nkeys = (int64_t)ncol * 8 + 1;
        dev_free(bstart_dev);
        bstart_dev = dev_alloc<int64_t>(nkeys + 1);
        HIPCHK(hipMemsetAsync(dcnt + 7, 0, 5 * 8, st));
        build_buckets(g, vol, colour, ncol, bin_lane(), bin_wave(), bin_block(), class_nodes, bstart_dev, dcnt + 8,
                      scr, st, keep);
        bstart.assign(nkeys + 1, 0);
        if (l.n > 0) HIPCHK(hipMemcpyAsync(bstart.data(), bstart_dev, (nkeys + 1) * 8, hipMemcpyDeviceToHost, st));
        // active entries = nnz minus rows made of a single self-loop
        if (l.n > 0)
            hipLaunchKernelGGL(k_count_loop_only, dim3((unsigned)(cdiv(l.n, 256) < kCountGrid ? cdiv(l.n, 256) : kCountGrid)),
                               dim3(256), 0, st, g, dcnt + 7);
        HIPCHK(hipMemcpyAsync(hbuf + 8, dcnt + 7, 5 * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        // first position of bin b of class c (b = 4: the next class)
        auto bs = [&](int64_t c, int b) { return bstart[8 * c + 2 * b]; };
        active_nodes = l.n > 0 ? bstart[(size_t)ncol * 8] : 0;
        launch_node_recs(g, class_nodes, active_nodes, noderec, l.sig, st);
        active_entries = l.nnz - hbuf[8];
        for (int b = 0; b < 4; ++b) {
            bin_entries[b] = hbuf[9 + b];
            bin_nodes[b] = 0;
            for (int32_t c = 0; c < ncol; ++c) bin_nodes[b] += bs(c, b + 1) - bs(c, b);
        }
        // hubs: degrees to the host, then per-hub table and block layout
        classes.assign(ncol, ClassRange());
        int64_t H = 0;
        for (int32_t c = 0; c < ncol; ++c) H += bs(c, 4) - bs(c, 3);
        std::vector<int64_t> deg(H > 0 ? H : 1), pos;
        pos.reserve(H);
        if (H > 0) {
            ensure_hub_nodes(H);
            scr.reserve(align_up(H * 8));
            int64_t *ddeg = (int64_t *)scr.get(H * 8);
            int64_t o = 0;
            for (int32_t c = 0; c < ncol; ++c) {
                int64_t b = bs(c, 3), cnt = bs(c, 4) - b;
                if (cnt > 0) launch_hub_degrees(g, class_nodes, vol, b, cnt, ddeg + o, hub_u + o, st);
                for (int64_t i = 0; i < cnt; ++i) pos.push_back(b + i);
                o += cnt;
            }
            HIPCHK(hipMemcpyAsync(deg.data(), ddeg, H * 8, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        // per hub: one workgroup (rows up to kSingleMaxRow with vol(u) < 2^31), or
        // chunks of kHubInsChunk entries and 2^pbits buckets of ~kHubBucketTarget
        // entries with staging and (bucket, chunk) table offsets within its class;
        // per workgroup of each launch: its hub
        std::vector<int32_t> hpos(H > 0 ? H : 1), hch(H > 0 ? H : 1, 0), hpb(H > 0 ? H : 1, 0), shub, rhub, ihub,
            ahub;
        std::vector<int64_t> hins(H > 0 ? H : 1, 0), hagg(H > 0 ? H : 1, 0), hstg(H > 0 ? H : 1, 0),
            hbk(H > 0 ? H : 1, 0), hins_abs(H > 0 ? H : 1, 0), hagg_abs(H > 0 ? H : 1, 0),
            hred_abs(H > 0 ? H : 1, 0);
        int64_t max_stg = 0, max_bk = 0, max_ins = 0, max_agg = 0, hg = 0;
        sgl_nodes = sgl_entries = 0;
        for (int32_t c = 0; c < ncol; ++c) {
            ClassRange &cr = classes[c];
            for (int b = 0; b < 4; ++b) {
                cr.begin[b] = bs(c, b);
                cr.count[b] = bs(c, b + 1) - bs(c, b);
            }
            cr.quad = bstart[8 * c + 3] - bstart[8 * c + 2];
            cr.blk_short = bstart[8 * c + 5] - bstart[8 * c + 4];
            cr.hub_first = hg;
            cr.hub_count = cr.count[3];
            cr.sgl_base = (int64_t)shub.size();
            cr.red_base = (int64_t)rhub.size();
            cr.ins_base = (int64_t)ihub.size();
            cr.agg_base = (int64_t)ahub.size();
            int64_t stg = 0, bk = 0, ins = 0, agg = 0;
            for (int64_t i = 0; i < cr.hub_count; ++i, ++hg) {
                hpos[hg] = (int32_t)pos[hg];
                int64_t d = deg[hg] < 0 ? -deg[hg] : deg[hg];
                if (deg[hg] > 0 && d <= single_max_row()) {
                    shub.push_back((int32_t)hg);
                    ++sgl_nodes;
                    sgl_entries += d;
                    continue;
                }
                hred_abs[hg] = (int64_t)rhub.size();
                rhub.insert(rhub.end(), (size_t)cdiv(d, kHubMarkSlice), (int32_t)hg);
                int64_t ch = cdiv(d, kHubInsChunk);
                int pb = ceil_log2((uint64_t)cdiv(d, kHubBucketTarget));
                if (pb > kHubMaxPBits) pb = kHubMaxPBits;
                hch[hg] = (int32_t)ch;
                hpb[hg] = pb;
                hins[hg] = ins;
                hagg[hg] = agg;
                hins_abs[hg] = (int64_t)ihub.size();
                hagg_abs[hg] = (int64_t)ahub.size();
                hstg[hg] = stg;
                hbk[hg] = bk;
                ihub.insert(ihub.end(), (size_t)ch, (int32_t)hg);
                ahub.insert(ahub.end(), (size_t)1 << pb, (int32_t)hg);
                ins += ch;
                agg += 1LL << pb;
                stg += ch * kHubInsChunk;
                bk += ch << pb;
            }
            cr.sgl_count = (int64_t)shub.size() - cr.sgl_base;
            cr.red_count = (int64_t)rhub.size() - cr.red_base;
            cr.ins_blocks = ins;
            cr.agg_blocks = agg;
            max_stg = stg > max_stg ? stg : max_stg;
            max_bk = bk > max_bk ? bk : max_bk;
            max_ins = ins > max_ins ? ins : max_ins;
            max_agg = agg > max_agg ? agg : max_agg;
        }
        if (H > 0) {
            ensure_hub_capacity(H, max_stg, max_bk, max_ins, max_agg, (int64_t)ihub.size(), (int64_t)ahub.size(),
                                (int64_t)shub.size(), (int64_t)rhub.size());
            HIPCHK(hipMemcpyAsync(hub_pos, hpos.data(), H * 4, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(nchunk, hch.data(), H * 4, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(pbits, hpb.data(), H * 4, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(ins_first, hins.data(), H * 8, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(agg_first, hagg.data(), H * 8, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(stg_off, hstg.data(), H * 8, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(bkt_off, hbk.data(), H * 8, hipMemcpyHostToDevice, st));
            if (!ihub.empty()) HIPCHK(hipMemcpyAsync(ins_hub, ihub.data(), ihub.size() * 4, hipMemcpyHostToDevice, st));
            if (!ahub.empty()) HIPCHK(hipMemcpyAsync(agg_hub, ahub.data(), ahub.size() * 4, hipMemcpyHostToDevice, st));
            if (!shub.empty()) HIPCHK(hipMemcpyAsync(sgl_hub, shub.data(), shub.size() * 4, hipMemcpyHostToDevice, st));
            if (!rhub.empty()) HIPCHK(hipMemcpyAsync(red_hub, rhub.data(), rhub.size() * 4, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(ins_abs, hins_abs.data(), H * 8, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(agg_abs, hagg_abs.data(), H * 8, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(red_abs, hred_abs.data(), H * 8, hipMemcpyHostToDevice, st));
            launch_hub_plans(g, hub_arrays(), l.sig, ins_abs, agg_abs, red_abs, (int64_t)shub.size(),
                             (int64_t)ihub.size(), (int64_t)ahub.size(), (int64_t)rhub.size(), splan, pplan, aplan,
                             rplan, st);
            HIPCHK(hipStreamSynchronize(st));
        }
        sched = true;
        if (opt.timing && events.size() < kEv * (size_t)ncol) {
            size_t old = events.size();
            events.resize(kEv * (size_t)ncol);
            // timing-only events (read after a stream synchronisation): no
            // system-scope fence
            for (size_t i = old; i < events.size(); ++i)
                HIPCHK(hipEventCreateWithFlags(&events[i], hipEventDisableSystemFence));
        }
    }

    MoveState move_state(bool count_cand) {
        MoveState ms;
        ms.zeta = zeta; ms.volC = volC; ms.vol = vol; ms.class_nodes = class_nodes; ms.move_to = move_to;
        ms.rec = noderec;
        if (L().colp) {
            ms.colp = L().colp; ms.zetap = zetap; ms.volCp = volCp; ms.sig = L().sig; ms.ord = L().ord;
        }
        ms.S = S; ms.wide_lim = wide_lim; ms.moves_dev = dcnt; ms.cand_dev = count_cand ? dcnt + 1 : nullptr;
        ms.cand_sgl = count_cand ? dcnt + 13 : nullptr;
        ms.dec_dev = count_cand ? dcnt + 16 : nullptr;
        ms.gp = gp();
        ms.gq = gq();
        if (batch) { ms.gid = L().gid; ms.gS = gS; ms.gwl = gwl; ms.gmoved = bgmoved; }
        if (!lp_mode && sctl) {
            ms.dw = dw; ms.slack = slack; ms.kslack = kslack; ms.tstamp = tstamp; ms.sctl = sctl;
        }
        if (lp_mode) {
            // scores (w(u,X) << 32) + t(u,X): S = 2^32, no vol(u) term, 64-bit
            // while vol(u) (>= every w(u,X)) is below 2^31
            ms.active = active;
            ms.lp_seed = lp_seed;
            ms.lp_level = cur;
            ms.S = (int64_t)1 << 32;
            ms.gp = 0;
            ms.gq = 1;
            ms.wide_lim = INT32_MAX;
        }
        return ms;
    }
    HubArrays hub_arrays() {
        HubArrays ha;
        ha.hub_pos = hub_pos; ha.hub_u = hub_u; ha.sgl_hub = sgl_hub; ha.red_hub = red_hub; ha.ins_hub = ins_hub;
        ha.agg_hub = agg_hub;
        ha.ins_first = ins_first; ha.agg_first = agg_first; ha.nchunk = nchunk;
        ha.pbits = pbits; ha.stg_off = stg_off; ha.bkt_off = bkt_off; ha.stg_x = stg_x; ha.stg_w = stg_w;
        ha.bkt = bkt; ha.wd_part = wd_part; ha.part = part; ha.hub_base = hub_base;
        ha.hub_skip = hub_skip; ha.hub_clk = hub_clk;
        ha.splan = splan; ha.pplan = pplan; ha.aplan = aplan; ha.rplan = rplan;
        ha.agg_max_keys = opt.agg_max_keys > 0 ? opt.agg_max_keys : 0;
        ha.agg_tile = opt.agg_tile > 0 ? opt.agg_tile : 0;
        return ha;
    }

    // ---------------------------------------------------------------- sweeps
    // The class steps of classes [c0, c1) on stream s (decide launches, apply).
    // With aux (kAux streams; branches 1: the partitioned-hub kernels, 2: every
    // kernel group), a class's kernel groups split into branches: after a fork
    // event on s, each branch but the first runs on an aux stream, and the
    // apply waits for all of them through join events.  The decide kernels
    // only read the state the class starts from and write their own class
    // positions, so their order does not matter.
    void launch_classes(int32_t c0, int32_t c1, const MoveState &ms, const HubArrays &ha, const GraphView &g,
                        bool fw, bool timing, unsigned mask, hipStream_t s, const hipStream_t *aux = nullptr,
                        int branches = 0) {
        for (int32_t c = c0; c < c1; ++c) {
            const ClassRange &cr = classes[c];
            const hipEvent_t *ev = timing ? &events[kEv * (size_t)c] : nullptr;
            unsigned part[5];
            int np = 0;
            if (aux) {
                const unsigned present = (cr.count[0] > 0 ? 1u : 0u) | (cr.count[1] > 0 ? 2u : 0u) |
                                         (cr.count[2] > 0 ? 4u : 0u) | (cr.sgl_count > 0 ? 8u : 0u) |
                                         (cr.red_count > 0 ? 16u : 0u);
                if (branches == 2) {
                    for (const unsigned grp : kBranchGroups)
                        if (present & grp) part[np++] = present & grp;
                } else {
                    if (present & 15u) part[np++] = present & 15u;
                    if (present & 16u) part[np++] = 16u;
                }
            }
            if (np >= 2) {
                const int k = c % kForkRing;
                HIPCHK(hipEventRecord(fork_ev[k], s));
                for (int i = 1; i < np; ++i) {
                    HIPCHK(hipStreamWaitEvent(aux[i - 1], fork_ev[k], 0));
                    launch_class_step(g, ms, cr, ha, fw, ev, mask, aux[i - 1], part[i]);
                    HIPCHK(hipEventRecord(join_ev[i - 1][k], aux[i - 1]));
                }
                launch_class_step(g, ms, cr, ha, fw, ev, mask, s, part[0]);
                for (int i = 1; i < np; ++i) HIPCHK(hipStreamWaitEvent(s, join_ev[i - 1][k], 0));
            } else {
                launch_class_step(g, ms, cr, ha, fw, ev, mask, s);
            }
            launch_apply(g, ms, ha, cr, s);
        }
    }
    void ensure_hub_streams() {
        if (hub_cap_st[0]) return;
        for (int a = 0; a < kAux; ++a) HIPCHK(hipStreamCreateWithFlags(&hub_cap_st[a], hipStreamNonBlocking));
        for (int i = 0; i < kForkRing; ++i) {
            HIPCHK(hipEventCreateWithFlags(&fork_ev[i], hipEventDisableTiming));
            for (int a = 0; a < kAux; ++a) HIPCHK(hipEventCreateWithFlags(&join_ev[a][i], hipEventDisableTiming));
        }
    }

    // Captures the launches of a whole sweep into sweep_exec.  Every kernel
    // argument is fixed while the plan lives (build_plan drops the graph), and
    // the counters a sweep reads back are cleared outside the graph.
    void capture_sweep(const MoveState &ms, const HubArrays &ha, const GraphView &g, bool fw) {
        if (!cap_st) HIPCHK(hipStreamCreateWithFlags(&cap_st, hipStreamNonBlocking));
        if (opt.hub_stream) ensure_hub_streams();
        HIPCHK(hipStreamBeginCapture(cap_st, hipStreamCaptureModeRelaxed));
        hipGraph_t gr = nullptr;
        try {
            launch_classes(0, ncol, ms, ha, g, fw, false, 0, cap_st, opt.hub_stream ? hub_cap_st : nullptr,
                           opt.hub_stream);
        } catch (...) {
            (void)hipStreamEndCapture(cap_st, &gr);
            if (gr) (void)hipGraphDestroy(gr);
            throw;
        }
        HIPCHK(hipStreamEndCapture(cap_st, &gr));
        hipError_t e = hipGraphInstantiate(&sweep_exec, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (e != hipSuccess) sweep_exec = nullptr;
        HIPCHK(e);
    }

    // allow_graph: a whole sweep may be replayed from (or captured into) the
    // sweep graph
    int64_t run_classes(int32_t c0, int32_t c1, bool allow_graph = false) {
        if (!sched) build_schedule();
        if (L().colp && layout_dirty) {  // zeta or volC changed outside the apply
            sync_layout(L().n, zeta, volC, L().sig, zetap, volCp, st);
            layout_dirty = false;
        }
        HIPCHK(hipMemsetAsync(dcnt, 0, 5 * 8, st));
        HIPCHK(hipMemsetAsync(dcnt + 13, 0, 8, st));
        HIPCHK(hipMemsetAsync(dcnt + 16, 0, 10 * 8, st));
        bool timing = opt.timing != 0;
        MoveState ms = move_state(timing);
        HubArrays ha = hub_arrays();
        GraphView g = L().view();
        bool fw = opt.int_mode == PLM_INT_128;
        // timing_kernel k in 1..5: only kernel group k - 1
        const int tk = opt.timing_kernel;
        const unsigned mask = tk == 0 ? 0x1fu : (1u << (tk - 1));
        if (allow_graph && opt.graph_sweeps && !timing && c0 == 0 && c1 == ncol && ncol > 0) {
            if (!sweep_exec) capture_sweep(ms, ha, g, fw);
            HIPCHK(hipGraphLaunch(sweep_exec, st));
        } else {
            // one stream: a fork and a join per class cost more than the overlap
            // gains when issued one by one (inside a graph they are edges)
            launch_classes(c0, c1, ms, ha, g, fw, timing, mask, st);
        }
        HIPCHK(hipMemcpyAsync(hbuf, dcnt, 5 * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(hbuf + 5, dcnt + 13, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(hbuf + 32, dcnt + 16, 10 * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        int64_t moves = hbuf[0];
        if (timing && cur < PLM_MAX_LEVELS) {
            // per bin: lane, wavefront, workgroup, hub (one-workgroup + partitioned)
            double bin_t[4] = {0, 0, 0, 0}, sgl_t = 0;
            int64_t launches = 0;
            for (int32_t c = c0; c < c1; ++c) {
                const ClassRange &cr = classes[c];
                const bool ran[5] = {cr.count[0] > 0, cr.count[1] > 0, cr.count[2] > 0, cr.sgl_count > 0,
                                     cr.red_count > 0};
                float t[5] = {0, 0, 0, 0, 0};
                for (int b = 0; b < 5; ++b)
                    if (((mask >> b) & 1u) && ran[b])
                        HIPCHK(hipEventElapsedTime(&t[b], events[kEv * (size_t)c + 2 * b],
                                                   events[kEv * (size_t)c + 2 * b + 1]));
                if (((mask >> 4) & 1u) && ran[4]) {  // + the agg launch
                    float ta = 0;
                    HIPCHK(hipEventElapsedTime(&ta, events[kEv * (size_t)c + 10], events[kEv * (size_t)c + 11]));
                    t[4] += ta;
                }
                for (int b = 0; b < 3; ++b) bin_t[b] += t[b];
                bin_t[3] += t[3] + t[4];
                sgl_t += t[3];
                for (int b = 0; b < 3; ++b) {
                    launches += cr.count[b] > 0 ? 1 : 0;
                    stats.kernel_launches[cur][b] += cr.count[b] > 0 ? 1 : 0;
                }
                launches += (cr.sgl_count > 0 ? 1 : 0) + (cr.red_count > 0 ? 2 : 0);
                stats.kernel_launches[cur][3] += cr.sgl_count > 0 ? 1 : 0;
                stats.kernel_launches[cur][4] += cr.red_count > 0 ? 1 : 0;
            }
            // algorithmic bytes (whole sweeps only): per entry the column, the
            // weight and the community of the neighbour; per distinct candidate
            // its community volume (none in label propagation); per node
            // offsets, own community, vol(u), vol(D) and the class list entry
            int wb = L().wkind == 0 ? 0 : (L().wkind == 1 ? 4 : 8);
            bool whole = c0 == 0 && c1 == ncol;
            const double per_cand = lp_mode ? 0.0 : 8.0;
            // PLM counts the rows actually scanned: a settled node costs its
            // class entry, moved weight, slack, clock stamp and vol(u) (36 bytes)
            const int64_t *dec = hbuf + 32;
            last_ms = last_bytes = 0;
            for (int b = 0; b < 4; ++b) {
                double bytes = 0.0;
                if (whole && lp_mode)
                    bytes = (double)bin_entries[b] * (8.0 + wb) + 32.0 * (double)bin_nodes[b];
                else if (whole)
                    bytes = (double)dec[4 + b] * (8.0 + wb) + per_cand * (double)hbuf[1 + b] + 32.0 * (double)dec[b] +
                            36.0 * (double)(bin_nodes[b] - dec[b]);
                last_ms += bin_t[b];
                last_bytes += bytes;
                if (lp_mode) continue;
                stats.bin_ms[cur][b] += bin_t[b];
                stats.bin_bytes[cur][b] += bytes;
                stats.decide_ms[cur] += bin_t[b];
                stats.decide_bytes[cur] += bytes;
            }
            if (!lp_mode) {
                stats.hub_single_ms[cur] += sgl_t;
                if (whole) {
                    stats.hub_single_bytes[cur] += (double)dec[9] * (8.0 + wb) + 8.0 * (double)hbuf[5] +
                                                   32.0 * (double)dec[8] + 36.0 * (double)(sgl_nodes - dec[8]);
                    for (int b = 0; b < 4; ++b) {
                        stats.decided_nodes[cur] += dec[b];
                        stats.decided_entries[cur] += dec[4 + b];
                        stats.settled_nodes[cur] += bin_nodes[b] - dec[b];
                    }
                }
                stats.decide_launches[cur] += launches;
            }
        }
        return moves;
    }

    // one sweep (with allow_graph, replayed from the graph captured at the
    // plan's first sweep)
    int64_t sweep(bool allow_graph = false) {
        settle_before();
        // every sweep of a plan replays the graph captured at its first sweep
        int64_t mv = run_classes(0, ncol_or_build(), allow_graph);
        ++sweeps;
        if (skip_armed && cur < PLM_MAX_LEVELS) ++stats.settle_sweeps[cur];
        settle_after(mv);
        return mv;
    }
    // before class steps (a sweep, or one class): arm when opt.settle = 1, and
    // re-arm (clock back to 0) before the clock could wrap (at most 2S per
    // sweep; a single class step counts as a sweep here)
    void settle_before() {
        if (!settle_usable()) return;
        const unsigned __int128 next = (unsigned __int128)(armed_sweeps + 1) * 2u * (uint64_t)S;
        if ((!skip_armed && opt.settle == 1) || (skip_armed && (next >> 63))) arm();
    }
    // after them: arm once a sweep moved at most n / kSettleDiv nodes on the
    // input level, n / kSettleDivCoarse on coarse levels (opt.settle = 0)
    void settle_after(int64_t moved) {
        const int64_t div = cur == 0 ? kSettleDiv : kSettleDivCoarse;
        if (skip_armed) ++armed_sweeps;
        else if (settle_usable() && opt.settle == 0 && moved * div <= L().n) arm();
    }

    // Move phase of the current level: sweeps until one moves nothing, at
    // most max_sweeps.  A sweep is a deterministic function of zeta (volumes
    // follow from it; colouring and class order are fixed), so when the state
    // after sweep s equals the state after sweep s - 2, sweeps s + 1, s + 2, ...
    // alternate between the states of sweeps s - 1 and s, moving as many nodes
    // as those did.  The phase then takes the state the last allowed sweep
    // would leave, without running the rest; *skipped receives their number.
    // Returns the moves of all max_sweeps (or fewer) sweeps.
    int64_t move_phase(int64_t *skipped) {
        const int64_t n = L().n;
        *skipped = 0;
        disarm();
        std::vector<int64_t> mv;
        int64_t moves = 0;
        for (int32_t s = 0; s < opt.max_sweeps; ++s) {
            int64_t m = sweep(true);
            mv.push_back(m);
            moves += m;
            if (m == 0) break;
            if (n == 0 || s + 1 == opt.max_sweeps) continue;
            if (!snap[0]) {
                snap[0] = dev_alloc<int32_t>(n0);
                snap[1] = dev_alloc<int32_t>(n0);
            }
            int32_t *prev2 = snap[s & 1];  // state after sweep s - 2
            if (s >= 2 && mv[s] == mv[s - 2]) {
                int32_t *flag = (int32_t *)(dcnt + 14);
                HIPCHK(hipMemsetAsync(flag, 0, 4, st));
                launch_differ(zeta, prev2, n, flag, st);
                HIPCHK(hipMemcpyAsync(hbuf + 16, flag, 4, hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                if (*(int32_t *)(hbuf + 16) == 0) {
                    const int64_t rest = opt.max_sweeps - 1 - s;
                    for (int64_t k = 1; k <= rest; ++k) moves += (k & 1) ? mv[s - 1] : mv[s];
                    if (rest & 1) {  // the last sweep leaves the state of sweep s - 1
                        HIPCHK(hipMemcpyAsync(zeta, snap[(s - 1) & 1], n * 4, hipMemcpyDeviceToDevice, st));
                        launch_comm_vol(zeta, vol, n, volC, st);
                        layout_dirty = true;
                        HIPCHK(hipStreamSynchronize(st));
                    }
                    disarm();  // the recorded slacks belong to the other state
                    sweeps += (int32_t)rest;
                    *skipped = rest;
                    break;
                }
            }
            HIPCHK(hipMemcpyAsync(prev2, zeta, n * 4, hipMemcpyDeviceToDevice, st));  // now the state after sweep s
        }
        return moves;
    }
    int32_t ncol_or_build() {
        if (!sched) build_schedule();
        return ncol;
    }

    // ---------------------------------------------------------------- coarsening
    int64_t coarsen() {
        LevelData &l = L();
        dev_free(l.pi);
        l.pi = dev_alloc<int32_t>(l.n);
        int64_t k = build_relabel(zeta, l.n, l.pi, scr, hbuf, st);
        LevelData nl;
        nl.n = k;
        nl.nnz = build_contraction(l.view(), l.pi, k, &nl.off, &nl.col, (int64_t **)&nl.w, scr, hbuf, st, nullptr,
                                   opt.pack_bits);
        nl.wkind = 2;
        nl.diag_mult = 1;
        // drop any deeper levels left from an earlier run
        while ((int)levels.size() > cur + 1) {
            levels.back().release();
            levels.pop_back();
        }
        levels.push_back(nl);
        ++cur;
        init_level();
        return k;
    }

    void reset() {
        while (levels.size() > 1) {
            levels.back().release();
            levels.pop_back();
        }
        dev_free(levels[0].pi);
        cur = 0;
        std::memset(&stats, 0, sizeof(stats));
        if (batch) set_active_all();
        init_level();
    }
    void set_active_all() {
        act_h.resize(G);
        for (int64_t g = 0; g < G; ++g) act_h[g] = g;
        HIPCHK(hipMemcpyAsync(act, act_h.data(), G * 8, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }

    void record_level(int64_t communities, double t_sched, double t_sweep, double t_coarsen, int64_t moves) {
        if (cur >= PLM_MAX_LEVELS) return;
        stats.levels = cur + 1;
        stats.n[cur] = L().n;
        stats.nnz[cur] = L().nnz;
        stats.loops[cur] = loops;
        stats.colours[cur] = ncol;
        stats.sweeps[cur] = sweeps;
        stats.communities[cur] = communities;
        stats.moves[cur] = moves;
        stats.schedule_ms[cur] = t_sched;
        stats.sweep_ms[cur] = t_sweep;
        for (int b = 0; b < 4; ++b) {
            stats.bin_nodes[cur][b] = bin_nodes[b];
            stats.bin_entries[cur][b] = bin_entries[b];
        }
        stats.hub_single_nodes[cur] = sgl_nodes;
        stats.hub_single_entries[cur] = sgl_entries;
        stats.coarsen_ms[cur] += t_coarsen;
    }

    // Algorithm 3 (Algorithm 4 with opt.refine) from level 0; leaves canonical
    // labels in lab_out (device)
    int32_t run(int32_t *lab_out) {
        reset();
        return descend(lab_out, 0, opt.refine != 0);
    }

    // From the current level `floor` (with its singletons set up): move phases
    // and coarsening until the communities stop merging (max_levels counts
    // from floor); with refine, the move phases after prolongation back down
    // to floor (Algorithm 4); then the communities of the input nodes through
    // the level maps, as canonical labels in lab_out.  Returns the levels.
    int32_t descend(int32_t *lab_out, int floor, bool refine) {
        int32_t done_levels = 0;
        for (;;) {
            double t0 = now_ms();
            build_schedule();
            if (refine) {  // refine_up below reuses it
                LevelData &l = L();
                if (!l.colour_kept && l.n > 0) l.colour_kept = dev_alloc<int32_t>(l.n);
                if (l.n > 0) HIPCHK(hipMemcpyAsync(l.colour_kept, colour, l.n * 4, hipMemcpyDeviceToDevice, st));
                l.ncol_kept = ncol;
            }
            double t1 = now_ms();
            int64_t skipped = 0;
            int64_t moves = move_phase(&skipped);
            if (cur < PLM_MAX_LEVELS) stats.cycle_sweeps[cur] = skipped;
            double t2 = now_ms();
            ++done_levels;
            bool last_allowed = opt.max_levels > 0 && done_levels >= opt.max_levels;
            int64_t k = count_communities(zeta, L().n, scr, hbuf, st);
            if (k == L().n || last_allowed) {
                record_level(k, t1 - t0, t2 - t1, 0, moves);
                break;
            }
            record_level(k, t1 - t0, t2 - t1, 0, moves);
            double t3 = now_ms();
            int prev = cur;
            coarsen();
            if (prev < PLM_MAX_LEVELS) stats.coarsen_ms[prev] = now_ms() - t3;
        }
        if (refine && cur > floor) refine_up(floor);
        // prolong: input node -> current level node -> community
        int64_t n = n0;
        if (n > 0) {
            if (cur == 0) {
                HIPCHK(hipMemcpyAsync(lab, zeta, n * 4, hipMemcpyDeviceToDevice, st));
            } else {
                HIPCHK(hipMemcpyAsync(lab, levels[0].pi, n * 4, hipMemcpyDeviceToDevice, st));
                for (int l = 1; l < cur; ++l) launch_compose(lab, levels[l].pi, n, st);
                launch_compose(lab, zeta, n, st);
            }
            build_canonical(lab, n, lab_out, scr, st);
        }
        return done_levels;
    }

    // PLMR (Algorithm 4), on the way back up: at each level l below the
    // deepest, down to floor, u takes the community of its coarse node pi_l(u)
    // (named by that community's id on level l + 1, which is below n_l), and a
    // move phase (same colouring, same sweep rule) starts from there.  Leaves
    // level floor's communities in zeta.
    void refine_up(int floor) {
        for (int l = cur - 1; l >= floor; --l) {
            double t0 = now_ms();
            const int64_t nl = levels[l].n;
            if (nl > 0) {
                HIPCHK(hipMemcpyAsync(move_to, levels[l].pi, nl * 4, hipMemcpyDeviceToDevice, st));
                launch_compose(move_to, zeta, nl, st);  // move_to[u] = zeta_{l+1}[pi_l[u]]
                HIPCHK(hipMemcpyAsync(zeta, move_to, nl * 4, hipMemcpyDeviceToDevice, st));
            }
            cur = l;
            LevelData &lv = L();
            launch_volumes(lv.view(), vol, dcnt + 5, dcnt + 6, st);
            HIPCHK(hipMemcpyAsync(hbuf, dcnt + 5, 16, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (hbuf[0] != S) throw Error{PLM_E_STATE, "internal: level weight differs during refinement"};
            max_vol = hbuf[1];
            wide_lim = wide_limit(S);
            if (opt.int_mode == PLM_INT_64 && max_vol > wide_lim)
                throw Error{PLM_E_STATE, "int_mode PLM_INT_64: S * vol(u) reaches 2^62 at this level"};
            launch_comm_vol(zeta, vol, nl, volC, st);
            layout_dirty = true;
            sched = false;
            sweeps = 0;
            // the colouring this level had on the way down (kept by descend)
            if (nl > 0) HIPCHK(hipMemcpyAsync(colour, lv.colour_kept, nl * 4, hipMemcpyDeviceToDevice, st));
            ncol = lv.ncol_kept;
            build_plan(nullptr);
            int64_t skipped = 0;
            int64_t moves = move_phase(&skipped);
            if (l < PLM_MAX_LEVELS) {
                stats.ref_cycle_sweeps[l] = skipped;
                stats.ref_sweeps[l] = sweeps;
                stats.ref_moves[l] = moves;
                stats.ref_ms[l] = now_ms() - t0;
            }
        }
    }

    // Label propagation (Algorithm 1) on the current level from singleton
    // labels: colour classes (Jones-Plassmann, whatever opt.schedule says) and
    // tie keys drawn with seed, every node with a
    // non-loop neighbour active at the start, iterations while more than
    // n * 10^-5 labels changed in the last one (at most max_iters).  Leaves the
    // labels (node ids) in zeta; upd (host, may be null) receives the changes
    // per iteration.  Returns the iterations.
    int32_t plp_level(uint64_t seed, int32_t max_iters, int64_t *upd) {
        LevelData &l = L();
        double t0 = now_ms();
        if (!active) active = dev_alloc<uint8_t>(n0 > 0 ? n0 : 1);
        launch_iota(zeta, l.n, st);
        layout_dirty = true;
        // nodes without non-loop neighbours are outside the class buckets, so
        // marking every node active is the same as marking those with one
        if (l.n > 0) HIPCHK(hipMemsetAsync(active, 1, l.n, st));
        build_schedule(seed, PLM_SCHEDULE_COLOUR);  // label propagation always runs on colour classes
        lp_mode = true;
        lp_seed = seed;
        int64_t updated = l.n;
        int32_t it = 0;
        try {
            while (updated * 100000 > l.n && it < max_iters) {
                updated = run_classes(0, ncol, true);
                if (upd) upd[it] = updated;
                if (opt.timing) {
                    stats.lp_decide_ms += last_ms;
                    if (it == 0) {
                        stats.lp_first_ms += last_ms;
                        stats.lp_first_bytes += last_bytes;
                    }
                }
                stats.lp_updates += updated;
                ++it;
            }
        } catch (...) {
            lp_mode = false;
            throw;
        }
        lp_mode = false;
        sched = false;  // the move phase draws its own classes
        stats.lp_runs += 1;
        stats.lp_iterations += it;
        stats.lp_ms += now_ms() - t0;
        return it;
    }

    // EPP(b, PLP, PLMR) (Algorithm 5); defined after create_impl, which it
    // uses for the contexts of its concurrent base runs
    int32_t epp(int32_t b, int32_t plp_iters, int32_t *lab_out, int64_t *cores_out);

    // Modularity of the current level's partition zeta, on the current graph:
    // contraction keeps every intra-community weight (coarse self-loops hold
    // the doubled diagonal) and every community volume, so the two integers of
    // Equation (3.1) equal those of the input nodes' labels
    double modularity_current() {
        __int128 num, den;
        if (modularity_parts(L().view(), vol, zeta, S, scr, hbuf, &num, &den, st) != 0)
            throw Error{PLM_E_STATE, "internal: community id out of range"};
        if (S == 0) return 0.0;
        return (double)num / (double)den;
    }
    double modularity_of(const int32_t *labels_dev) {
        __int128 num, den;
        if (modularity_parts(levels[0].view(), vol0, labels_dev, S, scr, hbuf, &num, &den, st) != 0)
            throw Error{PLM_E_ARG, "labels must lie in [0, n)"};
        if (S == 0) return 0.0;
        return (double)num / (double)den;
    }

    // per graph of a batch level (input graph ids act), the level it joined at;
    // null while every graph of the level started at level 0
    void set_shifts(LevelData &lv, const std::vector<int64_t> &act_ids) {
        dev_free(lv.gshift);
        std::vector<int32_t> sh(act_ids.size());
        bool any = false;
        for (size_t a = 0; a < act_ids.size(); ++a) {
            sh[a] = bshift_h[act_ids[a]];
            any = any || sh[a] != 0;
        }
        if (!any) return;
        lv.gshift = dev_alloc<int32_t>((int64_t)sh.size());
        HIPCHK(hipMemcpyAsync(lv.gshift, sh.data(), sh.size() * 4, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }

    // The graphs that finished at this level, one by one over their own input
    // node range: canonical labels (first occurrence) and modularity from
    // their local labels in bout; reported through hooks->done.
    void report_finished(BatchHooks *hooks, const std::vector<int64_t> &fin, const std::vector<int32_t> &glev) {
        const GraphView g0 = levels[0].view();
        if (!bcanon) bcanon = dev_alloc<int32_t>(n0);
        std::vector<int64_t> Sg(G);
        HIPCHK(hipMemcpyAsync(Sg.data(), gS0, G * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        unsigned long long *acc = dcnt + 26;
        for (int64_t g : fin) {
            const int64_t a = gbase0_h[g], n = gbase0_h[g + 1] - a;
            if (n > 0) build_canonical(bout + a, n, bcanon + a, scr, st);
            graph_modularity_parts(g0, a, n, bout + a, vol0, bnewid + a, acc, st);
            HIPCHK(hipMemcpyAsync(hbuf + 40, acc, 3 * 8, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            double q = 0.0;
            if (Sg[g] != 0) {
                unsigned __int128 s2 = ((unsigned __int128)(uint64_t)hbuf[42] << 64) | (uint64_t)hbuf[41];
                __int128 num = (__int128)Sg[g] * (__int128)hbuf[40] - (__int128)s2;
                __int128 den = (__int128)Sg[g] * (__int128)Sg[g];
                q = (double)num / (double)den;
            }
            hooks->done(g, bcanon + a, n, q, glev[g]);
        }
    }

    // reallocates a device array for new_n elements, keeping its first keep
    template <typename T>
    void regrow(T *&p, int64_t new_n, int64_t keep) {
        T *q = dev_alloc<T>(new_n);
        if (p && keep > 0) HIPCHK(hipMemcpyAsync(q, p, (size_t)keep * sizeof(T), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        dev_free(p);
        p = q;
    }

    // Continuous batching: graphs join the batch at the level boundary just
    // set up (cur >= 1), each at level 0 of its own.  Its input CSR is
    // validated and appended to the input union (levels[0]); converted to the
    // coarse format (int64 weights, self-loops doubled) it is appended to the
    // current level, whose per-graph level shift for it is cur, so that its
    // priorities hash its own level and it stops after its own max_levels.
    // codes/msgs: per offered graph 0 or the reason it was refused.
    void batch_append(const std::vector<JoinGraph> &js, std::vector<int> &codes, std::vector<std::string> &msgs) {
        struct Tmp {
            int64_t n = 0, nnz = 0, S = 0;
            int64_t *off = nullptr, *vol = nullptr;
            int32_t *col = nullptr, *w = nullptr;
        };
        std::vector<Tmp> ok;
        codes.assign(js.size(), PLM_OK);
        msgs.assign(js.size(), std::string());
        auto free_tmp = [&](Tmp &t) { dev_free(t.off); dev_free(t.vol); dev_free(t.col); dev_free(t.w); };
        int64_t addS = 0, addN = 0;
        try {
            for (size_t i = 0; i < js.size(); ++i) {
                const JoinGraph &j = js[i];
                Tmp t;
                t.n = j.n;
                t.nnz = j.nnz;
                t.off = dev_alloc<int64_t>(j.n + 1);
                t.col = dev_alloc<int32_t>(j.nnz);
                if (j.w) t.w = dev_alloc<int32_t>(j.nnz);
                t.vol = dev_alloc<int64_t>(j.n);
                const hipMemcpyKind kind = j.mem_kind == PLM_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
                HIPCHK(hipMemcpyAsync(t.off, j.off, (size_t)(j.n + 1) * 8, kind, st));
                if (j.nnz > 0) HIPCHK(hipMemcpyAsync(t.col, j.col, (size_t)j.nnz * 4, kind, st));
                if (j.w && j.nnz > 0) HIPCHK(hipMemcpyAsync(t.w, j.w, (size_t)j.nnz * 4, kind, st));
                GraphView v;
                v.n = t.n; v.nnz = t.nnz; v.off = t.off; v.col = t.col; v.w = t.w; v.wkind = t.w ? 1 : 0;
                v.diag_mult = 2;
                uint32_t bad = opt.validate ? validate_graph(v, scr, hbuf, st) : 0u;
                if (!bad) {
                    launch_volumes(v, t.vol, dcnt + 5, dcnt + 6, st);
                    HIPCHK(hipMemcpyAsync(hbuf, dcnt + 5, 8, hipMemcpyDeviceToHost, st));
                    HIPCHK(hipStreamSynchronize(st));
                    t.S = hbuf[0];
                }
                if (bad) {
                    codes[i] = PLM_E_GRAPH;
                    msgs[i] = "invalid graph";
                } else if ((unsigned __int128)(uint64_t)S + (uint64_t)addS + (uint64_t)t.S >= ((unsigned __int128)1 << 62)) {
                    codes[i] = PLM_E_BUDGET;
                    msgs[i] = "the batch's total weight would reach 2^62";
                } else if (n0 + addN + t.n >= (1LL << 31)) {
                    codes[i] = PLM_E_BUDGET;
                    msgs[i] = "the batch would exceed 2^31 nodes";
                }
                if (codes[i] != PLM_OK) {
                    free_tmp(t);
                    continue;
                }
                addS += t.S;
                addN += t.n;
                ok.push_back(t);
            }
            if (ok.empty()) return;
            const int64_t J = (int64_t)ok.size();
            int64_t nA = 0, eA = 0;
            bool weighted = levels[0].wkind == 1;
            for (auto &t : ok) {
                nA += t.n;
                eA += t.nnz;
                weighted = weighted || t.w != nullptr;
            }
            LevelData &b0 = levels[0];
            const int64_t n0o = n0, e0o = b0.nnz, Go = G;
            const int64_t n1 = n0o + nA, e1 = e0o + eA, G1 = Go + J;
            // ---- the input union
            regrow(b0.off, n1 + 1, n0o + 1);
            regrow(b0.col, e1, e0o);
            if (weighted) {
                if (b0.wkind == 1) {
                    int32_t *w0 = (int32_t *)b0.w;
                    regrow(w0, e1, e0o);
                    b0.w = w0;
                } else {
                    int32_t *w0 = dev_alloc<int32_t>(e1);
                    launch_fill_i32(w0, e0o, 1, st);
                    b0.w = w0;
                    b0.wkind = 1;
                }
            }
            int64_t nb = n0o, eb = e0o;
            for (auto &t : ok) {
                launch_append_off(b0.off + nb, t.off, t.n, eb, st);
                launch_append_input(b0.col + eb, weighted ? (int32_t *)b0.w + eb : nullptr, t.col, t.w, t.nnz, nb, st);
                gbase0_h.push_back(nb + t.n);
                nb += t.n;
                eb += t.nnz;
            }
            b0.n = n1;
            b0.nnz = e1;
            regrow(b0.gbase, G1 + 1, 0);
            HIPCHK(hipMemcpyAsync(b0.gbase, gbase0_h.data(), (G1 + 1) * 8, hipMemcpyHostToDevice, st));
            regrow(b0.gid, n1, 0);
            launch_fill_gid(b0.gbase, G1, n1, b0.gid, st);
            // ---- per input node and per input graph
            regrow(vol0, n1, n0o);
            regrow(lab, n1, n0o);
            regrow(bout, n1, n0o);
            launch_fill_i32(bout + n0o, nA, 0, st);
            nb = n0o;
            for (auto &t : ok) {
                if (t.n > 0) HIPCHK(hipMemcpyAsync(vol0 + nb, t.vol, t.n * 8, hipMemcpyDeviceToDevice, st));
                nb += t.n;
            }
            regrow(gS0, G1, Go);
            regrow(gwl0, G1, Go);
            {
                std::vector<int64_t> s(J), wl(J);
                for (int64_t k = 0; k < J; ++k) {
                    s[k] = ok[k].S;
                    unsigned __int128 sg = (unsigned __int128)(uint64_t)s[k] * (unsigned __int128)(uint64_t)gmax();
                    wl[k] = sg == 0 ? INT64_MAX : ((sg >> 62) ? 0 : (int64_t)(((1ULL << 62) - 1) / (uint64_t)sg));
                }
                HIPCHK(hipMemcpyAsync(gS0 + Go, s.data(), J * 8, hipMemcpyHostToDevice, st));
                HIPCHK(hipMemcpyAsync(gwl0 + Go, wl.data(), J * 8, hipMemcpyHostToDevice, st));
            }
            regrow(vol, n1, 0);
            regrow(volC, n1, 0);
            regrow(zeta, n1, 0);
            regrow(colour, n1, 0);
            regrow(class_nodes, n1, 0);
            regrow(noderec, n1, 0);
            regrow(move_to, n1, 0);
            regrow(bflag, n1, 0);
            regrow(bnewid, n1 + 1, 0);
            dev_free(bscan);
            bscan = dev_alloc<uint8_t>((int64_t)scan_scratch_bytes(n1 > 0 ? n1 : 1));
            dev_free(bcanon);
            regrow(act, G1, 0);
            regrow(gS, G1, 0);
            regrow(gwl, G1, 0);
            regrow(bstatus, G1, 0);
            regrow(bkeep, G1, 0);
            regrow(bsweep, G1, 0);
            regrow(bI2, G1, 0);
            regrow(bsq, 2 * G1, 0);
            regrow(bgmoved, G1, 0);
            regrow(bgath, 2 * (G1 + 1), 0);
            // ---- the current level
            LevelData &l = L();
            const int64_t nc = l.n, ec = l.nnz, A = (int64_t)act_h.size();
            std::vector<int64_t> lb(A + 1);
            HIPCHK(hipMemcpyAsync(lb.data(), l.gbase, (A + 1) * 8, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            regrow(l.off, nc + nA + 1, nc + 1);
            regrow(l.col, ec + eA, ec);
            int64_t *lw = (int64_t *)l.w;
            regrow(lw, ec + eA, ec);
            l.w = lw;
            // nodes of the new graphs at this level: right after the level's own
            nb = nc;
            eb = ec;
            int64_t ib = n0o;
            for (int64_t k = 0; k < J; ++k) {
                Tmp &t = ok[k];
                launch_append_off(l.off + nb, t.off, t.n, eb, st);
                launch_append_coarse(l.col + eb, lw + eb, t.off, t.n, t.col, t.w, t.nnz, nb, st);
                launch_iota_from(lab + ib, t.n, nb, st);  // input node -> its node at this level
                nb += t.n;
                eb += t.nnz;
                ib += t.n;
                lb.push_back(nb);
                act_h.push_back(Go + k);
                bshift_h.push_back(cur);
            }
            l.n = nc + nA;
            l.nnz = ec + eA;
            regrow(l.gbase, A + J + 1, 0);
            HIPCHK(hipMemcpyAsync(l.gbase, lb.data(), (A + J + 1) * 8, hipMemcpyHostToDevice, st));
            regrow(l.gid, l.n, 0);
            launch_fill_gid(l.gbase, A + J, l.n, l.gid, st);
            HIPCHK(hipMemcpyAsync(act, act_h.data(), (A + J) * 8, hipMemcpyHostToDevice, st));
            set_shifts(l, act_h);
            n0 = n1;
            G = G1;
            S += addS;
            for (auto &t : ok) free_tmp(t);
            ok.clear();
            init_level();  // volumes, graph weights, singletons of the grown level
        } catch (...) {
            for (auto &t : ok) free_tmp(t);
            throw;
        }
    }

    // Algorithm 3 on every graph of a batch at once.  All graphs still active
    // are at the same level; a graph whose communities stop merging (or that
    // reached max_levels) gets its labels at that level and leaves the next.
    // Results per graph equal those of a separate run: priorities, gains and
    // coarse ids are all local to each graph, and once a graph's sweep makes
    // no move, further sweeps of the batch leave it unchanged.
    // canon_out (device, n0): labels canonical within each graph.
    // With hooks (request server): at every level boundary graphs may join,
    // each starting at level 0 of its own (batch_append), and every graph is
    // reported through hooks->done at the level it finishes; canon_out, q_out
    // and levels_out are then unused.
    void run_batch(int32_t *canon_out, double *q_out, int32_t *levels_out, BatchHooks *hooks = nullptr) {
        reset();
        bshift_h.assign(G, 0);
        int64_t n0v = n0;
        if (hooks && n0v > 0) launch_fill_i32(bout, n0v, 0, st);  // keys of unfinished graphs stay in range
        std::vector<uint8_t> status(G, 0), keep;
        std::vector<int64_t> gath, nbase, nact;
        std::vector<int32_t> glev(G, 0);
        launch_iota(lab, n0v, st);
        std::vector<int32_t> gmoved;
        std::vector<uint8_t> sweeping;
        std::vector<int64_t> ebound;
        for (int32_t depth = 1;; ++depth) {
            double t0 = now_ms();
            build_schedule();
            double t1 = now_ms();
            LevelData &l = L();
            int64_t A = (int64_t)act_h.size();
            // entries of each graph of the level (row ranges are contiguous)
            ebound.resize(A + 1);
            launch_gather_i64(l.off, l.gbase, A + 1, bgath, st);
            HIPCHK(hipMemcpyAsync(ebound.data(), bgath, (A + 1) * 8, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemsetAsync(bgmoved, 0, A * 4, st));
            HIPCHK(hipStreamSynchronize(st));
            sweeping.assign(A, 1);
            int64_t planned = ebound[A] - ebound[0];
            int64_t moves = 0;
            for (int32_t s = 0; s < opt.max_sweeps; ++s) {
                int64_t mv = sweep(true);
                moves += mv;
                if (mv == 0) break;
                // a graph whose sweep moved nothing is done at this level (a
                // further sweep would repeat the same decisions): its nodes
                // leave the class buckets once the live entries have shrunk
                gmoved.resize(A);
                HIPCHK(hipMemcpyAsync(gmoved.data(), bgmoved, A * 4, hipMemcpyDeviceToHost, st));
                HIPCHK(hipMemsetAsync(bgmoved, 0, A * 4, st));
                HIPCHK(hipStreamSynchronize(st));
                int64_t live = 0;
                for (int64_t a = 0; a < A; ++a) {
                    if (!gmoved[a]) sweeping[a] = 0;
                    if (sweeping[a]) live += ebound[a + 1] - ebound[a];
                }
                if (s + 1 < opt.max_sweeps && (double)live < kReplanFraction * (double)planned) {
                    HIPCHK(hipMemcpyAsync(bsweep, sweeping.data(), A, hipMemcpyHostToDevice, st));
                    build_plan(bsweep);
                    planned = live;
                }
            }
            double t2 = now_ms();
            // communities of each graph: ranks of community ids at the graph bounds
            batch_relabel(zeta, l.n, l.gid, nullptr, bflag, bnewid, nullptr, bscan, st);
            launch_gather_i64(bnewid, l.gbase, A + 1, bgath, st);
            gath.resize(A + 1);
            HIPCHK(hipMemcpyAsync(gath.data(), bgath, (A + 1) * 8, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            const int64_t *nid = gath.data();
            std::vector<int64_t> abase(A + 1);
            HIPCHK(hipMemcpyAsync(abase.data(), l.gbase, (A + 1) * 8, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            keep.assign(A, 0);
            nbase.assign(1, 0);
            nact.clear();
            std::vector<int64_t> finished;
            for (int64_t a = 0; a < A; ++a) {
                int64_t ka = nid[a + 1] - nid[a], na = abase[a + 1] - abase[a];
                int64_t g = act_h[a];
                glev[g] = depth - bshift_h[g];  // levels of g's own run so far
                const bool last = opt.max_levels > 0 && glev[g] >= opt.max_levels;
                if (ka == na || last) {
                    finished.push_back(g);
                    status[g] = 1;
                } else {
                    status[g] = 0;
                    keep[a] = 1;
                    nact.push_back(g);
                    nbase.push_back(nbase.back() + ka);
                }
            }
            record_level(nid[A] - nid[0], t1 - t0, t2 - t1, 0, moves);
            double t3 = now_ms();
            HIPCHK(hipMemcpyAsync(bstatus, status.data(), G, hipMemcpyHostToDevice, st));
            if (A > 0) HIPCHK(hipMemcpyAsync(bkeep, keep.data(), A, hipMemcpyHostToDevice, st));
            int64_t A2 = (int64_t)nact.size();
            if (A2 > 0) {
                dev_free(l.pi);
                l.pi = dev_alloc<int32_t>(l.n);
                batch_relabel(zeta, l.n, l.gid, bkeep, bflag, bnewid, l.pi, bscan, st);
            }
            launch_batch_step(n0v, levels[0].gid, bstatus, l.gid, l.gbase, zeta, l.pi, lab, bout, st);
            HIPCHK(hipStreamSynchronize(st));
            if (hooks && !finished.empty()) report_finished(hooks, finished, glev);
            for (int64_t a = 0; a < A; ++a)
                if (!keep[a]) status[act_h[a]] = 2;
            if (A2 == 0) break;
            int64_t k = nbase.back();
            LevelData nl;
            nl.n = k;
            try {
                nl.nnz = build_contraction(l.view(), l.pi, k, &nl.off, &nl.col, (int64_t **)&nl.w, scr, hbuf, st, bkeep,
                                           opt.pack_bits);
                nl.wkind = 2;
                nl.diag_mult = 1;
                nl.gbase = dev_alloc<int64_t>(A2 + 1);
                nl.gid = dev_alloc<int32_t>(k);
                HIPCHK(hipMemcpyAsync(nl.gbase, nbase.data(), (A2 + 1) * 8, hipMemcpyHostToDevice, st));
                launch_fill_gid(nl.gbase, A2, k, nl.gid, st);
                set_shifts(nl, nact);
                act_h = nact;
                HIPCHK(hipMemcpyAsync(act, act_h.data(), A2 * 8, hipMemcpyHostToDevice, st));
                HIPCHK(hipStreamSynchronize(st));
            } catch (...) {
                nl.release();
                throw;
            }
            while ((int)levels.size() > cur + 1) {
                levels.back().release();
                levels.pop_back();
            }
            levels.push_back(nl);
            int prev = cur++;
            init_level();
            if (prev < PLM_MAX_LEVELS) stats.coarsen_ms[prev] = now_ms() - t3;
            if (hooks && depth <= opt.join) {  // joins at the first opt.join level boundaries
                std::vector<JoinGraph> js = hooks->join();
                if (!js.empty()) {
                    std::vector<int> codes;
                    std::vector<std::string> msgs;
                    batch_append(js, codes, msgs);
                    status.resize(G, 0);
                    glev.resize(G, 0);
                    n0v = n0;
                    hooks->joined(codes, msgs);
                }
            }
        }
        if (hooks) return;
        // labels canonical within each graph; per-graph modularity on the input
        const GraphView g0 = levels[0].view();
        if (n0v > 0) batch_canonical(n0v, g0.gid, g0.gbase, bout, bflag, move_to, canon_out, scr, st);
        if (q_out) {
            // keys (bflag) = first input node of the graph + local label
            batch_modularity_parts(g0, g0.gid, bflag, vol0, G, bnewid, bI2, bsq, st);
            std::vector<uint64_t> I2(G), sq(2 * G);
            std::vector<int64_t> Sg(G);
            HIPCHK(hipMemcpyAsync(I2.data(), bI2, G * 8, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(sq.data(), bsq, G * 16, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(Sg.data(), gS0, G * 8, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int64_t g = 0; g < G; ++g) {
                if (Sg[g] == 0) { q_out[g] = 0.0; continue; }
                unsigned __int128 s2 = ((unsigned __int128)sq[2 * g + 1] << 64) | sq[2 * g];
                __int128 num = (__int128)Sg[g] * (__int128)(int64_t)I2[g] - (__int128)s2;
                __int128 den = (__int128)Sg[g] * (__int128)Sg[g];
                q_out[g] = (double)num / (double)den;
            }
        }
        if (levels_out)
            for (int64_t g = 0; g < G; ++g) levels_out[g] = glev[g];
    }
};

// ------------------------------------------------------------------ C ABI
namespace {

const char *const kBinsMsg =
    "bins must satisfy 1 <= bin_lane <= 16, bin_lane <= bin_wave <= 512, bin_wave <= bin_block <= 4096 (0: tuned)";

int check_options(const plm_options &o, std::string &msg) {
    if (o.max_sweeps < 1) { msg = "max_sweeps must be >= 1"; return PLM_E_ARG; }
    if (o.max_levels < 0) { msg = "max_levels must be >= 0"; return PLM_E_ARG; }
    if (o.schedule != PLM_SCHEDULE_COLOUR && o.schedule != PLM_SCHEDULE_SEQUENTIAL) { msg = "bad schedule"; return PLM_E_ARG; }
    if (o.int_mode < 0 || o.int_mode > 2) { msg = "bad int_mode"; return PLM_E_ARG; }
    if (o.timing_kernel < 0 || o.timing_kernel > 5) { msg = "timing_kernel must lie in [0, 5]"; return PLM_E_ARG; }
    if (o.refine != 0 && o.refine != 1) { msg = "refine must be 0 or 1"; return PLM_E_ARG; }
    if (o.graph_sweeps != 0 && o.graph_sweeps != 1) { msg = "graph_sweeps must be 0 or 1"; return PLM_E_ARG; }
    if (o.hub_stream < 0 || o.hub_stream > 2) { msg = "hub_stream must be 0, 1 or 2"; return PLM_E_ARG; }
    if (o.colour_tail != 0 && o.colour_tail != 1) { msg = "colour_tail must be 0 or 1"; return PLM_E_ARG; }
    if (o.hub_row_max < 0 || o.hub_row_max > kSingleMaxRow) {
        msg = "hub_row_max must be 0 or lie in [1, 12288]";
        return PLM_E_ARG;
    }
    if (o.agg_max_keys != 0 && (o.agg_max_keys < 32 || o.agg_max_keys > 1536)) {
        msg = "agg_max_keys must be 0 or lie in [32, 1536]";
        return PLM_E_ARG;
    }
    if (o.agg_tile < 0 || o.agg_tile > 512) { msg = "agg_tile must be 0 or lie in [1, 512]"; return PLM_E_ARG; }
    if (o.settle < -1 || o.settle > 1) { msg = "settle must be -1, 0 or 1"; return PLM_E_ARG; }
    if (o.join < 0) { msg = "join must be >= 0"; return PLM_E_ARG; }
    if (o.layout < -1 || o.layout > 1) { msg = "layout must be -1, 0 or 1"; return PLM_E_ARG; }
    if (o.pack_bits < -1 || o.pack_bits == 1 || o.pack_bits > 62) {
        msg = "pack_bits must be -1, 0 or lie in [2, 62]";
        return PLM_E_ARG;
    }
    if (!(o.gamma_num == 0 && o.gamma_den == 0) &&
        (o.gamma_num < 0 || o.gamma_den < 1 || o.gamma_num >= 65536 || o.gamma_den >= 65536)) {
        msg = "gamma must satisfy 0 <= gamma_num < 2^16, 1 <= gamma_den < 2^16";
        return PLM_E_ARG;
    }
    // each bin in range here; their order once the zeros are filled (check_bins)
    if (o.bin_lane < 0 || o.bin_wave < 0 || o.bin_block < 0 || o.bin_lane > 16 || o.bin_wave > 512 ||
        o.bin_block > 4096) {
        msg = kBinsMsg;
        return PLM_E_ARG;
    }
    return PLM_OK;
}

int check_bins(const plm_options &o, std::string &msg) {
    if (o.bin_lane > o.bin_wave || o.bin_wave > o.bin_block) {
        msg = kBinsMsg;
        return PLM_E_ARG;
    }
    return PLM_OK;
}

template <typename F>
plm_status guarded(plm_ctx *ctx, F f) {
    if (!ctx) return PLM_E_ARG;
    try {
        ctx->err.clear();
        f();
        return PLM_OK;
    } catch (const Error &e) {
        ctx->err = e.msg;
        return e.code;
    } catch (const std::exception &e) {
        ctx->err = e.what();
        return PLM_E_NOMEM;
    }
}

void copy_in(void *dst, const void *src, size_t bytes, int mem_kind, hipStream_t st) {
    if (bytes == 0) return;
    HIPCHK(hipMemcpyAsync(dst, src, bytes, mem_kind == PLM_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          st));
}
void copy_out(void *dst, const void *src, size_t bytes, int mem_kind, hipStream_t st) {
    if (bytes == 0) return;
    HIPCHK(hipMemcpyAsync(dst, src, bytes, mem_kind == PLM_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          st));
}

// Address of the current device's static workspace, looked up once per device
// (with that device current) at context creation.
void *noalloc_workspace() {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocDevices) throw Error{PLM_E_DEVICE, "device index beyond the workspace table"};
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            throw Error{PLM_E_DEVICE, std::string("hipGetSymbolAddress of the static workspace failed: ") +
                                          hipGetErrorString(e)};
        }
        g_noalloc_ptr[dev] = p;
    }
    return g_noalloc_ptr[dev];
}

}  // namespace

extern "C" {

void plm_default_options(plm_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->max_sweeps = 32;
    o->max_levels = 0;
    o->schedule = PLM_SCHEDULE_COLOUR;
    o->validate = 1;
    o->colour_seed = 0;
    o->int_mode = PLM_INT_AUTO;
    o->bin_lane = 0;  // 0: the tuned table's value, else the compiled default
    o->bin_wave = 0;
    o->bin_block = 0;
    o->hub_row_max = 0;
    o->timing = 0;
    o->gamma_num = 1;
    o->gamma_den = 1;
    o->graph_sweeps = 1;
    o->hub_stream = 2;
    o->colour_tail = 1;
}

}  // extern "C"

namespace {

// ---------------------------------------------------------------- tuned bins
// Degree-bin thresholds and the one-workgroup hub limit left at 0 come from
// the table the tuner (tune.py) writes beside the library, tuned_bins.txt
// (PLM_TUNED_TABLE names another file): rows "kind max_nnz bin_lane bin_wave
// bin_block hub_row_max", kind batch or single, max_nnz 0 = any size; the
// first row of the context's kind whose max_nnz covers its entries applies.
// Without a table or a matching row, the compiled defaults 16 / 512 / 4096 /
// 12288 apply.  Rows outside the valid ranges are ignored.
struct TunedRow {
    bool batch;
    int64_t max_nnz;
    int32_t lane, wave, block, hub_max;
};
std::vector<TunedRow> g_tuned;
std::string g_tuned_source;
std::once_flag g_tuned_once;

bool bins_valid(int64_t a, int64_t b, int64_t c, int64_t h) {
    return a >= 1 && b >= 1 && c >= 1 && h >= 1 && a <= 16 && b <= 512 && c <= 4096 && a <= b && b <= c &&
           h <= kSingleMaxRow;
}

void load_tuned() {
    std::string path;
    if (const char *e = std::getenv("PLM_TUNED_TABLE")) {
        path = e;
    } else {
        Dl_info info;
        if (dladdr((void *)&load_tuned, &info) && info.dli_fname) {
            std::string so = info.dli_fname;
            size_t k = so.rfind('/');
            path = (k == std::string::npos ? std::string(".") : so.substr(0, k)) + "/tuned_bins.txt";
        }
    }
    std::ifstream f(path);
    if (!f) return;
    std::string line;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream is(line);
        std::string kind;
        TunedRow r;
        if (!(is >> kind >> r.max_nnz >> r.lane >> r.wave >> r.block >> r.hub_max)) continue;
        if (kind != "batch" && kind != "single") continue;
        if (r.max_nnz < 0 || !bins_valid(r.lane, r.wave, r.block, r.hub_max)) continue;
        r.batch = kind == "batch";
        g_tuned.push_back(r);
    }
    if (!g_tuned.empty()) g_tuned_source = path;
}

// Fills the bin thresholds of o left at 0: from the tuned table's row for
// (batch, nnz), else the compiled defaults.  A mix with the caller's own
// values that breaks the bin order falls back to the compiled defaults for
// the zero fields.
void resolve_bins(plm_options &o, bool batch, int64_t nnz) {
    if (o.bin_lane > 0 && o.bin_wave > 0 && o.bin_block > 0 && o.hub_row_max > 0) return;
    std::call_once(g_tuned_once, load_tuned);
    const TunedRow *row = nullptr;
    for (const TunedRow &r : g_tuned)
        if (r.batch == batch && (r.max_nnz == 0 || nnz <= r.max_nnz)) { row = &r; break; }
    const int32_t dl = 16, dw = 512, db = 4096, dh = (int32_t)kSingleMaxRow;
    plm_options t = o;
    if (t.bin_lane <= 0) t.bin_lane = row ? row->lane : dl;
    if (t.bin_wave <= 0) t.bin_wave = row ? row->wave : dw;
    if (t.bin_block <= 0) t.bin_block = row ? row->block : db;
    if (t.hub_row_max <= 0) t.hub_row_max = row ? row->hub_max : dh;
    if (!bins_valid(t.bin_lane, t.bin_wave, t.bin_block, t.hub_row_max)) {
        t = o;
        if (t.bin_lane <= 0) t.bin_lane = dl;
        if (t.bin_wave <= 0) t.bin_wave = dw;
        if (t.bin_block <= 0) t.bin_block = db;
        if (t.hub_row_max <= 0) t.hub_row_max = dh;
    }
    o = t;
}

// Shared by plm_create (G = 0) and plm_batch_create (G >= 1 graphs on the node
// ranges node_base[0..G]).
// adopt: offsets/cols/weights are device buffers from hipMalloc that the new
// context takes over (freed with it, also when creation fails) instead of copying
plm_status create_impl(plm_ctx **out, int64_t G, const int64_t *node_base, int64_t n, int64_t nnz,
                       const int64_t *offsets, const int32_t *cols, const int32_t *weights, int32_t mem_kind,
                       void *hip_stream, const plm_options *opt, bool adopt = false, bool borrow = false) {
    g_create_error.clear();
    if (out) *out = nullptr;
    auto fail = [&](int code, const std::string &m) {
        g_create_error = m;
        return code;
    };
    // adopted buffers not yet handed to a level are freed on every error path
    auto release_adopted = [&]() {
        if (!adopt) return;
        adopt = false;
        (void)hipFree(const_cast<int64_t *>(offsets));
        (void)hipFree(const_cast<int32_t *>(cols));
        if (weights) (void)hipFree(const_cast<int32_t *>(weights));
    };
    auto fail_adopt = [&](int code, const std::string &m) {
        release_adopted();
        return fail(code, m);
    };
    if (!out) return fail_adopt(PLM_E_ARG, "out is NULL");
    if (n < 0 || n >= (1LL << 31)) return fail_adopt(PLM_E_ARG, "n must lie in [0, 2^31)");
    if (nnz < 0 || nnz >= (1LL << 40)) return fail_adopt(PLM_E_ARG, "nnz must lie in [0, 2^40)");
    if (!offsets) return fail_adopt(PLM_E_ARG, "offsets is NULL");
    if (nnz > 0 && !cols) return fail_adopt(PLM_E_ARG, "cols is NULL");
    if (mem_kind != PLM_MEM_HOST && mem_kind != PLM_MEM_DEVICE) return fail_adopt(PLM_E_ARG, "bad mem_kind");
    plm_options o;
    plm_default_options(&o);
    if (opt) o = *opt;
    std::string m;
    int rc = check_options(o, m);
    if (rc) return fail_adopt(rc, m);
    if (o.gamma_num == 0 && o.gamma_den == 0) o.gamma_num = o.gamma_den = 1;
    resolve_bins(o, G > 0, nnz);
    rc = check_bins(o, m);
    if (rc) return fail_adopt(rc, m);
    if (G > 0) {
        if (o.refine) return fail_adopt(PLM_E_ARG, "batched runs do not refine");
        if (o.schedule != PLM_SCHEDULE_COLOUR) return fail_adopt(PLM_E_ARG, "batched runs use the colour schedule");
        if (o.int_mode == PLM_INT_64) return fail_adopt(PLM_E_ARG, "batched runs take int_mode auto or 128");
        if (node_base[0] != 0) return fail_adopt(PLM_E_ARG, "node_base[0] must be 0");
        for (int64_t g = 0; g < G; ++g)
            if (node_base[g + 1] < node_base[g]) return fail_adopt(PLM_E_ARG, "node_base must be non-decreasing");
    }
    if (mem_kind == PLM_MEM_HOST) {
        if (offsets[0] != 0 || offsets[n] != nnz) return fail_adopt(PLM_E_GRAPH, "offsets[0] must be 0 and offsets[n] = nnz");
    }
    plm_ctx *c = nullptr;
    try {
        c = new plm_ctx();
        std::memset(&c->stats, 0, sizeof(c->stats));
        c->st = (hipStream_t)hip_stream;
        c->scr.set_stream(c->st);
        c->opt = o;
        c->mem_kind = mem_kind;
        c->n0 = n;
        HIPCHK(hipHostMalloc((void **)&c->hbuf, kHostWords * sizeof(int64_t), hipHostMallocDefault));
        c->noalloc_ws = noalloc_workspace();
        LevelData l0;
        l0.n = n;
        l0.nnz = nnz;
        l0.wkind = weights ? 1 : 0;
        l0.diag_mult = 2;
        if (adopt || borrow) {
            l0.off = const_cast<int64_t *>(offsets);
            l0.col = const_cast<int32_t *>(cols);
            l0.w = const_cast<int32_t *>(weights);
            l0.borrowed = borrow;
            adopt = false;  // owned by the level from here on (or by the lender)
            c->levels.push_back(l0);
        } else {
            l0.off = dev_alloc<int64_t>(n + 1);
            l0.col = dev_alloc<int32_t>(nnz);
            if (weights) l0.w = dev_alloc<int32_t>(nnz);
            c->levels.push_back(l0);
            copy_in(l0.off, offsets, (size_t)(n + 1) * 8, mem_kind, c->st);
            copy_in(l0.col, cols, (size_t)nnz * 4, mem_kind, c->st);
            if (weights) copy_in(l0.w, weights, (size_t)nnz * 4, mem_kind, c->st);
        }
        HIPCHK(hipStreamSynchronize(c->st));
        if (G > 0) {
            c->batch = true;
            c->G = G;
            c->gbase0_h.assign(node_base, node_base + G + 1);
            LevelData &b0 = c->levels[0];
            b0.gbase = dev_alloc<int64_t>(G + 1);
            b0.gid = dev_alloc<int32_t>(n);
            HIPCHK(hipMemcpyAsync(b0.gbase, node_base, (G + 1) * 8, hipMemcpyHostToDevice, c->st));
            launch_fill_gid(b0.gbase, G, n, b0.gid, c->st);
            c->gS0 = dev_alloc<int64_t>(G); c->gwl0 = dev_alloc<int64_t>(G);
            c->act = dev_alloc<int64_t>(G); c->gS = dev_alloc<int64_t>(G); c->gwl = dev_alloc<int64_t>(G);
            c->bflag = dev_alloc<int32_t>(n); c->bout = dev_alloc<int32_t>(n);
            c->bnewid = dev_alloc<int64_t>(n + 1); c->bgath = dev_alloc<int64_t>(2 * (G + 1));
            c->bscan = dev_alloc<uint8_t>((int64_t)scan_scratch_bytes(n > 0 ? n : 1));
            c->bstatus = dev_alloc<uint8_t>(G); c->bkeep = dev_alloc<uint8_t>(G);
            c->bI2 = dev_alloc<unsigned long long>(G); c->bsq = dev_alloc<unsigned long long>(2 * G);
            c->bsweep = dev_alloc<uint8_t>(G); c->bgmoved = dev_alloc<int32_t>(G);
            HIPCHK(hipMemsetAsync(c->bgmoved, 0, G * 4, c->st));
            HIPCHK(hipStreamSynchronize(c->st));
        }
        if (o.validate) {
            uint32_t bad = validate_graph(c->levels[0].view(), c->scr, c->hbuf, c->st);
            if (!bad && G > 0)
                bad = batch_validate(c->levels[0].view(), c->levels[0].gid, c->levels[0].gbase, c->scr, c->hbuf,
                                     c->st);
            if (bad) {
                std::string why;
                if (bad & 16u) why += " offsets not monotone or not spanning [0, nnz];";
                if (bad & 1u) why += " column index out of range;";
                if (bad & 2u) why += " non-positive weight;";
                if (bad & 4u) why += " row not strictly ascending (duplicate or unsorted);";
                if (bad & 8u) why += " not symmetric (missing or unequal mirror entry);";
                if (bad & 32u) why += " edge between two graphs of the batch;";
                throw Error{PLM_E_GRAPH, "invalid graph:" + why};
            }
        }
        c->vol0 = dev_alloc<int64_t>(n);
        c->vol = dev_alloc<int64_t>(n);
        c->volC = dev_alloc<int64_t>(n);
        c->zeta = dev_alloc<int32_t>(n);
        c->colour = dev_alloc<int32_t>(n);
        c->class_nodes = dev_alloc<int32_t>(n);
        c->noderec = dev_alloc<NodeRec>(n);
        c->move_to = dev_alloc<int32_t>(n);
        c->lab = dev_alloc<int32_t>(n);
        c->dcnt = dev_alloc<unsigned long long>(32);
        HIPCHK(hipMemsetAsync(c->dcnt, 0, 32 * 8, c->st));
        if (!c->batch && o.settle >= 0 && n > 0) {
            c->dw = dev_alloc<uint64_t>(n);
            c->slack = dev_alloc<int64_t>(n);
            c->kslack = dev_alloc<int64_t>(n);
            c->tstamp = dev_alloc<uint64_t>(n);
            c->sctl = dev_alloc<unsigned long long>(2);
            HIPCHK(hipMemsetAsync(c->sctl, 0, 16, c->st));
        }
        if (c->batch) c->set_active_all();
        c->init_level();
    } catch (const Error &e) {
        delete c;
        release_adopted();
        return fail(e.code, e.msg);
    } catch (const std::exception &e) {
        delete c;
        release_adopted();
        return fail(PLM_E_NOMEM, e.what());
    }
    *out = c;
    return PLM_OK;
}

}  // namespace

// Batched run with hooks: graphs join at level boundaries and are reported as
// they finish (continuous batching of the request server in serve.hip).
plm_status plm_internal_batch_serve(plm_ctx *ctx, plm::BatchHooks *hooks) {
    return guarded(ctx, [&] {
        if (!ctx->batch || !hooks) throw Error{PLM_E_STATE, "internal: serving needs a batched context and hooks"};
        ctx->run_batch(nullptr, nullptr, nullptr, hooks);
    });
}

// Batched context over a disjoint-union CSR already in device memory (hipMalloc
// buffers the context adopts; used by the request server in serve.hip).
plm_status plm_internal_batch_adopt(plm_ctx **out, int64_t G, const int64_t *node_base, int64_t nnz, int64_t *off,
                                    int32_t *col, int32_t *w, void *hip_stream, const plm_options *opt) {
    return create_impl(out, G, node_base, node_base[G], nnz, off, col, w, PLM_MEM_DEVICE, hip_stream, opt, true);
}


// EPP(b, PLP, PLMR) (Algorithm 5): b label-propagation runs with seeds
// colour_seed .. colour_seed + b - 1 on the input graph, their core groups
// (Equation (3.2), named by their smallest member), the graph contracted by
// the core groups as level 1, PLMR from there (max_levels counted from level
// 1; level 0 is not refined), and the communities prolonged to the input
// nodes (canonical labels in lab_out).  Returns the PLMR levels.
// The base runs are independent, so they run concurrently: each on a context
// of its own (reading this context's input graph, with its own state, a
// stream of its own and a host thread driving it), as the paper runs its
// ensemble members in parallel;
// each gives exactly the labels of a run alone, and the core groups combine
// them in seed order.
int32_t plm_ctx::epp(int32_t b, int32_t plp_iters, int32_t *lab_out, int64_t *cores_out) {
    reset();
    const int64_t n = n0;
    *cores_out = 0;
    if (n == 0) return 1;
    EnsembleWork wk;
    int32_t *grp = nullptr;
    std::vector<plm_ctx *> runs(b, nullptr);
    std::vector<hipStream_t> rst(b, nullptr);
    std::vector<int32_t *> base(b, nullptr);
    auto release = [&]() {
        dev_free(wk.keys); dev_free(wk.keys_alt); dev_free(wk.vals); dev_free(wk.vals_alt); dev_free(wk.first);
        dev_free(grp);
        if (wk.scratch) (void)hipFree(wk.scratch);
        wk.scratch = nullptr;
        for (int32_t i = 0; i < b; ++i) {
            if (runs[i]) plm_destroy(runs[i]);
            runs[i] = nullptr;
            if (rst[i]) (void)hipStreamDestroy(rst[i]);
            rst[i] = nullptr;
            dev_free(base[i]);
        }
    };
    double t_ens = 0;
    int64_t k = 0;
    try {
        // the base runs' contexts: same graph and options, no validation, no
        // settled-node skip (label propagation keeps its own active set)
        plm_options o = opt;
        o.validate = 0;
        o.timing = 0;
        o.settle = -1;
        o.refine = 0;
        o.hub_stream = 0;  // one stream per base run: the runs are the concurrency
        o.layout = -1;     // the runs read the input in place: no per-run copies of it
        const LevelData &l0 = levels[0];
        HIPCHK(hipStreamSynchronize(st));
        for (int32_t i = 0; i < b; ++i) {
            HIPCHK(hipStreamCreateWithFlags(&rst[i], hipStreamNonBlocking));
            const plm_status rc = create_impl(&runs[i], 0, nullptr, n, l0.nnz, l0.off, l0.col,
                                              (const int32_t *)l0.w, PLM_MEM_DEVICE, rst[i], &o, false, true);
            if (rc != PLM_OK) throw Error{rc, "base run context: " + g_create_error};
            base[i] = dev_alloc<int32_t>(n);
        }
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        std::vector<std::exception_ptr> errs(b);
        std::vector<std::thread> ts;
        const double t_plp = now_ms();
        for (int32_t i = 0; i < b; ++i) {
            ts.emplace_back([&, i] {
                try {
                    HIPCHK(hipSetDevice(dev));
                    plm_ctx *c = runs[i];
                    c->plp_level(opt.colour_seed + (uint64_t)i, plp_iters, nullptr);
                    HIPCHK(hipMemcpyAsync(base[i], c->zeta, n * 4, hipMemcpyDeviceToDevice, c->st));
                    HIPCHK(hipStreamSynchronize(c->st));
                } catch (...) {
                    errs[i] = std::current_exception();
                }
            });
        }
        for (auto &t : ts) t.join();
        for (auto &e : errs)
            if (e) std::rethrow_exception(e);
        for (int32_t i = 0; i < b; ++i) {
            stats.lp_runs += runs[i]->stats.lp_runs;
            stats.lp_iterations += runs[i]->stats.lp_iterations;
            stats.lp_updates += runs[i]->stats.lp_updates;
        }
        stats.lp_ms += now_ms() - t_plp;
        wk.keys = dev_alloc<uint64_t>(n); wk.keys_alt = dev_alloc<uint64_t>(n);
        wk.vals = dev_alloc<int32_t>(n); wk.vals_alt = dev_alloc<int32_t>(n); wk.first = dev_alloc<int32_t>(n);
        wk.scratch = (void *)dev_alloc<uint8_t>((int64_t)ensemble_scratch_bytes(n));
        grp = dev_alloc<int32_t>(n);
        double t1 = now_ms();
        for (int32_t i = 0; i < b; ++i) ensemble_refine(grp, base[i], n, i == 0, wk, st);
        HIPCHK(hipStreamSynchronize(st));
        t_ens += now_ms() - t1;
        t1 = now_ms();
        HIPCHK(hipMemcpyAsync(zeta, grp, n * 4, hipMemcpyDeviceToDevice, st));
        layout_dirty = true;
        HIPCHK(hipStreamSynchronize(st));
        // the colouring of level 0 for the statistics (the base runs coloured
        // with their own seeds): that of the first base run
        const int32_t ncol0 = runs[0]->ncol;
        release();
        const int64_t loops0 = loops;
        k = coarsen();
        stats.levels = 1;
        stats.n[0] = n;
        stats.nnz[0] = levels[0].nnz;
        stats.loops[0] = loops0;
        stats.colours[0] = ncol0;
        stats.communities[0] = k;
        stats.coarsen_ms[0] = now_ms() - t1;
        stats.ens_ms = t_ens;
        stats.ens_cores = k;
    } catch (...) {
        release();
        throw;
    }
    *cores_out = k;
    return descend(lab_out, 1, true);
}

namespace {

void reject_batch(plm_ctx *ctx, const char *what) {
    if (ctx->batch) throw Error{PLM_E_STATE, std::string(what) + " does not apply to a batched context"};
}

}  // namespace

extern "C" {

plm_status plm_create(plm_ctx **out, int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *cols,
                      const int32_t *weights, int32_t mem_kind, void *hip_stream, const plm_options *opt) {
    return create_impl(out, 0, nullptr, n, nnz, offsets, cols, weights, mem_kind, hip_stream, opt);
}

plm_status plm_batch_create(plm_ctx **out, int64_t num_graphs, const int64_t *node_base, int64_t nnz,
                            const int64_t *offsets, const int32_t *cols, const int32_t *weights, int32_t mem_kind,
                            void *hip_stream, const plm_options *opt) {
    if (num_graphs < 1 || num_graphs >= (1LL << 31) || !node_base) {
        g_create_error = "num_graphs must lie in [1, 2^31) and node_base must not be NULL";
        if (out) *out = nullptr;
        return PLM_E_ARG;
    }
    return create_impl(out, num_graphs, node_base, node_base[num_graphs], nnz, offsets, cols, weights, mem_kind,
                       hip_stream, opt);
}

plm_status plm_batch_run(plm_ctx *ctx, int32_t *labels, double *q_out, int32_t *levels_out) {
    return guarded(ctx, [&] {
        if (!ctx->batch) throw Error{PLM_E_STATE, "plm_batch_run needs a context from plm_batch_create"};
        int64_t n = ctx->n0;
        int32_t *canon = dev_alloc<int32_t>(n);
        try {
            ctx->run_batch(canon, q_out, levels_out);
            if (labels) copy_out(labels, canon, (size_t)n * 4, ctx->mem_kind, ctx->st);
            HIPCHK(hipStreamSynchronize(ctx->st));
        } catch (...) {
            dev_free(canon);
            throw;
        }
        dev_free(canon);
    });
}

plm_status plm_move_sweep(plm_ctx *ctx, int64_t *moves_out) {
    return guarded(ctx, [&] {
        int64_t mv = ctx->sweep();
        if (moves_out) *moves_out = mv;
    });
}

plm_status plm_move_class(plm_ctx *ctx, int32_t c, int64_t *moves_out) {
    return guarded(ctx, [&] {
        int32_t nc = ctx->ncol_or_build();
        if (c < 0 || c >= nc) throw Error{PLM_E_ARG, "class index out of range"};
        if (ctx->skip_armed || ctx->opt.settle == 1) ctx->settle_before();
        int64_t mv = ctx->run_classes(c, c + 1);
        if (ctx->skip_armed) ++ctx->armed_sweeps;
        if (moves_out) *moves_out = mv;
    });
}

plm_status plm_coarsen(plm_ctx *ctx, int64_t *n_coarse_out) {
    return guarded(ctx, [&] {
        reject_batch(ctx, "plm_coarsen");
        int64_t k = ctx->coarsen();
        if (n_coarse_out) *n_coarse_out = k;
    });
}

plm_status plm_run(plm_ctx *ctx, int32_t *labels, double *q_out, int32_t *levels_out) {
    return guarded(ctx, [&] {
        reject_batch(ctx, "plm_run");
        int64_t n = ctx->n0;
        int32_t *canon = dev_alloc<int32_t>(n);
        try {
            int32_t lv = ctx->run(canon);
            double q = 0.0;
            if (q_out) q = ctx->modularity_current();
            if (labels) copy_out(labels, canon, (size_t)n * 4, ctx->mem_kind, ctx->st);
            HIPCHK(hipStreamSynchronize(ctx->st));
            if (q_out) *q_out = q;
            if (levels_out) *levels_out = lv;
        } catch (...) {
            dev_free(canon);
            throw;
        }
        dev_free(canon);
    });
}

plm_status plm_plp(plm_ctx *ctx, int32_t max_iters, int32_t *labels, double *q_out, int32_t *iters_out,
                   int64_t *updates_out) {
    return guarded(ctx, [&] {
        reject_batch(ctx, "plm_plp");
        if (max_iters < 1 || max_iters > 64) throw Error{PLM_E_ARG, "max_iters must lie in [1, 64]"};
        int64_t n = ctx->n0;
        int32_t *canon = dev_alloc<int32_t>(n);
        try {
            ctx->reset();
            int64_t upd[64];
            int32_t it = ctx->plp_level(ctx->opt.colour_seed, max_iters, upd);
            if (n > 0) build_canonical(ctx->zeta, n, canon, ctx->scr, ctx->st);
            double q = 0.0;
            if (q_out) q = ctx->modularity_of(canon);
            if (labels) copy_out(labels, canon, (size_t)n * 4, ctx->mem_kind, ctx->st);
            HIPCHK(hipStreamSynchronize(ctx->st));
            if (q_out) *q_out = q;
            if (iters_out) *iters_out = it;
            if (updates_out)
                for (int32_t i = 0; i < it; ++i) updates_out[i] = upd[i];
        } catch (...) {
            dev_free(canon);
            throw;
        }
        dev_free(canon);
    });
}

plm_status plm_epp(plm_ctx *ctx, int32_t ensemble_size, int32_t plp_iters, int32_t *labels, double *q_out,
                   int32_t *levels_out, int64_t *cores_out) {
    return guarded(ctx, [&] {
        reject_batch(ctx, "plm_epp");
        if (ensemble_size < 1 || ensemble_size > 1024) throw Error{PLM_E_ARG, "ensemble_size must lie in [1, 1024]"};
        if (plp_iters < 1 || plp_iters > 64) throw Error{PLM_E_ARG, "plp_iters must lie in [1, 64]"};
        int64_t n = ctx->n0;
        int32_t *canon = dev_alloc<int32_t>(n);
        try {
            int64_t cores = 0;
            int32_t lv = ctx->epp(ensemble_size, plp_iters, canon, &cores);
            double q = 0.0;
            if (q_out) q = ctx->modularity_of(canon);
            if (labels) copy_out(labels, canon, (size_t)n * 4, ctx->mem_kind, ctx->st);
            HIPCHK(hipStreamSynchronize(ctx->st));
            if (q_out) *q_out = q;
            if (levels_out) *levels_out = lv;
            if (cores_out) *cores_out = cores;
        } catch (...) {
            dev_free(canon);
            throw;
        }
        dev_free(canon);
    });
}

plm_status plm_modularity(plm_ctx *ctx, const int32_t *labels, int32_t mem_kind, double *q_out) {
    return guarded(ctx, [&] {
        reject_batch(ctx, "plm_modularity");
        if (!labels && ctx->n0 > 0) throw Error{PLM_E_ARG, "labels is NULL"};
        if (mem_kind != PLM_MEM_HOST && mem_kind != PLM_MEM_DEVICE) throw Error{PLM_E_ARG, "bad mem_kind"};
        int64_t n = ctx->n0;
        const int32_t *dl = labels;
        int32_t *tmp = nullptr;
        if (mem_kind == PLM_MEM_HOST && n > 0) {
            tmp = dev_alloc<int32_t>(n);
            HIPCHK(hipMemcpyAsync(tmp, labels, n * 4, hipMemcpyHostToDevice, ctx->st));
            dl = tmp;
        }
        try {
            double q = ctx->modularity_of(dl);
            if (q_out) *q_out = q;
        } catch (...) {
            dev_free(tmp);
            throw;
        }
        dev_free(tmp);
    });
}

plm_status plm_modularity_noalloc(plm_ctx *ctx, const int32_t *labels, double *q_out) {
    return guarded(ctx, [&] {
        reject_batch(ctx, "plm_modularity_noalloc");
        if (!labels && ctx->n0 > 0) throw Error{PLM_E_ARG, "labels is NULL"};
        if (ctx->n0 > kNoAllocMaxNodes)
            throw Error{PLM_E_ARG, "plm_modularity_noalloc takes at most 2^23 nodes (its static workspace)"};
        if (!ctx->noalloc_ws) throw Error{PLM_E_STATE, "no workspace address for this context's device"};
        if (modularity_ws_bytes(ctx->n0) > kNoAllocBytes) throw Error{PLM_E_STATE, "internal: workspace too small"};
        if (ctx->n0 > 0) {
            hipPointerAttribute_t at;
            hipError_t e = hipPointerGetAttributes(&at, labels);
            if (e != hipSuccess) (void)hipGetLastError();
            if (e != hipSuccess || at.type != hipMemoryTypeDevice)
                throw Error{PLM_E_ARG, "labels must be device memory"};
        }
        __int128 num, den;
        if (modularity_parts_ws(ctx->levels[0].view(), ctx->vol0, labels, ctx->S, ctx->noalloc_ws, ctx->hbuf, &num,
                                &den, ctx->st) != 0)
            throw Error{PLM_E_ARG, "labels must lie in [0, n)"};
        if (q_out) *q_out = ctx->S == 0 ? 0.0 : (double)num / (double)den;
    });
}

plm_status plm_get_options(plm_ctx *ctx, plm_options *out) {
    return guarded(ctx, [&] {
        if (!out) throw Error{PLM_E_ARG, "out is NULL"};
        *out = ctx->opt;
    });
}

plm_status plm_resolve_options(plm_options *o, int32_t batched, int64_t nnz) {
    if (!o || nnz < 0) return PLM_E_ARG;
    std::string m;
    const int rc = check_options(*o, m);
    if (rc) return rc;
    resolve_bins(*o, batched != 0, nnz);
    return check_bins(*o, m);
}

const char *plm_tuned_table(void) {
    std::call_once(g_tuned_once, load_tuned);
    return g_tuned_source.c_str();
}

plm_status plm_reset(plm_ctx *ctx) {
    return guarded(ctx, [&] { ctx->reset(); });
}

void plm_destroy(plm_ctx *ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->st);
    delete ctx;
}

const char *plm_last_error(const plm_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

plm_status plm_level_info(plm_ctx *ctx, plm_level_info_t *out) {
    return guarded(ctx, [&] {
        if (!out) throw Error{PLM_E_ARG, "out is NULL"};
        LevelData &l = ctx->L();
        out->level = ctx->cur;
        out->colours = ctx->sched ? ctx->ncol : 0;
        out->n = l.n;
        out->nnz = l.nnz;
        out->S = ctx->S;
        out->sweeps = ctx->sweeps;
        out->weight_kind = l.wkind;
        out->communities = count_communities(ctx->zeta, l.n, ctx->scr, ctx->hbuf, ctx->st);
        out->max_vol = ctx->max_vol;
    });
}

plm_status plm_get_state(plm_ctx *ctx, int32_t *zeta, int64_t *volc, int32_t *colour, int32_t mem_kind) {
    return guarded(ctx, [&] {
        if (mem_kind != PLM_MEM_HOST && mem_kind != PLM_MEM_DEVICE) throw Error{PLM_E_ARG, "bad mem_kind"};
        int64_t n = ctx->L().n;
        if (colour && !ctx->sched) ctx->build_schedule();
        if (zeta) copy_out(zeta, ctx->zeta, n * 4, mem_kind, ctx->st);
        if (volc) copy_out(volc, ctx->volC, n * 8, mem_kind, ctx->st);
        if (colour) copy_out(colour, ctx->colour, n * 4, mem_kind, ctx->st);
        HIPCHK(hipStreamSynchronize(ctx->st));
    });
}

plm_status plm_get_graph(plm_ctx *ctx, int64_t *offsets, int32_t *cols, int64_t *weights, int32_t mem_kind) {
    return guarded(ctx, [&] {
        if (mem_kind != PLM_MEM_HOST && mem_kind != PLM_MEM_DEVICE) throw Error{PLM_E_ARG, "bad mem_kind"};
        LevelData &l = ctx->L();
        if (offsets) copy_out(offsets, l.off, (l.n + 1) * 8, mem_kind, ctx->st);
        if (cols) copy_out(cols, l.col, l.nnz * 4, mem_kind, ctx->st);
        if (weights && l.nnz > 0) {
            if (l.wkind == 2 && l.diag_mult == 1) {
                copy_out(weights, l.w, l.nnz * 8, mem_kind, ctx->st);
            } else {
                int64_t *tmp = dev_alloc<int64_t>(l.nnz);
                hipLaunchKernelGGL(k_export_w, dim3((unsigned)cdiv(cdiv(l.nnz, 16), 256)), dim3(256), 0, ctx->st,
                                   l.view(), tmp);
                copy_out(weights, tmp, l.nnz * 8, mem_kind, ctx->st);
                HIPCHK(hipStreamSynchronize(ctx->st));
                dev_free(tmp);
            }
        }
        HIPCHK(hipStreamSynchronize(ctx->st));
    });
}

plm_status plm_get_stats(plm_ctx *ctx, plm_stats_t *out) {
    return guarded(ctx, [&] {
        if (!out) throw Error{PLM_E_ARG, "out is NULL"};
        *out = ctx->stats;
    });
}

}  // extern "C"
