// level.h - launchers of the per-level kernels, the move sweep and coarsening.
#pragma once

#include "plm_internal.h"

namespace plm {

// ---- level.hip
void launch_volumes(const GraphView &g, int64_t *vol, unsigned long long *S_dev, unsigned long long *maxvol_dev,
                    hipStream_t st);
// Colours the level (schedule 0: Jones-Plassmann; 1: priority rank) into
// colour[n]; returns the number of classes.  host_counters: 480 pinned int32.
// use_tail: small frontiers run as one workgroup's back-to-back rounds.
int32_t build_colouring(const GraphView &g, uint64_t seed, int32_t level, int schedule, int32_t *colour,
                        Scratch &scr, int32_t *host_counters, int32_t *jp_rounds, hipStream_t st, bool use_tail);
// Sorts nodes by (colour, degree bin, short row first) into class_nodes;
// bstart_dev[8*ncol+2] receives bucket starts (bucket 8c+2b+s = bin b of class
// c, s = 1 for the wavefront-bin rows longer than kQuadRow and the
// workgroup-bin rows longer than kBlockShortRow; bucket 8*ncol holds
// nodes that cannot move).
// bin_entries[4]: CSR entries of the movable nodes of each bin (added to).
// Nodes of the wave and block bins whose vol(u) does not fit 32 bits go to the
// hub bin (the tables of those bins sum in 32 bits).  keep (batched runs, else
// null): nodes of graphs g with keep[g.gid[u]] == 0 are left out (sentinel key).
void build_buckets(const GraphView &g, const int64_t *vol, const int32_t *colour, int32_t ncol, int64_t b0,
                   int64_t b1, int64_t b2, int32_t *class_nodes, int64_t *bstart_dev,
                   unsigned long long *bin_entries, Scratch &scr, hipStream_t st, const uint8_t *keep = nullptr);

// wavefront-bin rows up to this length take 16 lanes per node (four nodes per
// wavefront) instead of a whole wavefront
constexpr int64_t kQuadRow = 64;
// workgroup-bin rows up to this length take a 256-thread workgroup and a
// smaller table
constexpr int64_t kBlockShortRow = 2048;

// ---- move.hip
// per class position: its node and the node's row, written with the buckets
// and read by the per-node decide kernels in place of the node id and its two
// row offsets (one coalesced load instead of a load and two dependent ones)
struct NodeRec {
    int64_t e0;
    int32_t len, u;
    int32_t s, pad;  // s: u's index in the sweep layout (u itself without one)
};

struct MoveState {
    int32_t *zeta;         // community of each node
    int64_t *volC;         // community volumes
    const int64_t *vol;    // node volumes
    const int32_t *class_nodes;
    const NodeRec *rec = nullptr;  // per class position (see NodeRec)
    // sweep layout (large single graphs; null otherwise): the per-entry
    // community gathers and the community-volume reads of the decide kernels go
    // through copies ordered by descending degree, so that the few nodes most
    // entries point to share cache lines.  sig = a node's index in that order,
    // ord its inverse; colp[e] = sig[col[e]]; zetap[sig[u]] = sig[zeta[u]];
    // volCp[sig[c]] = volC[c].  Candidates are ranked, tie-broken and reported
    // by their original ids (ord), so decisions are those of the graph's own ids.
    const int32_t *colp = nullptr;
    int32_t *zetap = nullptr;
    int64_t *volCp = nullptr;
    const int32_t *sig = nullptr, *ord = nullptr;
    int32_t *move_to;      // per class position: target community or -1
    int64_t S;
    int64_t wide_lim;      // vol(u) > wide_lim needs 128-bit gains
    unsigned long long *moves_dev;  // move counter
    unsigned long long *cand_dev;   // distinct candidates evaluated per bin [4] (may be null)
    unsigned long long *cand_sgl;   // of those in the hub bin, the one-workgroup hubs' (may be null)
    // nodes decided (not settled) and their row entries: [bin], [4 + bin], and
    // of the hub bin the one-workgroup hubs' [8], [9] (may be null)
    unsigned long long *dec_dev = nullptr;
    // batched runs: graph of each node, and per graph S and the 64-bit limit
    const int32_t *gid = nullptr;
    const int64_t *gS = nullptr;
    const int64_t *gwl = nullptr;
    int32_t *gmoved = nullptr;  // set to 1 for the graph of every node that moves
    // resolution gamma = gp / gq: S is scaled by gq, vol(u) multipliers by gp
    int64_t gp = 1, gq = 1;
    // label propagation (Algorithm 1), set for the label-propagation kernels
    // only: active flag of each node, and seed and level of the tie keys
    uint8_t *active = nullptr;
    uint64_t lp_seed = 0;
    int32_t lp_level = 0;
    // settled nodes (move phases of single-graph PLM; null otherwise; the
    // bound is in move.hip).  While sctl[0] != 0: node u last stayed when the
    // moved-volume clock sctl[1] (+= 2 vol(m) per move m) read tstamp[u], with
    // every gain at most -slack[u] and kslack[u] = min(slack, score of
    // staying) (-1 if negative); dw[u] is the edge weight to neighbours that
    // moved since (>= 2^63: u must be decided).
    uint64_t *dw = nullptr;
    int64_t *slack = nullptr;
    int64_t *kslack = nullptr;
    uint64_t *tstamp = nullptr;
    unsigned long long *sctl = nullptr;  // [0] on, [1] moved-volume clock (wraps mod 2^64)
};

__device__ __forceinline__ int64_t node_S(const MoveState &ms, int32_t u) { return ms.gid ? ms.gS[ms.gid[u]] : ms.S; }
__device__ __forceinline__ int64_t node_wl(const MoveState &ms, int32_t u) {
    return ms.gid ? ms.gwl[ms.gid[u]] : ms.wide_lim;
}

// One class step: decide (per bin) then apply.  Counts (bin sizes) come from
// the host copy of the bucket starts.
struct ClassRange {
    int64_t begin[4], count[4];  // per bin
    int64_t quad = 0;            // the first quad nodes of the wavefront bin have rows of at most kQuadRow
    int64_t blk_short = 0;       // the first blk_short nodes of the workgroup bin have rows of at most kBlockShortRow
    // hubs of this class in the level's hub arrays
    int64_t hub_first = 0, hub_count = 0;
    int64_t ins_blocks = 0, agg_blocks = 0;
    // first entries of this class in the level's per-workgroup hub lists:
    // single-workgroup hubs, reduce workgroups of the partitioned hubs (one
    // per kHubMarkSlice entries of each row), their chunk and bucket
    // workgroups
    int64_t sgl_base = 0, sgl_count = 0, red_base = 0, red_count = 0, ins_base = 0, agg_base = 0;
};

// Launch plans of the hub kernels, one record per workgroup (filled on the
// device from the per-hub arrays once per plan): a workgroup finds its node,
// row slice and staging offsets with one load instead of a chain of dependent
// ones (workgroup -> hub -> node -> row offsets).
struct HubSglPlan {    // one-workgroup hub
    int64_t e0, e1;    // row of u
    int32_t u, pos;    // node, class position
    int32_t s, pad;    // u's index in the sweep layout
};
struct HubPartPlan {   // chunk workgroup of a partitioned hub
    int64_t c0;        // first entry of the chunk
    int64_t stg;       // staging offset of the chunk (class area)
    int64_t bkt;       // offset of the hub's (bucket, chunk) words (class area)
    int32_t u, hg, k, len, nch, pb, pos, s;  // node, hub, chunk, entries, chunks, log2 buckets, class position,
                                             // u's index in the sweep layout
};
struct HubAggPlan {    // bucket workgroup of a partitioned hub
    int64_t bkt;       // offset of this bucket's words, one per chunk (class area)
    int64_t stg;       // staging offset of the hub (class area)
    int64_t wd;        // first chunk workgroup of the hub (class-relative): its w(u, D) shares
    int32_t u, hg, p, nch;
    int32_t s, pad;    // u's index in the sweep layout
};
struct HubRedPlan {    // reduce of a partitioned hub (in the apply launch), one per slice of its row
    int64_t agg;       // first bucket workgroup of the hub (class-relative)
    int64_t wd;        // first chunk workgroup of the hub (class-relative)
    int64_t s0, s1;    // the slice of u's row this workgroup marks (or activates) when u moves
    int32_t u, hg, nagg, nch, k, s;  // k: slice (0 applies the move); s: u's index in the sweep layout
};

struct HubArrays {
    const int32_t *hub_pos;    // class position of each hub
    const int32_t *hub_u;      // node of each hub
    const int32_t *sgl_hub;    // hubs taken by one workgroup (level-wide list)
    const int32_t *red_hub;    // partitioned hubs (level-wide list)
    const int32_t *ins_hub;    // hub of each chunk workgroup (level-wide list)
    const int32_t *agg_hub;    // hub of each bucket workgroup (level-wide list)
    const int64_t *ins_first;  // first chunk workgroup of each hub (class-relative prefix)
    const int64_t *agg_first;  // first bucket workgroup of each hub (class-relative prefix)
    const int32_t *nchunk;     // chunks of each hub
    const int32_t *pbits;      // log2 of the bucket count of each hub
    const int64_t *stg_off;    // staging offset (entries) of each hub within the class area
    const int64_t *bkt_off;    // offset of each hub's (bucket, chunk) words within the class area
    int32_t *stg_x;            // staging: community of each entry
    int64_t *stg_w;            // staging: weight of each entry
    uint32_t *bkt;             // (start << 16 | count) per (bucket, chunk), bucket-major
    int64_t *wd_part;          // per chunk workgroup: its share of w(u, D \ u)
    int64_t *hub_base;         // per hub: vol(D \ u) at the start of its class
    unsigned long long *part;  // per bucket workgroup: score hi, score lo, X, slack of the bucket
    int32_t *hub_skip;         // per hub: 1 = settled in its current class step (written by agg)
    uint64_t *hub_clk;         // per hub: the moved-volume clock at the start of its class step
    const HubSglPlan *splan = nullptr;   // per workgroup of the level-wide lists above
    const HubPartPlan *pplan = nullptr;
    const HubAggPlan *aplan = nullptr;
    const HubRedPlan *rplan = nullptr;
    // lowered limits of the bucket workgroups (0 = the compiled ones): new
    // communities per pass, and chunks flattened at once
    int32_t agg_max_keys = 0, agg_tile = 0;
};

constexpr int64_t kHubInsChunk = 1024;  // entries per hub chunk workgroup
constexpr int kHubMaxPBits = 12;        // at most 4096 buckets per hub
constexpr int64_t kHubBucketTarget = 1024;  // entries per hash bucket (one agg workgroup each)
constexpr int64_t kHubMarkSlice = 16384;  // row entries per reduce workgroup of a partitioned hub
constexpr int64_t kSingleMaxRow = 12288;  // hubs up to this row length (and vol < 2^31) take one workgroup

// ev (may be null): per kernel group (lane, wavefront, workgroup, one-workgroup
// hub, partitioned hub) a start and a stop event, taken by the group's first
// and last dispatch, for the groups whose bit is set in ev_mask and that launch
// ms.active non-null: the label-propagation variant (ms.S = 2^32, ms.gp = 0,
// ms.gq = 1, ms.wide_lim = INT32_MAX)
// groups: bit i launches kernel group i (lane, wavefront, workgroup,
// one-workgroup hub, partitioned hub)
void launch_class_step(const GraphView &g, const MoveState &ms, const ClassRange &cr, const HubArrays &ha,
                       bool force_wide, const hipEvent_t *ev, unsigned ev_mask, hipStream_t st,
                       unsigned groups = 0x1fu);
// The moves of a class: reduce and apply of its partitioned hubs, and the
// apply of every other decided move (all class positions)
void launch_apply(const GraphView &g, const MoveState &ms, const HubArrays &ha, const ClassRange &cr,
                  hipStream_t st);
// row lengths (negated when vol(u) >= 2^31) and nodes of the hubs at class
// positions [begin, begin + count)
// rec[i] = (row start, row length, node) of class_nodes[i], i < count
void launch_node_recs(const GraphView &g, const int32_t *class_nodes, int64_t count, NodeRec *rec,
                      const int32_t *sig, hipStream_t st);
// sweep layout of a level: ord = nodes by descending degree (ties by id),
// sig its inverse, colp[e] = sig[col[e]] (keys/vals/alt: 4 n-word scratch
// arrays, rs: radix scratch for n items)
void build_layout(const GraphView &g, int32_t *sig, int32_t *ord, int32_t *colp, uint32_t *keys, int32_t *vals,
                  uint32_t *keys_alt, int32_t *vals_alt, void *rs, hipStream_t st);
// zetap[sig[u]] = sig[zeta[u]], volCp[sig[u]] = volC[u] for u < n
void sync_layout(int64_t n, const int32_t *zeta, const int64_t *volC, const int32_t *sig, int32_t *zetap,
                 int64_t *volCp, hipStream_t st);
// fills the launch plans of the level-wide hub lists (ins_abs / agg_abs /
// red_abs: first list index of each hub's chunk / bucket / reduce workgroups)
void launch_hub_plans(const GraphView &g, const HubArrays &ha, const int32_t *sig, const int64_t *ins_abs,
                      const int64_t *agg_abs, const int64_t *red_abs, int64_t n_sgl, int64_t n_ins, int64_t n_agg, int64_t n_red, HubSglPlan *sp, HubPartPlan *pp,
                      HubAggPlan *ap, HubRedPlan *rp, hipStream_t st);
void launch_hub_degrees(const GraphView &g, const int32_t *class_nodes, const int64_t *vol, int64_t begin,
                        int64_t count, int64_t *deg_out, int32_t *u_out, hipStream_t st);

// ---- coarsen.hip
// pi[u] = rank of zeta[u] among non-empty communities; returns k.
int64_t build_relabel(const int32_t *zeta, int64_t n, int32_t *pi, Scratch &scr, int64_t *host_i64,
                      hipStream_t st);
// Contracts g by pi into a coarse CSR (doubled diagonal, int64 weights, rows
// ascending).  Allocates *coff/*ccol/*cw with hipMalloc.  Returns nnz'.
// keep (batched runs, else null): rows of graphs g with keep[g.gid[u]] == 0
// are left out.
int64_t build_contraction(const GraphView &g, const int32_t *pi, int64_t k, int64_t **coff, int32_t **ccol,
                          int64_t **cw, Scratch &scr, int64_t *host_i64, hipStream_t st,
                          const uint8_t *keep = nullptr, int pack_bits = 0);
// lab[v] = map[lab[v]] for v < n
void launch_compose(int32_t *lab, const int32_t *map, int64_t n, hipStream_t st);
void launch_iota(int32_t *a, int64_t n, hipStream_t st);
// *flag = 1 if a[0..n) and b[0..n) differ (the caller clears *flag)
void launch_differ(const int32_t *a, const int32_t *b, int64_t n, int32_t *flag, hipStream_t st);
// community volumes of a partition with ids in [0, n)
void launch_comm_vol(const int32_t *zeta, const int64_t *vol, int64_t n, int64_t *volC, hipStream_t st);
void launch_copy_vol(int64_t *dst, const int64_t *src, int64_t n, hipStream_t st);
// canonical relabel by first occurrence, into out
void build_canonical(const int32_t *lab, int64_t n, int32_t *out, Scratch &scr, hipStream_t st);
// numerator/denominator of Equation (3.1) on level 0 for labels; returns
// status 0, or -1 when a label is out of range
int modularity_parts(const GraphView &g0, const int64_t *vol0, const int32_t *labels, int64_t S, Scratch &scr,
                     int64_t *host_i64, __int128 *num, __int128 *den, hipStream_t st);
// The same with caller workspace ws of modularity_ws_bytes(g0.n) bytes (no
// allocation; its counters are cleared by kernels, not memset nodes).
size_t modularity_ws_bytes(int64_t n);
int modularity_parts_ws(const GraphView &g0, const int64_t *vol0, const int32_t *labels, int64_t S, void *ws,
                        int64_t *host_i64, __int128 *num, __int128 *den, hipStream_t st);
// counts distinct values of zeta
int64_t count_communities(const int32_t *zeta, int64_t n, Scratch &scr, int64_t *host_i64, hipStream_t st);
// validation of an input CSR; returns 0 or an error code bit set
uint32_t validate_graph(const GraphView &g, Scratch &scr, int64_t *host_i64, hipStream_t st);

// ---- ensemble.hip
// Work arrays of ensemble_refine for n nodes (device): keys and keys_alt
// uint64[n], vals, vals_alt and first int32[n], ensemble_scratch_bytes(n) of
// scratch.
struct EnsembleWork {
    uint64_t *keys = nullptr, *keys_alt = nullptr;
    int32_t *vals = nullptr, *vals_alt = nullptr, *first = nullptr;
    void *scratch = nullptr;
};
size_t ensemble_scratch_bytes(int64_t n);
// Refines the core groups grp[n] (each node's group named by its smallest
// member) by the labels lab[n] (ids in [0, n)) of one more base solution;
// first_solution: grp is not read, the groups become those of lab.
void ensemble_refine(int32_t *grp, const int32_t *lab, int64_t n, bool first_solution, EnsembleWork &wk,
                     hipStream_t st);

// ---- batch.hip
void launch_gather_i64(const int64_t *a, const int64_t *idx, int64_t count, int64_t *out, hipStream_t st);
void batch_relabel(const int32_t *zeta, int64_t n, const int32_t *gid, const uint8_t *keep, int32_t *flag,
                   int64_t *newid, int32_t *pi, void *scan_scratch, hipStream_t st);
void launch_fill_gid(const int64_t *base, int64_t A, int64_t n, int32_t *gid, hipStream_t st);
void launch_batch_step(int64_t n0, const int32_t *gid0, const uint8_t *status, const int32_t *gid,
                       const int64_t *base, const int32_t *zeta, const int32_t *pi, int32_t *lab, int32_t *out,
                       hipStream_t st);
void launch_graph_S(const int64_t *vol, const int64_t *base, int64_t A, int64_t gmax, int64_t *S, int64_t *wl,
                    hipStream_t st);
void batch_canonical(int64_t n0, const int32_t *gid0, const int64_t *gbase0, const int32_t *local, int32_t *keys,
                     int32_t *rank, int32_t *out, Scratch &scr, hipStream_t st);
void batch_modularity_parts(const GraphView &g0, const int32_t *gid0, const int32_t *key, const int64_t *vol0,
                            int64_t G, int64_t *volL, unsigned long long *I2, unsigned long long *sq, hipStream_t st);
uint32_t batch_validate(const GraphView &g, const int32_t *gid0, const int64_t *gbase0, Scratch &scr,
                        int64_t *host_i64, hipStream_t st);
// joins (batch.hip): offsets dst[0..n] = ebase + off[0..n]; input-level
// entries (columns + nbase, weights or unit weights when w is not null);
// coarse-level entries (columns + nbase, int64 weights with the self-loop
// doubled); a[i] = first + i; a[i] = x
void launch_append_off(int64_t *dst, const int64_t *off, int64_t n, int64_t ebase, hipStream_t st);
void launch_append_input(int32_t *col, int32_t *w, const int32_t *jcol, const int32_t *jw, int64_t nnz, int64_t nbase,
                         hipStream_t st);
void launch_append_coarse(int32_t *col, int64_t *w, const int64_t *joff, int64_t n, const int32_t *jcol,
                          const int32_t *jw, int64_t nnz, int64_t nbase, hipStream_t st);
void launch_iota_from(int32_t *a, int64_t n, int64_t first, hipStream_t st);
void launch_fill_i32(int32_t *a, int64_t n, int32_t x, hipStream_t st);
// modularity parts of the graph on nodes [a, a + n) of a union (global column
// ids) for local labels lab[0..n): acc3 = [I2, sum vol(C)^2 lo, hi]; volL: n
// words of scratch
void graph_modularity_parts(const GraphView &g0, int64_t a, int64_t n, const int32_t *lab, const int64_t *vol0,
                            int64_t *volL, unsigned long long *acc3, hipStream_t st);

}  // namespace plm
