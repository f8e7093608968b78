/*
 * plm.h - C ABI of libplm: the local-moving sweep and the coarsening of the
 * Parallel Louvain Method (PLM) for modularity-based community detection
 * (Staudt & Meyerhenke, "Engineering Parallel Algorithms for Community
 * Detection in Massive Networks", section III-B, Algorithms 2 and 3), on an
 * AMD Instinct MI355X (gfx950).
 *
 * ---------------------------------------------------------------- graph input
 * An undirected graph G = (V, E) with positive integer weights (section III
 * opening paragraph takes real positive weights; this library takes integers so
 * that every gain is exact) as a symmetric CSR:
 *   offsets[n+1] int64, offsets[0] = 0, offsets[n] = nnz, non-decreasing;
 *   cols[nnz]    int32, each row strictly ascending (so no duplicates);
 *   weights[nnz] int32 > 0, or NULL for unit weights.
 * Every non-loop edge {u,v} appears as (u,v,w) and (v,u,w) with equal w.  A
 * self-loop is given once, as (u,u,w(u,u)); the library counts it twice in
 * vol(u) as section III-B defines the node volume.
 * n < 2^31.  The total weight S = sum of volumes = 2 w(E) must stay below 2^62.
 *
 * ---------------------------------------------------------------- schedule
 * The paper moves nodes asynchronously in parallel (section III-B, discussion of
 * Algorithm 3).  This library fixes the order so that every result is
 * reproducible bit for bit:
 *   - priority of node u at level l: (H(seed ^ (l << 40) ^ u), u), H = SplitMix64
 *     (Steele, Lea & Flood 2014), compared lexicographically;
 *   - colour of u = smallest colour not used by a higher-priority neighbour
 *     (Jones-Plassmann = greedy colouring in descending priority);
 *   - a sweep visits the colour classes in ascending order; all nodes of one
 *     class decide against the community volumes at the start of the class and
 *     their moves are applied together (classes are independent sets, so no
 *     decision sees a neighbour's move within the class);
 *   - node u in community D scores each neighbouring community X != D by
 *       gain(X) = S (w(u,X) - w(u,D\u)) - vol(u) (vol(X) - vol(D\u)),
 *     which is 2 w(E)^2 times the paper's Delta-mod (section III-B); it moves to
 *     the highest gain if that gain is > 0, ties going to the lowest X;
 *   - a level ends after a sweep with no move or after max_sweeps sweeps; the
 *     run descends iff the number of communities dropped below the node count;
 *     coarse node ids are the community ids in ascending order.
 * Output labels are canonical: numbered by first occurrence in node order.
 *
 * ---------------------------------------------------------------- conventions
 * Every call returns a plm_status (0 = OK, < 0 = error) and never throws.  On
 * error, plm_last_error(ctx) describes it (plm_last_error(NULL) after a failed
 * plm_create).  Pointers tagged mem_kind are host memory (PLM_MEM_HOST) or
 * device memory of the current HIP device (PLM_MEM_DEVICE).  Device work runs
 * on the stream given at plm_create (NULL = the null stream); every call
 * returns after that work is complete.  A context is used by one host thread at
 * a time; several contexts may share a device.
 */
#ifndef PLM_H
#define PLM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct plm_ctx plm_ctx;
typedef int32_t plm_status;

enum {
    PLM_OK = 0,
    PLM_E_ARG = -1,     /* bad argument or option */
    PLM_E_GRAPH = -2,   /* input is not a valid symmetric CSR (validate = 1) */
    PLM_E_NOMEM = -3,   /* device or host allocation failed */
    PLM_E_DEVICE = -4,  /* a HIP call failed */
    PLM_E_BUDGET = -5,  /* reserved for admission control */
    PLM_E_STATE = -6    /* call not valid in the context's current state */
};

enum { PLM_MEM_HOST = 0, PLM_MEM_DEVICE = 1 };
enum { PLM_SCHEDULE_COLOUR = 0, PLM_SCHEDULE_SEQUENTIAL = 1 };
enum { PLM_INT_AUTO = 0, PLM_INT_64 = 1, PLM_INT_128 = 2 };

typedef struct {
    int32_t max_sweeps;   /* sweeps per level, >= 1; default 32 */
    int32_t max_levels;   /* move phases per run; 0 = until no community merges */
    int32_t schedule;     /* PLM_SCHEDULE_COLOUR (default) or PLM_SCHEDULE_SEQUENTIAL:
                             one node per class in priority order, which is the
                             sequential local moving of Blondel et al. */
    int32_t validate;     /* 1 (default): check the CSR at plm_create */
    uint64_t colour_seed; /* seed of the priority hash; default 0 */
    int32_t int_mode;     /* PLM_INT_AUTO: 64-bit gains where S*vol(u) < 2^62, else
                             128-bit; PLM_INT_128: always 128-bit (same results);
                             PLM_INT_64: 64-bit only, PLM_E_STATE if unsafe */
    /* Degree bins (scheduling of the per-node community accumulation).  0
     * (the default) takes the value of the tuned table: tuned_bins.txt beside
     * the library (written by the package's tune.py; the environment variable
     * PLM_TUNED_TABLE names another file), whose first row of the context's
     * kind (batch or single graph) covering its entry count applies; without
     * one, the compiled defaults 16 / 512 / 4096 (and 12288 for hub_row_max).
     * Any setting gives the same results.  plm_get_options reports the values
     * a context took. */
    int32_t bin_lane;     /* rows up to this length: one lane per node (1..16) */
    int32_t bin_wave;     /* rows up to this length: one wavefront per node (..512) */
    int32_t bin_block;    /* rows up to this length: one workgroup per node (..4096);
                             longer rows ("hubs"): one 1024-thread workgroup up to
                             hub_row_max entries, else several workgroups per node.
                             Rows of the wavefront and workgroup bins whose vol(u)
                             reaches 2^31 also take the hub path. */
    int32_t timing;       /* 1: time the move-decide launches with HIP events */
    int32_t timing_kernel; /* with timing: 0 = every kernel group of every class step;
                              k = 1..5 = only group k (lane, wavefront, workgroup,
                              one-workgroup hub, partitioned hub), so timing costs
                              less.  Each group is timed by events attached to its
                              launches (the partitioned group's two launches each
                              by their own pair) */
    int32_t refine;        /* 1: PLMR (Algorithm 4): after each prolongation, a move
                              phase on that level starting from the prolonged
                              communities (same colour classes and sweep rule);
                              plm_run only (batches and servers: PLM_E_ARG) */
    /* resolution gamma = gamma_num / gamma_den (the gamma of section III-B;
     * default 1/1, 0/0 also means 1): the gain becomes S dw - gamma vol(u) dvol,
     * computed exactly as gamma_den S dw - gamma_num vol(u) dvol.
     * 0 <= gamma_num, 1 <= gamma_den, both < 2^16; with gamma != 1 the total
     * weight must satisfy S^2 max(num, den) < 2^126 (PLM_E_ARG at creation).
     * The reported Q stays the plain modularity (gamma = 1). */
    int32_t gamma_num;
    int32_t gamma_den;
    int32_t graph_sweeps;  /* 1 (default): the sweeps of a level's move phase and
                              the iterations of label propagation replay their
                              launches from a HIP graph captured once per plan;
                              0: every launch is issued one by one.  Same results.
                              Timed runs (timing = 1) always launch one by one.  While
                              a capture runs (on private non-blocking streams), HIP
                              refuses synchronous copies on the legacy default
                              stream from other host threads of the process. */
    int32_t hub_stream;    /* branches of a captured sweep: 2 (default): a class's
                              kernel groups run as three branches (lane, wavefront
                              and one-workgroup hub; workgroup; partitioned hub),
                              joined before the class's moves apply; 1: only the
                              partitioned-hub kernels branch off; 0: one chain.
                              Same results. */
    int32_t colour_tail;   /* 1 (default): once a colouring round's frontier is
                              small, the following rounds run back to back inside
                              one workgroup (one launch for many rounds); 0: every
                              round is a grid launch.  Same colours. */
    /* Limits of the partitioned hub path (section III-B's per-node community
     * accumulation spread over several workgroups).  hub_row_max is tuned like
     * the bins above; agg_max_keys and agg_tile are lowered only to exercise
     * rarely reached branches on small graphs (same results, slower).  0 = the
     * tuned value / the default of each. */
    int32_t hub_row_max;   /* hub-bin rows longer than this (1..12288; compiled
                              default 12288) take the partitioned path instead of
                              one 1024-thread workgroup */
    int32_t agg_max_keys;  /* distinct communities one bucket workgroup takes in a
                              pass before it splits the bucket into sub-partition
                              passes (default 1536, else 32..1536) */
    int32_t agg_tile;      /* chunks whose bucket segments a bucket workgroup
                              flattens at once (default 512, else 1..512) */
    int32_t settle;        /* settled nodes (single-graph move phases): a node none
                              of whose neighbours moved since it last stayed, with
                              a margin its gains cannot have lost to the community
                              volumes that changed meanwhile, keeps its community
                              without a new scan of its row.  0 (default): enabled
                              once a sweep of the phase moved at most n/16 nodes
                              (n/1024 on coarse levels); 1: from the first sweep;
                              -1: never.  Same results. */
    int32_t join;          /* request servers (plm_server_create) only: k >= 1 =
                              continuous batching: a running batch takes queued
                              requests in at its first k level boundaries (each starts
                              at level 0 of its own, so its result is that of its own
                              run) and reports every request as soon as its run ends;
                              batches then always run on the server's worker threads.
                              0 (default): a batch is fixed when it starts and reports
                              at its end. */
    int32_t layout;        /* sweep layout of single graphs: the move sweeps read
                              neighbour communities and community volumes through
                              copies ordered by descending degree (built once per
                              level: 4 bytes per entry and 20 per node), ranking and
                              reporting candidates by their own ids, so results are
                              unchanged.  0 (default): graphs of more than 2^27
                              entries; 1: every single graph; -1: never.  Batches
                              never. */
    int32_t pack_bits;     /* coarsening of levels with 32-bit or unit weights: a
                              (coarse row, coarse column) key and its weight are
                              sorted as one 64-bit word when every entry's weight
                              fits the bits the two ids leave free (a merged weight
                              too large for them is split over several words of
                              the key).  0 (default): all free bits; k in [2, 62]:
                              at most k of them (more splits; lowered only to
                              exercise the split on small graphs); -1: never
                              (key-weight pairs).  Same coarse graph. */
} plm_options;

/* Fills *opt with the defaults above. */
void plm_default_options(plm_options *opt);

/* The options a context runs with, after the tuned table filled the degree
 * bins left at 0. */
plm_status plm_get_options(plm_ctx *ctx, plm_options *out);

/* Path of the tuned table in use ("" when none was found or none of its rows
 * is valid).  The table is read once per process. */
const char *plm_tuned_table(void);

/* Fills the degree bins of *opt left at 0 as a context would: batched != 0
 * for plm_batch_create, nnz its entry count.  No device work.  PLM_E_ARG for
 * invalid options. */
plm_status plm_resolve_options(plm_options *opt, int32_t batched, int64_t nnz);

/* Creates a context holding a private copy of the graph (inputs may be freed
 * as soon as the call returns) and the level-0 state: vol(u) (section III-B),
 * singleton communities, colour classes.  offsets/cols/weights are host or
 * device pointers per mem_kind.  hip_stream is a hipStream_t or NULL.
 * opt NULL = defaults.  Errors: PLM_E_ARG (null pointers, n < 0, n >= 2^31,
 * bad options), PLM_E_GRAPH (invalid CSR, checked when opt->validate),
 * PLM_E_NOMEM, PLM_E_DEVICE.  On error *out is NULL. */
plm_status plm_create(plm_ctx **out, int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *cols,
                      const int32_t *weights, int32_t mem_kind, void *hip_stream, const plm_options *opt);

/* One sweep of Algorithm 2 (move) over all colour classes of the current
 * level; *moves_out = nodes moved.  Errors: PLM_E_STATE (int-mode overflow). */
plm_status plm_move_sweep(plm_ctx *ctx, int64_t *moves_out);

/* One class step of the current level (class c in [0, colours)). */
plm_status plm_move_class(plm_ctx *ctx, int32_t c, int64_t *moves_out);

/* Coarsening (section III-B, implementation): contracts each community of the
 * current level into one node (inter-community weights summed, intra-community
 * weight kept as a self-loop) and makes the coarse graph the current level with
 * singleton communities.  *n_coarse_out = number of coarse nodes. */
plm_status plm_coarsen(plm_ctx *ctx, int64_t *n_coarse_out);

/* Full PLM (Algorithm 3; with opt.refine, PLMR, Algorithm 4) from level 0:
 * move, coarsen while communities merge, prolong.  labels[n] (mem_kind of the context's input) receives canonical
 * labels; *q_out their modularity; *levels_out the number of move phases.  Any
 * output pointer may be NULL. */
plm_status plm_run(plm_ctx *ctx, int32_t *labels, double *q_out, int32_t *levels_out);

/* Label propagation, PLP (Algorithm 1), on the input graph from singleton
 * labels.  Nodes are visited class by class in the colour classes drawn with
 * opt.colour_seed (level 0), each class deciding against the labels at its
 * start; a node takes the label of largest weight among its non-loop
 * neighbours, keeps its own label when that one attains the maximum, and
 * otherwise breaks ties by the largest key t(v, l) = upper 32 bits of
 * SplitMix64(H(v) ^ l) (H: the node's priority hash), then the lowest label.
 * Only active nodes are visited (Algorithm 1); iterations continue while more
 * than n * 10^-5 labels changed, at most max_iters (in [1, 64]) times.
 * labels[n] (mem_kind of the context's input) receives canonical labels,
 * *q_out their modularity, *iters_out the iterations, updates_out[i] (host,
 * max_iters entries) the labels changed in iteration i.  Outputs may be NULL.
 * Leaves the context at level 0.  Errors: PLM_E_ARG, PLM_E_STATE (batched
 * context), PLM_E_NOMEM, PLM_E_DEVICE. */
plm_status plm_plp(plm_ctx *ctx, int32_t max_iters, int32_t *labels, double *q_out, int32_t *iters_out,
                   int64_t *updates_out);

/* Ensemble preprocessing EPP(b, PLP, PLMR) (Algorithm 5): ensemble_size = b
 * (in [1, 1024]) PLP runs as in plm_plp with colour seeds colour_seed ..
 * colour_seed + b - 1 and at most plp_iters (in [1, 64]) iterations each; the
 * core groups of their labels (Equation (3.2): two nodes share a group iff
 * every run gives them the same label), numbered by ascending smallest
 * member; the input contracted by the core groups as level 1; PLMR
 * (Algorithm 4) on it from level 1 (priorities of levels 1, 2, ...;
 * opt.max_levels counts from level 1; level 0 is not refined) with the
 * context's gamma; and the communities prolonged to the input nodes.
 * labels[n] receives canonical labels, *q_out their modularity on the input,
 * *levels_out the PLMR levels, *cores_out the number of core groups.
 * Outputs may be NULL.  Errors as plm_plp. */
plm_status plm_epp(plm_ctx *ctx, int32_t ensemble_size, int32_t plp_iters, int32_t *labels, double *q_out,
                   int32_t *levels_out, int64_t *cores_out);

/* Modularity, Equation (3.1), of labels[n] (values in [0, n), host or device
 * per mem_kind) on the input graph, computed as (S*I2 - sum vol(C)^2) / S^2
 * with exact 128-bit numerator and denominator converted once to double and
 * divided.  PLM_E_ARG for labels out of range. */
plm_status plm_modularity(plm_ctx *ctx, const int32_t *labels, int32_t mem_kind, double *q_out);

/* plm_modularity without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same value as plm_modularity, bit for bit.
 * labels: device memory (n int32, values in [0, n)).  Its workspace (the
 * volume of every label and four counters) is a static device array of
 * PLM_NOALLOC_MAX_NODES * 8 + 256 bytes (64 MiB + 256 B) per device, held
 * until the process ends and whose address is taken at plm_create; so the
 * input graph may have at most PLM_NOALLOC_MAX_NODES nodes (else PLM_E_ARG)
 * and a batched context is PLM_E_STATE.  Every call on a device shares that
 * device's workspace (each call clears what it uses, with kernels): calls that
 * overlap on one device race, so callers serialise them.  PLM_E_ARG for labels
 * out of range or NULL. */
#define PLM_NOALLOC_MAX_NODES (1LL << 23)
plm_status plm_modularity_noalloc(plm_ctx *ctx, const int32_t *labels, double *q_out);

/* ---------------------------------------------------------------- batches
 * Many independent graphs run Algorithm 3 together, each with the result of a
 * separate plm_run on it (same labels, modularity and number of levels): the
 * move phases of all graphs share launches, and a graph whose communities stop
 * merging leaves the later levels.
 *
 * plm_batch_create: num_graphs >= 1 graphs, graph g owning the nodes
 * node_base[g] .. node_base[g+1]-1 (node_base: host array of num_graphs + 1
 * non-decreasing values, node_base[0] = 0; empty graphs allowed).  The CSR
 * (offsets[node_base[num_graphs] + 1], cols, weights as for plm_create) is the
 * disjoint union with global node ids; with opt->validate an entry joining two
 * graphs is PLM_E_GRAPH.  Batched contexts take the colour schedule and
 * int_mode auto or 128 (else PLM_E_ARG); the sum of all graphs' S = 2 w(E)
 * must stay below 2^62.  plm_move_sweep, plm_move_class, plm_reset and the
 * inspection calls apply; plm_coarsen, plm_run and plm_modularity return
 * PLM_E_STATE. */
plm_status plm_batch_create(plm_ctx **out, int64_t num_graphs, const int64_t *node_base, int64_t nnz,
                            const int64_t *offsets, const int32_t *cols, const int32_t *weights, int32_t mem_kind,
                            void *hip_stream, const plm_options *opt);

/* Algorithm 3 on every graph of a batched context.  labels[n] (mem_kind of the
 * input) receives each graph's canonical labels, numbered from 0 within the
 * graph; q_out[num_graphs] (host) each graph's modularity, Equation (3.1)
 * computed as in plm_modularity (0 for a graph without edges);
 * levels_out[num_graphs] (host) each graph's number of move phases.  Any
 * output may be NULL.  PLM_E_STATE on a context from plm_create. */
plm_status plm_batch_run(plm_ctx *ctx, int32_t *labels, double *q_out, int32_t *levels_out);

/* ---------------------------------------------------------------- serving
 * A request server over the batched engine: each request is one graph (CSR as
 * for plm_create); its result equals plm_run on it, whatever it is batched
 * with.  plm_server_step admits queued requests in submission order while
 * their resident footprint (CSR, per-node state and contraction buffers:
 * 8(n+1) + 4 nnz (+4 nnz with weights) + 128 n + 64 nnz bytes) fits what
 * hbm_budget_bytes leaves beside the batches still running and their entries
 * fit max_batch_entries (with nothing running, at least one request), copies
 * them side by side into device memory, runs them as one batch
 * (plm_batch_run) and completes them.  max_inflight (1..16) batches may run
 * at once: with 1, the batch runs inside plm_server_step on hip_stream; with
 * k >= 2, the server's k worker threads each run batches on a stream of their
 * own (without sweep graphs), plm_server_step only admits and hands over (when
 * a worker is free), and the batches' kernels share the device.  Results stay in device memory until
 * plm_server_result fetches them.  The options are those of the batches
 * (colour schedule, int_mode auto or 128, else PLM_E_ARG).  The client calls
 * a server from one host thread at a time. */
typedef struct plm_server plm_server;

typedef struct {
    int64_t queued;        /* submitted, not yet admitted */
    int64_t completed;     /* completed since creation */
    int64_t batches;       /* steps that ran a batch */
    int64_t held_results;  /* completed or failed, not yet fetched */
    int64_t budget_bytes;
    int64_t inflight;      /* batches admitted and not finished */
    int64_t running;       /* requests in those batches */
    int64_t resident_bytes; /* their footprint, charged against the budget */
    int64_t joined;        /* requests that joined a running batch (opt.join) */
} plm_server_info_t;

/* Errors: PLM_E_ARG (budget or entry cap <= 0, max_inflight outside [1, 16],
 * options not valid for batches), PLM_E_DEVICE (worker streams). */
plm_status plm_server_create(plm_server **out, int64_t hbm_budget_bytes, int64_t max_batch_entries,
                             int32_t max_inflight, void *hip_stream, const plm_options *opt);

/* Queues one graph without copying it: offsets/cols/weights (mem_kind) must
 * stay valid and unchanged until the request's result is ready.  Checks
 * offsets[0] = 0 and offsets[n] = nnz (PLM_E_GRAPH); a request whose footprint
 * alone exceeds the budget is refused (PLM_E_BUDGET).  *request_id identifies
 * it in plm_server_result. */
plm_status plm_server_submit(plm_server *s, int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *cols,
                             const int32_t *weights, int32_t mem_kind, int64_t *request_id);

/* Admits one batch (nothing when the queue is empty, every worker is busy, or
 * the first queued request does not fit beside the running batches) and, with
 * max_inflight = 1, runs it; *completed_out = requests completed or failed
 * since the previous step or wait.  A request that fails (invalid graph,
 * allocation) is completed with its error, reported by plm_server_result;
 * when validation refuses a batch of several requests, they are queued again
 * at the front and run one per batch, so that only the invalid ones fail. */
plm_status plm_server_step(plm_server *s, int32_t *completed_out);

/* Blocks until no batch is in flight; *completed_out as for plm_server_step. */
plm_status plm_server_wait(plm_server *s, int32_t *completed_out);

/* *ready_out = 0 while the request waits.  Once it has run: its canonical
 * labels[n] (mem_kind; NULL to discard), *q_out and *levels_out as plm_run
 * gives them, *ready_out = 1, and the request is released (its id becomes
 * unknown, PLM_E_ARG).  A failed request returns its error here, once. */
plm_status plm_server_result(plm_server *s, int64_t request_id, int32_t *labels, int32_t mem_kind, double *q_out,
                             int32_t *levels_out, int32_t *ready_out);

plm_status plm_server_info(plm_server *s, plm_server_info_t *out);
void plm_server_destroy(plm_server *s);
const char *plm_server_last_error(const plm_server *s);

/* Resets the context to level 0 with singleton communities. */
plm_status plm_reset(plm_ctx *ctx);

void plm_destroy(plm_ctx *ctx);

/* Message of the last error on ctx (thread-local create error when ctx is
 * NULL).  Valid until the next call on the same context. */
const char *plm_last_error(const plm_ctx *ctx);

/* ---------------------------------------------------------------- inspection */
typedef struct {
    int32_t level;        /* current level, 0 = input graph */
    int32_t colours;      /* colour classes of the current level (0 before built) */
    int64_t n, nnz;       /* current level */
    int64_t S;            /* total volume 2 w(E), level invariant */
    int32_t sweeps;       /* sweeps done at the current level */
    int32_t weight_kind;  /* 0 unit, 1 int32 (input level), 2 int64 (coarse) */
    int64_t communities;  /* distinct communities at the current level */
    int64_t max_vol;      /* largest node volume at the current level */
} plm_level_info_t;

plm_status plm_level_info(plm_ctx *ctx, plm_level_info_t *out);

/* Copies the current level's community ids (int32[n]), community volumes
 * (int64[n]) and colours (int32[n]); NULL skips an output. */
plm_status plm_get_state(plm_ctx *ctx, int32_t *zeta, int64_t *volc, int32_t *colour, int32_t mem_kind);

/* Copies the current level's CSR: offsets int64[n+1], cols int32[nnz] and
 * weights int64[nnz] with every self-loop entry carrying twice the self-loop
 * weight (so vol(u) is the row sum).  NULL skips an output. */
plm_status plm_get_graph(plm_ctx *ctx, int64_t *offsets, int32_t *cols, int64_t *weights, int32_t mem_kind);

/* Per-run counters of the last plm_run (or of the sweeps since plm_reset). */
#define PLM_MAX_LEVELS 64
typedef struct {
    int32_t levels;
    int32_t pad;
    int64_t n[PLM_MAX_LEVELS], nnz[PLM_MAX_LEVELS], colours[PLM_MAX_LEVELS];
    int64_t sweeps[PLM_MAX_LEVELS], communities[PLM_MAX_LEVELS];
    int64_t moves[PLM_MAX_LEVELS];        /* summed over the level's sweeps */
    double schedule_ms[PLM_MAX_LEVELS];   /* colouring + class bucketing (host clock) */
    double sweep_ms[PLM_MAX_LEVELS];      /* all sweeps of the level (host clock) */
    double coarsen_ms[PLM_MAX_LEVELS];    /* relabel + contraction (host clock) */
    /* with opt.timing: device time of the move-decide launches (HIP events) and
     * their count, and the algorithmic bytes those launches had to move. */
    double decide_ms[PLM_MAX_LEVELS];
    int64_t decide_launches[PLM_MAX_LEVELS];
    double decide_bytes[PLM_MAX_LEVELS];
    int64_t schedule_rounds[PLM_MAX_LEVELS];  /* Jones-Plassmann rounds */
    double colour_ms[PLM_MAX_LEVELS];         /* colouring part of schedule_ms */
    /* with opt.timing, per degree bin (lane, wavefront, workgroup, hub) */
    double bin_ms[PLM_MAX_LEVELS][4];
    double bin_bytes[PLM_MAX_LEVELS][4];
    int64_t bin_nodes[PLM_MAX_LEVELS][4];     /* nodes of the level in each bin */
    int64_t bin_entries[PLM_MAX_LEVELS][4];   /* their CSR entries */
    int64_t loops[PLM_MAX_LEVELS];            /* self-loop entries of the level */
    /* the part of the hub bin taken by one workgroup per hub (rows of at most
     * 12288 entries with vol(u) < 2^31); the rest of the bin is partitioned */
    double hub_single_ms[PLM_MAX_LEVELS];
    double hub_single_bytes[PLM_MAX_LEVELS];
    int64_t hub_single_nodes[PLM_MAX_LEVELS];
    int64_t hub_single_entries[PLM_MAX_LEVELS];
    /* with opt.timing: class steps that launched each kernel (lane, wavefront,
     * workgroup, one-workgroup hub, partitioned hub) */
    int64_t kernel_launches[PLM_MAX_LEVELS][5];
    /* with opt.refine: the move phase after prolongation at each level */
    int64_t ref_sweeps[PLM_MAX_LEVELS];
    int64_t ref_moves[PLM_MAX_LEVELS];
    double ref_ms[PLM_MAX_LEVELS];            /* prolongation + schedule + sweeps (host clock) */
    /* label propagation: plm_plp, and the base solutions of plm_epp */
    int64_t lp_runs, lp_iterations;
    int64_t lp_updates;        /* label changes over all iterations */
    double lp_ms;              /* host clock, colouring included */
    double lp_decide_ms;       /* with opt.timing: device time of the decide launches */
    double lp_first_ms;        /* with opt.timing: that time in the first iteration of each run */
    double lp_first_bytes;     /* algorithmic bytes of those first iterations (every node active) */
    /* plm_epp: core-group combination (host clock) and the core groups */
    double ens_ms;
    int64_t ens_cores;
    /* sweeps counted in sweeps[] (ref_sweeps[]) but not executed: the state
     * after a sweep equalled the state two sweeps before, so every later sweep
     * up to max_sweeps alternates between the last two states, and the level
     * ends in the state its last sweep would leave (the result and the move
     * counts are those of running them) */
    int64_t cycle_sweeps[PLM_MAX_LEVELS];
    int64_t ref_cycle_sweeps[PLM_MAX_LEVELS];
    /* settled nodes (opt.settle): sweeps of the level's move phase run with the
     * skip armed; with opt.timing, over all sweeps of the level: node decisions
     * taken (rows scanned), their row entries, and decisions skipped because
     * the node was settled */
    int64_t settle_sweeps[PLM_MAX_LEVELS];
    int64_t decided_nodes[PLM_MAX_LEVELS];
    int64_t decided_entries[PLM_MAX_LEVELS];
    int64_t settled_nodes[PLM_MAX_LEVELS];
} plm_stats_t;

plm_status plm_get_stats(plm_ctx *ctx, plm_stats_t *out);

#ifdef __cplusplus
}
#endif

#endif /* PLM_H */
