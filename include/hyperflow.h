/*
 * hyperflow.h -- C ABI of the MI355X (gfx950) hypergraph max-flow / min-cut
 * library (libhyperflow.so).
 *
 * Problem (paper: section "Preliminaries", paragraphs "Flows" and "Flows on
 * Hypergraphs"; section "Network Construction"): given a hypergraph
 * H = (V, E, w) with integer net weights w(e) >= 1, a source set S and a
 * sink set T of vertices, compute
 *
 *   F = min over X with S <= X <= V \ T of  sum of w(e) over nets e that
 *       have a pin in X and a pin outside X,
 *
 * which equals the maximum flow of the Lawler expansion (every net e becomes
 * e_in -> e_out with capacity w(e); every pin u has infinite arcs
 * u -> e_in and e_out -> u), with S contracted into one source and T into one
 * sink.  Nets holding both a source and a sink pin are always cut and count
 * in F; single-pin and empty nets never count.
 *
 * Method (paper, section "Parallel Maximum Flow Algorithm"): synchronous
 * rounds of push-relabel over a compacted frontier of active nodes, with
 * exact global relabeling by reverse residual BFS from the sinks; the
 * arcs (u, e_in) carry capacity w(e) during the preflow (paragraph
 * "Restricting Capacities").  The solve stops at a maximum preflow; the
 * source side is the forward residual BFS of the uncapped network seeded
 * with the sources and every non-terminal node that still holds excess
 * (paragraph "Source-Side Cut").  The reported side is the unique
 * inclusion-minimal minimum cut, so results do not depend on the schedule.
 *
 * All capacities, flows and labels are exact int32; the flow value is int64.
 *
 * Memory kinds: mem_kind 0 = host pointers, 1 = device pointers (for example
 * torch.Tensor.data_ptr() of a CUDA/HIP tensor on the current device).
 * Streams: hip_stream is a hipStream_t (NULL = the null stream).  Every call
 * is stream-ordered on that stream and returns after its results are ready.
 *
 * Ownership: the caller owns every buffer it passes; create copies the
 * inputs into library-owned device memory, released by destroy.  Outputs are
 * written into caller buffers only when the call returns FP_OK.
 *
 * Threads: a handle must not be used by two threads at once.  Different
 * handles are independent.
 */
#ifndef HYPERFLOW_H
#define HYPERFLOW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fp_problem fp_problem; /* opaque, library-owned */

typedef enum {
  FP_OK = 0,
  FP_ERR_INVALID = -1,  /* malformed input (see flow_problem_create)          */
  FP_ERR_OVERFLOW = -2, /* sum of net weights exceeds INT32_MAX, or the
                           network does not fit 31-bit node ids            */
  FP_ERR_STATE = -3,    /* call not valid in the handle's current state     */
  FP_ERR_DEVICE = -4,   /* HIP runtime error or a failed internal check     */
  FP_ERR_OOM = -5,      /* device allocation failed                         */
  FP_ERR_ABORTED = -6   /* round budget exhausted before the flow was found */
} fp_status;

/* Tuning and debugging knobs.  A NULL pointer, or 0 in a field, selects the
 * default.  None of them changes any result. */
typedef struct {
  int32_t relabel_factor_x16; /* global relabel once (factor/16) * N relabels
                                 accumulated since the last one (N = number of
                                 network nodes); default 16 = once per N     */
  int32_t round_budget;       /* stop with FP_ERR_ABORTED after this many
                                 discharge rounds in one solve; 0 = no limit */
  int32_t debug_checks;       /* 1 = verify preflow and labelling invariants
                                 after every round (slow; test use)          */
  int32_t tail_threshold;     /* frontier size at or below which a single
                                 workgroup runs the rounds; default 256      */
  int32_t group_lanes;        /* lanes per small frontier vertex: 4, 8 or
                                 16 (small net nodes get half, at least 4);
                                 default 16                                  */
  int32_t big_degree;         /* nodes with more arcs go wave-per-node;
                                 default 32                                  */
  int32_t profile;            /* 1 = time every kernel launch with HIP events,
                                 2 = only the reverse-BFS level kernel (see
                                 flow_problem_kernel_times)                  */
  int32_t gr_interval;        /* also relabel globally after this many rounds
                                 since the last global relabel; default 16,
                                 -1 = only by relabel count and stale flow  */
  int32_t stale_rounds;       /* also relabel globally once the flow value
                                 stayed unchanged for this many rounds with a
                                 small frontier (paper, paragraph "Avoid
                                 Pushing Flow Back"); default 500, -1 = off  */
  int32_t bottom_up_min;      /* reverse-BFS levels with at least this many
                                 nodes are expanded without atomics and the
                                 next level is collected by a sweep over the
                                 labels; default N/50 (at least 1024),
                                 -1 = never                                  */
  int32_t bfs_arc_parallel;   /* 1 = BFS levels split work per arc (prefix sum
                                 over the level's arc counts) instead of per
                                 node; default 0                             */
  int32_t pull_min;           /* reverse-BFS levels with at least this many
                                 nodes run bottom-up: every unlabelled node
                                 looks for a residual arc into the level
                                 (stops at the first); 0 = never            */
  int32_t tail_gr_interval;   /* rounds between global relabels while the
                                 frontier fits the single-workgroup loop
                                 (tail_threshold); default 4 * gr_interval,
                                 -1 = gr_interval                            */
  int32_t bfs_flat;           /* expanded reverse-BFS levels spread the arcs
                                 of a wave's 64 nodes over its lanes; 1 = on
                                 (default), -1 = a fixed group of lanes per
                                 node (group_lanes)                          */
  int32_t bfs_marks;          /* expanded reverse-BFS levels mark reached
                                 nodes in a byte array and the collect sweep
                                 writes their labels; 1 = on, -1 = labels
                                 written during the expansion (default)     */
  int32_t relabel_blocking;   /* 1 = a node pushed to in a round does not
                                 relabel in that round (the paper's blocking
                                 fix of the push-relabel conflict, section
                                 "A Bug in the Synchronous Algorithm");
                                 0 = it relabels to at most its label + 2,
                                 which keeps every label valid (default)    */
  int32_t bfs_xcd;            /* expanded reverse-BFS levels scan their arcs
                                 and hand each head to the workgroups of the
                                 XCD that owns its slice of the labels (1024-
                                 node chunks dealt round-robin to the eight
                                 XCDs), which label it in their own L2;
                                 1 = on for networks of 1 M nodes or more
                                 (about 8 (|pins| + |nets|) bytes of extra
                                 device memory), 2 = on for every size,
                                 -1 = off (default: measured slower)         */
} fp_options;

/* Counters of the last solve (cumulative over warm-started solves). */
typedef struct {
  int64_t rounds;           /* discharge rounds                              */
  int64_t tail_rounds;      /* of which run by the single-workgroup loop     */
  int64_t relabels;         /* relabel operations                            */
  int64_t global_relabels;  /* reverse-BFS global relabels                   */
  int64_t bfs_levels;       /* BFS levels over all global relabels and cuts  */
  int64_t restarts;         /* termination checks that found active nodes    */
  int64_t host_syncs;       /* host round trips                              */
  int64_t flow_value;       /* current flow value                            */
  int64_t alg_bytes;        /* algorithmic bytes moved by the discharge,
                               relabel and BFS kernels since the handle was
                               created (device counters: a node's own fields
                               once, an arc's fields per scanned arc)        */
  int64_t reserved[7];
} fp_stats;

/*
 * flow_problem_create: validate the hypergraph and terminals, copy them to
 * the device and build the device layout (net CSR, vertex incidence CSR).
 *
 *   num_vertices  |V| >= 1
 *   num_nets      |E| >= 0
 *   net_offsets   |E|+1 int32; net_offsets[0] = 0, nondecreasing; the pins
 *                 of net e are pins[net_offsets[e] .. net_offsets[e+1])
 *   pins          net_offsets[|E|] vertex ids in [0, |V|), no vertex twice
 *                 inside one net
 *   net_weights   |E| int32, each >= 1, sum <= INT32_MAX
 *   sources       num_sources >= 1 vertex ids (repeats allowed)
 *   sinks         num_sinks >= 1 vertex ids, disjoint from the sources
 *   mem_kind      memory kind of all input pointers (0 host, 1 device)
 *   opts          NULL for defaults
 *   out           receives the handle on FP_OK, NULL otherwise
 *
 * Errors: FP_ERR_INVALID for any violated condition above, FP_ERR_OVERFLOW
 * for too large weights or sizes, FP_ERR_OOM, FP_ERR_DEVICE.  A failed
 * create leaves nothing allocated.
 */
fp_status flow_problem_create(int32_t num_vertices, int32_t num_nets,
                              const int32_t *net_offsets, const int32_t *pins,
                              const int32_t *net_weights, const int32_t *sources,
                              int32_t num_sources, const int32_t *sinks,
                              int32_t num_sinks, int32_t mem_kind,
                              const fp_options *opts, void *hip_stream,
                              fp_problem **out);

/*
 * maxflow_solve: push-relabel to a maximum preflow of the current S, T
 * (paper, section "Synchronous Parallel Push-Relabel" with the terminating
 * global relabel of section "A Bug in the Synchronous Algorithm").  The
 * first call starts from the zero flow; after flow_problem_pierce it
 * continues from the previous flow and labels (warm start, paragraph
 * "Maintain Distance Labels").
 *
 *   flow_value  host out: maximum flow value = minimum cut weight
 *
 * Errors: FP_ERR_ABORTED when opts->round_budget is exhausted (the handle
 * then holds a valid preflow and may be solved again), FP_ERR_DEVICE.
 */
fp_status maxflow_solve(fp_problem *problem, void *hip_stream, int64_t *flow_value);

/*
 * mincut_source_side: minimal source side of the minimum cut after a solve
 * (paper, paragraph "Source-Side Cut"; forward BFS ignores the (u, e_in)
 * capacity restriction as the paragraph "Restricting Capacities" states).
 *
 *   mem_kind     memory kind of the two output buffers
 *   vertex_side  |V| bytes: 1 if the vertex is in the minimal source side
 *   net_side     |E| bytes or NULL: bit 0 = e_in reachable from the source
 *                side (the net has a pin in it), bit 1 = e_out reachable
 *                (every pin of a non-empty net is in it)
 *
 * Errors: FP_ERR_STATE before a successful solve, FP_ERR_DEVICE (an
 * internal check found a sink reachable, i.e. the preflow was not maximum).
 */
fp_status mincut_source_side(fp_problem *problem, void *hip_stream, int32_t mem_kind,
                             uint8_t *vertex_side, uint8_t *net_side);

/*
 * flow_batch_solve: solve many independent problems with the same device
 * phases as maxflow_solve, all at once (default batch plan below: the
 * union schedule).  Problems may differ in size.  Equivalent to
 * flow_batch_create (no cut outputs, default configuration),
 * flow_batch_run and flow_batch_destroy.
 *
 *   problems     count handles created on the current device, pairwise
 *                distinct
 *   skip         count bytes or NULL; skip[i] != 0 leaves problem i alone
 *                and reports flow_values[i] = -1
 *   flow_values  host out, count entries
 *
 * The union schedule leaves the handles as they were (each problem is
 * solved inside the union network from the zero flow of its current
 * terminals); a batch plan with vertex_sides returns the minimal source
 * sides as well, and the workers schedule (schedule = 2) leaves every
 * solved handle as after maxflow_solve.  Errors: FP_ERR_INVALID,
 * FP_ERR_ABORTED (a problem's round budget ran out; the others are solved),
 * FP_ERR_DEVICE.
 */
fp_status flow_batch_solve(fp_problem *const *problems, int32_t count,
                           const uint8_t *skip, void *hip_stream,
                           int64_t *flow_values);

/*
 * Batch plans: many independent problems solved at once, the pattern of
 * the paper's refinement scheduler (section "Parallel Active Block
 * Scheduling").  Three schedules:
 *   1 (union, the default)  the kept problems are copied into one network,
 *                their disjoint union, and solved once with the device-wide
 *                kernels: every launch of the solve works on all problems
 *                at once (one global relabel is one BFS over every problem,
 *                one round discharges all of their frontiers), and small
 *                problems cost no launches of their own.  The union's
 *                minimal minimum cut is the union of the problems' minimal
 *                minimum cuts, and a problem's flow value is the weight of
 *                its nets that cut cuts (checked against the union's flow
 *                value).  Kept problems that do not fit one union
 *                (union_pins, 31-bit ids) go to several, in index order.
 *                Each run starts from the zero flow of every problem's
 *                current terminals (same results as a warm start) and leaves
 *                the problems' own handles untouched; the problems' round
 *                budgets do not apply to it.
 *   2 (workers)  problems are taken from a shared queue, largest (pins +
 *                network nodes) first, by `streams` host workers, each
 *                driving the single-problem path on a HIP stream of its own,
 *                so the kernels and host round trips of different problems
 *                overlap; every solved handle then behaves as after
 *                maxflow_solve.
 *   3 (workgroups)  one persistent launch, replayed from a captured HIP
 *                graph: each workgroup takes the next problem (largest
 *                first) from a device counter and solves it alone, from the
 *                zero flow of its current terminals to the terminating
 *                global relabel and, with with_cut, its source side, with
 *                workgroup barriers only (no launches or host round trips
 *                per problem: suited to many small problems).  The relabel
 *                interval is gr_interval (0 = 16); relabel work and
 *                stale-flow limits are the first problem's options.  Every solved
 *                handle then behaves as after maxflow_solve; round budgets
 *                and debug checks do not apply.
 */
typedef struct fp_batch fp_batch; /* opaque, library-owned */

typedef struct {
  int32_t group_lanes;   /* lanes per small frontier node: 4, 8 or 16;
                            0 = 8                                          */
  int32_t reserved0;     /* must be 0                                       */
  int32_t gr_interval;   /* rounds between global relabels, -1 = off;
                            0 = 8 for the union, 16 for the workgroups,
                            each problem's own option for the workers      */
  int32_t reserved1;     /* must be 0                                       */
  int32_t streams;       /* workers schedule: concurrent workers (streams),
                            1..64; 0 = 4                                   */
  int32_t schedule;      /* 1 = union, 2 = workers, 3 = workgroups;
                            0 = union                                      */
  int32_t union_pins;    /* union schedule: at most this many pins per
                            union (bounds its device memory); 0 = as many
                            as 31-bit ids allow                            */
  int32_t wg_threads;    /* workgroups schedule: threads per workgroup,
                            256 or 1024; 0 = 1024                          */
} fp_batch_config;

/*
 * flow_batch_create: plan a batch over count distinct problems.
 *
 *   vertex_sides, net_sides  count device pointers each, or NULL: where
 *                flow_batch_run(..., with_cut = 1, ...) writes problem i's
 *                minimal source side (layout as mincut_source_side; a NULL
 *                entry of net_sides skips that output)
 *   config       NULL for defaults
 *
 * The pointer arrays are copied; the buffers they point to must stay valid
 * while the plan is used.  Errors: FP_ERR_INVALID, FP_ERR_OOM, FP_ERR_DEVICE.
 */
fp_status flow_batch_create(fp_problem *const *problems, int32_t count,
                            uint8_t *const *vertex_sides, uint8_t *const *net_sides,
                            const fp_batch_config *config, void *hip_stream,
                            fp_batch **out);

/*
 * flow_batch_run: solve every problem not skipped (workers schedule: warm, a
 * problem that was solved or pierced before continues from its flow, a
 * fresh or reset one starts from zero, and every solved handle behaves as
 * after maxflow_solve; union schedule: see above), and with with_cut = 1
 * also write its minimal source side.  flow_values as in flow_batch_solve.
 * Skipped problems are not touched.  Errors as flow_batch_solve;
 * FP_ERR_INVALID when with_cut = 1 but the plan has no vertex_sides.
 */
fp_status flow_batch_run(fp_batch *batch, const uint8_t *skip, int32_t with_cut,
                         void *hip_stream, int64_t *flow_values);

/*
 * flow_batch_tune: time candidate configurations (schedule and number of
 * streams or threads per workgroup, lanes per node, global relabel
 * interval) on this batch, each run from the zero flow (the better of two
 * runs; with the source sides when the plan has vertex_sides), and keep the
 * fastest.  With a cache_path (or NULL), a
 * configuration stored under the batch's signature (device, problem count,
 * total pins, total network nodes) is reused without timing, and a newly
 * timed one is appended.  Ends with a run of the chosen configuration (with
 * the workers schedule every problem is then solved).  chosen may be NULL.
 */
fp_status flow_batch_tune(fp_batch *batch, void *hip_stream, const char *cache_path,
                          fp_batch_config *chosen);

/* Current configuration of the plan (host out). */
fp_status flow_batch_get_config(const fp_batch *batch, fp_batch_config *out);

/* Release the plan (the problems stay).  NULL is ignored. */
void flow_batch_destroy(fp_batch *batch);

/*
 * flow_release_cached_memory: free the device pools and pinned control
 * blocks that destroyed handles left for reuse.  Handles keep working; the
 * library keeps at most 4 GiB of released pools per process and reuses a
 * block for a new handle it covers without wasting more than half of it.
 * Waits for the current device to be idle.
 */
void flow_release_cached_memory(void);

/*
 * flow_problem_reset: forget the flow; the next solve starts from the zero
 * flow with the handle's current terminals.  Used to time or re-tune solves
 * of the same problem.
 */
fp_status flow_problem_reset(fp_problem *problem);

/*
 * flow_problem_sink_side: maximal sink side of the minimum cut after a
 * solve -- the vertices that can still reach a sink in the residual network
 * (paper, algorithm "FlowCutter Core": backward residual BFS from T; the
 * uncapped network, as for the source side).  It is the complement of the
 * union of all minimum-cut source sides, so it does not depend on the
 * schedule.
 *
 *   mem_kind     memory kind of vertex_side
 *   vertex_side  |V| bytes: 1 if the vertex reaches a sink
 *
 * Errors: FP_ERR_STATE before a successful solve, FP_ERR_DEVICE (an
 * internal check found a source that reaches a sink).
 */
fp_status flow_problem_sink_side(fp_problem *problem, void *hip_stream, int32_t mem_kind,
                                 uint8_t *vertex_side);

/*
 * flow_problem_pierce: turn vertices into terminals for the next solve of an
 * incremental sequence (paper, section "Flow-Based Refinement", algorithm
 * "FlowCutter Core"; paragraphs "Sink-Side Piercing" and "Maintain Distance
 * Labels").  side 0: every vertex of the current minimal source side plus
 * the given vertices becomes a source; side 1: every vertex of the current
 * maximal sink side plus the given vertices becomes a sink, and excess held
 * by new sinks is added to the flow value.  The flow is kept (flows on the
 * pin arcs of new sources are cancelled and a net gaining its first source
 * pin receives its contracted source arc's w(e)), so the next
 * maxflow_solve continues from it.
 *
 *   vertices  n host vertex ids (none may be a terminal of the other side;
 *             terminals of the pierced side are ignored)
 *
 * Errors: FP_ERR_STATE before a successful solve, FP_ERR_INVALID (nothing
 * is changed then).
 */
fp_status flow_problem_pierce(fp_problem *problem, int32_t side, const int32_t *vertices,
                              int32_t n, void *hip_stream);

/* Result of flow_problem_flowcutter. */
typedef struct {
  int64_t flow;          /* cut weight of the returned bipartition            */
  int64_t source_weight; /* c(X) of the returned source side X                */
  int64_t sink_weight;   /* c(V \ X)                                         */
  int32_t iterations;    /* maximum flows computed by the run so far (all
                            calls of a continued run)                       */
  int32_t status;        /* 0 balanced, 1 no piercing vertex left (the last
                            cut is returned), 2 iteration cap (the last
                            source side is returned)                        */
  int32_t side;          /* 0: X = S_r (minimal source side); 1: X = V \ T_r
                            (complement of the maximal sink side)           */
  int32_t augmenting;    /* piercing steps that could not avoid an augmenting
                            path                                             */
  int32_t first_balanced; /* iteration of the first balanced cut, 0 if none  */
  int32_t slice_iterations; /* iterations run by this call (= trace entries
                               written)                                     */
  int32_t resumable;     /* 1 when this call stopped at its iteration limit
                            before the run ended: flow_problem_flowcutter_
                            continue resumes it                             */
  int32_t reserved32;
  int64_t reserved[2];
} fp_cutter_result;

/* One FlowCutter iteration. */
typedef struct {
  int32_t side;          /* side pierced (0 source, 1 sink); -1 when the
                            iteration ended the run                          */
  int32_t node;          /* piercing vertex, -1 if none                       */
  int64_t flow;          /* maximum flow value of the iteration               */
  int64_t source_weight; /* c(S_r)                                            */
  int64_t sink_weight;   /* c(T_r)                                            */
  int32_t count;         /* vertices pierced (node is the smallest); 0 when
                            the iteration ended the run                      */
  int32_t reserved;
} fp_cutter_step;

/*
 * flow_problem_flowcutter: FlowCutter on the problem's current terminals
 * (paper, section "Flow-Based Refinement": algorithm "FlowCutter Core" and
 * paragraphs "Piercing" and "Bulk Piercing"), every flow warm started from
 * the previous one.  Each iteration solves the maximum flow,
 * derives S_r and T_r, and stops when (S_r, V \ S_r) or else
 * (V \ T_r, T_r) is balanced: c(X) <= max_source_weight and
 * c(V \ X) <= max_sink_weight.  Otherwise the lighter of S_r and T_r
 * (source side on ties) becomes the terminal set plus one piercing vertex:
 * the smallest-id pin, outside S_r and T_r, of a net cut by that side's
 * bipartition; else the smallest-id vertex outside S_r and T_r; else the
 * smallest-id such cut-net pin on the other side that is not a terminal yet
 * (an augmenting path follows).  A pierce of a vertex outside S_r and T_r
 * keeps the flow maximum: the next iteration skips the solve and only grows
 * the pierced side's reachable set.
 *
 * Bulk piercing (bulk_percent = beta in percent, 1..99; 0 = one vertex per
 * iteration), in integer arithmetic: only when the pierced side has no
 * candidate avoiding an augmenting path and after that side's first three
 * pierces.  Each side measures the weight its reachable set gained per
 * pierced vertex (the gain taken at the next iteration) and keeps a goal:
 * the term starts at c(V) / 2 - c(side) at the side's first bulk iteration
 * and is multiplied by beta every bulk iteration; goal = term + what the
 * previous goal missed.  The side then takes the
 * max(1, goal * pierced / gained) smallest-id augmenting candidates (all of
 * them if fewer).
 *
 * Most balanced cut (most_balanced = 1; paragraph "Most Balanced Cut"): from
 * the first balanced iteration on, the run keeps piercing as long as no
 * augmenting path is created -- the lighter side takes its free boundary
 * pin, else any free vertex, by the rule above; no solve is needed -- and
 * stops when no vertex outside S_r and T_r is left (or at the iteration
 * cap).  Every iteration offers (S_r, V \ S_r) and then (V \ T_r, T_r);
 * among the balanced ones the run returns the one whose heavier side
 * max(c(X), c(V \ X)) is lightest, the first one found on ties.  The cut
 * weight is the flow value of the first balanced iteration.  (The paper
 * repeats this with randomized choices; this is one deterministic pass.)
 *
 *   vertex_weights  host, |V| ints >= 0
 *   max_iterations  >= 1
 *   bulk_percent    0..99
 *   most_balanced   0 or 1
 *   mem_kind        memory kind of vertex_side
 *   vertex_side     |V| bytes: the returned source side X
 *   result          host out
 *   trace           host, max_iterations entries, or NULL
 *
 * Schedule: unless the handle was created with these options set, the
 * run's warm solves relabel globally every 8 rounds (gr_interval), every 16
 * in the single-workgroup loop (tail_gr_interval), and claim every BFS level
 * (bottom_up_min off); the handle keeps these settings afterwards.
 *
 * The handle keeps the final terminals and flow.  Errors: FP_ERR_INVALID,
 * FP_ERR_ABORTED (a solve ran out of its round budget), FP_ERR_DEVICE.
 */
fp_status flow_problem_flowcutter(fp_problem *problem, const int32_t *vertex_weights,
                                  int64_t max_source_weight, int64_t max_sink_weight,
                                  int32_t max_iterations, int32_t bulk_percent,
                                  int32_t most_balanced, void *hip_stream, int32_t mem_kind,
                                  uint8_t *vertex_side, fp_cutter_result *result,
                                  fp_cutter_step *trace);

/*
 * flow_problem_flowcutter_continue: resume the FlowCutter run of the last
 * flow_problem_flowcutter call on this handle after it stopped at its
 * iteration limit (result->resumable = 1), for up to max_iterations more
 * iterations, exactly as one uninterrupted run would go on: the bounds,
 * bulk-piercing goals and most balanced cut so far are kept in the handle
 * (a caller can so run FlowCutter in slices, e.g. under a time limit as the
 * paper's scheduler aborts long flow computations, section "Parallel
 * Active Block Scheduling", paragraph "Implementation Details").  The
 * vertex weights are those of the starting call.  trace receives this
 * call's iterations (result->slice_iterations entries); result->iterations
 * counts the whole run.  Other calls on the handle in between are allowed
 * (the next iteration then re-derives its sides).
 *
 * Errors: FP_ERR_STATE when there is no run to continue, FP_ERR_INVALID,
 * FP_ERR_ABORTED, FP_ERR_DEVICE.
 */
fp_status flow_problem_flowcutter_continue(fp_problem *problem, int32_t max_iterations,
                                           void *hip_stream, int32_t mem_kind,
                                           uint8_t *vertex_side, fp_cutter_result *result,
                                           fp_cutter_step *trace);

/*
 * flow_problem_terminals: the current terminal sets (after piercing, section
 * "Flow-Based Refinement", algorithm "FlowCutter Core": the pierced side's
 * reachable set plus the piercing vertices become terminals).
 *
 *   mem_kind  memory kind of roles
 *   roles     |V| bytes: 0 free, 1 source, 2 sink
 *
 * Errors: FP_ERR_INVALID, FP_ERR_DEVICE.
 */
fp_status flow_problem_terminals(fp_problem *problem, void *hip_stream, int32_t mem_kind,
                                 uint8_t *roles);

/*
 * Learned pruning scorer (pattern of the paper's pruning rules, section
 * "Parallel Active Block Scheduling", paragraph "Implementation Details":
 * unpromising block-pair flow problems are skipped).  A perceptron
 * 12 -> 64 -> 64 -> 1 with ReLU hidden units maps a problem's features to
 * the probability that refining it improves the cut; it is trained on the
 * outcomes of the plain run-everything schedule with the mean binary
 * cross-entropy on logits and full-batch Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8).  Everything runs in FP32 on the device; the feature
 * normalization statistics are computed in FP64.
 *
 * Parameters (FP_SCORER_PARAMS floats, row-major): W1 [64 x 12], b1 [64],
 * W2 [64 x 64], b2 [64], W3 [64], b3.  Features: n x 12 int64, row-major,
 * non-negative; each is transformed by log1p and z-scored with the mean and
 * population deviation of the data given to scorer_fit_normalization (a
 * deviation below 1e-9 is replaced by 1).  mem_kind applies to features,
 * labels and probabilities (0 host, 1 device).
 */
#define FP_SCORER_PARAMS 5057
typedef struct fp_scorer fp_scorer; /* opaque, library-owned */

/* init_params: host, FP_SCORER_PARAMS finite floats (the caller draws the
 * initialization).  Errors: FP_ERR_INVALID, FP_ERR_OOM, FP_ERR_DEVICE. */
fp_status scorer_create(const float *init_params, void *hip_stream, fp_scorer **out);

/* Normalization statistics from n >= 1 samples. */
fp_status scorer_fit_normalization(fp_scorer *scorer, const int64_t *features, int32_t n,
                                   int32_t mem_kind, void *hip_stream);

/* Gradient (host, FP_SCORER_PARAMS) and mean loss (host) of the current
 * parameters on n labelled samples (labels 0 or 1).  FP_ERR_STATE before
 * the normalization is fitted. */
fp_status scorer_gradient(fp_scorer *scorer, const int64_t *features, const float *labels,
                          int32_t n, int32_t mem_kind, void *hip_stream, float *gradient,
                          float *loss);

/* `steps` full-batch Adam steps with learning rate lr; losses (host, steps
 * entries, or NULL) receives the loss before each step. */
fp_status scorer_train(fp_scorer *scorer, const int64_t *features, const float *labels,
                       int32_t n, int32_t mem_kind, int32_t steps, float lr, void *hip_stream,
                       float *losses);

/* Probabilities of n samples (memory kind mem_kind). */
fp_status scorer_predict(fp_scorer *scorer, const int64_t *features, int32_t n,
                         int32_t mem_kind, void *hip_stream, float *probabilities);

/* Parameters (host) and normalization (host, 12 means then 12 deviations,
 * may be NULL). */
fp_status scorer_get_params(const fp_scorer *scorer, float *params, double *mean_std);

/* Load parameters and, if mean_std is not NULL, the normalization.
 * FP_ERR_INVALID for non-finite values or non-positive deviations (the
 * caller then keeps the plain schedule). */
fp_status scorer_set_params(fp_scorer *scorer, const float *params, const double *mean_std);

void scorer_destroy(fp_scorer *scorer);

/* Counters of the handle (host out). */
fp_status flow_problem_stats(const fp_problem *problem, fp_stats *out);

/*
 * Per-kernel timing when opts->profile = 1: for up to max_kinds kernel kinds
 * writes the kernel name, launch count, summed milliseconds (HIP events on
 * the launch stream) and algorithmic bytes moved (counted on the device).
 * Returns the number of kinds, or a negative fp_status.
 */
int32_t flow_problem_kernel_times(const fp_problem *problem, int32_t max_kinds,
                                  const char **names, int64_t *launches,
                                  double *milliseconds, double *bytes);

/*
 * flow_problem_export_state: copy the current flow state to host buffers
 * (any pointer may be NULL), for certificates and tests.
 *
 *   f_in    |P| ints: flow on (u, e_in) of each pin slot (net-CSR order)
 *   f_out   |P| ints: flow on (e_out, u) of each pin slot
 *   f_b     |E| ints: flow on (e_in, e_out)
 *   labels  |V| + 2|E| ints: distance labels of vertices, then e_in / e_out
 *           of each net interleaved (e_in of net e at |V| + 2e)
 *   excess  same layout as labels
 */
fp_status flow_problem_export_state(fp_problem *problem, void *hip_stream, int32_t *f_in,
                                    int32_t *f_out, int32_t *f_b, int32_t *labels,
                                    int32_t *excess);

/* Release all device memory of the handle.  NULL is ignored. */
void flow_problem_destroy(fp_problem *problem);

/*
 * maxflow_mincut_noalloc: for callers that cannot allocate memory (code
 * recorded into a HIP graph, tight serving loops, runtimes that forbid
 * allocation after start-up).  Computes what flow_problem_create,
 * maxflow_solve, mincut_source_side and flow_problem_destroy compute, in one
 * call that allocates nothing: all device state lives in a file-scope device
 * array of 64 MiB per GPU (problems up to roughly 700,000 pins) that the
 * library holds until the process ends, and the host mirror of its control
 * block in a file-scope host array.  Default options.
 *
 *   inputs       as flow_problem_create, all in memory kind mem_kind
 *   flow_value   host out: maximum flow value = minimum cut weight
 *   vertex_side  |V| bytes, net_side |E| bytes or NULL: as
 *                mincut_source_side, in memory kind mem_kind
 *
 * The array is shared by every call on a GPU and keeps the last call's
 * contents (each call clears what it needs): calls that overlap on one GPU,
 * from several threads or on several streams, race and must be serialised
 * by the caller.  Errors: as flow_problem_create, maxflow_solve and
 * mincut_source_side; FP_ERR_OVERFLOW when the problem needs more than the
 * array holds (the message gives both sizes).
 */
fp_status maxflow_mincut_noalloc(int32_t num_vertices, int32_t num_nets,
                                 const int32_t *net_offsets, const int32_t *pins,
                                 const int32_t *net_weights, const int32_t *sources,
                                 int32_t num_sources, const int32_t *sinks, int32_t num_sinks,
                                 int32_t mem_kind, void *hip_stream, int64_t *flow_value,
                                 uint8_t *vertex_side, uint8_t *net_side);

/*
 * Flow problems of block pairs, built on the device (paper, section
 * "Network Construction": paragraphs "Region Growing", "Construction
 * Algorithms" and "Identical Net Removal").  For each pair (i, j) of blocks
 * of a k-way partition two breadth-first searches grow B_i inside block i
 * and B_j inside block j, starting from the block's pins on the nets with
 * pins in both blocks; each search visits a level in increasing vertex id
 * and adds vertices while the side's weight stays within its cap and at
 * least one vertex of the block stays outside, and stops for good at the
 * first vertex that does not fit.  The pair's flow problem has the n region
 * vertices (local ids 0..n-1 in increasing global id), the source s = n
 * (block i outside the region, contracted) and the sink t = n + 1 (block j
 * outside); each net with a region pin keeps its region pins and gains s
 * (t) when it has a pin of block i (j) outside the region; pins of other
 * blocks are dropped; nets left with fewer than two pins or with both s
 * and t are discarded; nets keep increasing global id and list their pins
 * in increasing local id.  With flags bit 0 nets with equal pin sets are
 * merged into the one of smallest global id, carrying the sum of their
 * weights (this changes no cut).
 */
typedef struct fp_regions fp_regions; /* opaque, library-owned */

/*
 * flow_regions_build: the flow problems of num_pairs block pairs.
 *
 *   num_vertices, num_nets, net_offsets, pins, net_weights   the hypergraph,
 *                as flow_problem_create (pins of a net distinct)
 *   vertex_weights  num_vertices weights >= 1
 *   blocks       num_vertices block ids in [0, k), 2 <= k <= 64
 *   pairs        host, 2 * num_pairs distinct block ids (i, j) per pair
 *   caps         host, 2 * num_pairs weight caps (>= 0) of B_i and B_j
 *                (the caller's policy, e.g. the paper's
 *                (1 + alpha eps) ceil(c(V_i u V_j) / 2) - c(other block))
 *   flags        bit 0: merge identical nets; other bits must be 0
 *   mem_kind     of the hypergraph, vertex weights and blocks
 *
 * Every step runs on the device; the call returns when the problems are
 * built.  Errors: FP_ERR_INVALID (malformed input; the message names it),
 * FP_ERR_OVERFLOW (more than 2^31 - 1 touched nets or pins in all, or a
 * merged weight beyond INT32_MAX), FP_ERR_OOM, FP_ERR_DEVICE.
 */
fp_status flow_regions_build(int32_t num_vertices, int32_t num_nets,
                             const int32_t *net_offsets, const int32_t *pins,
                             const int32_t *net_weights, const int32_t *vertex_weights,
                             const int32_t *blocks, int32_t k, int32_t num_pairs,
                             const int32_t *pairs, const int64_t *caps, int32_t flags,
                             int32_t mem_kind, void *hip_stream, fp_regions **out);

/* Facts of pair `pair`, 16 entries: n, num_vertices (n + 2), num_nets,
 * num_pins, cut_before (weight of the built nets cut by the current
 * bipartition: a pin of block i or s and a pin of block j or t), boundary
 * (level-0 vertices of both searches), c(B_i), c(B_j), seven net-size bins
 * of the built nets (2, 3-4, 5-8, 9-16, 17-64, 65-256, more), nets merged. */
fp_status flow_regions_info(const fp_regions *regions, int32_t pair, int64_t *info);

/* Copy pair `pair`'s problem into caller buffers of memory kind mem_kind
 * (any pointer may be NULL): net_offsets[num_nets + 1], pins[num_pins]
 * (local ids), net_weights[num_nets], vertex_weights[n + 2] (s and t weigh
 * what their blocks keep outside the region), vertex_ids[n] (global id of
 * each region vertex), net_ids[num_nets] (global id of each net). */
fp_status flow_regions_export(const fp_regions *regions, int32_t pair, int32_t mem_kind,
                              void *hip_stream, int32_t *net_offsets, int32_t *pins,
                              int32_t *net_weights, int32_t *vertex_weights,
                              int32_t *vertex_ids, int32_t *net_ids);

/* A flow problem handle of pair `pair` (sources {n}, sinks {n + 1}),
 * created from the device copy as flow_problem_create with mem_kind 1. */
fp_status flow_regions_problem(const fp_regions *regions, int32_t pair, const fp_options *opts,
                               void *hip_stream, fp_problem **out);

/*
 * flow_regions_solve: the minimum cuts of every pair not skipped, solved as
 * disjoint-union networks built straight from the regions' device arrays
 * (one network unless 31-bit ids or a network's INT32_MAX weight sum would
 * be exceeded), like the union schedule of a batch plan but without a
 * handle per pair.  flow_values (host, num_pairs): each kept pair's maximum
 * flow, -1 where skip[q] != 0 (skip may be NULL).  The minimal source sides
 * are kept with the regions (flow_regions_source_side, flow_partition_apply
 * with vertex_sides = NULL) until the next solve.  Errors: FP_ERR_INVALID,
 * FP_ERR_OOM, FP_ERR_DEVICE.
 */
fp_status flow_regions_solve(fp_regions *regions, const uint8_t *skip, void *hip_stream,
                             int64_t *flow_values);

/* Pair `pair`'s minimal source side from the last flow_regions_solve: n
 * bytes, 1 = region vertex in X, memory kind mem_kind.  FP_ERR_STATE before
 * any solve. */
fp_status flow_regions_source_side(const fp_regions *regions, int32_t pair, int32_t mem_kind,
                                   void *hip_stream, uint8_t *vertex_side);

void flow_regions_destroy(fp_regions *regions);

/*
 * A k-way partition on the device, to which the results of block-pair
 * refinements are applied (paper, section "Parallel Active Block
 * Scheduling", paragraph "Apply Moves").  It holds a copy of the
 * hypergraph, the block of every vertex, the pin count of every net in every
 * block and the block weights.
 */
typedef struct fp_partition fp_partition; /* opaque, library-owned */

/* flow_partition_create: inputs as flow_regions_build (2 <= k <= 4096),
 * all in memory kind mem_kind; copied.  Device memory: about
 * 4 (num_nets * k + 3 |pins| + 3 num_vertices) bytes.  Errors:
 * FP_ERR_INVALID, FP_ERR_OOM, FP_ERR_DEVICE. */
fp_status flow_partition_create(int32_t num_vertices, int32_t num_nets,
                                const int32_t *net_offsets, const int32_t *pins,
                                const int32_t *net_weights, const int32_t *vertex_weights,
                                const int32_t *blocks, int32_t k, int32_t mem_kind,
                                void *hip_stream, fp_partition **out);

/*
 * flow_partition_apply: apply the pairs' results in pair order.
 *
 *   regions         built by flow_regions_build on the same hypergraph and k,
 *                   from the partition the results refine
 *   vertex_sides    host array of num_pairs device pointers: pair q's
 *                   minimal source side X over its n region vertices (as
 *                   written by mincut_source_side or a batch plan); NULL =
 *                   the sides of the regions' last flow_regions_solve
 *   expected_gains  host, num_pairs: cut_before - F of each pair
 *   lmax            the balance bound of every block
 *   status, gains, moved   host outputs per pair (any may be NULL):
 *                   status 0 = not tried (expected gain <= 0), 1 = applied,
 *                   2 = rejected (block i or j would exceed lmax),
 *                   3 = reverted (exact gain < 0); gains = exact change of
 *                   sum w(e) (lambda(e) - 1) (0 unless 1 or 3); moved =
 *                   moves applied (or undone)
 *
 * For pair (i, j): a region vertex of block i outside X moves to j, one of
 * block j inside X moves to i; moves whose vertex left its block since the
 * regions were built are dropped; if block i or j would exceed lmax nothing
 * is applied; otherwise all moves are applied and, when the exact gain is
 * negative, undone.  One workgroup runs the sequences in order on the
 * device.  Errors: FP_ERR_INVALID, FP_ERR_OOM, FP_ERR_DEVICE.
 */
fp_status flow_partition_apply(fp_partition *partition, const fp_regions *regions,
                               const uint8_t *const *vertex_sides,
                               const int64_t *expected_gains, int64_t lmax, void *hip_stream,
                               int32_t *status, int64_t *gains, int32_t *moved);

/* Copy out the blocks (num_vertices, memory kind mem_kind), the k block
 * weights (host) and the objective sum w(e) (lambda(e) - 1) (host); any
 * pointer may be NULL. */
fp_status flow_partition_get(fp_partition *partition, int32_t mem_kind, void *hip_stream,
                             int32_t *blocks, int64_t *block_weights, int64_t *objective);

/*
 * flow_partition_refine: refinement rounds around the batched solver (the
 * paper's algorithm "Parallel Flow-Based Refinement" and section
 * "Parallel Active Block Scheduling"), as synchronous rounds on the device:
 * the block pairs with cut weight >= min_cut and an active block (all
 * blocks are active at first), heaviest cut first (then block ids), get
 * regions with side caps min(alpha / 2 * cut, (100 + alpha eps) / 100 *
 * ceil((c(V_i) + c(V_j)) / 2) - c(other block)) (flow_regions_build), are
 * solved at once by the union schedule (minimum cuts; expected gain =
 * cut_before - F) and applied in that order by flow_partition_apply with
 * Lmax = floor((100 + eps) ceil(c(V) / k) / 100); the blocks of every pair
 * applied with a positive gain are active in the next round.  The rounds
 * stop when no pair is left, after max_rounds, or when a round improves
 * sum w(e) (lambda(e) - 1) by less than min_improvement_ppm parts per
 * million.  k <= 64.
 *
 *   objective_per_round   host, max_rounds + 1 entries or NULL: the
 *                         objective before the first round and after each
 */
typedef struct {
  int32_t max_rounds;          /* 0 = 16                                      */
  int32_t min_cut;             /* 0 = 10 (the paper's pruning rule)            */
  int32_t alpha;               /* region scale; 0 = 16                         */
  int32_t eps_percent;         /* imbalance in percent; 0 = 3                  */
  int32_t min_improvement_ppm; /* 0 = 1000 (0.1 %, the paper's stop rule)      */
  int32_t max_pairs;           /* pairs per round at most; 0 = all             */
  int32_t merge_identical;     /* 1 = merge identical nets in the regions      */
  int32_t reserved;            /* must be 0                                    */
} fp_refine_config;

typedef struct {
  int64_t objective_before, objective_after;
  int64_t moves;               /* moves applied (not undone)                   */
  int32_t rounds;
  int32_t pairs_tried, pairs_applied, pairs_reverted, pairs_unbalanced;
  int32_t reserved[3];
} fp_refine_result;

fp_status flow_partition_refine(fp_partition *partition, const fp_refine_config *config,
                                void *hip_stream, fp_refine_result *result,
                                int64_t *objective_per_round);

void flow_partition_destroy(fp_partition *partition);

/* Message of the last failed call on this thread ("" if none). */
const char *fp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HYPERFLOW_H */
