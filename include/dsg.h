/*
 * dsg.h -- C ABI of the MI355X densest-subgraph peeling library (libdsg.so).
 *
 * The library runs the iterated load-weighted peeling of Greedy++
 * (Sukprasert, Liu, Dhulipala, Shun, "Practical Parallel Algorithms for
 * Near-Optimal Densest Subgraphs on Massive Graphs", arXiv 2311.04333) on one
 * AMD Instinct MI355X (gfx950).  Three orderings are provided:
 *
 *   DSG_SEQ  -- exact sequential Greedy++ (Algorithm 2 with the load ordering
 *               of Section 2): one vertex at a time, minimum of load+degree,
 *               ties to the lower vertex id.
 *   DSG_PEEL -- the parallel ordering of ParallelGreedy++ (Section 3.3):
 *               round-synchronous peeling.  Each round peels every remaining
 *               vertex with load+degree <= (1 + eps) * (round minimum), and
 *               eps = eps_num/eps_den is exact.  Effects of one round's
 *               peels on degrees are delayed to the end of the round.
 *               Positions inside a round follow ascending vertex id, so a
 *               same-round edge is charged to its lower-id endpoint.
 *   DSG_SORT -- GreedySorting++ / ParallelGreedySorting++ (Sections 3.2,
 *               3.3): order by the load at the start of the iteration,
 *               ties to the lower id.
 *   DSG_PEEL_MONO -- DSG_PEEL with the bucketing of the exact k-core
 *               algorithm that the paper's parallel implementation uses
 *               (Section 3.1): the round bound only grows within an
 *               iteration.  Round r peels every remaining vertex with
 *               load+degree <= d_r, d_r = max(d_{r-1}, (1 + eps) * (round
 *               minimum)); d starts afresh in each iteration.  With eps = 0
 *               this is "peel everything at or below d, raise d when nothing
 *               is left there".  Fewer rounds than DSG_PEEL when degrees fall
 *               below the bound already reached.
 *
 * Every ordering feeds the same density-and-load computation (Algorithm 3):
 * each edge charges its earlier endpoint, the suffix sums give
 * |E(S_i)| of every suffix S_i of the order, the best suffix density of the
 * iteration is kept as an exact (edges, vertices) pair, and the loads grow by
 * the charges.  The best subgraph found so far is replaced only by a
 * strictly denser one (Algorithm 2), starting from the input graph itself.
 *
 * Conventions
 *   - Every call returns dsg_status.  No C++ exception crosses this ABI.
 *     dsg_last_error() returns a message for the calling thread's last
 *     failure.
 *   - "d_" pointers are device pointers (HIP, on the context's device).
 *     "h_" pointers are host pointers.  The caller owns all of them.
 *   - The graph is an undirected simple graph given as a symmetric int32
 *     CSR: offsets[n+1], adj[nnz], nnz = 2m, every row strictly increasing,
 *     no self-loops, and every u in row v has v in row u.  Isolated vertices
 *     are allowed.
 *   - The library allocates no device memory.  All device state lives in
 *     one caller-provided workspace of dsg_workspace_bytes() bytes, which
 *     must stay alive (with the CSR) until dsg_graph_destroy.  The one
 *     exception is dsg_par_run_noalloc, which uses a static device array of
 *     the library instead of a workspace.
 *   - Work is enqueued asynchronously on the context's HIP stream.  The
 *     dsg_get_* calls synchronise that stream before reading.
 *   - Handles are not thread-safe; use one context per host thread.
 */
#ifndef DSG_H
#define DSG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DSG_OK = 0,
    DSG_EINVAL = -1,    /* bad argument or invalid CSR (message says which) */
    DSG_ENOMEM = -2,    /* workspace smaller than dsg_workspace_bytes() */
    DSG_EDEVICE = -3,   /* HIP runtime error (message has the HIP error string) */
    DSG_EOVERFLOW = -4, /* the run could overflow the 31-bit device loads */
    DSG_ESTATE = -5,    /* call not valid in the handle's state */
    DSG_EBUSY = -6      /* server admission refused (over the HBM budget) */
} dsg_status;

typedef enum { DSG_SEQ = 0, DSG_PEEL = 1, DSG_SORT = 2, DSG_PEEL_MONO = 3 } dsg_variant;

/* flags for dsg_graph_create */
#define DSG_VALIDATE 1 /* check every CSR property listed above on the device */
/* Hub order: the graph renumbers its vertices internally by non-increasing
 * degree (ties by id) and keeps a renumbered copy of the CSR in its
 * workspace (dsg_workspace_bytes_ex).  In a skewed graph most adjacency
 * entries point at a few high-degree vertices; numbered first, their
 * per-vertex state shares a few cache lines, so the neighbour gathers of the
 * PEEL and SORT sweeps mostly hit the L2.  Every result (loads, orders,
 * digests, best set, densities) is reported in the caller's ids and is
 * identical to the result without the flag: ties between vertices still go
 * to the smaller caller id. */
#define DSG_HUB_ORDER 2

typedef struct dsg_ctx dsg_ctx;
typedef struct dsg_graph dsg_graph;

/* Context: binds a device and a stream.  hip_stream is a hipStream_t (for
 * example torch.cuda.current_stream().cuda_stream); NULL means the null
 * stream.  Fails with DSG_EDEVICE if the device cannot be used. */
dsg_status dsg_ctx_create(int device, void* hip_stream, dsg_ctx** out);
dsg_status dsg_ctx_destroy(dsg_ctx* ctx);

/* Bytes of workspace a graph of n vertices and nnz CSR entries needs, with
 * room for t_cap recorded iterations (per-iteration densities and digests).
 * n >= 1, 0 <= nnz <= 2^31 - 2^16 (int32 edge positions with a chunk of headroom), t_cap >= 1. */
dsg_status dsg_workspace_bytes(int32_t n, int64_t nnz, int32_t t_cap, int64_t* bytes);

/* The same for a graph created with `flags`: DSG_HUB_ORDER adds the
 * renumbered CSR and the two permutations, 4 (n + 1) + 4 nnz + 8 n bytes
 * (rounded up to 256-byte regions).  Other flags add nothing. */
dsg_status dsg_workspace_bytes_ex(int32_t n, int64_t nnz, int32_t t_cap, int32_t flags, int64_t* bytes);

/* Bind a CSR already resident on the device.  d_workspace must be 256-byte
 * aligned and hold at least dsg_workspace_bytes_ex(n, nnz, t_cap, flags)
 * bytes.  The state is reset: loads 0, best = the input graph (iteration 0).
 * With DSG_VALIDATE the CSR is checked and an invalid one gives DSG_EINVAL.
 * With DSG_HUB_ORDER the caller's CSR is read only here (it is renumbered
 * into the workspace); otherwise it must stay resident and unchanged while
 * the graph exists.  This call synchronises the stream (it reads the
 * maximum degree). */
dsg_status dsg_graph_create(dsg_ctx* ctx, int32_t n, int64_t nnz, const int32_t* d_offsets, const int32_t* d_adj,
                            void* d_workspace, int64_t workspace_bytes, int32_t t_cap, int32_t flags,
                            dsg_graph** out);

/* Run T more iterations of the given variant (T >= 0), appending to the
 * current state: loads and best carry over, so run(a) then run(b) equals
 * run(a + b).  eps = eps_num / eps_den with eps_num >= 0, eps_den >= 1; only
 * DSG_PEEL and DSG_PEEL_MONO read it.  DSG_SEQ requires n <= 16000 (its state
 * sits in LDS); DSG_PEEL and DSG_PEEL_MONO require n < 2^26.
 * Fails with DSG_EINVAL if the recorded iterations would exceed t_cap, and
 * with DSG_EOVERFLOW if (iterations + 1) * max_degree could reach 2^31.
 * Asynchronous: returns once the work is enqueued. */
dsg_status dsg_run(dsg_graph* g, int32_t T, int32_t eps_num, int32_t eps_den, dsg_variant variant);

/* Certificate-driven stop (Section 4.4): runs iterations of the variant one at
 * a time, at most T_max, and stops after the first one whose certificate
 * holds.  After t iterations since the last dsg_reset every densest subgraph
 * S* has rho(S*) <= L_t / t, where L_t is the largest load (each iteration
 * charges every edge of S* to an endpoint inside S*).  The certificate is
 *     L_t * best_vertices * tol_den <= t * best_edges * (tol_den + tol_num),
 * i.e. L_t / t <= (1 + tol) * rho(best), which proves the best subgraph found
 * is within a factor 1 + tol of the optimum.  *iters gets the iterations this
 * call ran, *certified 1 if it stopped on the certificate (0 if it ran T_max
 * without it).  Exact integer arithmetic.  Synchronous: it waits for every
 * iteration to read the certificate.  Errors as dsg_run, and DSG_EDEVICE if a
 * kernel consistency check fired. */
dsg_status dsg_run_until(dsg_graph* g, int32_t T_max, int32_t eps_num, int32_t eps_den, dsg_variant variant,
                         int32_t tol_num, int32_t tol_den, int32_t* iters, int32_t* certified);

/* Loads to 0, best to the input graph, history cleared.  Asynchronous. */
dsg_status dsg_reset(dsg_graph* g);

/* Wait for everything enqueued on the graph's stream.  Returns DSG_EDEVICE if a
 * kernel-side consistency check (bounded round loop, sweep item bounds)
 * fired during the work. */
dsg_status dsg_sync(dsg_graph* g);

/* Best subgraph so far: its edge and vertex counts, the iteration that found
 * it (0 = the input graph) and its index i in that iteration's order (the
 * set is the suffix of the order from position i). */
dsg_status dsg_get_best(dsg_graph* g, int64_t* edges, int64_t* verts, int32_t* iter, int32_t* index);

/* h_mask[v] = 1 if v belongs to the best subgraph, else 0 (n bytes). */
dsg_status dsg_get_best_mask(dsg_graph* g, uint8_t* h_mask);

/* Current loads (n int64 values). */
dsg_status dsg_get_loads(dsg_graph* g, int64_t* h_loads);

/* Per-iteration best suffix (edges, vertices, index), oldest first.  Writes
 * min(cap, count) entries of each non-NULL array.  *count gets the number
 * of iterations recorded. */
dsg_status dsg_get_iter_densities(dsg_graph* g, int64_t* h_edges, int64_t* h_verts, int32_t* h_index, int32_t cap,
                                  int32_t* count);

/* Order of the last iteration: h_round[v] = its peeling round (DSG_PEEL, DSG_PEEL_MONO) or
 * its position (DSG_SEQ, DSG_SORT), h_pos[v] = its position.  Either
 * pointer may be NULL.  *n_rounds gets the number of rounds of that
 * iteration (n for DSG_SEQ and DSG_SORT). */
dsg_status dsg_get_order(dsg_graph* g, int32_t* h_round, int32_t* h_pos, int32_t* n_rounds);

/* Per-iteration order digests, oldest first: the sum mod 2^64 over all v of
 * mix64(((uint64_t)v << 32) | (uint32_t)round[v]).  Here mix64(z) is the
 * SplitMix64 output function applied to z + 0x9E3779B97F4A7C15, and round
 * is as in dsg_get_order.  Also the number of rounds of each iteration
 * (h_rounds may be NULL). */
dsg_status dsg_get_iter_digests(dsg_graph* g, uint64_t* h_digest, int32_t* h_rounds, int32_t cap, int32_t* count);

/* Width and certificate diagnostics (Section 4.4): per recorded iteration,
 * the empirical width w_t = max over v of the iteration's load increase
 * (rho* <= w_t <= max degree), and the largest load after it, L_t.  After t
 * iterations since the last reset, rho* <= L_t / t (the load-based upper
 * bound), so the best density found is certified within a factor
 * (L_t / t) / rho(best).  cap entries at most; *count = recorded
 * iterations.  Waits for the work. */
dsg_status dsg_get_iter_bounds(dsg_graph* g, int32_t* h_width, int64_t* h_load_max, int32_t cap, int32_t* count);

/* Release the handle.  Caller memory (CSR, workspace) is not freed. */
dsg_status dsg_graph_destroy(dsg_graph* g);

/* Device time of the last dsg_run, in milliseconds (HIP events around the
 * enqueued work of that call, on the graph's stream).  The call waits for
 * the work to finish. */
dsg_status dsg_last_run_ms(dsg_graph* g, float* ms);

/* Tuning of the PEEL round loop; results do not depend on it.  Both
 * thresholds count the adjacency entries of a round's frontier, and -1
 * selects the default.
 *  - bucket_min_edges: from this size on, a round applies its neighbour-degree
 *    decrements through owner buckets.  The buckets cover ranges of up to
 *    32768 vertex ids (at most 2048 ranges, enough for every n the PEEL path
 *    accepts): contiguous blocks of ids, or under DSG_HUB_ORDER the first
 *    2^16 ids dealt one by one and the rest by 32-id lines, round robin (with
 *    65536 ids per range when n > 2^24 and every vertex past the first 2^16
 *    ids has degree below 2^16).  Each
 *    range is summed by one block in an LDS histogram after an extra grid
 *    barrier.  Smaller rounds apply the decrements with per-chunk aggregated
 *    device atomics.  Default 2^20 (2^17 under DSG_HUB_ORDER); 0 buckets
 *    every round.
 *  - coarse_min_edges: from this size on, a round sweeps 4096-edge chunks;
 *    smaller rounds sweep 1024-edge chunks, so that more blocks share them.
 *    Default 2^20; 0 = always coarse.
 * The setting is kept across dsg_reset.  Returns DSG_EINVAL for a value below
 * -1 or a NULL graph. */
dsg_status dsg_set_peel_tuning(dsg_graph* g, int64_t bucket_min_edges, int64_t coarse_min_edges);

/* Tuning of the SORT sweep; results do not depend on it.  With coarse ranks
 * the sweep first compares 4-bit position classes of about equal degree
 * mass, kept in an n/2-byte table (held by an XCD's L2 up to n = 2^22, by
 * the MALL above), and loads the neighbour's full position only when the
 * classes are equal.  Without them it loads every neighbour's position.
 * coarse_ranks: -1 = on for 2^19 <= n < 2^26 (the default), 0 = off, 1 = on
 * (ignored for n >= 2^26).
 * The setting is kept across dsg_reset.  DSG_EINVAL for other values or a
 * NULL graph. */
dsg_status dsg_set_sort_tuning(dsg_graph* g, int32_t coarse_ranks);

/* How DSG_PEEL and DSG_PEEL_MONO rounds find their frontier; results do not
 * depend on it.
 *   0 = full list: every round scans every alive vertex, and the positions
 *       come out of the round loop itself.
 *   1 = near list: the alive vertices whose priority is at most a near bound
 *       B (B = 5/4 of a round's threshold, plus one, reset whenever a
 *       threshold passes it) are kept in a list of their own, and a round
 *       whose threshold is at most B scans only that list; other rounds scan
 *       every alive vertex and reset B.  Vertices join the list as a
 *       decrement takes them to B or below.  The positions are sorted by round
 *       after the loop.  Pays off where many rounds peel few vertices out of
 *       many alive ones (large sparse graphs).
 *  -1 = near list from n >= 2^23 vertices, full list below (the default).
 * Kept across dsg_reset.  DSG_EINVAL for other values or a NULL graph. */
dsg_status dsg_set_peel_select(dsg_graph* g, int32_t mode);

/* Optional graph replay (off by default).  When on, dsg_run captures the
 * launches of its T iterations once into a HIP graph (on a private stream of
 * the graph object, at the default priority) and launches the instantiated
 * graph on the context's stream.  A later dsg_run with the same T, eps,
 * variant, history position and load bound (as after dsg_reset), and the
 * same tuning, replays it without re-issuing the launches; any other call
 * captures anew.  Results are the same as without replay.  The captured
 * launches hold no memset nodes.  If the runtime refuses to capture a launch,
 * dsg_run runs eagerly and keeps doing so until replay is switched on again.
 * Kernel timing (dsg_set_kernel_timing) runs eagerly. */
dsg_status dsg_set_graph_replay(dsg_graph* g, int32_t enable);

/* *state = 1 when a captured run is cached, 0 when replay is off or nothing
 * is captured yet, -1 when capture was refused (runs are eager). */
dsg_status dsg_get_graph_replay(dsg_graph* g, int32_t* state);

/* Optional per-launch timing of each iteration's dominant kernel (the PEEL
 * round loop, the SORT sweep, the SEQ peel): HIP events are recorded on the
 * graph's stream right before and after every such launch of later dsg_run
 * calls.  Off by default (enable = 0). */
dsg_status dsg_set_kernel_timing(dsg_graph* g, int32_t enable);

/* Sum of the timed launch durations of the last dsg_run, in milliseconds, and
 * the number of timed launches (0 when timing is off).  Waits for the work. */
dsg_status dsg_get_kernel_timing(dsg_graph* g, float* total_ms, int32_t* launches);

/* ------------------------------------------------- Pruning-and-Refining
 * Algorithm 1 (Section 3) with exact k-core pruning, the "PaR" of
 * PaRGreedy++ and PaRSorting++:
 *   cores, k_max <- Coreness(G);  L <- ceil(k_max / 2);  G <- getCore(G, L);
 *   S <- G;  then T times: S' <- one Greedy++ iteration of `variant` on G
 *   (loads persist across iterations for the vertices that stay);  if
 *   rho(S') > rho(S): S <- S', L <- max(L, rho(S)), G <- getCore(G, ceil L).
 * getCore(G, j) is the subgraph induced by the vertices whose core number in
 * the input graph is >= j, renumbered in input order (so lowest-id ties
 * resolve as on the input).  The core numbers come from dsg_coreness's
 * pass.  All device memory is the caller's workspace
 * (dsg_par_workspace_bytes); the input CSR is only read. */
typedef struct {
    int64_t best_edges;   /* |E(S)| of the best subgraph found */
    int64_t best_verts;   /* |S| */
    int32_t best_iter;    /* iteration that found it, 1..T; 0 = the initial ceil(k_max/2)-core */
    int32_t kmax;         /* largest core number of the input graph */
    int32_t level;        /* final core level ceil(L) */
    int32_t prunes;       /* prunes after the initial one */
    int32_t final_n;      /* vertices of the last refined graph */
    int32_t pad;
    int64_t final_nnz;    /* adjacency entries of the last refined graph */
} dsg_par_result;

/* Core numbers (Coreness, Section 2) of a symmetric int32 CSR on the device:
 * one PEEL pass with zero loads, eps = 0 and monotone round thresholds (every
 * round peels all alive vertices whose degree is at most the largest round
 * minimum so far, as bucketing does; those vertices' core number is that
 * value).  Workspace: dsg_par_workspace_bytes(n, nnz, 1).  flags:
 * DSG_VALIDATE.  Writes *kmax, h_core (n int32, optional), *rounds (optional)
 * and *round_loop_ms (optional: device time of the round loop; timing it
 * adds two events).  Synchronous.  DSG_EINVAL / DSG_EDEVICE as dsg_par_run. */
dsg_status dsg_coreness(dsg_ctx* ctx, int32_t n, int64_t nnz, const int32_t* d_offsets, const int32_t* d_adj,
                        void* d_workspace, int64_t workspace_bytes, int32_t flags, int32_t* h_core, int32_t* kmax,
                        int32_t* rounds, float* round_loop_ms);

/* Device workspace bytes for dsg_par_run.  1 <= n < 2^26, 0 <= nnz <=
 * 2^31 - 2^16, T >= 0.  About four int32 per entry plus the graph state. */
dsg_status dsg_par_workspace_bytes(int32_t n, int64_t nnz, int32_t T, int64_t* bytes);

/* Runs the framework on the symmetric int32 CSR (d_offsets, d_adj) (device,
 * not modified), with T refinement iterations of `variant` (eps_num/eps_den
 * used by DSG_PEEL and DSG_PEEL_MONO).  flags: DSG_VALIDATE checks the input CSR as
 * dsg_graph_create does.  Synchronous on the context's stream.  Host
 * outputs, each optional (NULL to skip): per iteration t = 1..T the edges,
 * vertices and index of S' (h_iter_edges, h_iter_verts, h_iter_index) and
 * the size and core level of the graph it refined (h_iter_n, h_iter_nnz as
 * undirected edges, h_iter_level); the best set's membership in input ids
 * (h_best_mask, n bytes); the core numbers (h_core, n int32).  Errors:
 * DSG_EINVAL (arguments, too small a workspace, invalid CSR, DSG_SEQ on a
 * refined graph above 16000 vertices), DSG_EOVERFLOW ((T + 1) * max_degree
 * >= 2^31), DSG_EDEVICE. */
dsg_status dsg_par_run(dsg_ctx* ctx, int32_t n, int64_t nnz, const int32_t* d_offsets, const int32_t* d_adj,
                       void* d_workspace, int64_t workspace_bytes, int32_t T, int32_t eps_num, int32_t eps_den,
                       dsg_variant variant, int32_t flags, dsg_par_result* result, int64_t* h_iter_edges,
                       int64_t* h_iter_verts, int32_t* h_iter_index, int32_t* h_iter_n, int64_t* h_iter_nnz,
                       int32_t* h_iter_level, uint8_t* h_best_mask, int32_t* h_core);

/* Approximate k-core pruning (Definition "c-Approx k-Core Decomposition",
 * Corollary apxkmax, and the frameworks PaRApxSorting++ and PaRApxGreedy++
 * of Section 4, "Implementations").  The paper cites the decomposition it
 * uses without describing it; here it is round-synchronous peeling with a
 * monotone geometric bound, the Coreness pass run with eps = c - 1: round r
 * peels every alive vertex whose degree is at most
 *   D_r = max(D_{r-1}, floor(c * minimum degree among the alive vertices)),
 * and khat(v) = D at v's round.  Then core(v) <= khat(v) <= c * core(v)
 * (the first vertex of the core(v)-core to go has degree >= core(v) when it
 * goes; every vertex alive at a round has core number >= that round's
 * minimum degree), so it is a c-approximate decomposition.  c = 3/2 is the
 * ratio the paper's experiments use.
 *   first cut: L <- ceil(khat_max / (2c)) = ceil(khat_max * c_den / (2 c_num)),
 *              G <- {v : khat(v) >= L}, which holds every densest subgraph;
 *   then_exact = 0 (PaRApxSorting++ with DSG_SORT): the re-cuts of Algorithm 1
 *              use khat at level ceil(L) (valid since khat >= core);
 *   then_exact = 1 (PaRApxGreedy++ with DSG_PEEL): exact core numbers of the
 *              cut graph (equal to the input's at every level >= L), then the
 *              cut to max(L, ceil(k_max / 2)) and exact re-cuts, so every
 *              refined graph, and every result, is that of dsg_par_run; only
 *              the exact Coreness pass runs on the smaller graph.
 * result->kmax is khat_max (then_exact = 0) or the exact k_max; h_core holds
 * the core numbers the cuts use, in input ids (khat, or the exact numbers of
 * the cut graph with 0 outside it); h_apx_core (n int32, optional) holds
 * khat.  1 < c_num / c_den, c_num <= 2^20.  Other arguments, workspace,
 * outputs and errors as dsg_par_run. */
typedef struct {
    int32_t apx_kmax;   /* largest approximate core number */
    int32_t apx_level;  /* level of the first (approximate) cut */
    int32_t apx_n;      /* vertices of the approximate cut */
    int32_t pad;
    int64_t apx_nnz;    /* adjacency entries of the approximate cut */
} dsg_par_apx;

dsg_status dsg_par_run_apx(dsg_ctx* ctx, int32_t n, int64_t nnz, const int32_t* d_offsets, const int32_t* d_adj,
                           void* d_workspace, int64_t workspace_bytes, int32_t T, int32_t eps_num, int32_t eps_den,
                           dsg_variant variant, int32_t flags, int32_t then_exact, int32_t c_num, int32_t c_den,
                           dsg_par_result* result, dsg_par_apx* apx, int64_t* h_iter_edges, int64_t* h_iter_verts,
                           int32_t* h_iter_index, int32_t* h_iter_n, int64_t* h_iter_nnz, int32_t* h_iter_level,
                           uint8_t* h_best_mask, int32_t* h_core, int32_t* h_apx_core);

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): dsg_par_run
 * without a workspace.  Its kernels use a static device array of
 * DSG_NOALLOC_SCRATCH_BYTES instead, one per GPU, which the library holds from
 * its load until the process ends.  The call allocates nothing: no device or
 * pinned memory, no streams or events, no handles (the HIP objects of the
 * context excepted, made by dsg_ctx_create).  The graph must satisfy
 * dsg_par_workspace_bytes(n, nnz, T) <= DSG_NOALLOC_SCRATCH_BYTES, else
 * DSG_ENOMEM with the needed size in the message (e.g. n = 2^18 with 8.4M
 * CSR entries at T = 50 fits; n = 2^20 with 16.8M does not).  Every call on one
 * GPU shares that GPU's scratch and leaves its contents behind; each call
 * initialises what it reads, so calls in sequence are independent, but calls
 * that overlap on one GPU (two host threads, or two contexts on different
 * streams) race and give undefined results.  Arguments, outputs, results and
 * other errors as dsg_par_run; DSG_EDEVICE if the scratch address could not be
 * resolved on the context's device. */
#define DSG_NOALLOC_SCRATCH_BYTES (256LL << 20)

dsg_status dsg_par_run_noalloc(dsg_ctx* ctx, int32_t n, int64_t nnz, const int32_t* d_offsets, const int32_t* d_adj,
                               int32_t T, int32_t eps_num, int32_t eps_den, dsg_variant variant, int32_t flags,
                               dsg_par_result* result, int64_t* h_iter_edges, int64_t* h_iter_verts,
                               int32_t* h_iter_index, int32_t* h_iter_n, int64_t* h_iter_nnz, int32_t* h_iter_level,
                               uint8_t* h_best_mask, int32_t* h_core);

/* ------------------------------------------------------------------ batches
 * Many independent graphs peeled in one persistent launch (DSG_PEEL rule).
 * Each graph's results are bit-identical to running it alone through
 * dsg_graph_create + dsg_run with the same T and eps.  Blocks of the
 * persistent kernel take whole graphs from a device work queue, largest
 * (by nnz) first, and run all of a graph's iterations with block barriers
 * only. */
typedef struct dsg_batch dsg_batch;

typedef struct {
    const int32_t* d_offsets; /* n + 1 entries, device */
    const int32_t* d_adj;     /* nnz entries, device */
    int32_t n;                /* >= 1 */
    int32_t T;                /* iterations each dsg_batch_run appends (>= 0) */
    int64_t nnz;              /* [0, 2^31 - 2^16] */
    int32_t eps_num;          /* eps = eps_num / eps_den, eps_num >= 0 */
    int32_t eps_den;          /* >= 1 */
} dsg_batch_graph;

/* Workspace bytes for these graphs with t_cap recorded iterations each. */
dsg_status dsg_batch_workspace_bytes(const dsg_batch_graph* graphs, int32_t count, int32_t t_cap, int64_t* bytes);

/* Bind count >= 1 graphs (host array of descriptors, copied; the device CSR
 * arrays must stay alive).  Every CSR gets the offsets and range checks of
 * dsg_graph_create, and with DSG_VALIDATE the full check.  The first bad
 * graph gives DSG_EINVAL and its index in the message.  Synchronises the
 * stream. */
dsg_status dsg_batch_create(dsg_ctx* ctx, const dsg_batch_graph* graphs, int32_t count, int32_t t_cap,
                            void* d_workspace, int64_t workspace_bytes, int32_t flags, dsg_batch** out);

/* Schedule of the persistent kernel: cfg 0 = 256 threads per block with
 * 1024-edge sweep chunks, 1 = 512 / 2048, 2 = 1024 / 4096; blocks_per_cu
 * caps residency (the occupancy limit applies too).  Chosen by the
 * autotuner; default (0, 4). */
dsg_status dsg_batch_set_config(dsg_batch* b, int32_t cfg, int32_t blocks_per_cu);

/* One persistent launch: every graph runs its T more iterations (state
 * carries over as with dsg_run).  DSG_EINVAL if a graph would exceed t_cap,
 * DSG_EOVERFLOW under the same load bound as dsg_run.  Asynchronous. */
dsg_status dsg_batch_run(dsg_batch* b);

/* Every graph back to loads 0, best = its input graph, no history. */
dsg_status dsg_batch_reset(dsg_batch* b);

/* Per-graph results; i in [0, count).  Same meaning as the dsg_get_*
 * calls of a single graph.  Each waits for the stream. */
dsg_status dsg_batch_get_best(dsg_batch* b, int32_t i, int64_t* edges, int64_t* verts, int32_t* iter, int32_t* index);
dsg_status dsg_batch_get_best_mask(dsg_batch* b, int32_t i, uint8_t* h_mask);
dsg_status dsg_batch_get_loads(dsg_batch* b, int32_t i, int64_t* h_loads);
dsg_status dsg_batch_get_iter_densities(dsg_batch* b, int32_t i, int64_t* h_edges, int64_t* h_verts, int32_t* h_index,
                                        int32_t cap, int32_t* count);
dsg_status dsg_batch_get_iter_digests(dsg_batch* b, int32_t i, uint64_t* h_digest, int32_t* h_rounds, int32_t cap,
                                      int32_t* count);

/* Device time of the last dsg_batch_run in milliseconds (waits). */
dsg_status dsg_batch_last_run_ms(dsg_batch* b, float* ms);

dsg_status dsg_batch_destroy(dsg_batch* b);

/* ------------------------------------------------------------------ serving
 * Continuous batching of a request stream (DSG_PEEL rule).  One persistent
 * kernel runs on a stream of its own.  Each request (a host CSR plus T and
 * eps) is admitted if its HBM footprint fits the caller-provided pool and a
 * ring slot is free; otherwise DSG_EBUSY.  It is copied to the device,
 * published to a request ring in pinned host memory, and claimed by the
 * first idle block.  So requests that arrive while others run start as soon
 * as a block frees up.  Results equal those of the same graph run alone
 * with dsg_run.  The CSR's offsets and entry range are checked on the host
 * at submit. */
typedef struct dsg_server dsg_server;

/* d_pool: caller-owned device memory (256-byte aligned) that the server
 * sub-allocates (first fit) for admitted requests.  ring_size >= 1 bounds
 * the requests in flight.  Allocates the pinned ring (host memory) and two
 * streams (kernel, copies), both at the default priority. */
dsg_status dsg_server_create(dsg_ctx* ctx, void* d_pool, int64_t pool_bytes, int32_t ring_size, dsg_server** out);

/* Bytes one request (with its CSR copy) occupies in the pool. */
dsg_status dsg_server_footprint(int32_t n, int64_t nnz, int32_t T, int64_t* bytes);

/* Launch the persistent kernel (cfg 0 = 256 threads / 1024-edge chunks,
 * 1 = 512 / 2048; blocks_per_cu >= 1).  It exits on dsg_server_stop, after
 * idle_seconds with nothing to do, or after max_seconds in total.  A request
 * that was admitted but never claimed (published just as an idle kernel
 * exited) is run by the next dsg_server_start, oldest first. */
dsg_status dsg_server_start(dsg_server* s, int32_t cfg, int32_t blocks_per_cu, double idle_seconds,
                            double max_seconds);

/* Admit one request; copies the host CSR (h_offsets[n+1], h_adj[nnz]) to
 * the pool before returning.  T >= 1, (T + 1) * max_degree < 2^31.
 * DSG_EBUSY when the pool or the ring is full (retry after releasing
 * results); DSG_ESTATE if the kernel is not running. */
dsg_status dsg_server_submit(dsg_server* s, const int32_t* h_offsets, const int32_t* h_adj, int32_t n, int64_t nnz,
                             int32_t T, int32_t eps_num, int32_t eps_den, uint64_t* ticket);

/* Resident graphs: register a CSR that stays on the device (caller-owned,
 * alive until dsg_server_destroy), checked like dsg_graph_create (flags:
 * DSG_VALIDATE).  Only before dsg_server_start.  Requests against it need
 * no copy and no host-side check, so admission is O(1) host work. */
dsg_status dsg_server_register(dsg_server* s, const int32_t* d_offsets, const int32_t* d_adj, int32_t n, int64_t nnz,
                               int32_t flags, int32_t* graph_id);

/* Admit one request against a registered graph (errors as dsg_server_submit). */
dsg_status dsg_server_submit_registered(dsg_server* s, int32_t graph_id, int32_t T, int32_t eps_num, int32_t eps_den,
                                        uint64_t* ticket);

/* Tickets whose results are ready (up to cap); each is reported once. */
dsg_status dsg_server_poll(dsg_server* s, uint64_t* h_tickets, int32_t cap, int32_t* count);

/* Copy a finished request's results: best[4] = (edges, vertices, iteration,
 * index); per-iteration arrays of length T (any may be NULL); h_loads
 * (n int64, may be NULL). */
dsg_status dsg_server_fetch(dsg_server* s, uint64_t ticket, int64_t* best, int64_t* h_edges, int64_t* h_verts,
                            int32_t* h_index, uint64_t* h_digest, int32_t* h_rounds, int64_t* h_loads);

/* Free a finished request's pool memory and ring slot. */
dsg_status dsg_server_release(dsg_server* s, uint64_t ticket);

/* Ask the kernel to finish the queue and exit; waits for it. */
dsg_status dsg_server_stop(dsg_server* s);

/* Stops the kernel if running, frees the pinned ring and streams. */
dsg_status dsg_server_destroy(dsg_server* s);

/* Message for the calling thread's last failed call ("" if none). */
const char* dsg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DSG_H */
