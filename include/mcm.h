/*
 * mcm.h -- maximum-cardinality matching in bipartite graphs on one MI355X
 * (gfx950), after Deveci, Kaya, Ucar and Catalyurek, "GPU accelerated
 * maximum cardinality matching algorithms for bipartite graphs".
 *
 * Method (paper, section 3): starting from a given (typically greedy)
 * matching, repeat phases until a phase finds nothing:
 *   - a level-synchronous alternating BFS from every unmatched column over
 *     the column-compressed pattern, recording for each reached row the
 *     column it was reached from (predecessor) and, per BFS tree, its root
 *     column (Algorithm 2 "GPUBFS"; Algorithm 4 "GPUBFS-WR" adds the root
 *     and stops expanding a tree once its root has found an unmatched row);
 *   - Alternate (Algorithm 3): from every unmatched row found, flip the
 *     matched/unmatched edges back along the predecessor chain to the
 *     root.  Walks of one tree that share a way to the root either stop
 *     where another walk already flipped (the check of Algorithm 3, option
 *     "alternate" "classic") or flip the shared part alike (option "fast",
 *     the default on low-degree graphs), and then the last flip of the
 *     column where they join wins;
 *   - FixMatching: unmatch every row whose column no longer points back.
 * APFB (the default driver) keeps expanding BFS levels until the frontier
 * is empty; APsB stops at the first level that finds an unmatched row
 * (Algorithm 1 and the text after it).  On termination no augmenting path
 * is left, so the matching is maximum (Berge's theorem, section 2).
 *
 * Conventions shared by every entry point
 *   - Graph: CSC.  colptr[ncols+1] with colptr[0] = 0, non-decreasing,
 *     colptr[ncols] = nnz < 2^31; rowind[nnz] with 0 <= rowind[j] < nrows.
 *     Rows of a column may come in any order; duplicates are tolerated.
 *   - Matching: cmatch[ncols], rmatch[nrows], int32; cmatch[c] = r and
 *     rmatch[r] = c for a matched pair, -1 for an unmatched vertex (the
 *     problem statement of Algorithm 1).
 *   - Unless stated otherwise, array arguments are DEVICE pointers owned by
 *     the caller; the library never frees caller memory and keeps no
 *     pointer to it after the call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls that return a result synchronise that stream before returning.
 *   - Errors: a negative return value is an mcm_status; mcm_strerror()
 *     gives the message of the calling thread's last error.  No C++
 *     exception crosses this interface.
 *   - Concurrency: entry points may be called from several host threads.
 *     Calls on the same stream share one library workspace and are
 *     serialised; calls on different streams use separate workspaces (each
 *     grows to the largest graph it has served, until mcm_shutdown) and may
 *     run at the same time.
 *     The library keeps at most one cooperative (whole-device) launch in
 *     flight in the process: mcm_match, mcm_konig_cover and mcm_bfs_levels
 *     on graphs above the one-workgroup size, the multi-graph launches of
 *     mcm_match_batched and of a request server take turns; a server's
 *     large requests wait while another caller's launch runs.
 */
#ifndef MCM_H
#define MCM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MCM_OK = 0,
    MCM_EINVAL = -1,     /* bad argument or malformed CSC (see mcm_set_option "validate") */
    MCM_ENOMEM = -2,     /* device or host allocation failed */
    MCM_EHIP = -3,       /* a HIP runtime call failed */
    MCM_EBADINIT = -4,   /* initial matching inconsistent or not on edges (validate=1 only) */
    MCM_EINTERNAL = -5,  /* watchdog: a phase or level bound was exceeded, or a device wait timed out */
    MCM_ENOTMAX = -6     /* mcm_konig_cover: the given matching admits an augmenting path */
} mcm_status;

/*
 * mcm_match -- maximum matching of one graph (paper, Algorithm 1 driven as
 * APFB by default, BFS kernel GPUBFS-WR of Algorithm 4, Alternate of
 * Algorithm 3, FixMatching).
 *
 *   ncols, nrows   number of column and row vertices (>= 0)
 *   colptr         [ncols+1] device, CSC column pointers
 *   rowind         [nnz] device, row indices; may be NULL only when nnz == 0
 *   init_cmatch    [ncols] device, initial matching, or NULL
 *   init_rmatch    [nrows] device, or NULL; both NULL = empty matching,
 *                  exactly one NULL is MCM_EINVAL.  Must be a matching of
 *                  the graph (checked only with option validate=1).
 *   out_cmatch     [ncols] device, receives a maximum matching; may alias
 *                  init_cmatch
 *   out_rmatch     [nrows] device; may alias init_rmatch
 *   stream         hipStream_t as void*
 *
 * Returns |M| >= 0, or a negative mcm_status.  ncols == 0 or nrows == 0
 * returns 0 with both outputs filled with -1.  The matching returned is a
 * maximum matching; which one depends on the schedule of the concurrent
 * flips (the paper's Alternate races by design), its size does not.
 */
int64_t mcm_match(int32_t ncols, int32_t nrows, const int32_t *colptr, const int32_t *rowind,
                  const int32_t *init_cmatch, const int32_t *init_rmatch,
                  int32_t *out_cmatch, int32_t *out_rmatch, void *stream);

/*
 * mcm_match_noalloc -- mcm_match for callers that cannot allocate memory:
 * code under stream capture, tight serving loops, harnesses that forbid
 * device allocation.  Same arguments, options, results and status codes as
 * mcm_match (the same kernels run), but the call allocates nothing: the
 * working state of the match lives in one fixed device array of 64 MiB
 * that the library holds on each device it runs on until the process ends
 * (looked up once per device on the first call there), and the host side
 * uses static memory.
 *
 * Limit: the graph's state must fit that array: 32 B per row, 12 B per
 * column and 32 B per frontier-queue entry (one per column, plus one per 64
 * edges when columns are split; see option "split"), plus about 260 KB of
 * control and barrier lines -- about 800 000 vertices per side at 4 edges
 * per column.  A larger graph returns MCM_ENOMEM with the sizes in the
 * message, before anything is launched.
 *
 * Calls on one device share its array; overlapping calls would race on it,
 * so the library makes them take turns (a per-device lock held until the
 * call's stream has finished with the array).  The array keeps the last
 * call's contents, which the next call does not read.  No per-phase record
 * (mcm_last_phases) and no kernel timing (kernel_ms reads 0) are kept.
 */
int64_t mcm_match_noalloc(int32_t ncols, int32_t nrows, const int32_t *colptr, const int32_t *rowind,
                          const int32_t *init_cmatch, const int32_t *init_rmatch,
                          int32_t *out_cmatch, int32_t *out_rmatch, void *stream);

/*
 * One graph of a batch.  Offsets are element offsets into the packed
 * arrays of mcm_match_batched: column pointers of graph g are
 * colptr_all[colptr_off .. colptr_off+ncols] (ncols+1 entries, local
 * values starting at 0), its rows rowind_all[rowind_off ..) (local row
 * ids), its column state *_cmatch_all[col_off ..) and row state
 * *_rmatch_all[row_off ..).
 */
typedef struct {
    int32_t ncols, nrows;
    int64_t colptr_off, rowind_off, col_off, row_off;
} mcm_graph;

/*
 * mcm_match_batched -- maximum matchings of many independent graphs in one
 * device launch (one persistent kernel drains a work queue of graphs,
 * largest first; each graph is matched by one workgroup with the same
 * phases as mcm_match).  Members with ncols + nrows above both the option
 * "multi_threshold" (default 2^15) and twice the batch's vertices per
 * resident workgroup are matched instead, after the
 * workgroup kernel on the same stream, by one cooperative launch whose
 * groups of "multi_group" blocks (default: an eighth of the CUs) take them
 * from a queue.  Defined to equal calling mcm_match on each graph: the per-graph
 * cardinalities are identical.
 *
 *   ngraphs            >= 0
 *   graphs             [ngraphs] HOST array of descriptors (copied)
 *   colptr_all, rowind_all           device, packed CSC of every graph
 *   init_cmatch_all, init_rmatch_all device, packed initial matchings, or
 *                                    both NULL (all empty)
 *   out_cmatch_all, out_rmatch_all   device, packed outputs (may alias init)
 *   out_card           [ngraphs] HOST, receives |M_g|, or NULL
 *   stream             hipStream_t as void*
 *
 * Returns sum_g |M_g| >= 0 or a negative mcm_status.  Graph ranges must
 * not overlap in the output arrays.
 */
int64_t mcm_match_batched(int32_t ngraphs, const mcm_graph *graphs,
                          const int32_t *colptr_all, const int32_t *rowind_all,
                          const int32_t *init_cmatch_all, const int32_t *init_rmatch_all,
                          int32_t *out_cmatch_all, int32_t *out_rmatch_all,
                          int64_t *out_card, void *stream);

/*
 * Batch plans: the descriptors of a fixed set of graphs are uploaded once
 * and the launch sequence of mcm_match_batched (control reset, the
 * one-workgroup-per-graph kernel for every member, whatever its size,
 * result copies) is captured in a hipGraph
 * that every mcm_batch_plan_run replays.  The arrays named at creation stay
 * bound to the plan: between runs the caller may change their contents
 * (new initial matchings, even new graphs of the same sizes) but not the
 * pointers.  With option "autotune" = "1" creation times every candidate
 * configuration (mapping thread/wave x workgroup 256/512/1024 threads x
 * wavefront batch 1/8/32 entries) on the plan's own graphs and keeps the
 * fastest; the choice is cached per device and size class, in the file
 * named by option "tuning" if set, and reused by later plans and by
 * mcm_match_batched (mapping "auto").
 *
 *   mcm_batch_plan_create  same arguments as mcm_match_batched (no stream,
 *                          no card array); *plan receives the handle.
 *                          Returns MCM_OK or a negative mcm_status.  The
 *                          plan owns its workspace (device memory of about
 *                          28 bytes per row and 36 per column).
 *   mcm_batch_plan_run     replays the plan on `stream`, synchronises it,
 *                          writes |M_g| into out_card (HOST [ngraphs], or
 *                          NULL); returns sum |M_g| or a negative status.
 *   mcm_batch_plan_info    JSON description of the chosen configuration.
 *   mcm_batch_plan_destroy releases everything (NULL is accepted).
 */
typedef struct mcm_batch_plan mcm_batch_plan;

int64_t mcm_batch_plan_create(int32_t ngraphs, const mcm_graph *graphs,
                              const int32_t *colptr_all, const int32_t *rowind_all,
                              const int32_t *init_cmatch_all, const int32_t *init_rmatch_all,
                              int32_t *out_cmatch_all, int32_t *out_rmatch_all,
                              mcm_batch_plan **plan);
int64_t mcm_batch_plan_run(mcm_batch_plan *plan, int64_t *out_card, void *stream);
int mcm_batch_plan_info(const mcm_batch_plan *plan, char *buf, int32_t len);
int mcm_batch_plan_destroy(mcm_batch_plan *plan);

/*
 * mcm_cheap_init -- a cheap initial matching computed on the device (the
 * paper starts every algorithm from a cheap greedy matching, section 4).
 * Parallel greedy: each column takes the first row of its stored adjacency
 * that it can claim while still unmatched; the result is a maximal
 * matching, schedule dependent (it generally differs from the sequential
 * mcm_cheap_init_host).  cmatch[ncols], rmatch[nrows]: DEVICE outputs.
 * Returns |M0| or a negative mcm_status.
 */
int64_t mcm_cheap_init(int32_t ncols, int32_t nrows, const int32_t *colptr, const int32_t *rowind,
                       int32_t *cmatch, int32_t *rmatch, void *stream);

/*
 * Serving: a continuous-batching request server.  Requests (one graph each,
 * HOST CSC arrays) are admitted in arrival order while their device
 * footprint (inputs, outputs and workspace, about 4(nc+1) + 4 nnz + 12 nc +
 * 28 nr bytes plus queue space) fits the HBM budget; later requests wait in
 * the queue until memory returns.  A worker thread copies admitted inputs
 * to the device on a copy stream and keeps launching the batched matcher
 * over every admitted request whose inputs have arrived, while new requests
 * are admitted and copied; requests with nc + nr above 2^15 go, up to 64
 * per launch, to one cooperative launch whose groups of blocks (an eighth
 * of the CUs each) take them from a queue.  Every request starts from the device cheap matching and ends
 * with a maximum matching of its graph, copied back into the caller's
 * arrays; its memory is then released.
 *
 *   mcm_server_create  budget in bytes (> 0), largest batch per launch (>= 1)
 *   mcm_server_submit  colptr[ncols+1], rowind[nnz]: HOST inputs;
 *                      cmatch[ncols], rmatch[nrows]: HOST outputs.  All four
 *                      must stay valid until the request is polled done
 *                      (pinned memory makes the copies asynchronous).
 *                      Returns a ticket > 0, MCM_ENOMEM if the request alone
 *                      exceeds the budget, MCM_EINVAL for bad arguments.
 *   mcm_server_poll    waits up to wait_ms (0 = no wait) for the ticket;
 *                      returns 1 (done: outputs written, *info filled, the
 *                      ticket is released), 0 (not yet) or a negative status
 *   mcm_server_stats_get  counters of the server
 *   mcm_server_destroy    stops the worker; outstanding requests are dropped
 * Times in mcm_request_info are milliseconds since the server was created.
 */
typedef struct mcm_server mcm_server;

typedef struct {
    int64_t card;        /* |M| */
    double submit_ms;    /* request submitted */
    double admit_ms;     /* memory granted, input copy started */
    double start_ms;     /* its launch was queued */
    double done_ms;      /* results on the host */
    int32_t path;        /* 0 batched launch (one workgroup), 1 whole device */
    int32_t batch_size;  /* requests in the same launch */
} mcm_request_info;

typedef struct {
    int64_t submitted, completed, rejected, queued, in_flight;
    int64_t bytes_in_use, peak_bytes, budget_bytes;
    int64_t launches_batched, launches_grid, max_batch_seen;
} mcm_server_stats;

int64_t mcm_server_create(int64_t hbm_budget_bytes, int32_t max_batch, mcm_server **server);
int64_t mcm_server_submit(mcm_server *server, int32_t ncols, int32_t nrows, const int32_t *colptr,
                          const int32_t *rowind, int32_t *cmatch, int32_t *rmatch);
int64_t mcm_server_poll(mcm_server *server, int64_t ticket, mcm_request_info *info, double wait_ms);
int mcm_server_stats_get(mcm_server *server, mcm_server_stats *out);
int mcm_server_destroy(mcm_server *server);

/*
 * mcm_konig_cover -- minimum vertex cover certifying a maximum matching
 * (Konig's theorem; section 2 states the Berge criterion it rests on).
 * Runs one complete alternating BFS from every unmatched column (GPUBFS,
 * no early exit).  If it reaches an unmatched row the matching is not
 * maximum and MCM_ENOTMAX is returned.  Otherwise, with Z_C the reached
 * columns: col_in_cover[c] = 1 iff c is matched and not in Z_C, and
 * row_in_cover[r] = 1 iff r is adjacent to Z_C.
 *
 *   cmatch, rmatch      device, a matching of the graph (not modified)
 *   col_in_cover        [ncols] device uint8 output
 *   row_in_cover        [nrows] device uint8 output
 * Returns |K| (equal to |M|) or a negative mcm_status.
 */
int64_t mcm_konig_cover(int32_t ncols, int32_t nrows, const int32_t *colptr, const int32_t *rowind,
                        const int32_t *cmatch, const int32_t *rmatch,
                        uint8_t *col_in_cover, uint8_t *row_in_cover, void *stream);

/*
 * mcm_bfs_levels -- one complete alternating BFS phase from every unmatched
 * column of the given matching, without early exit and without
 * augmentation (the level sets that GPUBFS of Algorithm 2 builds one
 * launch per level).  Inspection and testing aid.
 *
 *   col_level  [ncols] device output: BFS level of each column (unmatched
 *              columns 0, a column reached through its matched row one more
 *              than the column that reached that row), -1 if not reached
 *   row_pred   [nrows] device output: the column that reached each row
 *              (one of several when several columns of the same level are
 *              adjacent), -1 if not reached
 * Returns the number of unmatched rows reached, or a negative mcm_status.
 */
int64_t mcm_bfs_levels(int32_t ncols, int32_t nrows, const int32_t *colptr, const int32_t *rowind,
                       const int32_t *cmatch, const int32_t *rmatch,
                       int32_t *col_level, int32_t *row_pred, void *stream);

/*
 * mcm_bfs_forest -- one complete BFS phase of the form mcm_match would run
 * (GPUBFS-WR of Algorithm 4 by default, GPUBFS of Algorithm 2 with option
 * "bfs" "plain"), without augmentation and strictly level-synchronous (one
 * BFS level per grid level), from every unmatched column of the given
 * matching.  It exposes the forest the phase grows, for inspection and for
 * checking the GPUBFS-WR invariants: with the early exit, a tree whose root
 * has found an unmatched row stops growing one level later, the columns
 * reached are a subset of those GPUBFS reaches, and every column's root is
 * the root of the column that reached its matched row.  The options
 * "endpoints" ("one": one end per root), "claim" ("max"), "flush"
 * ("defer") and "wr_check" select the same forms as for mcm_match ("auto"
 * means the plain default here).
 *
 *   col_level  [ncols] device output: the level at which each column
 *              entered the BFS (0 for unmatched columns), -1 if not reached
 *   col_root   [ncols] device output: the unmatched column at the root of
 *              its tree (itself for an unmatched column), -1 if not reached
 *   row_pred   [nrows] device output: the column that claimed each row,
 *              -1 if not reached
 *   ends       [nrows] device output: the unmatched rows reached that
 *              Alternate would start from, in the first entries
 * Returns the number of ends, or a negative mcm_status.
 */
int64_t mcm_bfs_forest(int32_t ncols, int32_t nrows, const int32_t *colptr, const int32_t *rowind,
                       const int32_t *cmatch, const int32_t *rmatch,
                       int32_t *col_level, int32_t *col_root, int32_t *row_pred, int32_t *ends,
                       void *stream);

/*
 * mcm_cheap_init_host -- the greedy initial matching that precedes every
 * run in the paper's experiments (section 4): columns in index order, each
 * takes the first row of its stored adjacency that is still unmatched.
 * HOST arrays; cmatch[ncols] and rmatch[nrows] are overwritten.
 * Returns |M0| or MCM_EINVAL.
 */
int64_t mcm_cheap_init_host(int32_t ncols, int32_t nrows, const int32_t *colptr, const int32_t *rowind,
                            int32_t *cmatch, int32_t *rmatch);

/*
 * mcm_set_option / mcm_get_option -- process-wide settings (strings).
 *   "driver"    "apfb" (default) | "apsb"      Algorithm 1 with or without
 *                                              the stop at the first level
 *                                              that finds an unmatched row
 *   "bfs"       "wr" (default) | "plain"       GPUBFS-WR (Algorithm 4) or
 *                                              GPUBFS (Algorithm 2)
 *   "endpoints" "auto" (default) | "one" | "all"
 *                                              with WR: Alternate starts
 *                                              from one reached unmatched
 *                                              row per root (the first), or
 *                                              from all of them; auto = one
 *                                              under APsB, all under APFB
 *                                              (section 3, the improvement
 *                                              of GPUBFS-WR with root and
 *                                              bfs_array)
 *   "mapping"   "auto" (default) | "thread" | "wave"
 *                                              frontier column per lane, or
 *                                              edges of 64 columns balanced
 *                                              across a wavefront
 *   "loop"      "auto" (default) | "device" | "host"
 *                                              BFS level loop in one
 *                                              persistent launch with grid
 *                                              barriers, or one launch per
 *                                              level
 *   "claim"     "auto" (default) | "max" | "probe"
 *                                              how a BFS claims a row (the
 *                                              visited check of Algorithm 2,
 *                                              made atomic): one 64-bit
 *                                              atomic maximum of the phase
 *                                              stamp, or a load of the row
 *                                              word then a compare-and-swap
 *                                              (fewer atomics on rows with
 *                                              many edges); auto = max when
 *                                              the graph has at most 8 edges
 *                                              per row on average.  mcm_match
 *                                              above the one-workgroup size
 *                                              only; max keeps 8 bytes per
 *                                              row more workspace
 *   "flush"     "auto" (default) | "defer" | "atomic"
 *                                              how a level of the persistent
 *                                              loop reserves its next
 *                                              frontier: with the counter
 *                                              barrier's own addition, the
 *                                              entries written after
 *                                              arriving and checked by their
 *                                              readers, and the barriers
 *                                              between two such levels
 *                                              without memory fences (defer;
 *                                              needs "barrier" "counter"), or
 *                                              with one queue atomic per
 *                                              workgroup before arriving;
 *                                              auto = defer when the graph
 *                                              has at most 8 edges per row
 *                                              on average
 *   "wr_check"  "auto" (default) | "early" | "late"
 *                                              where GPUBFS-WR tests whether
 *                                              an entry's root already has a
 *                                              path (wave mapping): before
 *                                              the entry's edges are read,
 *                                              or beside each edge visit;
 *                                              auto = late for graphs with
 *                                              at most 8 edges per row on
 *                                              average, early otherwise
 *                                              (late outside mcm_match)
 *   "alternate" "auto" (default) | "fast" | "classic"
 *                                              mcm_match's Alternate
 *                                              (Algorithm 3): a claim also
 *                                              records the row that held the
 *                                              claiming column, so a walk
 *                                              step loads pred and that row
 *                                              together (fast; walks that
 *                                              share a way to the root flip
 *                                              it alike and FixMatching
 *                                              settles their junction), or
 *                                              reads cmatch after pred and
 *                                              stops where another walk
 *                                              passed (classic, as printed);
 *                                              auto = fast with GPUBFS-WR
 *                                              on graphs with at most 8
 *                                              edges per row on average,
 *                                              classic otherwise
 *   "local_levels" "auto" (default) | "0".."16" levels of mcm_match's
 *                                              persistent loop (not the
 *                                              multi-graph launch of
 *                                              batches and the server): a
 *                                              wavefront expands the
 *                                              columns it has just reached
 *                                              (its newest 64 staged entries)
 *                                              up to this many times more
 *                                              before the grid barrier, so a
 *                                              barrier covers several BFS
 *                                              layers of such chains; 0 =
 *                                              strictly level-synchronous as
 *                                              in Algorithm 1 (BFS trees are
 *                                              then shortest-path trees; the
 *                                              matching is maximum either
 *                                              way); auto = 16 with probe
 *                                              claims, 6 with atomic-maximum
 *                                              claims
 *   "local_edges" "1024" (default) | "0".."1048576"
 *                                              a local level takes only the
 *                                              newest staged entries whose
 *                                              edges add up to at most this
 *                                              many (at least one entry); the
 *                                              rest wait for the next grid
 *                                              level, where every wavefront
 *                                              shares them; 0 = the newest 64
 *   "roots"     "auto" (default) | "list" | "scan"
 *                                              mcm_match's root scan of a
 *                                              phase: every column (scan),
 *                                              or only the previous phase's
 *                                              roots, listed as they are
 *                                              found (a matched column never
 *                                              becomes unmatched); auto =
 *                                              the list while the previous
 *                                              phase had at most ncols/16
 *                                              roots, else every column
 *   "fix"       "auto" (default) | "list" | "scan"
 *                                              mcm_match's FixMatching:
 *                                              every row (scan), or only the
 *                                              rows the walks of the phase
 *                                              wrote or stopped at (list;
 *                                              every row when more rows were
 *                                              reported than nrows); auto =
 *                                              the list in phases that found
 *                                              at most nrows/64 ends
 *   "schedule"  "levels" (default) | "async" | "auto"
 *                                              mcm_match's BFS under APFB:
 *                                              level-synchronous, or
 *                                              level-free (one phase-long
 *                                              queue, no grid barrier between
 *                                              levels; measured slower, see
 *                                              the design notes); auto =
 *                                              levels
 *   "keep", "take"  "128", "64" (defaults)     level-free BFS: entries a
 *                                              wavefront keeps before
 *                                              handing older ones on (1..192),
 *                                              and expands per step (1..64)
 *   "validate"  "0" (default) | "1"            check CSC and init on device
 *   "stats"     "0" (default) | "1"            count scanned edges etc.
 *   "tuning"    path of an autotuner cache file (JSON lines) or ""
 *   "autotune"  "0" (default) | "1"            batch plans time candidates
 *   "fuse"      "on" (default) | "off"         mcm_match with probe claims: a
 *                                              phase that does not list its
 *                                              roots expands them (BFS level
 *                                              0) as its root scan finds
 *                                              them, instead of enqueueing
 *                                              them for a level of their own
 *   "wg_lds"    "on" (default) | "off"         mcm_match's one-workgroup path
 *                                              (graphs with ncols + nrows at
 *                                              most wg_threshold) keeps the
 *                                              pattern, row words and
 *                                              per-vertex state in the
 *                                              workgroup's LDS when they fit
 *                                              there (4 (ncols + 1) + 4 nnz +
 *                                              12 nrows + 8 ncols bytes, up to
 *                                              what the LDS staging leaves)
 *   "block", "blocks_per_cu", "wg_block", "wg_threshold", "small_max",
 *   "batch_min", "split", "timeout_s", "max_blocks", "level_entries",
 *   "idle_sleep", "barrier", "multi_threshold", "multi_group"
 *                                              launch-shape details (see
 *                                              the host driver)
 * Return MCM_OK or MCM_EINVAL (unknown key or value).  mcm_get_option
 * writes the current value into buf (NUL-terminated, truncated to len).
 */
int mcm_set_option(const char *key, const char *value);
int mcm_get_option(const char *key, char *buf, int32_t len);

/*
 * mcm_last_phases -- the per-phase record of the last mcm_match call on this
 * process that ran with option "stats" = "1" on the device-loop or
 * host-loop path (graphs above the one-workgroup size): for phase i,
 * levels[i] = BFS levels expanded and ends[i] = unmatched rows reached
 * (augmenting-path ends; 0 in the last phase, whose complete BFS found
 * none).  This is the per-iteration view the paper plots for its variants
 * (section 4, the figure of BFS levels per iteration).
 *
 *   levels, ends   HOST [cap] arrays (may be NULL when cap == 0)
 *   cap            entries to write at most (>= 0)
 *
 * Returns the number of phases recorded (at most 4096; it may exceed cap),
 * 0 if the last call kept no record, or MCM_EINVAL.
 */
int64_t mcm_last_phases(int32_t *levels, int32_t *ends, int64_t cap);

/* Counters of the last mcm_match / mcm_match_batched call on this process. */
typedef struct {
    int64_t phases;          /* phases run, including the last one that found nothing */
    int64_t levels;          /* BFS levels expanded, summed over phases */
    int64_t edges_scanned;   /* adjacency entries read by BFS (stats=1) */
    int64_t cols_expanded;   /* frontier columns expanded (stats=1) */
    int64_t cols_claimed;    /* columns inserted into a next frontier (stats=1) */
    int64_t rows_found;      /* unmatched rows reached, summed over phases (stats=1) */
    int64_t alt_steps;       /* Alternate loop iterations (stats=1) */
    int64_t fix_resets;      /* rows reset by FixMatching (stats=1) */
    int64_t roots;           /* frontier roots enqueued, summed over phases (stats=1) */
    double  t_expand_ms;     /* block 0 of the persistent launch (stats=1): expanding levels, */
    double  t_flush_ms;      /*   handing staged queue entries over, */
    double  t_barrier_ms;    /*   waiting in grid barriers, */
    double  t_small_ms;      /*   running single-workgroup levels, */
    double  t_augment_ms;    /*   in Alternate and FixMatching */
    int64_t init_card;       /* |M| of the initial matching (mcm_match; -1 after a batched call) */
    int64_t card;            /* |M| returned */
    double  kernel_ms;       /* device time of the matching, HIP events */
    int32_t loop;            /* 0 = device-side level loop, 1 = host-side */
    int32_t mapping;         /* 0 = thread, 1 = wave */
    int64_t claims_tried;    /* compare-and-swaps on rows the probe saw unreached (stats=1);
                                claims_tried - cols_claimed - rows_found were lost to another lane;
                                with claim = max: atomic maxima on rows not yet stamped */
    int32_t claim;           /* row claims used: 0 = probe + compare-and-swap, 1 = atomic maximum */
    int32_t flush;           /* grid levels: 0 = queue atomic, 1 = deferred (counter barrier) */
    int32_t wr_check;        /* GPUBFS-WR root test: 0 = before the scan, 1 = beside each edge visit */
    int32_t alternate;       /* Alternate: 0 = classic, 1 = along the rows recorded at the claims */
    int64_t pass_bytes;      /* per-phase passes under the fixed byte model (stats=1): 4 B and 1/8 B per
                                column the root scan reads, 8 B per row FixMatching reads */
    int32_t schedule;        /* BFS of mcm_match: 0 = level-synchronous, 1 = level-free */
    int32_t local_levels;    /* local levels of the device loop's grid levels (0 on other paths) */
} mcm_stats;

int mcm_last_stats(mcm_stats *out);

/* Message for a status code, or the calling thread's last error message. */
const char *mcm_strerror(int64_t status);

/* Library version string. */
const char *mcm_version(void);

/*
 * mcm_shutdown -- releases everything the library holds on every device:
 * workspaces, pinned host buffers, events, and the batch plans and request
 * servers the caller has not destroyed (a later destroy call on such a
 * handle does nothing).  Call it before the process tears down the HIP
 * runtime (the Python binding registers it with atexit).  The library may
 * be used again afterwards; it allocates anew.  Returns MCM_OK.
 */
int mcm_shutdown(void);

#ifdef __cplusplus
}
#endif
#endif /* MCM_H */
