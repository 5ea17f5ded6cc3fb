/*
 * bpida.h -- Block-Parallel IDA* on AMD Instinct MI355X (gfx950).
 *
 * Method: Horie & Fukunaga, "Block-Parallel IDA* for GPUs" (SoCS 2017),
 * Alg. 1 (BPIDA* and BPDFS) with the all-optimal-solutions completion of the
 * final f-limited iteration (Sec. 6.1).  The domain is the sliding-tile
 * puzzle with the Manhattan distance heuristic (Sec. 1, Sec. 3).  All search
 * work runs in HIP kernels: ingest (validate, pack, h), root split
 * (CreateRootSet), the block-parallel f-limited DFS (BPDFS: one subtree per
 * workgroup, the DFS stack in LDS, one wavefront expanding per round either
 * 16 nodes x 4 moves, Alg. 1's thread-to-action map, or 64 nodes, one per
 * lane with its four moves, the batched default) and the per-limit reduction
 * of node counts and next limits.
 *
 * Conventions shared by every entry point:
 *   - a state is width*width bytes, row-major; byte p is the tile at cell p,
 *     0 is the blank; the goal holds tile p at cell p;
 *   - moves are blank moves U, L, R, D, unit cost; a move that undoes the
 *     one that produced a node is not generated (parent pruning);
 *   - h = Manhattan distance of the non-blank tiles;
 *   - the f-limits are h0, h0+2, ... (Manhattan changes by exactly 1 per
 *     move and keeps the parity of the path length, so no other limit can
 *     occur); the final limit, the optimal length, is searched to completion
 *     so that every count is unique (unless the first_solution option asks
 *     for Alg. 1's stop at the first goal).
 *
 * Thread safety: calls may come from several host threads; they are
 * serialised inside the library (one shared device workspace per device).
 * Errors never abort and no C++ exception crosses this interface.
 */
#ifndef BPIDA_H
#define BPIDA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Columns of the per-limit node-count matrix: limit h0 + 2j goes in column j. */
#define BPIDA_MAX_THRESHOLDS 64

/* Board widths: 3 (8-puzzle), 4 (15-puzzle), 5 (24-puzzle).  The batched
 * mode takes all three (4 bits per tile for 3x3 and 4x4, 5 bits for 5x5);
 * the plain mode and the server take width 4 only. */
#define BPIDA_MIN_WIDTH 3
#define BPIDA_MAX_WIDTH 5

enum bpida_status {
  BPIDA_OK = 0,
  BPIDA_EINVAL = -1,      /* bad argument, or a state that is not a permutation */
  BPIDA_EUNSOLVABLE = -2, /* permutation parity and blank parity disagree       */
  BPIDA_ELIMIT = -3,      /* more than BPIDA_MAX_THRESHOLDS limits, or past the
                             max_threshold option; counts of the limits that
                             were completed are kept                            */
  BPIDA_ENOMEM = -4,      /* device allocation failed, a per-workgroup spill
                             area (plain) or the work queue (batched) overflowed */
  BPIDA_EDEVICE = -5,     /* no usable gfx950 device, or a HIP call failed      */
  BPIDA_EINTERNAL = -6,   /* a consistency check failed (next limit != L + 2),
                             or a persistent launch stopped by its watchdog or
                             time budget                                        */
  BPIDA_EAGAIN = -7,      /* server: the request ring is full; retry later     */
};

/*
 * Solve n_instances puzzles given in host memory (BPIDA*, Alg. 1).
 *
 * states     host, n_instances * width * width bytes (layout above).
 * width      side of the board: 3, 4 or 5 (batched mode), 4 (plain mode;
 *            another width is BPIDA_EINVAL there).
 * out_len    host, n_instances int32: optimal solution length, or -1 for an
 *            instance that is invalid, unsolvable or stopped by a limit.
 * out_nodes_per_threshold
 *            host, n_instances * BPIDA_MAX_THRESHOLDS uint64, row-major:
 *            [i][j] = nodes expanded by the f-limited iteration with limit
 *            h0(i) + 2j (start, interior and goal nodes included); columns
 *            past instance i's last completed limit are 0.
 * Returns BPIDA_OK if every instance was solved, otherwise the first negative
 * code met in instance order; the other instances are still solved.  Argument
 * errors (null pointers, n_instances < 0, unsupported width) are reported
 * before any device work and leave the outputs untouched.  Synchronous.  The
 * caller owns all buffers; nothing is retained after return.
 */
int bpida_solve(const uint8_t *states, int32_t n_instances, int32_t width, int32_t *out_len,
                uint64_t *out_nodes_per_threshold);

/* Bytes per returned path: moves of the blank, U, L, R, D = 0..3, one per
 * byte, 0xFF past the path's end. */
#define BPIDA_MAX_PATH 256

/*
 * As bpida_solve (batched mode, one board width) plus one optimal path per
 * instance: Alg. 1's BPDFS returns the goal "and its parents as a shortest
 * path".  out_path: host, n_instances * BPIDA_MAX_PATH bytes; row i holds
 * out_len[i] moves of the blank (U, L, R, D = 0..3) leading from state i to
 * the goal, then 0xFF (all 0xFF for an instance that is invalid, unsolvable,
 * capped, or already the goal).  The path is the lexicographically smallest
 * optimal move sequence (U < L < R < D), so it is unique: the first goal a
 * sequential depth-first search in that move order meets at the optimal
 * limit.  It is rebuilt after the solve by exact-limit probes: per move, each
 * legal child of the current state is searched at the single limit "moves
 * left - 1" (first goal only), and the first child that reaches the goal is
 * taken; the probes of all instances run in one batched launch per move.
 * out_len and out_nodes_per_threshold are those of bpida_solve (all optimal
 * solutions in the final limit unless the first_solution option is set).
 * Return value as bpida_solve; BPIDA_EINTERNAL if some probe round found no
 * child one step closer (never expected).  Synchronous.
 */
int bpida_solve_paths(const uint8_t *states, int32_t n_instances, int32_t width, int32_t *out_len,
                      uint64_t *out_nodes_per_threshold, uint8_t *out_path);

/*
 * As bpida_solve_paths with every buffer in device memory of the current
 * device (d_path: n * BPIDA_MAX_PATH bytes), ordered on `hip_stream`; returns
 * after the results are in place (one host read of the lengths between the
 * solve and the probes, and one at the end).
 */
int bpida_solve_paths_device(const uint8_t *d_states, int32_t n_instances, int32_t width,
                             int32_t *d_len, uint64_t *d_nodes, uint8_t *d_path, void *hip_stream);

/*
 * As bpida_solve for a batch that mixes board widths, always in batched mode
 * (one persistent launch for all of them).  widths: host, n int32 in 3..5.
 * states: host, the instances' bytes back to back (instance i takes
 * widths[i]^2 bytes).  Outputs as in bpida_solve.  5x5 instances need an LDS
 * stack of at least 1024 entries (the default), 3x3 of 256, 4x4 of 512 with
 * 64-node rounds; a smaller one is BPIDA_EINVAL.
 */
int bpida_solve_mixed(const uint8_t *states, const int32_t *widths, int32_t n_instances,
                      int32_t *out_len, uint64_t *out_nodes_per_threshold);

/*
 * As bpida_solve_mixed with the states and outputs in device memory of the
 * current device (d_states: the instances' bytes back to back; d_len, d_nodes
 * as in bpida_solve_device) and the widths in host memory (n int32 in 3..5;
 * the host lays out the split trees from them).  Work is ordered on
 * `hip_stream` (NULL = the null stream); returns after the results are in
 * d_len and d_nodes, with the first failing status in instance order.
 */
int bpida_solve_mixed_device(const uint8_t *d_states, const int32_t *widths, int32_t n_instances,
                             int32_t *d_len, uint64_t *d_nodes, void *hip_stream);

/*
 * As bpida_solve, with every buffer in device memory of the current device:
 * d_states (n * width * width bytes), d_len (n int32), d_nodes
 * (n * BPIDA_MAX_THRESHOLDS uint64).  Validation runs on the device; the
 * per-instance status is written to d_len (-1) and the return value is the
 * first failing code.  Work is ordered on `hip_stream` (a hipStream_t, NULL =
 * the null stream); the call returns after the results are in d_len and
 * d_nodes (plain mode: the limit loop reads 16 bytes per limit back to the
 * host; batched mode: one read of the per-instance status after the launch).
 */
int bpida_solve_device(const uint8_t *d_states, int32_t n_instances, int32_t width,
                       int32_t *d_len, uint64_t *d_nodes, void *hip_stream);

/*
 * Enqueue a batched solve (mode option ignored: always the persistent
 * launch) on `hip_stream` and return without waiting: no host
 * synchronisation and no copy to the host, so the call can be recorded into a
 * HIP graph and replayed.  Buffers as in bpida_solve_device, plus d_status
 * (device, n int32): 1 = solved, otherwise a negative bpida_status for that
 * instance (a queue overflow marks every instance BPIDA_ENOMEM).  The
 * library's device workspace is sized on the first call for a given n and
 * options and then reused; a call that would have to grow it while the stream
 * is capturing returns BPIDA_EINVAL (make one uncaptured call first).
 * Returns BPIDA_OK once the work is enqueued, or an argument/device error.
 * Concurrent solves on one device share the workspace: calls are serialised,
 * but enqueued work from two calls must not overlap on different streams.
 */
int bpida_solve_device_async(const uint8_t *d_states, int32_t n_instances, int32_t width,
                             int32_t *d_len, uint64_t *d_nodes, int32_t *d_status,
                             void *hip_stream);

/*
 * As bpida_solve_device_async, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The call allocates nothing: every buffer the solve
 * needs besides the caller's inputs and outputs (ingested states, split
 * tree, interior histograms, work queue, per-instance search state) is
 * carved from one fixed device array of BPIDA_NOALLOC_SCRATCH_BYTES per
 * GPU, which the library holds until the process ends.  Buffers, options,
 * ordering and d_status as in bpida_solve_device_async (batched mode, one
 * board width).  The work queue sized from the batch is shrunk to fit the
 * array when needed (not below the seeds plus 1024 chunks; a queue_capacity
 * option is kept as set); a queue that then overflows marks every instance
 * BPIDA_ENOMEM in d_status.  Returns BPIDA_ENOMEM, before any device work,
 * if the batch's buffers do not fit (e.g. 4096 4x4 instances fit at the
 * default split depth 6, about 1500 at depth 8).  Every call on one GPU
 * shares that GPU's array: two calls whose enqueued work overlaps in time
 * (on two streams with no ordering between them) race and give wrong
 * results; order them on one stream.  The array keeps the last call's
 * contents; each call initialises everything it reads.
 */
#define BPIDA_NOALLOC_SCRATCH_BYTES (128u << 20)
int bpida_solve_device_noalloc(const uint8_t *d_states, int32_t n_instances, int32_t width,
                               int32_t *d_len, uint64_t *d_nodes, int32_t *d_status,
                               void *hip_stream);

/*
 * Continuous-batching server (one per process).  bpida_server_start launches
 * a persistent search kernel on `hip_stream` (NULL: a stream of the
 * library's own) and returns at once; the kernel keeps running, admitting
 * requests as they arrive, until bpida_server_stop.  Requests travel through
 * a ring of `ring_capacity` slots (rounded up to a power of two, >= 64) in
 * pinned host memory; at most `max_inflight` requests are searched at the
 * same time (each holds a device slot: split tree, counts, outputs), and a
 * request that arrives while others are on the GPU is admitted as soon as a
 * slot frees and the queued frontier is within its budget (option
 * admit_backlog), its subtrees sharing the work queue with theirs.  Options
 * (split depth, nodes per round, ring capacity, grid size, budget_ms) are
 * read at start.  The launch ends when the host has asked to stop and every
 * admitted request is answered, or after budget_ms.
 */
int bpida_server_start(int32_t width /* 4 */, int32_t max_inflight, int32_t ring_capacity,
                       void *hip_stream);

/*
 * Queue one start state (host, width*width bytes).  Writes the request's
 * ticket.  Returns BPIDA_OK, BPIDA_EAGAIN if the ring holds ring_capacity
 * requests whose results have not been collected yet, or BPIDA_EINVAL.
 * Invalid or unsolvable states are answered with that status.
 */
int bpida_server_submit(const uint8_t *state, uint64_t *ticket);

/*
 * Collect the answer of `ticket`: returns 1 and fills out_len, out_nodes
 * (host, BPIDA_MAX_THRESHOLDS uint64 as in bpida_solve) and status (1 solved,
 * else a negative bpida_status; BPIDA_ENOMEM if the work queue overflowed
 * while this request was searched, its length then -1) once it is ready; 0 while it is pending;
 * BPIDA_EINVAL for an unknown or already collected ticket.  Answers stay
 * readable after bpida_server_stop until the next bpida_server_start.
 */
int bpida_server_poll(uint64_t ticket, int32_t *out_len, uint64_t *out_nodes, int32_t *status);

/*
 * Ask the server to finish, wait until every admitted request is answered
 * and the launch has ended.  Returns BPIDA_OK, or the run's error
 * (BPIDA_ENOMEM: work queue overflow; BPIDA_EINTERNAL: time budget spent).
 */
int bpida_server_stop(void);

/*
 * Set a tuning or control option for subsequent calls (process-wide).
 *   "mode"               1 = batched (default): one persistent launch searches
 *                        all instances through all limits from a device work
 *                        queue with work donation between workgroups and
 *                        the limit advanced on the device; 0 = plain: Alg. 1
 *                        as printed, one search launch per instance and limit,
 *                        one subtree root per workgroup, no balancing
 *   "frontier_depth"     depth D of the root split, 0..16, or -1 (default):
 *                        10 in plain mode, 6 in batched mode
 *   "lds_stack_capacity" DFS stack entries per workgroup in LDS: 128, 256,
 *                        512, 640, 672, 768, 1024 or 2048, or -1 (default): 512
 *                        for 16-node rounds, 1024 for 64-node rounds (64-node
 *                        rounds need at least 512 on 4x4 and 1024 on 5x5, 256
 *                        on 3x3; 640, 672 and 768 only for batched 64-node
 *                        rounds with one-wave workgroups, where they let 24,
 *                        20 and 20 waves share a compute unit instead of 16;
 *                        at 672 the 4x4 stack interleaves each entry's state
 *                        and meta word, one instruction less per child; other
 *                        combinations are BPIDA_EINVAL at solve time); deeper
 *                        entries spill to HBM (plain) or to the work queue
 *                        (batched).  A smaller stack spills more: with 512
 *                        entries, batches of thousands of 4x4 instances can
 *                        overflow the default work queue (BPIDA_ENOMEM)
 *   "nodes_per_round"    batched mode: 64 (default) pops one node per lane and
 *                        each lane tries the four moves; 16 uses Alg. 1's map
 *                        (lane l expands node l/4 with move l%4).
 *   "wg_size"            batched mode and server: threads per workgroup of the
 *                        persistent kernel, 64 (default), 128 or 256: 1, 2 or
 *                        4 waves, each with its own LDS stack, taking its own
 *                        work and never waiting for the others (Sec. 5's
 *                        block = one warp, several per workgroup); 128 and 256
 *                        need 64-node rounds and a stack of 512+ entries.
 *                        Results do not depend on it.
 *   "plain_nodes_per_round"
 *                        plain mode: 16 (default, Alg. 1's map) or 64 (the
 *                        batched kernel's round: one node per lane; needs an
 *                        LDS stack of at least 512 entries, default 1024)
 *   "spill_capacity"     plain mode: per-workgroup HBM spill entries, a
 *                        multiple of 64 (default 16384)
 *   "queue_capacity"     batched mode: queue slots of 64 entries (rounded up
 *                        to a power of two, at least 64; 0 = sized from the
 *                        batch); a queue that stays full while a workgroup
 *                        pushes makes the call return BPIDA_ENOMEM
 *   "watchdog_ms"        batched mode: an idle workgroup that sees no work
 *                        queue activity for this long while instances remain
 *                        stops and the call returns BPIDA_EINTERNAL (default
 *                        20000)
 *   "budget_ms"          batched mode: every workgroup of the persistent launch
 *                        stops after this long and the call returns
 *                        BPIDA_EINTERNAL (default 600000)
 *   "max_workgroups"     cap on the persistent search grid (0 = occupancy)
 *   "max_threshold"      stop with BPIDA_ELIMIT before a limit above this
 *                        (-1 = none, default)
 *   "donate_every"       batched mode: rounds between a workgroup's checks
 *                        for waiting workgroups to donate to (a power of
 *                        two in 4..1024, default 128)
 *   "start_threshold"    first f-limit to search: -1 (default) = h0; else the
 *                        smallest h0 + 2j >= the value.  Columns of skipped
 *                        limits stay 0.  out_len is then the first searched
 *                        limit that holds a goal: the optimal length only if
 *                        the start does not exceed it.
 *   "static_lb"          plain mode: 1 (default) re-splits, between limits, every
 *                        root whose repetition count exceeded the average of
 *                        the searched roots (Sec. 5, BPIDA*'s static load
 *                        balancing): it is replaced by the nodes of its
 *                        subtree at the first depth holding at least
 *                        load / average of them (at most 64); 0 keeps the
 *                        root set of the split.  Counts are exact either way.
 *   "first_solution"     0 (default): the final limit runs to completion (all
 *                        optimal solutions, Sec. 6.1), so every count is
 *                        unique.  1: the final limit stops at its first goal
 *                        (Alg. 1 as printed): out_len and the counts of the
 *                        earlier limits are unchanged; the final column
 *                        holds the nodes expanded before the search stopped
 *                        (at most the all-solutions count, and it varies
 *                        from run to run).
 *   "seed_chunk"         batched mode: roots per chunk when a limit is seeded
 *                        into the work queue: 8, 16, 32 or 64 (default)
 *   "queue_chunk"        batched mode: entries per donated chunk, 16, 32 or
 *                        64 (default); a donation splits the oldest
 *                        2 x queue_chunk entries of the donor's stack
 *                        alternately.  Overflow spills always move 64.
 *   "donate_min"         batched mode: smallest LDS stack (entries) that
 *                        donates (2..2048; -1 = four rounds' worth of pops,
 *                        at most half the stack: 256 for 64-node rounds, the
 *                        default).  Too small a value ships pieces of work
 *                        that cost more to move than they hold; one the stack
 *                        seldom reaches stops donation altogether.
 *   "admit_backlog"      server: the HBM frontier budget of admission.  A
 *                        request is admitted only while at most this many
 *                        chunks of 64 entries wait in the work queue beyond
 *                        the workgroups waiting for work (-1, the default:
 *                        half the queue's slots; 0: no limit), besides the
 *                        instance-slot budget max_inflight
 *   "push_spin"          batched mode and server: polls (of about 64 clocks
 *                        each) a push waits for a full work-queue slot before
 *                        it gives up and the pushed entries are lost (1..2^24,
 *                        default 65536).  A small value makes a full queue
 *                        lose work at once: a batched call then reports
 *                        BPIDA_ENOMEM, and the server answers each request
 *                        that lost work with status BPIDA_ENOMEM (never with
 *                        counts short of the true ones) and keeps serving.
 * Returns BPIDA_OK, or BPIDA_EINVAL for an unknown key or a bad value.
 */
int bpida_set_option(const char *key, int64_t value);

/* Current value of an option, or INT64_MIN for an unknown key. */
int64_t bpida_get_option(const char *key);

/*
 * Statistics of the last completed solve call on this process:
 *   out[0] search rounds (pop-expand-push cycles, the repetitions of BPDFS's
 *          loop), summed over workgroups and limits
 *   out[1] nodes expanded by the search kernel (interior split nodes excluded)
 *   out[2] entries moved from LDS to HBM (plain: spills; batched: donated
 *          or spilled chunks x 64)
 *   out[3] search-kernel launches
 *   out[4] search-kernel time in microseconds (device events, summed)
 *   out[5] plain mode: largest per-workgroup spill stack seen, in entries;
 *          batched mode: most chunks queued at once (seen at a push)
 *   out[6] batched mode: chunks pushed to the work queue (seeds excluded)
 *   out[7] batched mode: chunks popped from the work queue
 *   out[8..10] batched mode: microseconds summed over workgroups spent
 *          searching, taking work from the queue, and idle
 *   out[11] batched mode: donations made because workgroups were idle
 *   out[12] batched mode: workgroups in the persistent grid
 *   out[13] batched mode: error bits (1 queue full while seeding, 2 entries
 *          dropped, 4 idle watchdog, 8 deadline, 16 queue ring full,
 *          32 LDS stack overrun, 256 split check)
 *   out[14] batched mode: work-queue slots (chunks of 64 entries)
 *   out[15] plain mode: roots added by the static load balancing
 *   out[16] split-tree roots read (once per root and searched limit: the
 *          algorithmic HBM reads of the search, 16 bytes each)
 *   out[17] batched mode: 5x5 chunks taken from the work queue
 * n = number of slots to fill (<= 20).  Returns BPIDA_OK or BPIDA_EINVAL.
 */
int bpida_last_stats(uint64_t *out, int32_t n);

/* Static, human-readable text for a status code. */
const char *bpida_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* BPIDA_H */
