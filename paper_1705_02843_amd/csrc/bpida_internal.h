// bpida_internal.h -- layouts shared by the library's host driver and kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include <algorithm>

namespace bpida {

// ---------------------------------------------------------------------------
// 15-puzzle encoding (width 4).
//   tiles: 16 nibbles, nibble p (bits 4p..4p+3) = tile at cell p.
//   goal:  tile p at cell p.
//   moves: blank moves U=0 (-4), L=1 (-1), R=2 (+1), D=3 (+4); inverse 3-a.
// ---------------------------------------------------------------------------
constexpr uint64_t kGoal4 = 0xFEDCBA9876543210ull;

// Bit 4*b + a is set iff move a keeps a blank at cell b on the board.
constexpr uint64_t make_move_mask4() {
  uint64_t m = 0;
  for (int b = 0; b < 16; ++b) {
    const int r = b >> 2, c = b & 3;
    if (r > 0) m |= 1ull << (4 * b + 0);
    if (c > 0) m |= 1ull << (4 * b + 1);
    if (c < 3) m |= 1ull << (4 * b + 2);
    if (r < 3) m |= 1ull << (4 * b + 3);
  }
  return m;
}
constexpr uint64_t kMoveMask4 = make_move_mask4();

// Manhattan delta table (Sec. 3 heuristic, applied incrementally).  Move a
// slides the tile t standing at the blank's neighbour n into the blank's
// cell b.  Only one coordinate of t changes: its row for U/D, its column
// for L/R.  With ct = that coordinate of t's goal cell (= of t) and cn = that
// coordinate of n, the tile's distance grows by one iff it moves away from
// its goal coordinate, otherwise it shrinks by one.  Bits 16a + 4ct + cn hold
// "grows" for move a.
constexpr uint64_t make_dh_table4() {
  uint64_t tab = 0;
  for (int a = 0; a < 4; ++a)
    for (int ct = 0; ct < 4; ++ct)
      for (int cn = 0; cn < 4; ++cn) {
        // coordinate after the move: U moves the tile down (+1), D up (-1),
        // L moves it right (+1), R left (-1)
        const int step = (a == 0 || a == 1) ? 1 : -1;
        const int before = ct > cn ? ct - cn : cn - ct;
        const int cafter = cn + step;
        const int after = ct > cafter ? ct - cafter : cafter - ct;
        if (after > before) tab |= 1ull << (16 * a + 4 * ct + cn);
      }
  return tab;
}
constexpr uint64_t kDhTable4 = make_dh_table4();

// A node of the split tree, and a subtree root of the search.
//   meta bits 0..4 blank cell, 5..7 forbidden move (inverse of the move that
//   produced the node; 4 = none), 8..15 g, 16..23 h.
struct alignas(16) Node {
  uint64_t tiles;
  uint32_t meta;
  uint32_t f;  // g + h
};

// The first f-limit searched: h0, or the smallest h0 + 2j >= start when the
// caller asks to start higher (start < 0: h0).
__host__ __device__ inline int first_limit(int h0, int start) {
  return start <= h0 ? h0 : h0 + ((start - h0 + 1) & ~1);
}

__host__ __device__ inline uint32_t node_meta(int blank, int forbid, int g, int h) {
  return (uint32_t)blank | ((uint32_t)forbid << 5) | ((uint32_t)g << 8) | ((uint32_t)h << 16);
}

// Split-tree node of the batched path, any width (5x5 states take 125 bits).
struct alignas(8) NodeW {
  uint64_t lo, hi;  // packed state: bits 0..63, 64..127
  uint32_t meta;    // as Node
  uint32_t f;
};

// Ingest result of the batched path, any width.
struct InstW {
  uint64_t lo, hi;
  int32_t blank;
  int32_t h0;
  int32_t status;  // bpida_status
  int32_t width;
};

// Ingest result per instance.
struct Inst {
  uint64_t tiles;
  int32_t blank;
  int32_t h0;
  int32_t status;  // bpida_status
  int32_t pad;
};

// Per-workgroup partial of one search launch.
struct Partial {
  uint64_t nodes;    // nodes popped (expanded)
  uint64_t rounds;   // pop-expand-push cycles
  uint64_t spilled;  // entries moved LDS -> HBM
  int32_t fmin;      // smallest f of a pruned child or skipped root
  int32_t goals;     // goal nodes expanded
  int32_t err;       // nonzero: spill area overflow
  int32_t spill_hw;  // high-water mark of the spill stack
};

// Per-limit result read back by the host driver.
struct LimitResult {
  uint64_t nodes;   // interior + searched nodes at this limit
  int32_t fnext;    // next limit (must be limit + 2 unless found)
  int32_t found;    // a goal was expanded
  int32_t err;      // spill overflow in some workgroup
  int32_t spill_hw;
  uint64_t rounds;
  uint64_t spilled;
  uint64_t searched;  // nodes expanded by the search kernel alone
};

constexpr int kHistBins = 256;  // f values 0..255 of the split tree's interior
constexpr int kMaxPath = 256;   // moves per returned path (limits stay below 256)
constexpr int kMaxLimit = 255;  // slack and f fit in 8 bits
constexpr int kMaxDepth = 16;  // deepest root split
constexpr int kWalkCells = 25;  // walk-count table: [width - 3][cell][first forbidden move][length]
constexpr int kWalkStride = kWalkCells * 5 * (kMaxDepth + 1);

// Exact split-tree level sizes: v[w - 3][c][f][d] = number of blank walks of
// length d from cell c of a width-w board that never undo their previous
// move and whose first move is not f (f = 4: any first move): every level of
// the parent-pruned tree of a root with forbidden move f, no duplicate
// elimination.
struct WalkTable {
  int32_t v[3][kWalkCells][5][kMaxDepth + 1];
};

// Offset of the row (cell, first forbidden move) inside one width's table.
__host__ __device__ constexpr int walk_row(int cell, int forbid) {
  return (cell * 5 + forbid) * (kMaxDepth + 1);
}

constexpr WalkTable make_walk_table() {
  WalkTable t{};
  for (int w = 3; w <= 5; ++w)
    for (int blank = 0; blank < w * w; ++blank)
      for (int f0 = 0; f0 <= 4; ++f0) {
      // cur[c][f]: walks ending at cell c whose next move may not be f (4: any)
      int64_t cur[kWalkCells][5] = {};
      cur[blank][f0] = 1;
      for (int d = 0; d <= kMaxDepth; ++d) {
        int64_t tot = 0, nxt[kWalkCells][5] = {};
        for (int c = 0; c < w * w; ++c)
          for (int fb = 0; fb < 5; ++fb) {
            const int64_t m = cur[c][fb];
            if (!m) continue;
            tot += m;
            const int r = c / w, col = c % w;
            for (int a = 0; a < 4; ++a) {
              const bool ok = a == 0 ? r > 0 : a == 1 ? col > 0 : a == 2 ? col < w - 1 : r < w - 1;
              if (!ok || a == fb) continue;
              const int n = c + (a == 0 ? -w : a == 1 ? -1 : a == 2 ? 1 : w);
              nxt[n][3 - a] += m;
            }
          }
        t.v[w - 3][blank][f0][d] = (int32_t)(tot < INT32_MAX ? tot : INT32_MAX);
        for (int c = 0; c < kWalkCells; ++c)
          for (int fb = 0; fb < 5; ++fb) cur[c][fb] = nxt[c][fb];
      }
    }
  return t;
}

// ---------------------------------------------------------------------------
// Batched persistent search (bpida_batch.hip).
// ---------------------------------------------------------------------------
constexpr int kQChunk = 64;  // stack entries per queue chunk

// One queue slot: up to 64 stack entries of one instance at its current limit.
// Queue error bits after which work is lost (1 queue full while seeding,
// 2 entries dropped, 16 a ticket lost): the batched call reports
// BPIDA_ENOMEM and its workgroups stop early.
constexpr int32_t kErrFatal = 1 | 2 | 16;

// Bits 64..127 of a 5x5 chunk's states live in a parallel array (BatchArgs::hi),
// so a 3x3 or 4x4 chunk moves 6 cache lines, not 10.
struct alignas(128) QChunk {
  uint64_t tiles[kQChunk];  // packed states, bits 0..63
  uint16_t meta[kQChunk];
  int32_t inst;
  int32_t count;
  int32_t wide;  // 1: a 5x5 chunk, whose high words are in BatchArgs::hi
};

// Per-slot control words of the queue ring, for the next ticket t to use the
// slot: seq == 4t free for producer t, 4t + 1 claimed by it, 4t + 2 holds
// ticket t's chunk; abandoned = 1 + the largest ticket whose producer gave up
// on this slot (ring full for its whole bounded wait), 0 if none.
struct SlotCtl {
  uint64_t seq;
  uint64_t abandoned;
};

// Per-instance search state.
struct InstState {
  int32_t limit;        // current f-limit
  int32_t col;          // output column of the current limit
  int32_t done;         // 0 searching, 1 solved, 2 no goal within an exact limit,
                        // < 0 bpida_status
  int32_t outstanding;  // chunks queued or held at the current limit
  uint64_t nodes;       // nodes expanded by the search at the current limit
  int32_t fmin;         // smallest pruned f at the current limit
  int32_t goals;        // goals expanded at the current limit
  int64_t root_off;     // first root of this instance in the split tree buffer
  int32_t nroots;
  int32_t width;        // board width 3, 4 or 5
  int32_t stop;         // first-solution mode: a goal was expanded, drop the rest
  int32_t lost;         // some of this instance's work was dropped (queue full):
                        // its counts are void (server mode answers BPIDA_ENOMEM)
};

// Queue control block and run counters.  The fields that many workgroups
// touch concurrently sit on separate 128-byte lines.
struct QueueCtl {
  alignas(128) uint64_t head;
  alignas(128) uint64_t tail;
  alignas(128) int32_t remaining;  // instances still searching
  alignas(128) int32_t seed_next;  // next instance whose first limit is to be seeded
  alignas(128) int32_t err;  // 1: queue full while seeding, 2: entries dropped,
                             // 4: idle watchdog, 8: deadline passed, 16: ring full
  alignas(128) uint64_t rounds;
  uint64_t searched, pushes, pops;
  uint64_t t_work, t_queue, t_idle;  // wall-clock ticks summed over workgroups
  uint64_t voluntary;                // donations made because workgroups idled
  uint64_t qmax;                     // most chunks queued at once (seen at a push)
  uint64_t roots_read;               // split-tree roots read while seeding limits
  uint64_t chunks_read_wide;         // 5x5 chunks taken (their high words read too)
};

// ---------------------------------------------------------------------------
// Continuous-batching server: requests arrive through a ring in pinned host
// memory while the persistent kernel runs; each is admitted into a free
// instance slot (the device-memory budget), searched alongside the others
// and answered through a result ring in pinned host memory.
// ---------------------------------------------------------------------------
struct ServerReq {
  uint8_t state[16];
};

struct ServerRes {
  uint64_t seq;     // ticket + 1 once the fields below are final
  int32_t len;      // optimal length or -1
  int32_t status;   // 1 solved, < 0 bpida_status
  uint64_t nodes[64];
};

struct ServerHostCtl {
  alignas(128) uint64_t req_tail;      // requests published (host writes)
  alignas(128) int32_t stop;           // host asks the server to finish
  alignas(128) uint64_t req_admitted;  // requests copied to the device (device writes)
};

struct ServerArgs {
  ServerHostCtl* host;  // pinned host memory
  const ServerReq* req; // pinned ring of requests
  ServerRes* res;       // pinned ring of results
  uint64_t ring_mask;   // ring capacity - 1
  int32_t slots;        // instance slots (in-flight budget)
  int32_t depth;        // root split depth
  int64_t stride;       // split-tree nodes per slot
  int32_t* busy;        // per slot: 1 while a request occupies it
  uint64_t* ticket;     // per slot: request ticket
  const int32_t* walks; // walk counts per start cell and length, width 4
  int32_t* admitter;    // 0 until a workgroup takes the admitter role
  int32_t* in_flight;   // admitted, not yet answered
  int64_t backlog_max;  // the HBM frontier budget: a request is admitted only
                        // while at most this many chunks wait in the work queue
                        // beyond the waiting workgroups (<= 0: no limit)
};

struct BatchArgs {
  QueueCtl* q;
  SlotCtl* seq;        // per slot sequence number and abandoned-ticket mark
  QChunk* slots;
  uint64_t* hi;        // per slot 64 words: bits 64..127 of a 5x5 chunk (null: no 5x5 instance)
  uint64_t qmask;      // capacity - 1 (capacity a power of two)
  InstState* is;
  const NodeW* tree;
  const uint32_t* hist;
  const int32_t* goal_g;
  int32_t* out_len;
  uint64_t* out_nodes;  // n x 64
  int32_t n;
  int32_t max_limit;
  uint64_t idle_ticks;   // an idle workgroup gives up after this many wall-clock ticks
  uint64_t budget_ticks; // every workgroup stops this many ticks after it starts
  uint32_t donate_mask;  // donation checks run when (round & donate_mask) == 0
  int32_t donate_min;    // only stacks of at least this many entries donate (<= 0: 4 rounds of pops, <= ring / 2)
  int32_t donate_window; // a donation splits the oldest min(window, stack) entries (2 x chunk)
  int32_t first_solution; // nonzero: the final limit stops at its first goal
  int32_t start_limit;    // first f-limit to search (< 0: h0)
  int32_t seed_chunk;     // roots per seeded chunk (8..64)
  const int32_t* exact_limit;  // null, or per instance the one f-limit to search
                               // (status 1: a goal within it, 2: none)
  int32_t push_spin;     // polls of a full slot before a push gives its ticket up
  int32_t server;        // nonzero: continuous-batching server (srv below)
  ServerArgs srv;
};

hipError_t launch_server_setup(const BatchArgs& A, hipStream_t s);
// Device address of the walk-count table (a constant-initialised device
// variable: no allocation).
hipError_t walk_table_device(const int32_t** out);

hipError_t launch_batch_setup(const BatchArgs& A, const InstW* d_inst, const int64_t* d_root_off,
                              const int32_t* d_nroots, hipStream_t s);
hipError_t launch_ingestw(const uint8_t* d_states, const int64_t* d_byte_off, const int32_t* d_widths,
                          int width, int n, InstW* d_inst, hipStream_t s);
hipError_t launch_splitw(const InstW* d_inst, int n, int depth, const int64_t* d_tree_off,
                         int64_t stride, const int32_t* d_walks, const uint8_t* d_forbid,
                         NodeW* d_tree, uint32_t* d_hist, int32_t* d_goal_g, int32_t* d_err,
                         int64_t* d_root_off, int32_t* d_nroots, hipStream_t s);
hipError_t launch_batch4(int lds_cap, int npl, int wpg, int grid, const BatchArgs& A, hipStream_t s);
hipError_t launch_batch_status(const InstState* d_is, int n, const QueueCtl* d_q,
                               const int32_t* d_split_err, int32_t* d_status, hipStream_t s);
int batch4_max_blocks_per_cu(int lds_cap, int npl, int wpg);

// Path reconstruction by exact-limit probes (bpida_path.hip).
hipError_t launch_path_init(const uint8_t* d_states, const int32_t* d_len, int n, int nn,
                            uint8_t* d_cur, int32_t* d_left, uint8_t* d_prev, uint8_t* d_path,
                            hipStream_t s);
hipError_t launch_path_probe(const uint8_t* d_cur, const int32_t* d_left, const uint8_t* d_prev, int n,
                             int w, uint8_t* d_probe, int32_t* d_probe_limit, uint8_t* d_probe_forbid,
                             hipStream_t s);
hipError_t launch_path_select(const uint8_t* d_probe, const int32_t* d_status, const int32_t* d_len,
                              int n, int nn, uint8_t* d_cur, int32_t* d_left, uint8_t* d_prev,
                              uint8_t* d_path, int32_t* d_err, hipStream_t s);

// Kernel launchers (bpida_kernels.hip).
hipError_t launch_ingest4(const uint8_t* d_states, int n, Inst* d_inst, hipStream_t s);
hipError_t launch_split4(const Inst* d_inst, int n, int depth, const int64_t* d_tree_off,
                         int64_t stride, const int32_t* d_walks, Node* d_tree, uint32_t* d_hist,
                         int32_t* d_goal_g, int32_t* d_err, int64_t* d_root_off, int32_t* d_nroots,
                         hipStream_t s);
hipError_t launch_search4(int lds_cap, int npl, int grid, const Node* d_roots, int nroots, int limit,
                          int32_t* d_cursor, uint64_t* d_spill_tiles, uint16_t* d_spill_meta,
                          int spill_cap, Partial* d_part, int32_t* d_stop, uint32_t* d_load,
                          hipStream_t s);
// Static load balancing of the plain path (bpida_lb.hip): plan (average
// load, per-root split depth and size, offsets, total) and emit (the new
// root list; interior nodes into the histogram and the interior-goal depth).
hipError_t launch_lb_plan(const Node* d_roots, const uint32_t* d_load, int nroots, int limit,
                          uint64_t* d_avg, int32_t* d_level, int32_t* d_count, int64_t* d_off,
                          int64_t* d_total, hipStream_t s);
hipError_t launch_lb_emit(const Node* d_roots, int nroots, const int32_t* d_level,
                          const int32_t* d_count, const int64_t* d_off, Node* d_out,
                          uint32_t* d_hist, int32_t* d_goal_g, int32_t* d_err, hipStream_t s);
hipError_t launch_reduce(const Partial* d_part, int nwg, const uint32_t* d_hist_i,
                         const int32_t* d_goal_g_i, int limit, int col, uint64_t* d_nodes_row,
                         int32_t* d_cursor, LimitResult* d_res, hipStream_t s);
hipError_t launch_fill_outputs(int32_t* d_len, uint64_t* d_nodes, int n, hipStream_t s);
hipError_t launch_set_len(int32_t* d_len_i, int32_t value, hipStream_t s);
hipError_t launch_zero_i32(int32_t* d_p, int n, hipStream_t s);
hipError_t launch_zero_words(void* d_p, size_t bytes, hipStream_t s);
int search4_max_blocks_per_cu(int lds_cap, int npl);

}  // namespace bpida
