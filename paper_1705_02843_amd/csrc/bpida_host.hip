// bpida_host.hip -- C ABI and host driver of Block-Parallel IDA* (Alg. 1).
//
// The host side does what Alg. 1's BPIDA* function does on the CPU: it
// launches the root split once (CreateRootSet), starts at limit h0
// (DecideFirstLimit) and repeats one search launch per f-limit, one subtree
// per workgroup (parallelForByBlocks), reading back 48 bytes per limit to
// decide whether to stop.  Every node expansion, count and minimum is
// computed by the kernels in bpida_kernels.hip.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/bpida.h"
#include "bpida_internal.h"

namespace bpida {
namespace {

enum { kModePlain = 0, kModeBatched = 1 };

struct Options {
  int64_t mode = kModeBatched;
  int64_t frontier_depth = -1;  // -1: 10 for plain, 6 for batched
  int64_t nodes_per_round = 64; // batched mode: 16 (4 lanes per node) or 64
  int64_t queue_capacity = 0;   // chunks; 0: sized from the batch
  int64_t watchdog_ms = 20000;  // idle workgroups give up after this long
  int64_t budget_ms = 600000;   // the persistent launch stops after this long
  int64_t lds_stack_capacity = -1;  // -1: 512 for 16-node rounds, 1024 for 64
  int64_t spill_capacity = 16384;
  int64_t max_workgroups = 0;
  int64_t max_threshold = -1;
  int64_t donate_every = 128;  // batched mode: rounds between donation checks
  int64_t donate_min = -1;     // batched mode: smallest stack that donates (-1: 4 rounds of pops, <= ring / 2)
  int64_t queue_chunk = 64;    // batched mode: entries per donated chunk (16, 32 or 64)
  int64_t first_solution = 0;  // 1: the final limit stops at its first goal (Alg. 1 as printed)
  int64_t static_lb = 1;       // plain mode: re-split heavy roots between limits (Sec. 5)
  int64_t start_threshold = -1; // first f-limit to search (-1: h0)
  int64_t seed_chunk = 64;      // batched mode: roots per seeded chunk (8, 16, 32, 64)
  int64_t push_spin = 65536;    // batched mode: polls of a full queue slot before a push gives up
  int64_t plain_nodes_per_round = 16;  // plain mode: 16 (Alg. 1's lane map) or 64
  int64_t wg_size = 64;         // batched mode: threads per workgroup (1, 2 or 4 independent waves)
  int64_t admit_backlog = -1;   // server: queued chunks above which admission waits (-1: half the queue, 0: none)
};

std::mutex g_mu;  // serialises solves and option changes
Options g_opt;
constexpr int kStats = 20;
uint64_t g_stats[kStats] = {0};

// Set while the caller's stream is capturing a graph: buffers may not grow.
bool g_no_alloc = false;

// Grow-only device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t want) {
    if (want <= bytes) return hipSuccess;
    if (g_no_alloc) return hipErrorInvalidValue;
    if (p) {
      hipError_t e = hipFree(p);
      if (e != hipSuccess) return e;
      p = nullptr;
      bytes = 0;
    }
    size_t b = std::max<size_t>(want, 256);
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return e;
    }
    bytes = b;
    return hipSuccess;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

struct Workspace {
  int device = -1;
  int num_cu = 0;
  int wall_khz = 100000;
  bool arch_ok = false;
  uint64_t qcap = 0;  // queue slots of the last batched launch
  DevBuf inst, tree, tree_off, hist, goal_g, err, cursor, part, spill_t, spill_m, res, stop;
  DevBuf qctl, qseq, qslots, qhi, istate, root_off, nroots, status;
  // non-backtracking walk counts per width (3, 4, 5), start cell and length:
  // the device table (d_walks) and its host copy
  const int32_t* d_walks = nullptr;
  WalkTable h_walks = make_walk_table();
  DevBuf treew, winst, tree_offw, widths, byte_off;
  DevBuf h2d_states, out_len, out_nodes, out_path;
  // path reconstruction: current states, moves left, previous moves, probes
  DevBuf p_cur, p_left, p_prev, p_probe, p_limit, p_forbid, p_len, p_nodes, p_status, p_err;
  DevBuf lb_load, lb_roots[2], lb_level, lb_count, lb_off, lb_avg, lb_total;
  LimitResult* h_res = nullptr;  // pinned
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

Workspace g_ws;

int map_err(hipError_t e) {
  if (e == hipSuccess) return BPIDA_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return BPIDA_ENOMEM;
  return BPIDA_EDEVICE;
}

// Number of non-backtracking blank walks of each length 0..depth from cell
// `blank` of the 15-puzzle board (the exact size of each split-tree level).
void level_sizes(int blank, int depth, int32_t* out) {
  for (int d = 0; d <= depth; ++d) out[d] = g_ws.h_walks.v[1][blank][4][d];
}

int ensure_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return BPIDA_EDEVICE;
  }
  if (g_ws.device == dev) return g_ws.arch_ok ? BPIDA_OK : BPIDA_EDEVICE;
  if (g_ws.device >= 0) return BPIDA_EDEVICE;  // one device per process
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return BPIDA_EDEVICE;
  }
  g_ws.device = dev;
  g_ws.num_cu = prop.multiProcessorCount;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
    g_ws.wall_khz = khz;
  g_ws.arch_ok = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
  if (!g_ws.arch_ok) return BPIDA_EDEVICE;
  if (hipHostMalloc((void**)&g_ws.h_res, sizeof(LimitResult), hipHostMallocDefault) != hipSuccess)
    return BPIDA_ENOMEM;
  if (hipEventCreate(&g_ws.ev0) != hipSuccess || hipEventCreate(&g_ws.ev1) != hipSuccess)
    return BPIDA_EDEVICE;
  if (walk_table_device(&g_ws.d_walks) != hipSuccess) {
    (void)hipGetLastError();
    return BPIDA_EDEVICE;
  }
  return BPIDA_OK;
}

int cap_for(const Options& O, int npl) {
  if (O.lds_stack_capacity > 0) return (int)O.lds_stack_capacity;
  return npl == 64 ? 1024 : 512;
}

int depth_for(const Options& O) {
  if (O.frontier_depth >= 0) return (int)O.frontier_depth;
  return O.mode == kModePlain ? 10 : 6;
}

int run_batched(const uint8_t* d_states, int n, int32_t* d_len, uint64_t* d_nodes, hipStream_t st,
                const Options& O, int width = 4, const int32_t* h_widths = nullptr);

// The plain BPIDA* driver (Alg. 1 as printed: one search launch per f-limit
// and instance, one root per workgroup, no dynamic balancing).  All buffers
// are device buffers; outputs are written on `st`.
int run_plain(const uint8_t* d_states, int n, int32_t* d_len, uint64_t* d_nodes, hipStream_t st,
              const Options& O, int width = 4) {
  if (O.mode == kModeBatched) return run_batched(d_states, n, d_len, d_nodes, st, O, width);
  if (width != 4) return BPIDA_EINVAL;  // the plain path is the 15-puzzle kernel
  Workspace& W = g_ws;
  uint64_t stats[kStats] = {0};
  hipError_t e;
#define HIPCHK(x)              \
  do {                         \
    e = (x);                   \
    if (e != hipSuccess) {     \
      (void)hipGetLastError(); \
      return map_err(e);       \
    }                          \
  } while (0)

  HIPCHK(launch_fill_outputs(d_len, d_nodes, n, st));
  if (n == 0) return BPIDA_OK;
  const int D = depth_for(O);
  const int pnpl = (int)O.plain_nodes_per_round;
  const int cap = cap_for(O, pnpl);
  const int spill_cap = (int)O.spill_capacity;

  // a1: ingest
  HIPCHK(W.inst.ensure(sizeof(Inst) * (size_t)n));
  HIPCHK(launch_ingest4(d_states, n, W.inst.as<Inst>(), st));
  std::vector<Inst> inst((size_t)n);
  HIPCHK(hipMemcpyAsync(inst.data(), W.inst.p, sizeof(Inst) * (size_t)n, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));

  // a3: split-tree layout (exact level sizes per instance)
  const int L1 = kMaxDepth + 1;
  std::vector<int32_t> lc((size_t)n * L1, 0);
  std::vector<int64_t> off((size_t)n + 1, 0);
  std::vector<int64_t> root_off((size_t)n, 0);
  for (int i = 0; i < n; ++i) {
    int32_t* row = lc.data() + (size_t)i * L1;
    if (inst[i].status == 0) level_sizes(inst[i].blank, D, row);
    else row[0] = 1;
    int64_t tot = 0;
    for (int d = 0; d <= D; ++d) {
      if (d == D) root_off[i] = off[i] + tot;
      tot += row[d];
    }
    off[i + 1] = off[i] + tot;
  }
  HIPCHK(W.tree.ensure(sizeof(Node) * (size_t)off[n]));
  HIPCHK(W.tree_off.ensure(sizeof(int64_t) * (size_t)n));
  HIPCHK(W.hist.ensure(sizeof(uint32_t) * kHistBins * (size_t)n));
  HIPCHK(W.goal_g.ensure(sizeof(int32_t) * (size_t)n));
  HIPCHK(W.err.ensure(sizeof(int32_t)));
  HIPCHK(hipMemcpyAsync(W.tree_off.p, off.data(), sizeof(int64_t) * (size_t)n, hipMemcpyHostToDevice, st));
  HIPCHK(launch_zero_i32(W.err.as<int32_t>(), 1, st));
  HIPCHK(launch_split4(W.inst.as<Inst>(), n, D, W.tree_off.as<int64_t>(), 0,
                       W.d_walks + kWalkStride,
                       W.tree.as<Node>(), W.hist.as<uint32_t>(), W.goal_g.as<int32_t>(),
                       W.err.as<int32_t>(), nullptr, nullptr, st));
  int32_t split_err = 0;
  HIPCHK(hipMemcpyAsync(&split_err, W.err.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (split_err) return BPIDA_EINTERNAL;

  // a4..a9: persistent search grid and its scratch
  int per_cu = search4_max_blocks_per_cu(cap, pnpl);
  if (per_cu <= 0) return BPIDA_EINVAL;
  int64_t max_grid = (int64_t)per_cu * W.num_cu;
  if (O.max_workgroups > 0) max_grid = std::min<int64_t>(max_grid, O.max_workgroups);
  HIPCHK(W.part.ensure(sizeof(Partial) * (size_t)max_grid));
  HIPCHK(W.spill_t.ensure(sizeof(uint64_t) * (size_t)max_grid * spill_cap));
  HIPCHK(W.spill_m.ensure(sizeof(uint16_t) * (size_t)max_grid * spill_cap));
  HIPCHK(W.cursor.ensure(sizeof(int32_t)));
  HIPCHK(W.stop.ensure(sizeof(int32_t)));
  // static load balancing: a root list grows to at most lb_cap entries
  int64_t max_roots = 0;
  for (int i = 0; i < n; ++i) max_roots = std::max<int64_t>(max_roots, lc[(size_t)i * L1 + D]);
  const int64_t lb_cap = O.static_lb ? max_roots * 32 + 4096 : 0;
  if (O.static_lb) {
    HIPCHK(W.lb_load.ensure(sizeof(uint32_t) * (size_t)lb_cap));
    HIPCHK(W.lb_roots[0].ensure(sizeof(Node) * (size_t)lb_cap));
    HIPCHK(W.lb_roots[1].ensure(sizeof(Node) * (size_t)lb_cap));
    HIPCHK(W.lb_level.ensure(sizeof(int32_t) * (size_t)lb_cap));
    HIPCHK(W.lb_count.ensure(sizeof(int32_t) * (size_t)lb_cap));
    HIPCHK(W.lb_off.ensure(sizeof(int64_t) * (size_t)lb_cap));
    HIPCHK(W.lb_avg.ensure(2 * sizeof(uint64_t)));
    HIPCHK(W.lb_total.ensure(sizeof(int64_t)));
  }
  HIPCHK(W.res.ensure(sizeof(LimitResult)));
  HIPCHK(launch_zero_i32(W.cursor.as<int32_t>(), 1, st));

  int rc = BPIDA_OK;
  for (int i = 0; i < n; ++i) {
    int code = inst[i].status;
    if (code == BPIDA_OK) {
      int nroots = lc[(size_t)i * L1 + D];
      const Node* roots = W.tree.as<Node>() + root_off[i];
      int pong = 0;
      int L = first_limit(inst[i].h0, (int)O.start_threshold);
      code = BPIDA_ELIMIT;
      for (int j = (L - inst[i].h0) / 2; j < BPIDA_MAX_THRESHOLDS; ++j) {
        if (L > kMaxLimit || (O.max_threshold >= 0 && L > O.max_threshold)) break;
        const int grid = (int)std::min<int64_t>(nroots, max_grid);
        uint32_t* load = nullptr;
        if (O.static_lb) {
          load = W.lb_load.as<uint32_t>();
          HIPCHK(launch_zero_i32((int32_t*)load, nroots, st));
        }
        int32_t* stop = nullptr;
        if (O.first_solution) {
          stop = W.stop.as<int32_t>();
          HIPCHK(launch_zero_i32(stop, 1, st));
        }
        HIPCHK(hipEventRecord(W.ev0, st));
        HIPCHK(launch_search4(cap, pnpl, grid, roots, nroots, L, W.cursor.as<int32_t>(),
                              W.spill_t.as<uint64_t>(), W.spill_m.as<uint16_t>(), spill_cap,
                              W.part.as<Partial>(), stop, load, st));
        HIPCHK(hipEventRecord(W.ev1, st));
        HIPCHK(launch_reduce(W.part.as<Partial>(), grid, W.hist.as<uint32_t>() + (size_t)i * kHistBins,
                             W.goal_g.as<int32_t>() + i, L, j, d_nodes + (size_t)i * BPIDA_MAX_THRESHOLDS,
                             W.cursor.as<int32_t>(), W.res.as<LimitResult>(), st));
        HIPCHK(hipMemcpyAsync(W.h_res, W.res.p, sizeof(LimitResult), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        float ms = 0.f;
        if (grid > 0 && hipEventElapsedTime(&ms, W.ev0, W.ev1) == hipSuccess)
          stats[4] += (uint64_t)(ms * 1000.0f);
        const LimitResult R = *W.h_res;
        stats[0] += R.rounds;
        stats[1] += R.searched;
        stats[2] += R.spilled;
        stats[3] += grid > 0 ? 1 : 0;
        stats[16] += (uint64_t)nroots;  // every root is read once per limit
        stats[5] = std::max<uint64_t>(stats[5], (uint64_t)R.spill_hw);
        if (R.err) {
          code = BPIDA_ENOMEM;
          break;
        }
        if (R.found) {
          HIPCHK(launch_set_len(d_len + i, L, st));
          code = BPIDA_OK;
          break;
        }
        if (R.fnext != L + 2) {
          code = BPIDA_EINTERNAL;
          break;
        }
        // (every limit, small ones included: the re-splits compound, each
        // refining the root set the next, larger limits inherit)
        if (O.static_lb && nroots > 0) {
          // Sec. 5: re-split the roots whose repetition count exceeded the
          // average, for the next iteration
          HIPCHK(launch_lb_plan(roots, load, nroots, L, W.lb_avg.as<uint64_t>(),
                                W.lb_level.as<int32_t>(), W.lb_count.as<int32_t>(),
                                W.lb_off.as<int64_t>(), W.lb_total.as<int64_t>(), st));
          int64_t total = 0;
          HIPCHK(hipMemcpyAsync(&total, W.lb_total.p, sizeof total, hipMemcpyDeviceToHost, st));
          HIPCHK(hipStreamSynchronize(st));
          if (total > nroots && total <= lb_cap) {
            Node* out = W.lb_roots[pong].as<Node>();
            HIPCHK(launch_zero_i32(W.err.as<int32_t>(), 1, st));
            HIPCHK(launch_lb_emit(roots, nroots, W.lb_level.as<int32_t>(), W.lb_count.as<int32_t>(),
                                  W.lb_off.as<int64_t>(), out,
                                  W.hist.as<uint32_t>() + (size_t)i * kHistBins,
                                  W.goal_g.as<int32_t>() + i, W.err.as<int32_t>(), st));
            int32_t lb_err = 0;
            HIPCHK(hipMemcpyAsync(&lb_err, W.err.p, sizeof lb_err, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (lb_err) {
              code = BPIDA_EINTERNAL;
              break;
            }
            stats[15] += (uint64_t)(total - nroots);
            roots = out;
            nroots = (int)total;
            pong ^= 1;
          }
        }
        L = R.fnext;
      }
    }
    if (code != BPIDA_OK && rc == BPIDA_OK) rc = code;
  }
  HIPCHK(hipStreamSynchronize(st));
  memcpy(g_stats, stats, sizeof stats);
#undef HIPCHK
  return rc;
}

// Enqueues the whole batched solve on `st`; per-instance status (1 solved,
// < 0 bpida_status) lands in d_status.  No host synchronisation, no copy to
// the host: the sequence can be recorded into a HIP graph.
// Split-tree nodes per instance of width w at depth D (the largest level
// total over start cells) and the largest root count.
void tree_size(const Workspace& W, int w, int D, int64_t* stride, int64_t* max_roots) {
  *stride = 0;
  *max_roots = 0;
  for (int c = 0; c < w * w; ++c) {
    int64_t tot = 0;
    for (int d = 0; d <= D; ++d) tot += W.h_walks.v[w - 3][c][4][d];
    *stride = std::max(*stride, tot);
    *max_roots = std::max<int64_t>(*max_roots, W.h_walks.v[w - 3][c][4][D]);
  }
}

// Whether a width can run with this LDS stack option.  3x3 and 5x5
// instances always run 64-node rounds; a 5x5 state takes two entries, so its
// stack holds cap / 2 of them.  A 64-node round can add 192 entries, so a
// stack of 256 spills on almost every round: the spilled chunks, taken
// oldest first, turn the search breadth-first and the work queue grows
// without bound on 4x4 and 5x5 trees (measured: 2 million chunks were not
// enough).  3x3 trees are small enough for 256.
bool ring_fits(int w, int cap, int npl) {
  if (w == 3) return cap >= 256;
  if (w == 4) return npl == 16 || cap >= 512;
  return cap / 2 >= 512;
}

// Sizes of one batched solve.  Every buffer depends on n, the widths and D
// only, and no value travels back to the host before the persistent launch:
// the whole solve is one stream-ordered sequence of kernels.
struct BatchPlan {
  int n = 0, width = 4, D = 0, npl = 64, cap = 1024, sc = 64, wpg = 1;
  bool any5 = false;
  int64_t tree_nodes = 0, stride = 0, seed_chunks = 0, grid = 0;
  uint64_t qcap = 64;       // queue slots (a power of two)
  uint64_t qwant = 64;      // the default queue size (queue_capacity option, or sized from the batch)
  std::vector<int64_t> toff, boff;  // mixed widths: split-tree and byte offsets per instance
};

// Device buffers of one batched solve.
struct BatchBufs {
  InstW* winst = nullptr;
  NodeW* treew = nullptr;
  uint32_t* hist = nullptr;
  int32_t* goal_g = nullptr;
  int32_t* err = nullptr;
  int64_t* root_off = nullptr;
  int32_t* nroots = nullptr;
  QueueCtl* qctl = nullptr;
  SlotCtl* qseq = nullptr;
  QChunk* qslots = nullptr;
  uint64_t* qhi = nullptr;  // 5x5 high words (any5 only)
  InstState* istate = nullptr;
  int32_t* widths = nullptr;    // mixed widths only
  int64_t* byte_off = nullptr;  // mixed widths only
  int64_t* tree_offw = nullptr; // mixed widths only
};

int plan_batched(int n, int width, const int32_t* h_widths, const Options& O, int num_cu,
                 BatchPlan* P) {
  const Workspace& W = g_ws;
  P->n = n;
  P->width = width;
  P->D = depth_for(O);
  P->npl = (int)O.nodes_per_round;
  P->cap = cap_for(O, P->npl);
  P->wpg = (int)(O.wg_size / 64);
  const int per_cu = batch4_max_blocks_per_cu(P->cap, P->npl, P->wpg);
  if (per_cu <= 0) return BPIDA_EINVAL;  // unsupported capacity for this round width
  P->any5 = width == 5;
  P->tree_nodes = P->seed_chunks = P->stride = 0;
  if (!h_widths) {
    int64_t mr = 0;
    tree_size(W, width, P->D, &P->stride, &mr);
    if (!ring_fits(width, P->cap, P->npl)) return BPIDA_EINVAL;
    P->tree_nodes = P->stride * n;
    P->seed_chunks = (int64_t)n * ((mr + kQChunk - 1) / kQChunk);
  } else {
    P->toff.assign((size_t)n, 0);
    P->boff.assign((size_t)n, 0);
    int64_t bytes = 0;
    for (int i = 0; i < n; ++i) {
      const int w = h_widths[i];
      if (w < 3 || w > 5 || !ring_fits(w, P->cap, P->npl)) return BPIDA_EINVAL;
      P->any5 = P->any5 || w == 5;
      int64_t sw = 0, mr = 0;
      tree_size(W, w, P->D, &sw, &mr);
      P->toff[i] = P->tree_nodes;
      P->boff[i] = bytes;
      P->tree_nodes += sw;
      bytes += (int64_t)w * w;
      P->seed_chunks += (mr + kQChunk - 1) / kQChunk;
    }
  }
  P->grid = (int64_t)per_cu * num_cu;
  if (O.max_workgroups > 0) P->grid = std::min<int64_t>(P->grid, O.max_workgroups);
  // Default queue size: the seeds plus, per wave, room for the chunks its
  // stack overflows into.  Smaller stacks spill more (64-node rounds on
  // a 512-entry stack spill ~10x more than on 1024), and a 5x5 subtree's
  // stack runs deeper on a stack of half as many entries (measured peaks:
  // about 6 chunks per workgroup for 4x4 batches on 1024 entries, 36 for
  // 5x5).  Smaller seed chunks were measured not to help (the grid fills
  // through donation within the first rounds), so 64 is the default.
  P->sc = (int)O.seed_chunk;
  P->seed_chunks *= kQChunk / P->sc;
  const int64_t per_wg = P->any5 ? 64 : std::min<int64_t>(64, std::max<int64_t>(16, 32768 / P->cap));
  const uint64_t want = O.queue_capacity > 0 ? (uint64_t)O.queue_capacity
                                              : (uint64_t)(P->seed_chunks + P->grid * P->wpg * per_wg + 1024);
  uint64_t q = 64;
  while (q < want) q <<= 1;
  P->qcap = P->qwant = q;
  return BPIDA_OK;
}

// Lays the buffers of plan P out from byte address `base` (256-byte aligned
// pieces) and returns the bytes used; base = 0 only measures.
size_t carve_batched(uintptr_t base, const BatchPlan& P, BatchBufs* B) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> uintptr_t {
    const uintptr_t p = base + off;
    off += (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    return p;
  };
  const size_t n = (size_t)P.n;
  B->winst = (InstW*)take(sizeof(InstW) * n);
  B->treew = (NodeW*)take(sizeof(NodeW) * (size_t)P.tree_nodes);
  B->hist = (uint32_t*)take(sizeof(uint32_t) * kHistBins * n);
  B->goal_g = (int32_t*)take(sizeof(int32_t) * n);
  B->err = (int32_t*)take(sizeof(int32_t));
  B->root_off = (int64_t*)take(sizeof(int64_t) * n);
  B->nroots = (int32_t*)take(sizeof(int32_t) * n);
  B->qctl = (QueueCtl*)take(sizeof(QueueCtl));
  B->qseq = (SlotCtl*)take(sizeof(SlotCtl) * P.qcap);
  B->qslots = (QChunk*)take(sizeof(QChunk) * P.qcap);
  B->qhi = P.any5 ? (uint64_t*)take(sizeof(uint64_t) * kQChunk * P.qcap) : nullptr;
  B->istate = (InstState*)take(sizeof(InstState) * n);
  if (!P.toff.empty()) {
    B->widths = (int32_t*)take(sizeof(int32_t) * n);
    B->byte_off = (int64_t*)take(sizeof(int64_t) * n);
    B->tree_offw = (int64_t*)take(sizeof(int64_t) * n);
  }
  return off;
}

// The buffers of plan P from the library's grow-only workspace.
int alloc_batched(const BatchPlan& P, BatchBufs* B) {
  Workspace& W = g_ws;
  const size_t n = (size_t)P.n;
  if (W.winst.ensure(sizeof(InstW) * n) != hipSuccess ||
      W.treew.ensure(sizeof(NodeW) * (size_t)P.tree_nodes) != hipSuccess ||
      W.hist.ensure(sizeof(uint32_t) * kHistBins * n) != hipSuccess ||
      W.goal_g.ensure(sizeof(int32_t) * n) != hipSuccess || W.err.ensure(sizeof(int32_t)) != hipSuccess ||
      W.root_off.ensure(sizeof(int64_t) * n) != hipSuccess ||
      W.nroots.ensure(sizeof(int32_t) * n) != hipSuccess ||
      W.qctl.ensure(sizeof(QueueCtl)) != hipSuccess ||
      W.qseq.ensure(sizeof(SlotCtl) * P.qcap) != hipSuccess ||
      W.qslots.ensure(sizeof(QChunk) * P.qcap) != hipSuccess ||
      (P.any5 && W.qhi.ensure(sizeof(uint64_t) * kQChunk * P.qcap) != hipSuccess) ||
      W.istate.ensure(sizeof(InstState) * n) != hipSuccess)
    return g_no_alloc ? BPIDA_EINVAL : BPIDA_ENOMEM;
  if (!P.toff.empty() &&
      (W.widths.ensure(sizeof(int32_t) * n) != hipSuccess ||
       W.byte_off.ensure(sizeof(int64_t) * n) != hipSuccess ||
       W.tree_offw.ensure(sizeof(int64_t) * n) != hipSuccess))
    return g_no_alloc ? BPIDA_EINVAL : BPIDA_ENOMEM;
  B->winst = W.winst.as<InstW>();
  B->treew = W.treew.as<NodeW>();
  B->hist = W.hist.as<uint32_t>();
  B->goal_g = W.goal_g.as<int32_t>();
  B->err = W.err.as<int32_t>();
  B->root_off = W.root_off.as<int64_t>();
  B->nroots = W.nroots.as<int32_t>();
  B->qctl = W.qctl.as<QueueCtl>();
  B->qseq = W.qseq.as<SlotCtl>();
  B->qslots = W.qslots.as<QChunk>();
  B->qhi = P.any5 ? W.qhi.as<uint64_t>() : nullptr;
  B->istate = W.istate.as<InstState>();
  if (!P.toff.empty()) {
    B->widths = W.widths.as<int32_t>();
    B->byte_off = W.byte_off.as<int64_t>();
    B->tree_offw = W.tree_offw.as<int64_t>();
  }
  return BPIDA_OK;
}

// Enqueues the whole batched solve of plan P on `st` into buffers B;
// per-instance status (1 solved, < 0 bpida_status) lands in d_status.  No
// host synchronisation and no copy to the host except the mixed-width
// tables: the sequence can be recorded into a HIP graph.  `walks` is the
// device walk-count table.
int enqueue_batched_into(const uint8_t* d_states, int32_t* d_len, uint64_t* d_nodes,
                         int32_t* d_status, hipStream_t st, const Options& O, const BatchPlan& P,
                         const BatchBufs& B, const int32_t* walks, const int32_t* h_widths,
                         hipEvent_t ev0, hipEvent_t ev1, int wall_khz,
                         const int32_t* exact_limit = nullptr, const uint8_t* root_forbid = nullptr) {
  hipError_t e;
#define HIPCHK(x)              \
  do {                         \
    e = (x);                   \
    if (e != hipSuccess) {     \
      (void)hipGetLastError(); \
      return map_err(e);       \
    }                          \
  } while (0)
  const int n = P.n;
  HIPCHK(launch_fill_outputs(d_len, d_nodes, n, st));
  if (n == 0) return BPIDA_OK;
  if (h_widths) {
    HIPCHK(hipMemcpyAsync(B.widths, h_widths, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(B.byte_off, P.boff.data(), sizeof(int64_t) * (size_t)n, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(B.tree_offw, P.toff.data(), sizeof(int64_t) * (size_t)n, hipMemcpyHostToDevice, st));
  }
  HIPCHK(launch_ingestw(d_states, h_widths ? B.byte_off : nullptr, h_widths ? B.widths : nullptr,
                        P.width, n, B.winst, st));
  HIPCHK(launch_zero_i32(B.err, 1, st));
  HIPCHK(launch_splitw(B.winst, n, P.D, h_widths ? B.tree_offw : nullptr, P.stride, walks, root_forbid,
                       B.treew, B.hist, B.goal_g, B.err, B.root_off, B.nroots, st));
  HIPCHK(launch_zero_words(B.qctl, sizeof(QueueCtl), st));

  BatchArgs A;
  memset(&A, 0, sizeof A);
  A.q = B.qctl;
  A.seq = B.qseq;
  A.slots = B.qslots;
  A.hi = B.qhi;
  A.qmask = P.qcap - 1;
  A.is = B.istate;
  A.tree = B.treew;
  A.hist = B.hist;
  A.goal_g = B.goal_g;
  A.out_len = d_len;
  A.out_nodes = d_nodes;
  A.n = n;
  A.server = 0;
  A.max_limit = (int)(O.max_threshold >= 0 ? std::min<int64_t>(O.max_threshold, kMaxLimit) : kMaxLimit);
  A.idle_ticks = (uint64_t)O.watchdog_ms * (uint64_t)wall_khz;
  A.budget_ticks = (uint64_t)O.budget_ms * (uint64_t)wall_khz;
  A.donate_mask = (uint32_t)O.donate_every - 1u;
  A.donate_min = (int32_t)O.donate_min;
  A.donate_window = 2 * (int32_t)O.queue_chunk;
  A.first_solution = (int32_t)O.first_solution;
  A.start_limit = (int32_t)O.start_threshold;
  A.seed_chunk = P.sc;
  A.push_spin = (int32_t)O.push_spin;
  A.exact_limit = exact_limit;
  HIPCHK(launch_batch_setup(A, B.winst, B.root_off, B.nroots, st));
  if (ev0) HIPCHK(hipEventRecord(ev0, st));
  HIPCHK(launch_batch4(P.cap, P.npl, P.wpg, (int)P.grid, A, st));
  if (ev1) HIPCHK(hipEventRecord(ev1, st));
  HIPCHK(launch_batch_status(A.is, n, A.q, B.err, d_status, st));
  return BPIDA_OK;
#undef HIPCHK
}

int enqueue_batched(const uint8_t* d_states, int n, int32_t* d_len, uint64_t* d_nodes,
                    int32_t* d_status, hipStream_t st, const Options& O, bool timed,
                    int64_t* grid_out, int width = 4, const int32_t* h_widths = nullptr) {
  Workspace& W = g_ws;
  if (n == 0) return map_err(launch_fill_outputs(d_len, d_nodes, n, st));
  BatchPlan P;
  int rc = plan_batched(n, width, h_widths, O, W.num_cu, &P);
  if (rc != BPIDA_OK) return rc;
  BatchBufs B;
  rc = alloc_batched(P, &B);
  if (rc != BPIDA_OK) return rc;
  W.qcap = P.qcap;
  *grid_out = P.grid;
  return enqueue_batched_into(d_states, d_len, d_nodes, d_status, st, O, P, B, W.d_walks, h_widths,
                              timed ? W.ev0 : nullptr, timed ? W.ev1 : nullptr, W.wall_khz);
}

// The batched driver: enqueue, then wait and read the status back.
int run_batched(const uint8_t* d_states, int n, int32_t* d_len, uint64_t* d_nodes, hipStream_t st,
                const Options& O, int width, const int32_t* h_widths) {
  Workspace& W = g_ws;
  uint64_t stats[kStats] = {0};
  hipError_t e;
#define HIPCHK(x)              \
  do {                         \
    e = (x);                   \
    if (e != hipSuccess) {     \
      (void)hipGetLastError(); \
      return map_err(e);       \
    }                          \
  } while (0)
  if (n == 0) {
    HIPCHK(launch_fill_outputs(d_len, d_nodes, n, st));
    return BPIDA_OK;
  }
  HIPCHK(W.status.ensure(sizeof(int32_t) * (size_t)n));
  int64_t grid = 0;
  int rc0 = enqueue_batched(d_states, n, d_len, d_nodes, W.status.as<int32_t>(), st, O, true, &grid,
                            width, h_widths);
  if (rc0 != BPIDA_OK) return rc0;
  std::vector<int32_t> status((size_t)n);
  QueueCtl qc;
  int32_t split_err = 0;
  HIPCHK(hipMemcpyAsync(status.data(), W.status.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&qc, W.qctl.p, sizeof(QueueCtl), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&split_err, W.err.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, W.ev0, W.ev1) == hipSuccess) stats[4] = (uint64_t)(ms * 1000.0f);
  stats[0] = qc.rounds;
  stats[1] = qc.searched;
  stats[2] = qc.pushes * kQChunk;
  stats[3] = 1;
  stats[6] = qc.pushes;
  stats[7] = qc.pops;
  stats[8] = qc.t_work / (uint64_t)std::max(1, W.wall_khz / 1000);  // microseconds
  stats[9] = qc.t_queue / (uint64_t)std::max(1, W.wall_khz / 1000);
  stats[10] = qc.t_idle / (uint64_t)std::max(1, W.wall_khz / 1000);
  stats[11] = qc.voluntary;
  stats[5] = qc.qmax;
  stats[12] = (uint64_t)grid;
  stats[13] = (uint64_t)(uint32_t)qc.err | ((uint64_t)(split_err != 0) << 8);
  stats[14] = W.qcap;
  stats[16] = qc.roots_read;
  stats[17] = qc.chunks_read_wide;
  memcpy(g_stats, stats, sizeof stats);
  int rc = BPIDA_OK;
  for (int i = 0; i < n && rc == BPIDA_OK; ++i)
    if (status[i] != 1) rc = status[i];
  return rc;
#undef HIPCHK
}

// One optimal path per instance: the batched solve, then one round of
// exact-limit probes per move (bpida_path.hip).  Probes of a round run as one
// batched solve of 4 n boards, each at the single limit (moves left - 1),
// with the move back to the parent forbidden at its root and the search
// stopping at its first goal.  Statistics stay those of the solve.
int run_paths(const uint8_t* d_states, int n, int width, int32_t* d_len, uint64_t* d_nodes,
              uint8_t* d_path, hipStream_t st, const Options& O) {
  Workspace& W = g_ws;
  hipError_t e;
#define HIPCHK(x)              \
  do {                         \
    e = (x);                   \
    if (e != hipSuccess) {     \
      (void)hipGetLastError(); \
      return map_err(e);       \
    }                          \
  } while (0)
  Options Ob = O;
  Ob.mode = kModeBatched;
  const int rc = run_batched(d_states, n, d_len, d_nodes, st, Ob, width);
  uint64_t solve_stats[kStats];
  memcpy(solve_stats, g_stats, sizeof solve_stats);
  if (n == 0) return rc;
  const int nn = width * width;
  std::vector<int32_t> len((size_t)n);
  HIPCHK(hipMemcpyAsync(len.data(), d_len, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  int maxlen = 0;
  for (int i = 0; i < n; ++i) maxlen = std::max(maxlen, (int)len[i]);
  const size_t np = 4 * (size_t)n;
  if (W.p_cur.ensure((size_t)n * nn) != hipSuccess || W.p_left.ensure(sizeof(int32_t) * (size_t)n) != hipSuccess ||
      W.p_prev.ensure((size_t)n) != hipSuccess || W.p_probe.ensure(np * nn) != hipSuccess ||
      W.p_limit.ensure(sizeof(int32_t) * np) != hipSuccess || W.p_forbid.ensure(np) != hipSuccess ||
      W.p_len.ensure(sizeof(int32_t) * np) != hipSuccess ||
      W.p_nodes.ensure(sizeof(uint64_t) * BPIDA_MAX_THRESHOLDS * np) != hipSuccess ||
      W.p_status.ensure(sizeof(int32_t) * np) != hipSuccess || W.p_err.ensure(sizeof(int32_t)) != hipSuccess)
    return BPIDA_ENOMEM;
  HIPCHK(launch_path_init(d_states, d_len, n, nn, W.p_cur.as<uint8_t>(), W.p_left.as<int32_t>(),
                          W.p_prev.as<uint8_t>(), d_path, st));
  HIPCHK(launch_zero_i32(W.p_err.as<int32_t>(), 1, st));
  Options Op = Ob;
  Op.first_solution = 1;
  Op.start_threshold = -1;
  Op.max_threshold = -1;
  BatchPlan P;
  int prc = plan_batched((int)np, width, nullptr, Op, W.num_cu, &P);
  if (prc != BPIDA_OK) return prc;
  BatchBufs B;
  prc = alloc_batched(P, &B);
  if (prc != BPIDA_OK) return prc;
  for (int step = 0; step < maxlen; ++step) {
    HIPCHK(launch_path_probe(W.p_cur.as<uint8_t>(), W.p_left.as<int32_t>(), W.p_prev.as<uint8_t>(), n,
                             width, W.p_probe.as<uint8_t>(), W.p_limit.as<int32_t>(),
                             W.p_forbid.as<uint8_t>(), st));
    prc = enqueue_batched_into(W.p_probe.as<uint8_t>(), W.p_len.as<int32_t>(), W.p_nodes.as<uint64_t>(),
                               W.p_status.as<int32_t>(), st, Op, P, B, W.d_walks, nullptr, nullptr,
                               nullptr, W.wall_khz, W.p_limit.as<int32_t>(), W.p_forbid.as<uint8_t>());
    if (prc != BPIDA_OK) return prc;
    HIPCHK(launch_path_select(W.p_probe.as<uint8_t>(), W.p_status.as<int32_t>(), d_len, n, nn,
                              W.p_cur.as<uint8_t>(), W.p_left.as<int32_t>(), W.p_prev.as<uint8_t>(),
                              d_path, W.p_err.as<int32_t>(), st));
  }
  int32_t perr = 0;
  HIPCHK(hipMemcpyAsync(&perr, W.p_err.p, sizeof perr, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  memcpy(g_stats, solve_stats, sizeof solve_stats);
  if (perr) return rc != BPIDA_OK ? rc : BPIDA_EINTERNAL;
  return rc;
#undef HIPCHK
}

int check_opts(int width) {
  if (width < BPIDA_MIN_WIDTH || width > BPIDA_MAX_WIDTH) return BPIDA_EINVAL;
  return BPIDA_OK;
}

}  // namespace
}  // namespace bpida

using namespace bpida;

extern "C" int bpida_solve(const uint8_t* states, int32_t n_instances, int32_t width,
                           int32_t* out_len, uint64_t* out_nodes_per_threshold) {
  try {
    if (!states || !out_len || !out_nodes_per_threshold || n_instances < 0) return BPIDA_EINVAL;
    if (check_opts(width) != BPIDA_OK) return BPIDA_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    const Options O = g_opt;
    const size_t n = (size_t)n_instances;
    if (n == 0) return BPIDA_OK;
    int rc = ensure_device();
    if (rc != BPIDA_OK) return rc;
    Workspace& W = g_ws;
    hipStream_t st = nullptr;
    const size_t bytes = n * (size_t)width * (size_t)width;
    if (W.h2d_states.ensure(bytes) != hipSuccess || W.out_len.ensure(n * sizeof(int32_t)) != hipSuccess ||
        W.out_nodes.ensure(n * BPIDA_MAX_THRESHOLDS * sizeof(uint64_t)) != hipSuccess)
      return BPIDA_ENOMEM;
    if (hipMemcpyAsync(W.h2d_states.p, states, bytes, hipMemcpyHostToDevice, st) != hipSuccess)
      return BPIDA_EDEVICE;
    rc = run_plain(W.h2d_states.as<uint8_t>(), (int)n, W.out_len.as<int32_t>(),
                   W.out_nodes.as<uint64_t>(), st, O, width);
    if (hipMemcpyAsync(out_len, W.out_len.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(out_nodes_per_threshold, W.out_nodes.p, n * BPIDA_MAX_THRESHOLDS * sizeof(uint64_t),
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return BPIDA_EDEVICE;
    return rc;
  } catch (const std::bad_alloc&) {
    return BPIDA_ENOMEM;
  } catch (...) {
    return BPIDA_EINTERNAL;
  }
}

extern "C" int bpida_solve_paths(const uint8_t* states, int32_t n_instances, int32_t width,
                                 int32_t* out_len, uint64_t* out_nodes_per_threshold, uint8_t* out_path) {
  try {
    if (!states || !out_len || !out_nodes_per_threshold || !out_path || n_instances < 0)
      return BPIDA_EINVAL;
    if (check_opts(width) != BPIDA_OK) return BPIDA_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    const Options O = g_opt;
    const size_t n = (size_t)n_instances;
    if (n == 0) return BPIDA_OK;
    int rc = ensure_device();
    if (rc != BPIDA_OK) return rc;
    Workspace& W = g_ws;
    hipStream_t st = nullptr;
    const size_t bytes = n * (size_t)width * (size_t)width;
    if (W.h2d_states.ensure(bytes) != hipSuccess || W.out_len.ensure(n * sizeof(int32_t)) != hipSuccess ||
        W.out_nodes.ensure(n * BPIDA_MAX_THRESHOLDS * sizeof(uint64_t)) != hipSuccess ||
        W.out_path.ensure(n * BPIDA_MAX_PATH) != hipSuccess)
      return BPIDA_ENOMEM;
    if (hipMemcpyAsync(W.h2d_states.p, states, bytes, hipMemcpyHostToDevice, st) != hipSuccess)
      return BPIDA_EDEVICE;
    rc = run_paths(W.h2d_states.as<uint8_t>(), (int)n, width, W.out_len.as<int32_t>(),
                   W.out_nodes.as<uint64_t>(), W.out_path.as<uint8_t>(), st, O);
    if (hipMemcpyAsync(out_len, W.out_len.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(out_nodes_per_threshold, W.out_nodes.p, n * BPIDA_MAX_THRESHOLDS * sizeof(uint64_t),
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(out_path, W.out_path.p, n * BPIDA_MAX_PATH, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return BPIDA_EDEVICE;
    return rc;
  } catch (const std::bad_alloc&) {
    return BPIDA_ENOMEM;
  } catch (...) {
    return BPIDA_EINTERNAL;
  }
}

extern "C" int bpida_solve_paths_device(const uint8_t* d_states, int32_t n_instances, int32_t width,
                                        int32_t* d_len, uint64_t* d_nodes, uint8_t* d_path,
                                        void* hip_stream) {
  try {
    if (!d_states || !d_len || !d_nodes || !d_path || n_instances < 0) return BPIDA_EINVAL;
    if (check_opts(width) != BPIDA_OK) return BPIDA_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    const Options O = g_opt;
    if (n_instances == 0) return BPIDA_OK;
    int rc = ensure_device();
    if (rc != BPIDA_OK) return rc;
    return run_paths(d_states, n_instances, width, d_len, d_nodes, d_path, (hipStream_t)hip_stream, O);
  } catch (const std::bad_alloc&) {
    return BPIDA_ENOMEM;
  } catch (...) {
    return BPIDA_EINTERNAL;
  }
}

extern "C" int bpida_solve_mixed(const uint8_t* states, const int32_t* widths, int32_t n_instances,
                                 int32_t* out_len, uint64_t* out_nodes_per_threshold) {
  try {
    if (!states || !widths || !out_len || !out_nodes_per_threshold || n_instances < 0) return BPIDA_EINVAL;
    size_t bytes = 0;
    for (int32_t i = 0; i < n_instances; ++i) {
      if (widths[i] < BPIDA_MIN_WIDTH || widths[i] > BPIDA_MAX_WIDTH) return BPIDA_EINVAL;
      bytes += (size_t)widths[i] * (size_t)widths[i];
    }
    std::lock_guard<std::mutex> lk(g_mu);
    Options O = g_opt;
    O.mode = kModeBatched;
    const size_t n = (size_t)n_instances;
    if (n == 0) return BPIDA_OK;
    int rc = ensure_device();
    if (rc != BPIDA_OK) return rc;
    Workspace& W = g_ws;
    hipStream_t st = nullptr;
    if (W.h2d_states.ensure(bytes) != hipSuccess || W.out_len.ensure(n * sizeof(int32_t)) != hipSuccess ||
        W.out_nodes.ensure(n * BPIDA_MAX_THRESHOLDS * sizeof(uint64_t)) != hipSuccess)
      return BPIDA_ENOMEM;
    if (hipMemcpyAsync(W.h2d_states.p, states, bytes, hipMemcpyHostToDevice, st) != hipSuccess)
      return BPIDA_EDEVICE;
    rc = run_batched(W.h2d_states.as<uint8_t>(), (int)n, W.out_len.as<int32_t>(),
                     W.out_nodes.as<uint64_t>(), st, O, 0, widths);
    if (hipMemcpyAsync(out_len, W.out_len.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(out_nodes_per_threshold, W.out_nodes.p, n * BPIDA_MAX_THRESHOLDS * sizeof(uint64_t),
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return BPIDA_EDEVICE;
    return rc;
  } catch (const std::bad_alloc&) {
    return BPIDA_ENOMEM;
  } catch (...) {
    return BPIDA_EINTERNAL;
  }
}

extern "C" int bpida_solve_mixed_device(const uint8_t* d_states, const int32_t* widths,
                                        int32_t n_instances, int32_t* d_len, uint64_t* d_nodes,
                                        void* hip_stream) {
  try {
    if (!d_states || !widths || !d_len || !d_nodes || n_instances < 0) return BPIDA_EINVAL;
    for (int32_t i = 0; i < n_instances; ++i)
      if (widths[i] < BPIDA_MIN_WIDTH || widths[i] > BPIDA_MAX_WIDTH) return BPIDA_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Options O = g_opt;
    O.mode = kModeBatched;
    if (n_instances == 0) return BPIDA_OK;
    int rc = ensure_device();
    if (rc != BPIDA_OK) return rc;
    return run_batched(d_states, n_instances, d_len, d_nodes, (hipStream_t)hip_stream, O, 0, widths);
  } catch (const std::bad_alloc&) {
    return BPIDA_ENOMEM;
  } catch (...) {
    return BPIDA_EINTERNAL;
  }
}

extern "C" int bpida_solve_device(const uint8_t* d_states, int32_t n_instances, int32_t width,
                                  int32_t* d_len, uint64_t* d_nodes, void* hip_stream) {
  try {
    if (!d_states || !d_len || !d_nodes || n_instances < 0) return BPIDA_EINVAL;
    if (check_opts(width) != BPIDA_OK) return BPIDA_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    const Options O = g_opt;
    if (n_instances == 0) return BPIDA_OK;
    int rc = ensure_device();
    if (rc != BPIDA_OK) return rc;
    return run_plain(d_states, n_instances, d_len, d_nodes, (hipStream_t)hip_stream, O, width);
  } catch (const std::bad_alloc&) {
    return BPIDA_ENOMEM;
  } catch (...) {
    return BPIDA_EINTERNAL;
  }
}

// ---------------------------------------------------------------------------
// Continuous-batching server.
// ---------------------------------------------------------------------------
namespace bpida {
namespace {

struct Server {
  bool running = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  uint64_t ring = 0;
  ServerHostCtl* host = nullptr;
  ServerReq* req = nullptr;
  ServerRes* res = nullptr;
  std::vector<uint8_t> collected;
  uint64_t tail = 0, min_uncollected = 0;
  DevBuf qctl, qseq, qslots, istate, tree, hist, goal_g, out_len, out_nodes, busy, ticket, admitter,
      inflight;
  int64_t grid = 0;
};

Server g_srv;

void free_server_host(Server& V) {
  if (V.host) (void)hipHostFree(V.host);
  if (V.req) (void)hipHostFree(V.req);
  if (V.res) (void)hipHostFree(V.res);
  V.host = nullptr;
  V.req = nullptr;
  V.res = nullptr;
}

}  // namespace
}  // namespace bpida

extern "C" int bpida_server_start(int32_t width, int32_t max_inflight, int32_t ring_capacity,
                                  void* hip_stream) {
  try {
    if (width != 4 || max_inflight < 1 || max_inflight > (1 << 16) ||
        ring_capacity < 1 || ring_capacity > (1 << 20))
      return BPIDA_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Server& V = g_srv;
    if (V.running) return BPIDA_EINVAL;
    int rc = ensure_device();
    if (rc != BPIDA_OK) return rc;
    Workspace& W = g_ws;
    Options O = g_opt;
    O.mode = kModeBatched;
    const int D = depth_for(O);
    const int npl = (int)O.nodes_per_round;
    const int cap = cap_for(O, npl);
    const int wpg = (int)(O.wg_size / 64);
    const int per_cu = batch4_max_blocks_per_cu(cap, npl, wpg);
    if (per_cu <= 0 || !ring_fits(4, cap, npl)) return BPIDA_EINVAL;
    int64_t grid = (int64_t)per_cu * W.num_cu;
    if (O.max_workgroups > 0) grid = std::min<int64_t>(grid, O.max_workgroups);
    if (grid * wpg < 2) return BPIDA_EINVAL;  // one admitter plus at least one searcher
    int64_t stride = 0, max_roots = 0;
    tree_size(W, 4, D, &stride, &max_roots);
    const int64_t S = max_inflight;
    uint64_t ring = 64;
    while (ring < (uint64_t)ring_capacity) ring <<= 1;
    const int sc_srv = (int)O.seed_chunk;
    uint64_t qcap = 64;
    // as a batch: the seeds of every slot plus, per workgroup, room for the
    // chunks its stack overflows into (smaller stacks spill more)
    const int64_t per_wg = std::min<int64_t>(64, std::max<int64_t>(16, 32768 / cap));
    const uint64_t want = O.queue_capacity > 0
                              ? (uint64_t)O.queue_capacity
                              : (uint64_t)(S * ((max_roots + sc_srv - 1) / sc_srv) + grid * wpg * per_wg + 1024);
    while (qcap < want) qcap <<= 1;
    free_server_host(V);
    if (V.qctl.ensure(sizeof(QueueCtl)) != hipSuccess || V.qseq.ensure(sizeof(SlotCtl) * qcap) != hipSuccess ||
        V.qslots.ensure(sizeof(QChunk) * qcap) != hipSuccess ||
        V.istate.ensure(sizeof(InstState) * S) != hipSuccess ||
        V.tree.ensure(sizeof(NodeW) * S * stride) != hipSuccess ||
        V.hist.ensure(sizeof(uint32_t) * kHistBins * S) != hipSuccess ||
        V.goal_g.ensure(sizeof(int32_t) * S) != hipSuccess ||
        V.out_len.ensure(sizeof(int32_t) * S) != hipSuccess ||
        V.out_nodes.ensure(sizeof(uint64_t) * 64 * S) != hipSuccess ||
        V.busy.ensure(sizeof(int32_t) * S) != hipSuccess ||
        V.ticket.ensure(sizeof(uint64_t) * S) != hipSuccess ||
        V.admitter.ensure(sizeof(int32_t)) != hipSuccess || V.inflight.ensure(sizeof(int32_t)) != hipSuccess)
      return BPIDA_ENOMEM;
    const unsigned fl = hipHostMallocCoherent | hipHostMallocMapped;
    if (hipHostMalloc((void**)&V.host, sizeof(ServerHostCtl), fl) != hipSuccess ||
        hipHostMalloc((void**)&V.req, sizeof(ServerReq) * ring, fl) != hipSuccess ||
        hipHostMalloc((void**)&V.res, sizeof(ServerRes) * ring, fl) != hipSuccess) {
      (void)hipGetLastError();
      free_server_host(V);
      return BPIDA_ENOMEM;
    }
    memset((void*)V.host, 0, sizeof(ServerHostCtl));
    memset((void*)V.req, 0, sizeof(ServerReq) * ring);
    memset((void*)V.res, 0, sizeof(ServerRes) * ring);
    V.ring = ring;
    V.collected.assign(ring, 0);
    V.tail = 0;
    V.min_uncollected = 0;
    V.grid = grid;
    if (hip_stream) {
      V.stream = (hipStream_t)hip_stream;
      V.own_stream = false;
    } else if (!V.stream || !V.own_stream) {
      if (hipStreamCreateWithFlags(&V.stream, hipStreamNonBlocking) != hipSuccess) return BPIDA_EDEVICE;
      V.own_stream = true;
    }
    BatchArgs A;
    memset(&A, 0, sizeof A);
    A.q = V.qctl.as<QueueCtl>();
    A.seq = V.qseq.as<SlotCtl>();
    A.slots = V.qslots.as<QChunk>();
    A.qmask = qcap - 1;
    A.is = V.istate.as<InstState>();
    A.tree = V.tree.as<NodeW>();
    A.hist = V.hist.as<uint32_t>();
    A.goal_g = V.goal_g.as<int32_t>();
    A.out_len = V.out_len.as<int32_t>();
    A.out_nodes = V.out_nodes.as<uint64_t>();
    A.n = 0;
    A.max_limit = (int)(O.max_threshold >= 0 ? std::min<int64_t>(O.max_threshold, kMaxLimit) : kMaxLimit);
    A.idle_ticks = ~0ull;  // waiting for requests is not a stall
    A.budget_ticks = (uint64_t)O.budget_ms * (uint64_t)W.wall_khz;
    A.donate_mask = (uint32_t)O.donate_every - 1u;
    A.donate_min = (int32_t)O.donate_min;
    A.donate_window = 2 * (int32_t)O.queue_chunk;
    A.first_solution = (int32_t)O.first_solution;
    A.start_limit = (int32_t)O.start_threshold;
    A.seed_chunk = sc_srv;
    A.push_spin = (int32_t)O.push_spin;
    A.server = 1;
    A.srv.host = V.host;
    A.srv.req = V.req;
    A.srv.res = V.res;
    A.srv.ring_mask = ring - 1;
    A.srv.slots = (int32_t)S;
    A.srv.depth = D;
    A.srv.stride = stride;
    A.srv.busy = V.busy.as<int32_t>();
    A.srv.ticket = V.ticket.as<uint64_t>();
    A.srv.walks = W.d_walks + kWalkStride;
    A.srv.admitter = V.admitter.as<int32_t>();
    A.srv.in_flight = V.inflight.as<int32_t>();
    A.srv.backlog_max = O.admit_backlog < 0 ? (int64_t)(qcap / 2) : O.admit_backlog;
    if (launch_zero_words(V.qctl.p, sizeof(QueueCtl), V.stream) != hipSuccess ||
        launch_server_setup(A, V.stream) != hipSuccess ||
        launch_batch4(cap, npl, wpg, (int)grid, A, V.stream) != hipSuccess) {
      (void)hipGetLastError();
      return BPIDA_EDEVICE;
    }
    V.running = true;
    return BPIDA_OK;
  } catch (const std::bad_alloc&) {
    return BPIDA_ENOMEM;
  } catch (...) {
    return BPIDA_EINTERNAL;
  }
}

extern "C" int bpida_server_submit(const uint8_t* state, uint64_t* ticket) {
  if (!state || !ticket) return BPIDA_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  Server& V = g_srv;
  if (!V.running) return BPIDA_EINVAL;
  const uint64_t admitted = __atomic_load_n(&V.host->req_admitted, __ATOMIC_ACQUIRE);
  if (V.tail - V.min_uncollected >= V.ring || V.tail - admitted >= V.ring) return BPIDA_EAGAIN;
  memcpy(V.req[V.tail & (V.ring - 1)].state, state, 16);
  std::atomic_thread_fence(std::memory_order_release);
  __atomic_store_n(&V.host->req_tail, V.tail + 1, __ATOMIC_RELEASE);
  *ticket = V.tail++;
  return BPIDA_OK;
}

extern "C" int bpida_server_poll(uint64_t ticket, int32_t* out_len, uint64_t* out_nodes,
                                 int32_t* status) {
  if (!out_len || !out_nodes || !status) return BPIDA_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  Server& V = g_srv;
  if (!V.res || ticket >= V.tail || ticket < V.min_uncollected || V.collected[ticket & (V.ring - 1)])
    return BPIDA_EINVAL;
  const ServerRes* r = V.res + (ticket & (V.ring - 1));
  if (__atomic_load_n(&r->seq, __ATOMIC_ACQUIRE) != ticket + 1) return 0;
  *out_len = r->len;
  *status = r->status;
  memcpy(out_nodes, (const void*)r->nodes, sizeof(uint64_t) * 64);
  V.collected[ticket & (V.ring - 1)] = 1;
  while (V.min_uncollected < V.tail && V.collected[V.min_uncollected & (V.ring - 1)]) {
    V.collected[V.min_uncollected & (V.ring - 1)] = 0;
    ++V.min_uncollected;
  }
  return 1;
}

extern "C" int bpida_server_stop(void) {
  try {
    std::lock_guard<std::mutex> lk(g_mu);
    Server& V = g_srv;
    if (!V.running) return BPIDA_EINVAL;
    __atomic_store_n(&V.host->stop, 1, __ATOMIC_RELEASE);
    QueueCtl qc;
    if (hipStreamSynchronize(V.stream) != hipSuccess ||
        hipMemcpy(&qc, V.qctl.p, sizeof(QueueCtl), hipMemcpyDeviceToHost) != hipSuccess) {
      (void)hipGetLastError();
      V.running = false;
      return BPIDA_EDEVICE;
    }
    V.running = false;
    uint64_t stats[kStats] = {0};
    stats[0] = qc.rounds;
    stats[1] = qc.searched;
    stats[2] = qc.pushes * kQChunk;
    stats[3] = 1;
    stats[6] = qc.pushes;
    stats[7] = qc.pops;
    stats[11] = qc.voluntary;
    stats[12] = (uint64_t)V.grid;
    stats[13] = (uint64_t)(uint32_t)qc.err;
    memcpy(g_stats, stats, sizeof stats);
    if (qc.err & kErrFatal) return BPIDA_ENOMEM;
    if (qc.err) return BPIDA_EINTERNAL;
    return BPIDA_OK;
  } catch (...) {
    return BPIDA_EINTERNAL;
  }
}

extern "C" int bpida_solve_device_async(const uint8_t* d_states, int32_t n_instances, int32_t width,
                                        int32_t* d_len, uint64_t* d_nodes, int32_t* d_status,
                                        void* hip_stream) {
  try {
    if (!d_states || !d_len || !d_nodes || !d_status || n_instances < 0) return BPIDA_EINVAL;
    if (check_opts(width) != BPIDA_OK) return BPIDA_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    const Options O = g_opt;
    if (n_instances == 0) return BPIDA_OK;
    int rc = ensure_device();
    if (rc != BPIDA_OK) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
      (void)hipGetLastError();
      return BPIDA_EDEVICE;
    }
    g_no_alloc = cs != hipStreamCaptureStatusNone;
    int64_t grid = 0;
    Options Ob = O;
    Ob.mode = kModeBatched;
    rc = enqueue_batched(d_states, n_instances, d_len, d_nodes, d_status, st, Ob, false, &grid, width);
    g_no_alloc = false;
    return rc;
  } catch (const std::bad_alloc&) {
    g_no_alloc = false;
    return BPIDA_ENOMEM;
  } catch (...) {
    g_no_alloc = false;
    return BPIDA_EINTERNAL;
  }
}

extern "C" int bpida_set_option(const char* key, int64_t value) {
  if (!key) return BPIDA_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  const std::string k(key);
  if (k == "mode") {
    if (value != kModePlain && value != kModeBatched) return BPIDA_EINVAL;
    g_opt.mode = value;
  } else if (k == "budget_ms") {
    if (value < 1 || value > 36000000) return BPIDA_EINVAL;
    g_opt.budget_ms = value;
  } else if (k == "watchdog_ms") {
    if (value < 1 || value > 3600000) return BPIDA_EINVAL;
    g_opt.watchdog_ms = value;
  } else if (k == "queue_capacity") {
    if (value < 0 || value > (int64_t(1) << 24)) return BPIDA_EINVAL;
    g_opt.queue_capacity = value;
  } else if (k == "frontier_depth") {
    if (value < -1 || value > kMaxDepth) return BPIDA_EINVAL;
    g_opt.frontier_depth = value;
  } else if (k == "lds_stack_capacity") {
    if (value != -1 && value != 128 && value != 256 && value != 512 && value != 640 &&
        value != 672 && value != 768 && value != 1024 && value != 2048)
      return BPIDA_EINVAL;
    g_opt.lds_stack_capacity = value;
  } else if (k == "nodes_per_round") {
    if (value != 16 && value != 64) return BPIDA_EINVAL;
    g_opt.nodes_per_round = value;
  } else if (k == "spill_capacity") {
    if (value < 64 || value > (1 << 24) || value % 64) return BPIDA_EINVAL;
    g_opt.spill_capacity = value;
  } else if (k == "max_workgroups") {
    if (value < 0 || value > (1 << 20)) return BPIDA_EINVAL;
    g_opt.max_workgroups = value;
  } else if (k == "max_threshold") {
    if (value < -1 || value > kMaxLimit) return BPIDA_EINVAL;
    g_opt.max_threshold = value;
  } else if (k == "donate_every") {
    if (value < 4 || value > 1024 || (value & (value - 1))) return BPIDA_EINVAL;
    g_opt.donate_every = value;
  } else if (k == "seed_chunk") {
    if (value != 8 && value != 16 && value != 32 && value != 64) return BPIDA_EINVAL;
    g_opt.seed_chunk = value;
  } else if (k == "start_threshold") {
    if (value < -1 || value > kMaxLimit) return BPIDA_EINVAL;
    g_opt.start_threshold = value;
  } else if (k == "static_lb") {
    if (value != 0 && value != 1) return BPIDA_EINVAL;
    g_opt.static_lb = value;
  } else if (k == "first_solution") {
    if (value != 0 && value != 1) return BPIDA_EINVAL;
    g_opt.first_solution = value;
  } else if (k == "queue_chunk") {
    if (value != 16 && value != 32 && value != 64) return BPIDA_EINVAL;
    g_opt.queue_chunk = value;
  } else if (k == "admit_backlog") {
    if (value < -1 || value > (int64_t(1) << 24)) return BPIDA_EINVAL;
    g_opt.admit_backlog = value;
  } else if (k == "wg_size") {
    if (value != 64 && value != 128 && value != 256) return BPIDA_EINVAL;
    g_opt.wg_size = value;
  } else if (k == "plain_nodes_per_round") {
    if (value != 16 && value != 64) return BPIDA_EINVAL;
    g_opt.plain_nodes_per_round = value;
  } else if (k == "push_spin") {
    if (value < 1 || value > (int64_t(1) << 24)) return BPIDA_EINVAL;
    g_opt.push_spin = value;
  } else if (k == "donate_min") {
    if (value != -1 && (value < 2 || value > 2048)) return BPIDA_EINVAL;
    g_opt.donate_min = value;
  } else {
    return BPIDA_EINVAL;
  }
  return BPIDA_OK;
}

extern "C" int64_t bpida_get_option(const char* key) {
  if (!key) return INT64_MIN;
  std::lock_guard<std::mutex> lk(g_mu);
  const std::string k(key);
  if (k == "mode") return g_opt.mode;
  if (k == "queue_capacity") return g_opt.queue_capacity;
  if (k == "watchdog_ms") return g_opt.watchdog_ms;
  if (k == "budget_ms") return g_opt.budget_ms;
  if (k == "frontier_depth") return g_opt.frontier_depth;
  if (k == "lds_stack_capacity") return g_opt.lds_stack_capacity;
  if (k == "nodes_per_round") return g_opt.nodes_per_round;
  if (k == "spill_capacity") return g_opt.spill_capacity;
  if (k == "max_workgroups") return g_opt.max_workgroups;
  if (k == "max_threshold") return g_opt.max_threshold;
  if (k == "donate_every") return g_opt.donate_every;
  if (k == "donate_min") return g_opt.donate_min;
  if (k == "queue_chunk") return g_opt.queue_chunk;
  if (k == "first_solution") return g_opt.first_solution;
  if (k == "static_lb") return g_opt.static_lb;
  if (k == "start_threshold") return g_opt.start_threshold;
  if (k == "seed_chunk") return g_opt.seed_chunk;
  if (k == "push_spin") return g_opt.push_spin;
  if (k == "plain_nodes_per_round") return g_opt.plain_nodes_per_round;
  if (k == "wg_size") return g_opt.wg_size;
  if (k == "admit_backlog") return g_opt.admit_backlog;
  return INT64_MIN;
}

extern "C" int bpida_last_stats(uint64_t* out, int32_t n) {
  if (!out || n < 0 || n > kStats) return BPIDA_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  for (int i = 0; i < n; ++i) out[i] = g_stats[i];
  return BPIDA_OK;
}

extern "C" const char* bpida_strerror(int code) {
  switch (code) {
    case BPIDA_OK: return "ok";
    case BPIDA_EINVAL: return "invalid argument or state";
    case BPIDA_EUNSOLVABLE: return "unsolvable state (parity)";
    case BPIDA_ELIMIT: return "f-limit cap reached";
    case BPIDA_ENOMEM: return "out of device memory or spill area";
    case BPIDA_EDEVICE: return "no usable gfx950 device or HIP failure";
    case BPIDA_EINTERNAL: return "internal consistency check failed";
    case BPIDA_EAGAIN: return "server request ring full, try again";
    default: return "unknown status";
  }
}

// ---------------------------------------------------------------------------
// Batched solve that allocates nothing: every buffer is carved from one
// fixed device array per GPU, `scratch`.  Host code never uses the array's
// name as a device address: its address on each device comes from
// hipGetSymbolAddress, taken once per device with that device current.
// ---------------------------------------------------------------------------
namespace bpida {
namespace {

static __device__ __align__(256) uint8_t scratch[BPIDA_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxNoAllocDevices = 64;

struct NoAllocDevice {
  bool init = false;
  int rc = BPIDA_OK;
  uint8_t* ptr = nullptr;         // device address of `scratch` on this device
  const int32_t* walks = nullptr; // device address of the walk-count table
  int num_cu = 0;
  int wall_khz = 100000;
};

NoAllocDevice g_noalloc[kMaxNoAllocDevices];

// Once per device, with the device current: its properties and the device
// addresses of the scratch array and the walk table.
int noalloc_init(int dev) {
  NoAllocDevice& D = g_noalloc[dev];
  if (D.init) return D.rc;
  D.init = true;
  D.rc = BPIDA_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return D.rc;
  }
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return D.rc;
  D.num_cu = prop.multiProcessorCount;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
    D.wall_khz = khz;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return D.rc;
  }
  D.ptr = static_cast<uint8_t*>(p);
  if (walk_table_device(&D.walks) != hipSuccess || !D.walks) {
    (void)hipGetLastError();
    return D.rc;
  }
  D.rc = BPIDA_OK;
  return D.rc;
}

}  // namespace
}  // namespace bpida

extern "C" int bpida_solve_device_noalloc(const uint8_t* d_states, int32_t n_instances, int32_t width,
                                          int32_t* d_len, uint64_t* d_nodes, int32_t* d_status,
                                          void* hip_stream) {
  try {
    if (!d_states || !d_len || !d_nodes || !d_status || n_instances < 0) return BPIDA_EINVAL;
    if (check_opts(width) != BPIDA_OK) return BPIDA_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Options O = g_opt;
    O.mode = kModeBatched;
    if (n_instances == 0) return BPIDA_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxNoAllocDevices) {
      (void)hipGetLastError();
      return BPIDA_EDEVICE;
    }
    int rc = noalloc_init(dev);
    if (rc != BPIDA_OK) return rc;
    const NoAllocDevice& D = g_noalloc[dev];
    BatchPlan P;
    rc = plan_batched(n_instances, width, nullptr, O, D.num_cu, &P);
    if (rc != BPIDA_OK) return rc;
    // A queue sized from the batch may not fit: shrink it, never below the
    // seeds plus 1024 chunks (a queue that then overflows while searching
    // reports BPIDA_ENOMEM per instance); a queue_capacity option is kept.
    BatchBufs B;
    uint64_t qmin = 64;
    while (qmin < (uint64_t)P.seed_chunks + 1024) qmin <<= 1;
    while (O.queue_capacity == 0 && P.qcap > qmin &&
           carve_batched(0, P, &B) > (size_t)BPIDA_NOALLOC_SCRATCH_BYTES)
      P.qcap >>= 1;
    if (carve_batched(0, P, &B) > (size_t)BPIDA_NOALLOC_SCRATCH_BYTES) return BPIDA_ENOMEM;
    carve_batched((uintptr_t)D.ptr, P, &B);
    return enqueue_batched_into(d_states, d_len, d_nodes, d_status, (hipStream_t)hip_stream, O, P, B,
                                D.walks, nullptr, nullptr, nullptr, D.wall_khz);
  } catch (const std::bad_alloc&) {
    return BPIDA_ENOMEM;
  } catch (...) {
    return BPIDA_EINTERNAL;
  }
}
