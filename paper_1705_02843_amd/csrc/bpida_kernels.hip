// bpida_kernels.hip -- gfx950 kernels of Block-Parallel IDA* (15-puzzle).
//
//   ingest4  validate + pack + Manhattan h of each start state
//   split4   CreateRootSet (Alg. 1): the parent-pruned search tree expanded
//            level by level to depth D, no duplicate elimination; the
//            interior nodes are binned by f, the depth-D nodes become roots
//   search4  BPDFS (Alg. 1): one subtree per workgroup of one wave64; the
//            DFS stack lives in LDS; each round pops up to 16 nodes
//            (parallelPop with #threads / #actions = 64 / 4), lane l expands
//            node l/4 with move l%4 (the threadID mod #actions map), and the
//            surviving children are pushed with a ballot + mbcnt prefix
//            (atomicPut; one wave makes it a single linearizable step)
//   search64 the same launch with 64-node rounds: one popped node per lane,
//            its four moves unrolled (the batched kernel's round)
//   reduce   per-limit node total, next limit and goal flag (the min/stat
//            combine that Alg. 1 performs across its parallel blocks)
#include <limits.h>

#include "bpida_board.h"
#include "bpida_internal.h"
#include "bpida_round.h"

namespace bpida {

// ---------------------------------------------------------------------------
// ingest4: one thread per instance.
// ---------------------------------------------------------------------------
__global__ void ingest4_kernel(const uint8_t* __restrict__ states, int n, Inst* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint8_t* s = states + (size_t)i * 16;
  uint32_t v[16];
  uint32_t seen = 0;
  bool ok = true;
  int blank = 0;
  for (int p = 0; p < 16; ++p) {
    v[p] = s[p];
    if (v[p] >= 16 || (seen >> v[p]) & 1u) ok = false;
    seen |= 1u << (v[p] & 15u);
    if (v[p] == 0) blank = p;
  }
  Inst r;
  r.tiles = 0;
  r.blank = blank;
  r.h0 = 0;
  r.pad = 0;
  if (!ok) {
    r.status = -1;  // BPIDA_EINVAL
    out[i] = r;
    return;
  }
  uint32_t inv = 0;
  int h = 0;
  uint64_t tiles = 0;
  for (int p = 0; p < 16; ++p) {
    for (int q = p + 1; q < 16; ++q) inv ^= (v[p] > v[q]) ? 1u : 0u;
    tiles |= (uint64_t)v[p] << (4 * p);
    if (v[p] != 0) {
      const int dr = (p >> 2) - (int)(v[p] >> 2), dc = (p & 3) - (int)(v[p] & 3);
      h += (dr < 0 ? -dr : dr) + (dc < 0 ? -dc : dc);
    }
  }
  // solvable iff permutation parity == parity of the blank's distance to 0
  const uint32_t bpar = (uint32_t)((blank >> 2) + (blank & 3)) & 1u;
  r.tiles = tiles;
  r.h0 = h;
  r.status = (inv == bpar) ? 0 : -2;  // BPIDA_EUNSOLVABLE
  out[i] = r;
}

hipError_t launch_ingest4(const uint8_t* d_states, int n, Inst* d_inst, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(ingest4_kernel, dim3((n + 127) / 128), dim3(128), 0, s, d_states, n, d_inst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Shared move helper of the split kernel (scalar per thread).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int move_delta(int a) { return a == 0 ? -4 : a == 1 ? -1 : a == 2 ? 1 : 4; }

__device__ __forceinline__ int dh_grows(int a, uint32_t t, int n) {
  const int sh = (a == 0 || a == 3) ? 2 : 0;
  const uint32_t idx = (((t >> sh) & 3u) << 2) | (((uint32_t)n >> sh) & 3u);
  return (int)((kDhTable4 >> (16 * a + idx)) & 1ull);
}

// ---------------------------------------------------------------------------
// split4: one workgroup of 256 threads per instance.  Level d of the tree is
// stored after levels 0..d-1 in the instance's region (tree_off[i], or
// i * stride when tree_off is null).  Level sizes are exact: walks[c][d] is
// the number of non-backtracking blank walks of length d from cell c; a
// level whose fill differs from it raises `err`.  The depth-D level holds
// the roots; their offset and count go to root_off / nroots when given.
// ---------------------------------------------------------------------------
constexpr int kSplitThreads = 256;

__global__ __launch_bounds__(kSplitThreads) void split4_kernel(
    const Inst* __restrict__ inst, int depth, const int64_t* __restrict__ tree_off, int64_t stride,
    const int32_t* __restrict__ walks, Node* __restrict__ tree, uint32_t* __restrict__ hist,
    int32_t* __restrict__ goal_g, int32_t* __restrict__ err, int64_t* __restrict__ root_off,
    int32_t* __restrict__ nroots) {
  const int i = blockIdx.x;
  const Inst I = inst[i];
  __shared__ uint32_t h_lds[kHistBins];
  __shared__ int32_t fill;
  __shared__ int32_t gmin;
  for (int k = threadIdx.x; k < kHistBins; k += kSplitThreads) h_lds[k] = 0;
  if (threadIdx.x == 0) {
    gmin = INT_MAX;
    fill = 0;
  }
  const int64_t region = tree_off ? tree_off[i] : (int64_t)i * stride;
  Node* base = tree + region;
  if (I.status != 0) {
    __syncthreads();
    for (int k = threadIdx.x; k < kHistBins; k += kSplitThreads) hist[(size_t)i * kHistBins + k] = 0;
    if (threadIdx.x == 0) {
      goal_g[i] = INT_MAX;
      if (root_off) root_off[i] = region;
      if (nroots) nroots[i] = 0;
    }
    return;
  }
  const int32_t* lc = walks + walk_row(I.blank, 4);
  if (threadIdx.x == 0) {
    Node r;
    r.tiles = I.tiles;
    r.meta = node_meta(I.blank, 4, 0, I.h0);
    r.f = (uint32_t)I.h0;
    base[0] = r;
  }
  __syncthreads();
  int64_t lvl = 0;  // start of the current level inside base
  for (int d = 0; d < depth; ++d) {
    const int cnt = lc[d];
    const int64_t next = lvl + cnt;
    for (int k = threadIdx.x; k < cnt; k += kSplitThreads) {
      const Node nd = base[lvl + k];
      const int b = nd.meta & 31, fb = (nd.meta >> 5) & 7;
      const int g = (nd.meta >> 8) & 255, h = (nd.meta >> 16) & 255;
      atomicAdd(&h_lds[min(g + h, kHistBins - 1)], 1u);
      if (nd.tiles == kGoal4) atomicMin(&gmin, g);
      for (int a = 0; a < 4; ++a) {
        if (!((kMoveMask4 >> (4 * b + a)) & 1ull) || a == fb) continue;
        const int nn = b + move_delta(a);
        const uint32_t t = (uint32_t)(nd.tiles >> (4 * nn)) & 15u;
        const int h2 = h + (dh_grows(a, t, nn) ? 1 : -1);
        Node c;
        c.tiles = nd.tiles + ((uint64_t)t << (4 * b)) - ((uint64_t)t << (4 * nn));
        c.meta = node_meta(nn, 3 - a, g + 1, h2);
        c.f = (uint32_t)(g + 1 + h2);
        const int slot = atomicAdd(&fill, 1);
        if (slot < lc[d + 1]) base[next + slot] = c;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      if (fill != lc[d + 1]) atomicOr(err, 1);
      fill = 0;
    }
    lvl = next;
    __syncthreads();
  }
  for (int k = threadIdx.x; k < kHistBins; k += kSplitThreads) hist[(size_t)i * kHistBins + k] = h_lds[k];
  if (threadIdx.x == 0) {
    goal_g[i] = gmin;
    if (root_off) root_off[i] = region + lvl;
    if (nroots) nroots[i] = lc[depth];
  }
}

hipError_t launch_split4(const Inst* d_inst, int n, int depth, const int64_t* d_tree_off,
                         int64_t stride, const int32_t* d_walks, Node* d_tree, uint32_t* d_hist,
                         int32_t* d_goal_g, int32_t* d_err, int64_t* d_root_off, int32_t* d_nroots,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(split4_kernel, dim3(n), dim3(kSplitThreads), 0, s, d_inst, depth, d_tree_off,
                     stride, d_walks, d_tree, d_hist, d_goal_g, d_err, d_root_off, d_nroots);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// search4: BPDFS.  Persistent grid: each workgroup (one wave64) takes subtree
// roots through an atomic cursor and searches each to completion.
//
// LDS stack: a ring of CAP entries, SoA (u64 tiles, u16 meta), positions
// [bot, top) used.  Stack meta: bits 0..4 blank, 5..7 forbidden move
// (4 = none), 8..15 slack = limit - g - h (>= 0; a child has slack - 1 - dh).
// When a round could overflow the ring, the 64 oldest entries move to this
// workgroup's HBM spill stack; when fewer than 16 entries remain and the
// spill stack is not empty, 64 entries come back below bot.  Every entry is
// popped exactly once, so the node count is exact in any order.
// ---------------------------------------------------------------------------
constexpr int kChunk = 64;



template <int CAP>
__global__ __launch_bounds__(64) void search4_kernel(const Node* __restrict__ roots, int nroots,
                                                     int limit, int32_t* __restrict__ cursor,
                                                     uint64_t* __restrict__ spill_tiles,
                                                     uint16_t* __restrict__ spill_meta,
                                                     int spill_cap, Partial* __restrict__ part,
                                                     int32_t* __restrict__ stop,
                                                     uint32_t* __restrict__ load) {
  // stop: null, or (first-solution mode) a flag the workgroup that expands a
  // goal sets; the others see it within 64 rounds and drop their work.
  // load: null, or per root the repetitions of the round loop its subtree
  // took (the work estimate of the static load balancing)
  static_assert((CAP & (CAP - 1)) == 0 && CAP >= 128, "ring size");
  __shared__ uint64_t st[CAP];
  __shared__ uint16_t sm[CAP];

  const int lane = threadIdx.x;
  const LaneMap M = make_lane_map(lane);

  uint64_t* sp_t = spill_tiles + (size_t)blockIdx.x * spill_cap;
  uint16_t* sp_m = spill_meta + (size_t)blockIdx.x * spill_cap;

  uint64_t expanded = 0, rounds = 0, spilled = 0;
  int goals = 0;
  int fmin = INT_MAX;  // per lane
  int err = 0;
  int spill_hw = 0;

  bool stopped = false;
  for (;;) {
    if (stop && wave_bcast(lane == 0 ? __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0))
      break;
    int r = 0;
    if (lane == 0) r = atomicAdd(cursor, 1);
    r = __builtin_amdgcn_readfirstlane(__shfl(r, 0, 64));
    if (r >= nroots) break;
    const Node R = roots[r];
    if ((int)R.f > limit) {
      fmin = min(fmin, (int)R.f);
      continue;
    }
    if (lane == 0) {
      st[0] = R.tiles;
      sm[0] = (uint16_t)((R.meta & 0xFFu) | ((uint32_t)(limit - (int)R.f) << 8));
    }
    WAVE_SYNC();
    const uint64_t rounds0 = rounds;
    uint32_t top = 1, bot = 0;  // unsigned ring positions: they wrap
    int sp = 0;
    for (;;) {
      int avail = (int)(top - bot);
      if (avail < 16 && sp > 0 && avail + kChunk <= CAP) {
        sp -= kChunk;
        bot -= kChunk;
        const uint32_t p = (bot + (uint32_t)lane) & (CAP - 1);
        st[p] = sp_t[sp + lane];
        sm[p] = sp_m[sp + lane];
        avail += kChunk;
        WAVE_SYNC();
      }
      if (avail == 0) break;
      if (avail + 32 > CAP) {
        if (sp + kChunk > spill_cap) {
          err = 1;  // entries are dropped; the host reports BPIDA_ENOMEM
        } else {
          const uint32_t p = (bot + (uint32_t)lane) & (CAP - 1);
          sp_t[sp + lane] = st[p];
          sp_m[sp + lane] = sm[p];
          sp += kChunk;
          spilled += kChunk;
          spill_hw = max(spill_hw, sp);
        }
        bot += kChunk;
        avail -= kChunk;
        WAVE_SYNC();
      }
      // parallelPop + expand + atomicPut
      const int kp = min(avail, 16);
      top = bp_round<CAP>(st, sm, top, kp, limit, M, goals, fmin);
      expanded += (uint64_t)kp;
      rounds += 1;
      if (stop) {
        if (goals > 0) {
          if (lane == 0) __hip_atomic_store(stop, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          stopped = true;
          break;
        }
        if ((rounds & 63u) == 0 &&
            wave_bcast(lane == 0 ? __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0)) {
          stopped = true;
          break;
        }
      }
    }
    if (load && lane == 0) load[r] = (uint32_t)min<uint64_t>(rounds - rounds0, 0xFFFFFFFFull);
    if (stopped) break;
  }
  fmin = wave_min(fmin);
  if (lane == 0) {
    Partial P;
    P.nodes = expanded;
    P.rounds = rounds;
    P.spilled = spilled;
    P.fmin = fmin;
    P.goals = goals;
    P.err = err;
    P.spill_hw = spill_hw;
    part[blockIdx.x] = P;
  }
}

// search64: as search4 (persistent grid, roots through the cursor, HBM spill
// stack per workgroup, first-solution stop flag, per-root round counts for
// the static load balancing), with 64-node rounds on a linear LDS stack
// [0, top) (the round's stores are branch-free, under the keep mask).  The
// oldest 64 entries go to the spill stack when the largest round (128 new
// entries: three children a node; the start node, alone in the first round,
// may have four) might not fit; when fewer than 64 entries remain, the last
// spilled chunk comes back below them.
template <int CAP>
__global__ __launch_bounds__(64) void search64_kernel(const Node* __restrict__ roots, int nroots,
                                                      int limit, int32_t* __restrict__ cursor,
                                                      uint64_t* __restrict__ spill_tiles,
                                                      uint16_t* __restrict__ spill_meta,
                                                      int spill_cap, Partial* __restrict__ part,
                                                      int32_t* __restrict__ stop,
                                                      uint32_t* __restrict__ load) {
  static_assert((CAP & (CAP - 1)) == 0 && CAP >= 512, "stack size for 64-node rounds");
  // the width-4 round's stack (its layout for this size)
  __shared__ __attribute__((aligned(16))) uint64_t lds[stack4_bytes<CAP>() / 8];
  uint64_t* st = lds;
  constexpr uint32_t kCap = CAP;
  // largest growth of one round: at most 3 children a node (a unit starts
  // from one root, whose round cannot overflow)
  constexpr uint32_t kGrow = 2 * 64;

  const int lane = threadIdx.x;
  uint64_t* sp_t = spill_tiles + (size_t)blockIdx.x * spill_cap;
  uint16_t* sp_m = spill_meta + (size_t)blockIdx.x * spill_cap;

  uint64_t expanded = 0, rounds = 0, spilled = 0;
  int goals = 0;
  int fmin = INT_MAX;
  int err = 0;
  int spill_hw = 0;

  const RoundConsts4 rk = make_round_consts4();
  bool stopped = false;
  for (;;) {
    if (stop && wave_bcast(lane == 0 ? __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0))
      break;
    int r = 0;
    if (lane == 0) r = atomicAdd(cursor, 1);
    r = wave_bcast(r);
    if (r >= nroots) break;
    const Node R = roots[r];
    if ((int)R.f > limit) {
      fmin = min(fmin, (int)R.f);
      continue;
    }
    // (the width-4 round's meta layout)
    if (lane == 0) e4_put<CAP>(st, 0, R.tiles, meta4_in((R.meta & 0xFFu) | ((uint32_t)(limit - (int)R.f) << 8)));
    WAVE_SYNC();
    const uint64_t rounds0 = rounds;
    uint32_t top = 1;
    int sp = 0;
    for (;;) {
      if (top < 64u && sp > 0) {
        // the last spilled chunk comes back below the remaining entries
        uint64_t t = 0;
        uint32_t m = 0;
        if ((uint32_t)lane < top) {
          t = e4_tile<CAP>(st, lane);
          m = e4_meta<CAP>(st, lane);
        }
        WAVE_SYNC();
        if ((uint32_t)lane < top) e4_put<CAP>(st, 64 + lane, t, m);
        sp -= 64;
        e4_put<CAP>(st, lane, sp_t[sp + lane], sp_m[sp + lane]);
        top += 64u;
        WAVE_SYNC();
      }
      if (top == 0) break;
      if (top + kGrow > kCap) {
        if (sp + 64 > spill_cap) {
          err = 1;  // entries are dropped; the host reports BPIDA_ENOMEM
        } else {
          sp_t[sp + lane] = e4_tile<CAP>(st, lane);
          sp_m[sp + lane] = (uint16_t)e4_meta<CAP>(st, lane);
          sp += 64;
          spilled += 64;
          spill_hw = max(spill_hw, sp);
        }
        WAVE_SYNC();
        move_down4<CAP>(st, 0u, 64u, top - 64u);
        top -= 64u;
      }
      const int kp = (int)min(top, 64u);
      top = bp_round64_4<CAP, false>(st, top, kp, goals, rk);
      expanded += (uint64_t)kp;
      rounds += 1;
      if (!stop) {
        // all-solutions search: full rounds back to back while the stack
        // holds 64 entries and has room for their children (no spill or
        // refill due); counts are added once at the end
        uint64_t gm = 0;  // lanes that expanded a goal (only "any" matters)
        uint32_t n = 0;
        while (top - 64u <= kCap - kGrow - 64u) {
          top = bp_round64_4<CAP, true>(st, top, 64, gm, rk);
          ++n;
        }
        if (gm != 0) goals += 1;
        expanded += 64ull * n;
        rounds += n;
      } else {
        if (goals > 0) {
          if (lane == 0) __hip_atomic_store(stop, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          stopped = true;
          break;
        }
        if ((rounds & 63u) == 0 &&
            wave_bcast(lane == 0 ? __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0)) {
          stopped = true;
          break;
        }
      }
    }
    if (load && lane == 0) load[r] = (uint32_t)min<uint64_t>(rounds - rounds0, 0xFFFFFFFFull);
    if (stopped) break;
  }
  // 64-node rounds do not track pruned f: every pruned child has f = limit + 2
  // (all slacks are even), and a limit below the optimum always prunes one
  if (expanded > 0) fmin = min(fmin, limit + 2);
  fmin = wave_min(fmin);
  if (lane == 0) {
    Partial P;
    P.nodes = expanded;
    P.rounds = rounds;
    P.spilled = spilled;
    P.fmin = fmin;
    P.goals = goals;
    P.err = err;
    P.spill_hw = spill_hw;
    part[blockIdx.x] = P;
  }
}

template <int CAP>
static hipError_t launch_search4_t(int grid, const Node* d_roots, int nroots, int limit,
                                   int32_t* d_cursor, uint64_t* d_st, uint16_t* d_sm, int spill_cap,
                                   Partial* d_part, int32_t* d_stop, uint32_t* d_load, hipStream_t s) {
  hipLaunchKernelGGL(search4_kernel<CAP>, dim3(grid), dim3(64), 0, s, d_roots, nroots, limit,
                     d_cursor, d_st, d_sm, spill_cap, d_part, d_stop, d_load);
  return hipGetLastError();
}

template <int CAP>
static hipError_t launch_search64_t(int grid, const Node* d_roots, int nroots, int limit,
                                    int32_t* d_cursor, uint64_t* d_st, uint16_t* d_sm, int spill_cap,
                                    Partial* d_part, int32_t* d_stop, uint32_t* d_load, hipStream_t s) {
  hipLaunchKernelGGL(search64_kernel<CAP>, dim3(grid), dim3(64), 0, s, d_roots, nroots, limit,
                     d_cursor, d_st, d_sm, spill_cap, d_part, d_stop, d_load);
  return hipGetLastError();
}

hipError_t launch_search4(int lds_cap, int npl, int grid, const Node* d_roots, int nroots, int limit,
                          int32_t* d_cursor, uint64_t* d_spill_tiles, uint16_t* d_spill_meta,
                          int spill_cap, Partial* d_part, int32_t* d_stop, uint32_t* d_load,
                          hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (npl == 64) {
    switch (lds_cap) {
#define CASE(C)                                                                                 \
  case C:                                                                                       \
    return launch_search64_t<C>(grid, d_roots, nroots, limit, d_cursor, d_spill_tiles,          \
                                d_spill_meta, spill_cap, d_part, d_stop, d_load, s);
      CASE(512) CASE(1024) CASE(2048)
#undef CASE
      default:
        return hipErrorInvalidValue;
    }
  }
  if (npl != 16) return hipErrorInvalidValue;
  switch (lds_cap) {
#define CASE(C)                                                                                 \
  case C:                                                                                       \
    return launch_search4_t<C>(grid, d_roots, nroots, limit, d_cursor, d_spill_tiles,           \
                               d_spill_meta, spill_cap, d_part, d_stop, d_load, s);
    CASE(128) CASE(256) CASE(512) CASE(1024) CASE(2048)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

int search4_max_blocks_per_cu(int lds_cap, int npl) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  if (npl == 64) {
    switch (lds_cap) {
      case 512: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, search64_kernel<512>, 64, 0); break;
      case 1024: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, search64_kernel<1024>, 64, 0); break;
      case 2048: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, search64_kernel<2048>, 64, 0); break;
      default: break;
    }
    return e == hipSuccess ? nb : 0;
  }
  if (npl != 16) return 0;
  switch (lds_cap) {
    case 128: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, search4_kernel<128>, 64, 0); break;
    case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, search4_kernel<256>, 64, 0); break;
    case 512: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, search4_kernel<512>, 64, 0); break;
    case 1024: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, search4_kernel<1024>, 64, 0); break;
    case 2048: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, search4_kernel<2048>, 64, 0); break;
    default: break;
  }
  return e == hipSuccess ? nb : 0;
}

// ---------------------------------------------------------------------------
// reduce: one workgroup of 256 threads combines the partials of one search
// launch with the split tree's interior nodes at this limit, writes the
// node count into the output row, re-arms the root cursor and leaves a
// 48-byte result for the host driver.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void reduce_kernel(const Partial* __restrict__ part, int nwg,
                                                     const uint32_t* __restrict__ hist,
                                                     const int32_t* __restrict__ goal_g, int limit,
                                                     int col, uint64_t* __restrict__ nodes_row,
                                                     int32_t* __restrict__ cursor,
                                                     LimitResult* __restrict__ res) {
  __shared__ uint64_t s_nodes[256], s_rounds[256], s_spilled[256], s_searched[256];
  __shared__ int32_t s_fmin[256], s_goals[256], s_err[256], s_hw[256];
  const int tid = threadIdx.x;
  uint64_t nodes = 0, rounds = 0, spilled = 0;
  int fmin = INT_MAX, goals = 0, err = 0, hw = 0;
  for (int k = tid; k < nwg; k += 256) {
    const Partial P = part[k];
    nodes += P.nodes;
    rounds += P.rounds;
    spilled += P.spilled;
    fmin = min(fmin, P.fmin);
    goals += P.goals;
    err |= P.err;
    hw = max(hw, P.spill_hw);
  }
  const uint64_t searched = nodes;
  // interior nodes of the split tree: expanded at this limit iff f <= limit
  for (int f = tid; f < kHistBins; f += 256) {
    if (f <= limit) nodes += hist[f];
    else if (hist[f] != 0) fmin = min(fmin, f);
  }
  s_nodes[tid] = nodes; s_rounds[tid] = rounds; s_spilled[tid] = spilled; s_searched[tid] = searched;
  s_fmin[tid] = fmin; s_goals[tid] = goals; s_err[tid] = err; s_hw[tid] = hw;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      s_nodes[tid] += s_nodes[tid + o];
      s_rounds[tid] += s_rounds[tid + o];
      s_spilled[tid] += s_spilled[tid + o];
      s_searched[tid] += s_searched[tid + o];
      s_fmin[tid] = min(s_fmin[tid], s_fmin[tid + o]);
      s_goals[tid] += s_goals[tid + o];
      s_err[tid] |= s_err[tid + o];
      s_hw[tid] = max(s_hw[tid], s_hw[tid + o]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    const int found = (s_goals[0] > 0 || *goal_g <= limit) ? 1 : 0;
    nodes_row[col] = s_nodes[0];
    LimitResult R;
    R.nodes = s_nodes[0];
    R.fnext = s_fmin[0];
    R.found = found;
    R.err = s_err[0];
    R.spill_hw = s_hw[0];
    R.rounds = s_rounds[0];
    R.spilled = s_spilled[0];
    R.searched = s_searched[0];
    *res = R;
    *cursor = 0;
  }
}

hipError_t launch_reduce(const Partial* d_part, int nwg, const uint32_t* d_hist_i,
                         const int32_t* d_goal_g_i, int limit, int col, uint64_t* d_nodes_row,
                         int32_t* d_cursor, LimitResult* d_res, hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, s, d_part, nwg, d_hist_i, d_goal_g_i,
                     limit, col, d_nodes_row, d_cursor, d_res);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Output initialisation: len = -1, node rows = 0.
// ---------------------------------------------------------------------------
__global__ void fill_outputs_kernel(int32_t* __restrict__ len, uint64_t* __restrict__ nodes, int n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < (int64_t)n * 64) nodes[k] = 0;
  if (k < n) len[k] = -1;
}

hipError_t launch_fill_outputs(int32_t* d_len, uint64_t* d_nodes, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t tot = (int64_t)n * 64;
  hipLaunchKernelGGL(fill_outputs_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                     d_len, d_nodes, n);
  return hipGetLastError();
}

__global__ void set_len_kernel(int32_t* len, int32_t v) { *len = v; }

hipError_t launch_set_len(int32_t* d_len_i, int32_t value, hipStream_t s) {
  hipLaunchKernelGGL(set_len_kernel, dim3(1), dim3(1), 0, s, d_len_i, value);
  return hipGetLastError();
}

__global__ void zero_i32_kernel(int32_t* p, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0;
}

hipError_t launch_zero_i32(int32_t* d_p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d_p, n);
  return hipGetLastError();
}

__global__ void zero_words_kernel(uint32_t* p, size_t n) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0u;
}

hipError_t launch_zero_words(void* d_p, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 4;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     (uint32_t*)d_p, n);
  return hipGetLastError();
}

}  // namespace bpida
