// bpida_round.h -- one fetch-evaluate-expand round of BPDFS (Alg. 1) for a
// single wave64 on an LDS ring stack, shared by the search kernels.
#pragma once

#include <limits.h>

#include "bpida_internal.h"

namespace bpida {

// Orders this wave's LDS accesses across lanes: LDS executes one wave's
// operations in issue order, so a compiler-level barrier plus a wavefront
// fence is all that is needed between a lane's store and another lane's load.
#define WAVE_SYNC()                                        \
  do {                                                     \
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront"); \
    __builtin_amdgcn_wave_barrier();                       \
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront"); \
  } while (0)

// Lane of this thread within its wave64 (workgroups of the batched kernel
// may hold several independent waves).
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

// Orders this wave's LDS and global accesses across its lanes, like a
// workgroup barrier in a one-wave workgroup, without waiting for the other
// waves of the workgroup (which run independently).
#define WAVE_SYNC_MEM()                                    \
  do {                                                     \
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup"); \
    __builtin_amdgcn_wave_barrier();                       \
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup"); \
  } while (0)

// Per-lane constants of the lane -> (popped entry, move) map: lane l expands
// entry l/4 with move l%4 (the threadID mod #actions rule of Alg. 1).
struct LaneMap {
  int e;         // popped entry handled by this lane (0..15)
  int a;         // move: U, L, R, D = 0..3
  int delta;     // cell offset of the move
  uint32_t sh;   // 2: the move changes rows, 0: columns
  uint32_t tab;  // this move's 16-bit Manhattan "grows" table
};

__device__ __forceinline__ LaneMap make_lane_map(int lane) {
  LaneMap M;
  M.e = lane >> 2;
  M.a = lane & 3;
  M.delta = M.a == 0 ? -4 : M.a == 1 ? -1 : M.a == 2 ? 1 : 4;
  M.sh = (M.a == 0 || M.a == 3) ? 2u : 0u;
  M.tab = (uint32_t)(kDhTable4 >> (16 * M.a)) & 0xFFFFu;
  return M;
}

// Stack entry meta (16 bits): bits 0..4 blank cell, 5..7 forbidden move
// (inverse of the producing move, 4 = none), 8..15 slack = limit - g - h.
// Because Manhattan changes by exactly one per move, a child's slack is
// slack - 1 - dh, i.e. slack (tile moved toward its goal) or slack - 2, and
// f_new <= limit  <=>  child slack >= 0.
__device__ __forceinline__ uint16_t stack_meta(int blank, int forbid, int slack) {
  return (uint16_t)((uint32_t)blank | ((uint32_t)forbid << 5) | ((uint32_t)slack << 8));
}

// One round on the ring [bot, top) of capacity CAP (power of two).  Pops
// kp = min(16, top - bot) entries from the top (parallelPop), tests them for
// the goal, generates all legal non-undoing children and pushes those with
// f <= limit at the top (atomicPut: ballot + mbcnt prefix, one wave-wide
// step).  Returns the new top.  The caller guarantees top - bot + 2*kp <= CAP.
// Ring positions are unsigned and wrap; only top - bot is ever compared.
template <int CAP>
__device__ __forceinline__ uint32_t bp_round(uint64_t* st, uint16_t* sm, uint32_t top, int kp, int limit,
                                             const LaneMap& M, int& goals, int& fmin) {
  const uint32_t base = top - (uint32_t)kp;
  const uint32_t idx = (base + (uint32_t)M.e) & (CAP - 1);
  const uint64_t s = st[idx];
  const uint32_t m = sm[idx];
  const bool act = M.e < kp;
  // goal test on expansion: the popped node is counted and expanded like
  // any other; all its children exceed the limit
  goals += __popcll(__ballot(act && M.a == 0 && s == kGoal4));
  // applicability: the blank stays on the board and the move does not undo
  // the parent move
  const int b = (int)(m & 31u);
  const int fb = (int)((m >> 5) & 7u);
  const int slack = (int)(m >> 8);
  const bool legal = act && ((kMoveMask4 >> (4 * (b & 15) + M.a)) & 1ull) && M.a != fb;
  // successor: tile t at the neighbour cell n slides into the blank's cell
  const int n = (b + M.delta) & 15;
  const uint32_t t = (uint32_t)(s >> (4 * n)) & 15u;
  const uint32_t up = (M.tab >> ((((t >> M.sh) & 3u) << 2) | (((uint32_t)n >> M.sh) & 3u))) & 1u;
  const int slack2 = slack - 2 * (int)up;
  const bool keep = legal && slack2 >= 0;
  if (legal && slack2 < 0) fmin = min(fmin, limit - slack2);
  const uint64_t cs = s + ((uint64_t)t << (4 * b)) - ((uint64_t)t << (4 * n));
  const uint32_t cm = (uint32_t)n | ((uint32_t)(3 - M.a) << 5) | ((uint32_t)slack2 << 8);
  const uint64_t km = __ballot(keep);
  const uint32_t off = __builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
  if (keep) {
    const uint32_t p = (base + off) & (CAP - 1);
    st[p] = cs;
    sm[p] = (uint16_t)cm;
  }
  WAVE_SYNC();
  return base + (uint32_t)__popcll(km);
}

// Moves LDS stack entries [src, src + n) down to [dst, dst + n), dst < src,
// 64 at a time in ascending order: every entry is read before anything is
// written over it.
template <typename S>
__device__ __forceinline__ void move_down(S* st, uint16_t* sm, uint32_t dst, uint32_t src, uint32_t n) {
  const uint32_t lane = (uint32_t)lane_id();
  for (uint32_t i = 0; i < n; i += 64u) {
    const uint32_t k = i + lane;
    if (k < n) {
      const S t = st[src + k];
      const uint16_t m = sm[src + k];
      st[dst + k] = t;
      sm[dst + k] = m;
    }
  }
  WAVE_SYNC();
}

__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int wave_bcast(int v) {
  return __builtin_amdgcn_readfirstlane(v);
}

}  // namespace bpida
