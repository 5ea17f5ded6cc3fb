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

// Stack entry meta (16 bits): bits 0..3 blank cell, 4..6 forbidden move
// (inverse of the producing move, 4 = none), 8..15 slack = limit - g - h.
// Because Manhattan changes by exactly one per move, a child's slack is
// slack - 1 - dh, i.e. slack (tile moved toward its goal) or slack - 2, and
// f_new <= limit  <=>  child slack >= 0.
__device__ __forceinline__ uint16_t stack_meta(int blank, int forbid, int slack) {
  return (uint16_t)((uint32_t)blank | ((uint32_t)forbid << 4) | ((uint32_t)slack << 8));
}

// One round on the ring [bot, top) of capacity CAP (power of two).  Pops
// kp = min(16, top - bot) entries from the top (parallelPop), tests them for
// the goal, generates all legal non-undoing children and pushes those with
// f <= limit at the top (atomicPut: ballot + mbcnt prefix, one wave-wide
// step).  Returns the new top.  The caller guarantees top - bot + 2*kp <= CAP.
template <int CAP>
__device__ __forceinline__ int bp_round(uint64_t* st, uint16_t* sm, int top, int kp, int limit,
                                        const LaneMap& M, int& goals, int& fmin) {
  const int base = top - kp;
  const int idx = (base + M.e) & (CAP - 1);
  const uint64_t s = st[idx];
  const uint32_t m = sm[idx];
  const bool act = M.e < kp;
  // goal test on expansion: the popped node is counted and expanded like
  // any other; all its children exceed the limit
  goals += __popcll(__ballot(act && M.a == 0 && s == kGoal4));
  // applicability: the blank stays on the board and the move does not undo
  // the parent move
  const int b = (int)(m & 15u);
  const int fb = (int)((m >> 4) & 7u);
  const int slack = (int)(m >> 8);
  const bool legal = act && ((kMoveMask4 >> (4 * b + M.a)) & 1ull) && M.a != fb;
  // successor: tile t at the neighbour cell n slides into the blank's cell
  const int n = (b + M.delta) & 15;
  const uint32_t t = (uint32_t)(s >> (4 * n)) & 15u;
  const uint32_t up = (M.tab >> ((((t >> M.sh) & 3u) << 2) | (((uint32_t)n >> M.sh) & 3u))) & 1u;
  const int slack2 = slack - 2 * (int)up;
  const bool keep = legal && slack2 >= 0;
  if (legal && slack2 < 0) fmin = min(fmin, limit - slack2);
  const uint64_t cs = s + ((uint64_t)t << (4 * b)) - ((uint64_t)t << (4 * n));
  const uint32_t cm = (uint32_t)n | ((uint32_t)(3 - M.a) << 4) | ((uint32_t)slack2 << 8);
  const uint64_t km = __ballot(keep);
  const int off = __builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
  if (keep) {
    const int p = (base + off) & (CAP - 1);
    st[p] = cs;
    sm[p] = (uint16_t)cm;
  }
  WAVE_SYNC();
  return base + __popcll(km);
}

// One round with one popped node per lane (kp = min(64, top - bot) nodes):
// each lane tries the four moves in turn with the move's constants known at
// compile time, so a node is decoded once and the successor is one shifted
// add.  Sliding tile t from cell n into the blank's cell b changes the packed
// state by t * (16^b - 16^n): for U (n = b - 4) that is +(65535 t) << 4n, for
// L (n = b - 1) +(15 t) << 4n, for R (n = b + 1) -(15 t) << 4b and for D
// (n = b + 4) -(65535 t) << 4b.  The Manhattan delta reads the move's 16-bit
// table slice at (coordinate of t's goal) * 4 + (coordinate of n); the
// neighbour's coordinate is b's plus a constant step, folded into a shifted
// copy of the slice.  Children are pushed move by move with a ballot + mbcnt
// prefix.  The caller guarantees top - bot + 3*kp <= CAP (at most four
// children per node, one of which reuses the popped slot).
template <int CAP, int A>
__device__ __forceinline__ void bp_move(uint64_t* st, uint16_t* sm, int& out, const uint64_t s,
                                        uint32_t b, uint32_t b4, uint32_t rb, uint32_t cb,
                                        uint32_t lm, int slack, uint32_t& anyup) {
  constexpr int delta = A == 0 ? -4 : A == 1 ? -1 : A == 2 ? 1 : 4;
  constexpr bool vert = A == 0 || A == 3;
  constexpr int step = (A == 0 || A == 1) ? -1 : 1;  // coordinate of n minus that of b
  constexpr uint32_t tab = (uint32_t)(kDhTable4 >> (16 * A)) & 0xFFFFu;
  constexpr uint32_t tab2 = step < 0 ? (tab << 1) : (tab >> 1);
  constexpr uint32_t K = vert ? 65535u : 15u;
  const uint32_t sh_n = (b4 + (uint32_t)(4 * delta)) & 63u;  // 4n (garbage if illegal)
  const uint32_t t = (uint32_t)(s >> sh_n) & 15u;
  const uint32_t ct = vert ? (t >> 2) : (t & 3u);
  const uint32_t up = (tab2 >> ((ct << 2) + (vert ? rb : cb))) & 1u;
  const int slack2 = slack - (int)(up << 1);
  const uint32_t legal = (lm >> A) & 1u;
  anyup |= legal & up;
  const bool keep = legal != 0u && slack2 >= 0;
  const uint64_t d = (uint64_t)(K * t) << (A < 2 ? sh_n : b4);  // K * t < 2^20
  const uint64_t cs = A < 2 ? s + d : s - d;
  // n | (3 - A) << 4 | slack2 << 8, with n = b + delta on a legal move
  const uint32_t cm = ((uint32_t)slack2 << 8) + b + (uint32_t)(delta + ((3 - A) << 4));
  const uint64_t km = __builtin_amdgcn_ballot_w64(keep);
  if (keep) {
    const uint32_t off = __builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
    // byte offset of slot (out + off) mod CAP in the u64 array; the u16 meta
    // array is indexed by the same slot
    const uint32_t p8 = (((uint32_t)out << 3) + (off << 3)) & (uint32_t)(8 * CAP - 1);
    *(uint64_t*)((char*)st + p8) = cs;
    *(uint16_t*)((char*)sm + (p8 >> 2)) = (uint16_t)cm;
  }
  out += __popcll(km);
}

// `smax` tracks, per lane, the largest slack of a pruned child.  A child is
// pruned only when its tile moves away from its goal (slack - 2 < 0), so a
// node's pruned children all have slack - 2.
template <int CAP>
__device__ __forceinline__ int bp_round64(uint64_t* st, uint16_t* sm, int top, int kp,
                                          int& goals, int& smax) {
  const int lane = threadIdx.x;
  const int base = top - kp;
  const int idx = (base + lane) & (CAP - 1);
  const uint64_t s = st[idx];
  const uint32_t m = sm[idx];
  const bool act = lane < kp;
  goals += __popcll(__builtin_amdgcn_ballot_w64(act && s == kGoal4));
  const uint32_t b = m & 15u;
  const uint32_t fb = (m >> 4) & 7u;
  const int slack = (int)(m >> 8);
  // legal moves of the blank at b, without the one undoing the parent move
  // (fb = 4, no parent, clears nothing inside the 4-bit mask)
  const uint32_t lm = act ? ((uint32_t)(kMoveMask4 >> (4 * b)) & 15u) & ~(1u << fb) : 0u;
  const uint32_t b4 = b << 2, rb = b >> 2, cb = b & 3u;
  uint32_t anyup = 0;
  int out = base;
  bp_move<CAP, 0>(st, sm, out, s, b, b4, rb, cb, lm, slack, anyup);
  bp_move<CAP, 1>(st, sm, out, s, b, b4, rb, cb, lm, slack, anyup);
  bp_move<CAP, 2>(st, sm, out, s, b, b4, rb, cb, lm, slack, anyup);
  bp_move<CAP, 3>(st, sm, out, s, b, b4, rb, cb, lm, slack, anyup);
  if (anyup != 0u && slack < 2) smax = max(smax, slack - 2);
  WAVE_SYNC();
  return out;
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
