// bpida_board.h -- sliding-tile boards of width 3, 4 and 5 for the batched
// search: packed state type, goal, move legality, the Manhattan delta table
// and the one-node-per-lane round of BPDFS (Alg. 1).
//
// Packing: cell p holds its tile in bits [BITS*p, BITS*p + BITS): 4 bits per
// tile in a u64 for 3x3 and 4x4, 5 bits per tile in a 128-bit word for 5x5.
// The goal holds tile p at cell p.  Moves are blank moves U, L, R, D = 0..3
// (cell offsets -W, -1, +1, +W), inverse 3 - a.
#pragma once

#include <limits.h>
#include <stdint.h>

#include <type_traits>

#include "bpida_round.h"

namespace bpida {

template <int W>
struct Board {
  static_assert(W >= 3 && W <= 5, "width");
  static constexpr int N = W * W;
  static constexpr int BITS = W == 5 ? 5 : 4;
  using S = typename std::conditional<W == 5, unsigned __int128, uint64_t>::type;
  static constexpr uint32_t MASK = (1u << BITS) - 1u;

  static constexpr S goal() {
    S g = 0;
    for (int p = 0; p < N; ++p) g |= (S)p << (BITS * p);
    return g;
  }

  // Move a slides the tile t at the blank's neighbour n into the blank's
  // cell b.  Only one coordinate of t changes (its row for U/D, its column
  // for L/R).  Bit (ct * W + cn) of table(a) says whether that coordinate
  // moves away from the tile's goal coordinate ct, given the neighbour's
  // coordinate cn (the tile's distance then grows by one, else it shrinks).
  static constexpr uint32_t table(int a) {
    uint32_t tab = 0;
    const int step = (a == 0 || a == 1) ? 1 : -1;  // U, L move the tile +1; R, D -1
    for (int ct = 0; ct < W; ++ct)
      for (int cn = 0; cn < W; ++cn) {
        const int before = ct > cn ? ct - cn : cn - ct;
        const int ca = cn + step;
        const int after = ct > ca ? ct - ca : ca - ct;
        if (after > before) tab |= 1u << (ct * W + cn);
      }
    return tab;
  }

  // Bit a set iff move a keeps a blank at cell b on the board.
  static __device__ __forceinline__ uint32_t legal(uint32_t b) {
    const uint32_t r = b / W, c = b - r * W;
    return (r > 0 ? 1u : 0u) | (c > 0 ? 2u : 0u) | (c < W - 1 ? 4u : 0u) | (r < W - 1 ? 8u : 0u);
  }
};

// One move for every lane of a 64-node round (see bp_round64w).
template <int W, int CAP, int A>
__device__ __forceinline__ void bp_move_w(typename Board<W>::S* st, uint16_t* sm, int& out,
                                          const typename Board<W>::S s, uint32_t b, uint32_t rb,
                                          uint32_t cb, uint32_t lm, int slack, uint32_t& anyup) {
  using B = Board<W>;
  using S = typename B::S;
  constexpr int delta = A == 0 ? -W : A == 1 ? -1 : A == 2 ? 1 : W;
  constexpr bool vert = A == 0 || A == 3;
  constexpr int step = (A == 0 || A == 1) ? -1 : 1;  // neighbour coordinate minus blank's
  constexpr uint32_t tab = B::table(A);
  // index (ct * W + cb) reads bit (ct * W + cb + step) of the table
  constexpr uint32_t tab2 = step < 0 ? (tab << 1) : (tab >> 1);
  constexpr uint32_t K = vert ? ((1u << (B::BITS * W)) - 1u) : B::MASK;
  const uint32_t n = b + (uint32_t)delta;  // wraps (and is unused) when illegal
  const uint32_t sh_n = (B::BITS * n) & (8u * sizeof(S) - 1u);
  const uint32_t t = (uint32_t)(s >> sh_n) & B::MASK;
  const uint32_t ct = vert ? t / W : t % W;
  const uint32_t up = (tab2 >> ((ct * W + (vert ? rb : cb)) & 31u)) & 1u;
  const int slack2 = slack - (int)(up << 1);
  const uint32_t legal = (lm >> A) & 1u;
  anyup |= legal & up;
  const bool keep = legal != 0u && slack2 >= 0;
  // successor: t moves from n to b, i.e. the packed word changes by
  // t * (base^b - base^n) = +/- (K * t) << (BITS * min(b, n))
  const S d = (S)(K * t) << (A < 2 ? sh_n : B::BITS * b);
  const S cs = A < 2 ? s + d : s - d;
  // stack meta: n | (3 - A) << 5 | slack2 << 8 (n = b + delta on a legal move)
  const uint32_t cm = ((uint32_t)slack2 << 8) + b + (uint32_t)(delta + ((3 - A) << 5));
  const uint64_t km = __builtin_amdgcn_ballot_w64(keep);
  if (keep) {
    const uint32_t off = __builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
    const uint32_t p = ((uint32_t)out + off) & (uint32_t)(CAP - 1);
    st[p] = cs;
    sm[p] = (uint16_t)cm;
  }
  out += __popcll(km);
}

// One BPDFS round with one popped node per lane, for any board width: pops
// kp = min(64, top - bot) nodes, tests them for the goal and pushes every
// legal, non-undoing child with f <= limit.  The caller guarantees
// top - bot + 3*kp <= CAP.  `smax` tracks the largest slack of a pruned
// child (always slack - 2 of a node whose tile moves away from its goal).
template <int W, int CAP>
__device__ __forceinline__ int bp_round64w(typename Board<W>::S* st, uint16_t* sm, int top, int kp,
                                           int& goals, int& smax) {
  using B = Board<W>;
  using S = typename B::S;
  const int lane = threadIdx.x;
  const int base = top - kp;
  const int idx = (base + lane) & (CAP - 1);
  const S s = st[idx];
  const uint32_t m = sm[idx];
  const bool act = lane < kp;
  goals += __popcll(__builtin_amdgcn_ballot_w64(act && s == B::goal()));
  const uint32_t b = m & 31u;
  const uint32_t fb = (m >> 5) & 7u;
  const int slack = (int)(m >> 8);
  const uint32_t lm = act ? B::legal(b) & ~(1u << fb) : 0u;
  const uint32_t rb = b / W, cb = b - rb * W;
  uint32_t anyup = 0;
  int out = base;
  bp_move_w<W, CAP, 0>(st, sm, out, s, b, rb, cb, lm, slack, anyup);
  bp_move_w<W, CAP, 1>(st, sm, out, s, b, rb, cb, lm, slack, anyup);
  bp_move_w<W, CAP, 2>(st, sm, out, s, b, rb, cb, lm, slack, anyup);
  bp_move_w<W, CAP, 3>(st, sm, out, s, b, rb, cb, lm, slack, anyup);
  if (anyup != 0u && slack < 2) smax = max(smax, slack - 2);
  WAVE_SYNC();
  return out;
}

}  // namespace bpida
