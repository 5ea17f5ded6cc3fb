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

  // Index parts of the blank's cell b used by up(): for width 4 the row and
  // 4 * column, else the row and the column.
  static constexpr __host__ __device__ uint32_t row_part(uint32_t b) { return W == 4 ? b >> 2 : b / W; }
  static constexpr __host__ __device__ uint32_t col_part(uint32_t b) {
    return W == 4 ? (b & 3u) << 2 : b % W;
  }

  // 1 iff move a takes the tile it slides away from the tile's goal cell.
  // x holds the tile (its number t) in its low BITS bits; higher bits are
  // ignored.  The tile sits at the blank's neighbour and only one of its
  // coordinates changes; the table bit for (goal coordinate, neighbour
  // coordinate) is read with the neighbour's coordinate taken as the
  // blank's + step, i.e. from a shifted table.  For width 4, ct * 4 = t & 12
  // (rows) and, on a transposed table, the index is 4 * cb | ct with
  // ct = t & 3 (columns): one AND-OR per move.
  template <int A>
  static constexpr __host__ __device__ uint32_t up(uint32_t x, uint32_t rowp, uint32_t colp) {
    constexpr bool vert = A == 0 || A == 3;
    constexpr int step = (A == 0 || A == 1) ? -1 : 1;  // neighbour coordinate minus blank's
    constexpr uint32_t tab = table(A);
    if constexpr (W == 4) {
      if constexpr (vert) {
        constexpr uint32_t t2 = step < 0 ? (tab << 1) : (tab >> 1);
        return (t2 >> ((x & 12u) | rowp)) & 1u;
      } else {
        constexpr uint32_t tt = transposed(tab);
        constexpr uint32_t t2 = step < 0 ? (tt << 4) : (tt >> 4);
        return (t2 >> ((x & 3u) | colp)) & 1u;
      }
    } else {
      constexpr uint32_t t2 = step < 0 ? (tab << 1) : (tab >> 1);
      const uint32_t t = x & MASK;
      const uint32_t ct = vert ? t / W : t % W;
      return (t2 >> ((ct * W + (vert ? rowp : colp)) & 31u)) & 1u;
    }
  }

  // table(a) with its two coordinates swapped: bit (cn * W + ct).
  static constexpr uint32_t transposed(uint32_t tab) {
    uint32_t t = 0;
    for (int ct = 0; ct < W; ++ct)
      for (int cn = 0; cn < W; ++cn)
        if ((tab >> (ct * W + cn)) & 1u) t |= 1u << (cn * W + ct);
    return t;
  }

  // Bit a set iff move a keeps a blank at cell b on the board.
  static __device__ __forceinline__ uint32_t legal(uint32_t b) {
    const uint32_t r = b / W, c = b - r * W;
    return (r > 0 ? 1u : 0u) | (c > 0 ? 2u : 0u) | (c < W - 1 ? 4u : 0u) | (r < W - 1 ? 8u : 0u);
  }
};

// Legal moves per blank cell, 4 bits per cell (bit a: move a keeps the
// blank on the board), for boards of at most 16 cells.
template <int W>
constexpr uint64_t legal_table() {
  uint64_t t = 0;
  for (int p = 0; p < W * W && p < 16; ++p) {
    const int r = p / W, c = p % W;
    const uint64_t m = (r > 0 ? 1u : 0u) | (c > 0 ? 2u : 0u) | (c < W - 1 ? 4u : 0u) |
                       (r < W - 1 ? 8u : 0u);
    t |= m << (4 * p);
  }
  return t;
}

// Compile-time proof of the lookups against their definitions: for every
// blank cell, tile and legal move, up() equals "the tile's Manhattan
// distance to its goal cell grows", and legal_table equals the board edges.
template <int W>
constexpr bool check_lookups() {
  using B = Board<W>;
  for (int b = 0; b < W * W; ++b) {
    const int r = b / W, c = b % W;
    const bool lg[4] = {r > 0, c > 0, c < W - 1, r < W - 1};
    const int dn[4] = {-W, -1, 1, W};
    if (W * W <= 16) {
      uint32_t m = 0;
      for (int a = 0; a < 4; ++a) m |= lg[a] ? 1u << a : 0u;
      if (((legal_table<W>() >> (4 * b)) & 15u) != m) return false;
    }
    for (int a = 0; a < 4; ++a) {
      if (!lg[a]) continue;
      const int n = b + dn[a];
      for (int t = 1; t < W * W; ++t) {
        const int gr = t / W, gc = t % W;
        const int before = (gr > n / W ? gr - n / W : n / W - gr) + (gc > n % W ? gc - n % W : n % W - gc);
        const int after = (gr > r ? gr - r : r - gr) + (gc > c ? gc - c : c - gc);
        const uint32_t want = after > before ? 1u : 0u;
        // garbage above the tile's bits must not matter
        const uint32_t x = (uint32_t)t | (0xABCD00u << B::BITS);
        uint32_t got = 0;
        const uint32_t rp = B::row_part((uint32_t)b), cp = B::col_part((uint32_t)b);
        if (a == 0) got = B::template up<0>(x, rp, cp);
        if (a == 1) got = B::template up<1>(x, rp, cp);
        if (a == 2) got = B::template up<2>(x, rp, cp);
        if (a == 3) got = B::template up<3>(x, rp, cp);
        if (got != want) return false;
      }
    }
  }
  return true;
}
static_assert(check_lookups<3>() && check_lookups<4>() && check_lookups<5>(),
              "move tables disagree with the board");

// 24-bit unsigned product kept in 32 bits (the operands are a tile number and
// a constant below 2^20), so the compiler does not widen it to 64 bits.
__device__ __forceinline__ uint32_t mul_u24(uint32_t k, uint32_t t) {
  uint32_t r;
  asm("v_mul_u32_u24 %0, %1, %2" : "=v"(r) : "v"(k), "v"(t));
  return r;
}

// 24-bit signed product (k = -K for a constant K below 2^24, t a tile).
__device__ __forceinline__ uint32_t mul_i24(int k, uint32_t t) {
  uint32_t r;
  asm("v_mul_i32_i24 %0, %1, %2" : "=v"(r) : "v"(k), "v"(t));
  return r;
}

// a * b + c on 24-bit signed a, b (one instruction; the compiler would
// otherwise shift and subtract).
__device__ __forceinline__ uint32_t mad_i24(uint32_t a, int b, uint32_t c) {
  uint32_t r;
  asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
  return r;
}

// v where the lane's bit of the wave mask lm is set, else 0: the mask is read
// from scalar registers, with no per-lane compare.
__device__ __forceinline__ uint32_t sel_lanes(uint64_t lm, uint32_t v) {
  // the mask is wave-uniform; readfirstlane tells the compiler so (and
  // folds away when it already knows)
  const uint64_t m = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(lm >> 32)) << 32) |
                     (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)lm);
  uint32_t r;
  asm("v_cndmask_b32 %0, 0, %1, %2" : "=v"(r) : "v"(v), "s"(m));
  return r;
}

// Hides a value's known bits from the optimiser (no instruction is emitted).
// Used where the compiler would otherwise re-derive one condition in two
// forms, or keep a shift-amount mask the hardware applies anyway.
__device__ __forceinline__ uint32_t opaque(uint32_t v) {
  asm("" : "+v"(v));
  return v;
}

// The same for a 64-bit value; also a way to keep a constant in vector
// registers (as the operand of a 64-bit compare or shift it would be
// reloaded into scalar registers every round).
__device__ __forceinline__ uint64_t opaque64(uint64_t v) {
  asm("" : "+v"(v));
  return v;
}

// Hides a wave-uniform 32-bit constant from the optimiser and keeps it in a
// scalar register (the operand of a class test below would otherwise be
// folded into a mask-and-compare pair).
__device__ __forceinline__ uint32_t opaque_s(uint32_t v) {
  asm("" : "+s"(v));
  return v;
}

// ---------------------------------------------------------------------------
// The width-4 64-node round.
//
// Its stack meta word is laid out for the round: slack / 2 in bits 0..5,
// bits 6..7 zero, the blank cell in bits 8..11 and the forbidden move as a
// one-hot mask in bits 12..15 (0: none).  m >> 6 then holds 4 x blank in
// its low six bits (all that a 64-bit shift reads), byte 0 is slack / 2
// and byte 1 the blank plus the mask, and a child's slack / 2 is its
// parent's minus a borrow.  Slack / 2 fits six bits: f never falls below h0 along a
// path (Manhattan distance is consistent) and a limit is at most h0 + 126
// (64 limits).  Queue chunks and split-tree roots carry the common layout
// (blank | forbidden << 5 | slack << 8); meta4_in and meta4_out convert at
// the stack's edges.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr uint32_t meta4_in(uint32_t m) {
  const uint32_t fb = (m >> 5) & 7u;
  return ((m >> 9) & 63u) | ((m & 15u) << 8) | ((fb < 4u ? 1u << fb : 0u) << 12);
}
__host__ __device__ constexpr uint32_t meta4_out(uint32_t m) {
  const uint32_t f = (m >> 12) & 15u;
  const uint32_t fb = f == 0u ? 4u : f == 1u ? 0u : f == 2u ? 1u : f == 4u ? 2u : 3u;
  return ((m >> 8) & 15u) | (fb << 5) | ((m & 63u) << 9);
}
constexpr bool check_meta4() {
  for (uint32_t b = 0; b < 16; ++b)
    for (uint32_t f = 0; f <= 4; ++f)
      for (uint32_t s = 0; s <= 126; s += 2) {
        const uint32_t m = b | (f << 5) | (s << 8);
        const uint32_t k = meta4_in(m);
        if (meta4_out(k) != m || (k & 63u) != s / 2 || ((k >> 6) & 63u) != 4 * b ||
            ((k >> 12) & 15u) != (f < 4u ? 1u << f : 0u) || k > 0xFFFFu)
          return false;
      }
  return true;
}
static_assert(check_meta4(), "width-4 stack meta does not round-trip");

// Width-4 stacks of 64-node rounds come in two layouts.  Split (most sizes):
// CAP 8-byte states, then CAP 2-byte meta words, 10 bytes an entry.
// Interleaved (672 entries): entry i holds its state at bytes
// 12i .. 12i + 7 (two dwords) and its meta word at 12i + 8, so that one
// address serves both (one instruction less per child and per node, 20 %
// more LDS per entry, i.e. fewer waves per compute unit at a given size).
// st is the stack's base.
template <int CAP>
constexpr bool stack4_interleaved() {
  return CAP == 672;
}
template <int CAP>
constexpr uint32_t stack4_bytes() {
  return (stack4_interleaved<CAP>() ? 12u : 10u) * (uint32_t)CAP;
}
constexpr uint32_t kEntry4 = 12;
template <int CAP>
__device__ __forceinline__ uint64_t e4_tile(const uint64_t* st, uint32_t i) {
  if constexpr (stack4_interleaved<CAP>()) {
    const uint32_t* p = (const uint32_t*)((const char*)st + kEntry4 * i);
    return (uint64_t)p[0] | ((uint64_t)p[1] << 32);
  } else {
    return st[i];
  }
}
template <int CAP>
__device__ __forceinline__ uint32_t e4_meta(const uint64_t* st, uint32_t i) {
  if constexpr (stack4_interleaved<CAP>()) return *(const uint16_t*)((const char*)st + kEntry4 * i + 8);
  else return ((const uint16_t*)(st + CAP))[i];
}
template <int CAP>
__device__ __forceinline__ void e4_put(uint64_t* st, uint32_t i, uint64_t t, uint32_t m) {
  if constexpr (stack4_interleaved<CAP>()) {
    uint32_t* p = (uint32_t*)((char*)st + kEntry4 * i);
    p[0] = (uint32_t)t;
    p[1] = (uint32_t)(t >> 32);
    *(uint16_t*)(p + 2) = (uint16_t)m;
  } else {
    st[i] = t;
    ((uint16_t*)(st + CAP))[i] = (uint16_t)m;
  }
}

// Moves width-4 stack entries [src, src + n) down to [dst, dst + n), dst <
// src, 64 at a time in ascending order: every entry is read before anything
// is written over it.
template <int CAP>
__device__ __forceinline__ void move_down4(uint64_t* st, uint32_t dst, uint32_t src, uint32_t n) {
  const uint32_t lane = (uint32_t)lane_id();
  for (uint32_t i = 0; i < n; i += 64u) {
    const uint32_t k = i + lane;
    if (k < n) {
      const uint64_t t = e4_tile<CAP>(st, src + k);
      const uint32_t m = e4_meta<CAP>(st, src + k);
      e4_put<CAP>(st, dst + k, t, m);
    }
  }
  WAVE_SYNC();
}

// r * 12 + c in one instruction (r below 2^24).
__device__ __forceinline__ uint32_t mad12(uint32_t r, uint32_t c) {
  uint32_t d;
  asm("v_mad_u32_u24 %0, %1, 12, %2" : "=v"(d) : "v"(r), "s"(c));
  return d;
}

// Move A of the width-4 round takes tile t away from its goal cell (tile t's
// goal cell is t): the coordinate that changes is the row for U and D, the
// column for L and R, and the tile moves away when its goal coordinate lies
// behind the neighbour's, seen from the blank.  With the blank's row part
// b & 12, b | 3 and its column b & 3 these are single compares:
//   U: t >> 2 < row(b)      <=> t < (b & 12)
//   D: t >> 2 > row(b)      <=> t > (b | 3)
//   L: t & 3  < col(b),   R: t & 3 > col(b).
template <int A>
__host__ __device__ constexpr bool up4(uint32_t t, uint32_t b) {
  return A == 0 ? t < (b & 12u) : A == 1 ? (t & 3u) < (b & 3u) : A == 2 ? (t & 3u) > (b & 3u) : t > (b | 3u);
}
template <int A>
constexpr bool check_up4() {
  using B = Board<4>;
  for (uint32_t b = 0; b < 16; ++b) {
    if (((legal_table<4>() >> (4 * b + A)) & 1u) == 0) continue;  // (any value serves)
    for (uint32_t t = 1; t < 16; ++t)
      if (up4<A>(t, b) != (B::template up<A>(t, B::row_part(b), B::col_part(b)) != 0)) return false;
  }
  return true;
}
static_assert(check_up4<0>() && check_up4<1>() && check_up4<2>() && check_up4<3>(),
              "width-4 compares disagree with Board::up");

// Constants of the width-4 round, set once per unit: the goal and the
// legal-move table in vector registers (as operands of a 64-bit compare or
// shift they would be reloaded into scalar registers every round), and one
// float per move whose IEEE class is bit A of a class test's mask (signaling
// NaN, quiet NaN, -infinity, -normal), so that a class test against a node's
// 4-bit move mask says whether move A is in it.
struct RoundConsts4 {
  uint64_t goal;
  uint64_t legal;
  uint32_t cls[4];
  uint32_t nk[4];  // per move, minus its child's meta increment (vector registers)
};

// Move A's child meta increment: blank + delta, forbidden move 3 - A.
template <int A>
constexpr int meta4_step() {
  return (A == 0 ? -4 : A == 1 ? -1 : A == 2 ? 1 : 4) * 256 + (4096 << (3 - A));
}

__device__ __forceinline__ RoundConsts4 make_round_consts4() {
  RoundConsts4 k;
  k.goal = opaque64(Board<4>::goal());
  k.legal = opaque64(legal_table<4>());
  k.cls[0] = opaque_s(0x7F800001u);  // signaling NaN: class bit 0
  k.cls[1] = opaque_s(0x7FC00000u);  // quiet NaN: class bit 1
  k.cls[2] = opaque_s(0xFF800000u);  // -infinity: class bit 2
  k.cls[3] = opaque_s(0xBF800000u);  // -1.0, a negative normal: class bit 3
  k.nk[0] = opaque((uint32_t)-meta4_step<0>());
  k.nk[1] = opaque((uint32_t)-meta4_step<1>());
  k.nk[2] = opaque((uint32_t)-meta4_step<2>());
  k.nk[3] = opaque((uint32_t)-meta4_step<3>());
  return k;
}

// Byte address of an LDS object (its offset in the workgroup's LDS).
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

// Lanes whose mask lm holds the IEEE class of the float with bits c (one
// compare into a scalar register pair; written out because the compiler
// turns the ballot of a class test into a select and a second compare).
__device__ __forceinline__ uint64_t class_lanes(uint32_t c, uint32_t lm) {
  uint64_t r;
  asm("v_cmp_class_f32_e64 %0, %1, %2" : "=s"(r) : "s"(c), "v"(lm));
  return r;
}

// Lanes whose byte 0 of v is nonzero (one compare with a byte select).
__device__ __forceinline__ uint64_t byte0_lanes(uint32_t v) {
  uint64_t r;
  asm("v_cmp_ne_u32_sdwa %0, %1, 0 src0_sel:BYTE_0 src1_sel:DWORD" : "=s"(r) : "v"(v));
  return r;
}

// K AND byte 1 of v (one instruction with a byte select).
template <int K>
__device__ __forceinline__ uint32_t and_byte1(uint32_t v) {
  uint32_t r;
  asm("v_and_b32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1"
      : "=v"(r)
      : "i"(K), "v"(v));
  return r;
}

// The up compare, keep mask and child meta of one width-4 move, with the
// compare's lane mask in VCC: up = x < y (LT) or x > y; keep = legal and
// not (up and not roomy); meta = base - nk - up, one subtract with the
// borrow taken from VCC (nk: the move's meta increment, negated, in a vector
// register; the borrow-in already uses the one scalar operand the
// instruction may read, so the constant cannot be a literal).
template <bool LT>
__device__ __forceinline__ void keep_meta(uint32_t x, uint32_t y, uint64_t legal, uint64_t roomy,
                                          uint32_t base, uint32_t nk, uint64_t& keep, uint32_t& meta) {
  uint64_t away_short;
  if constexpr (LT) {
    asm("v_cmp_lt_u32_e32 vcc, %[x], %[y]\n\t"
        "s_andn2_b64 %[t], vcc, %[r]\n\t"
        "s_andn2_b64 %[k], %[l], %[t]\n\t"
        "v_subb_co_u32_e32 %[m], vcc, %[b], %[nk], vcc"
        : [k] "=&s"(keep), [m] "=v"(meta), [t] "=&s"(away_short)
        : [x] "v"(x), [y] "v"(y), [l] "s"(legal), [r] "s"(roomy), [b] "v"(base), [nk] "v"(nk)
        : "vcc", "scc");
  } else {
    asm("v_cmp_gt_u32_e32 vcc, %[x], %[y]\n\t"
        "s_andn2_b64 %[t], vcc, %[r]\n\t"
        "s_andn2_b64 %[k], %[l], %[t]\n\t"
        "v_subb_co_u32_e32 %[m], vcc, %[b], %[nk], vcc"
        : [k] "=&s"(keep), [m] "=v"(meta), [t] "=&s"(away_short)
        : [x] "v"(x), [y] "v"(y), [l] "s"(legal), [r] "s"(roomy), [b] "v"(base), [nk] "v"(nk)
        : "vcc", "scc");
  }
}

// Per-node values of the width-4 round shared by its four moves.
struct Node4 {
  uint32_t shb;    // 4 x blank in the low six bits (higher bits are ignored)
  uint32_t sr_lo;  // low word of s >> 4b: the cells after the blank
  uint32_t su_hi;  // high word of s << (63 - 4b): the cells before it
  uint32_t lm;     // bit A (A < 4): move A is legal and does not undo the parent's
  uint32_t b12;    // blank & 12, blank | 3, blank & 3: the up compares' bounds
  uint32_t b3;
  uint32_t bc;
  uint32_t mbase;  // the meta word without its forbidden-move mask
  uint64_t roomy;  // lanes with slack >= 2 (a child may move a tile away)
};

// One move of the width-4 round for every lane (see bp_round64_4).
template <int CAP, int A>
__device__ __forceinline__ void bp_move4(uint64_t* st, uint32_t& out, const uint64_t s, const Node4& c,
                                         const RoundConsts4& rk) {
  constexpr int delta = A == 0 ? -4 : A == 1 ? -1 : A == 2 ? 1 : 4;
  constexpr uint32_t K = (A == 0 || A == 3) ? 0xFFFFu : 15u;
  // cell b + d sits at bits 4d of s >> 4b (d > 0), and at bits 63 + 4d - 32
  // of the high word of s << (63 - 4b) (d < 0): one extract gives the tile
  uint32_t x;
  if constexpr (A == 0) x = (c.su_hi >> 15) & 15u;
  else if constexpr (A == 1) x = (c.su_hi >> 27) & 15u;
  else if constexpr (A == 2) x = (c.sr_lo >> 4) & 15u;
  else x = (c.sr_lo >> 16) & 15u;
  const uint32_t t = opaque(x);
  // the move takes t away from its goal cell (up4): U t < b & 12, L
  // (t & 3) < b & 3, R (t & 3) > b & 3, D t > b | 3
  const uint32_t ux = (A == 1 || A == 2) ? (t & 3u) : t;
  const uint32_t uy = A == 0 ? c.b12 : A == 3 ? c.b3 : c.bc;
  // legal and not undoing: one class test of move A's constant against lm
  const uint64_t lg = class_lanes(rk.cls[A], c.lm);
  // kept: legal, and approaching its goal or with slack to spare (an away
  // move costs 2 of slack; slack is even, so 0 prunes it); child meta:
  // slack / 2 minus up (a borrow), blank n, forbidden 3 - A
  uint64_t km;
  uint32_t cm;
  keep_meta<(A == 0 || A == 1)>(ux, uy, lg, c.roomy, c.mbase, rk.nk[A], km, cm);
  // successor: t moves from n = b + delta to b, i.e. the packed word changes
  // by +/- (K * t) << (4 * min(b, n))
  uint64_t cs;
  if constexpr (A >= 2) {
    // the subtraction as the addition of -K t sign-extended to 64 bits
    const uint32_t nkt = mul_i24(-(int)K, t);
    cs = s + (((0xFFFFFFFFull << 32) | nkt) << (c.shb & 63u));
  } else {
    const uint32_t kt = mul_u24(K, t);
    cs = s + ((uint64_t)kt << ((c.shb + (uint32_t)(4 * delta)) & 63u));
  }
  const uint32_t r =
      __builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
  // entry out + r (below CAP: the caller leaves room for the largest round).
  // The stores run under the keep mask with no branch around them; the
  // compiler would put a skip jump around stores in a divergent branch, so
  // the asm sets EXEC to the mask, stores and restores EXEC itself.
  uint64_t saved;
  if constexpr (stack4_interleaved<CAP>()) {
    const uint32_t as = lds_addr(st) + mad12(r, out * kEntry4);
    asm volatile(
        "s_and_saveexec_b64 %0, %1\n\t"
        "ds_write2_b32 %2, %3, %4 offset1:1\n\t"
        "ds_write_b16 %2, %5 offset:8\n\t"
        "s_mov_b64 exec, %0"
        : "=&s"(saved)
        : "s"(km), "v"(as), "v"((uint32_t)cs), "v"((uint32_t)(cs >> 32)), "v"(cm)
        : "memory", "scc");
  } else {
    // (the meta array follows the CAP states)
    const uint32_t pst = (r + out) << 3;
    const uint32_t as = lds_addr(st) + pst;
    const uint32_t am = lds_addr(st) + (pst >> 2);
    asm volatile(
        "s_and_saveexec_b64 %0, %1\n\t"
        "ds_write_b64 %2, %3\n\t"
        "ds_write_b16 %4, %5 offset:%6\n\t"
        "s_mov_b64 exec, %0"
        : "=&s"(saved)
        : "s"(km), "v"(as), "v"(cs), "v"(am), "v"(cm), "i"(CAP * 8)
        : "memory", "scc");
  }
  out += (uint32_t)__popcll(km);
}

// One BPDFS round of the width-4 board with one popped node per lane: pops
// kp = min(64, top) nodes from a stack of entries [0, top) (either layout
// above, meta words in the width-4 layout), tests them for the goal and pushes
// every legal, non-undoing child with f <= limit.  The caller guarantees
// that the children fit, top + 2*kp <= CAP; FULL: kp = 64 and `goals` is a
// 64-bit mask that collects the lanes that expanded a goal, else a count.
// Pruned children are not tracked: every slack on the stack is even (f
// keeps the parity of h0, and so does the limit), so a child is pruned only
// from slack 0, moving a tile away from its goal, and its f is the limit + 2.
template <int CAP, bool FULL, typename G>
__device__ __forceinline__ uint32_t bp_round64_4(uint64_t* st, uint32_t top, int kp, G& goals,
                                                 const RoundConsts4& rk) {
  const int lane = lane_id();
  const uint32_t base = top - (uint32_t)kp;
  uint64_t s;
  uint32_t m;
  if constexpr (stack4_interleaved<CAP>()) {
    const uint32_t pe = opaque(mad12((uint32_t)lane, base * kEntry4));
    const uint32_t* pp = (const uint32_t*)((const char*)st + pe);
    s = (uint64_t)pp[0] | ((uint64_t)pp[1] << 32);
    m = *(const uint16_t*)(pp + 2);
  } else {
    const uint32_t pst = opaque((base + (uint32_t)lane) << 3);
    s = *(const uint64_t*)((const char*)st + pst);
    m = *(const uint16_t*)((const char*)(st + CAP) + (pst >> 2));
  }
  const uint64_t actm = FULL || kp >= 64 ? ~0ull : ((1ull << kp) - 1ull);
  const uint64_t gm = __builtin_amdgcn_uicmpl(s, rk.goal, 32);
  if constexpr (FULL) goals |= gm;
  else goals += __popcll(gm & actm);
  Node4 c;
  c.shb = opaque(m >> 6);
  c.sr_lo = (uint32_t)(s >> (c.shb & 63u));
  c.su_hi = (uint32_t)((s << (~c.shb & 63u)) >> 32);
  // legal moves minus the forbidden one; bits above 3 (the next cells'
  // legal moves) are left in: the class tests read only bits 0..3
  const uint32_t lm = (uint32_t)(rk.legal >> (c.shb & 63u)) & ~(m >> 12);
  // lanes past kp keep nothing
  c.lm = FULL ? lm : sel_lanes(actm, lm);
  c.roomy = byte0_lanes(m);  // slack / 2 != 0
  c.b12 = and_byte1<12>(m);  // byte 1 = blank | mask << 4
  c.b3 = c.b12 | 3u;
  c.bc = and_byte1<3>(m);
  c.mbase = m & 0x0FFFu;
  uint32_t out = base;
  bp_move4<CAP, 0>(st, out, s, c, rk);
  bp_move4<CAP, 1>(st, out, s, c, rk);
  bp_move4<CAP, 2>(st, out, s, c, rk);
  bp_move4<CAP, 3>(st, out, s, c, rk);
  WAVE_SYNC();
  return out;
}

// Per-node values shared by the four moves of a 64-node round (widths 3
// and 5).
struct NodeCtx {
  uint32_t b;      // blank cell
  uint32_t shb;    // BITS * b
  uint32_t rowi;   // vertical moves: the blank's row (table index part)
  uint32_t coli;   // horizontal moves: the blank's column
  uint32_t lmx;    // bit (A + 4 up): move A survives the f test
  uint32_t mbase;  // slack << 8 | blank
};

// One move for every lane of a 64-node round (see bp_round64w).
template <int W, int CAP, int A, bool MASKED>
__device__ __forceinline__ void bp_move_w(typename Board<W>::S* st, uint16_t* sm, uint32_t& out,
                                          const typename Board<W>::S s, const NodeCtx& c) {
  using B = Board<W>;
  using S = typename B::S;
  constexpr int delta = A == 0 ? -W : A == 1 ? -1 : A == 2 ? 1 : W;
  constexpr bool vert = A == 0 || A == 3;
  constexpr uint32_t K = vert ? ((1u << (B::BITS * W)) - 1u) : B::MASK;
  // shift to the neighbour's cell; it wraps (and the tile is unused) when
  // the move is illegal, and needs no mask on a legal one
  const uint32_t shu = c.shb + (uint32_t)(B::BITS * delta);
  const uint32_t x = (uint32_t)(s >> (shu & (8u * sizeof(S) - 1u)));
  const uint32_t tile = x & B::MASK;  // the neighbour's tile t
  const uint32_t up = B::template up<A>(x, c.rowi, c.coli);  // 1: t moves away from its goal cell
  const uint32_t kb = opaque((c.lmx >> (A + 4 * up)) & 1u);
  const uint64_t km = __builtin_amdgcn_uicmp(kb, 0u, 33);  // lanes with kb != 0
  // MASKED (64-bit states): every lane builds its child (a vector
  // instruction costs the same for any number of active lanes) and only the
  // lanes that keep it store, under the mask; no branch.  Otherwise (5x5)
  // the child is built in a branch that the compiler skips when no lane
  // keeps the move.
  if (MASKED || kb != 0u) {
    // successor: t moves from n to b, i.e. the packed word changes by
    // t * (base^b - base^n) = +/- (K * t) << (BITS * min(b, n))
    S cs;
    if constexpr (A >= 2 && sizeof(S) == 8) {
      // the subtraction as the addition of -K t sign-extended to 64 bits:
      // one 64-bit add instead of a subtract with borrow
      const uint32_t nkt = mul_i24(-(int)K, tile);
      cs = s + (((0xFFFFFFFFull << 32) | nkt) << (c.shb & 63u));
    } else {
      uint32_t kt;
      if constexpr (K < (1u << 24)) kt = mul_u24(K, tile);
      else kt = K * tile;  // 5x5 rows: K = 2^25 - 1
      const S d = (S)kt << ((A < 2 ? shu : c.shb) & (8u * sizeof(S) - 1u));
      cs = A < 2 ? s + d : s - d;
    }
    // stack meta: n | (3 - A) << 5 | (slack - 2 up) << 8
    const uint32_t cm = mad_i24(up, -512, c.mbase) + (uint32_t)(delta + ((3 - A) << 5));
    const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
    // byte offsets into the stack: entry out + r (below CAP: the caller
    // leaves room for the largest round)
    constexpr uint32_t LS = sizeof(S) == 8 ? 3 : 4;
    const uint32_t pst = (r + out) << LS;
    if constexpr (MASKED) {
      // the two stores under the keep mask, with no branch around them (the
      // meta array follows the CAP tiles: sm == st + CAP).  The compiler
      // would put a skip jump around stores in a divergent branch; this asm
      // sets EXEC to the mask, stores and restores EXEC itself.
      const uint32_t as = lds_addr(st) + pst;
      const uint32_t am = lds_addr(st) + (pst >> (LS - 1));
      uint64_t saved;
      asm volatile(
          "s_and_saveexec_b64 %0, %1\n\t"
          "ds_write_b64 %2, %3\n\t"
          "ds_write_b16 %4, %5 offset:%6\n\t"
          "s_mov_b64 exec, %0"
          : "=&s"(saved)
          : "s"(km), "v"(as), "v"(cs), "v"(am), "v"(cm), "i"(CAP * (int)sizeof(S))
          : "memory", "scc");
    } else {
      *(S*)((char*)st + pst) = cs;
      *(uint16_t*)((char*)sm + (pst >> (LS - 1))) = (uint16_t)cm;
    }
  }
  out += (uint32_t)__popcll(km);
}

// One BPDFS round with one popped node per lane, for boards of width 3 and
// 5 (width 4 has its own round above, with its own stack meta layout): pops
// kp = min(64, top) nodes from a stack of entries [0, top), tests them for
// the goal and pushes every legal, non-undoing child with f <= limit.  The
// caller guarantees that the children fit, top + 2*kp <= CAP (three
// children a node at most; only a root, expanded in a unit's first round
// from at most 64 entries, can have four; no position wraps); FULL: it also
// guarantees kp = 64, so no lane is idle, and passes a 64-bit mask that
// collects the lanes that expanded a goal.  The round does not track the f
// of pruned children: every slack on the stack is even (f keeps the parity
// of h0, and so does the limit), so a child is pruned only from slack 0,
// moving a tile away from its goal, and its f is the limit + 2.
template <int W, int CAP, bool MASKED, bool FULL, typename G>
__device__ __forceinline__ uint32_t bp_round64w(typename Board<W>::S* st, uint16_t* sm, uint32_t top, int kp,
                                           G& goals, const RoundConsts4& rk) {
  if constexpr (W == 4) {
    return bp_round64_4<CAP, FULL>(st, top, kp, goals, rk);
  } else {
    using B = Board<W>;
    using S = typename B::S;
    const int lane = lane_id();
    const uint32_t base = top - (uint32_t)kp;
    constexpr uint32_t LS = sizeof(S) == 8 ? 3 : 4;
    const uint32_t pst = opaque((base + (uint32_t)lane) << LS);
    const S s = *(const S*)((const char*)st + pst);
    const uint32_t m = *(const uint16_t*)((const char*)sm + (pst >> (LS - 1)));
    const uint64_t actm = FULL || kp >= 64 ? ~0ull : ((1ull << kp) - 1ull);
    uint64_t gm;
    if constexpr (sizeof(S) == 8) gm = __builtin_amdgcn_uicmpl((uint64_t)s, (uint64_t)B::goal(), 32);
    else gm = __builtin_amdgcn_ballot_w64(s == B::goal());
    // goals: a count (int), or (FULL) the union of the rounds' goal masks
    if constexpr (FULL) goals |= gm;
    else goals += __popcll(gm & actm);
    NodeCtx c;
    c.b = m & 31u;
    const uint32_t fb = (m >> 5) & 7u;
    c.shb = opaque(B::BITS * c.b);
    uint32_t lm;
    if constexpr (W * W <= 16) lm = (uint32_t)(legal_table<W>() >> (4u * c.b)) & ~(1u << fb) & 15u;
    else lm = B::legal(c.b) & ~(1u << fb);
    c.coli = B::col_part(c.b);
    c.rowi = B::row_part(c.b);
    // moves that survive: any legal one if its tile approaches its goal, and
    // only with slack >= 2 if it moves away (bits 0..3 and 4..7 of lm * 17);
    // lanes past kp keep nothing
    const bool roomy = m >= (2u << 8);
    if constexpr (FULL) c.lmx = mul_u24(lm, roomy ? 17u : 1u);
    else c.lmx = mul_u24(lm, sel_lanes(actm, roomy ? 17u : 1u));
    c.mbase = (m & 0xFF00u) | c.b;
    uint32_t out = base;
    bp_move_w<W, CAP, 0, MASKED>(st, sm, out, s, c);
    bp_move_w<W, CAP, 1, MASKED>(st, sm, out, s, c);
    bp_move_w<W, CAP, 2, MASKED>(st, sm, out, s, c);
    bp_move_w<W, CAP, 3, MASKED>(st, sm, out, s, c);
    WAVE_SYNC();
    return out;
  }
}

}  // namespace bpida
