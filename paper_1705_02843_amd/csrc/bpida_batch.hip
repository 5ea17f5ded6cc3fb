// bpida_batch.hip -- batched, persistent Block-Parallel IDA* for gfx950.
//
// One launch searches every instance of a batch through all of its f-limits.
// Work lives in a device queue of chunks (up to 64 stack entries of one
// instance at one limit).  A workgroup (one wave64) pops a chunk into its LDS
// stack and runs BPDFS rounds (Alg. 1) on it; it gives the 64 oldest entries
// of its stack back to the queue when its stack would overflow LDS, or when
// other workgroups are idle and the queue holds fewer chunks than there are
// workgroups waiting for work (donation; the paper's BPIDA* balances statically, its
// intra-block donation idea for PFullLB is applied here across workgroups).
//
// Per instance, `outstanding` counts its chunks that are queued or held by a
// workgroup at the current limit.  The workgroup whose decrement brings it to
// zero completes the limit on the device: it adds the split tree's interior
// nodes, writes the node count of the limit, stops on a goal (all optimal
// solutions: the limit has been searched to completion), and otherwise
// advances the limit by 2 and seeds the instance's subtree roots again.
#include <limits.h>

#include "bpida_board.h"
#include "bpida_internal.h"
#include "bpida_round.h"

namespace bpida {

#define AGENT __HIP_MEMORY_SCOPE_AGENT

// The split kernels' level sizes, built at compile time.
__device__ WalkTable g_walk_table = make_walk_table();

hipError_t walk_table_device(const int32_t** out) {
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_walk_table));
  *out = static_cast<const int32_t*>(p);
  return e;
}

__device__ __forceinline__ uint64_t ld_relaxed(uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, AGENT);
}
__device__ __forceinline__ int32_t ld_relaxed(int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, AGENT);
}
// The value lane 0 loads, in every lane: a branch on it is uniform (a
// per-lane load, even of one address, makes the compiler treat the branch
// as divergent).
__device__ __forceinline__ int32_t ld_wave(int32_t* p) {
  return __builtin_amdgcn_readfirstlane(ld_relaxed(p));
}

// ---------------------------------------------------------------------------
// Ticket queue of chunks.  Producers and consumers take tickets with a
// fetch-and-add on tail / head (no compare-and-swap loops on those two
// counters, which collapse under thousands of contending workgroups).  Slot
// k of the ring carries the state of ticket t = the next ticket to use it:
// 4t free for producer t, 4t + 1 claimed by producer t (being written),
// 4t + 2 holds the chunk of ticket t.  An idle wave takes one consumer ticket
// and then polls only its own slot, so waiting waves do not contend on a
// shared line; head - tail = waiting waves - queued chunks, which is what a
// busy wave reads to decide whether to donate.  Every operation is done by a
// whole wave: lane 0 handles tickets, all lanes move the 64 entries.
//
// A producer whose slot is still occupied after A.push_spin polls gives its
// ticket up and raises the slot's `abandoned` mark to at least t + 1.  A
// consumer holding ticket t whose slot is free for t while the mark is past
// t hands the slot on to ticket t + capacity with a compare-and-swap (the
// producer claims it with one too, so exactly one of them wins; a late
// producer that loses gives up as well).  A lost ticket therefore never
// strands a consumer and the ring keeps working; the lost chunk's work is
// gone, its instance is marked lost and the call reports BPIDA_ENOMEM.
// ---------------------------------------------------------------------------
constexpr uint64_t kNoTicket = ~0ull;

__device__ __forceinline__ uint64_t bcast64(uint64_t v) {
  const uint32_t lo = (uint32_t)wave_bcast((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)wave_bcast((int)(uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ bool cas64(uint64_t* p, uint64_t expect, uint64_t want) {
  return __hip_atomic_compare_exchange_strong(p, &expect, want, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                              AGENT);
}

// Returns false if the ring stayed full for the whole bounded wait (the
// entries were not queued).  `hi` is stored only for 5x5 chunks (wide), in
// the slot's row of A.hi.
__device__ bool q_push(const BatchArgs& A, uint64_t tile, uint64_t hi, uint16_t meta, int count,
                       int inst, bool wide) {
  const int lane = lane_id();
  QueueCtl* q = A.q;
  const uint64_t mask = A.qmask;
  uint64_t pos = 0;
  int ok = 0;
  if (lane == 0) {
    pos = __hip_atomic_fetch_add(&q->tail, (uint64_t)1, __ATOMIC_RELAXED, AGENT);
    const uint64_t h = ld_relaxed(&q->head);
    if (pos + 1 > h) __hip_atomic_fetch_max(&q->qmax, pos + 1 - h, __ATOMIC_RELAXED, AGENT);
    SlotCtl* sc = A.seq + (pos & mask);
    for (int k = 0; k < A.push_spin; ++k) {
      const uint64_t v = ld_relaxed(&sc->seq);
      if (v == 4 * pos) {
        ok = cas64(&sc->seq, 4 * pos, 4 * pos + 1) ? 1 : 0;
        break;
      }
      if (v > 4 * pos) break;  // handed on past this ticket by its consumer
      __builtin_amdgcn_s_sleep(1);
    }
    if (!ok) {
      __hip_atomic_fetch_max(&sc->abandoned, pos + 1, __ATOMIC_RELAXED, AGENT);
      atomicOr(&q->err, 16);  // ticket lost: the call reports BPIDA_ENOMEM
    }
  }
  ok = wave_bcast(ok);
  if (!ok) return false;
  pos = bcast64(pos);
  // the slot's previous consumer released it; order the new payload after
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  QChunk* c = A.slots + (pos & mask);
  c->tiles[lane] = tile;
  if (wide) A.hi[(pos & mask) * kQChunk + lane] = hi;
  c->meta[lane] = meta;
  if (lane == 0) {
    c->inst = inst;
    c->count = count;
    c->wide = wide ? 1 : 0;
  }
  WAVE_SYNC_MEM();  // every lane's stores precede lane 0's release
  if (lane == 0) __hip_atomic_store(&A.seq[pos & mask].seq, 4 * pos + 2, __ATOMIC_RELEASE, AGENT);
  return true;
}

// Takes a consumer ticket if `ticket` holds none, then checks whether that
// ticket's chunk has arrived.  Returns true with the chunk, or false (the
// ticket is kept for the next call, or dropped if its producer gave up).
__device__ bool q_take(const BatchArgs& A, uint64_t& ticket, uint64_t& tile, uint64_t& hi,
                       uint16_t& meta, int& count, int& inst) {
  const int lane = lane_id();
  QueueCtl* q = A.q;
  const uint64_t mask = A.qmask;
  int ready = 0;
  if (lane == 0) {
    if (ticket == kNoTicket) ticket = __hip_atomic_fetch_add(&q->head, (uint64_t)1, __ATOMIC_RELAXED, AGENT);
    SlotCtl* sc = A.seq + (ticket & mask);
    const uint64_t v = ld_relaxed(&sc->seq);
    ready = v == 4 * ticket + 2;
    if (!ready && v == 4 * ticket && ld_relaxed(&sc->abandoned) > ticket &&
        cas64(&sc->seq, 4 * ticket, 4 * (ticket + mask + 1))) {
      // a producer of this slot gave up at or after this ticket: hand the
      // slot on and take a new ticket next time
      ticket = kNoTicket;
    }
  }
  ticket = bcast64(ticket);
  if (!wave_bcast(ready)) return false;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const QChunk* c = A.slots + (ticket & mask);
  tile = c->tiles[lane];
  meta = c->meta[lane];
  count = wave_bcast(c->count);
  inst = wave_bcast(c->inst);
  // the high words only for a 5x5 chunk: a 4x4 chunk reads 6 lines, not 10
  const int wide = wave_bcast(c->wide);
  hi = wide ? A.hi[(ticket & mask) * kQChunk + lane] : 0ull;
  if (wide && lane == 0) __hip_atomic_fetch_add(&q->chunks_read_wide, (uint64_t)1, __ATOMIC_RELAXED, AGENT);
  WAVE_SYNC_MEM();  // all lanes have read the slot before it is handed back
  if (lane == 0)
    __hip_atomic_store(&A.seq[ticket & mask].seq, 4 * (ticket + mask + 1), __ATOMIC_RELEASE, AGENT);
  ticket = kNoTicket;
  return true;
}

// ---------------------------------------------------------------------------
// Limit bookkeeping, executed by one wave.
// ---------------------------------------------------------------------------

// Pushes the roots of instance i with f <= limit as chunks, under a guard
// unit so that the limit cannot complete while seeding.  Returns true if the
// guard's release brought the instance's outstanding count to zero, i.e. the
// caller must complete the limit itself.
// `stage` (128 u64) and `stage_m` (64 u16) are LDS the caller does not use
// while seeding (its LDS stack is empty whenever a limit is seeded).
__device__ bool seed_limit(const BatchArgs& A, int i, uint64_t* stage, uint16_t* stage_m) {
  const int lane = lane_id();
  InstState* S = A.is + i;
  const int L = S->limit;
  const bool wide = S->width == 5;
  if (lane == 0) __hip_atomic_store(&S->outstanding, 1, __ATOMIC_RELAXED, AGENT);
  const NodeW* roots = A.tree + S->root_off;
  // first-solution mode: a goal inside the split tree ends the search at
  // this limit without searching any subtree
  const int nroots = (A.first_solution && A.goal_g[i] <= L) ? 0 : S->nroots;
  int fm = INT_MAX;
  bool full = false;
  for (int base = 0; base < nroots && !full; base += 64) {
    const int r = base + lane;
    NodeW R;
    R.lo = 0;
    R.hi = 0;
    R.meta = 0;
    R.f = 0;
    bool keep = false;
    if (r < nroots) {
      R = roots[r];
      keep = (int)R.f <= L;
      if (!keep) fm = min(fm, (int)R.f);
    }
    const uint64_t km = __ballot(keep);
    const int cnt = __popcll(km);
    if (cnt == 0) continue;
    // compact the kept roots into lanes 0..cnt-1 through LDS
    const int off = __builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32),
                                              __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
    if (keep) {
      stage[off] = R.lo;
      stage[64 + off] = R.hi;
      stage_m[off] = stack_meta((int)(R.meta & 31u), (int)((R.meta >> 5) & 7u), L - (int)R.f);
    }
    WAVE_SYNC();
    // chunks of seed_chunk roots: smaller seeds when a batch has few roots
    // per workgroup, so the whole grid has work from the start
    const int sc = A.seed_chunk > 0 ? A.seed_chunk : kQChunk;
    for (int p0 = 0; p0 < cnt && !full; p0 += sc) {
      const int pc = min(sc, cnt - p0);
      const uint64_t t = lane < pc ? stage[p0 + lane] : 0ull;
      const uint64_t th = lane < pc ? stage[64 + p0 + lane] : 0ull;
      const uint16_t m = lane < pc ? stage_m[p0 + lane] : (uint16_t)0;
      if (lane == 0) __hip_atomic_fetch_add(&S->outstanding, 1, __ATOMIC_RELAXED, AGENT);
      if (!q_push(A, t, th, m, pc, i, wide)) {
        full = true;  // the remaining roots are dropped; the call reports BPIDA_ENOMEM
        if (lane == 0) {
          __hip_atomic_fetch_add(&S->outstanding, -1, __ATOMIC_RELAXED, AGENT);
          __hip_atomic_store(&S->lost, 1, __ATOMIC_RELAXED, AGENT);
          atomicOr(&A.q->err, 1);
        }
      }
    }
    WAVE_SYNC();
  }
  fm = wave_min(fm);
  int last = 0;
  if (lane == 0) {
    if (nroots) __hip_atomic_fetch_add(&A.q->roots_read, (uint64_t)nroots, __ATOMIC_RELAXED, AGENT);
    if (fm != INT_MAX) __hip_atomic_fetch_min(&S->fmin, fm, __ATOMIC_RELAXED, AGENT);
    last = __hip_atomic_fetch_add(&S->outstanding, -1, __ATOMIC_ACQ_REL, AGENT) == 1;
  }
  return wave_bcast(last) != 0;
}

// Server mode: copy slot i's answer into the pinned result ring, publish it,
// and free the slot.  Executed by one wave after the slot's outputs are final.
__device__ void emit_result(const BatchArgs& A, int i, int status) {
  const int lane = lane_id();
  const ServerArgs& V = A.srv;
  WAVE_SYNC_MEM();  // the slot's output row, written by lane 0, is visible
  const uint64_t t = V.ticket[i];
  ServerRes* r = V.res + (t & V.ring_mask);
  r->nodes[lane] = A.out_nodes[(size_t)i * 64 + lane];
  if (lane == 0) {
    r->len = A.out_len[i];
    r->status = status;
  }
  WAVE_SYNC_MEM();
  if (lane == 0) {
    __hip_atomic_store(&r->seq, t + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&V.busy[i], 0, __ATOMIC_RELEASE, AGENT);
    __hip_atomic_fetch_add(V.in_flight, -1, __ATOMIC_RELEASE, AGENT);
  }
}

// Completes the current limit of instance i (its outstanding count is zero
// and this wave observed it), then advances it.  Loops while a new limit
// has no queued work.
__device__ void complete_limit(const BatchArgs& A, int i, uint64_t* stage, uint16_t* stage_m) {
  const int lane = lane_id();
  InstState* S = A.is + i;
  for (;;) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int L = S->limit;
    const int col = S->col;
    // interior nodes of the split tree (depth < D) expanded at this limit
    const uint32_t* h = A.hist + (size_t)i * kHistBins;
    uint64_t interior = 0;
    int fm = INT_MAX;
    for (int f = lane; f < kHistBins; f += 64) {
      const uint32_t c = h[f];
      if (f <= L) interior += c;
      else if (c) fm = min(fm, f);
    }
    for (int o = 32; o > 0; o >>= 1) interior += __shfl_xor(interior, o, 64);
    fm = wave_min(fm);
    int state = 0;  // 0: advance, 1: solved, <0: error code
    if (lane == 0) {
      const uint64_t total = ld_relaxed(&S->nodes) + interior;
      A.out_nodes[(size_t)i * 64 + col] = total;
      const int goals = ld_relaxed(&S->goals);
      const int fnext = min(fm, ld_relaxed(&S->fmin));
      if (ld_relaxed(&S->lost)) {
        state = -4;  // BPIDA_ENOMEM: work of this limit was dropped, its counts are void
      } else if (goals > 0 || A.goal_g[i] <= L) {
        A.out_len[i] = L;
        state = 1;
      } else if (fnext != L + 2) {
        state = -6;  // BPIDA_EINTERNAL
      } else if (A.exact_limit) {
        state = 2;  // one limit only, and no goal within it
      } else if (col + 1 >= 64 || L + 2 > A.max_limit) {
        state = -3;  // BPIDA_ELIMIT
      }
      if (state != 0) {
        __hip_atomic_store(&S->done, state, __ATOMIC_RELAXED, AGENT);
        if (!A.server) __hip_atomic_fetch_add(&A.q->remaining, -1, __ATOMIC_RELEASE, AGENT);
      } else {
        S->limit = L + 2;
        S->col = col + 1;
        __hip_atomic_store(&S->nodes, (uint64_t)0, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&S->fmin, INT_MAX, __ATOMIC_RELAXED, AGENT);
        __hip_atomic_store(&S->goals, 0, __ATOMIC_RELAXED, AGENT);
      }
    }
    state = wave_bcast(state);
    if (state != 0) {
      if (A.server) emit_result(A, i, state);
      return;
    }
    WAVE_SYNC_MEM();
    if (!seed_limit(A, i, stage, stage_m)) return;
  }
}

// ---------------------------------------------------------------------------
// Server admission, executed by the one workgroup holding the admitter role.
// ---------------------------------------------------------------------------

// Validate and pack a state of 16 bytes (in pinned host memory) with one wave.
__device__ Inst wave_ingest4(const uint8_t* src) {
  const int lane = lane_id();
  const uint32_t v = lane < 16 ? (uint32_t)src[lane] : 0u;
  // permutation: every value 0..15 exactly once
  uint32_t seen = lane < 16 && v < 16 ? (1u << v) : 0u;
  for (int o = 32; o > 0; o >>= 1) seen |= __shfl_xor(seen, o, 64);
  const uint64_t valid = __builtin_amdgcn_ballot_w64(lane < 16 && v < 16);
  const uint64_t blank_m = __builtin_amdgcn_ballot_w64(lane < 16 && v == 0);
  // inversions: lane p counts q > p with v[q] < v[p]
  uint32_t inv = 0;
  for (int q = 0; q < 16; ++q) {
    const uint32_t vq = (uint32_t)__shfl((int)v, q, 64);
    inv += (lane < 16 && q > lane && vq < v) ? 1u : 0u;
  }
  int h = 0;
  if (lane < 16 && v != 0) {
    const int dr = (lane >> 2) - (int)(v >> 2), dc = (lane & 3) - (int)(v & 3);
    h = (dr < 0 ? -dr : dr) + (dc < 0 ? -dc : dc);
  }
  uint64_t word = lane < 16 ? (uint64_t)(v & 15u) << (4 * lane) : 0ull;
  for (int o = 32; o > 0; o >>= 1) {
    inv += (uint32_t)__shfl_xor((int)inv, o, 64);
    h += __shfl_xor(h, o, 64);
    word |= (uint64_t)__shfl_xor((long long)word, o, 64);
  }
  Inst I;
  I.tiles = word;
  I.blank = blank_m ? (int)__builtin_ctzll(blank_m) : 0;
  I.h0 = h;
  I.pad = 0;
  if (seen != 0xFFFFu || valid != 0xFFFFull) I.status = -1;  // BPIDA_EINVAL
  else {
    const uint32_t bpar = (uint32_t)((I.blank >> 2) + (I.blank & 3)) & 1u;
    I.status = ((inv & 1u) == bpar) ? 0 : -2;  // BPIDA_EUNSOLVABLE
  }
  return I;
}

// The root split of one instance with one wave (CreateRootSet; same tree as
// split4_kernel): levels 0..depth of the parent-pruned tree are written to
// base[], interior nodes binned by f in hist_lds (256 entries of LDS).
// Returns the first root's index inside base; the root count is
// walks[blank][depth].
__device__ int64_t wave_split4(const Inst& I, int depth, const int32_t* walks, NodeW* base,
                               uint32_t* hist_lds, uint32_t* hist_out, int32_t* goal_g_out) {
  const int lane = lane_id();
  for (int k = lane; k < kHistBins; k += 64) hist_lds[k] = 0;
  if (lane == 0) {
    NodeW r;
    r.lo = I.tiles;
    r.hi = 0;
    r.meta = node_meta(I.blank, 4, 0, I.h0);
    r.f = (uint32_t)I.h0;
    base[0] = r;
  }
  WAVE_SYNC_MEM();
  const int32_t* lc = walks + walk_row(I.blank, 4);
  int gmin = INT_MAX;
  int64_t lvl = 0;
  for (int d = 0; d < depth; ++d) {
    const int cnt = lc[d];
    const int64_t next = lvl + cnt;
    int64_t fill = next;
    for (int k0 = 0; k0 < cnt; k0 += 64) {
      const int k = k0 + lane;
      NodeW nd;
      nd.lo = 0;
      nd.hi = 0;
      nd.meta = 0;
      nd.f = 0;
      if (k < cnt) nd = base[lvl + k];
      const int b = (int)(nd.meta & 31u), fb = (int)((nd.meta >> 5) & 7u);
      const int g = (int)((nd.meta >> 8) & 255u), h = (int)((nd.meta >> 16) & 255u);
      if (k < cnt) {
        atomicAdd(&hist_lds[min(g + h, kHistBins - 1)], 1u);
        if (nd.lo == kGoal4) gmin = min(gmin, g);
      }
      for (int a = 0; a < 4; ++a) {
        const bool ok = k < cnt && ((kMoveMask4 >> (4 * b + a)) & 1ull) && a != fb;
        const int nn = (b + (a == 0 ? -4 : a == 1 ? -1 : a == 2 ? 1 : 4)) & 15;
        const uint32_t t = (uint32_t)(nd.lo >> (4 * nn)) & 15u;
        const int sh = (a == 0 || a == 3) ? 2 : 0;
        const uint32_t idx = (((t >> sh) & 3u) << 2) | (((uint32_t)nn >> sh) & 3u);
        const int h2 = h + (((kDhTable4 >> (16 * a + idx)) & 1ull) ? 1 : -1);
        const uint64_t km = __builtin_amdgcn_ballot_w64(ok);
        const int off = __builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
        if (ok && fill + off < next + lc[d + 1]) {  // the level's exact size bounds it
          NodeW c;
          c.lo = nd.lo + ((uint64_t)t << (4 * b)) - ((uint64_t)t << (4 * nn));
          c.hi = 0;
          c.meta = node_meta(nn, 3 - a, g + 1, h2);
          c.f = (uint32_t)(g + 1 + h2);
          base[fill + off] = c;
        }
        fill += __popcll(km);
      }
    }
    WAVE_SYNC_MEM();  // this level's children are visible to the whole wave
    lvl = next;
  }
  gmin = wave_min(gmin);
  for (int k = lane; k < kHistBins; k += 64) hist_out[k] = hist_lds[k];
  if (lane == 0) *goal_g_out = gmin;
  WAVE_SYNC_MEM();
  return lvl;
}

// Admits requests until the host asks to stop and nothing is in flight.
__device__ void admitter_loop(const BatchArgs& A, uint64_t* st, uint16_t* sm, uint64_t deadline) {
  const int lane = lane_id();
  const ServerArgs& V = A.srv;
  QueueCtl* q = A.q;
  uint32_t* hist_lds = (uint32_t*)st;  // the stack is unused by the admitter
  uint64_t head = 0;
  int cursor = 0;
  for (;;) {
    if (wall_clock64() > deadline) {
      if (lane == 0) {
        atomicOr(&q->err, 8);
        __hip_atomic_store(&q->remaining, 0, __ATOMIC_RELEASE, AGENT);
      }
      return;
    }
    uint64_t tail = 0;
    int stop = 0, busy_all = 0;
    if (lane == 0) {
      tail = __hip_atomic_load(&V.host->req_tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
      stop = __hip_atomic_load(&V.host->stop, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    tail = bcast64(tail);
    stop = wave_bcast(stop);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // request bytes published before req_tail
    if (tail == head) {
      if (stop) {
        int inflight = 0;
        if (lane == 0) inflight = __hip_atomic_load(V.in_flight, __ATOMIC_ACQUIRE, AGENT);
        if (wave_bcast(inflight) == 0) {
          if (lane == 0) __hip_atomic_store(&q->remaining, 0, __ATOMIC_RELEASE, AGENT);
          return;
        }
      }
      __builtin_amdgcn_s_sleep(32);
      continue;
    }
    // the HBM frontier budget: while more chunks wait in the work queue than
    // the budget allows, the searching workgroups are behind, and a new
    // request's seeds (and later spills) could overflow it; wait
    if (V.backlog_max > 0) {
      int64_t backlog = 0;
      if (lane == 0) backlog = (int64_t)(ld_relaxed(&q->tail) - ld_relaxed(&q->head));
      backlog = (int64_t)bcast64((uint64_t)backlog);
      if (backlog > V.backlog_max) {
        __builtin_amdgcn_s_sleep(32);
        continue;
      }
    }
    // a free instance slot (the in-flight budget); wait if none
    int slot = -1;
    for (int k0 = 0; k0 < V.slots && slot < 0; k0 += 64) {
      const int j = (cursor + k0 + lane) % V.slots;
      const bool fr = k0 + lane < V.slots &&
                      __hip_atomic_load(&V.busy[j], __ATOMIC_ACQUIRE, AGENT) == 0;
      const uint64_t fm = __builtin_amdgcn_ballot_w64(fr);
      if (fm) slot = (cursor + k0 + (int)__builtin_ctzll(fm)) % V.slots;
    }
    if (slot < 0) {
      busy_all = 1;
      __builtin_amdgcn_s_sleep(32);
      continue;
    }
    (void)busy_all;
    cursor = (slot + 1) % V.slots;
    const Inst I = wave_ingest4(V.req[head & V.ring_mask].state);
    if (lane == 0) {
      __hip_atomic_store(&V.host->req_admitted, head + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
      V.busy[slot] = 1;
      V.ticket[slot] = head;
      __hip_atomic_fetch_add(V.in_flight, 1, __ATOMIC_RELAXED, AGENT);
    }
    A.out_nodes[(size_t)slot * 64 + lane] = 0;
    if (lane == 0) A.out_len[slot] = -1;
    InstState S;
    S.limit = first_limit(I.h0, A.start_limit);
    S.col = (S.limit - I.h0) / 2;
    S.done = I.status;
    S.outstanding = 0;
    S.nodes = 0;
    S.fmin = INT_MAX;
    S.goals = 0;
    S.stop = 0;
    S.lost = 0;
    S.root_off = (int64_t)slot * V.stride;
    S.nroots = 0;
    S.width = 4;
    if (I.status == 0) {
      NodeW* base = const_cast<NodeW*>(A.tree) + (int64_t)slot * V.stride;
      const int64_t r0 = wave_split4(I, V.depth, V.walks, base, hist_lds,
                                     const_cast<uint32_t*>(A.hist) + (size_t)slot * kHistBins,
                                     const_cast<int32_t*>(A.goal_g) + slot);
      S.root_off += r0;
      S.nroots = V.walks[walk_row(I.blank, 4) + V.depth];
      // a first limit past the cap or past the 64 output columns
      if (S.limit > A.max_limit || S.col >= 64) S.done = -3;  // BPIDA_ELIMIT
    }
    if (lane == 0) A.is[slot] = S;
    WAVE_SYNC_MEM();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (S.done != 0) emit_result(A, slot, S.done);
    else if (seed_limit(A, slot, st, sm)) complete_limit(A, slot, st, sm);
    ++head;
  }
}

// Adds this workgroup's counts for the unit of instance i it held and
// releases the unit; completes the limit if it was the last unit.
__device__ void release_unit(const BatchArgs& A, int i, uint64_t expanded, int goals, int fmin,
                             uint64_t* stage, uint16_t* stage_m) {
  const int lane = lane_id();
  InstState* S = A.is + i;
  fmin = wave_min(fmin);
  int last = 0;
  if (lane == 0) {
    if (expanded) __hip_atomic_fetch_add(&S->nodes, expanded, __ATOMIC_RELAXED, AGENT);
    if (goals) __hip_atomic_fetch_add(&S->goals, goals, __ATOMIC_RELAXED, AGENT);
    if (fmin != INT_MAX) __hip_atomic_fetch_min(&S->fmin, fmin, __ATOMIC_RELAXED, AGENT);
    last = __hip_atomic_fetch_add(&S->outstanding, -1, __ATOMIC_ACQ_REL, AGENT) == 1;
  }
  if (wave_bcast(last)) complete_limit(A, i, stage, stage_m);
}

// ---------------------------------------------------------------------------
// The persistent kernel.
// ---------------------------------------------------------------------------
// Per-workgroup run counters.
struct WgCounters {
  uint64_t rounds = 0, pushes = 0, voluntary = 0;
};

// Searches one unit (the chunk already in LDS entries [0, cnt)) of an
// instance of width W until its stack is empty: BPDFS rounds, with spills
// to the queue when LDS would overflow and donations to waiting workgroups.
// NPL = nodes popped per round: 16 (lane l expands node l/4 with move l%4,
// Alg. 1's thread -> action map; width 4 only) or 64 (one node per lane,
// four moves each).  Returns false if the time budget ran out (abandoned).
template <int W, int CAP, int NPL, bool FS>
__device__ bool run_unit(const BatchArgs& A, int inst, int limit, typename Board<W>::S* st,
                         uint16_t* sm, int cnt, WgCounters& wc, uint32_t& tick, uint64_t deadline,
                         uint64_t& expanded, int& goals, int& fmin) {
  static_assert(NPL == 64 || W == 4, "16-node rounds are the 4x4 map");
  static_assert(NPL == 64 ? CAP >= 256 : ((CAP & (CAP - 1)) == 0 && CAP >= 128), "stack size");
  using S = typename Board<W>::S;
  const int lane = lane_id();
  QueueCtl* q = A.q;
  const bool wide = W == 5;
  // largest growth of one round: a node has at most 3 children (its parent's
  // cell is excluded).  Only a root of the split (depth 0) has no parent and
  // may have 4, and a root is expanded in the unit's first round, which
  // starts from one chunk (at most 64 entries) and so cannot overflow.
  constexpr int kGrow = NPL == 16 ? 32 : 2 * 64;
  // 64-node rounds on 3x3 and 4x4 stacks store without branches (under the
  // keep mask)
  constexpr bool kMasked = NPL == 64 && sizeof(S) == 8;
  // the width-4 64-node round keeps its stack in its own layout (its own
  // meta word; 12-byte interleaved entries at 672 entries); chunks carry
  // the common meta word
  constexpr bool kMeta4 = NPL == 64 && W == 4;
  constexpr int kCap = CAP;
  const LaneMap M = make_lane_map(lane);
  const RoundConsts4 rk = make_round_consts4();
  // Donating from a shallow stack hands over pieces too small to pay for the
  // transfer; a threshold the stack seldom reaches stops donation and leaves
  // subtrees on one workgroup.  Default: four rounds' worth of pops, at most
  // half the stack.
  const int dmin = A.donate_min > 0 ? A.donate_min : min(4 * NPL, CAP / 2);
  // The LDS stack holds entries [0, top), the oldest at 0.  Entries taken
  // from the bottom (spills, donations) make the rest move down, so a
  // position never wraps and a round addresses the stack without a mask.
  uint32_t top = (uint32_t)cnt;
  if (FS && wave_bcast(lane == 0 ? ld_relaxed(&A.is[inst].stop) : 0)) top = 0;
  // The deadline, donation and first-solution polls come every
  // min(64, donate_every) rounds, a period that divides each of theirs; the
  // rounds in between test only whether the next round needs a spill.
  const uint32_t poll_mask = min(A.donate_mask, 63u);
  while (top != 0) {
    int avail = (int)top;
    ++tick;
    const bool poll = (tick & poll_mask) == 0;
    if (poll) {
      if ((tick & 1023u) == 0) {
        // the time budget is spent, or work was dropped somewhere (every
        // count is void and the call reports BPIDA_ENOMEM): stop instead of
        // searching on
        const bool late = wall_clock64() > deadline;
        if (late || (!A.server && (ld_wave(&q->err) & kErrFatal))) {
          if (late && lane == 0) atomicOr(&q->err, 8);
          return false;
        }
      }
      if (avail + kGrow <= kCap && avail >= dmin && (tick & A.donate_mask) == 0) {
        // donation when workgroups wait on tickets no queued chunk covers:
        // the oldest min(window, avail) entries (the shallowest, largest
        // subtrees) are split alternately, so donor and receiver each keep
        // about half
        int want = 0;
        if (lane == 0) want = (int64_t)(ld_relaxed(&q->head) - ld_relaxed(&q->tail)) > 0;
        if (wave_bcast(want)) {
          const int w = min(avail, A.donate_window) & ~1;
          const int h = w >> 1;
          // (positions up to 127: inside the stack's storage, read for every lane)
          S tg, tk;
          uint16_t mg, mk;
          if constexpr (kMeta4) {
            tg = (S)e4_tile<CAP>((uint64_t*)st, 2 * lane);
            tk = (S)e4_tile<CAP>((uint64_t*)st, 2 * lane + 1);
            mg = (uint16_t)e4_meta<CAP>((uint64_t*)st, 2 * lane);
            mk = (uint16_t)e4_meta<CAP>((uint64_t*)st, 2 * lane + 1);
          } else {
            tg = st[2 * lane];
            tk = st[2 * lane + 1];
            mg = sm[2 * lane];
            mk = sm[2 * lane + 1];
          }
          WAVE_SYNC();
          if (lane == 0) __hip_atomic_fetch_add(&A.is[inst].outstanding, 1, __ATOMIC_RELAXED, AGENT);
          if (q_push(A, (uint64_t)tg, wide ? (uint64_t)((unsigned __int128)tg >> 64) : 0ull,
                     kMeta4 ? (uint16_t)meta4_out(mg) : mg, h, inst, wide)) {
            wc.pushes += 1;
            wc.voluntary += 1;
            // the kept half becomes the bottom, the entries above the window
            // close up behind it
            if constexpr (kMeta4) {
              if (lane < h) e4_put<CAP>((uint64_t*)st, lane, (uint64_t)tk, mk);
              WAVE_SYNC();
              move_down4<CAP>((uint64_t*)st, (uint32_t)h, (uint32_t)w, top - (uint32_t)w);
            } else {
              if (lane < h) {
                st[lane] = tk;
                sm[lane] = mk;
              }
              move_down(st, sm, (uint32_t)h, (uint32_t)w, top - (uint32_t)w);
            }
            top -= (uint32_t)h;
            avail -= h;
          } else if (lane == 0) {
            __hip_atomic_fetch_add(&A.is[inst].outstanding, -1, __ATOMIC_RELAXED, AGENT);
          }
        }
      }
    }
    if (avail + kGrow > kCap) {
      // LDS could overflow: move the oldest entries to the queue, 64 at a
      // time, until the largest round fits.
      do {
        const S t = kMeta4 ? (S)e4_tile<CAP>((uint64_t*)st, lane) : st[lane];
        const uint16_t m = kMeta4 ? (uint16_t)e4_meta<CAP>((uint64_t*)st, lane) : sm[lane];
        WAVE_SYNC();
        if (lane == 0) __hip_atomic_fetch_add(&A.is[inst].outstanding, 1, __ATOMIC_RELAXED, AGENT);
        if (q_push(A, (uint64_t)t, wide ? (uint64_t)((unsigned __int128)t >> 64) : 0ull,
                   kMeta4 ? (uint16_t)meta4_out(m) : m, 64, inst, wide)) {
          wc.pushes += 1;
        } else if (lane == 0) {
          __hip_atomic_fetch_add(&A.is[inst].outstanding, -1, __ATOMIC_RELAXED, AGENT);
          __hip_atomic_store(&A.is[inst].lost, 1, __ATOMIC_RELAXED, AGENT);
          atomicOr(&q->err, 2);  // entries dropped: the call reports BPIDA_ENOMEM
        }
        if constexpr (kMeta4) move_down4<CAP>((uint64_t*)st, 0u, 64u, top - 64u);
        else move_down(st, sm, 0u, 64u, top - 64u);
        top -= 64u;
        avail -= 64;
      } while (avail + kGrow > kCap);
    }
    const int kp = min(avail, NPL);
    if constexpr (NPL == 16) {
      top = bp_round<CAP>((uint64_t*)st, sm, top, kp, limit, M, goals, fmin);
    } else {
      top = bp_round64w<W, CAP, kMasked, false>(st, sm, top, kp, goals, rk);
    }
    // the spill above keeps every round inside the stack; a round that ended
    // past it would have overwritten entries (reported, never silent)
    if (top > (uint32_t)kCap) atomicOr(&q->err, 32);  // every lane: a uniform branch
    expanded += (uint64_t)kp;
    wc.rounds += 1;
    if constexpr (FS) {
      // first-solution mode (Alg. 1 returns at its first goal): the unit that
      // expands a goal stops its instance; the others see the flag within 64
      // rounds and drop their stacks
      if (goals > 0) {
        if (lane == 0) __hip_atomic_store(&A.is[inst].stop, 1, __ATOMIC_RELAXED, AGENT);
        break;
      }
      if (poll && (tick & 63u) == 0 && wave_bcast(lane == 0 ? ld_relaxed(&A.is[inst].stop) : 0))
        break;
    }
    if constexpr (NPL == 64) {
      // Full rounds with nothing else to test: while the stack holds 64
      // entries and has room for their children (the condition under which
      // the round above needs no spill) and no poll is due, 64-node rounds
      // run back to back; their counts are added once at the end.  The
      // first-solution search also leaves after a round that expanded a goal
      // (a test of the wave's goal mask, uniform), and stops its instance
      // outside the loop.
      const uint32_t n = (uint32_t)__builtin_amdgcn_readfirstlane((int)(poll_mask - (tick & poll_mask)));
      uint32_t r = 0;
      uint64_t gm = 0;  // lanes that expanded a goal (only "any" matters)
      for (;;) {
        if (r >= n) break;
        if (top - 64u > (uint32_t)(kCap - kGrow - 64)) break;
        top = bp_round64w<W, CAP, kMasked, true>(st, sm, top, 64, gm, rk);
        ++r;
        if constexpr (FS) {
          if (gm != 0) break;
        }
      }
      if (gm != 0) goals += 1;
      tick += r;
      expanded += 64ull * r;
      wc.rounds += r;
      if constexpr (FS) {
        if (goals > 0) {
          if (lane == 0) __hip_atomic_store(&A.is[inst].stop, 1, __ATOMIC_RELAXED, AGENT);
          break;
        }
      }
    }
  }
  // 64-node rounds: a pruned child always has f = limit + 2 (bp_round64w),
  // and every limit below the optimum prunes one: below the optimum, a path
  // of approaching moves from a slack-0 node cannot reach the goal, so it
  // ends at a node whose remaining moves all go away and are pruned
  if (NPL == 64) fmin = limit + 2;
  return true;
}

// The persistent kernel.  A workgroup holds WPG independent waves (Sec. 5's
// block = one warp, WPG times over): each wave has its own stack and takes
// its own work, and no wave ever waits for another.  LDS per wave: CAP
// entries of u64 tiles + u16 meta for widths 3 and 4 (10 bytes an entry;
// 12 for width 4 in the interleaved layout, which then sizes the stack for
// every width), CAP/2 entries of 128-bit tiles + u16 meta for width 5; the
// width is read per chunk from the instance.
//
// Waves per SIMD a one-wave workgroup's 64-node stack allows (LDS: 160 KB
// per compute unit): 24 per compute unit at 640 entries, 20 at 672
// (interleaved) and 768, 16 at 1024.  The launch bound keeps the vector
// registers within that occupancy (at most 80 per lane at 6 waves per SIMD,
// 96 at 5), capped at 6.
template <int CAP, int NPL>
constexpr int batch_waves_per_simd() {
  constexpr int w = NPL != 64 ? 1 : (int)(163840u / stack4_bytes<CAP>()) / 4;
  return w > 6 ? 6 : w < 1 ? 1 : w;
}

template <int CAP, int NPL, int WPG, bool FS>
__global__ __launch_bounds__(64 * WPG, (batch_waves_per_simd<CAP, NPL>())) void batch4_kernel(BatchArgs A) {
  static_assert(CAP % 16 == 0 && (NPL == 64 || (CAP & (CAP - 1)) == 0), "stack size");
  static_assert(NPL == 16 || NPL == 64, "nodes per round");
  static_assert(NPL == 16 || CAP >= 256, "stack too small for 64-node rounds");
  static_assert(WPG == 1 || WPG == 2 || WPG == 4, "waves per workgroup");
  // u64 words of one wave's stack: 10 bytes an entry, or 12 with the
  // interleaved width-4 layout of 64-node rounds
  constexpr int kWords = (int)((NPL == 64 ? stack4_bytes<CAP>() : 10u * CAP) / 8u);
  __shared__ __attribute__((aligned(16))) uint64_t lds[WPG * kWords];
  uint64_t* st = lds + (WPG == 1 ? 0 : (int)(threadIdx.x >> 6) * kWords);  // widths 3, 4: CAP tiles
  uint16_t* sm = (uint16_t*)(st + CAP);        // CAP (or CAP/2) meta words
  unsigned __int128* st5 = (unsigned __int128*)st;  // width 5: CAP/2 tiles
  const int lane = lane_id();
  QueueCtl* q = A.q;

  if (A.server) {
    int role = 0;
    if (lane == 0) role = atomicCAS(A.srv.admitter, 0, 1) == 0;
    if (wave_bcast(role)) {
      admitter_loop(A, st, sm, wall_clock64() + A.budget_ticks);
      return;
    }
  }

  // Seed the first limit of every instance through a shared cursor: all
  // instances are seeded by workgroups that are running, whatever part of
  // the grid is resident.
  for (;;) {
    int i = 0;
    if (lane == 0) i = __hip_atomic_fetch_add(&q->seed_next, 1, __ATOMIC_RELAXED, AGENT);
    i = wave_bcast(i);
    if (i >= A.n) break;
    if (ld_wave(&q->err) & kErrFatal) break;  // work already lost: stop seeding
    if (A.is[i].done != 0) continue;
    if (seed_limit(A, i, st, sm)) complete_limit(A, i, st, sm);
  }

  WgCounters wc;
  uint64_t searched = 0, pops = 0;
  uint64_t t_work = 0, t_queue = 0, t_idle = 0;
  uint64_t t_mark = wall_clock64();
  bool idle = false;
  uint64_t idle_since = 0, idle_act = 0;
  uint32_t tick = 0;
  int backoff = 1;
  uint64_t ticket = kNoTicket;  // consumer ticket held while idle
  const uint64_t deadline = wall_clock64() + A.budget_ticks;

  for (;;) {
    uint64_t t, th;
    uint16_t m;
    int cnt, inst;
    if (!q_take(A, ticket, t, th, m, cnt, inst)) {
      if (ld_wave(&q->remaining) <= 0) break;
      if (!A.server && (ld_wave(&q->err) & kErrFatal)) break;
      const uint64_t now = wall_clock64();
      // queue activity seen by this idle workgroup (lane 0's view)
      uint64_t act = 0;
      if (lane == 0) act = ld_relaxed(&q->head) + ld_relaxed(&q->tail);
      act = (uint64_t)(uint32_t)wave_bcast((int)(uint32_t)act);
      if (!idle) {
        idle = true;
        idle_since = now;
        idle_act = act;
        backoff = 1;
      } else if (act != idle_act) {
        idle_since = now;  // the queue moved: work is being shared
        idle_act = act;
      } else if (now - idle_since > A.idle_ticks || now > deadline) {
        // no queue activity for the whole watchdog period although
        // instances remain, or the run's time budget is spent
        if (lane == 0) atomicOr(&q->err, now > deadline ? 8 : 4);
        break;
      }
      // exponential backoff (1 .. 8 x 4096 clocks) keeps idle workgroups
      // from flooding the queue's cache lines
      for (int k = 0; k < backoff; ++k) __builtin_amdgcn_s_sleep(64);
      backoff = min(backoff * 2, 8);
      const uint64_t now2 = wall_clock64();
      t_idle += now2 - t_mark;
      t_mark = now2;
      continue;
    }
    idle = false;
    backoff = 1;
    pops += 1;
    {
      const uint64_t now = wall_clock64();
      t_queue += now - t_mark;
      t_mark = now;
    }
    const int limit = A.is[inst].limit;
    const int width = A.is[inst].width;
    uint64_t expanded = 0;
    int goals = 0, fmin = INT_MAX;
    bool ok = true;
    if (width == 4) {
      if (lane < cnt) {
        // the 64-node round's stack has its own layout
        if constexpr (NPL == 64) {
          e4_put<CAP>(st, lane, t, meta4_in(m));
        } else {
          st[lane] = t;
          sm[lane] = m;
        }
      }
      WAVE_SYNC();
      ok = run_unit<4, CAP, NPL, FS>(A, inst, limit, st, sm, cnt, wc, tick, deadline,
                                             expanded, goals, fmin);
    } else if (width == 3) {
      if constexpr (CAP >= 256) {
        if (lane < cnt) {
          st[lane] = t;
          sm[lane] = m;
        }
        WAVE_SYNC();
        ok = run_unit<3, CAP, 64, FS>(A, inst, limit, st, sm, cnt, wc, tick, deadline,
                                              expanded, goals, fmin);
      }
    } else {
      if constexpr (CAP / 2 >= 256) {
        if (lane < cnt) {
          st5[lane] = (unsigned __int128)t | ((unsigned __int128)th << 64);
          sm[lane] = m;
        }
        WAVE_SYNC();
        ok = run_unit<5, CAP / 2, 64, FS>(A, inst, limit, st5, sm, cnt, wc, tick,
                                                  deadline, expanded, goals, fmin);
      }
    }
    if (!ok) break;
    const uint64_t now = wall_clock64();
    t_work += now - t_mark;
    t_mark = now;
    release_unit(A, inst, expanded, goals, fmin, st, sm);
    searched += expanded;
  }
  if (lane == 0) {
    atomicAdd((unsigned long long*)&q->rounds, (unsigned long long)wc.rounds);
    atomicAdd((unsigned long long*)&q->searched, (unsigned long long)searched);
    atomicAdd((unsigned long long*)&q->pushes, (unsigned long long)wc.pushes);
    atomicAdd((unsigned long long*)&q->pops, (unsigned long long)pops);
    atomicAdd((unsigned long long*)&q->t_work, (unsigned long long)t_work);
    atomicAdd((unsigned long long*)&q->t_queue, (unsigned long long)t_queue);
    atomicAdd((unsigned long long*)&q->t_idle, (unsigned long long)t_idle);
    atomicAdd((unsigned long long*)&q->voluntary, (unsigned long long)wc.voluntary);
  }
}

// ---------------------------------------------------------------------------
// Set-up: per-instance state, queue sequence numbers and counters.
// ---------------------------------------------------------------------------
__global__ void batch_setup_kernel(BatchArgs A, const InstW* __restrict__ inst,
                                   const int64_t* __restrict__ root_off,
                                   const int32_t* __restrict__ nroots) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k <= (int64_t)A.qmask) {
    A.seq[k].seq = 4 * (uint64_t)k;
    A.seq[k].abandoned = 0;
  }
  if (k < A.n) {
    InstState S;
    S.limit = first_limit(inst[k].h0, A.start_limit);
    S.col = (S.limit - inst[k].h0) / 2;
    S.done = inst[k].status;  // 0 = to search
    if (A.exact_limit) {
      // one limit only: a limit below h0 or of the other parity has no path
      // of exactly that length
      S.limit = A.exact_limit[k];
      S.col = 0;
      if (S.done == 0 && (S.limit < inst[k].h0 || ((S.limit - inst[k].h0) & 1))) S.done = 2;
    }
    S.outstanding = 0;
    S.nodes = 0;
    S.fmin = INT_MAX;
    S.goals = 0;
    S.stop = 0;
    S.lost = 0;
    S.root_off = root_off[k];
    S.nroots = nroots[k];
    S.width = inst[k].width;
    if (S.done == 0 && (S.limit > A.max_limit || S.col >= 64)) S.done = -3;  // BPIDA_ELIMIT
    A.is[k] = S;
    if (S.done == 0) atomicAdd(&A.q->remaining, 1);
  }
}

// Per-instance status: 1 solved, < 0 a bpida_status.  A failed split or a
// queue that overflowed (its dropped work invalidates every count) marks
// every instance; a watchdog or deadline stop marks the unfinished ones.
__global__ void batch_status_kernel(const InstState* __restrict__ is, int n,
                                    const QueueCtl* __restrict__ q,
                                    const int32_t* __restrict__ split_err, int32_t* __restrict__ st) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int32_t done = is[k].done;
  int32_t v = done;
  if (*split_err) v = -6;                    // BPIDA_EINTERNAL
  else if (q->err & kErrFatal) v = -4;      // BPIDA_ENOMEM
  else if (q->err & 32) v = -6;             // LDS stack overrun: BPIDA_EINTERNAL
  else if (done == 0) v = -6;               // stopped by the watchdog or the deadline
  st[k] = v;
}

// ---------------------------------------------------------------------------
// Ingest and root split of the batched path, any width.
// ---------------------------------------------------------------------------

// One thread per instance: validate (a permutation of 0..w*w-1 whose parity
// matches the blank's distance from cell 0), pack, Manhattan h0.  States are
// w*w bytes at byte_off[i] (or i*w*w); widths[i] (or `width`) per instance.
__global__ void ingestw_kernel(const uint8_t* __restrict__ states, const int64_t* __restrict__ byte_off,
                               const int32_t* __restrict__ widths, int width, int n,
                               InstW* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int w = widths ? widths[i] : width;
  InstW r;
  r.lo = 0;
  r.hi = 0;
  r.blank = 0;
  r.h0 = 0;
  r.status = -1;  // BPIDA_EINVAL
  r.width = w;
  if (w < 3 || w > 5) {
    out[i] = r;
    return;
  }
  const int nn = w * w;
  const int bits = w == 5 ? 5 : 4;
  const uint8_t* s = states + (byte_off ? byte_off[i] : (int64_t)i * nn);
  uint32_t seen = 0;
  bool ok = true;
  unsigned __int128 word = 0;
  int blank = 0, h = 0;
  uint32_t inv = 0;
  for (int p = 0; p < nn; ++p) {
    const uint32_t v = s[p];
    if (v >= (uint32_t)nn || ((seen >> v) & 1u)) ok = false;
    seen |= 1u << (v & 31u);
    if (v == 0) blank = p;
    word |= (unsigned __int128)(v & 31u) << (bits * p);
    if (v != 0 && v < (uint32_t)nn) {
      const int dr = p / w - (int)v / w, dc = p % w - (int)v % w;
      h += (dr < 0 ? -dr : dr) + (dc < 0 ? -dc : dc);
    }
    for (int q = 0; q < p; ++q) inv ^= (uint32_t)(s[q] > v);
  }
  if (ok) {
    const uint32_t bpar = (uint32_t)(blank / w + blank % w) & 1u;
    r.status = inv == bpar ? 0 : -2;  // BPIDA_EUNSOLVABLE
    r.lo = (uint64_t)word;
    r.hi = (uint64_t)(word >> 64);
    r.blank = blank;
    r.h0 = h;
  }
  out[i] = r;
}

hipError_t launch_ingestw(const uint8_t* d_states, const int64_t* d_byte_off, const int32_t* d_widths,
                          int width, int n, InstW* d_inst, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(ingestw_kernel, dim3((n + 127) / 128), dim3(128), 0, s, d_states, d_byte_off,
                     d_widths, width, n, d_inst);
  return hipGetLastError();
}

constexpr int kSplitThreadsW = 256;

// The parent-pruned tree of one instance to depth D, level after level
// (CreateRootSet, no duplicate elimination); the workgroup's instance has
// width W and its start may not make move fb0 first (4: any move).  Level
// sizes come from the walk-count table of that width.
template <int W>
__device__ void split_impl(const InstW& I, int fb0, int depth, const int32_t* walks, NodeW* base,
                           uint32_t* h_lds, int32_t* fill, int32_t* gmin, int32_t* err,
                           int64_t* lvl_out) {
  using B = Board<W>;
  using S = typename B::S;
  const int32_t* lc = walks + walk_row(I.blank, fb0);
  if (threadIdx.x == 0) {
    NodeW r;
    r.lo = I.lo;
    r.hi = I.hi;
    r.meta = node_meta(I.blank, fb0, 0, I.h0);
    r.f = (uint32_t)I.h0;
    base[0] = r;
  }
  __syncthreads();
  int64_t lvl = 0;
  for (int d = 0; d < depth; ++d) {
    const int cnt = lc[d];
    const int64_t next = lvl + cnt;
    for (int k = threadIdx.x; k < cnt; k += kSplitThreadsW) {
      const NodeW nd = base[lvl + k];
      S s = (S)nd.lo;
      if constexpr (W == 5) s |= (S)nd.hi << 64;
      const uint32_t b = nd.meta & 31u, fb = (nd.meta >> 5) & 7u;
      const int g = (int)((nd.meta >> 8) & 255u), h = (int)((nd.meta >> 16) & 255u);
      atomicAdd(&h_lds[min(g + h, kHistBins - 1)], 1u);
      if (s == B::goal()) atomicMin(gmin, g);
      const uint32_t lm = B::legal(b) & ~(1u << fb);
      for (int a = 0; a < 4; ++a) {
        if (!((lm >> a) & 1u)) continue;
        const int delta = a == 0 ? -W : a == 1 ? -1 : a == 2 ? 1 : W;
        const uint32_t nn = b + (uint32_t)delta;
        const uint32_t t = (uint32_t)(s >> (B::BITS * nn)) & B::MASK;
        const bool vert = a == 0 || a == 3;
        const uint32_t ct = vert ? t / W : t % W, cn = vert ? nn / W : nn % W;
        const int up = (int)((B::table(a) >> (ct * W + cn)) & 1u);
        const int h2 = h + (up ? 1 : -1);
        const S cs = s + ((S)t << (B::BITS * b)) - ((S)t << (B::BITS * nn));
        NodeW c;
        c.lo = (uint64_t)cs;
        c.hi = W == 5 ? (uint64_t)((unsigned __int128)cs >> 64) : 0ull;
        c.meta = node_meta((int)nn, 3 - a, g + 1, h2);
        c.f = (uint32_t)(g + 1 + h2);
        const int slot = atomicAdd(fill, 1);
        if (slot < lc[d + 1]) base[next + slot] = c;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      if (*fill != lc[d + 1]) atomicOr(err, 1);
      *fill = 0;
    }
    lvl = next;
    __syncthreads();
  }
  *lvl_out = lvl;
}

// One workgroup of 256 threads per instance; the instance's region is
// tree_off[i] (or i * stride).  `walks` = [width - 3][cell][first forbidden
// move][length] counts; `forbid` (null: none) = per instance the move its
// start may not make first (4: any).
__global__ __launch_bounds__(kSplitThreadsW) void splitw_kernel(
    const InstW* __restrict__ inst, int depth, const int64_t* __restrict__ tree_off, int64_t stride,
    const int32_t* __restrict__ walks, const uint8_t* __restrict__ forbid, NodeW* __restrict__ tree,
    uint32_t* __restrict__ hist, int32_t* __restrict__ goal_g, int32_t* __restrict__ err,
    int64_t* __restrict__ root_off, int32_t* __restrict__ nroots) {
  const int i = blockIdx.x;
  const InstW I = inst[i];
  const int fb0 = forbid ? min((int)forbid[i], 4) : 4;
  __shared__ uint32_t h_lds[kHistBins];
  __shared__ int32_t fill;
  __shared__ int32_t gmin;
  for (int k = threadIdx.x; k < kHistBins; k += kSplitThreadsW) h_lds[k] = 0;
  if (threadIdx.x == 0) {
    gmin = INT_MAX;
    fill = 0;
  }
  const int64_t region = tree_off ? tree_off[i] : (int64_t)i * stride;
  NodeW* base = tree + region;
  int64_t lvl = 0;
  if (I.status == 0) {
    const int32_t* wk = walks + (size_t)(I.width - 3) * kWalkStride;
    if (I.width == 3) split_impl<3>(I, fb0, depth, wk, base, h_lds, &fill, &gmin, err, &lvl);
    else if (I.width == 4) split_impl<4>(I, fb0, depth, wk, base, h_lds, &fill, &gmin, err, &lvl);
    else split_impl<5>(I, fb0, depth, wk, base, h_lds, &fill, &gmin, err, &lvl);
  } else {
    __syncthreads();
  }
  for (int k = threadIdx.x; k < kHistBins; k += kSplitThreadsW) hist[(size_t)i * kHistBins + k] = h_lds[k];
  if (threadIdx.x == 0) {
    goal_g[i] = gmin;
    root_off[i] = region + lvl;
    nroots[i] = I.status == 0
                    ? walks[(size_t)(I.width - 3) * kWalkStride + walk_row(I.blank, fb0) + depth]
                    : 0;
  }
}

hipError_t launch_splitw(const InstW* d_inst, int n, int depth, const int64_t* d_tree_off,
                         int64_t stride, const int32_t* d_walks, const uint8_t* d_forbid,
                         NodeW* d_tree, uint32_t* d_hist, int32_t* d_goal_g, int32_t* d_err,
                         int64_t* d_root_off, int32_t* d_nroots, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(splitw_kernel, dim3(n), dim3(kSplitThreadsW), 0, s, d_inst, depth, d_tree_off,
                     stride, d_walks, d_forbid, d_tree, d_hist, d_goal_g, d_err, d_root_off,
                     d_nroots);
  return hipGetLastError();
}

// Server set-up: queue sequence numbers, free instance slots, one sentinel in
// `remaining` (cleared by the admitter when the server shuts down).
__global__ void server_setup_kernel(BatchArgs A) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k <= (int64_t)A.qmask) {
    A.seq[k].seq = 4 * (uint64_t)k;
    A.seq[k].abandoned = 0;
  }
  if (k < A.srv.slots) A.srv.busy[k] = 0;
  if (k == 0) {
    A.q->remaining = 1;
    *A.srv.admitter = 0;
    *A.srv.in_flight = 0;
  }
}

hipError_t launch_server_setup(const BatchArgs& A, hipStream_t s) {
  const int64_t work = std::max<int64_t>((int64_t)A.qmask + 1, A.srv.slots);
  hipLaunchKernelGGL(server_setup_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_batch_setup(const BatchArgs& A, const InstW* d_inst, const int64_t* d_root_off,
                              const int32_t* d_nroots, hipStream_t s) {
  const int64_t work = std::max<int64_t>((int64_t)A.qmask + 1, A.n);
  hipLaunchKernelGGL(batch_setup_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, A,
                     d_inst, d_root_off, d_nroots);
  return hipGetLastError();
}

hipError_t launch_batch_status(const InstState* d_is, int n, const QueueCtl* d_q,
                               const int32_t* d_split_err, int32_t* d_status, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_status_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d_is, n, d_q,
                     d_split_err, d_status);
  return hipGetLastError();
}

// The first-solution search is a kernel of its own: with both unit loops in
// one kernel the register allocation of each suffers.
template <int CAP, int NPL, int WPG>
static hipError_t launch_batch_t(int grid, const BatchArgs& A, hipStream_t s) {
  if (A.first_solution)
    hipLaunchKernelGGL((batch4_kernel<CAP, NPL, WPG, true>), dim3(grid), dim3(64 * WPG), 0, s, A);
  else
    hipLaunchKernelGGL((batch4_kernel<CAP, NPL, WPG, false>), dim3(grid), dim3(64 * WPG), 0, s, A);
  return hipGetLastError();
}

template <int CAP, int NPL, int WPG>
static int occupancy_t() {
  int nb = 0, nf = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch4_kernel<CAP, NPL, WPG, false>, 64 * WPG, 0) !=
          hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nf, batch4_kernel<CAP, NPL, WPG, true>, 64 * WPG, 0) !=
          hipSuccess)
    return 0;
  return nb < nf ? nb : nf;  // the grid suits either kernel
}

// Supported (stack capacity, nodes per round, waves per workgroup) triples.
#define BATCH_CONFIGS(X)                                                                         \
  X(128, 16, 1) X(256, 16, 1) X(512, 16, 1) X(1024, 16, 1) X(2048, 16, 1) X(256, 64, 1)          \
  X(512, 64, 1) X(640, 64, 1) X(672, 64, 1) X(768, 64, 1) X(1024, 64, 1) X(2048, 64, 1)    \
  X(512, 64, 2) X(1024, 64, 2) X(2048, 64, 2)                                                     \
  X(512, 64, 4) X(1024, 64, 4) X(2048, 64, 4)

hipError_t launch_batch4(int lds_cap, int npl, int wpg, int grid, const BatchArgs& A, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
#define X(C, N, G) \
  if (lds_cap == C && npl == N && wpg == G) return launch_batch_t<C, N, G>(grid, A, s);
  BATCH_CONFIGS(X)
#undef X
  return hipErrorInvalidValue;
}

int batch4_max_blocks_per_cu(int lds_cap, int npl, int wpg) {
#define X(C, N, G) \
  if (lds_cap == C && npl == N && wpg == G) return occupancy_t<C, N, G>();
  BATCH_CONFIGS(X)
#undef X
  return 0;
}

}  // namespace bpida
