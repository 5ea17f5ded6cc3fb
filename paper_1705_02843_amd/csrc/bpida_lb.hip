// bpida_lb.hip -- BPIDA*'s static load balancing for the plain path.
//
// Sec. 5: BPIDA* re-balances its root set between f-limited iterations the
// way PStaticLB does (Sec. 4, UpdateRootSet), with the work under a root
// estimated by the number of repetitions of BPDFS's loop it took in the
// previous iteration.  A root whose load exceeds the average load is split:
// its subtree is expanded until at least load / average nodes are
// generated, and those nodes replace it.
//
// Here the expansion is breadth-first and without duplicate elimination (the
// same tree as the root split, so every count stays exact): a heavy root is
// replaced by all nodes of its subtree at the first depth that holds at least
// ceil(load / average) of them (at most kLbMaxPieces; at most kLbMaxLevels
// levels).  The root and the nodes above that depth become interior nodes:
// their f goes into the instance's f-histogram, so they are counted at every
// later limit that admits them, and a goal among them is recorded like a goal
// inside the split tree.  Roots are then handed to workgroups through the
// search kernel's cursor (dynamic assignment) rather than by load sums.
#include "bpida_internal.h"

namespace bpida {

namespace {

constexpr int kLbMaxPieces = 64;
constexpr int kLbMaxLevels = 10;
constexpr int kDelta4[4] = {-4, -1, 1, 4};

// Number of non-backtracking blank walks of length j from (blank, forbidden
// move) for j = 1, 2, ...: the first j whose count reaches k, with that count
// (or kLbMaxLevels and its count).
__device__ void split_depth(int blank, int forbid, int k, int* level, int* count) {
  uint32_t cur[16][5], nxt[16][5];
  for (int c = 0; c < 16; ++c)
    for (int f = 0; f < 5; ++f) cur[c][f] = 0;
  cur[blank][forbid] = 1;
  for (int j = 1; j <= kLbMaxLevels; ++j) {
    for (int c = 0; c < 16; ++c)
      for (int f = 0; f < 5; ++f) nxt[c][f] = 0;
    uint32_t total = 0;
    for (int c = 0; c < 16; ++c)
      for (int f = 0; f < 5; ++f) {
        const uint32_t v = cur[c][f];
        if (!v) continue;
        for (int a = 0; a < 4; ++a) {
          if (a == f || !((kMoveMask4 >> (4 * c + a)) & 1ull)) continue;
          nxt[c + kDelta4[a]][3 - a] += v;
          total += v;
        }
      }
    for (int c = 0; c < 16; ++c)
      for (int f = 0; f < 5; ++f) cur[c][f] = nxt[c][f];
    if ((int)total >= k || j == kLbMaxLevels) {
      *level = j;
      *count = (int)total;
      return;
    }
  }
}

// Sum and number of the loads of the roots searched at `limit` (f <= limit).
__global__ __launch_bounds__(1024) void lb_average_kernel(const Node* __restrict__ roots,
                                                          const uint32_t* __restrict__ load,
                                                          int nroots, int limit,
                                                          uint64_t* __restrict__ out) {
  __shared__ uint64_t s_sum[1024];
  __shared__ uint32_t s_cnt[1024];
  uint64_t sum = 0;
  uint32_t cnt = 0;
  for (int r = threadIdx.x; r < nroots; r += blockDim.x)
    if ((int)roots[r].f <= limit) {
      sum += load[r];
      cnt += 1;
    }
  s_sum[threadIdx.x] = sum;
  s_cnt[threadIdx.x] = cnt;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s_sum[threadIdx.x] += s_sum[threadIdx.x + o];
      s_cnt[threadIdx.x] += s_cnt[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s_sum[0];
    out[1] = s_cnt[0];
  }
}

// Per root: the split depth (0 = kept as it is) and the number of roots it
// becomes.
__global__ void lb_count_kernel(const Node* __restrict__ roots, const uint32_t* __restrict__ load,
                                int nroots, int limit, const uint64_t* __restrict__ avg_in,
                                int32_t* __restrict__ level, int32_t* __restrict__ count) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nroots) return;
  const uint64_t n = avg_in[1];
  const uint64_t avg = n ? (avg_in[0] + n - 1) / n : 0;
  const Node R = roots[r];
  int lv = 0, c = 1;
  if ((int)R.f <= limit && avg > 0 && load[r] > avg) {
    const uint64_t want = (load[r] + avg - 1) / avg;
    const int k = (int)(want < (uint64_t)kLbMaxPieces ? want : (uint64_t)kLbMaxPieces);
    split_depth((int)(R.meta & 31u), (int)((R.meta >> 5) & 7u), k, &lv, &c);
  }
  level[r] = lv;
  count[r] = c;
}

// Exclusive prefix sum of count[0..n) into off, and the total, by one
// workgroup of 1024 threads (each scans a contiguous segment).
__global__ __launch_bounds__(1024) void lb_scan_kernel(const int32_t* __restrict__ count, int n,
                                                       int64_t* __restrict__ off,
                                                       int64_t* __restrict__ total) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int seg = (n + 1023) / 1024;
  const int b = t * seg, e = min(n, b + seg);
  int64_t s = 0;
  for (int k = b; k < e; ++k) s += count[k];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int64_t acc = 0;
    for (int k = 0; k < 1024; ++k) {
      const int64_t v = part[k];
      part[k] = acc;
      acc += v;
    }
    *total = acc;
  }
  __syncthreads();
  int64_t acc = part[t];
  for (int k = b; k < e; ++k) {
    off[k] = acc;
    acc += count[k];
  }
}

// Per root: copy it, or enumerate its subtree to its split depth (depth
// first, moves in U, L, R, D order): the nodes at that depth become roots,
// the ones above it interior nodes.
__global__ void lb_emit_kernel(const Node* __restrict__ roots, int nroots,
                               const int32_t* __restrict__ level, const int32_t* __restrict__ count,
                               const int64_t* __restrict__ off, Node* __restrict__ out, uint32_t* __restrict__ hist,
                               int32_t* __restrict__ goal_g, int32_t* __restrict__ err) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nroots) return;
  const Node R = roots[r];
  const int lv = level[r];
  Node* dst = out + off[r];
  if (lv == 0) {
    dst[0] = R;
    return;
  }
  uint64_t s[kLbMaxLevels + 1];
  int blank[kLbMaxLevels + 1], forbid[kLbMaxLevels + 1], g[kLbMaxLevels + 1],
      h[kLbMaxLevels + 1], next[kLbMaxLevels + 1];
  s[0] = R.tiles;
  blank[0] = (int)(R.meta & 31u);
  forbid[0] = (int)((R.meta >> 5) & 7u);
  g[0] = (int)((R.meta >> 8) & 255u);
  h[0] = (int)((R.meta >> 16) & 255u);
  next[0] = 0;
  int d = 0;
  int64_t w = 0;
  // the root itself is now an interior node
  atomicAdd(&hist[min(g[0] + h[0], kHistBins - 1)], 1u);
  if (h[0] == 0 && s[0] == kGoal4) atomicMin(goal_g, g[0]);
  while (d >= 0) {
    const int a = next[d];
    if (a == 4) {
      --d;
      continue;
    }
    next[d] = a + 1;
    const int b = blank[d];
    if (a == forbid[d] || !((kMoveMask4 >> (4 * b + a)) & 1ull)) continue;
    const int n = b + kDelta4[a];
    const uint32_t t = (uint32_t)(s[d] >> (4 * n)) & 15u;
    const bool vert = a == 0 || a == 3;
    const uint32_t ct = vert ? t >> 2 : t & 3u;
    const uint32_t cn = vert ? (uint32_t)n >> 2 : (uint32_t)n & 3u;
    const int grows = (int)((kDhTable4 >> (16 * a + 4 * ct + cn)) & 1ull);
    const uint64_t cs = s[d] + ((uint64_t)t << (4 * b)) - ((uint64_t)t << (4 * n));
    const int cg = g[d] + 1, ch = h[d] + (grows ? 1 : -1);
    if (d + 1 == lv) {
      Node c;
      c.tiles = cs;
      c.meta = node_meta(n, 3 - a, cg, ch);
      c.f = (uint32_t)(cg + ch);
      if (w < count[r]) dst[w] = c;  // never past the planned slots
      ++w;
    } else {
      ++d;
      s[d] = cs;
      blank[d] = n;
      forbid[d] = 3 - a;
      g[d] = cg;
      h[d] = ch;
      next[d] = 0;
      atomicAdd(&hist[min(cg + ch, kHistBins - 1)], 1u);
      if (ch == 0 && cs == kGoal4) atomicMin(goal_g, cg);
    }
  }
  if (w != count[r]) atomicOr(err, 1);  // the enumeration must match the plan
}

}  // namespace

hipError_t launch_lb_plan(const Node* d_roots, const uint32_t* d_load, int nroots, int limit,
                          uint64_t* d_avg, int32_t* d_level, int32_t* d_count, int64_t* d_off,
                          int64_t* d_total, hipStream_t s) {
  if (nroots <= 0) return hipSuccess;
  hipLaunchKernelGGL(lb_average_kernel, dim3(1), dim3(1024), 0, s, d_roots, d_load, nroots, limit,
                     d_avg);
  hipLaunchKernelGGL(lb_count_kernel, dim3((nroots + 255) / 256), dim3(256), 0, s, d_roots, d_load,
                     nroots, limit, d_avg, d_level, d_count);
  hipLaunchKernelGGL(lb_scan_kernel, dim3(1), dim3(1024), 0, s, d_count, nroots, d_off, d_total);
  return hipGetLastError();
}

hipError_t launch_lb_emit(const Node* d_roots, int nroots, const int32_t* d_level,
                          const int32_t* d_count, const int64_t* d_off, Node* d_out,
                          uint32_t* d_hist, int32_t* d_goal_g, int32_t* d_err, hipStream_t s) {
  if (nroots <= 0) return hipSuccess;
  hipLaunchKernelGGL(lb_emit_kernel, dim3((nroots + 255) / 256), dim3(256), 0, s, d_roots, nroots,
                     d_level, d_count, d_off, d_out, d_hist, d_goal_g, d_err);
  return hipGetLastError();
}

}  // namespace bpida
