// bpida_path.hip -- one optimal path per instance (Alg. 1's BPDFS returns
// the goal "and its parents").
//
// The search keeps no ancestry on its stacks (entries move between
// workgroups through spills and donations), so the path is rebuilt after
// the solve, one move per step, by exact-limit probes: with k moves left from
// the current state s (k = opt(s)), every legal move a that does not undo
// the previous one gives a probe "does s.a reach the goal in exactly k - 1
// moves?", which is the batched search at the single f-limit k - 1 with the
// move back to s forbidden at the probe's root, stopping at its first goal.
// The step takes the first move, in U, L, R, D order, whose probe finds a
// goal: the path is the lexicographically smallest optimal move sequence,
// which is unique.  These kernels build the probes of a step and apply its
// outcome; the probes of all instances of a step run in one batched launch.
#include <stdint.h>

#include "bpida_internal.h"

namespace bpida {

// Per instance: current state = start, moves left = optimal length (or -1),
// no previous move, empty path.
__global__ void path_init_kernel(const uint8_t* __restrict__ states, const int32_t* __restrict__ len,
                                 int n, int nn, uint8_t* __restrict__ cur, int32_t* __restrict__ left,
                                 uint8_t* __restrict__ prev, uint8_t* __restrict__ path) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < (int64_t)n * nn) cur[k] = states[k];
  if (k < (int64_t)n * kMaxPath) path[k] = 0xFF;
  if (k < n) {
    left[k] = len[k];
    prev[k] = 4;
  }
}

// Probe 4i + a = the current state of instance i after blank move a, with
// limit left - 1 and move 3 - a forbidden at its root; a probe that does not
// apply (instance done, move off the board or undoing the previous move) is
// an all-zero board, which the ingest rejects before any search.
__global__ void path_probe_kernel(const uint8_t* __restrict__ cur, const int32_t* __restrict__ left,
                                  const uint8_t* __restrict__ prev, int n, int w,
                                  uint8_t* __restrict__ probe, int32_t* __restrict__ probe_limit,
                                  uint8_t* __restrict__ probe_forbid) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= 4 * n) return;
  const int i = j >> 2, a = j & 3, nn = w * w;
  const uint8_t* s = cur + (size_t)i * nn;
  uint8_t* out = probe + (size_t)j * nn;
  int blank = 0;
  for (int p = 0; p < nn; ++p)
    if (s[p] == 0) blank = p;
  const int r = blank / w, c = blank % w;
  const bool on_board = a == 0 ? r > 0 : a == 1 ? c > 0 : a == 2 ? c < w - 1 : r < w - 1;
  const bool use = left[i] > 0 && on_board && a != 3 - (int)prev[i];
  for (int p = 0; p < nn; ++p) out[p] = use ? s[p] : 0;
  if (use) {
    const int nb = blank + (a == 0 ? -w : a == 1 ? -1 : a == 2 ? 1 : w);
    out[blank] = s[nb];
    out[nb] = 0;
  }
  probe_limit[j] = use ? left[i] - 1 : 0;
  probe_forbid[j] = (uint8_t)(3 - a);
}

// Applies a step: the first move whose probe found a goal (status 1) is
// appended to the path and its probe becomes the current state.  An
// instance with moves left and no such move sets *err (an inconsistency:
// a state at distance k always has a neighbour at distance k - 1).
__global__ void path_select_kernel(const uint8_t* __restrict__ probe,
                                   const int32_t* __restrict__ status, const int32_t* __restrict__ len,
                                   int n, int nn, uint8_t* __restrict__ cur, int32_t* __restrict__ left,
                                   uint8_t* __restrict__ prev, uint8_t* __restrict__ path,
                                   int32_t* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || left[i] <= 0) return;
  int pick = -1;
  for (int a = 3; a >= 0; --a)
    if (status[4 * i + a] == 1) pick = a;
  if (pick < 0) {
    atomicOr(err, 1);
    left[i] = 0;
    return;
  }
  const int step = len[i] - left[i];
  if (step >= 0 && step < kMaxPath) path[(size_t)i * kMaxPath + step] = (uint8_t)pick;
  const uint8_t* src = probe + (size_t)(4 * i + pick) * nn;
  for (int p = 0; p < nn; ++p) cur[(size_t)i * nn + p] = src[p];
  left[i] -= 1;
  prev[i] = (uint8_t)pick;
}

hipError_t launch_path_init(const uint8_t* d_states, const int32_t* d_len, int n, int nn,
                            uint8_t* d_cur, int32_t* d_left, uint8_t* d_prev, uint8_t* d_path,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t work = (int64_t)n * std::max(nn, kMaxPath);
  hipLaunchKernelGGL(path_init_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, d_states,
                     d_len, n, nn, d_cur, d_left, d_prev, d_path);
  return hipGetLastError();
}

hipError_t launch_path_probe(const uint8_t* d_cur, const int32_t* d_left, const uint8_t* d_prev, int n,
                             int w, uint8_t* d_probe, int32_t* d_probe_limit, uint8_t* d_probe_forbid,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(path_probe_kernel, dim3((4 * n + 255) / 256), dim3(256), 0, s, d_cur, d_left,
                     d_prev, n, w, d_probe, d_probe_limit, d_probe_forbid);
  return hipGetLastError();
}

hipError_t launch_path_select(const uint8_t* d_probe, const int32_t* d_status, const int32_t* d_len,
                              int n, int nn, uint8_t* d_cur, int32_t* d_left, uint8_t* d_prev,
                              uint8_t* d_path, int32_t* d_err, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(path_select_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d_probe, d_status,
                     d_len, n, nn, d_cur, d_left, d_prev, d_path, d_err);
  return hipGetLastError();
}

}  // namespace bpida
