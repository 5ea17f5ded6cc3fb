/*
 * ida_oracle.c -- sequential CPU IDA* used as the correctness oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or calls
 * this file; only the test suite, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header or table with the GPU library.
 *
 * What it computes (Horie & Fukunaga, "Block-Parallel IDA* for GPUs"):
 *   IDA* (Sec. 1; the per-iteration f-limited DFS of Alg. 2, function DFS,
 *   without load balancing) on the sliding-tile puzzle with the Manhattan
 *   distance heuristic (Sec. 3).  The block-parallel search of Alg. 1 must
 *   expand exactly the same node set in every f-limited iteration (Sec. 6.1:
 *   parallel and sequential IDA* agree on non-final iterations, and the
 *   all-optimal-solutions mode removes the difference in the final one).
 *
 * Readings taken where the paper is silent (all stated in the design notes):
 *   - goal: tile p at position p, blank (0) at position 0;
 *   - moves are blank moves U, L, R, D (0..3), the inverse of a is 3-a, unit
 *     cost (the cost(a) term of Alg. 1);
 *   - "applicable" = blank stays on the board and a does not undo the move
 *     that generated the node (parent pruning); the start has no parent move;
 *   - Manhattan distance excludes the blank;
 *   - the first limit is h(start) (DecideFirstLimit);
 *   - goal test on expansion (Alg. 1 and Alg. 2 test the popped node);
 *   - the final iteration runs to completion (Sec. 6.1, all optimal
 *     solutions), so its count is unique; a first-solution mode instead
 *     returns at the first goal expanded, as Alg. 1 is printed (the count of
 *     the final iteration is then that of this sequential U, L, R, D order);
 *   - "expanded" = every node the DFS visits, start and goal nodes included.
 *
 * Output per instance: the optimal length, the sequence of f-limits used and
 * the number of nodes expanded under each of them, and optionally one
 * optimal path (Alg. 1's BPDFS returns the goal "and its parents"): the moves
 * from the start to the first goal the DFS expands.  The final limit is the
 * optimal length and every pruned subtree holds no goal within it, so the
 * depth-first order U, L, R, D makes that path the lexicographically
 * smallest optimal move sequence (unique, whichever final-limit mode runs).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_ITERS 64
#define ORACLE_MAX_PATH 256 /* moves per path (f-limits stay below 256) */
#define ORACLE_MAX_WIDTH 5
#define ORACLE_MAX_CELLS (ORACLE_MAX_WIDTH * ORACLE_MAX_WIDTH)

enum {
  ORACLE_OK = 0,
  ORACLE_EINVAL = -1,      /* bad arguments or not a permutation          */
  ORACLE_EUNSOLVABLE = -2, /* wrong permutation parity                     */
  ORACLE_ELIMIT = -3,      /* more than ORACLE_MAX_ITERS f-limits, or the  */
                           /* caller's limit cap was passed                */
  ORACLE_EHCHECK = -4,     /* check mode: incremental h != full h          */
};

/* ---- the heuristic (Sec. 3: Manhattan distance) ----------------------- */

/* Distance of `tile` standing at `pos` from its goal position `tile`. */
static int md_tile(int w, int tile, int pos) {
  int dr = pos / w - tile / w;
  int dc = pos % w - tile % w;
  return (dr < 0 ? -dr : dr) + (dc < 0 ? -dc : dc);
}

/* Sum over all non-blank tiles. */
static int md_full(int w, const uint8_t *s) {
  int h = 0;
  for (int p = 0; p < w * w; ++p)
    if (s[p] != 0) h += md_tile(w, s[p], p);
  return h;
}

static int is_goal(int w, const uint8_t *s) {
  for (int p = 0; p < w * w; ++p)
    if (s[p] != p) return 0;
  return 1;
}

/* ---- the f-limited depth-first search ---------------------------------- */

typedef struct {
  int w;
  int limit;        /* current f-limit                                     */
  uint64_t count;   /* nodes expanded in this iteration                    */
  int found;        /* a goal was expanded in this iteration               */
  int fmin;         /* smallest f of a pruned child (next f-limit)         */
  int check;        /* recompute h from scratch at every node              */
  int first;        /* first-solution mode: stop at the first goal         */
  int hbad;         /* check mode found a mismatch                         */
  uint8_t s[ORACLE_MAX_CELLS];
  uint8_t moves[ORACLE_MAX_PATH]; /* moves from the start to the current node */
  uint8_t *path;    /* null, or where the first goal's moves are copied    */
  int path_len;     /* moves copied to path (-1: none yet)                 */
} search_t;

/* Blank at `blank`, path cost g, heuristic h, `last` = move that produced
 * this node or -1 at the start. */
static void dfs(search_t *S, int blank, int g, int h, int last) {
  const int w = S->w;
  S->count++;
  if (S->check && md_full(w, S->s) != h) S->hbad = 1;
  if (h == 0 && is_goal(w, S->s)) {
    if (!S->found && S->path && g <= ORACLE_MAX_PATH) {
      /* the first goal of this iteration: its path is the current moves */
      memcpy(S->path, S->moves, (size_t)g);
      S->path_len = g;
    }
    S->found = 1;
    if (S->first) return; /* first solution: the search ends here */
  }                       /* all solutions: continue */
  const int r = blank / w, c = blank % w;
  for (int a = 0; a < 4; ++a) {
    if (S->first && S->found) return;
    if (last >= 0 && a == 3 - last) continue; /* undoes the parent move */
    int n;
    if (a == 0) { if (r == 0) continue; n = blank - w; }
    else if (a == 1) { if (c == 0) continue; n = blank - 1; }
    else if (a == 2) { if (c == w - 1) continue; n = blank + 1; }
    else { if (r == w - 1) continue; n = blank + w; }
    const int t = S->s[n];
    /* tile t slides from n into the blank's cell */
    const int hc = h - md_tile(w, t, n) + md_tile(w, t, blank);
    const int f = g + 1 + hc; /* unit move cost */
    if (f > S->limit) {
      if (f < S->fmin) S->fmin = f;
      continue;
    }
    S->s[blank] = (uint8_t)t;
    S->s[n] = 0;
    if (g < ORACLE_MAX_PATH) S->moves[g] = (uint8_t)a;
    dfs(S, n, g + 1, hc, a);
    S->s[n] = (uint8_t)t;
    S->s[blank] = 0;
  }
}

/* Permutation parity (number of inversions mod 2) over all w*w entries,
 * blank included. */
static int perm_parity(int nn, const uint8_t *s) {
  int inv = 0;
  for (int i = 0; i < nn; ++i)
    for (int j = i + 1; j < nn; ++j)
      if (s[i] > s[j]) inv ^= 1;
  return inv;
}

/* Solvable iff permutation parity == parity of the blank's taxicab distance
 * from position 0 (each move is one transposition and moves the blank one
 * cell, so both parities flip together; the converse is checked
 * exhaustively on 3x3 by the tests). */
int oracle_check_state(const uint8_t *s, int32_t w) {
  if (w < 2 || w > ORACLE_MAX_WIDTH || !s) return ORACLE_EINVAL;
  const int nn = w * w;
  int seen[ORACLE_MAX_CELLS] = {0};
  int blank = -1;
  for (int p = 0; p < nn; ++p) {
    if (s[p] >= nn || seen[s[p]]) return ORACLE_EINVAL;
    seen[s[p]] = 1;
    if (s[p] == 0) blank = p;
  }
  const int bd = blank / w + blank % w;
  if (perm_parity(nn, s) != (bd & 1)) return ORACLE_EUNSOLVABLE;
  return ORACLE_OK;
}

int32_t oracle_manhattan(const uint8_t *s, int32_t w) { return md_full(w, s); }

/* Solve one instance.  limits[j], nodes[j] for j < *niter; path (null, or
 * ORACLE_MAX_PATH bytes): the moves of the first goal expanded, 0xFF after. */
static int solve_one(const uint8_t *start, int w, int check, int first, int max_limit,
                     int32_t *len, int32_t *limits, uint64_t *nodes, int32_t *niter,
                     uint8_t *path) {
  *len = -1;
  *niter = 0;
  for (int j = 0; j < ORACLE_MAX_ITERS; ++j) { limits[j] = 0; nodes[j] = 0; }
  if (path) memset(path, 0xFF, ORACLE_MAX_PATH);
  int rc = oracle_check_state(start, w);
  if (rc != ORACLE_OK) return rc;
  search_t S;
  memset(&S, 0, sizeof S);
  S.w = w;
  S.check = check;
  S.first = first;
  S.path = path;
  S.path_len = -1;
  memcpy(S.s, start, (size_t)(w * w));
  int blank = 0;
  while (start[blank] != 0) ++blank;
  const int h0 = md_full(w, start);
  int L = h0; /* DecideFirstLimit */
  for (int j = 0; j < ORACLE_MAX_ITERS; ++j) {
    if (max_limit >= 0 && L > max_limit) return ORACLE_ELIMIT;
    S.limit = L;
    S.count = 0;
    S.found = 0;
    S.fmin = 1 << 30;
    dfs(&S, blank, 0, h0, -1);
    limits[j] = L;
    nodes[j] = S.count;
    *niter = j + 1;
    if (S.hbad) return ORACLE_EHCHECK;
    if (S.found) { *len = L; return ORACLE_OK; }
    L = S.fmin;
  }
  return ORACLE_ELIMIT;
}

/* ---- batch driver: instances spread over host threads ------------------ */

typedef struct {
  const uint8_t *states;
  int n, w, check, first, max_limit;
  int32_t *len, *limits, *niter, *status;
  uint64_t *nodes;
  uint8_t *paths; /* null, or n * ORACLE_MAX_PATH */
  int next; /* shared cursor, taken under the lock */
  pthread_mutex_t mu;
} batch_t;

static void *worker(void *arg) {
  batch_t *B = (batch_t *)arg;
  for (;;) {
    pthread_mutex_lock(&B->mu);
    int i = B->next++;
    pthread_mutex_unlock(&B->mu);
    if (i >= B->n) break;
    const int nn = B->w * B->w;
    B->status[i] = solve_one(B->states + (size_t)i * nn, B->w, B->check, B->first, B->max_limit,
                             &B->len[i],
                             B->limits + (size_t)i * ORACLE_MAX_ITERS,
                             B->nodes + (size_t)i * ORACLE_MAX_ITERS, &B->niter[i],
                             B->paths ? B->paths + (size_t)i * ORACLE_MAX_PATH : NULL);
  }
  return NULL;
}

/*
 * states     host, n * width*width bytes, row-major, 0 = blank
 * out_len    host, n: optimal length, -1 on error
 * out_limits host, n * 64: f-limit of iteration j (0 past the last)
 * out_nodes  host, n * 64: nodes expanded in iteration j (0 past the last)
 * out_niter  host, n: iterations run
 * out_status host, n: ORACLE_* code per instance
 * nthreads   worker threads (<= 0: one)
 * check      nonzero: recompute h from scratch at every node
 * max_limit  stop with ORACLE_ELIMIT before an f-limit above this (< 0: none)
 * first      nonzero: the final iteration returns at its first goal
 * out_path   host, n * 256 or null: the moves (U, L, R, D = 0..3) of the
 *            first goal expanded, 0xFF past the length
 * Returns ORACLE_OK if every instance solved, else the first failing code.
 */
int oracle_solve_paths(const uint8_t *states, int32_t n, int32_t width, int32_t *out_len,
                       int32_t *out_limits, uint64_t *out_nodes, int32_t *out_niter,
                       int32_t *out_status, int32_t nthreads, int32_t check, int32_t max_limit,
                       int32_t first, uint8_t *out_path) {
  if (!states || !out_len || !out_limits || !out_nodes || !out_niter || !out_status || n < 0 ||
      width < 2 || width > ORACLE_MAX_WIDTH)
    return ORACLE_EINVAL;
  batch_t B;
  B.states = states; B.n = n; B.w = width; B.check = check; B.first = first;
  B.max_limit = max_limit;
  B.paths = out_path;
  B.len = out_len; B.limits = out_limits; B.nodes = out_nodes; B.niter = out_niter;
  B.status = out_status; B.next = 0;
  pthread_mutex_init(&B.mu, NULL);
  if (nthreads < 1) nthreads = 1;
  if (nthreads > n) nthreads = n > 0 ? n : 1;
  pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
  if (!th) return ORACLE_EINVAL;
  for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, worker, &B);
  worker(&B);
  for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(th);
  pthread_mutex_destroy(&B.mu);
  for (int i = 0; i < n; ++i)
    if (out_status[i] != ORACLE_OK) return out_status[i];
  return ORACLE_OK;
}

int oracle_solve(const uint8_t *states, int32_t n, int32_t width, int32_t *out_len,
                 int32_t *out_limits, uint64_t *out_nodes, int32_t *out_niter,
                 int32_t *out_status, int32_t nthreads, int32_t check, int32_t max_limit,
                 int32_t first) {
  return oracle_solve_paths(states, n, width, out_len, out_limits, out_nodes, out_niter,
                            out_status, nthreads, check, max_limit, first, NULL);
}
