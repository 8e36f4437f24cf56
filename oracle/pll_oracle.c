/*
 * Plain sequential CPU oracle for Pruned Landmark Labeling.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the GPU
 * library never does and shares no code, header or table with it.
 *
 * Source: T. Akiba, Y. Iwata, Y. Yoshida, "Fast Exact Shortest-Path Distance
 * Queries on Large Networks by Pruned Landmark Labeling", SIGMOD 2013.
 *
 * What it computes, step by step, in the paper's order:
 *   O0  validation; vertex ranks from the order; adjacency in rank space with
 *       every row sorted (Section 4.5.1, "Sorting Labels": hubs are stored
 *       as ranks, so labels come out sorted).
 *   O1  greedy choice of bit-parallel roots r and neighbour sets S_r
 *       (Section 5.4, last paragraph).
 *   O2  one bit-parallel BFS per root (Algorithm 3 / Section 5.2).
 *   O3  pruned BFSs from every vertex in rank order (Algorithms 1 and 2),
 *       pruning on bit-parallel labels first and normal labels second
 *       (Section 5.4), normal-label prune test with the root array T and
 *       per-BFS resets of only the touched entries (Section 4.5.1).
 *   O4  labels stored with a sentinel after the last entry (Section 4.5.2).
 *   O5  queries: bit-parallel part (Section 5.3) plus the merge join over
 *       sorted labels (Section 3.3).
 *
 * Readings of points the paper leaves open (each one also fixed on the GPU
 * side, so both compute the same bytes):
 *   - Algorithm 1 appends the visit distance of u and expands the neighbours
 *     of u (the printed pseudo-code has typos there; the prose of Section 4.2
 *     says what is meant).
 *   - A vertex is marked when it is enqueued, so it is tested at most once per
 *     BFS.
 *   - "Infinity" in the 8-bit arrays is 255.  A distance of 255 or more cannot
 *     be stored: a bit-parallel BFS that reaches distance 255, or a pruned BFS
 *     that would label a vertex at distance 255, fails with ORC_E_RANGE.
 *   - Bit-parallel roots: the lowest-rank vertex not yet used as a root or as
 *     a neighbour; S_r: its first (up to) 64 unused neighbours in ascending
 *     rank; bit j of a set stands for the (j+1)-th chosen neighbour.  When no
 *     vertex is left the slot is empty (distance 255, empty sets).
 *   - Pruned BFSs are not run from vertices used by the bit-parallel phase
 *     (their bit-parallel self-distance is 0, so they would prune themselves).
 *   - Self-loops are rejected (one would put v into its own S^0 set).
 *   - S^0 is stored as Section 5.1 defines it (disjoint from S^{-1}); the
 *     printed Algorithm 3 alone can leave S^{-1} members in it.
 *   - Query answers are min(QUERY, 255); 255 means unreachable.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_INF 255u
#define ORC_SENTINEL 0xFFFFFFFFu
#define ORC_BPW 64 /* bits per bit-parallel word (b in Section 5) */

enum { ORC_OK = 0, ORC_E_INVAL = -1, ORC_E_NOMEM = -2, ORC_E_RANGE = -3 };

/* counters, in this order */
enum {
  C_N = 0,          /* vertices */
  C_TBP,            /* bit-parallel slots requested */
  C_ENTRIES,        /* normal label entries (no sentinels) */
  C_BP_USED,        /* |B|: roots plus chosen neighbours */
  C_ROOTS,          /* pruned BFSs run */
  C_VISITED,        /* sum over roots of vertices dequeued */
  C_LABELED,        /* sum over roots of vertices labeled (== C_ENTRIES) */
  C_EDGES,          /* sum over roots of adjacency entries scanned */
  C_BP_PRUNED,      /* vertices pruned by the bit-parallel test */
  C_NORMAL_TESTS,   /* vertices that reached the normal-label test */
  C_LABEL_SCANNED,  /* label entries read by normal-label tests */
  C_ROOT_STAGED,    /* label entries of the roots written into T */
  C_BP_REACHED,     /* sum over slots of vertices reached */
  C_BP_EDGES,       /* sum over slots of adjacency entries scanned */
  C_BP_E0,          /* sum over slots of |E0| */
  C_BP_E1,          /* sum over slots of |E1| */
  C_MAX_DIST,       /* largest finite distance stored */
  ORC_NCOUNTERS
};

typedef struct {
  uint32_t *hub; /* hub ranks, ascending, then ORC_SENTINEL */
  uint8_t *dist;
  int64_t len;   /* entries, not counting the sentinel */
  int64_t cap;
} orc_label;

typedef struct orc_index {
  int32_t n, t_bp;
  int32_t *rank;      /* rank[v] for input id v */
  orc_label *lab;     /* indexed by rank */
  uint8_t *bp_d;      /* [n][t_bp], indexed by rank */
  uint64_t *bp_m1;    /* S^{-1} sets */
  uint64_t *bp_0;     /* S^{0} sets */
  int32_t *bp_root;   /* [t_bp]: rank of the root, -1 for an empty slot */
  int32_t *bp_nsel;   /* [t_bp]: |S_r| */
  int32_t *bp_sel;    /* [t_bp][64]: ranks of S_r in bit order */
  int32_t *root_visited; /* [n]: vertices dequeued by the pruned BFS of rank k */
  int32_t *root_labeled; /* [n]: vertices it labeled (Figure 4 quantities) */
  int64_t cnt[ORC_NCOUNTERS];
} orc_index;

/* ------------------------------------------------------------------------ */

static void label_free_all(orc_label *lab, int32_t n) {
  if (!lab) return;
  for (int32_t i = 0; i < n; i++) {
    free(lab[i].hub);
    free(lab[i].dist);
  }
  free(lab);
}

void orc_free(orc_index *x) {
  if (!x) return;
  free(x->rank);
  label_free_all(x->lab, x->n);
  free(x->bp_d);
  free(x->bp_m1);
  free(x->bp_0);
  free(x->bp_root);
  free(x->bp_nsel);
  free(x->bp_sel);
  free(x->root_visited);
  free(x->root_labeled);
  free(x);
}

/* append (h, d) and keep the sentinel after the last entry */
static int label_push(orc_label *L, uint32_t h, uint8_t d) {
  if (L->len + 2 > L->cap) {
    int64_t nc = L->cap ? 2 * L->cap : 4;
    uint32_t *nh = (uint32_t *)realloc(L->hub, (size_t)nc * sizeof(uint32_t));
    if (!nh) return ORC_E_NOMEM;
    L->hub = nh;
    uint8_t *nd = (uint8_t *)realloc(L->dist, (size_t)nc);
    if (!nd) return ORC_E_NOMEM;
    L->dist = nd;
    L->cap = nc;
  }
  L->hub[L->len] = h;
  L->dist[L->len] = d;
  L->len++;
  L->hub[L->len] = ORC_SENTINEL;
  L->dist[L->len] = (uint8_t)ORC_INF;
  return ORC_OK;
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* Distance via one bit-parallel slot (Section 5.3).  Returns an int that may
 * exceed 254; the caller takes the minimum. */
static int bp_slot_dist(uint8_t ds, uint64_t m1s, uint64_t m0s,
                        uint8_t dt, uint64_t m1t, uint64_t m0t) {
  int td = (int)ds + (int)dt;
  if (m1s & m1t)
    td -= 2;
  else if ((m0s & m1t) | (m1s & m0t))
    td -= 1;
  return td;
}

/* ------------------------------------------------------------------------ */
/* O0: validation and rank-space adjacency                                  */

static int validate(int32_t n, const int32_t *row_ptr, const int32_t *col,
                    const int32_t *order, int32_t t_bp) {
  if (n < 0 || t_bp < 0) return ORC_E_INVAL;
  if (n == 0) return ORC_OK;
  if (!row_ptr || !order) return ORC_E_INVAL;
  if (row_ptr[0] != 0) return ORC_E_INVAL;
  for (int32_t v = 0; v < n; v++)
    if (row_ptr[v + 1] < row_ptr[v]) return ORC_E_INVAL;
  if (row_ptr[n] > 0 && !col) return ORC_E_INVAL;
  for (int32_t v = 0; v < n; v++)
    for (int32_t j = row_ptr[v]; j < row_ptr[v + 1]; j++) {
      if (col[j] < 0 || col[j] >= n) return ORC_E_INVAL;
      if (col[j] == v) return ORC_E_INVAL; /* self-loop */
    }
  char *seen = (char *)calloc((size_t)n, 1);
  if (!seen) return ORC_E_NOMEM;
  int bad = 0;
  for (int32_t i = 0; i < n && !bad; i++) {
    if (order[i] < 0 || order[i] >= n || seen[order[i]]) bad = 1;
    else seen[order[i]] = 1;
  }
  free(seen);
  return bad ? ORC_E_INVAL : ORC_OK;
}

/* every edge (v,w) must have its reverse (w,v): binary search in sorted rows */
static int check_symmetric(int32_t n, const int64_t *off, const int32_t *adj) {
  for (int32_t v = 0; v < n; v++)
    for (int64_t j = off[v]; j < off[v + 1]; j++) {
      int32_t w = adj[j];
      int64_t lo = off[w], hi = off[w + 1];
      while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (adj[mid] < v) lo = mid + 1;
        else hi = mid;
      }
      if (lo == off[w + 1] || adj[lo] != v) return ORC_E_INVAL;
    }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* O1: greedy bit-parallel root and neighbour choice (Section 5.4)          */

static void choose_bp_roots(orc_index *x, const int64_t *off, const int32_t *adj,
                            char *used) {
  int32_t n = x->n, r = 0;
  for (int32_t i = 0; i < x->t_bp; i++) {
    while (r < n && used[r]) r++;
    x->bp_nsel[i] = 0;
    if (r == n) {
      x->bp_root[i] = -1;
      continue;
    }
    x->bp_root[i] = r;
    used[r] = 1;
    for (int64_t j = off[r]; j < off[r + 1] && x->bp_nsel[i] < ORC_BPW; j++) {
      int32_t w = adj[j];
      if (!used[w]) {
        used[w] = 1;
        x->bp_sel[(int64_t)i * ORC_BPW + x->bp_nsel[i]] = w;
        x->bp_nsel[i]++;
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* O2: bit-parallel BFS from r and S_r (Algorithm 3)                        */

static int bp_bfs(orc_index *x, int32_t slot, const int64_t *off, const int32_t *adj,
                  uint8_t *P, uint64_t *s1, uint64_t *s0, int32_t *q0, int32_t *q1,
                  int32_t *e0, int32_t *e1) {
  int32_t n = x->n, t = x->t_bp;
  int32_t r = x->bp_root[slot];
  if (r < 0) { /* empty slot */
    for (int32_t v = 0; v < n; v++) {
      x->bp_d[(int64_t)v * t + slot] = (uint8_t)ORC_INF;
      x->bp_m1[(int64_t)v * t + slot] = 0;
      x->bp_0[(int64_t)v * t + slot] = 0;
    }
    return ORC_OK;
  }
  for (int32_t v = 0; v < n; v++) {
    P[v] = (uint8_t)ORC_INF;
    s1[v] = 0;
    s0[v] = 0;
  }
  int64_t n0 = 0, n1 = 0;
  P[r] = 0;
  q0[n0++] = r;
  for (int32_t j = 0; j < x->bp_nsel[slot]; j++) {
    int32_t v = x->bp_sel[(int64_t)slot * ORC_BPW + j];
    P[v] = 1;
    s1[v] = (uint64_t)1 << j;
    q1[n1++] = v;
  }
  int64_t reached = 1 + n1;
  while (n0 > 0) {
    int64_t ne0 = 0, ne1 = 0;
    for (int64_t qi = 0; qi < n0; qi++) {
      int32_t v = q0[qi];
      int nextd = (int)P[v] + 1;
      for (int64_t j = off[v]; j < off[v + 1]; j++) {
        int32_t u = adj[j];
        x->cnt[C_BP_EDGES]++;
        if (P[u] == ORC_INF || (int)P[u] == nextd) {
          e1[2 * ne1] = v;
          e1[2 * ne1 + 1] = u;
          ne1++;
          if (P[u] == ORC_INF) {
            if (nextd >= (int)ORC_INF) return ORC_E_RANGE;
            P[u] = (uint8_t)nextd;
            q1[n1++] = u;
            reached++;
          }
        } else if (P[u] == P[v]) {
          e0[2 * ne0] = v;
          e0[2 * ne0 + 1] = u;
          ne0++;
        }
      }
    }
    /* all same-level edges first, then all edges to the next level */
    for (int64_t i = 0; i < ne0; i++) s0[e0[2 * i + 1]] |= s1[e0[2 * i]];
    for (int64_t i = 0; i < ne1; i++) {
      s1[e1[2 * i + 1]] |= s1[e1[2 * i]];
      s0[e1[2 * i + 1]] |= s0[e1[2 * i]];
    }
    x->cnt[C_BP_E0] += ne0;
    x->cnt[C_BP_E1] += ne1;
    /* Q0 <- Q1, Q1 <- empty */
    memcpy(q0, q1, (size_t)n1 * sizeof(int32_t));
    n0 = n1;
    n1 = 0;
  }
  x->cnt[C_BP_REACHED] += reached;
  /* The dynamic programme above can leave in S^0(v) members w of S^{-1}(v)
   * (w reaches v one step early on one parent and on time on another).
   * Section 5.1 defines S^{-1}, S^0 and S^{+1} as a partition of S_r, so
   * S^0 is reduced to its definition here.  No query answer depends on it:
   * such a bit only matters where S^{-1} and S^{-1} already intersect. */
  for (int32_t v = 0; v < n; v++) {
    x->bp_d[(int64_t)v * t + slot] = P[v];
    x->bp_m1[(int64_t)v * t + slot] = s1[v];
    x->bp_0[(int64_t)v * t + slot] = s0[v] & ~s1[v];
    if (P[v] != ORC_INF && P[v] > x->cnt[C_MAX_DIST]) x->cnt[C_MAX_DIST] = P[v];
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* O3: pruned BFSs (Algorithms 1 and 2)                                     */

/* Is u pruned when visited at distance d from root k?  Bit-parallel labels
 * first, then the normal label of u against T (Section 4.5.1, "Querying"). */
static int pruned_at(orc_index *x, int32_t k, int32_t u, int d, const uint8_t *T) {
  int32_t t = x->t_bp;
  const uint8_t *dk = x->bp_d + (int64_t)k * t, *du = x->bp_d + (int64_t)u * t;
  const uint64_t *m1k = x->bp_m1 + (int64_t)k * t, *m1u = x->bp_m1 + (int64_t)u * t;
  const uint64_t *m0k = x->bp_0 + (int64_t)k * t, *m0u = x->bp_0 + (int64_t)u * t;
  for (int32_t i = 0; i < t; i++) {
    if (dk[i] == ORC_INF || du[i] == ORC_INF) continue;
    if (bp_slot_dist(dk[i], m1k[i], m0k[i], du[i], m1u[i], m0u[i]) <= d) {
      x->cnt[C_BP_PRUNED]++;
      return 1;
    }
  }
  x->cnt[C_NORMAL_TESTS]++;
  const orc_label *L = &x->lab[u];
  x->cnt[C_LABEL_SCANNED] += L->len;
  int best = 1 << 20;
  for (int64_t i = 0; i < L->len; i++) {
    uint8_t th = T[L->hub[i]];
    if (th == ORC_INF) continue;
    int v = (int)L->dist[i] + (int)th;
    if (v < best) best = v;
  }
  return best <= d;
}

static int pruned_phase(orc_index *x, const int64_t *off, const int32_t *adj,
                        const char *used) {
  int32_t n = x->n;
  uint8_t *P = (uint8_t *)malloc((size_t)n);
  uint8_t *T = (uint8_t *)malloc((size_t)n);
  int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int rc = ORC_OK;
  if (!P || !T || !queue) {
    rc = ORC_E_NOMEM;
    goto done;
  }
  memset(P, (int)ORC_INF, (size_t)n); /* once, before the first BFS */
  memset(T, (int)ORC_INF, (size_t)n);
  for (int32_t k = 0; k < n && rc == ORC_OK; k++) {
    if (used[k]) continue;
    x->cnt[C_ROOTS]++;
    int64_t vis0 = x->cnt[C_VISITED], lab0 = x->cnt[C_LABELED];
    orc_label *Lk = &x->lab[k];
    for (int64_t i = 0; i < Lk->len; i++) T[Lk->hub[i]] = Lk->dist[i];
    x->cnt[C_ROOT_STAGED] += Lk->len;
    int64_t qh = 0, qt = 0;
    queue[qt++] = k;
    P[k] = 0;
    while (qh < qt) {
      int32_t u = queue[qh++];
      int d = P[u];
      x->cnt[C_VISITED]++;
      if (pruned_at(x, k, u, d, T)) continue;
      rc = label_push(&x->lab[u], (uint32_t)k, (uint8_t)d);
      if (rc != ORC_OK) break;
      x->cnt[C_LABELED]++;
      if (d > x->cnt[C_MAX_DIST]) x->cnt[C_MAX_DIST] = d;
      for (int64_t j = off[u]; j < off[u + 1]; j++) {
        int32_t w = adj[j];
        x->cnt[C_EDGES]++;
        if (P[w] != ORC_INF) continue;
        if (d + 1 >= (int)ORC_INF) {
          /* w sits at distance 255: fine only if it would be pruned */
          if (!pruned_at(x, k, w, d + 1, T)) {
            rc = ORC_E_RANGE;
            break;
          }
          continue;
        }
        P[w] = (uint8_t)(d + 1);
        queue[qt++] = w;
      }
      if (rc != ORC_OK) break;
    }
    /* reset only what this BFS touched (Section 4.5.1, "Initialization") */
    for (int64_t i = 0; i < qt; i++) P[queue[i]] = (uint8_t)ORC_INF;
    for (int64_t i = 0; i < Lk->len; i++) T[Lk->hub[i]] = (uint8_t)ORC_INF;
    x->root_visited[k] = (int32_t)(x->cnt[C_VISITED] - vis0);
    x->root_labeled[k] = (int32_t)(x->cnt[C_LABELED] - lab0);
  }
done:
  free(P);
  free(T);
  free(queue);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Public entry points                                                       */

/* Build the index.  flags bit 0: check that the graph is symmetric. */
int orc_build(int32_t n, const int32_t *row_ptr, const int32_t *col,
              const int32_t *order, int32_t t_bp, uint32_t flags, orc_index **out) {
  if (!out) return ORC_E_INVAL;
  *out = NULL;
  int rc = validate(n, row_ptr, col, order, t_bp);
  if (rc != ORC_OK) return rc;

  orc_index *x = (orc_index *)calloc(1, sizeof(orc_index));
  if (!x) return ORC_E_NOMEM;
  x->n = n;
  x->t_bp = t_bp;
  int64_t nn = n > 0 ? n : 1, tt = t_bp > 0 ? t_bp : 1;
  int64_t nnz = n > 0 ? row_ptr[n] : 0;
  x->rank = (int32_t *)malloc((size_t)nn * sizeof(int32_t));
  x->lab = (orc_label *)calloc((size_t)nn, sizeof(orc_label));
  x->bp_d = (uint8_t *)malloc((size_t)(nn * tt));
  x->bp_m1 = (uint64_t *)malloc((size_t)(nn * tt) * sizeof(uint64_t));
  x->bp_0 = (uint64_t *)malloc((size_t)(nn * tt) * sizeof(uint64_t));
  x->bp_root = (int32_t *)malloc((size_t)tt * sizeof(int32_t));
  x->bp_nsel = (int32_t *)malloc((size_t)tt * sizeof(int32_t));
  x->bp_sel = (int32_t *)malloc((size_t)(tt * ORC_BPW) * sizeof(int32_t));
  x->root_visited = (int32_t *)calloc((size_t)nn, sizeof(int32_t));
  x->root_labeled = (int32_t *)calloc((size_t)nn, sizeof(int32_t));
  int64_t *off = (int64_t *)malloc((size_t)(nn + 1) * sizeof(int64_t));
  int32_t *adj = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
  char *used = (char *)calloc((size_t)nn, 1);
  uint8_t *P = (uint8_t *)malloc((size_t)nn);
  uint64_t *s1 = (uint64_t *)malloc((size_t)nn * sizeof(uint64_t));
  uint64_t *s0 = (uint64_t *)malloc((size_t)nn * sizeof(uint64_t));
  int32_t *q0 = (int32_t *)malloc((size_t)nn * sizeof(int32_t));
  int32_t *q1 = (int32_t *)malloc((size_t)nn * sizeof(int32_t));
  int32_t *e0 = (int32_t *)malloc((size_t)(2 * (nnz > 0 ? nnz : 1)) * sizeof(int32_t));
  int32_t *e1 = (int32_t *)malloc((size_t)(2 * (nnz > 0 ? nnz : 1)) * sizeof(int32_t));
  if (!x->rank || !x->lab || !x->bp_d || !x->bp_m1 || !x->bp_0 || !x->bp_root ||
      !x->bp_nsel || !x->bp_sel || !x->root_visited || !x->root_labeled || !off || !adj || !used || !P || !s1 || !s0 || !q0 ||
      !q1 || !e0 || !e1) {
    rc = ORC_E_NOMEM;
    goto fail;
  }

  /* O0: ranks and the rank-space adjacency with sorted rows */
  for (int32_t i = 0; i < n; i++) x->rank[order[i]] = i;
  off[0] = 0;
  for (int32_t r = 0; r < n; r++) {
    int32_t v = order[r];
    int64_t deg = row_ptr[v + 1] - row_ptr[v];
    for (int64_t j = 0; j < deg; j++) adj[off[r] + j] = x->rank[col[row_ptr[v] + j]];
    qsort(adj + off[r], (size_t)deg, sizeof(int32_t), cmp_i32);
    off[r + 1] = off[r] + deg;
  }
  if (flags & 1u) {
    rc = check_symmetric(n, off, adj);
    if (rc != ORC_OK) goto fail;
  }

  /* O1 + O2 */
  choose_bp_roots(x, off, adj, used);
  for (int32_t i = 0; i < n; i++) x->cnt[C_BP_USED] += used[i] ? 1 : 0;
  for (int32_t s = 0; s < t_bp; s++) {
    rc = bp_bfs(x, s, off, adj, P, s1, s0, q0, q1, e0, e1);
    if (rc != ORC_OK) goto fail;
  }

  /* O3 + O4 */
  rc = pruned_phase(x, off, adj, used);
  if (rc != ORC_OK) goto fail;
  for (int32_t v = 0; v < n; v++) x->cnt[C_ENTRIES] += x->lab[v].len;
  /* a vertex with an empty label still gets its sentinel */
  for (int32_t v = 0; v < n; v++) {
    if (x->lab[v].cap == 0) {
      x->lab[v].hub = (uint32_t *)malloc(sizeof(uint32_t));
      x->lab[v].dist = (uint8_t *)malloc(1);
      if (!x->lab[v].hub || !x->lab[v].dist) {
        rc = ORC_E_NOMEM;
        goto fail;
      }
      x->lab[v].cap = 1;
      x->lab[v].hub[0] = ORC_SENTINEL;
      x->lab[v].dist[0] = (uint8_t)ORC_INF;
    }
  }
  x->cnt[C_N] = n;
  x->cnt[C_TBP] = t_bp;

  free(off); free(adj); free(used); free(P); free(s1); free(s0);
  free(q0); free(q1); free(e0); free(e1);
  *out = x;
  return ORC_OK;

fail:
  free(off); free(adj); free(used); free(P); free(s1); free(s0);
  free(q0); free(q1); free(e0); free(e1);
  orc_free(x);
  return rc;
}

/* O5: one query by ids.  Bit-parallel part (Section 5.3) and the merge join
 * of the two sorted labels that stops at the shared sentinel (Sections 3.3
 * and 4.5.2), each returned as an int (INF when it finds nothing). */
static void query_parts(const orc_index *x, int32_t s, int32_t t, int *bp_part,
                        int *normal_part) {
  int32_t rs = x->rank[s], rt = x->rank[t], tb = x->t_bp;
  int best = (int)ORC_INF;
  for (int32_t i = 0; i < tb; i++) {
    uint8_t ds = x->bp_d[(int64_t)rs * tb + i], dt = x->bp_d[(int64_t)rt * tb + i];
    if (ds == ORC_INF || dt == ORC_INF) continue;
    int v = bp_slot_dist(ds, x->bp_m1[(int64_t)rs * tb + i], x->bp_0[(int64_t)rs * tb + i],
                         dt, x->bp_m1[(int64_t)rt * tb + i], x->bp_0[(int64_t)rt * tb + i]);
    if (v < best) best = v;
  }
  *bp_part = best;
  best = (int)ORC_INF;
  const orc_label *A = &x->lab[rs], *B = &x->lab[rt];
  int64_t i = 0, j = 0;
  for (;;) {
    uint32_t ha = A->hub[i], hb = B->hub[j];
    if (ha == hb) {
      if (ha == ORC_SENTINEL) break;
      int v = (int)A->dist[i] + (int)B->dist[j];
      if (v < best) best = v;
      i++;
      j++;
    } else if (ha < hb) {
      i++;
    } else {
      j++;
    }
  }
  *normal_part = best;
}

static uint8_t query_one(const orc_index *x, int32_t s, int32_t t) {
  int a, b;
  query_parts(x, s, t, &a, &b);
  int best = a < b ? a : b;
  return (uint8_t)(best < (int)ORC_INF ? best : (int)ORC_INF);
}

/* Both parts of each query, unclamped (for pinning each part on its own). */
int orc_query_parts(const orc_index *x, const int32_t *pairs, int64_t q, int32_t *bp_part,
                    int32_t *normal_part) {
  if (!x || q < 0 || (q > 0 && (!pairs || !bp_part || !normal_part))) return ORC_E_INVAL;
  for (int64_t i = 0; i < 2 * q; i++)
    if (pairs[i] < 0 || pairs[i] >= x->n) return ORC_E_INVAL;
  for (int64_t i = 0; i < q; i++) {
    int a, b;
    query_parts(x, pairs[2 * i], pairs[2 * i + 1], &a, &b);
    bp_part[i] = a;
    normal_part[i] = b;
  }
  return ORC_OK;
}

int orc_query(const orc_index *x, const int32_t *pairs, int64_t q, uint8_t *out) {
  if (!x || q < 0 || (q > 0 && (!pairs || !out))) return ORC_E_INVAL;
  for (int64_t i = 0; i < 2 * q; i++)
    if (pairs[i] < 0 || pairs[i] >= x->n) return ORC_E_INVAL;
  for (int64_t i = 0; i < q; i++) out[i] = query_one(x, pairs[2 * i], pairs[2 * i + 1]);
  return ORC_OK;
}

int32_t orc_ncounters(void) { return ORC_NCOUNTERS; }

int orc_counters(const orc_index *x, int64_t *c, int32_t nc) {
  if (!x || !c) return ORC_E_INVAL;
  for (int32_t i = 0; i < nc && i < ORC_NCOUNTERS; i++) c[i] = x->cnt[i];
  return ORC_OK;
}

int64_t orc_num_entries(const orc_index *x) { return x ? x->cnt[C_ENTRIES] : -1; }

/* Export in rank order, without sentinels.  Any output pointer may be NULL. */
int orc_export(const orc_index *x, int64_t *off, uint32_t *hub, uint8_t *dist,
               uint8_t *bp_d, uint64_t *bp_m1, uint64_t *bp_0, int32_t *rank,
               int32_t *bp_root, int32_t *bp_nsel, int32_t *bp_sel) {
  if (!x) return ORC_E_INVAL;
  int64_t e = 0;
  for (int32_t v = 0; v < x->n; v++) {
    if (off) off[v] = e;
    const orc_label *L = &x->lab[v];
    if (hub) memcpy(hub + e, L->hub, (size_t)L->len * sizeof(uint32_t));
    if (dist) memcpy(dist + e, L->dist, (size_t)L->len);
    e += L->len;
  }
  if (off) off[x->n] = e;
  int64_t nb = (int64_t)x->n * x->t_bp;
  if (bp_d && nb) memcpy(bp_d, x->bp_d, (size_t)nb);
  if (bp_m1 && nb) memcpy(bp_m1, x->bp_m1, (size_t)nb * sizeof(uint64_t));
  if (bp_0 && nb) memcpy(bp_0, x->bp_0, (size_t)nb * sizeof(uint64_t));
  if (rank && x->n) memcpy(rank, x->rank, (size_t)x->n * sizeof(int32_t));
  if (bp_root && x->t_bp) memcpy(bp_root, x->bp_root, (size_t)x->t_bp * sizeof(int32_t));
  if (bp_nsel && x->t_bp) memcpy(bp_nsel, x->bp_nsel, (size_t)x->t_bp * sizeof(int32_t));
  if (bp_sel && x->t_bp)
    memcpy(bp_sel, x->bp_sel, (size_t)x->t_bp * ORC_BPW * sizeof(int32_t));
  return ORC_OK;
}

/* Per-root work of the pruned phase, indexed by rank (0 for vertices that
 * were bit-parallel roots or neighbours). */
int orc_root_counts(const orc_index *x, int32_t *visited, int32_t *labeled) {
  if (!x) return ORC_E_INVAL;
  if (visited && x->n) memcpy(visited, x->root_visited, (size_t)x->n * sizeof(int32_t));
  if (labeled && x->n) memcpy(labeled, x->root_labeled, (size_t)x->n * sizeof(int32_t));
  return ORC_OK;
}
