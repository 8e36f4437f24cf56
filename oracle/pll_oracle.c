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
 *   O6  shortest paths (Section 6, "Shortest-Path Queries"): every label
 *       entry (h, d) of v also keeps the parent of v in the pruned BFS tree
 *       of h, and a path is restored by ascending those trees.
 *   O7  directed graphs (Section 6, "Directed Graphs"): labels L_OUT(v) =
 *       {(u, d(v,u))} and L_IN(v) = {(u, d(u,v))}; from every vertex in rank
 *       order one pruned BFS along the edges (it labels L_IN of what it
 *       reaches, pruning with L_OUT(root) and L_IN(u)) and one against them
 *       (labels L_OUT, pruning with L_OUT(u) and L_IN(root)); d(s,t) is the
 *       merge of L_OUT(s) and L_IN(t).  Entries keep parents as in O6, so
 *       paths s -> t are restored through the best hub of that merge.
 *   O8  weighted graphs (Section 6, "Weighted Graphs"): the pruned BFS of
 *       Algorithm 1 becomes a pruned Dijkstra search (a binary heap, a vertex
 *       is tested and, if not pruned, labeled and relaxed when it is settled);
 *       no bit-parallel labels; distances are 32-bit.  Also for digraphs,
 *       with the two searches of O7.  Entries keep the parent in the search
 *       tree of the hub (chosen as in O6), so shortest paths come back as in
 *       O6.
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
 *   - The parent kept with (h, d) in L(v) is v's parent in the pruned BFS
 *     tree of h (Section 6; the printed text says "of u" where the tree is
 *     rooted at u: the parent of v is meant).  Every vertex that the BFS
 *     from h labeled at d - 1 and that has an edge to v is such a parent;
 *     the lowest-ranked one is kept, so the choice is unique (the root
 *     itself for its own entry).  For a digraph the edge runs in the
 *     search's direction; for weighted graphs the parent p is labeled at
 *     d - w(p, v).
 *   - Bit-parallel labels keep no tree (Section 6 treats normal labels only).
 *     When a bit-parallel slot gives the distance, the path is walked by
 *     scanning neighbours in ascending rank: towards the root r with the
 *     distances of the slot, towards a chosen neighbour w with w in S^{-1}
 *     (one step closer to w per level) or S^{0} (same distance as to r).
 */
#define _POSIX_C_SOURCE 199309L
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

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
  uint32_t *par; /* parent (rank) of this vertex in the BFS tree of the hub */
  int64_t len;   /* entries, not counting the sentinel */
  int64_t cap;
} orc_label;

typedef struct orc_index {
  int32_t n, t_bp;
  int32_t *rank;      /* rank[v] for input id v */
  orc_label *lab;     /* indexed by rank (L_OUT for a directed graph) */
  orc_label *lab_in;  /* L_IN of a directed graph, else NULL */
  uint8_t *bp_d;      /* [n][t_bp], indexed by rank */
  uint64_t *bp_m1;    /* S^{-1} sets */
  uint64_t *bp_0;     /* S^{0} sets */
  int32_t *bp_root;   /* [t_bp]: rank of the root, -1 for an empty slot */
  int32_t *bp_nsel;   /* [t_bp]: |S_r| */
  int32_t *bp_sel;    /* [t_bp][64]: ranks of S_r in bit order */
  int32_t *root_visited; /* [n]: vertices dequeued by the pruned BFS of rank k */
  int32_t *root_labeled; /* [n]: vertices it labeled (Figure 4 quantities) */
  int32_t *ord;          /* [n]: input id of rank r */
  /* wall-clock timing of the build (reporting only; no effect on labels) */
  int64_t ns_bp, ns_pruned;   /* bit-parallel phase, pruned phase */
  int32_t ck_step, nck;       /* checkpoint every ck_step roots, nck taken */
  int64_t *ck_ns;             /* [nck]: pruned-phase ns elapsed before rank i*ck_step */
  int64_t *off;          /* [n+1] rank-space adjacency (kept for paths) */
  int32_t *adj;
  int64_t cnt[ORC_NCOUNTERS];
} orc_index;

/* ------------------------------------------------------------------------ */

static void label_free_all(orc_label *lab, int32_t n) {
  if (!lab) return;
  for (int32_t i = 0; i < n; i++) {
    free(lab[i].hub);
    free(lab[i].dist);
    free(lab[i].par);
  }
  free(lab);
}

void orc_free(orc_index *x) {
  if (!x) return;
  free(x->rank);
  label_free_all(x->lab, x->n);
  label_free_all(x->lab_in, x->n);
  free(x->bp_d);
  free(x->bp_m1);
  free(x->bp_0);
  free(x->bp_root);
  free(x->bp_nsel);
  free(x->bp_sel);
  free(x->root_visited);
  free(x->root_labeled);
  free(x->ord);
  free(x->ck_ns);
  free(x->off);
  free(x->adj);
  free(x);
}

/* append (h, d, parent) and keep the sentinel after the last entry */
static int label_push(orc_label *L, uint32_t h, uint8_t d, uint32_t par) {
  if (L->len + 2 > L->cap) {
    int64_t nc = L->cap ? 2 * L->cap : 4;
    uint32_t *nh = (uint32_t *)realloc(L->hub, (size_t)nc * sizeof(uint32_t));
    if (!nh) return ORC_E_NOMEM;
    L->hub = nh;
    uint8_t *nd = (uint8_t *)realloc(L->dist, (size_t)nc);
    if (!nd) return ORC_E_NOMEM;
    L->dist = nd;
    uint32_t *np = (uint32_t *)realloc(L->par, (size_t)nc * sizeof(uint32_t));
    if (!np) return ORC_E_NOMEM;
    L->par = np;
    L->cap = nc;
  }
  L->hub[L->len] = h;
  L->dist[L->len] = d;
  L->par[L->len] = par;
  L->len++;
  L->hub[L->len] = ORC_SENTINEL;
  L->dist[L->len] = (uint8_t)ORC_INF;
  L->par[L->len] = ORC_SENTINEL;
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

static int64_t now_ns(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (int64_t)ts.tv_sec * 1000000000 + ts.tv_nsec;
}

/* Parent kept with (k, d) in L(u), d >= 1: the lowest-ranked p in row u of
 * (poff, padj) -- the vertices with an edge p -> u in the search -- whose
 * label holds (k, d - 1).  Roots run in rank order, so while the search
 * from k runs, an entry of k is the newest one of a label, and every vertex
 * at distance d - 1 has been labeled or pruned before u is taken. */
static uint32_t tree_parent(const orc_label *lab, const int64_t *poff, const int32_t *padj,
                            int32_t u, int32_t k, int d) {
  uint32_t best = ORC_SENTINEL;
  for (int64_t j = poff[u]; j < poff[u + 1]; j++) {
    const orc_label *L = &lab[padj[j]];
    if (L->len > 0 && L->hub[L->len - 1] == (uint32_t)k && L->dist[L->len - 1] == d - 1 &&
        (uint32_t)padj[j] < best)
      best = (uint32_t)padj[j];
  }
  return best;
}

/* root_limit: pruned BFSs run from ranks 0..root_limit-1 only. */
static int pruned_phase(orc_index *x, const int64_t *off, const int32_t *adj,
                        const char *used, int32_t root_limit) {
  int32_t n = x->n;
  /* visit distances in 16 bits, so that a vertex can be reached (and
   * tested) at distance 255; only labeling it there is out of range */
  uint16_t *P = (uint16_t *)malloc((size_t)n * sizeof(uint16_t));
  uint8_t *T = (uint8_t *)malloc((size_t)n);
  int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int rc = ORC_OK;
  if (!P || !T || !queue) {
    rc = ORC_E_NOMEM;
    goto done;
  }
  memset(P, 0xFF, (size_t)n * sizeof(uint16_t)); /* once, before the first BFS */
  memset(T, (int)ORC_INF, (size_t)n);
  int64_t t0 = now_ns();
  for (int32_t k = 0; k < root_limit && rc == ORC_OK; k++) {
    if (k % x->ck_step == 0) x->ck_ns[x->nck++] = now_ns() - t0;
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
      if (d >= (int)ORC_INF) { /* (k, 255) cannot be stored */
        rc = ORC_E_RANGE;
        break;
      }
      uint32_t par = d == 0 ? (uint32_t)k : tree_parent(x->lab, off, adj, u, k, d);
      rc = label_push(&x->lab[u], (uint32_t)k, (uint8_t)d, par);
      if (rc != ORC_OK) break;
      x->cnt[C_LABELED]++;
      if (d > x->cnt[C_MAX_DIST]) x->cnt[C_MAX_DIST] = d;
      for (int64_t j = off[u]; j < off[u + 1]; j++) {
        int32_t w = adj[j];
        x->cnt[C_EDGES]++;
        if (P[w] != 0xFFFF) continue;
        P[w] = (uint16_t)(d + 1);
        queue[qt++] = w;
      }
    }
    /* reset only what this BFS touched (Section 4.5.1, "Initialization") */
    for (int64_t i = 0; i < qt; i++) P[queue[i]] = 0xFFFF;
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

/* Build the index.  flags bit 0: check that the graph is symmetric.
 * root_limit (0..n): the pruned phase stops before the root of that rank.
 * By Theorem 4.1 the labels are then exactly the entries of the full
 * labels whose hub ranks below root_limit; root_limit = n is the full
 * build (orc_build). */
int orc_build_prefix(int32_t n, const int32_t *row_ptr, const int32_t *col,
                     const int32_t *order, int32_t t_bp, uint32_t flags, int32_t root_limit,
                     orc_index **out) {
  if (!out) return ORC_E_INVAL;
  *out = NULL;
  int rc = validate(n, row_ptr, col, order, t_bp);
  if (rc != ORC_OK) return rc;
  if (root_limit < 0 || root_limit > n) return ORC_E_INVAL;

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
  x->ck_step = (int32_t)((nn + 1023) / 1024);
  x->ck_ns = (int64_t *)calloc(1025, sizeof(int64_t));
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
      !x->bp_nsel || !x->bp_sel || !x->root_visited || !x->root_labeled || !x->ck_ns || !off || !adj || !used || !P || !s1 || !s0 || !q0 ||
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
  int64_t tb0 = now_ns();
  choose_bp_roots(x, off, adj, used);
  for (int32_t i = 0; i < n; i++) x->cnt[C_BP_USED] += used[i] ? 1 : 0;
  for (int32_t s = 0; s < t_bp; s++) {
    rc = bp_bfs(x, s, off, adj, P, s1, s0, q0, q1, e0, e1);
    if (rc != ORC_OK) goto fail;
  }
  int64_t tb1 = now_ns();
  x->ns_bp = tb1 - tb0;

  /* O3 + O4 */
  rc = pruned_phase(x, off, adj, used, root_limit);
  if (rc != ORC_OK) goto fail;
  x->ns_pruned = now_ns() - tb1;
  for (int32_t v = 0; v < n; v++) x->cnt[C_ENTRIES] += x->lab[v].len;
  /* a vertex with an empty label still gets its sentinel */
  for (int32_t v = 0; v < n; v++) {
    if (x->lab[v].cap == 0) {
      x->lab[v].hub = (uint32_t *)malloc(sizeof(uint32_t));
      x->lab[v].dist = (uint8_t *)malloc(1);
      x->lab[v].par = (uint32_t *)malloc(sizeof(uint32_t));
      if (!x->lab[v].hub || !x->lab[v].dist || !x->lab[v].par) {
        rc = ORC_E_NOMEM;
        goto fail;
      }
      x->lab[v].cap = 1;
      x->lab[v].hub[0] = ORC_SENTINEL;
      x->lab[v].dist[0] = (uint8_t)ORC_INF;
      x->lab[v].par[0] = ORC_SENTINEL;
    }
  }
  x->cnt[C_N] = n;
  x->cnt[C_TBP] = t_bp;

  /* keep the rank-space graph and the rank -> id map for path queries */
  x->ord = (int32_t *)malloc((size_t)nn * sizeof(int32_t));
  if (!x->ord) {
    rc = ORC_E_NOMEM;
    goto fail;
  }
  for (int32_t i = 0; i < n; i++) x->ord[i] = order[i];
  x->off = off;
  x->adj = adj;
  off = NULL;
  adj = NULL;

  free(used); free(P); free(s1); free(s0);
  free(q0); free(q1); free(e0); free(e1);
  *out = x;
  return ORC_OK;

fail:
  free(off); free(adj); free(used); free(P); free(s1); free(s0);
  free(q0); free(q1); free(e0); free(e1);
  orc_free(x);
  return rc;
}

int orc_build(int32_t n, const int32_t *row_ptr, const int32_t *col,
              const int32_t *order, int32_t t_bp, uint32_t flags, orc_index **out) {
  return orc_build_prefix(n, row_ptr, col, order, t_bp, flags, n, out);
}

/* Wall-clock times of a build (ns): bit-parallel phase, pruned phase, and
 * the pruned-phase time elapsed before every ck_step-th root.  Returns the
 * number of checkpoints (at most max_ck are copied). */
int32_t orc_times(const orc_index *x, int64_t *bp_ns, int64_t *pruned_ns, int32_t *ck_step,
                  int64_t *ck_ns, int32_t max_ck) {
  if (!x) return ORC_E_INVAL;
  if (bp_ns) *bp_ns = x->ns_bp;
  if (pruned_ns) *pruned_ns = x->ns_pruned;
  if (ck_step) *ck_step = x->ck_step;
  for (int32_t i = 0; ck_ns && i < x->nck && i < max_ck; i++) ck_ns[i] = x->ck_ns[i];
  return x->nck;
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
  const orc_label *A = &x->lab[rs], *B = x->lab_in ? &x->lab_in[rt] : &x->lab[rt];
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

/* ------------------------------------------------------------------------ */
/* O6: shortest paths (Section 6)                                            */

/* entry of hub h in L(v) (labels are sorted by hub rank), or -1 */
static int64_t find_hub(const orc_label *L, uint32_t h) {
  int64_t lo = 0, hi = L->len;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (L->hub[mid] < h) lo = mid + 1;
    else hi = mid;
  }
  return (lo < L->len && L->hub[lo] == h) ? lo : -1;
}

/* One step of a walk on bit-parallel slot i from c: the first neighbour x
 * (ascending rank) with d(x) == dc + ddx and, when bit != 0, that bit in
 * S^{-1}(x) (sel = 1) or S^{0}(x) (sel = 0).  -1 if there is none. */
static int32_t bp_step(const orc_index *x, int32_t c, int32_t i, int ddx, uint64_t bit, int sel) {
  int32_t tb = x->t_bp;
  int dc = x->bp_d[(int64_t)c * tb + i];
  for (int64_t j = x->off[c]; j < x->off[c + 1]; j++) {
    int32_t y = x->adj[j];
    if ((int)x->bp_d[(int64_t)y * tb + i] != dc + ddx) continue;
    if (!bit) return y;
    uint64_t m = sel ? x->bp_m1[(int64_t)y * tb + i] : x->bp_0[(int64_t)y * tb + i];
    if (m & bit) return y;
  }
  return -1;
}

/* Walk from c on slot i and write the visited ranks at out[pos], out[pos +
 * dir], ...  mode 0: towards the root (d decreases to 0); mode 1: towards
 * neighbour w (bit) with w in S^{-1}(c) (d decreases to 1, ends at w);
 * mode 2: towards w with w in S^{0}(c) (a step to a vertex one level closer
 * keeps w in S^{0}; a step within the level puts w in S^{-1}, mode 1 from
 * there).  Returns the number of vertices written, or -1. */
static int bp_walk(const orc_index *x, int32_t c, int32_t i, uint64_t bit, int mode,
                   int32_t *out, int pos, int dir) {
  int32_t tb = x->t_bp;
  int nw = 0;
  for (;;) {
    out[pos] = c;
    pos += dir;
    nw++;
    int dc = x->bp_d[(int64_t)c * tb + i];
    if (mode == 0) {
      if (dc == 0) return nw;
      c = bp_step(x, c, i, -1, 0, 0);
    } else if (mode == 1) {
      if (dc == 1) return nw; /* c is w: S^{-1}(w) = {w} at level 1 */
      c = bp_step(x, c, i, -1, bit, 1);
    } else {
      int32_t y = bp_step(x, c, i, -1, bit, 0);
      if (y < 0) {
        y = bp_step(x, c, i, 0, bit, 1);
        if (y >= 0) mode = 1;
      }
      c = y;
    }
    if (c < 0) return -1;
  }
}

/* Shortest path from s to t (input ids) into out[0..D] as input ids.
 * *len = D+1, 0 if t is unreachable (or 255 or more away), -(D+1) if
 * maxlen < D+1 (nothing written).  Returns ORC_OK, or ORC_E_RANGE if a walk
 * fails (it cannot on a correct index). */
static int path_one(const orc_index *x, int32_t s, int32_t t, int32_t maxlen, int32_t *out,
                    int32_t *len) {
  int32_t rs = x->rank[s], rt = x->rank[t], tb = x->t_bp;
  if (rs == rt) {
    if (maxlen < 1) {
      *len = -1;
      return ORC_OK;
    }
    out[0] = s;
    *len = 1;
    return ORC_OK;
  }
  /* normal part: best hub by the merge join (first one on ties) */
  const orc_label *A = &x->lab[rs], *B = &x->lab[rt];
  int best_n = 1 << 20, ia = -1, ib = -1;
  for (int64_t i = 0, j = 0;;) {
    uint32_t ha = A->hub[i], hb = B->hub[j];
    if (ha == hb) {
      if (ha == ORC_SENTINEL) break;
      int v = (int)A->dist[i] + (int)B->dist[j];
      if (v < best_n) {
        best_n = v;
        ia = (int)i;
        ib = (int)j;
      }
      i++;
      j++;
    } else if (ha < hb) {
      i++;
    } else {
      j++;
    }
  }
  /* bit-parallel part: best slot (lowest on ties) and its witness */
  int best_b = 1 << 20, bi = -1, kind = 0;
  uint64_t wbit = 0;
  for (int32_t i = 0; i < tb; i++) {
    uint8_t ds = x->bp_d[(int64_t)rs * tb + i], dt = x->bp_d[(int64_t)rt * tb + i];
    if (ds == ORC_INF || dt == ORC_INF) continue;
    uint64_t m1s = x->bp_m1[(int64_t)rs * tb + i], m0s = x->bp_0[(int64_t)rs * tb + i];
    uint64_t m1t = x->bp_m1[(int64_t)rt * tb + i], m0t = x->bp_0[(int64_t)rt * tb + i];
    int v = bp_slot_dist(ds, m1s, m0s, dt, m1t, m0t);
    if (v < best_b) {
      best_b = v;
      bi = i;
      kind = (int)ds + (int)dt - v;
      uint64_t m = kind == 2 ? (m1s & m1t) : kind == 1 ? ((m1s & m0t) ? (m1s & m0t) : (m0s & m1t)) : 0;
      wbit = m & (~m + 1); /* lowest set bit */
    }
  }
  int D = best_n <= best_b ? best_n : best_b;
  *len = 0;
  if (D >= (int)ORC_INF) return ORC_OK;
  if (maxlen < D + 1) {
    *len = -(D + 1);
    return ORC_OK;
  }
  int32_t *tmp = out; /* ranks first, mapped to ids at the end */
  if (best_n <= best_b) {
    uint32_t h = A->hub[ia];
    int ds = A->dist[ia], dt = B->dist[ib];
    int32_t c = rs;
    for (int k = 0; k <= ds; k++) {
      tmp[k] = c;
      if (k < ds) {
        int64_t e = find_hub(&x->lab[c], h);
        if (e < 0) return ORC_E_RANGE;
        c = (int32_t)x->lab[c].par[e];
        if ((uint32_t)c >= (uint32_t)x->n) return ORC_E_RANGE;
      }
    }
    c = rt;
    for (int k = 0; k < dt; k++) {
      tmp[D - k] = c;
      int64_t e = find_hub(&x->lab[c], h);
      if (e < 0) return ORC_E_RANGE;
      c = (int32_t)x->lab[c].par[e];
      if ((uint32_t)c >= (uint32_t)x->n) return ORC_E_RANGE;
    }
    if (c != (int32_t)h) return ORC_E_RANGE;
  } else {
    int ds = x->bp_d[(int64_t)rs * tb + bi], dt = x->bp_d[(int64_t)rt * tb + bi];
    uint64_t m1s = x->bp_m1[(int64_t)rs * tb + bi];
    int ms, mt; /* walk modes of the two halves */
    if (kind == 0) {
      ms = 0;
      mt = 0;
    } else if (kind == 2) {
      ms = 1;
      mt = 1;
    } else if (m1s & wbit) {
      ms = 1;
      mt = 2;
    } else {
      ms = 2;
      mt = 1;
    }
    /* the s half ends at the meeting vertex (r or w), written at position ls-1 */
    int ls = ms == 1 ? ds : ds + 1;
    int a = bp_walk(x, rs, bi, wbit, ms, tmp, 0, 1);
    if (a != ls) return ORC_E_RANGE;
    int lt = mt == 1 ? dt : dt + 1;
    /* the t half, written backwards from D; its last vertex is the meeting one */
    int b = bp_walk(x, rt, bi, wbit, mt, tmp, D, -1);
    if (b != lt || ls + lt - 1 != D + 1) return ORC_E_RANGE;
  }
  for (int k = 0; k <= D; k++) out[k] = x->ord[tmp[k]];
  *len = D + 1;
  return ORC_OK;
}

/* Shortest path s -> t of a directed index, as path_one: the best hub h of
 * the merge of L_OUT(s) and L_IN(t) (first on ties); the parents kept with
 * (h, .) in L_OUT lead from s along the arcs to h, those in L_IN lead from t
 * against the arcs back to h. */
static int path_one_directed(const orc_index *x, int32_t s, int32_t t, int32_t maxlen,
                             int32_t *out, int32_t *len) {
  int32_t rs = x->rank[s], rt = x->rank[t];
  if (rs == rt) {
    if (maxlen < 1) {
      *len = -1;
      return ORC_OK;
    }
    out[0] = s;
    *len = 1;
    return ORC_OK;
  }
  const orc_label *A = &x->lab[rs], *B = &x->lab_in[rt];
  int best = 1 << 20, ia = -1, ib = -1;
  for (int64_t i = 0, j = 0;;) {
    uint32_t ha = A->hub[i], hb = B->hub[j];
    if (ha == hb) {
      if (ha == ORC_SENTINEL) break;
      int v = (int)A->dist[i] + (int)B->dist[j];
      if (v < best) {
        best = v;
        ia = (int)i;
        ib = (int)j;
      }
      i++;
      j++;
    } else if (ha < hb) {
      i++;
    } else {
      j++;
    }
  }
  *len = 0;
  if (best >= (int)ORC_INF) return ORC_OK;
  int D = best;
  if (maxlen < D + 1) {
    *len = -(D + 1);
    return ORC_OK;
  }
  uint32_t h = A->hub[ia];
  int ds = A->dist[ia], dt = B->dist[ib];
  int32_t c = rs;
  for (int k = 0; k <= ds; k++) {
    out[k] = c;
    if (k < ds) {
      int64_t e = find_hub(&x->lab[c], h);
      if (e < 0) return ORC_E_RANGE;
      c = (int32_t)x->lab[c].par[e];
      if ((uint32_t)c >= (uint32_t)x->n) return ORC_E_RANGE;
    }
  }
  c = rt;
  for (int k = 0; k < dt; k++) {
    out[D - k] = c;
    int64_t e = find_hub(&x->lab_in[c], h);
    if (e < 0) return ORC_E_RANGE;
    c = (int32_t)x->lab_in[c].par[e];
    if ((uint32_t)c >= (uint32_t)x->n) return ORC_E_RANGE;
  }
  if (c != (int32_t)h) return ORC_E_RANGE;
  for (int k = 0; k <= D; k++) out[k] = x->ord[out[k]];
  *len = D + 1;
  return ORC_OK;
}

/* Paths of q pairs: row i of paths (maxlen ids) and lens[i] as path_one
 * (path_one_directed for a directed index). */
int orc_paths(const orc_index *x, const int32_t *pairs, int64_t q, int32_t maxlen,
              int32_t *paths, int32_t *lens) {
  if (!x || q < 0 || maxlen < 0 ||
      (q > 0 && (!pairs || !lens || (maxlen > 0 && !paths))))
    return ORC_E_INVAL;
  for (int64_t i = 0; i < 2 * q; i++)
    if (pairs[i] < 0 || pairs[i] >= x->n) return ORC_E_INVAL;
  for (int64_t i = 0; i < q; i++) {
    int rc = x->lab_in ? path_one_directed(x, pairs[2 * i], pairs[2 * i + 1], maxlen,
                                           paths + i * (int64_t)maxlen, &lens[i])
                       : path_one(x, pairs[2 * i], pairs[2 * i + 1], maxlen,
                                  paths + i * (int64_t)maxlen, &lens[i]);
    if (rc != ORC_OK) return rc;
  }
  return ORC_OK;
}

/* Parents of the exported label entries (ranks), same order as orc_export. */
int orc_export_parents(const orc_index *x, uint32_t *par) {
  if (!x || !par) return ORC_E_INVAL;
  int64_t e = 0;
  for (int32_t v = 0; v < x->n; v++) {
    const orc_label *L = &x->lab[v];
    if (L->len) memcpy(par + e, L->par, (size_t)L->len * sizeof(uint32_t));
    e += L->len;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* O7: directed graphs (Section 6)                                           */

/* min over (h, delta) of L with T[h] finite of delta + T[h] */
static int t_query(const orc_label *L, const uint8_t *T) {
  int best = 1 << 20;
  for (int64_t i = 0; i < L->len; i++) {
    uint8_t th = T[L->hub[i]];
    if (th == ORC_INF) continue;
    int v = (int)L->dist[i] + (int)th;
    if (v < best) best = v;
  }
  return best;
}

/* One pruned BFS from root k over adj (out-edges for the forward search,
 * in-edges for the reverse one; poff/padj: the other direction, whose row u
 * lists the vertices the search reaches u from).  T holds the root's label
 * on the other side; `own` receives (k, d) at every vertex it does not
 * prune. */
static int directed_bfs(orc_index *x, int32_t k, const int64_t *off, const int32_t *adj,
                        const int64_t *poff, const int32_t *padj, orc_label *own,
                        const orc_label *root_side, uint16_t *P, uint8_t *T, int32_t *queue) {
  const orc_label *Lk = &root_side[k];
  for (int64_t i = 0; i < Lk->len; i++) T[Lk->hub[i]] = Lk->dist[i];
  x->cnt[C_ROOT_STAGED] += Lk->len;
  int rc = ORC_OK;
  int64_t qh = 0, qt = 0;
  queue[qt++] = k;
  P[k] = 0;
  while (qh < qt && rc == ORC_OK) {
    int32_t u = queue[qh++];
    int d = P[u];
    x->cnt[C_VISITED]++;
    x->cnt[C_NORMAL_TESTS]++;
    x->cnt[C_LABEL_SCANNED] += own[u].len;
    if (t_query(&own[u], T) <= d) continue;
    if (d >= (int)ORC_INF) { /* (k, 255) cannot be stored */
      rc = ORC_E_RANGE;
      break;
    }
    /* the parent: u's predecessor on a path from k for the search along
     * the arcs, its successor on a path to k for the search against them */
    uint32_t par = d == 0 ? (uint32_t)k : tree_parent(own, poff, padj, u, k, d);
    rc = label_push(&own[u], (uint32_t)k, (uint8_t)d, par);
    if (rc != ORC_OK) break;
    x->cnt[C_LABELED]++;
    if (d > x->cnt[C_MAX_DIST]) x->cnt[C_MAX_DIST] = d;
    for (int64_t j = off[u]; j < off[u + 1]; j++) {
      int32_t w = adj[j];
      x->cnt[C_EDGES]++;
      if (P[w] != 0xFFFF) continue;
      P[w] = (uint16_t)(d + 1);
      queue[qt++] = w;
    }
  }
  for (int64_t i = 0; i < qt; i++) P[queue[i]] = 0xFFFF;
  for (int64_t i = 0; i < Lk->len; i++) T[Lk->hub[i]] = (uint8_t)ORC_INF;
  return rc;
}

/* Build the two labels of a directed graph (row_ptr/col: out-edges), in
 * rank order, forward search before reverse search for each root.  No
 * bit-parallel labels (Section 5 is written for undirected graphs). */
int orc_build_directed(int32_t n, const int32_t *row_ptr, const int32_t *col,
                       const int32_t *order, orc_index **out) {
  if (!out) return ORC_E_INVAL;
  *out = NULL;
  int rc = validate(n, row_ptr, col, order, 0);
  if (rc != ORC_OK) return rc;
  orc_index *x = (orc_index *)calloc(1, sizeof(orc_index));
  if (!x) return ORC_E_NOMEM;
  x->n = n;
  x->t_bp = 0;
  int64_t nn = n > 0 ? n : 1;
  int64_t nnz = n > 0 ? row_ptr[n] : 0, mm = nnz > 0 ? nnz : 1;
  x->rank = (int32_t *)malloc((size_t)nn * sizeof(int32_t));
  x->lab = (orc_label *)calloc((size_t)nn, sizeof(orc_label));
  x->lab_in = (orc_label *)calloc((size_t)nn, sizeof(orc_label));
  x->bp_d = (uint8_t *)malloc(1);
  x->bp_m1 = (uint64_t *)malloc(sizeof(uint64_t));
  x->bp_0 = (uint64_t *)malloc(sizeof(uint64_t));
  x->bp_root = (int32_t *)malloc(sizeof(int32_t));
  x->bp_nsel = (int32_t *)malloc(sizeof(int32_t));
  x->bp_sel = (int32_t *)malloc(sizeof(int32_t));
  x->root_visited = (int32_t *)calloc((size_t)nn, sizeof(int32_t));
  x->root_labeled = (int32_t *)calloc((size_t)nn, sizeof(int32_t));
  x->ord = (int32_t *)malloc((size_t)nn * sizeof(int32_t));
  int64_t *off = (int64_t *)calloc((size_t)(nn + 1), sizeof(int64_t));
  int32_t *adj = (int32_t *)malloc((size_t)mm * sizeof(int32_t));
  int64_t *ioff = (int64_t *)calloc((size_t)(nn + 1), sizeof(int64_t));
  int32_t *iadj = (int32_t *)malloc((size_t)mm * sizeof(int32_t));
  int64_t *fill = (int64_t *)calloc((size_t)nn, sizeof(int64_t));
  uint16_t *P = (uint16_t *)malloc((size_t)nn * sizeof(uint16_t));
  uint8_t *T = (uint8_t *)malloc((size_t)nn);
  int32_t *queue = (int32_t *)malloc((size_t)nn * sizeof(int32_t));
  if (!x->rank || !x->lab || !x->lab_in || !x->bp_d || !x->bp_m1 || !x->bp_0 || !x->bp_root ||
      !x->bp_nsel || !x->bp_sel || !x->root_visited || !x->root_labeled || !x->ord || !off ||
      !adj || !ioff || !iadj || !fill || !P || !T || !queue) {
    rc = ORC_E_NOMEM;
    goto done;
  }
  /* ranks; out-adjacency and its transpose (in-adjacency), rows sorted */
  for (int32_t i = 0; i < n; i++) {
    x->rank[order[i]] = i;
    x->ord[i] = order[i];
  }
  for (int32_t r = 0; r < n; r++) {
    int32_t v = order[r];
    int64_t deg = row_ptr[v + 1] - row_ptr[v];
    for (int64_t j = 0; j < deg; j++) adj[off[r] + j] = x->rank[col[row_ptr[v] + j]];
    qsort(adj + off[r], (size_t)deg, sizeof(int32_t), cmp_i32);
    off[r + 1] = off[r] + deg;
  }
  for (int64_t j = 0; j < nnz; j++) ioff[adj[j] + 1]++;
  for (int32_t r = 0; r < n; r++) ioff[r + 1] += ioff[r];
  for (int32_t r = 0; r < n; r++) /* sources in ascending rank: rows come out sorted */
    for (int64_t j = off[r]; j < off[r + 1]; j++) iadj[ioff[adj[j]] + fill[adj[j]]++] = r;
  memset(P, 0xFF, (size_t)nn * sizeof(uint16_t));
  memset(T, (int)ORC_INF, (size_t)nn);
  for (int32_t k = 0; k < n && rc == ORC_OK; k++) {
    x->cnt[C_ROOTS]++;
    int64_t vis0 = x->cnt[C_VISITED], lab0 = x->cnt[C_LABELED];
    rc = directed_bfs(x, k, off, adj, ioff, iadj, x->lab_in, x->lab, P, T, queue);
    if (rc == ORC_OK) rc = directed_bfs(x, k, ioff, iadj, off, adj, x->lab, x->lab_in, P, T, queue);
    x->root_visited[k] = (int32_t)(x->cnt[C_VISITED] - vis0);
    x->root_labeled[k] = (int32_t)(x->cnt[C_LABELED] - lab0);
  }
  if (rc != ORC_OK) goto done;
  for (int32_t v = 0; v < n; v++) x->cnt[C_ENTRIES] += x->lab[v].len + x->lab_in[v].len;
  x->cnt[C_N] = n;
  x->off = off;
  x->adj = adj;
  off = NULL;
  adj = NULL;
  *out = x;
  x = NULL;
done:
  free(off); free(adj); free(ioff); free(iadj); free(fill); free(P); free(T); free(queue);
  if (x) orc_free(x);
  return rc;
}

/* Parents of the L_IN entries of a directed index (ranks), in the order of
 * orc_export_in. */
int orc_export_in_parents(const orc_index *x, uint32_t *par) {
  if (!x || !x->lab_in || !par) return ORC_E_INVAL;
  int64_t e = 0;
  for (int32_t v = 0; v < x->n; v++) {
    const orc_label *L = &x->lab_in[v];
    if (L->len) memcpy(par + e, L->par, (size_t)L->len * sizeof(uint32_t));
    e += L->len;
  }
  return ORC_OK;
}

/* The in-labels of a directed index, in rank order, without sentinels. */
int orc_export_in(const orc_index *x, int64_t *entries, int64_t *off, uint32_t *hub,
                  uint8_t *dist) {
  if (!x || !x->lab_in) return ORC_E_INVAL;
  int64_t e = 0;
  for (int32_t v = 0; v < x->n; v++) {
    if (off) off[v] = e;
    const orc_label *L = &x->lab_in[v];
    if (hub && L->len) memcpy(hub + e, L->hub, (size_t)L->len * sizeof(uint32_t));
    if (dist && L->len) memcpy(dist + e, L->dist, (size_t)L->len);
    e += L->len;
  }
  if (off) off[x->n] = e;
  if (entries) *entries = e;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* O8: weighted graphs (Section 6, "Weighted Graphs")                        */
/*
 * Readings:
 *   - Edge weights are integers >= 1 (a weight of 0 is rejected); distances
 *     are uint32.  ORC_WINF = 2^32 - 1 means unreachable.
 *   - A relaxation whose distance would reach ORC_WINF is dropped, so a
 *     vertex at distance >= ORC_WINF from a root is treated as unreachable
 *     from it: the labels are exactly the unbounded ones with distance below
 *     ORC_WINF, and a query answer of ORC_WINF means unreachable or that far.
 *   - Sums of two distances are formed in 64 bits.
 */

#define ORC_WINF 0xFFFFFFFFu

typedef struct {
  uint32_t *hub; /* hub ranks, ascending, then ORC_SENTINEL */
  uint32_t *dist;
  uint32_t *par; /* parent (rank) of this vertex in the search tree of the hub */
  int64_t len, cap;
} orc_wlabel;

enum {
  W_N = 0,         /* vertices */
  W_ENTRIES,       /* label entries (both directions of a digraph) */
  W_ROOTS,         /* pruned searches run (two per root for a digraph) */
  W_SETTLED,       /* vertices settled (each tested once per search) */
  W_LABELED,       /* vertices labeled */
  W_EDGES,         /* adjacency entries relaxed from labeled vertices */
  W_PUSHES,        /* heap insertions (improvements of a tentative distance) */
  W_LABEL_SCANNED, /* label entries read by prune tests */
  W_MAX_DIST,      /* largest stored distance */
  ORC_WNCOUNTERS
};

typedef struct orc_windex {
  int32_t n, directed;
  int32_t *rank;
  int32_t *ord; /* input id of rank r */
  orc_wlabel *out; /* L of an undirected graph; L_OUT of a digraph */
  orc_wlabel *in;  /* L_IN of a digraph, else NULL */
  int64_t cnt[ORC_WNCOUNTERS];
} orc_windex;

static void wlabel_free_all(orc_wlabel *lab, int32_t n) {
  if (!lab) return;
  for (int32_t v = 0; v < n; v++) {
    free(lab[v].hub);
    free(lab[v].dist);
    free(lab[v].par);
  }
  free(lab);
}

void orc_wfree(orc_windex *x) {
  if (!x) return;
  wlabel_free_all(x->out, x->n);
  wlabel_free_all(x->in, x->n);
  free(x->rank);
  free(x->ord);
  free(x);
}

/* Append (h, d) and keep the sentinel after the last entry. */
static int wlabel_push(orc_wlabel *L, uint32_t h, uint32_t d, uint32_t par) {
  if (L->len + 2 > L->cap) {
    int64_t nc = L->cap ? 2 * L->cap : 4;
    uint32_t *nh = (uint32_t *)realloc(L->hub, (size_t)nc * sizeof(uint32_t));
    if (!nh) return ORC_E_NOMEM;
    L->hub = nh;
    uint32_t *nd = (uint32_t *)realloc(L->dist, (size_t)nc * sizeof(uint32_t));
    if (!nd) return ORC_E_NOMEM;
    L->dist = nd;
    uint32_t *np = (uint32_t *)realloc(L->par, (size_t)nc * sizeof(uint32_t));
    if (!np) return ORC_E_NOMEM;
    L->par = np;
    L->cap = nc;
  }
  L->hub[L->len] = h;
  L->dist[L->len] = d;
  L->par[L->len] = par;
  L->len++;
  L->hub[L->len] = ORC_SENTINEL;
  L->dist[L->len] = ORC_WINF;
  L->par[L->len] = ORC_SENTINEL;
  return ORC_OK;
}

/* Binary min-heap of (distance, vertex) keys packed as d << 32 | v. */
typedef struct {
  uint64_t *a;
  int64_t len, cap;
} wheap;

static int wheap_push(wheap *h, uint64_t key) {
  if (h->len == h->cap) {
    int64_t nc = h->cap ? 2 * h->cap : 64;
    uint64_t *na = (uint64_t *)realloc(h->a, (size_t)nc * sizeof(uint64_t));
    if (!na) return ORC_E_NOMEM;
    h->a = na;
    h->cap = nc;
  }
  int64_t i = h->len++;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h->a[p] <= key) break;
    h->a[i] = h->a[p];
    i = p;
  }
  h->a[i] = key;
  return ORC_OK;
}

static uint64_t wheap_pop(wheap *h) {
  uint64_t top = h->a[0], last = h->a[--h->len];
  int64_t i = 0;
  for (;;) {
    int64_t c = 2 * i + 1;
    if (c >= h->len) break;
    if (c + 1 < h->len && h->a[c + 1] < h->a[c]) c++;
    if (h->a[c] >= last) break;
    h->a[i] = h->a[c];
    i = c;
  }
  if (h->len) h->a[i] = last;
  return top;
}

/* Parent kept with (k, d) in L(u) of a weighted search, d >= 1: the
 * lowest-ranked p in row u of (poff, padj, pw) -- the edges p -> u of the
 * search, weight pw -- whose label's newest entry is (k, d - pw).  Weights
 * are at least 1, so every such p was settled (labeled or pruned) before
 * u. */
static uint32_t wtree_parent(const orc_wlabel *lab, const int64_t *poff, const int32_t *padj,
                             const uint32_t *pw, int32_t u, int32_t k, uint32_t d) {
  uint32_t best = ORC_SENTINEL;
  for (int64_t j = poff[u]; j < poff[u + 1]; j++) {
    const orc_wlabel *L = &lab[padj[j]];
    if (pw[j] <= d && L->len > 0 && L->hub[L->len - 1] == (uint32_t)k &&
        L->dist[L->len - 1] == d - pw[j] && (uint32_t)padj[j] < best)
      best = (uint32_t)padj[j];
  }
  return best;
}

/* One pruned Dijkstra search from root k over (off, adj, wgt): settled
 * vertices are tested against T (the root's labels from tlab, indexed by
 * hub) and their own labels in `lab`; a vertex that is not pruned gets
 * (k, d) in `lab` and relaxes its edges.  (poff, padj, pw): the edges in
 * the other direction (the same ones for an undirected graph), for the
 * parents.  D, T and settled are all-INF / zero on entry and on exit. */
static int weighted_search(orc_windex *x, int32_t k, const int64_t *off, const int32_t *adj,
                           const uint32_t *wgt, const int64_t *poff, const int32_t *padj,
                           const uint32_t *pw, orc_wlabel *lab, const orc_wlabel *tlab,
                           uint32_t *D, uint32_t *T, char *settled, int32_t *touched,
                           wheap *heap) {
  int rc = ORC_OK;
  const orc_wlabel *Lk = &tlab[k];
  for (int64_t i = 0; i < Lk->len; i++) T[Lk->hub[i]] = Lk->dist[i];
  int64_t nt = 0;
  heap->len = 0;
  D[k] = 0;
  touched[nt++] = k;
  rc = wheap_push(heap, (uint64_t)k);
  x->cnt[W_PUSHES]++;
  while (rc == ORC_OK && heap->len) {
    uint64_t key = wheap_pop(heap);
    int32_t u = (int32_t)(key & 0xFFFFFFFFu);
    uint32_t d = (uint32_t)(key >> 32);
    if (settled[u] || d != D[u]) continue; /* stale heap entry */
    settled[u] = 1;
    x->cnt[W_SETTLED]++;
    /* prune test: QUERY(v_k, u) over the labels so far (Section 4.5.1 T) */
    const orc_wlabel *L = &lab[u];
    x->cnt[W_LABEL_SCANNED] += L->len;
    int pruned = 0;
    for (int64_t i = 0; i < L->len && !pruned; i++) {
      uint32_t th = T[L->hub[i]];
      if (th != ORC_WINF && (uint64_t)L->dist[i] + th <= d) pruned = 1;
    }
    if (pruned) continue;
    uint32_t par = d == 0 ? (uint32_t)k : wtree_parent(lab, poff, padj, pw, u, k, d);
    rc = wlabel_push(&lab[u], (uint32_t)k, d, par);
    if (rc != ORC_OK) break;
    x->cnt[W_LABELED]++;
    if ((int64_t)d > x->cnt[W_MAX_DIST]) x->cnt[W_MAX_DIST] = d;
    for (int64_t j = off[u]; j < off[u + 1] && rc == ORC_OK; j++) {
      int32_t w = adj[j];
      x->cnt[W_EDGES]++;
      uint64_t nd = (uint64_t)d + wgt[j];
      if (nd >= ORC_WINF || settled[w] || nd >= D[w]) continue;
      if (D[w] == ORC_WINF) touched[nt++] = w;
      D[w] = (uint32_t)nd;
      rc = wheap_push(heap, nd << 32 | (uint64_t)w);
      x->cnt[W_PUSHES]++;
    }
  }
  for (int64_t i = 0; i < nt; i++) {
    D[touched[i]] = ORC_WINF;
    settled[touched[i]] = 0;
  }
  for (int64_t i = 0; i < Lk->len; i++) T[Lk->hub[i]] = ORC_WINF;
  return rc;
}

typedef struct {
  int32_t v;
  uint32_t w;
} wnbr;

static int cmp_wnbr(const void *a, const void *b) {
  const wnbr *x = (const wnbr *)a, *y = (const wnbr *)b;
  if (x->v != y->v) return x->v < y->v ? -1 : 1;
  return (x->w > y->w) - (x->w < y->w);
}

/* Rank-space adjacency with weights, each row sorted by (rank, weight). */
static void weighted_adjacency(const orc_windex *x, const int32_t *row_ptr, const int32_t *col,
                               const uint32_t *wgt, const int32_t *order, int64_t *off,
                               int32_t *adj, uint32_t *aw, wnbr *tmp) {
  int32_t n = x->n;
  off[0] = 0;
  for (int32_t r = 0; r < n; r++) {
    int32_t v = order[r];
    int64_t deg = row_ptr[v + 1] - row_ptr[v];
    for (int64_t j = 0; j < deg; j++) {
      tmp[j].v = x->rank[col[row_ptr[v] + j]];
      tmp[j].w = wgt[row_ptr[v] + j];
    }
    qsort(tmp, (size_t)deg, sizeof(wnbr), cmp_wnbr);
    for (int64_t j = 0; j < deg; j++) {
      adj[off[r] + j] = tmp[j].v;
      aw[off[r] + j] = tmp[j].w;
    }
    off[r + 1] = off[r] + deg;
  }
}

/* Weighted build.  flags bit 0: check that every edge (u, v, w) has its
 * reverse (v, u, w) (undirected only); bit 1: the CSR lists out-arcs of a
 * digraph (labels L_OUT and L_IN, Section 6). */
int orc_build_weighted(int32_t n, const int32_t *row_ptr, const int32_t *col,
                       const uint32_t *wgt, const int32_t *order, uint32_t flags,
                       orc_windex **out) {
  if (!out) return ORC_E_INVAL;
  *out = NULL;
  int rc = validate(n, row_ptr, col, order, 0);
  if (rc != ORC_OK) return rc;
  int64_t nnz = n > 0 ? row_ptr[n] : 0;
  if (nnz > 0 && !wgt) return ORC_E_INVAL;
  for (int64_t j = 0; j < nnz; j++)
    if (wgt[j] == 0) return ORC_E_INVAL;
  int directed = (flags & 2u) != 0;
  orc_windex *x = (orc_windex *)calloc(1, sizeof(orc_windex));
  if (!x) return ORC_E_NOMEM;
  x->n = n;
  x->directed = directed;
  int64_t nn = n > 0 ? n : 1, mm = nnz > 0 ? nnz : 1, maxdeg = 1;
  for (int32_t v = 0; v < n; v++)
    if (row_ptr[v + 1] - row_ptr[v] > maxdeg) maxdeg = row_ptr[v + 1] - row_ptr[v];
  x->rank = (int32_t *)malloc((size_t)nn * sizeof(int32_t));
  x->out = (orc_wlabel *)calloc((size_t)nn, sizeof(orc_wlabel));
  if (directed) x->in = (orc_wlabel *)calloc((size_t)nn, sizeof(orc_wlabel));
  int64_t *off = (int64_t *)calloc((size_t)(nn + 1), sizeof(int64_t));
  int32_t *adj = (int32_t *)malloc((size_t)mm * sizeof(int32_t));
  uint32_t *aw = (uint32_t *)malloc((size_t)mm * sizeof(uint32_t));
  int64_t *ioff = NULL;
  int32_t *iadj = NULL;
  uint32_t *iaw = NULL;
  wnbr *tmp = (wnbr *)malloc((size_t)maxdeg * sizeof(wnbr));
  uint32_t *D = (uint32_t *)malloc((size_t)nn * sizeof(uint32_t));
  uint32_t *T = (uint32_t *)malloc((size_t)nn * sizeof(uint32_t));
  char *settled = (char *)calloc((size_t)nn, 1);
  int32_t *touched = (int32_t *)malloc((size_t)nn * sizeof(int32_t));
  x->ord = (int32_t *)malloc((size_t)nn * sizeof(int32_t));
  wheap heap = {NULL, 0, 0};
  if (!x->rank || !x->out || (directed && !x->in) || !off || !adj || !aw || !tmp || !D || !T ||
      !settled || !touched || !x->ord) {
    rc = ORC_E_NOMEM;
    goto done;
  }
  for (int32_t i = 0; i < n; i++) {
    x->rank[order[i]] = i;
    x->ord[i] = order[i];
  }
  weighted_adjacency(x, row_ptr, col, wgt, order, off, adj, aw, tmp);
  if (!directed && (flags & 1u)) {
    /* every (r, s, w) has (s, r, w): rows are sorted by (rank, weight) */
    for (int32_t r = 0; r < n && rc == ORC_OK; r++)
      for (int64_t j = off[r]; j < off[r + 1]; j++) {
        int32_t s2 = adj[j];
        int found = 0;
        for (int64_t i = off[s2]; i < off[s2 + 1] && !found; i++)
          if (adj[i] == r && aw[i] == aw[j]) found = 1;
        if (!found) {
          rc = ORC_E_INVAL;
          break;
        }
      }
    if (rc != ORC_OK) goto done;
  }
  if (directed) {
    /* transpose: in-arcs of every vertex, sources in ascending rank */
    ioff = (int64_t *)calloc((size_t)(nn + 1), sizeof(int64_t));
    iadj = (int32_t *)malloc((size_t)mm * sizeof(int32_t));
    iaw = (uint32_t *)malloc((size_t)mm * sizeof(uint32_t));
    int64_t *fill = (int64_t *)calloc((size_t)nn, sizeof(int64_t));
    if (!ioff || !iadj || !iaw || !fill) {
      free(fill);
      rc = ORC_E_NOMEM;
      goto done;
    }
    for (int64_t j = 0; j < nnz; j++) ioff[adj[j] + 1]++;
    for (int32_t r = 0; r < n; r++) ioff[r + 1] += ioff[r];
    for (int32_t r = 0; r < n; r++)
      for (int64_t j = off[r]; j < off[r + 1]; j++) {
        int64_t p = ioff[adj[j]] + fill[adj[j]]++;
        iadj[p] = r;
        iaw[p] = aw[j];
      }
    free(fill);
  }
  for (int32_t r = 0; r < n; r++) {
    D[r] = ORC_WINF;
    T[r] = ORC_WINF;
  }
  for (int32_t k = 0; k < n && rc == ORC_OK; k++) {
    if (!directed) {
      x->cnt[W_ROOTS]++;
      rc = weighted_search(x, k, off, adj, aw, off, adj, aw, x->out, x->out, D, T, settled,
                           touched, &heap);
    } else {
      /* along the arcs: labels L_IN, root distances from L_OUT(k); then
       * against them: labels L_OUT, root distances from L_IN(k) */
      x->cnt[W_ROOTS] += 2;
      rc = weighted_search(x, k, off, adj, aw, ioff, iadj, iaw, x->in, x->out, D, T, settled,
                           touched, &heap);
      if (rc == ORC_OK)
        rc = weighted_search(x, k, ioff, iadj, iaw, off, adj, aw, x->out, x->in, D, T, settled,
                             touched, &heap);
    }
  }
  if (rc != ORC_OK) goto done;
  for (int32_t v = 0; v < n; v++)
    x->cnt[W_ENTRIES] += x->out[v].len + (directed ? x->in[v].len : 0);
  x->cnt[W_N] = n;
  *out = x;
  x = NULL;
done:
  free(off); free(adj); free(aw); free(ioff); free(iadj); free(iaw); free(tmp);
  free(D); free(T); free(settled); free(touched); free(heap.a);
  if (x) orc_wfree(x);
  return rc;
}

/* QUERY over sorted labels (Section 3.3 merge join), 64-bit sums. */
static uint32_t wquery_one(const orc_windex *x, int32_t s, int32_t t) {
  const orc_wlabel *A = &x->out[x->rank[s]];
  const orc_wlabel *B = x->directed ? &x->in[x->rank[t]] : &x->out[x->rank[t]];
  uint64_t best = ORC_WINF;
  if (!A->hub || !B->hub) return ORC_WINF;
  int64_t i = 0, j = 0;
  for (;;) {
    uint32_t ha = A->hub[i], hb = B->hub[j];
    if (ha == hb) {
      if (ha == ORC_SENTINEL) break;
      uint64_t v = (uint64_t)A->dist[i] + B->dist[j];
      best = v < best ? v : best;
      i++;
      j++;
    } else if (ha < hb) {
      i++;
    } else {
      j++;
    }
  }
  return (uint32_t)best;
}

int orc_wquery(const orc_windex *x, const int32_t *pairs, int64_t q, uint32_t *out) {
  if (!x || q < 0 || (q > 0 && (!pairs || !out))) return ORC_E_INVAL;
  for (int64_t i = 0; i < 2 * q; i++)
    if (pairs[i] < 0 || pairs[i] >= x->n) return ORC_E_INVAL;
  for (int64_t i = 0; i < q; i++) out[i] = wquery_one(x, pairs[2 * i], pairs[2 * i + 1]);
  return ORC_OK;
}

int32_t orc_wncounters(void) { return ORC_WNCOUNTERS; }

int orc_wcounters(const orc_windex *x, int64_t *c, int32_t nc) {
  if (!x || !c) return ORC_E_INVAL;
  for (int32_t i = 0; i < nc && i < ORC_WNCOUNTERS; i++) c[i] = x->cnt[i];
  return ORC_OK;
}

/* Labels in rank order without sentinels: side 0 = L (L_OUT of a digraph),
 * side 1 = L_IN.  *entries gets the count; NULL arrays skip the copy. */
int orc_wexport(const orc_windex *x, int32_t side, int64_t *entries, int64_t *off,
                uint32_t *hub, uint32_t *dist, int32_t *rank) {
  if (!x || (side == 1 && !x->in) || side < 0 || side > 1) return ORC_E_INVAL;
  const orc_wlabel *lab = side ? x->in : x->out;
  int64_t e = 0;
  for (int32_t v = 0; v < x->n; v++) {
    if (off) off[v] = e;
    const orc_wlabel *L = &lab[v];
    if (hub && L->len) memcpy(hub + e, L->hub, (size_t)L->len * sizeof(uint32_t));
    if (dist && L->len) memcpy(dist + e, L->dist, (size_t)L->len * sizeof(uint32_t));
    e += L->len;
  }
  if (off) off[x->n] = e;
  if (entries) *entries = e;
  if (rank && x->n) memcpy(rank, x->rank, (size_t)x->n * sizeof(int32_t));
  return ORC_OK;
}

/* entry of hub h in a weighted label (sorted by hub rank), or -1 */
static int64_t wfind_hub(const orc_wlabel *L, uint32_t h) {
  int64_t lo = 0, hi = L->len;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (L->hub[mid] < h) lo = mid + 1;
    else hi = mid;
  }
  return (lo < L->len && L->hub[lo] == h) ? lo : -1;
}

/* Vertices from rank c up the search tree of hub h (c first, h last) into
 * out[pos], out[pos + dir], ... (out may be NULL: count only).  Returns the
 * count, or -1 if a label lacks h (a broken index). */
static int64_t wascend(const orc_windex *x, const orc_wlabel *lab, int32_t c, uint32_t h,
                       int32_t *out, int64_t pos, int64_t dir, int64_t room) {
  int64_t cnt = 0;
  for (;;) {
    if (out && cnt < room) out[pos + dir * cnt] = x->ord[c];
    cnt++;
    if ((uint32_t)c == h) return cnt;
    if (cnt > x->n) return -1;
    int64_t e = wfind_hub(&lab[c], h);
    if (e < 0) return -1;
    c = (int32_t)lab[c].par[e];
    if ((uint32_t)c >= (uint32_t)x->n) return -1;
  }
}

/* Shortest path s -> t of a weighted index: the best hub h of the merge of
 * L(s) (L_OUT) and L(t) (L_IN), first on ties, then both search trees of h
 * ascended.  *len = vertices on the path, 0 if unreachable (or 2^32 - 1 or
 * more away), -(vertices) if maxlen is too small (nothing written). */
static int wpath_one(const orc_windex *x, int32_t s, int32_t t, int32_t maxlen, int32_t *out,
                     int32_t *len) {
  int32_t rs = x->rank[s], rt = x->rank[t];
  const orc_wlabel *A = &x->out[rs], *B = x->directed ? &x->in[rt] : &x->out[rt];
  const orc_wlabel *tl = x->directed ? x->in : x->out;
  *len = 0;
  if (rs == rt) {
    if (maxlen >= 1) out[0] = s;
    *len = maxlen >= 1 ? 1 : -1;
    return ORC_OK;
  }
  uint64_t best = ORC_WINF;
  uint32_t h = ORC_SENTINEL;
  for (int64_t i = 0, j = 0;;) {
    uint32_t ha = A->hub[i], hb = B->hub[j];
    if (ha == hb) {
      if (ha == ORC_SENTINEL) break;
      uint64_t v = (uint64_t)B->dist[j] + A->dist[i];
      if (v < best) {
        best = v;
        h = ha;
      }
      i++;
      j++;
    } else if (ha < hb) {
      i++;
    } else {
      j++;
    }
  }
  if (best >= ORC_WINF) return ORC_OK;
  int64_t cs = wascend(x, x->out, rs, h, NULL, 0, 1, 0);
  int64_t ct = wascend(x, tl, rt, h, NULL, 0, 1, 0);
  if (cs < 0 || ct < 0) return ORC_E_RANGE;
  int64_t total = cs + ct - 1; /* h counted once */
  if (total > maxlen) {
    *len = (int32_t)-total;
    return ORC_OK;
  }
  wascend(x, x->out, rs, h, out, 0, 1, total);
  wascend(x, tl, rt, h, out, total - 1, -1, total);
  *len = (int32_t)total;
  return ORC_OK;
}

int orc_wpaths(const orc_windex *x, const int32_t *pairs, int64_t q, int32_t maxlen,
               int32_t *paths, int32_t *lens) {
  if (!x || q < 0 || maxlen < 0 || (q > 0 && (!pairs || !lens || (maxlen > 0 && !paths))))
    return ORC_E_INVAL;
  for (int64_t i = 0; i < 2 * q; i++)
    if (pairs[i] < 0 || pairs[i] >= x->n) return ORC_E_INVAL;
  for (int64_t i = 0; i < q; i++) {
    int rc = wpath_one(x, pairs[2 * i], pairs[2 * i + 1], maxlen, paths + i * (int64_t)maxlen,
                       &lens[i]);
    if (rc != ORC_OK) return rc;
  }
  return ORC_OK;
}

/* Parents (ranks) of the exported entries of one side, as orc_wexport. */
int orc_wexport_parents(const orc_windex *x, int32_t side, uint32_t *par) {
  if (!x || !par || (side == 1 && !x->in) || side < 0 || side > 1) return ORC_E_INVAL;
  const orc_wlabel *lab = side ? x->in : x->out;
  int64_t e = 0;
  for (int32_t v = 0; v < x->n; v++) {
    const orc_wlabel *L = &lab[v];
    if (L->len) memcpy(par + e, L->par, (size_t)L->len * sizeof(uint32_t));
    e += L->len;
  }
  return ORC_OK;
}
