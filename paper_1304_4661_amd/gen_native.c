/* Preferential-attachment loop of the Barabasi-Albert input generator, in C
 * for speed.  It consumes the same uniform draws, in the same order, as the
 * Python loop in gen.py, so both give identical graphs. */
#include <stdint.h>

/* Vertices 0..m-1 start isolated, vertex m joins all of them, every later
 * vertex v draws targets from the endpoint multiset (index floor(u * size))
 * until it has m distinct ones.  us/vs receive m*(n-m) edges.  Returns the
 * number of uniforms used, or -1 if nu were not enough. */
int64_t ba_edges(int64_t n, int32_t m, const double *u, int64_t nu, int64_t *us, int64_t *vs,
                 int64_t *ends) {
  int64_t e = 0, bi = 0;
  for (int32_t j = 0; j < m; j++) {
    us[e] = m;
    vs[e] = j;
    ends[2 * e] = m;
    ends[2 * e + 1] = j;
    e++;
  }
  int64_t chosen[64];
  for (int64_t v = m + 1; v < n; v++) {
    const int64_t nends = 2 * e;
    int32_t c = 0;
    while (c < m) {
      if (bi >= nu) return -1;
      const int64_t t = ends[(int64_t)(u[bi++] * (double)nends)];
      int dup = 0;
      for (int32_t k = 0; k < c; k++) dup |= chosen[k] == t;
      if (!dup) chosen[c++] = t;
    }
    for (int32_t k = 0; k < m; k++) {
      us[e] = v;
      vs[e] = chosen[k];
      ends[2 * e] = v;
      ends[2 * e + 1] = chosen[k];
      e++;
    }
  }
  return bi;
}
