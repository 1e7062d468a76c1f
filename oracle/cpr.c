/*
 * PageRank oracle in plain C (float64, CPU, OpenMP over vertices).
 *
 * TEST INFRASTRUCTURE ONLY: called by the test suite (through oracle/cpr.py)
 * for graphs too large for the numpy oracle to finish in seconds; never by
 * the product path, and it shares no code with the HIP library.
 *
 * It computes exactly what oracle/pagerank.py computes, written out the same
 * plain way: the synchronous (Jacobi) sweep of the damped PageRank map
 *
 *   T(x)_v = (1 - alpha)/N + alpha * ( sum_{u -> v} x_u / outdeg(u) + D(x)/N ),
 *   D(x)   = sum of x_u over vertices u with outdeg(u) = 0,
 *
 * (the paper's pull-based PageRank of its evaluation section, with the
 * standard damped form and the dangling mass spread evenly), repeated from
 * x = 1/N until the L1 change of a sweep is below tol (its stopping rule with
 * a threshold).  Edges count with multiplicity; self-loops count in outdeg.
 * With a restart vertex s it is the personalised map of the batched queries
 * instead, from x = e_s:
 *
 *   P_s(x)_v = alpha * sum_{u -> v} x_u / outdeg(u) + [v = s] ((1 - alpha) + alpha D(x)).
 *
 * Each vertex's in-edge sum runs in edge order on one thread, and D and the
 * L1 change are summed over fixed vertex ranges in range order, so the result
 * does not depend on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CHUNKS 256

static void range_of(uint32_t n, int c, uint32_t* lo, uint32_t* hi) {
  *lo = (uint32_t)(((uint64_t)n * (uint64_t)c) / CHUNKS);
  *hi = (uint32_t)(((uint64_t)n * (uint64_t)(c + 1)) / CHUNKS);
}

/* Returns 0 on success, 1 on allocation failure, 2 on malformed input.
 * ptr[n+1], idx[m]: out-edge CSR.  restart: 0xFFFFFFFF for PageRank, else
 * the restart vertex of personalised PageRank.  x_out[n]: the last iterate (not
 * normalised).  sweeps_out: sweeps run, the confirming one included.
 * resid_out: L1 change of the last sweep. */
int cpr_jacobi(uint32_t n, uint64_t m, const uint64_t* ptr, const uint32_t* idx, uint32_t restart, double alpha,
               double tol, uint32_t max_sweeps, double* x_out, uint32_t* sweeps_out, double* resid_out) {
  const int personal = restart != 0xFFFFFFFFu;
  if (n == 0 || ptr[0] != 0 || ptr[n] != m || (personal && restart >= n)) return 2;
  for (uint64_t e = 0; e < m; ++e)
    if (idx[e] >= n) return 2;
  /* in-edge lists by a counting sort over destinations (sources ascending
   * within a destination, as they come from the CSR scan) */
  uint64_t* in_ptr = calloc((size_t)n + 1, sizeof(uint64_t));
  uint32_t* in_src = malloc((m ? m : 1) * sizeof(uint32_t));
  uint32_t* deg = malloc((size_t)n * sizeof(uint32_t));
  double* x = malloc((size_t)n * sizeof(double));
  double* xn = malloc((size_t)n * sizeof(double));
  double* contrib = malloc((size_t)n * sizeof(double));
  uint64_t* fill = malloc((size_t)n * sizeof(uint64_t));
  if (!in_ptr || !in_src || !deg || !x || !xn || !contrib || !fill) {
    free(in_ptr); free(in_src); free(deg); free(x); free(xn); free(contrib); free(fill);
    return 1;
  }
  for (uint32_t u = 0; u < n; ++u) deg[u] = (uint32_t)(ptr[u + 1] - ptr[u]);
  for (uint64_t e = 0; e < m; ++e) in_ptr[idx[e] + 1]++;
  for (uint32_t v = 0; v < n; ++v) in_ptr[v + 1] += in_ptr[v];
  memcpy(fill, in_ptr, (size_t)n * sizeof(uint64_t));
  for (uint32_t u = 0; u < n; ++u)
    for (uint64_t e = ptr[u]; e < ptr[u + 1]; ++e) in_src[fill[idx[e]]++] = u;

  for (uint32_t v = 0; v < n; ++v) x[v] = personal ? (v == restart ? 1.0 : 0.0) : 1.0 / (double)n;
  double part[CHUNKS];
  uint32_t sweeps = 0;
  double r = 0.0;
  while (sweeps < max_sweeps) {
    /* contributions and the dangling mass of the current iterate */
#pragma omp parallel for schedule(static)
    for (int c = 0; c < CHUNKS; ++c) {
      uint32_t lo, hi;
      range_of(n, c, &lo, &hi);
      double d = 0.0;
      for (uint32_t u = lo; u < hi; ++u) {
        if (deg[u]) {
          contrib[u] = x[u] / (double)deg[u];
        } else {
          contrib[u] = 0.0;
          d += x[u];
        }
      }
      part[c] = d;
    }
    double dang = 0.0;
    for (int c = 0; c < CHUNKS; ++c) dang += part[c];
    const double base = (1.0 - alpha) / (double)n;
    const double at_restart = (1.0 - alpha) + alpha * dang;
    /* pull every vertex's new value; the L1 change per range */
#pragma omp parallel for schedule(static)
    for (int c = 0; c < CHUNKS; ++c) {
      uint32_t lo, hi;
      range_of(n, c, &lo, &hi);
      double rc = 0.0;
      for (uint32_t v = lo; v < hi; ++v) {
        double s = 0.0;
        for (uint64_t e = in_ptr[v]; e < in_ptr[v + 1]; ++e) s += contrib[in_src[e]];
        const double y = personal ? alpha * s + (v == restart ? at_restart : 0.0) : base + alpha * (s + dang / (double)n);
        const double diff = y - x[v];
        rc += diff < 0 ? -diff : diff;
        xn[v] = y;
      }
      part[c] = rc;
    }
    r = 0.0;
    for (int c = 0; c < CHUNKS; ++c) r += part[c];
    double* t = x;
    x = xn;
    xn = t;
    ++sweeps;
    if (r < tol) break;
  }
  memcpy(x_out, x, (size_t)n * sizeof(double));
  *sweeps_out = sweeps;
  *resid_out = r;
  free(in_ptr); free(in_src); free(deg); free(x); free(xn); free(contrib); free(fill);
  return 0;
}
