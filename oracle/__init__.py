"""CPU oracle for delayed asynchronous PageRank and Bellman-Ford sweeps.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this package: only the test suite, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code, header, table or helper with the
HIP library; the only thing both sides read is the seeded input generator
(``graphgen``), which holds none of the method's arithmetic.

What it computes (Blanco, McMillan, Low, "Delayed Asynchronous Iterative Graph
Algorithms", HPEC 2021):

* ``pagerank`` - the damped PageRank fixed point the paper's pull sweeps
  converge to (the paper evaluates pull-based PageRank in its section on
  factors affecting delta), written as the plain Jacobi (synchronous) sweep of
  the introduction, plus a dense linear solve for tiny graphs and an a-posteriori
  error certificate.
* ``sssp`` - Bellman-Ford single-source shortest paths with 32-bit unsigned
  path lengths (same section), as the synchronous min-plus sweep, plus
  Dijkstra, Floyd-Warshall and an O(m) optimality certificate.
* ``schedule`` - a sequential emulation of the paper's delayed schedule
  (section III: thread-local buffers of delta values flushed to the global
  array when full or when the thread's block is done), used to pin the
  semantics of the three commit modes on tiny graphs.

Precision: float64 throughout for PageRank; exact integers (int64) for paths.
"""
from . import pagerank, sssp, schedule  # noqa: F401
