"""CPU oracle for exact fixed-radius near-neighbour search (SNN, Chen & Guettel).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.
The HIP product path never imports, links or calls it, and this package never
imports the product package: the two share no code.

What the oracle computes (the result definition every GPU path must match
bit for bit):

    N(q) = { i : S(p_i, q) <= fl(R*R) }

where inputs are promoted to float64 (exact) and S is the direct squared
distance of Section 4, eq. (ip1), evaluated in the recursion order the
rounding analysis of Section 4 uses: t_k = fl(p_k - q_k), then
s <- fl(s + fl(t_k * t_k)) for k = 0..d-1 left to right, with no fused
multiply-add.  The comparison is inclusive (Section 3.2 asks for
||p_i - q|| <= R and compares squares).  Returned distances are
fl32(sqrt(S)).  Rows are in query order; ids within a row are ascending
original row numbers (the paper leaves the order open).

Modules
-------
brute   O1: exhaustive search with the normative S ("brute force 2" of
        Section 6.1 with the direct form in place of gemv).
snn     O2: Algorithms 1 and 2 of Section 3 on the CPU -- centring, first
        principal component, sort by score, binary-searched window, the
        decomposition of eq. (ip2) -- plus a rigorous floating-point band in
        which decisions are re-taken with the normative S.
exact   O3: exact rational arithmetic on tiny inputs (fractions.Fraction).
dbscan  DBSCAN (the application of Section 6.4) on self-query neighbour
        lists: core points, clusters grown in index order, border points.

Pins: see tests/test_oracle_*.py.  Every function here is pinned by at least
one test that does not re-use its own formula (exact rationals, lattice
counts, closed-form statistics, values printed in Tables 1 and 2, the
Cauchy-Schwarz invariant of eq. (lower), the sigma_2 = 0 special case).
"""

from .brute import Neighbors, normative_sqdist, brute_radius
from .snn import SnnIndex, build_index, query as snn_query, first_principal_component
from .exact import exact_sqdist, exact_radius
from .dbscan import Clustering, dbscan, dbscan_from_neighbors

__all__ = [
    "Neighbors",
    "normative_sqdist",
    "brute_radius",
    "SnnIndex",
    "build_index",
    "snn_query",
    "first_principal_component",
    "exact_sqdist",
    "exact_radius",
    "Clustering",
    "dbscan",
    "dbscan_from_neighbors",
]
