"""DBSCAN on fixed-radius neighbour lists (the application of Section 6.4).

Test infrastructure only (see the package docstring).

Section 6.4 plugs SNN into scikit-learn's DBSCAN as its radius search and
reports that the clustering is unchanged, with min_samples fixed at 5 and
eps playing the role of the radius R.  The clustering is therefore DBSCAN
as that implementation defines it, restated here:

* the eps-neighbourhood of point i is N(i) = { j : S(p_j, p_i) <= fl(eps^2) }
  (the normative rule of the search, so i itself belongs to it);
* i is a core point iff |N(i)| >= min_samples (the point itself counts);
* points are visited in ascending index; each core point not yet labelled
  opens the next cluster (labels 0, 1, 2, ...), which is grown through core
  points only: every unlabelled member of the neighbourhood of a core point
  of the cluster joins it, and the growth continues from the members that
  are core points;
* points that no cluster reaches are noise (label -1).

A cluster is thus a connected component of the graph of core points joined
when one lies in the other's neighbourhood, plus the non-core points in the
neighbourhood of its core points; clusters are numbered in order of their
smallest core index, and a non-core point within reach of several clusters
takes the one numbered first.  Pins: tests/test_oracle_dbscan.py (against
scikit-learn's DBSCAN, and closed-form configurations).
"""

from __future__ import annotations

from collections import deque
from typing import NamedTuple

import numpy as np

from .brute import brute_radius


class Clustering(NamedTuple):
    labels: np.ndarray  # int32, n: cluster label or -1 (noise)
    core: np.ndarray  # bool, n


def dbscan_from_neighbors(row_ptr, col, min_samples: int) -> Clustering:
    """DBSCAN labels from neighbour lists (row i = N(i), self included).

    row_ptr: (n+1,) int, col: (nnz,) int.  The lists must be those of an
    all-points self-query, so membership is symmetric.
    """
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    n = row_ptr.shape[0] - 1
    if min_samples < 1:
        raise ValueError("min_samples must be >= 1")
    core = (row_ptr[1:] - row_ptr[:-1]) >= min_samples
    labels = np.full(n, -1, dtype=np.int32)
    next_label = 0
    for i in range(n):
        if labels[i] != -1 or not core[i]:
            continue
        labels[i] = next_label
        frontier = deque([i])  # core points of the cluster still to expand
        while frontier:
            c = frontier.popleft()
            for j in col[row_ptr[c]:row_ptr[c + 1]]:
                if labels[j] == -1:
                    labels[j] = next_label
                    if core[j]:
                        frontier.append(int(j))
        next_label += 1
    return Clustering(labels, core)


def dbscan(P, eps: float, min_samples: int) -> Clustering:
    """DBSCAN of the rows of P with the normative eps-neighbourhoods (O1)."""
    nb = brute_radius(P, P, eps)
    return dbscan_from_neighbors(nb.row_ptr, nb.col, min_samples)
