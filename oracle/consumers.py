"""Plain FP64 reference of the two consumers of the smallest eigenpairs that
Section 2 of the paper describes.

TEST INFRASTRUCTURE ONLY: the tests are its only users; the product library
never imports or executes anything here, and the two share no code.

* Spectral bisection (graph partitioning, Section 2): for prescribed sizes
  n1 + n2 = n, relaxing x_i = +-1/2 to real x with x'x = n/4 and
  e'x = (n1 - n2)/2 gives min x'Gx = n1 n2 lambda_2 / n, reached at
  x = (n1 - n2)/(2n) e + sqrt(n1 n2 / n) v_2 (v_2 the Fiedler vector).  The
  partition takes the n1 vertices where that x is smallest, i.e. where v_2
  is smallest; equal entries go by vertex index (a reading: the paper does
  not say how to round).  Its cut size is x'Gx for x_i = +-1/2, eq. (1), the
  sum of the weights of the edges between the two sides.
* Approximations of the pseudo-inverse G^+ (current-flow betweenness):
      T^(k) = sum_{j=2..k} (1/lambda_j) v_j v_j'
      S^(k) = (1/sigma) I - (1/sigma) v_1 v_1' + sum_{j=2..k} (1/lambda_j - 1/sigma) v_j v_j'
  (the paper's second expression of S^(k), which equals
  T^(k) + (1/sigma) sum_{j>k} v_j v_j' for a complete orthonormal set).
  Reading for graphs with several components: the zero pairs (one per
  component) take the place of v_1, and j runs over the positive ones.
"""
from __future__ import annotations

import numpy as np


def bisect(L, fiedler, n1):
    """part (0 for the n1 vertices with the smallest Fiedler entries, ties
    by index; 1 for the others) and the cut size, by plain loops over the
    sorted order and the edges."""
    n = L.n
    f = np.asarray(fiedler, dtype=np.float64)
    order = np.lexsort((np.arange(n), f))  # by value, then by index
    part = np.ones(n, dtype=np.int32)
    part[order[:n1]] = 0
    cut = 0.0
    for i in range(n):
        for p in range(L.rowptr[i], L.rowptr[i + 1]):
            j = int(L.col[p])
            if j > i and part[i] != part[j]:
                cut += -float(L.val[p])  # the weight of edge (i, j)
    return part, cut


def relaxed_optimum(n1, n, lam2, v2):
    """x = (n1 - n2)/(2n) e + sqrt(n1 n2 / n) v_2 and its value n1 n2 lambda_2 / n."""
    n2 = n - n1
    x = (n1 - n2) / (2.0 * n) * np.ones(n) + np.sqrt(n1 * n2 / n) * np.asarray(v2, dtype=np.float64)
    return x, n1 * n2 * lam2 / n


def pinv_T(evals, evecs, X):
    """T^(k) X = sum over the positive pairs of (1/lambda_j) v_j (v_j' X)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.zeros_like(X)
    for j, lam in enumerate(evals):
        if lam > 0.0:
            v = evecs[:, j]
            Y += np.outer(v, v @ X) / lam if X.ndim == 2 else v * (v @ X) / lam
    return Y


def pinv_S(evals, evecs, sigma, X):
    """S^(k) X = X/sigma - (1/sigma) sum over the zero pairs v (v'X)
    + sum over the positive pairs (1/lambda_j - 1/sigma) v_j (v_j' X)."""
    X = np.asarray(X, dtype=np.float64)
    Y = X / sigma
    for j, lam in enumerate(evals):
        v = evecs[:, j]
        c = (1.0 / lam - 1.0 / sigma) if lam > 0.0 else -1.0 / sigma
        Y = Y + (np.outer(v, v @ X) if X.ndim == 2 else v * (v @ X)) * c
    return Y
