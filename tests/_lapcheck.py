"""Comparison helpers shared by the tests: cluster-aware eigenpair checks.

Eigenvectors are unique only up to sign (simple eigenvalue) or rotation
(repeated or tightly clustered eigenvalues), so vectors are compared by the
largest principal angle between the spans of matching clusters.
"""
from __future__ import annotations

import numpy as np


def clusters(evals, rel_gap=1e-2, abs_gap=1e-9):
    """Group ascending eigenvalues: i and i+1 share a cluster when
    lam[i+1] - lam[i] < rel_gap * lam[i+1] + abs_gap."""
    out, cur = [], [0]
    for i in range(1, len(evals)):
        if evals[i] - evals[i - 1] < rel_gap * abs(evals[i]) + abs_gap:
            cur.append(i)
        else:
            out.append(cur)
            cur = [i]
    out.append(cur)
    return out


def orthonormal(X):
    q, _ = np.linalg.qr(X)
    return q


def sin_largest_angle(X, Y):
    """sin of the largest principal angle between span(X) and span(Y),
    measured as ||(I - P_Y) X||_2 with both bases orthonormalized;
    requires dim span(X) <= dim span(Y)."""
    Xo, Yo = orthonormal(X), orthonormal(Y)
    R = Xo - Yo @ (Yo.T @ Xo)
    return float(np.linalg.norm(R, 2)) if R.size else 0.0


def residuals(Lsp, evals, evecs):
    """||L x_j - lam_j x_j|| / ||x_j|| per pair."""
    R = Lsp @ evecs - evecs * evals[None, :]
    return np.linalg.norm(R, axis=0) / np.linalg.norm(evecs, axis=0)


def check_against_reference(evals, evecs, ref_evals, ref_evecs, *, val_rtol, val_atol=1e-12,
                            angle_tol, rel_gap=1e-2):
    """Compare k computed pairs with a reference that holds at least k pairs
    (more when the k-th sits inside a cluster).  Returns a dict of the
    worst errors; asserts the bounds."""
    k = len(evals)
    assert len(ref_evals) >= k
    err = np.abs(evals - ref_evals[:k])
    bound = val_rtol * np.abs(ref_evals[:k]) + val_atol
    assert np.all(err <= bound), f"eigenvalue mismatch: {err} vs bound {bound}"
    worst = 0.0
    for c in clusters(ref_evals, rel_gap):
        inside = [i for i in c if i < k]
        if not inside:
            continue
        # a cluster can only be compared when the reference shows where it
        # ends, i.e. holds the next, separated eigenvalue as well
        if max(c) + 1 >= len(ref_evals):
            continue
        s = sin_largest_angle(evecs[:, inside], ref_evecs[:, c])
        worst = max(worst, s)
        assert s <= angle_tol, f"subspace angle {s:.3e} > {angle_tol} in cluster {c}"
    return {"max_val_err": float(err.max()) if k else 0.0, "max_sin": worst}
