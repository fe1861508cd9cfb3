"""Plain FP64 reference of the Implicitly Restarted Lanczos Method on the
inverse (Section 3.1, Algorithm 1 right): Lanczos on G^+ (the inverse of G
on the complement of its zero space), each step solving G w = v by the
oracle's PCG, restarted so that the wanted (largest) Ritz values of G^+,
the reciprocals of the smallest nonzero eigenvalues of G, converge.

TEST INFRASTRUCTURE ONLY: the tests are its only users; the product library
never imports or executes anything here, and the two share no code.

Readings (the paper describes ARPACK's method without its details):
* restart: thick restart with the wanted Ritz vectors and the last Lanczos
  vector (Wu & Simon), which with exact shifts spans the same space as
  Sorensen's implicit restart; full reorthogonalization (classical
  Gram-Schmidt twice) keeps the basis orthonormal;
* the zero space: the normalized component indicators are the zero pairs
  (as in JD); v_1 and every Lanczos vector stay orthogonal to them, and
  the inner PCG solves on their complement (Q = the indicators, theta = 0);
* Krylov size m = max(3 (k - zeros), k - zeros + 6) (the paper: about three
  times the number of wanted pairs), p = wanted + (m - wanted) / 2 vectors
  kept at a restart;
* inner tolerance ||v - G w|| <= rtol_pcg ||v|| with rtol_pcg = 1e-12 (the
  paper: proportional to the accuracy wanted; a residual of G^+ is
  amplified by up to ||G|| in the residual of G);
* a pair is accepted with JD's certificate ||G u - lambda u|| <= tol
  min(lambda, 1), lambda = u'Gu from a fresh product; the run stops when
  every wanted pair holds it.
"""
from __future__ import annotations

import numpy as np

import oracle


def _zero_space(L):
    nc, lab = oracle.components(L)
    Z = np.zeros((L.n, nc))
    for c in range(nc):
        Z[lab == c, c] = 1.0
    return Z / np.sqrt(Z.sum(axis=0))


def irlm(L, k, tol, *, precond=oracle.PREC_JACOBI, rtol_pcg=1e-12, itmax_pcg=5000, m=None,
         max_restarts=200, seed=1):
    """(evals ascending, evecs n x k, info dict with restarts, lanczos_steps,
    inner iterations and products)."""
    n = L.n
    Z = _zero_space(L)
    nz = min(Z.shape[1], k)
    want = k - nz
    evals = [0.0] * nz
    evecs = [Z[:, c] for c in range(nz)]
    info = {"restarts": 0, "lanczos_steps": 0, "inner": 0, "mvp": 0}
    if want == 0:
        return np.array(evals), np.stack(evecs, axis=1), info
    if m is None:
        m = max(3 * want, want + 6)
    m = min(m, n - Z.shape[1])
    p = want + (m - want) // 2
    G = L.to_scipy()

    def solve(v):
        # G w = v on the complement of the zero space: the projected PCG of
        # Algorithm 2 step 8 with theta = 0 solves (G) t = -r for r = -v
        t, its, br = oracle.pcg_correction(L, 0.0, Z, -v, precond=precond, itmax=itmax_pcg, rtol=rtol_pcg)
        info["inner"] += its
        info["mvp"] += its
        return t

    # v_1: the seeded start vector of JD, orthogonal to the zero space, unit length
    v = np.array([oracle.start_value(seed, i) for i in range(n)])
    v -= Z @ (Z.T @ v)
    v /= np.linalg.norm(v)
    V = np.zeros((n, m + 1))
    V[:, 0] = v
    T = np.zeros((m, m))
    j0 = 0
    beta = 0.0
    for restart in range(max_restarts + 1):
        for j in range(j0, m):
            w = solve(V[:, j])
            info["lanczos_steps"] += 1
            # full reorthogonalization against V[:, :j+1] (twice) and the zero space
            h = V[:, :j + 1].T @ w
            w -= V[:, :j + 1] @ h
            h2 = V[:, :j + 1].T @ w
            w -= V[:, :j + 1] @ h2
            h += h2
            w -= Z @ (Z.T @ w)
            if j == j0 and j0 > 0:
                T[:j, j] = h[:j]  # the arrow of a thick restart
                T[j, :j] = h[:j]
            elif j > 0:
                T[j - 1, j] = T[j, j - 1] = h[j - 1]
            T[j, j] = h[j]
            beta = np.linalg.norm(w)
            V[:, j + 1] = w / beta
            if j + 1 < m:
                T[j, j + 1] = T[j + 1, j] = beta
        mu, Y = np.linalg.eigh(T)
        order = np.argsort(-mu)  # largest Ritz values of G^+ first
        mu, Y = mu[order], Y[:, order]
        U = V[:, :m] @ Y[:, :want]
        lam = 1.0 / mu[:want]
        ok = True
        res = []
        for i in range(want):
            u = U[:, i] / np.linalg.norm(U[:, i])
            gu = G @ u
            info["mvp"] += 1
            th = float(u @ gu)
            rn = float(np.linalg.norm(gu - th * u))
            res.append((th, rn, u))
            if rn > tol * min(th, 1.0):
                ok = False
        if ok:
            for th, rn, u in res:
                evals.append(th)
                evecs.append(u)
            info["restarts"] = restart
            order = np.argsort(evals)
            return np.array(evals)[order], np.stack(evecs, axis=1)[:, order], info
        # thick restart: the p largest Ritz vectors and the last Lanczos vector
        Vn = np.zeros_like(V)
        Vn[:, :p] = V[:, :m] @ Y[:, :p]
        Vn[:, p] = V[:, m]
        V = Vn
        T = np.zeros((m, m))
        T[np.arange(p), np.arange(p)] = mu[:p]
        s = beta * Y[m - 1, :p]
        T[:p, p] = s
        T[p, :p] = s
        j0 = p
    raise RuntimeError("IRLM did not converge")
