"""Geometric multigrid for the dense fractional-Laplacian system, plain
numpy (test infrastructure only, like the rest of ``oracle/``).

Sec. 5 (end) of arXiv:1708.03912 proposes geometric multigrid on nested
meshes as the solver whose iteration count stays bounded under refinement
(unlike Jacobi-preconditioned CG, whose count grows like n^(s/d)); the
paper gives no cycle details.  Reading used here and by the library:

* nested uniform refinements; the prolongation P_l takes a coarse P1
  function to the same function on the fine mesh (fine nodal values: the
  coarse value at inherited vertices, the mean of the two parents at edge
  midpoints), restricted to the DOFs of each level (Sec. 3 rule);
* Galerkin coarse operators A_{l-1} = P_l^T A_l P_l (no coarse quadrature);
* V(2,2) cycle, damped Jacobi smoothing with omega = 2/3, exact solve on the
  coarsest level (Cholesky);
* used as the preconditioner of CG (one cycle from a zero guess), which
  keeps the preconditioner symmetric positive definite.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

OMEGA = 2.0 / 3.0
NU = 2


def prolongation(parents, dofs_c, dofs_f, nv_c):
    """Dense P (n_f x n_c) between the DOF sets of two nested levels.
    parents: (nv_f, 2) coarse parent vertices of each fine vertex."""
    col = np.full(nv_c, -1)
    col[np.asarray(dofs_c)] = np.arange(len(dofs_c))
    P = np.zeros((len(dofs_f), len(dofs_c)))
    for r, v in enumerate(np.asarray(dofs_f)):
        a, b = parents[v]
        if a == b:
            if col[a] >= 0:
                P[r, col[a]] = 1.0
        else:
            for p in (a, b):
                if col[p] >= 0:
                    P[r, col[p]] += 0.5
    return P


def galerkin(A, P):
    return P.T @ A @ P


def _jacobi(A, d, x, b, steps):
    for _ in range(steps):
        x = x + OMEGA * (b - A @ x) / d
    return x


def vcycle(As, Ps, b, level=None, chol=None):
    """One V(NU, NU) cycle from x = 0 on level ``level`` (default: finest).
    As[l]: operators, coarsest first; Ps[l] prolongs level l-1 to l."""
    if level is None:
        level = len(As) - 1
    A = As[level]
    if level == 0:
        c = chol if chol is not None else scipy.linalg.cho_factor(A)
        return scipy.linalg.cho_solve(c, b)
    d = np.diag(A)
    x = _jacobi(A, d, np.zeros_like(b), b, NU)
    r = b - A @ x
    x = x + Ps[level] @ vcycle(As, Ps, Ps[level].T @ r, level - 1, chol)
    return _jacobi(A, d, x, b, NU)


def mg_pcg(As, Ps, b, rtol=1e-12, maxit=1000):
    """CG on As[-1] u = b preconditioned by one V-cycle; x0 = 0, stop at
    ||r|| <= rtol ||b||.  Returns (u, iterations)."""
    A = As[-1]
    chol = scipy.linalg.cho_factor(As[0])
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.linalg.norm(b)
    if bn == 0:
        return x, 0
    z = vcycle(As, Ps, r, chol=chol)
    p = z.copy()
    rz = r @ z
    for it in range(maxit):
        if np.linalg.norm(r) <= rtol * bn:
            return x, it
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = vcycle(As, Ps, r, chol=chol)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit


def hierarchy_operators(A_fine, parents_list, dofs_list, nv_list):
    """Galerkin operators of every level (coarsest first) and the
    prolongations, from the finest matrix and the nested-mesh data."""
    L = len(dofs_list)
    Ps = [None] * L
    for l in range(1, L):
        Ps[l] = prolongation(parents_list[l - 1], dofs_list[l - 1], dofs_list[l], nv_list[l - 1])
    As = [None] * L
    As[-1] = A_fine
    for l in range(L - 1, 0, -1):
        As[l - 1] = galerkin(As[l], Ps[l])
    return As, Ps
