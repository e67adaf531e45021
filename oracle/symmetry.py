"""Symmetry reduction of the stiffness matrix, plain numpy (test
infrastructure only, like the rest of ``oracle/``).

Sec. 7 (exploiting symmetry): for a rotation B with B^K = Id mapping the
domain and the data to themselves, symmetric functions u(Bx) = u(x) are
spanned by the orbit sums Phi_I = sum of the hat functions of the images of
a representative vertex I, and the bilinear form satisfies a(u, v) = K
a_omega(u, v) with the effective kernel over the sector.  The reduced
system is therefore written here from the full one, without the effective
kernel:

  A_red = P^T A_full P / K,    b_red = P^T b_full / K,

P the 0/1 matrix mapping each full DOF to the DOF of its representative.
This is the definition of the reduced operator.  The same operator as a
sum over cell pairs (what the effective kernel amounts to: every pair of
sector cells with each image of the second cell) is `assemble_reduced`:
pairs of the full mesh weighted by the mean of w_K, w_L (w = 1 on the
sector, 0 on the images), identical pairs and the boundary term by w_K,
vertices folded onto their representatives.  The two agree up to the
quadrature rules' lack of exact rotation invariance (rotated copies of a
pair can fall on either side of a distance-class threshold).
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def fold_matrix(dofs_full, vfold):
    """(P, reduced DOF vertices): P[i, I] = 1 if full DOF i (vertex
    dofs_full[i]) has the representative vertex of reduced DOF I."""
    dofs_full = np.asarray(dofs_full)
    rep = np.asarray(vfold)[dofs_full]
    red = np.unique(rep)
    col = np.searchsorted(red, rep)
    P = np.zeros((len(dofs_full), len(red)))
    P[np.arange(len(dofs_full)), col] = 1.0
    return P, red


def reduce(A_full, b_full, dofs_full, vfold, K):
    P, red = fold_matrix(dofs_full, vfold)
    return P.T @ A_full @ P / K, P.T @ b_full / K, red


def assemble_reduced(mesh, s, orders, vfold, T_omega, mode="paper", pre=None, rot=None, K=0):
    """Reduced matrix (representative DOFs, increasing vertex order) by the
    weighted pair sum over the full mesh (sector cells first).  With pre /
    rot / K (preimage sector cell and rotation index of every cell) one
    member of each equal couple of cross pairs (S, B^i T) ~ (T, B^-i S)
    counts, with weight 1."""
    nv = len(mesh["verts"])
    T = len(mesh["cells"])
    w = np.zeros(T)
    w[:T_omega] = 1.0
    An, cnt = O.assemble_full(mesh, s, orders, cell_w=w, cell_pre=pre, cell_rot=rot, sym_order=K)
    vfold = np.asarray(vfold)
    dofs = O.dof_nodes(nv, mesh["bfacets"], s, mode)
    red = np.unique(vfold[dofs])
    # fold the DOF rows and columns (entries of non-DOF vertices are never
    # used: for s >= 1/2 those of boundary vertices diverge)
    F = np.zeros((len(dofs), len(red)))
    pos = {v: i for i, v in enumerate(red)}
    for i, v in enumerate(dofs):
        F[i, pos[vfold[v]]] = 1.0
    return F.T @ An[np.ix_(dofs, dofs)] @ F, red, cnt


def load_vector_reduced(mesh, vfold, T_omega, red):
    """f = 1: sum over the sector cells around each representative of |K|/(d+1)."""
    d = mesh["dim"]
    V = np.asarray(mesh["verts"], dtype=np.float64).reshape(-1, d)
    C = np.asarray(mesh["cells"])
    pos = {int(v): i for i, v in enumerate(red)}
    b = np.zeros(len(red))
    for c in C[:T_omega]:
        P = V[c]
        if d == 1:
            meas = abs(P[1, 0] - P[0, 0])
        else:
            meas = 0.5 * abs((P[1, 0] - P[0, 0]) * (P[2, 1] - P[0, 1]) - (P[2, 0] - P[0, 0]) * (P[1, 1] - P[0, 1]))
        for v in c:
            r = int(vfold[v])
            if r in pos:
                b[pos[r]] += meas / (d + 1)
    return b
