"""Strong form of the fractional Laplacian of a P1 function and the
Babuska-Rheinboldt type error indicators, plain numpy (test
infrastructure only, like the rest of ``oracle/``).

Sec. 4 of arXiv:1708.03912 (lemma on the strong form, eq. 8 for
s != 1 - d/2; eq. 9, the logarithmic form, for d = 1, s = 1/2): for x in
the element K0,

  (-Delta)^s u(x) / C(d,s)
    =  1/(d+2s-2) int_{dK0} grad u|K0 . n |x-y|^{-(d+2s-2)} dy
     - u(x)/(2s)  int_{dK0} n . (x-y) |x-y|^{-(d+2s)} dy
     + sum_{K != K0} [ 1/(2s(d+2s-2)) int_{dK} grad u|K . n |x-y|^{-(d+2s-2)} dy
                       - 1/(2s) int_{dK} u(y) n . (x-y) |x-y|^{-(d+2s)} dy ]

with n the outward normal of each element (eq. 9: |x-y|^{-(d+2s-2)}/(d+2s-2)
becomes log(1/|x-y|), i.e. the coefficients 1/(d+2s-2) and 1/(2s(d+2s-2))
become 1 and 1/(2s)).  In d = 1 the boundary of an element is its two end
points and the boundary integrals are point values; and the indicators (eq. for
eta-hat_i) eta_i^2 = sum_{K containing node i} h_K^{2s} ||f - (-Delta)^s u||^2_{L2(K)}.

Rule (the paper says the edge integrals are regular and standard rules
apply; choices shared with the library): q-point Gauss-Legendre on every
edge, q_near points for the edges of K0 and of every element sharing a
vertex with K0, q_far points otherwise; the strong form is evaluated at the
k_eval x k_eval collapsed Gauss points of each element, which also give the
L2 norms.  Written per element and per edge as in the formula (no
cancellation across shared edges).
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def _elements(mesh):
    V = np.asarray(mesh["verts"], dtype=np.float64).reshape(-1, 2)
    C = np.asarray(mesh["cells"], dtype=np.int64)
    P = V[C]                                   # (T, 3, 2)
    a, b, c = P[:, 0], P[:, 1], P[:, 2]
    det = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1])
    return V, C, P, det


def _dim(mesh):
    return np.asarray(mesh["cells"]).shape[1] - 1


def eval_points(mesh, k_eval):
    """Evaluation points of every element.  d = 2: collapsed Gauss points,
    (T, k^2, 2) coordinates, (T, k^2, 3) barycentric coordinates and
    (T, k^2) weights times |K|.  d = 1: k Gauss-Legendre points, (T, k, 1),
    (T, k, 2) and (T, k)."""
    if _dim(mesh) == 1:
        V = np.asarray(mesh["verts"], dtype=np.float64).reshape(-1)
        C = np.asarray(mesh["cells"], dtype=np.int64)
        t, w = O.gauss_legendre01(k_eval)
        lam = np.stack([1 - t, t], axis=1)                            # (k, 2)
        X = (lam[None, :, :] * V[C][:, None, :]).sum(-1)[..., None]
        W = np.abs(V[C[:, 1]] - V[C[:, 0]])[:, None] * w[None, :]
        return X, np.broadcast_to(lam, (len(C), k_eval, 2)), W
    V, C, P, det = _elements(mesh)
    ux, uw = O.gauss_jacobi01(k_eval, 1.0, 0.0)
    vx, vw = O.gauss_legendre01(k_eval)
    lam, w = [], []
    for i in range(k_eval):
        for j in range(k_eval):
            l1, l2 = ux[i], (1 - ux[i]) * vx[j]
            lam.append((1 - l1 - l2, l1, l2))
            w.append(2 * uw[i] * vw[j])
    lam = np.array(lam)                        # (Q, 3)
    X = np.einsum("qa,tad->tqd", lam, P)
    W = np.abs(det)[:, None] * 0.5 * np.array(w)[None, :]
    return X, np.broadcast_to(lam, (len(C), len(lam), 3)), W


def _strong_form_1d(mesh, dofs, u, s, k_eval):
    """d = 1: each element [a, b] contributes at its two end points p with
    the outward normal n_p = sign(p - other end point)."""
    V = np.asarray(mesh["verts"], dtype=np.float64).reshape(-1)
    C = np.asarray(mesh["cells"], dtype=np.int64)
    nod = np.zeros(len(V))
    nod[np.asarray(dofs)] = u
    X, lam, _ = eval_points(mesh, k_eval)
    X = X[..., 0]                                                     # (T, k)
    ux = (lam * nod[C][:, None, :]).sum(-1)
    log_case = abs(s - 0.5) < 1e-15                                   # s = 1 - d/2
    d2 = 2.0 * s - 1.0
    out = np.zeros_like(X)
    for K in range(len(C)):
        a, b = V[C[K]]
        g = (nod[C[K, 1]] - nod[C[K, 0]]) / (b - a)                    # u' on K
        for p, q, up in ((a, b, nod[C[K, 0]]), (b, a, nod[C[K, 1]])):
            n = np.sign(p - q)
            dx = X - p
            r = np.abs(dx)
            gk = np.log(1.0 / r) if log_case else r ** (-d2)
            cg_own, cg = (1.0, 1.0 / (2 * s)) if log_case else (1.0 / d2, 1.0 / (2 * s * d2))
            ku = n * dx * r ** (-(1.0 + 2 * s))
            own = np.zeros(len(C), dtype=bool)
            own[K] = True
            out += np.where(own[:, None], cg_own * g * n * gk - ux / (2 * s) * ku,
                            cg * g * n * gk - up / (2 * s) * ku)
    return O.cdn(1, s) * out


def strong_form(mesh, dofs, u, s, k_eval=2, q_far=2, q_near=12, cells=None):
    """(-Delta)^s u_h at the evaluation points, (T, k_eval^d).  u: values on
    the DOFs (zero at the other vertices).  q_far / q_near: edge rules in
    d = 2 (unused in d = 1).  cells: evaluate only in these cells (rows in
    that order)."""
    if _dim(mesh) == 1:
        out = _strong_form_1d(mesh, dofs, u, s, k_eval)
        return out if cells is None else out[np.asarray(cells)]
    V, C, P, det = _elements(mesh)
    T = len(C)
    nod = np.zeros(len(V))
    nod[np.asarray(dofs)] = u
    U = nod[C]                                 # (T, 3)
    # gradient of u on each element: solve [b-a; c-a] g = [ub-ua; uc-ua]
    Ex = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]], axis=1)      # (T, 2, 2)
    du = np.stack([U[:, 1] - U[:, 0], U[:, 2] - U[:, 0]], axis=1)
    G = np.linalg.solve(Ex, du[..., None])[..., 0]                     # (T, 2)
    sgn = np.sign(det)                                                 # +1 counter-clockwise
    X, lam, _ = eval_points(mesh, k_eval)
    ux = np.einsum("tqa,ta->tq", lam, U)                               # u at the points
    tc = np.arange(T) if cells is None else np.asarray(cells)
    X, ux = X[tc], ux[tc]
    d2 = 2.0 * s                                                       # d + 2s - 2, d = 2
    tf, wf = O.gauss_legendre01(q_far)
    tn, wn = O.gauss_legendre01(q_near)
    out = np.zeros(X.shape[:2])
    vid = C
    for K in range(T):
        near = np.isin(vid[tc], vid[K]).any(axis=1)                    # target cells sharing a vertex with K
        for e in range(3):
            A_, B_ = P[K, e], P[K, (e + 1) % 3]
            ua, ub = U[K, e], U[K, (e + 1) % 3]
            dx, dy = B_ - A_
            N = sgn[K] * np.array([dy, -dx])                           # outward normal times |e|
            gN = G[K] @ N
            for (tq, wq, sel) in ((tf, wf, ~near), (tn, wn, near)):
                if not sel.any():
                    continue
                Xs = X[sel]                                            # (m, Q, 2)
                own = np.zeros(sel.sum(), dtype=bool)
                own[tc[sel] == K] = True
                Y = A_[None, :] + tq[:, None] * (B_ - A_)[None, :]     # (q, 2)
                Dv = Xs[:, :, None, :] - Y[None, None, :, :]           # (m, Q, q, 2)
                r2 = (Dv ** 2).sum(-1)
                kern = r2 ** (-(1.0 + s))                              # |x-y|^{-(d+2s)}
                kg = kern * r2                                         # |x-y|^{-(d+2s-2)}
                nd = Dv @ N                                            # n.(x-y) |e|
                uy = ua + tq * (ub - ua)
                Ig = (kg * wq).sum(-1) * gN                            # int grad u . n |x-y|^{-(d+2s-2)}
                Iu_own = (kern * nd * wq).sum(-1)                      # int n.(x-y) |x-y|^{-(d+2s)}
                Iu = (kern * nd * wq * uy).sum(-1)                     # int u(y) n.(x-y) ...
                val = np.where(own[:, None],
                               Ig / d2 - ux[sel] / (2 * s) * Iu_own,
                               Ig / (2 * s * d2) - Iu / (2 * s))
                out[sel] += val
    return O.cdn(2, s) * out


def indicators(mesh, dofs, u, s, Lu, k_eval=2, f=None):
    """eta_K^2 = h_K^{2s} ||f - Lu||^2_{L2(K)} (collapsed rule) and the nodal
    eta_i^2 = sum over the elements containing vertex i.  f: values at the
    evaluation points (default 1).  Returns (eta_K^2 (T,), eta_i^2 (nv,))."""
    _, _, W = eval_points(mesh, k_eval)
    fv = np.ones_like(Lu) if f is None else f
    C = np.asarray(mesh["cells"], dtype=np.int64)
    if _dim(mesh) == 1:
        V = np.asarray(mesh["verts"], dtype=np.float64).reshape(-1)
        h2 = (V[C[:, 1]] - V[C[:, 0]]) ** 2
    else:
        V, C, P, det = _elements(mesh)
        h2 = ((P[:, [1, 2, 0]] - P) ** 2).sum(-1).max(1)
    ek = h2 ** s * (W * (fv - Lu) ** 2).sum(1)
    en = np.zeros(len(V))
    for a in range(C.shape[1]):
        np.add.at(en, C[:, a], ek)
    return ek, en
