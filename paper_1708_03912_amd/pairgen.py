"""Seeded random inputs for the learned pair-integral surrogate.

Like ``meshgen`` this module only builds inputs -- pair geometries, values
of s and starting weights -- and holds none of the method's arithmetic.  It
is shared by the library's callers (benchmark, tests) and the oracle's
tests.

``sample_pairs`` draws separated triangle pairs of the kind that the order
rule of App. B puts into its closest classes (Sec. 5 element-pair
decomposition): both triangles shape-regular (every angle at least
``min_angle`` degrees), longest-edge ratio log-uniform in ``size_ratio``,
centroid distance over the larger longest edge uniform in ``r_range``, and
a gap of at least ``min_gap`` larger longest edges between the closed
triangles.  The whole pair is then scaled and shifted at random (the
surrogate's targets do not depend on that).

``glorot_params`` draws starting weights for the 9-64-64-21 network in the
padded layout the library uses (see ``param_layout``).
"""
from __future__ import annotations

import math

import numpy as np

NIN, NH, NOUT = 9, 64, 21   # network widths
KIN, KOUT = 32, 32          # padded input / output widths


def param_layout():
    """(name, shape) of the packed parameter vector, in order: W1 (NH x KIN,
    columns >= NIN zero), b1, W2 (NH x NH), b2, W3 (KOUT x NH, rows >= NOUT
    zero), b3 (KOUT, entries >= NOUT zero)."""
    return [("W1", (NH, KIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
            ("W3", (KOUT, NH)), ("b3", (KOUT,))]


def n_params():
    return sum(int(np.prod(sh)) for _, sh in param_layout())


def glorot_params(seed: int) -> np.ndarray:
    """Glorot-uniform weights (fan-in / fan-out of the unpadded layers),
    zero biases, zero padding; float64 vector of n_params()."""
    rng = np.random.default_rng(seed)
    out = []
    fans = {"W1": (NIN, NH), "W2": (NH, NH), "W3": (NH, NOUT)}
    for name, sh in param_layout():
        a = np.zeros(sh)
        if name in fans:
            fi, fo = fans[name]
            lim = math.sqrt(6.0 / (fi + fo))
            rows = NOUT if name == "W3" else sh[0]
            cols = NIN if name == "W1" else sh[1]
            a[:rows, :cols] = rng.uniform(-lim, lim, size=(rows, cols))
        out.append(a.ravel())
    return np.concatenate(out)


def _triangles(rng, m, min_angle):
    """m triangles (m, 3, 2) with longest edge 1, every angle >= min_angle
    degrees, random rotation and vertex order."""
    out = np.empty((m, 3, 2))
    i = 0
    while i < m:
        n = 2 * (m - i) + 16
        A = rng.uniform(min_angle, 180.0 - 2 * min_angle, n)
        B = rng.uniform(min_angle, 180.0, n)
        C = 180.0 - A - B
        ok = C >= min_angle
        A, B = np.radians(A[ok]), np.radians(B[ok])
        # vertices (0,0), (1,0) and the apex from the two base angles
        t = np.sin(B) / np.sin(A + B)
        P = np.zeros((len(A), 3, 2))
        P[:, 1, 0] = 1.0
        P[:, 2, 0] = t * np.cos(A)
        P[:, 2, 1] = t * np.sin(A)
        L = np.sqrt(((P[:, [1, 2, 0]] - P) ** 2).sum(-1)).max(1)
        P /= L[:, None, None]
        rot = rng.uniform(0, 2 * math.pi, len(A))
        c, s = np.cos(rot), np.sin(rot)
        P = np.stack([c[:, None] * P[..., 0] - s[:, None] * P[..., 1],
                      s[:, None] * P[..., 0] + c[:, None] * P[..., 1]], -1)
        perm = np.argsort(rng.random((len(A), 3)), axis=1)
        P = np.take_along_axis(P, perm[:, :, None].repeat(2, 2), 1)
        k = min(len(A), m - i)
        out[i:i + k] = P[:k]
        i += k
    return out


def _seg_dist(p, a, b):
    ab = b - a
    t = np.clip(((p - a) * ab).sum(-1) / (ab * ab).sum(-1), 0.0, 1.0)
    return np.sqrt(((p - (a + t[:, None] * ab)) ** 2).sum(-1))


def gap(X, Y):
    """Distance between two disjoint closed triangles (m, 3, 2) each: the
    smallest vertex-to-edge distance."""
    d = np.full(len(X), np.inf)
    for P, Q in ((X, Y), (Y, X)):
        for i in range(3):
            for j in range(3):
                d = np.minimum(d, _seg_dist(P[:, i], Q[:, j], Q[:, (j + 1) % 3]))
    return d


def sample_pairs(seed: int, m: int, r_range=(0.75, 3.0), size_ratio=(0.25, 4.0),
                 s_range=(0.05, 0.95), min_angle=25.0, min_gap=0.3, scale_range=(0.005, 1.0)):
    """m separated triangle pairs.  Returns X (m, 6), Y (m, 6) row-major
    vertex coordinates and s (m,)."""
    rng = np.random.default_rng(seed)
    Xs, Ys = [], []
    got = 0
    while got < m:
        n = 2 * (m - got) + 64
        K = _triangles(rng, n, min_angle)
        T = _triangles(rng, n, min_angle)
        lam = np.exp(rng.uniform(math.log(size_ratio[0]), math.log(size_ratio[1]), n))
        T *= lam[:, None, None]
        hm = np.maximum(1.0, lam)
        r = rng.uniform(r_range[0], r_range[1], n)
        ang = rng.uniform(0, 2 * math.pi, n)
        shift = K.mean(1) - T.mean(1) + (r * hm)[:, None] * np.stack([np.cos(ang), np.sin(ang)], 1)
        T += shift[:, None, :]
        ok = gap(K, T) >= min_gap * hm
        K, T = K[ok], T[ok]
        sc = np.exp(rng.uniform(math.log(scale_range[0]), math.log(scale_range[1]), len(K)))
        off = rng.uniform(-1, 1, (len(K), 2))
        K = K * sc[:, None, None] + off[:, None, :]
        T = T * sc[:, None, None] + off[:, None, :]
        Xs.append(K.reshape(-1, 6))
        Ys.append(T.reshape(-1, 6))
        got += len(K)
    X = np.concatenate(Xs)[:m]
    Y = np.concatenate(Ys)[:m]
    s = rng.uniform(s_range[0], s_range[1], m)
    return np.ascontiguousarray(X), np.ascontiguousarray(Y), s


def mesh_band_pairs(mesh, seed: int, m: int, r_max: float = 3.0, s_range=(0.05, 0.95)):
    """m separated element pairs of a triangle mesh (no common vertex) whose
    centroid distance is below r_max times the larger longest edge -- the
    pairs the closest classes of the order rule hold.  Each draw takes a
    random element K and a random such partner no larger than K.  Returns
    X (m, 6), Y (m, 6) vertex coordinates and s (m,) uniform in s_range."""
    from scipy.spatial import cKDTree
    V = np.asarray(mesh["verts"], dtype=np.float64)
    C = np.asarray(mesh["cells"], dtype=np.int64)
    P = V[C]
    cen = P.mean(1)
    h = np.sqrt(((P[:, [1, 2, 0]] - P) ** 2).sum(-1)).max(1)
    rng = np.random.default_rng(seed)
    tree = cKDTree(cen)
    Xs, Ys = [], []
    while len(Xs) < m:
        K = int(rng.integers(len(C)))
        idx = np.asarray(tree.query_ball_point(cen[K], r_max * h[K]), dtype=np.int64)
        idx = idx[(h[idx] <= h[K]) & (idx != K)]
        if len(idx):
            shared = (C[idx][:, :, None] == C[K][None, None, :]).any(-1).any(-1)
            idx = idx[~shared]
        if len(idx) == 0:
            continue
        j = int(idx[rng.integers(len(idx))])
        if ((cen[K] - cen[j]) ** 2).sum() >= (r_max * h[K]) ** 2:
            continue
        Xs.append(P[K].ravel())
        Ys.append(P[j].ravel())
    s = rng.uniform(s_range[0], s_range[1], m)
    return np.ascontiguousarray(Xs), np.ascontiguousarray(Ys), s
