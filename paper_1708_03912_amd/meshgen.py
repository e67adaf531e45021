"""Seeded synthetic meshes shaped like the paper's workloads.

This module only builds inputs: vertex coordinates, cells and boundary
facets.  It holds none of the method's arithmetic and is the one module
shared by the library's tests/benchmark and the oracle's tests.

Shapes (Sec. 7 of arXiv:1708.03912 uses the interval (-1,1), the unit disk
and an L-shaped domain; its adaptively refined meshes exist only as figures,
so seeded stand-ins are generated here):

* ``interval(N)``       -- uniform mesh of (-1,1) with N cells.
* ``disk(h, seed)``     -- unit disk: equispaced points on the circle, a
                           jittered hexagonal lattice inside, Delaunay.
* ``lshape(...)``       -- (-1,1)^2 minus [0,1)x(-1,0]: newest-vertex
                           bisection (conforming, no hanging nodes) graded
                           geometrically toward the re-entrant corner and the
                           boundary, size ratio up to 1:64.
* ``square3(N)``        -- structured three-direction mesh of (-1,1)^2.
* ``refine_uniform``,
  ``hierarchy``         -- nested uniform refinements (for multigrid), with
                           each fine vertex's coarse parents.

Every mesh is a dict with ``dim``, ``verts`` (nv x dim float64), ``cells``
(nc x (dim+1) int32) and ``bfacets`` (nb x dim int32).  Vertices and cells
are sorted along a Morton curve so that neighbouring indices are
neighbouring in space.
"""
from __future__ import annotations

import math

import numpy as np


def _morton_key(xy: np.ndarray, bits: int = 16) -> np.ndarray:
    lo = xy.min(axis=0)
    span = max(float((xy.max(axis=0) - lo).max()), 1e-300)
    q = np.floor((xy - lo) / span * ((1 << bits) - 1)).astype(np.uint64)
    key = np.zeros(len(xy), dtype=np.uint64)
    for b in range(bits):
        for d in range(xy.shape[1]):
            key |= ((q[:, d] >> np.uint64(b)) & np.uint64(1)) << np.uint64(xy.shape[1] * b + d)
    return key


def _finish(dim, verts, cells, bfacets, sort=True, want_perm=False):
    verts = np.asarray(verts, dtype=np.float64).reshape(-1, dim)
    cells = np.asarray(cells, dtype=np.int64).reshape(-1, dim + 1)
    bfacets = np.asarray(bfacets, dtype=np.int64).reshape(-1, dim)
    perm = np.arange(len(verts))
    if sort and dim == 2:
        perm = np.argsort(_morton_key(verts), kind="stable")
        inv = np.empty_like(perm)
        inv[perm] = np.arange(len(perm))
        verts = verts[perm]
        cells = inv[cells]
        bfacets = inv[bfacets]
        cen = verts[cells].mean(axis=1)
        cells = cells[np.argsort(_morton_key(cen), kind="stable")]
        # counter-clockwise orientation
        a, b, c = verts[cells[:, 0]], verts[cells[:, 1]], verts[cells[:, 2]]
        det = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1])
        neg = det < 0
        cells[neg] = cells[neg][:, [0, 2, 1]]
        bfacets = bfacets[np.lexsort((bfacets[:, 1], bfacets[:, 0]))]
    mesh = {"dim": dim, "verts": np.ascontiguousarray(verts),
            "cells": np.ascontiguousarray(cells, dtype=np.int32),
            "bfacets": np.ascontiguousarray(bfacets, dtype=np.int32)}
    return (mesh, perm) if want_perm else mesh


def refine_uniform(mesh):
    """One uniform refinement: every segment is halved, every triangle split
    into four by its edge midpoints (nested meshes for multigrid).  Returns
    (fine mesh, parents): parents[v] (nv_fine x 2, int32) are the two coarse
    vertices whose midpoint fine vertex v is, or (p, p) for a vertex inherited
    from coarse vertex p."""
    dim = mesh["dim"]
    V = np.asarray(mesh["verts"], dtype=np.float64).reshape(-1, dim)
    C = np.asarray(mesh["cells"], dtype=np.int64)
    B = np.asarray(mesh["bfacets"], dtype=np.int64)
    nv = len(V)
    if dim == 1:
        mid = nv + np.arange(len(C))
        verts = np.concatenate([V, 0.5 * (V[C[:, 0]] + V[C[:, 1]])])
        cells = np.concatenate([np.stack([C[:, 0], mid], 1), np.stack([mid, C[:, 1]], 1)])
        parents = np.concatenate([np.stack([np.arange(nv)] * 2, 1), C])
        # keep vertices ordered along the line
        order = np.argsort(verts[:, 0], kind="stable")
        inv = np.empty_like(order)
        inv[order] = np.arange(len(order))
        fine = _finish(1, verts[order], inv[cells], inv[B], sort=False)
        return fine, np.ascontiguousarray(parents[order], dtype=np.int32)
    edges = np.concatenate([C[:, [0, 1]], C[:, [1, 2]], C[:, [2, 0]]])
    key = np.sort(edges, axis=1)
    uniq, inv_e = np.unique(key, axis=0, return_inverse=True)
    inv_e = inv_e.reshape(-1)
    mid = nv + inv_e.reshape(3, -1).T  # midpoint of edges (01, 12, 20) of each cell
    verts = np.concatenate([V, 0.5 * (V[uniq[:, 0]] + V[uniq[:, 1]])])
    m01, m12, m20 = mid[:, 0], mid[:, 1], mid[:, 2]
    cells = np.concatenate([np.stack([C[:, 0], m01, m20], 1), np.stack([m01, C[:, 1], m12], 1),
                            np.stack([m20, m12, C[:, 2]], 1), np.stack([m01, m12, m20], 1)])
    bkey = np.sort(B, axis=1)
    pos = {tuple(e): i for i, e in enumerate(uniq.tolist())}
    bm = np.array([nv + pos[tuple(e)] for e in bkey.tolist()], dtype=np.int64)
    bf = np.concatenate([np.stack([B[:, 0], bm], 1), np.stack([bm, B[:, 1]], 1)])
    parents = np.concatenate([np.stack([np.arange(nv)] * 2, 1), uniq])
    fine, perm = _finish(2, verts, cells, bf, want_perm=True)
    return fine, np.ascontiguousarray(parents[perm], dtype=np.int32)


def hierarchy(mesh, levels: int):
    """Nested meshes [mesh, refine(mesh), ...] (levels meshes) and the
    parent arrays of levels 1 .. levels-1 (see refine_uniform)."""
    meshes, parents = [mesh], []
    for _ in range(levels - 1):
        m, p = refine_uniform(meshes[-1])
        meshes.append(m)
        parents.append(p)
    return meshes, parents


def interval(N: int, a: float = -1.0, b: float = 1.0):
    """Uniform mesh of (a,b) with N cells; boundary facets are the endpoints."""
    if a == -1.0 and b == 1.0 and (N & (N - 1)) == 0:
        x = -1.0 + np.arange(N + 1) * (2.0 / N)  # exact in binary
    else:
        x = np.linspace(a, b, N + 1)
    cells = np.stack([np.arange(N), np.arange(1, N + 1)], axis=1)
    return _finish(1, x[:, None], cells, [[0], [N]], sort=False)


def interval_graded(N: int, mu: float = 2.0):
    """Mesh of (-1,1) graded symmetrically toward both endpoints:
    x_i = -1 + (i/M)^mu on the left half (N = 2M cells)."""
    M = N // 2
    t = (np.arange(M + 1) / M) ** mu
    x = np.concatenate([-1.0 + t, (1.0 - t[::-1])[1:]])
    cells = np.stack([np.arange(2 * M), np.arange(1, 2 * M + 1)], axis=1)
    return _finish(1, x[:, None], cells, [[0], [2 * M]], sort=False)


def _boundary_edges(cells):
    from collections import Counter
    cnt = Counter()
    for c in cells:
        for i in range(3):
            e = tuple(sorted((int(c[i]), int(c[(i + 1) % 3]))))
            cnt[e] += 1
    return [e for e, k in cnt.items() if k == 1]


def disk(h: float, seed: int = 2, jitter: float = 0.15):
    """Quasi-uniform mesh of the unit disk.  N_b = round(2 pi / h) points on
    the circle; interior hexagonal lattice of spacing h clipped to
    r < 1 - 0.7 h, each point shifted by U(-jitter h, jitter h)^2 drawn from
    numpy.random.default_rng(seed); Delaunay triangulation (scipy), whose
    hull is the inscribed polygon."""
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(seed)
    nb = int(round(2 * math.pi / h))
    th = 2 * math.pi * np.arange(nb) / nb
    bpts = np.stack([np.cos(th), np.sin(th)], axis=1)
    ny = int(math.ceil(1.0 / (h * math.sqrt(3) / 2))) + 1
    pts = []
    for j in range(-ny, ny + 1):
        y = j * h * math.sqrt(3) / 2
        off = 0.5 * h if (j % 2) else 0.0
        nx = int(math.ceil(1.0 / h)) + 1
        xs = np.arange(-nx, nx + 1) * h + off
        pts.append(np.stack([xs, np.full_like(xs, y)], axis=1))
    ipts = np.concatenate(pts)
    ipts = ipts[np.hypot(ipts[:, 0], ipts[:, 1]) < 1.0 - 0.7 * h]
    ipts = ipts + rng.uniform(-jitter * h, jitter * h, size=ipts.shape)
    P = np.concatenate([bpts, ipts])
    tri = Delaunay(P)
    cells = tri.simplices
    bf = _boundary_edges(cells)
    return _finish(2, P, cells, bf)


def disk_symmetric(h: float, K: int, seed: int = 2, jitter: float = 0.15):
    """Unit-disk mesh invariant under the rotation B by 2 pi / K (K >= 2),
    built from a sector omega = {r <= 1, 0 <= phi <= 2 pi / K} and its
    images.  The sector holds the origin, points at radii j h on its two
    radial edges (the second edge the image of the first), points on the
    arc, and a jittered hexagonal lattice (numpy default_rng(seed)) kept
    0.5 h away from the edges; Delaunay on the sector, then rotated copies
    glued along the radial edges.  Returns (mesh, vfold, T_omega, pre, rot):
    the cells of omega come first (T_omega of them, in Morton order); copy i
    of sector cell c follows as cell i T_omega + c, with pre = c and rot = i
    (pre = c, rot = 0 on the sector); vfold maps every vertex to its
    representative (the omega vertex it is an image of, the first radial
    edge standing for the second)."""
    from scipy.spatial import Delaunay
    assert K >= 2
    al = 2 * math.pi / K
    rng = np.random.default_rng(seed)
    N = max(2, int(round(1.0 / h)))
    r = np.arange(1, N + 1) / N                       # radii on the edges (1 = the arc's end)
    e1 = np.stack([r, np.zeros_like(r)], 1)
    e2 = np.stack([r * math.cos(al), r * math.sin(al)], 1)
    nb = max(2, int(round(al / h)))
    th = al * np.arange(1, nb) / nb
    arc = np.stack([np.cos(th), np.sin(th)], 1)
    ny = int(math.ceil(1.0 / (h * math.sqrt(3) / 2))) + 1
    pts = []
    for j in range(-ny, ny + 1):
        y = j * h * math.sqrt(3) / 2
        off = 0.5 * h if (j % 2) else 0.0
        nx = int(math.ceil(1.0 / h)) + 1
        xs = np.arange(-nx, nx + 1) * h + off
        pts.append(np.stack([xs, np.full_like(xs, y)], 1))
    ip = np.concatenate(pts)
    ip = ip + rng.uniform(-jitter * h, jitter * h, size=ip.shape)
    rr = np.hypot(ip[:, 0], ip[:, 1])
    ph = np.mod(np.arctan2(ip[:, 1], ip[:, 0]), 2 * math.pi)
    d1 = rr * np.sin(np.minimum(ph, math.pi / 2))      # distance to the first edge (phi < pi/2)
    d2 = rr * np.sin(np.clip(al - ph, 0.0, math.pi / 2))
    keep = (rr < 1.0 - 0.7 * h) & (ph < al) & (d1 > 0.5 * h) & (d2 > 0.5 * h)
    ip = ip[keep]
    P = np.concatenate([[[0.0, 0.0]], e1, e2, arc, ip])
    n1 = len(e1)
    tri = Delaunay(P)
    cells = tri.simplices
    a = P[cells]
    area = 0.5 * np.abs((a[:, 1, 0] - a[:, 0, 0]) * (a[:, 2, 1] - a[:, 0, 1])
                        - (a[:, 2, 0] - a[:, 0, 0]) * (a[:, 1, 1] - a[:, 0, 1]))
    cells = cells[area > 1e-12 * h * h]
    used = np.unique(cells)
    assert len(used) == len(P), "every sector point must be a vertex"
    # sector cells along a Morton curve of their centroids (spatially
    # coherent order; the images keep it)
    cells = cells[np.argsort(_morton_key(P[cells].mean(1)), kind="stable")]
    # sector representatives: the second edge (indices 1 + n1 .. 2 n1) stands for the first
    rep_s = np.arange(len(P))
    rep_s[1 + n1:1 + 2 * n1] = np.arange(1, 1 + n1)
    # glue K rotated copies; a vertex is keyed by its rounded coordinates.
    # Copy i of sector point p stands for the sector vertex rep_s[p] (a
    # vertex shared by two copies gets the same answer from both).
    verts, vrep, key = [], {}, {}
    cell_all = []
    ids0 = None
    for i in range(K):
        c, s_ = math.cos(i * al), math.sin(i * al)
        Q = P @ np.array([[c, s_], [-s_, c]])
        ids = np.empty(len(P), dtype=np.int64)
        for p in range(len(P)):
            kk = (round(Q[p, 0] * 1e9), round(Q[p, 1] * 1e9))
            if kk not in key:
                key[kk] = len(verts)
                verts.append(Q[p])
            ids[p] = key[kk]
        if i == 0:
            ids0 = ids.copy()
        for p in range(len(P)):
            vrep[int(ids[p])] = int(ids0[rep_s[p]])
        cell_all.append(ids[cells])
    vrep = np.array([vrep[v] for v in range(len(verts))])
    C = np.concatenate(cell_all)
    V = np.array(verts)
    bf = _boundary_edges(C)
    Tw = len(cells)
    pre = np.tile(np.arange(Tw), K).astype(np.int32)
    rot = np.repeat(np.arange(K), Tw).astype(np.int32)
    return _finish(2, V, C, bf, sort=False), vrep.astype(np.int32), Tw, pre, rot


def disk_for_cells(T: int, seed: int = 2):
    """Disk mesh with about T triangles (T ~ 7.25 / h^2)."""
    return disk(math.sqrt(7.25 / T), seed=seed)


def square3(N: int, a: float = -1.0, b: float = 1.0):
    """Structured three-direction mesh of (a,b)^2: N x N squares, each cut
    by its (lower-left, upper-right) diagonal."""
    x = np.linspace(a, b, N + 1)
    X, Y = np.meshgrid(x, x, indexing="ij")
    verts = np.stack([X.ravel(), Y.ravel()], axis=1)
    idx = lambda i, j: i * (N + 1) + j
    cells = []
    for i in range(N):
        for j in range(N):
            cells.append((idx(i, j), idx(i + 1, j), idx(i + 1, j + 1)))
            cells.append((idx(i, j), idx(i + 1, j + 1), idx(i, j + 1)))
    cells = np.array(cells)
    bf = _boundary_edges(cells)
    return _finish(2, verts, cells, bf, sort=False) | {"N": N}


# ----------------------------------------------------------- L-shape NVB --

def _nvb_refine(verts, tris, marked_fn, max_pass=200, marked_ids=None):
    """Conforming newest-vertex bisection.  Each triangle (a,b,c) has its
    refinement edge (b,c) opposite the newest vertex a.  A triangle is
    bisected only together with the neighbour that shares its refinement
    edge as that neighbour's refinement edge (recursively refining the
    neighbour first), so no hanging nodes arise.  Passes refine the
    triangles that marked_fn selects until none is; with marked_ids, one
    pass bisects those triangles (indices into tris) once each."""
    verts = [tuple(v) for v in verts]
    tris = {i: tuple(t) for i, t in enumerate(tris)}
    nxt = len(tris)
    edge = {}

    def add(tid):
        a, b, c = tris[tid]
        for e in ((a, b), (b, c), (c, a)):
            edge.setdefault(tuple(sorted(e)), set()).add(tid)

    def rem(tid):
        a, b, c = tris[tid]
        for e in ((a, b), (b, c), (c, a)):
            edge[tuple(sorted(e))].discard(tid)

    for t in tris:
        add(t)
    mids = {}

    def midpoint(b, c):
        key = tuple(sorted((b, c)))
        if key not in mids:
            vb, vc = verts[b], verts[c]
            verts.append(((vb[0] + vc[0]) / 2, (vb[1] + vc[1]) / 2))
            mids[key] = len(verts) - 1
        return mids[key]

    def bisect(tid):
        nonlocal nxt
        a, b, c = tris[tid]
        m = midpoint(b, c)
        rem(tid)
        del tris[tid]
        t1, t2 = nxt, nxt + 1
        nxt += 2
        tris[t1] = (m, a, b)
        tris[t2] = (m, c, a)
        add(t1)
        add(t2)

    def refine(tid, depth=0):
        if tid not in tris:
            return
        a, b, c = tris[tid]
        key = tuple(sorted((b, c)))
        nb = [t for t in edge.get(key, ()) if t != tid]
        if nb:
            n = nb[0]
            na, nbv, ncv = tris[n]
            if tuple(sorted((nbv, ncv))) != key:
                refine(n, depth + 1)
                nb = [t for t in edge.get(key, ()) if t != tid]
                n = nb[0]
            bisect(tid)
            bisect(n)
        else:
            bisect(tid)

    if marked_ids is not None:
        for t in marked_ids:
            refine(int(t))
        return np.array(verts), np.array(list(tris.values()))
    for _ in range(max_pass):
        marked = [t for t, abc in tris.items() if marked_fn([verts[v] for v in abc])]
        if not marked:
            break
        for t in marked:
            refine(t)
    return np.array(verts), np.array(list(tris.values()))


def nvb_label(mesh):
    """Newest-vertex labels for a triangle mesh that has none: every cell is
    rotated (orientation kept) so that its longest edge joins columns 1 and
    2, the refinement edge of refine_marked."""
    V = np.asarray(mesh["verts"], dtype=np.float64)
    C = np.asarray(mesh["cells"], dtype=np.int64)
    L = np.stack([((V[C[:, (i + 1) % 3]] - V[C[:, (i + 2) % 3]]) ** 2).sum(1) for i in range(3)], 1)
    r = np.argmax(L, axis=1)  # vertex opposite the longest edge
    idx = (r[:, None] + np.arange(3)[None, :]) % 3
    out = dict(mesh)
    out["cells"] = np.ascontiguousarray(np.take_along_axis(C, idx, 1), dtype=np.int32)
    return out


def project_disk(xy):
    """Radial projection onto the unit circle (new boundary vertices of a
    disk mesh)."""
    xy = np.asarray(xy, dtype=np.float64)
    return xy / np.linalg.norm(xy, axis=-1, keepdims=True)


def refine_marked(mesh, marked, project=None):
    """Refine the marked cells (indices) of a mesh.  d = 1: each marked
    cell is halved.  d = 2: newest-vertex bisection with column 0 the newest
    vertex (see nvb_label), each marked cell bisected once, neighbours
    bisected as far as conformity requires; the children keep the labels.
    project (d = 2): maps the new boundary vertices (edge midpoints) onto
    the curved boundary, e.g. project_disk.  Returns the new (sorted)
    mesh."""
    dim = mesh["dim"]
    V = np.asarray(mesh["verts"], dtype=np.float64).reshape(-1, dim)
    C = np.asarray(mesh["cells"], dtype=np.int64)
    marked = np.unique(np.asarray(marked, dtype=np.int64))
    if dim == 1:
        keep = np.ones(len(C), dtype=bool)
        keep[marked] = False
        mid = len(V) + np.arange(len(marked))
        verts = np.concatenate([V[:, 0], 0.5 * (V[C[marked, 0], 0] + V[C[marked, 1], 0])])
        cells = np.concatenate([C[keep], np.stack([C[marked, 0], mid], 1), np.stack([mid, C[marked, 1]], 1)])
        order = np.argsort(verts, kind="stable")
        inv = np.empty_like(order)
        inv[order] = np.arange(len(order))
        cells = inv[cells]
        cells = cells[np.argsort(verts[order][cells].mean(1), kind="stable")]
        B = inv[np.asarray(mesh["bfacets"], dtype=np.int64)]
        return _finish(1, verts[order][:, None], cells, B, sort=False)
    verts, tris = _nvb_refine([tuple(v) for v in V], [tuple(t) for t in C.tolist()], None,
                              marked_ids=marked.tolist())
    bf = _boundary_edges(tris)
    if project is not None:
        nb = np.unique(np.asarray(bf, dtype=np.int64))
        nb = nb[nb >= len(V)]
        if len(nb):
            verts = np.array(verts, dtype=np.float64)
            verts[nb] = project(verts[nb])
    return _finish(2, verts, tris, bf)


def lshape(h_max: float = 0.1, gamma: float = 1.0, ratio: float = 64.0, R: float = 1.0):
    """L-shape (-1,1)^2 minus [0,1)x(-1,0], graded by newest-vertex
    bisection: refine K while its longest edge exceeds
    h_max * max(1/ratio, min(1, (rho(c_K)/R)^gamma)), rho = distance of the
    centroid to the re-entrant corner or the boundary, whichever is
    smaller.  Deterministic (no random numbers)."""
    V = [(-1, -1), (0, -1), (-1, 0), (0, 0), (1, 0), (-1, 1), (0, 1), (1, 1)]
    # three unit squares, cut along diagonals through the corner (0,0);
    # (newest vertex, refinement edge) = (right-angle corner, hypotenuse)
    T = [(1, 0, 3), (2, 3, 0),      # [-1,0]x[-1,0], diagonal (-1,-1)-(0,0)
         (2, 3, 5), (6, 5, 3),      # [-1,0]x[0,1],  diagonal (-1,1)-(0,0)
         (4, 3, 7), (6, 7, 3)]      # [0,1]x[0,1],   diagonal (0,0)-(1,1)

    def dist_boundary(x, y):
        # distance to the boundary of the L-shape (inside points)
        d = min(1 + x, 1 - x, 1 + y, 1 - y)
        if x >= 0 and y <= 0:
            return 0.0
        if x >= 0:  # upper right square: edge y = 0 for x in [0,1]
            d = min(d, y)
        if y <= 0:  # lower left square: edge x = 0 for y in [-1,0]
            d = min(d, -x)
        return max(d, 0.0)

    def marked(P):
        cx = sum(p[0] for p in P) / 3
        cy = sum(p[1] for p in P) / 3
        rho = min(math.hypot(cx, cy), dist_boundary(cx, cy))
        target = h_max * max(1.0 / ratio, min(1.0, (rho / R) ** gamma))
        hk = max(math.dist(P[i], P[(i + 1) % 3]) for i in range(3))
        return hk > target * 1.0000001

    verts, tris = _nvb_refine(V, T, marked)
    bf = _boundary_edges(tris)
    return _finish(2, verts, tris, bf)


def lshape_config3():
    """Graded L-shape with ~40k triangles and size ratio 1:64 toward the
    re-entrant corner and the boundary."""
    return lshape(0.3, 1.0, 64.0, 0.5)


def tiny(kind: str):
    """Small meshes for brute-force checks."""
    if kind == "one":
        return _finish(2, [(0, 0), (1, 0), (0.2, 0.9)], [(0, 1, 2)], [(0, 1), (1, 2), (0, 2)], sort=False)
    if kind == "two":
        v = [(0, 0), (1, 0), (0.3, 0.8), (1.1, 0.9)]
        return _finish(2, v, [(0, 1, 2), (1, 3, 2)], [(0, 1), (1, 3), (2, 3), (0, 2)], sort=False)
    if kind == "four":
        v = [(0, 0), (1, 0), (1, 1), (0, 1), (0.45, 0.55)]
        c = [(0, 1, 4), (1, 2, 4), (2, 3, 4), (3, 0, 4)]
        return _finish(2, v, c, [(0, 1), (1, 2), (2, 3), (0, 3)], sort=False)
    raise ValueError(kind)
