"""Adaptive refinement loop (Sec. 4 and Sec. 7 of arXiv:1708.03912):
solve on the current mesh, evaluate the strong form of the discrete
solution at the indicator points, form the Babuska-Rheinboldt indicators,
mark by the maximum strategy (threshold 0.8), refine, repeat.

Every numerical step runs in the library (assembly, solve, strong form,
indicators); marking and refinement are host mesh logic (meshgen).  The
right-hand side is f = 1.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import fraclap as F
from . import meshgen as M


def mark_max(eta_node, cells, theta=0.8):
    """Maximum marking on the nodal indicators: the vertices i with
    eta-hat_i >= theta max_j eta-hat_j (eta_node holds eta-hat_i^2); the
    cells to refine are their patches S_i."""
    eta = np.sqrt(np.maximum(np.asarray(eta_node, dtype=np.float64), 0.0))
    hot = eta >= theta * eta.max()
    return np.nonzero(hot[np.asarray(cells)].any(axis=1))[0]


@dataclass
class Step:
    n: int                  # DOFs
    cells: int
    estimator: float        # sum_i eta-hat_i^2
    e2: float | None        # squared energy error (if (f,u) is given)
    t_assemble: float       # seconds
    t_solve: float
    t_indicators: float
    iters: int
    extra: dict = field(default_factory=dict)


def adaptive_loop(mesh, s, steps, theta=0.8, opts=None, k_eval=2, q_far=2, q_near=12, rtol=1e-10,
                  fu=None, max_cells=None, project=None, cluster_sf=None, device=0):
    """Run `steps` solve-estimate-mark-refine cycles from `mesh`; returns the
    list of Step records and the last mesh.  fu = (f, u) of the exact
    solution, if known, gives the energy error by the identity of Sec. 7.
    project: map of new boundary vertices onto a curved boundary (d = 2).
    cluster_sf: None, or (m, eta, leaf) to evaluate the strong form's
    all-pairs part by the cluster method (d = 2), as Sec. 7 does.
    Stops early once the mesh would exceed max_cells."""
    if mesh["dim"] == 2:
        mesh = M.nvb_label(mesh)
    opts = opts if opts is not None else F.default_opts()
    out = []
    h = F.Handle(device)
    try:
        for it in range(steps):
            T = len(mesh["cells"])
            Q = k_eval ** mesh["dim"]
            h.set_mesh(mesh)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            n = h.assemble(s, opts)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            b = torch.empty(n, dtype=torch.float64, device="cuda")
            h.load_vector_one(b)
            u = torch.zeros_like(b)
            iters, _, _ = h.solve(b, u, rtol=rtol)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            Lu = torch.empty(T * Q, dtype=torch.float64, device="cuda")
            eta_c = torch.empty(T, dtype=torch.float64, device="cuda")
            eta_n = torch.empty(len(mesh["verts"]), dtype=torch.float64, device="cuda")
            if cluster_sf is not None and mesh["dim"] == 2:
                m, eta, leaf = cluster_sf
                h.strong_form_cluster(s, u, Lu, k_eval=k_eval, q_far=q_far, q_near=q_near, m=m, eta=eta, leaf=leaf)
            else:
                h.strong_form(s, u, Lu, k_eval=k_eval, q_far=q_far, q_near=q_near)
            h.indicators(s, Lu, eta_c, eta_n, k_eval=k_eval)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            e2 = h.energy_error2(fu, b, u) if fu is not None else None
            en = eta_n.cpu().numpy()
            out.append(Step(n, T, float(eta_c.sum().item()), e2, t1 - t0, t2 - t1, t3 - t2, iters))
            if it == steps - 1:
                break
            marked = mark_max(en, mesh["cells"], theta)
            new = M.refine_marked(mesh, marked, project=project)
            if max_cells is not None and len(new["cells"]) > max_cells:
                break
            mesh = new
    finally:
        h.close()
    return out, mesh
