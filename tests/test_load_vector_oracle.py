"""Pins of the oracle's load vectors b_i = int f phi_i (Sec. 2: the right-hand
side of the Galerkin system) for data other than f = 1.

`oracle.load_vector_fn` integrates f phi_i cell by cell with the collapsed
order-k triangle rule (2D) or k-point Gauss-Legendre (1D).  It is pinned
here against values it does not compute itself:

* f = 1: the exact sum over the cells of |K| / (d + 1) (`load_vector_one`);
* f linear: f is its own P1 interpolant, so b = M f(nodes) with the P1 mass
  matrix over all nodes (pinned on its own in the heat-step pins);
* f = cos(w . x + c): the closed form of int_K lambda_a exp(i w . x) dx
  by the Hermite-Genocchi formula.  On the reference simplex,
  int lambda_a exp(sum_j t_j z_j) dt is the derivative of the divided
  difference exp[z_0, .., z_d] with respect to z_a, i.e. the divided
  difference with z_a repeated, times d! |K| (z_j = i w . v_j), evaluated
  here in 40-digit arithmetic.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O
from paper_1708_03912_amd import meshgen as M


def _divdiff_exp(z):
    """exp[z_0, .., z_m] for nodes sorted so that equal nodes are adjacent
    (at most one node repeated once), by the recursive definition with
    f[z, z] = exp(z)."""
    z = list(z)
    m = len(z) - 1
    if m == 0:
        return mp.exp(z[0])
    if all(abs(zz - z[0]) == 0 for zz in z):
        return mp.exp(z[0]) / mp.factorial(m)
    if abs(z[-1] - z[0]) == 0:
        raise ValueError("repeated node must be adjacent to its copy")
    return (_divdiff_exp(z[1:]) - _divdiff_exp(z[:-1])) / (z[-1] - z[0])


def _exact_cos_load(mesh, omega, phase):
    """b_v = int cos(omega . x + phase) phi_v(x) dx over all nodes v, closed form."""
    mp.mp.dps = 40
    dim = mesh["dim"]
    V = np.asarray(mesh["verts"], dtype=np.float64).reshape(-1, dim)
    Cc = np.asarray(mesh["cells"]).reshape(-1, dim + 1)
    b = [mp.mpf(0)] * len(V)
    eph = mp.exp(1j * mp.mpf(phase))
    for cell in Cc:
        P = [V[c] for c in cell]
        z = [1j * sum(mp.mpf(omega[k]) * mp.mpf(float(p[k])) for k in range(dim)) for p in P]
        if dim == 1:
            meas = abs(mp.mpf(float(P[1][0])) - mp.mpf(float(P[0][0])))
            fac = meas            # d! |K|, d = 1
        else:
            a, bb, c = [[mp.mpf(float(t)) for t in p] for p in P]
            meas = abs((bb[0] - a[0]) * (c[1] - a[1]) - (c[0] - a[0]) * (bb[1] - a[1])) / 2
            fac = 2 * meas        # d! |K|, d = 2
        for a_loc, v in enumerate(cell):
            others = [z[j] for j in range(dim + 1) if j != a_loc]
            dd = _divdiff_exp([z[a_loc], z[a_loc]] + others)
            b[v] += mp.re(fac * dd * eph)
    return np.array([float(x) for x in b])


def _mesh2d():
    return M.disk_for_cells(120, seed=7)


def _mesh1d():
    x = np.sort(np.concatenate([[-1.0, 1.0], np.random.default_rng(3).uniform(-0.95, 0.95, 21)]))
    return {"dim": 1, "verts": x[:, None], "cells": np.stack([np.arange(22), np.arange(1, 23)], 1),
            "bfacets": np.array([[0], [22]])}


@pytest.mark.parametrize("dim", [1, 2])
def test_constant_is_load_vector_one(dim):
    mesh = _mesh2d() if dim == 2 else _mesh1d()
    dofs = np.arange(len(mesh["verts"]))
    for k in (1, 2, 4, 7):
        b = O.load_vector_fn(mesh, dofs, lambda x: np.ones(len(x)), k=k)
        b1 = O.load_vector_one(mesh, dofs)
        assert np.abs(b - b1).max() <= 1e-14 * np.abs(b1).max()


@pytest.mark.parametrize("dim", [1, 2])
def test_linear_is_mass_times_nodal(dim):
    mesh = _mesh2d() if dim == 2 else _mesh1d()
    nv = len(mesh["verts"])
    V = np.asarray(mesh["verts"], dtype=np.float64).reshape(nv, dim)
    Mfull = O.mass_matrix(mesh, np.arange(nv))
    dofs = O.dof_nodes(nv, mesh["bfacets"], 0.75)          # interior nodes only
    coef = [(0.3, -1.2, 2.5), (-2.0, 0.7, 0.1)]
    for c0, cx, cy in coef:
        if dim == 1:
            f = lambda x, c0=c0, cx=cx: c0 + cx * x[:, 0]
            nod = c0 + cx * V[:, 0]
        else:
            f = lambda x, c0=c0, cx=cx, cy=cy: c0 + cx * x[:, 0] + cy * x[:, 1]
            nod = c0 + cx * V[:, 0] + cy * V[:, 1]
        ref = (Mfull @ nod)[dofs]
        # the integrand f phi_i has degree 2: orders >= 2 integrate it exactly
        for k in (2, 4):
            b = O.load_vector_fn(mesh, dofs, f, k=k)
            assert np.abs(b - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("dim", [1, 2])
def test_cosine_closed_form(dim):
    mesh = _mesh2d() if dim == 2 else _mesh1d()
    nv = len(mesh["verts"])
    dofs = np.arange(nv)
    modes = [((math.pi * 1, math.pi * 2), 0.0), ((math.pi * 3, -math.pi * 1), 0.7)] if dim == 2 else \
            [((math.pi * 3,), 0.0), ((math.pi * 1.5,), -0.4)]
    for om, ph in modes:
        if dim == 2:
            f = lambda x, om=om, ph=ph: np.cos(om[0] * x[:, 0] + om[1] * x[:, 1] + ph)
        else:
            f = lambda x, om=om, ph=ph: np.cos(om[0] * x[:, 0] + ph)
        ref = _exact_cos_load(mesh, om, ph)
        scale = np.abs(ref).max()
        # a high order reproduces the closed form to rounding
        b12 = O.load_vector_fn(mesh, dofs, f, k=12)
        assert np.abs(b12 - ref).max() <= 1e-13 * scale
        # the order-4 rule used for the benchmark right-hand sides is close
        # (degree 7 exact) and the error falls with the order
        e4 = np.abs(O.load_vector_fn(mesh, dofs, f, k=4) - ref).max() / scale
        e2 = np.abs(O.load_vector_fn(mesh, dofs, f, k=2) - ref).max() / scale
        assert e4 <= 1e-4 and e4 < 2e-2 * e2


def test_cosine_sum_is_linear_in_the_modes():
    """A sum of cosine modes with coefficients c_m (the batched right-hand
    sides) is the same combination of the single-mode closed forms."""
    mesh = _mesh2d()
    nv = len(mesh["verts"])
    dofs = O.dof_nodes(nv, mesh["bfacets"], 0.75)
    ks = [(0, 0), (1, 0), (2, 3), (3, 1)]
    c = np.random.default_rng(11).standard_normal(len(ks))

    def f(x):
        return sum(cm * np.cos(math.pi * (k1 * x[:, 0] + k2 * x[:, 1])) for cm, (k1, k2) in zip(c, ks))

    ref = sum(cm * _exact_cos_load(mesh, (math.pi * k1, math.pi * k2), 0.0) for cm, (k1, k2) in zip(c, ks)
              if (k1, k2) != (0, 0))
    ref = ref + c[0] * O.load_vector_one(mesh, np.arange(nv))
    b = O.load_vector_fn(mesh, dofs, f, k=12)
    assert np.abs(b - ref[dofs]).max() <= 1e-13 * np.abs(ref).max()
