"""Implicit steps of the fractional heat equation (Sec. 5) on the GPU:
mass-shifted assembly A^s + mu M, the mass product, and backward Euler
steps against the CPU oracle's dense solves; the Sec. 5 lemma's bounded
iteration counts for dt = h^(2s)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1708_03912_amd import fraclap as F, meshgen as M  # noqa: E402

from test_gpu_parity import check_matrix, gpu_assemble, oracle_orders  # noqa: E402


def _hmax(mesh):
    V = np.asarray(mesh["verts"], dtype=np.float64).reshape(-1, mesh["dim"])
    if mesh["dim"] == 1:
        C = np.asarray(mesh["cells"])
        return float(np.abs(V[C[:, 1], 0] - V[C[:, 0], 0]).max())
    P = V[np.asarray(mesh["cells"])]
    return float(np.sqrt(((P[:, [1, 2, 0]] - P) ** 2).sum(-1)).max())


@pytest.mark.parametrize("name,s,mode", [("disk", 0.3, "paper"), ("disk", 0.75, "paper"),
                                         ("interval", 0.75, "interior"), ("lshape", 0.5, "interior")])
def test_mass_shift_parity(name, s, mode):
    mesh = {"disk": lambda: M.disk_for_cells(800, seed=2), "interval": lambda: M.interval(200),
            "lshape": lambda: M.lshape(0.4, 1.0, 4.0)}[name]()
    mu = 37.5
    o0 = F.make_opts(dof_mode=mode)
    o1 = F.make_opts(dof_mode=mode, mass_shift=mu)
    h0, h1 = gpu_assemble(mesh, s, o0), gpu_assemble(mesh, s, o1)
    A0, A1 = h0.export_matrix(), h1.export_matrix()
    Ao, dofs, _ = O.assemble(mesh, s, oracle_orders(o0), mode=mode)
    Mo = O.mass_matrix(mesh, dofs)
    check_matrix(A1, Ao + mu * Mo)
    # the shift itself, to rounding of the sum
    assert np.abs((A1 - A0) - mu * Mo).max() <= 1e-13 * np.abs(A1).max()
    h0.close()
    h1.close()


def test_mass_matvec_parity_and_errors():
    mesh = M.disk_for_cells(900, seed=7)
    h = F.Handle(0)
    h.set_mesh(mesh)
    x0 = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(F.FraclapError) as e:
        h.mass_matvec(x0, x0.clone())
    assert e.value.code == F.FL_ESTATE
    n = h.assemble(0.6)
    Ao, dofs, _ = O.assemble(mesh, 0.6, oracle_orders(F.default_opts()))
    assert len(dofs) == n
    Mo = O.mass_matrix(mesh, dofs)
    g = torch.Generator().manual_seed(3)
    x = torch.randn(n, generator=g, dtype=torch.float64)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    xd = x.cuda()
    h.mass_matvec(xd, y)
    ref = Mo @ x.numpy()
    assert np.abs(y.cpu().numpy() - ref).max() <= 1e-14 * np.abs(ref).max()
    with pytest.raises(F.FraclapError) as e:
        h.mass_matvec(xd, xd)
    assert e.value.code == F.FL_EINVAL
    with pytest.raises(F.FraclapError) as e:
        h.assemble(0.6, F.make_opts(mass_shift=-1.0))
    assert e.value.code == F.FL_EINVAL
    h.close()


@pytest.mark.parametrize("s", [0.4, 0.8])
def test_backward_euler_steps(s):
    """u^{k+1} = (M + dt A)^{-1} (M u^k + dt b), f = 1, u^0 = 0, solved as
    (A + M/dt) u^{k+1} = M u^k / dt + b on the GPU (Jacobi-PCG, rtol 1e-13)
    against the oracle's dense solves; the iterates approach the Poisson
    solution."""
    mesh = M.disk_for_cells(700, seed=9)
    dt = 0.02
    h = gpu_assemble(mesh, s, F.make_opts(mass_shift=1.0 / dt))
    n = h.n
    Ao, dofs, _ = O.assemble(mesh, s, oracle_orders(F.default_opts()))
    Mo = O.mass_matrix(mesh, dofs)
    bo = O.load_vector_one(mesh, dofs)
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    h.load_vector_one(b)
    u = torch.zeros(n, dtype=torch.float64, device="cuda")
    mu = torch.empty_like(u)
    uo = np.zeros(n)
    upois = O.solve_cholesky(Ao, bo)
    Aop = Ao + Mo / dt
    dist = []
    for _ in range(4):
        h.mass_matvec(u, mu)
        rhs = mu / dt + b
        unew = torch.zeros_like(u)
        it, rel, rc = h.solve(rhs, unew, rtol=1e-13)
        assert rc == F.FL_OK
        u = unew
        uo = O.solve_cholesky(Aop, Mo @ uo / dt + bo)
        e = u.cpu().numpy() - uo
        assert math.sqrt(e @ Aop @ e) <= 1e-10 * math.sqrt(uo @ Aop @ uo)
        dist.append(np.abs(uo - upois).max())
    assert all(dist[k + 1] < dist[k] for k in range(3))
    h.close()


def test_heat_iterations_bounded_under_refinement():
    """Sec. 5 lemma: with dt = h^(2s) the Jacobi-preconditioned system
    M + dt A^s has a condition number bounded under refinement, so the CG
    iteration count stays nearly flat from ~1000 to ~4000 cells, while the
    Poisson system's grows (s = 0.75)."""
    s = 0.75
    its = {}
    for T in (1000, 4000):
        mesh = M.disk_for_cells(T, seed=3)
        dt = _hmax(mesh) ** (2 * s)
        for name, mu in (("poisson", 0.0), ("heat", 1.0 / dt)):
            h = gpu_assemble(mesh, s, F.make_opts(mass_shift=mu))
            b = torch.empty(h.n, dtype=torch.float64, device="cuda")
            h.load_vector_one(b)
            u = torch.zeros_like(b)
            it, rel, rc = h.solve(b, u, rtol=1e-10)
            assert rc == F.FL_OK
            its[(name, T)] = it
            h.close()
    assert its[("heat", 4000)] <= 1.35 * its[("heat", 1000)], its
    assert its[("poisson", 4000)] >= 1.4 * its[("poisson", 1000)], its
