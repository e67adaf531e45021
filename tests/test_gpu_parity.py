"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bar (FP64): max|dA| <= 1e-10 max|A| and ||dA||_F <= 1e-10 ||A||_F for the
assembled matrix; ||u - u_oracle||_A <= 1e-10 ||u_oracle||_A for solves with
rtol <= 1e-13.  Both sides use the same quadrature rule (orders, classes,
regularised touching-pair rules); they share no code.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1708_03912_amd import fraclap as F, meshgen as M  # noqa: E402

TOL = 1e-10


def oracle_orders(o):
    nc = o.n_classes
    return O.Orders(k_touch=o.k_touch, k_touch_bnd=o.k_touch_bnd, theta=[o.theta[i] for i in range(nc)],
                    k_far=[o.k_far[i] for i in range(nc + 1)], k_far_bnd=[o.k_far_bnd[i] for i in range(nc + 1)])


def gpu_assemble(mesh, s, o):
    h = F.Handle(0)
    h.set_mesh(mesh)
    h.assemble(s, o)
    return h


def check_matrix(A, Ao):
    assert A.shape == Ao.shape
    assert np.all(np.isfinite(A))
    scale = np.abs(Ao).max()
    assert np.abs(A - Ao).max() <= TOL * scale
    assert np.linalg.norm(A - Ao) <= TOL * np.linalg.norm(Ao)


MESHES = {
    "interval256": lambda: M.interval(256),
    "interval_graded": lambda: M.interval_graded(200, 2.5),
    "interval3": lambda: M.interval(3, -0.5, 0.7),
    "disk_600": lambda: M.disk_for_cells(600),
    "disk_1500": lambda: M.disk_for_cells(1500, seed=5),
    "lshape_graded": lambda: M.lshape(0.4, 1.0, 4.0),
    "square3_ties": lambda: M.square3(12),
    "tiny_one": lambda: M.tiny("one"),
    "tiny_two": lambda: M.tiny("two"),
    "tiny_four": lambda: M.tiny("four"),
}


@pytest.mark.parametrize("mode", ["paper", "interior"])
@pytest.mark.parametrize("s", [0.25, 0.5, 0.75])
@pytest.mark.parametrize("name", list(MESHES))
def test_assembly_parity(name, s, mode):
    mesh = MESHES[name]()
    print(f"case {name} s={s} mode={mode}", flush=True)
    o = F.make_opts(dof_mode=mode)
    h = gpu_assemble(mesh, s, o)
    Ao, dofs, cnt = O.assemble(mesh, s, oracle_orders(o), mode=mode)
    assert np.array_equal(h.dofs(), dofs)
    st = h.stats()
    assert list(st.pairs_far)[:o.n_classes + 1] == list(cnt)
    if len(dofs):
        check_matrix(h.export_matrix(), Ao)
    h.close()


@pytest.mark.parametrize("s", [0.3, 0.75])
def test_assembly_parity_high_and_low_orders(s):
    mesh = M.disk_for_cells(500, seed=7)
    for o in (F.make_opts(k_touch=12, k_touch_bnd=10, theta=[1.2, 2.0, 4.0, 8.0, 16.0], k_far=[8, 7, 6, 5, 4, 3],
                          k_far_bnd=[8, 6, 5, 4, 3, 2]),
              F.make_opts(k_touch=1, k_touch_bnd=1, theta=[], k_far=[1], k_far_bnd=[1]),
              F.make_opts(with_boundary=0)):
        h = gpu_assemble(mesh, s, o)
        Ao, dofs, _ = O.assemble(mesh, s, oracle_orders(o), with_boundary=bool(o.with_boundary))
        check_matrix(h.export_matrix(), Ao)
        h.close()


def sampled_rows_parity(mesh, s, nrows, seed, mode="paper"):
    o = F.default_opts()
    o.dof_mode = F.FL_DOF_PAPER if mode == "paper" else F.FL_DOF_INTERIOR
    h = gpu_assemble(mesh, s, o)
    dofs = h.dofs()
    n = len(dofs)
    rng = np.random.default_rng(seed)
    rows = np.unique(np.concatenate([rng.choice(n, nrows, replace=False), [0, n - 1]]))
    A = h.matrix_view()
    Ag = A[torch.as_tensor(rows, device="cuda")].cpu().numpy()
    Af, _ = O.assemble_full(mesh, s, oracle_orders(o), rows=dofs[rows])
    Ao = Af[np.ix_(dofs[rows], dofs)]
    scale = np.abs(Ao).max()
    assert np.abs(Ag - Ao).max() <= TOL * scale
    # symmetry of the device matrix on the sampled rows
    col = A[:, torch.as_tensor(rows, device="cuda")].cpu().numpy().T
    assert np.abs(col - Ag).max() <= 1e-15 * 16 * scale
    h.close()


@pytest.mark.parametrize("s", [0.25, 0.75])
def test_config2_full_size_sampled_rows(s):
    """d=2 unit disk, ~8k triangles (the benchmark workload): sampled rows."""
    sampled_rows_parity(M.disk_for_cells(8000, seed=2), s, 10, 11)


def test_config5_disk_100k_sampled_rows():
    """d=2 unit disk with ~2e5 triangles: ~1e5 interior DOFs, an 80 GB FP64
    matrix on one device.  The oracle computes 8 sampled rows (all element
    pairs that reach them) without forming the matrix."""
    mesh = M.disk_for_cells(200000, seed=2)
    o = F.default_opts()
    o.dof_mode = F.FL_DOF_INTERIOR
    s = 0.75
    h = gpu_assemble(mesh, s, o)
    dofs = h.dofs()
    n = len(dofs)
    assert 95000 < n < 105000
    rng = np.random.default_rng(13)
    rows = np.unique(np.concatenate([rng.choice(n, 6, replace=False), [0, n - 1]]))
    A = h.matrix_view()
    Ag = A[torch.as_tensor(rows, device="cuda")].cpu().numpy()
    Ar, _ = O.assemble_full(mesh, s, oracle_orders(o), rows=dofs[rows], compact=True)
    Ao = Ar[:, dofs]
    scale = np.abs(Ao).max()
    assert np.abs(Ag - Ao).max() <= TOL * scale
    assert np.linalg.norm(Ag - Ao) <= TOL * np.linalg.norm(Ao)
    h.close()


def test_config3_lshape_full_size_sampled_rows():
    """d=2 graded L-shape, ~40k triangles, size ratio up to 1:64, s = 1/2."""
    mesh = M.lshape_config3()
    assert 35000 < len(mesh["cells"]) < 45000
    sampled_rows_parity(mesh, 0.5, 6, 12)


def test_matvec_and_solve_parity():
    mesh = M.disk_for_cells(1500, seed=5)
    for s in (0.25, 0.75):
        o = F.default_opts()
        h = gpu_assemble(mesh, s, o)
        n = h.n
        A = h.export_matrix()
        x = torch.rand(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        h.matvec(x, y)
        yr = A @ x.cpu().numpy()
        assert np.abs(y.cpu().numpy() - yr).max() <= 1e-13 * np.abs(yr).max()
        b = torch.empty(n, dtype=torch.float64, device="cuda")
        h.load_vector_one(b)
        Ao, dofs, _ = O.assemble(mesh, s, oracle_orders(o))
        bo = O.load_vector_one(mesh, dofs)
        assert np.abs(b.cpu().numpy() - bo).max() <= 1e-15
        u = torch.zeros_like(b)
        it, rel, rc = h.solve(b, u, rtol=1e-13)
        assert rc == F.FL_OK and rel <= 1e-13
        uo = O.solve_cholesky(Ao, bo)
        du = u.cpu().numpy() - uo
        assert math.sqrt(du @ Ao @ du) <= TOL * math.sqrt(uo @ Ao @ uo)
        # energy error against the closed form (Sec. 7 identity)
        fu = O.ball_fu(2, s)
        e2 = h.energy_error2(fu, b, u)
        Eo, e2o = O.energy_error(fu, bo, uo, Ao)
        assert abs(e2 - e2o) <= 1e-9 * fu
        # iteration count agrees with the oracle's PCG (same algorithm)
        _, ito, _ = O.pcg(Ao, bo, rtol=1e-13)
        assert abs(it - ito) <= 1
        h.close()


def test_config1_interval():
    """d=1, 256 cells, s = 0.75, f = 1: CG to 1e-12, closed-form energy error."""
    mesh = M.interval(256)
    o = F.default_opts()
    h = gpu_assemble(mesh, 0.75, o)
    Ao, dofs, _ = O.assemble(mesh, 0.75, oracle_orders(o))
    check_matrix(h.export_matrix(), Ao)
    b = torch.empty(h.n, dtype=torch.float64, device="cuda")
    h.load_vector_one(b)
    u = torch.zeros_like(b)
    it, rel, rc = h.solve(b, u, rtol=1e-12)
    _, ito, _ = O.pcg(Ao, O.load_vector_one(mesh, dofs), rtol=1e-12)
    assert abs(it - ito) <= 1 and rel <= 1e-12
    E = math.sqrt(h.energy_error2(O.ball_fu(1, 0.75), b, u))
    assert abs(E - 2.9403e-2) < 1e-5  # exact-matrix value 2.9433e-2; quadrature shifts the 4th digit
    h.close()


def test_error_paths():
    mesh = M.disk_for_cells(300)
    h = F.Handle(0)
    with pytest.raises(F.FraclapError) as e:
        h.assemble(0.5)
    assert e.value.code == F.FL_ESTATE
    h.set_mesh(mesh)
    for s in (0.0, 1.0, -0.1, float("nan")):
        with pytest.raises(F.FraclapError) as e:
            h.assemble(s)
        assert e.value.code == F.FL_EINVAL
    with pytest.raises(F.FraclapError) as e:
        h.assemble(0.5, F.make_opts(k_far=[9, 3, 2, 2]))
    assert e.value.code == F.FL_EINVAL
    with pytest.raises(F.FraclapError) as e:
        h.assemble(0.5, F.make_opts(theta=[2.0, 1.0], k_far=[3, 2, 2]))
    assert e.value.code == F.FL_EINVAL
    x = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(F.FraclapError) as e:
        h.matvec(x, x)
    assert e.value.code == F.FL_ESTATE
    n = h.assemble(0.75)
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    h.load_vector_one(b)
    u = torch.zeros_like(b)
    it, rel, rc = h.solve(b, u, rtol=1e-12, maxit=3)
    assert rc == F.FL_ENOCONV and it == 3
    b[5] = float("nan")
    with pytest.raises(F.FraclapError) as e:
        h.solve(b, u)
    assert e.value.code == F.FL_ENONFINITE
    bad = dict(mesh)
    bad["cells"] = mesh["cells"].copy()
    bad["cells"][3, 1] = len(mesh["verts"]) + 5
    with pytest.raises(F.FraclapError) as e:
        h.set_mesh(bad)
    assert e.value.code == F.FL_EMESH
    deg = dict(mesh)
    deg["cells"] = mesh["cells"].copy()
    deg["cells"][3, 1] = deg["cells"][3, 0]
    with pytest.raises(F.FraclapError) as e:
        h.set_mesh(deg)
    assert e.value.code == F.FL_EMESH
    nof = dict(mesh)
    nof["bfacets"] = np.vstack([mesh["bfacets"], [[0, len(mesh["verts"]) - 1]]]).astype(np.int32)
    with pytest.raises(F.FraclapError) as e:
        h.set_mesh(nof)
    assert e.value.code == F.FL_EMESH
    # scales outside the range of the FP64 kernel-power tables are refused
    for f in (2.0 ** -56, 2.0 ** 62):
        sc = dict(mesh)
        sc["verts"] = mesh["verts"] * f
        with pytest.raises(F.FraclapError) as e:
            h.set_mesh(sc)
        assert e.value.code == F.FL_EMESH
    ok = dict(mesh)
    ok["verts"] = mesh["verts"] * 2.0 ** -40
    h.set_mesh(ok)
    h.close()


def test_no_dofs():
    """One triangle with s >= 1/2: every vertex is on the boundary, n = 0."""
    h = F.Handle(0)
    h.set_mesh(M.tiny("one"))
    assert h.assemble(0.75) == 0
    b = torch.empty(0, dtype=torch.float64, device="cuda")
    it, rel, rc = h.solve(b, b.clone())
    assert it == 0 and rc == F.FL_OK
    h.close()


def test_repeatable():
    """Two assemblies agree to rounding (global atomics order the sums
    differently from run to run)."""
    mesh = M.disk_for_cells(1500, seed=5)
    h1 = gpu_assemble(mesh, 0.4, F.default_opts())
    h2 = gpu_assemble(mesh, 0.4, F.default_opts())
    A1, A2 = h1.export_matrix(), h2.export_matrix()
    assert np.abs(A1 - A2).max() <= 1e-14 * np.abs(A1).max()
    h1.close()
    h2.close()


@pytest.mark.parametrize("s", [0.3, 0.8])
def test_scale_homogeneity(s):
    """The bilinear form is homogeneous (Sec. 2, kernel |x-y|^(-d-2s)):
    scaling every coordinate by a power of two f multiplies the matrix by
    f^(d-2s) up to rounding.  Scales 2^-40 and 2^40 drive the separated-pair
    kernel powers far from 1 (both ends of their exponent tables)."""
    mesh = M.disk_for_cells(800, seed=3)
    A = gpu_assemble(mesh, s, F.default_opts())
    A1 = A.export_matrix()
    A.close()
    for e in (-40, 40):
        sc = dict(mesh)
        sc["verts"] = mesh["verts"] * 2.0 ** e
        h = gpu_assemble(sc, s, F.default_opts())
        Af = h.export_matrix() / 2.0 ** (e * (2 - 2 * s))
        h.close()
        assert np.abs(Af - A1).max() <= 1e-12 * np.abs(A1).max(), e


@pytest.mark.parametrize("s", [0.25, 0.75])
def test_mixed_precision_assembly_and_refined_solve(s):
    """FL_MIXED: separated pairs in FP32, FP64 everywhere else; the matrix
    stays within FP32 rounding of the FP64 one, and the refined solve reaches
    rtol on it with an energy-norm gap to the FP64 solution far below the
    discretisation error (equal error: gap <= 0.1 E)."""
    mesh = M.disk_for_cells(1500, seed=5)
    h64 = gpu_assemble(mesh, s, F.default_opts())
    hmx = gpu_assemble(mesh, s, F.make_opts(precision="mixed"))
    A64, Amx = h64.export_matrix(), hmx.export_matrix()
    assert np.abs(Amx - A64).max() <= 2e-6 * np.abs(A64).max()
    n = h64.n
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    h64.load_vector_one(b)
    u64, umx = torch.zeros_like(b), torch.zeros_like(b)
    h64.solve(b, u64, rtol=1e-12)
    it, rel, rc = hmx.solve(b, umx, rtol=1e-12)
    assert rc == F.FL_OK and rel <= 1e-12
    st = hmx.stats()
    assert st.last_outer >= 2
    fu = O.ball_fu(2, s)
    E = math.sqrt(h64.energy_error2(fu, b, u64))
    du = (umx - u64).cpu().numpy()
    gap = math.sqrt(du @ A64 @ du)
    assert gap <= 1e-3 * E
    # refined solution solves the mixed matrix to rtol
    r = b.cpu().numpy() - Amx @ umx.cpu().numpy()
    assert np.linalg.norm(r) <= 2e-12 * np.linalg.norm(b.cpu().numpy())
    h64.close()
    hmx.close()
