"""Batched path (several s, many right-hand sides) through the C ABI against
the CPU oracle.

* Matrices of fl_assemble_batch: the FP64 bar of the single-s path
  (max|dA| <= 1e-10 max|A|, ||dA||_F <= 1e-10 ||A||_F).
* Load vectors: same rule on both sides, relative 1e-12.
* fl_matmul, elementwise |Y - A_o X| <= g * sum_k |A_ik| |X_kc|
  + 1e-10 max|A| sum_k |X_kc| (the second term: the device matrix agrees
  with the oracle's A_o to 1e-10 max|A|), g from the storage and
  accumulation arithmetic:
    f64     g = n 2^-53
    f32     g = 2^-24 (A rounded to FP32) + n 2^-24 (FP32 accumulation,
            recursive-summation bound) ; X is given in FP32
    bf16    g = 2^-8 (A rounded to bf16, 8 significant bits, after the FP32
            rounding 2^-24) + 2^-24 + 2^-16 (X split into bf16 hi + lo:
            |x - hi| <= 2^-8 |x|, lo rounds that to 2^-8 relative) + n 2^-24
    bf16x2  g = 2^-16 (A as hi + lo) + 2^-24 + 2^-16 (X split) + 2^-16 (the
            dropped A_lo X_lo product) + n 2^-24
* fl_solve_batch at rtol 1e-13 (FP64 CG, or CG in FP32 arithmetic on the
  FP32 / bf16 matrix with FP64 solution and FP64 residual replacement):
  ||u - u_oracle||_A <= 1e-10 ||u_oracle||_A, the oracle solving its own
  matrix and load vector by Cholesky.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1708_03912_amd import fraclap as F, meshgen as M  # noqa: E402

TOL = 1e-10
SVALS = [0.1, 0.5, 0.9]


def orders():
    return O.Orders(k_touch=6, k_touch_bnd=6, theta=[1.5, 3.0, 6.0], k_far=[4, 3, 2, 2], k_far_bnd=[4, 3, 2, 2])


_cache = {}


def case(cells, seed=2):
    """mesh, oracle matrices (interior DOFs) for SVALS, DOF list"""
    key = (cells, seed)
    if key not in _cache:
        mesh = M.disk_for_cells(cells, seed=seed)
        mats = []
        for s in SVALS:
            A, dofs, _ = O.assemble(mesh, s, orders(), mode="interior")
            mats.append(A)
        _cache[key] = (mesh, mats, dofs)
    return _cache[key]


def batch_handle(mesh, svals=SVALS):
    h = F.Handle(0)
    h.set_mesh(mesh)
    h.assemble_batch(svals, F.make_opts(dof_mode="interior"))
    return h


def fourier_coeffs(nrhs, seed0=1000):
    return np.stack([np.random.default_rng(seed0 + m).standard_normal(16) for m in range(nrhs)])


def fourier_fn(coef):
    def f(x):
        x = np.atleast_2d(x)
        out = np.zeros(x.shape[0])
        for k1 in range(4):
            for k2 in range(4):
                out += coef[4 * k1 + k2] * np.cos(np.pi * (k1 * x[:, 0] + k2 * x[:, 1]))
        return out
    return f


@pytest.mark.parametrize("cells", [600, 1400])
def test_batch_matrices_match_oracle(cells):
    mesh, mats, dofs = case(cells)
    print(f"case batch matrices cells={cells}", flush=True)
    h = batch_handle(mesh)
    assert h.n == len(dofs)
    assert np.array_equal(h.dofs(), dofs)
    for j, Ao in enumerate(mats):
        A = h.export_batch_matrix(j)
        scale = np.abs(Ao).max()
        assert np.abs(A - Ao).max() <= TOL * scale
        assert np.linalg.norm(A - Ao) <= TOL * np.linalg.norm(Ao)
        # symmetric up to the summation order of the FP64 atomics
        assert np.abs(A - A.T).max() <= 1e-14 * scale
    h.close()


def test_batch_dof_sets_must_agree():
    mesh = M.disk_for_cells(300)
    h = F.Handle(0)
    h.set_mesh(mesh)
    with pytest.raises(F.FraclapError) as e:
        h.assemble_batch([0.25, 0.75], F.make_opts(dof_mode="paper"))
    assert e.value.code == F.FL_EINVAL
    # same side of 1/2 in paper mode is fine: all nodes
    n = h.assemble_batch([0.2, 0.3], F.make_opts(dof_mode="paper"))
    assert n == len(mesh["verts"])
    h.close()


def test_load_vectors_match_oracle():
    mesh, mats, dofs = case(1400)
    print("case load vectors", flush=True)
    h = batch_handle(mesh)
    n = h.n
    nrhs = 5
    coef = fourier_coeffs(nrhs)
    b = torch.zeros(nrhs, n, dtype=torch.float64, device="cuda")
    h.load_vector("fourier16", b, coef)
    bg = b.cpu().numpy()
    for c in range(nrhs):
        bo = O.load_vector_fn(mesh, dofs, fourier_fn(coef[c]), k=4)
        assert np.abs(bg[c] - bo).max() <= 1e-12 * np.abs(bo).max()
    # P1 nodal data of a linear function: the interpolant is the function, the
    # order-4 rule is exact for the degree-2 integrand
    V = np.asarray(mesh["verts"])
    lin = [(1.0, 0.0, 0.0), (0.3, -1.2, 2.5), (-2.0, 0.7, 0.1)]
    nod = np.stack([a + bx * V[:, 0] + by * V[:, 1] for a, bx, by in lin])
    b2 = torch.zeros(len(lin), n, dtype=torch.float64, device="cuda")
    h.load_vector("nodal", b2, nod)
    for c, (a, bx, by) in enumerate(lin):
        bo = O.load_vector_fn(mesh, dofs, lambda x, a=a, bx=bx, by=by: a + bx * x[:, 0] + by * x[:, 1], k=4)
        assert np.abs(b2[c].cpu().numpy() - bo).max() <= 1e-12 * np.abs(bo).max()
    b3 = torch.zeros(2, n, dtype=torch.float64, device="cuda")
    h.load_vector("one", b3)
    bo = O.load_vector_one(mesh, dofs)
    for c in range(2):
        assert np.abs(b3[c].cpu().numpy() - bo).max() <= 1e-14 * np.abs(bo).max()
    h.close()


def gemm_bound(dtype, n):
    u24 = 2.0 ** -24
    g = {"f64": n * 2.0 ** -53, "f32": u24 + n * u24, "bf16": 2.0 ** -8 + 2 * u24 + 2.0 ** -16 + n * u24,
         "bf16x2": 3 * 2.0 ** -16 + u24 + n * u24}
    return g[dtype]


def check_gemm(Y, Xq, Ao, dtype):
    """Y, Xq: (nrhs, n) rows = columns of the column-major operands."""
    n = Ao.shape[0]
    ref = Xq @ Ao                      # (A X)^T = X^T A, A symmetric
    mag = np.abs(Xq) @ np.abs(Ao)
    par = TOL * np.abs(Ao).max() * np.abs(Xq).sum(axis=1)[:, None]
    err = np.abs(Y - ref)
    assert np.all(np.isfinite(Y))
    assert np.all(err <= gemm_bound(dtype, n) * mag + par), (dtype, (err / (mag + 1e-300)).max())


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "bf16x2"])
def test_matmul_all_types(dtype):
    mesh, mats, dofs = case(1400)
    print(f"case matmul {dtype}", flush=True)
    h = batch_handle(mesh)
    n, ns, nrhs = h.n, len(SVALS), 37
    rng = np.random.default_rng(7)
    X = rng.standard_normal((ns, nrhs, n))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    Xt = torch.tensor(X, dtype=tdt, device="cuda")
    Yt = torch.full((ns, nrhs, n), float("nan"), dtype=tdt, device="cuda")
    h.matmul(Xt, Yt, dtype)
    Xq = Xt.double().cpu().numpy()
    Y = Yt.double().cpu().numpy()
    for j, Ao in enumerate(mats):
        check_gemm(Y[j], Xq[j], Ao, dtype)
    # one matrix of the batch
    Y1 = torch.full((nrhs, n), float("nan"), dtype=tdt, device="cuda")
    h.matmul(Xt[1].contiguous(), Y1, dtype, s_index=1)
    check_gemm(Y1.double().cpu().numpy(), Xq[1], mats[1], dtype)
    h.close()


def test_matmul_more_than_64_columns_and_tuner():
    mesh, mats, dofs = case(600)
    print("case matmul 70 columns + tuner", flush=True)
    h = batch_handle(mesh)
    n, ns, nrhs = h.n, len(SVALS), 70
    for dt in ("f64", "f32", "bf16", "bf16x2"):
        rows, best = h.autotune(dt)
        assert len(rows) >= 4 and 0 <= best < len(rows)
        assert all(r["ms"] > 0 for r in rows)
        assert rows[best]["ms"] == min(r["ms"] for r in rows)
    X = np.random.default_rng(3).standard_normal((ns, nrhs, n))
    Xt = torch.tensor(X, dtype=torch.float32, device="cuda")
    Yt = torch.full((ns, nrhs, n), float("nan"), dtype=torch.float32, device="cuda")
    h.matmul(Xt, Yt, "f32")
    Xq = Xt.double().cpu().numpy()
    for j, Ao in enumerate(mats):
        check_gemm(Yt[j].double().cpu().numpy(), Xq[j], Ao, "f32")
    h.close()


def a_norm_rel(A, u, uo):
    d = u - uo
    return np.sqrt(max(d @ A @ d, 0.0)) / np.sqrt(uo @ A @ uo)


@pytest.mark.parametrize("inner", ["f64", "f32", "bf16", "bf16x2"])
def test_solve_batch_matches_oracle(inner):
    mesh, mats, dofs = case(1400)
    print(f"case solve_batch inner={inner}", flush=True)
    h = batch_handle(mesh)
    n, ns, nrhs = h.n, len(SVALS), 6
    coef = fourier_coeffs(nrhs)
    b = torch.zeros(nrhs, n, dtype=torch.float64, device="cuda")
    h.load_vector("fourier16", b, coef)
    U = torch.full((ns, nrhs, n), float("nan"), dtype=torch.float64, device="cuda")
    it, rel, rc = h.solve_batch(b, U, rtol=1e-13, maxit=5000, inner=inner)
    assert rc == F.FL_OK, (it, rel)
    assert np.all(rel <= 1e-13)
    Ug = U.cpu().numpy()
    for c in range(nrhs):
        bo = O.load_vector_fn(mesh, dofs, fourier_fn(coef[c]), k=4)
        for j, Ao in enumerate(mats):
            uo = O.solve_cholesky(Ao, bo)
            assert a_norm_rel(Ao, Ug[j, c], uo) <= TOL, (j, c)
    # iteration counts grow with s (Sec. 5: condition number ~ h^{-2s})
    assert np.all(it > 0)
    assert it[2].mean() > it[0].mean()
    h.close()


def test_solve_batch_per_s_rhs_zero_column_and_chunks():
    mesh, mats, dofs = case(600)
    print("case solve_batch per-s rhs", flush=True)
    h = batch_handle(mesh)
    n, ns, nrhs = h.n, len(SVALS), 66
    rng = np.random.default_rng(11)
    Bm = rng.standard_normal((ns, nrhs, n))
    Bm[1, 5] = 0.0
    Bt = torch.tensor(Bm, device="cuda")
    U = torch.full((ns, nrhs, n), float("nan"), dtype=torch.float64, device="cuda")
    it, rel, rc = h.solve_batch(Bt, U, rtol=1e-13, maxit=5000, inner="bf16x2")
    assert rc == F.FL_OK
    Ug = U.cpu().numpy()
    assert np.all(Ug[1, 5] == 0.0) and it[1, 5] == 0
    for j in range(ns):
        for c in (0, 5, 63, 64, 65):
            if j == 1 and c == 5:
                continue
            uo = O.solve_cholesky(mats[j], Bm[j, c])
            assert a_norm_rel(mats[j], Ug[j, c], uo) <= TOL
    h.close()


def test_batch_errors_and_state():
    mesh = M.disk_for_cells(300)
    h = F.Handle(0)
    h.set_mesh(mesh)
    x = torch.zeros(1, 10, dtype=torch.float64, device="cuda")
    with pytest.raises(F.FraclapError) as e:
        h.matmul(x, x.clone(), "f64", s_index=0)
    assert e.value.code == F.FL_ESTATE
    n = h.assemble_batch([0.3, 0.6], F.make_opts(dof_mode="interior"))
    X = torch.zeros(2, 3, n, dtype=torch.float64, device="cuda")
    Y = torch.zeros_like(X)
    with pytest.raises(F.FraclapError) as e:
        h.matmul(X, Y, 7)
    assert e.value.code == F.FL_EINVAL
    with pytest.raises(F.FraclapError) as e:
        h.matmul(X[0], Y[0], "f64", s_index=2)
    assert e.value.code == F.FL_EINVAL
    # the single-s calls need fl_assemble
    with pytest.raises(F.FraclapError) as e:
        h.matvec(X[0, 0], Y[0, 0])
    assert e.value.code == F.FL_ESTATE
    # a new mesh drops the batch
    h.set_mesh(mesh)
    with pytest.raises(F.FraclapError) as e:
        h.matmul(X, Y, "f64")
    assert e.value.code == F.FL_ESTATE
    h.close()
