"""The symmetric product on sizes where a workgroup takes several block rows
(its column sums gathered over them in LDS): fl_matvec against the full
matrix's product (torch, FP64, both triangles read), and the FP64 and
mixed-precision CG against the true residual b - A u.  Disks of 6e4,
1.2e5 and 1.5e5 triangles (n ~ 3e4, 6e4, 7.4e4: 2, 8 and 16 block rows per
workgroup; the block counts 463 and 1163 leave a partial last workgroup
row)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1708_03912_amd import fraclap as F, meshgen as M  # noqa: E402


def _block_rows(n):
    # the grouping the library chooses for n unknowns (documented geometry)
    nb = (n + 63) // 64
    tiles = nb * (nb + 1) // 2
    m = max(3, min(16, tiles // 2048))
    R = 1
    while R < 16 and tiles // (m * 2 * R) >= 2048:
        R *= 2
    return R


@pytest.mark.parametrize("cells", [60000, 120000, 150000])
def test_grouped_product_and_cg(cells):
    mesh = M.disk_for_cells(cells, seed=7)
    s = 0.6
    h = F.Handle(0)
    h.set_mesh(mesh)
    n = h.assemble(s, F.make_opts(dof_mode="interior"))
    print(f"cells={cells} n={n} block rows per workgroup={_block_rows(n)}", flush=True)
    assert _block_rows(n) >= 2
    A = h.matrix_view()
    g = torch.Generator(device="cuda").manual_seed(cells)
    for trial in range(3):
        x = torch.rand(n, dtype=torch.float64, device="cuda", generator=g) - 0.5
        if trial == 2:
            x[: n // 3] = 0.0  # a vector zero on the leading blocks
        y = torch.empty_like(x)
        h.matvec(x, y)
        yr = torch.mv(A, x)
        err = float((y - yr).abs().max() / yr.abs().max())
        assert err <= 1e-13, err
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    h.load_vector_one(b)
    u = torch.zeros_like(b)
    it, rel, rc = h.solve(b, u, rtol=1e-10, maxit=20000)
    true_rel = float(torch.linalg.norm(b - torch.mv(A, u)) / torch.linalg.norm(b))
    print(f"  FP64 CG: {it} iterations, recursive {rel:.2e}, true {true_rel:.2e}", flush=True)
    assert rc == F.FL_OK and rel <= 1e-10 and true_rel <= 2e-10
    h.close()


def test_grouped_product_mixed_solve():
    """FP32 matrix (four columns per 16-byte load, two tiles per step) in
    the grouped layout: the refined solve reaches the FP64 tolerance."""
    mesh = M.disk_for_cells(120000, seed=8)
    s = 0.4
    h = F.Handle(0)
    h.set_mesh(mesh)
    n = h.assemble(s, F.make_opts(dof_mode="interior", precision="mixed"))
    assert _block_rows(n) >= 2
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    h.load_vector_one(b)
    u = torch.zeros_like(b)
    it, rel, rc = h.solve(b, u, rtol=1e-10, maxit=20000)
    A = h.matrix_view()
    true_rel = float(torch.linalg.norm(b - torch.mv(A, u)) / torch.linalg.norm(b))
    print(f"n={n} mixed solve: {it} iterations, {rel:.2e}, true {true_rel:.2e}", flush=True)
    assert rc == F.FL_OK and true_rel <= 2e-10
    h.close()
    assert np.isfinite(true_rel)
