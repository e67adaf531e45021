"""The cluster method's FP32 representation (fl_cluster_assemble with
precision FL_MIXED): the kernel and near blocks assembled in FP64, rounded
once to FP32 and kept so, products and sums in FP64.  Against the FP64
representation on the same mesh: the product to the FP32 rounding of the
blocks (relative 1e-6, below the cluster approximation's own error), the
operator symmetric to that level, the device bytes smaller, and CG on it
reaches the FP64 tolerance with an energy error equal to the FP64 one to
1e-5 relative; in 2D (m = 6, the 36-wide kernels) and 1D (m = 5)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1708_03912_amd import fraclap as F, meshgen as M  # noqa: E402


def _pair(mesh, s, m, leaf):
    hs = []
    for prec in ("fp64", "mixed"):
        h = F.Handle(0)
        h.set_mesh(mesh)
        n = h.cluster_assemble(s, F.make_opts(dof_mode="interior", precision=prec), m=m, eta=2.0, leaf=leaf)
        hs.append(h)
    return hs, n


@pytest.mark.parametrize("case", ["disk", "interval"])
def test_cluster_fp32_representation(case):
    if case == "disk":
        mesh, s, m, leaf = M.disk_for_cells(12000, seed=4), 0.6, 6, 32
    else:
        mesh, s, m, leaf = M.interval(2048), 0.3, 5, 16
    (h64, h32), n = _pair(mesh, s, m, leaf)
    b64, b32 = h64.cluster_info()["bytes"], h32.cluster_info()["bytes"]
    print(f"{case}: n={n} bytes fp64={b64} fp32={b32}", flush=True)
    assert b32 < 0.75 * b64
    g = torch.Generator(device="cuda").manual_seed(5)
    for _ in range(2):
        x = torch.rand(n, dtype=torch.float64, device="cuda", generator=g) - 0.5
        y64, y32 = torch.empty_like(x), torch.empty_like(x)
        h64.cluster_matvec(x, y64)
        h32.cluster_matvec(x, y32)
        err = float((y32 - y64).abs().max() / y64.abs().max())
        assert err <= 1e-6, err
    # symmetry: x . A y = y . A x to the FP32 rounding
    x = torch.rand(n, dtype=torch.float64, device="cuda", generator=g) - 0.5
    z = torch.rand(n, dtype=torch.float64, device="cuda", generator=g) - 0.5
    ax, az = torch.empty_like(x), torch.empty_like(x)
    h32.cluster_matvec(x, ax)
    h32.cluster_matvec(z, az)
    lhs, rhs = float(torch.dot(z, ax)), float(torch.dot(x, az))
    assert abs(lhs - rhs) <= 1e-6 * float(z.norm() * ax.norm())
    # the solve
    res = []
    for h in (h64, h32):
        bv = torch.empty(n, dtype=torch.float64, device="cuda")
        h.load_vector_one(bv)
        u = torch.zeros_like(bv)
        it, rel, rc = h.solve_cluster(bv, u, rtol=1e-10)
        assert rc == F.FL_OK and rel <= 1e-10
        res.append((it, float(torch.dot(bv, u))))
    print(f"  iterations fp64 {res[0][0]} fp32 {res[1][0]}; b.u {res[0][1]:.12e} {res[1][1]:.12e}", flush=True)
    assert abs(res[1][1] - res[0][1]) <= 1e-5 * abs(res[0][1])
    assert abs(res[1][0] - res[0][0]) <= max(3, res[0][0] // 20)
    h64.close()
    h32.close()
