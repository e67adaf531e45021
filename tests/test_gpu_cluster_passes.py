"""The cluster product's upward and downward passes (Sec. 6) in both of
their forms: shift coefficients staged through registers and LDS for
M = m^2 <= 64 (m = 3 and 6), read directly for larger M (m = 9).  On trees
of depth 7 and more, against the oracle's product to 1e-10; the same
product repeated after other vectors gives the same bits."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import cluster as H  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_1708_03912_amd import fraclap as F, meshgen as M  # noqa: E402

from test_gpu_parity import oracle_orders  # noqa: E402


@pytest.mark.parametrize("m,leaf", [(6, 8), (3, 10), (9, 8)])
def test_passes_parity_and_repeat(m, leaf):
    mesh, s, eta = M.disk_for_cells(3000, seed=4), 0.6, 2.0
    h = F.Handle(0)
    h.set_mesh(mesh)
    n = h.assemble(s, F.default_opts())
    h.cluster_build(m=m, eta=eta, leaf=leaf)
    info = h.cluster_info()
    A, dofs, _ = O.assemble(mesh, s, oracle_orders(F.default_opts()))
    Ho = H.build(mesh, dofs, A, s, m=m, eta=eta, leaf=leaf)
    print(f"m={m} (M={m * m}) leaf={leaf}: n={n} clusters={info['clusters']} leaves={info['leaves']}", flush=True)
    assert info["clusters"] == len(Ho.tree.clusters) and info["leaves"] == len(Ho.tree.leaves())
    rng = np.random.default_rng(m)
    xs = [rng.standard_normal(n) for _ in range(3)]
    first = None
    for k, x in enumerate(xs + [xs[0]]):
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        h.cluster_matvec(torch.tensor(x, device="cuda"), y)
        yg = y.cpu().numpy()
        if k == 0:
            first = yg.copy()
            yo = H.matvec(Ho, x)
            err = np.abs(yg - yo).max() / np.abs(yo).max()
            assert err <= 1e-10, err
        elif k < 3:
            yo = H.matvec(Ho, x)
            err = np.abs(yg - yo).max() / np.abs(yo).max()
            assert err <= 1e-10, err
        else:
            assert np.array_equal(yg.view(np.int64), first.view(np.int64))
    h.close()
