"""Symmetry reduction on the GPU (Sec. 7) against the oracle: the reduced
matrix (sector cells against every image) to 1e-10, its solution equal to
the full symmetric solution, and the pair count cut by about K."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from oracle import symmetry as SY  # noqa: E402
from paper_1708_03912_amd import fraclap as F, meshgen as M  # noqa: E402

from test_gpu_parity import oracle_orders  # noqa: E402


@pytest.mark.parametrize("K,s,couples", [(2, 0.3, False), (4, 0.75, False), (8, 0.5, False),
                                          (2, 0.75, True), (4, 0.3, True), (8, 0.5, True)])
def test_reduced_matrix_parity(K, s, couples):
    """couples: one member of each equal couple of cross pairs (preimage and
    rotation of every cell given) instead of both with weight 1/2."""
    mesh, vfold, Tw, pre, rot = M.disk_symmetric(0.2, K, seed=6)
    h = F.Handle(0)
    h.set_mesh(mesh)
    if couples:
        h.set_symmetry(K, Tw, vfold, pre, rot)
    else:
        h.set_symmetry(K, Tw, vfold)
    n = h.assemble(s, F.default_opts())
    A = h.export_matrix()
    kw = dict(pre=pre, rot=rot, K=K) if couples else {}
    Ao, red, _ = SY.assemble_reduced(mesh, s, oracle_orders(F.default_opts()), vfold, Tw, **kw)
    assert n == len(red)
    assert np.abs(A - Ao).max() <= 1e-10 * np.abs(Ao).max()
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    h.load_vector_one(b)
    bo = SY.load_vector_reduced(mesh, vfold, Tw, red)
    assert np.abs(b.cpu().numpy() - bo).max() <= 1e-14 * np.abs(bo).max()
    h.close()


def test_reduced_solution_is_the_full_one():
    """d = 2, K = 4, s = 0.75: CG on the reduced system gives the full
    mesh's solution at the representatives (up to the quadrature's lack of
    exact rotation invariance); one member of each couple of equal cross
    pairs: about 1/K of the full mesh's separated pairs."""
    K, s = 4, 0.75
    mesh, vfold, Tw, pre, rot = M.disk_symmetric(0.08, K, seed=7)
    hf = F.Handle(0)
    hf.set_mesh(mesh)
    nf = hf.assemble(s)
    stf = hf.stats()
    bf = torch.empty(nf, dtype=torch.float64, device="cuda")
    hf.load_vector_one(bf)
    uf = torch.zeros_like(bf)
    hf.solve(bf, uf, rtol=1e-12)
    dofs_full = hf.dofs()
    hr = F.Handle(0)
    hr.set_mesh(mesh)
    hr.set_symmetry(K, Tw, vfold, pre, rot)
    nr = hr.assemble(s)
    str_ = hr.stats()
    br = torch.empty(nr, dtype=torch.float64, device="cuda")
    hr.load_vector_one(br)
    ur = torch.zeros_like(br)
    hr.solve(br, ur, rtol=1e-12)
    red = hr.dofs()
    assert np.all(np.asarray(vfold)[red] == red)
    pos = np.searchsorted(dofs_full, red)
    u_full = uf.cpu().numpy()
    assert np.abs(ur.cpu().numpy() - u_full[pos]).max() <= 1e-7 * np.abs(u_full).max()
    # energies: K a_red(u, u) = a(u, u)
    y = torch.empty_like(ur)
    hr.matvec(ur, y)
    yf = torch.empty_like(uf)
    hf.matvec(uf, yf)
    er, ef = float(torch.dot(ur, y)), float(torch.dot(uf, yf))
    assert abs(K * er - ef) <= 1e-7 * ef
    far_f, far_r = sum(stf.pairs_far), sum(str_.pairs_far)
    # computed pairs: the weight-0 half of the cross pairs is skipped tile by
    # tile, so small meshes (few blocks per image copy) keep more of it
    assert far_r < 0.5 * far_f, (far_r, far_f)
    hf.close()
    hr.close()


def test_symmetry_errors():
    mesh, vfold, Tw, pre, rot = M.disk_symmetric(0.3, 2, seed=1)
    h = F.Handle(0)
    h.set_mesh(mesh)
    bad = np.array(vfold)
    bad[0] = len(bad)
    with pytest.raises(F.FraclapError) as e:
        h.set_symmetry(2, Tw, bad)
    assert e.value.code == F.FL_EMESH
    with pytest.raises(F.FraclapError) as e:
        h.set_symmetry(2, len(mesh["cells"]) + 1, vfold)
    assert e.value.code == F.FL_EINVAL
    bad_pre = np.array(pre)
    bad_pre[-1] = (bad_pre[-1] + 1) % Tw
    with pytest.raises(F.FraclapError) as e:
        h.set_symmetry(2, Tw, vfold, bad_pre, rot)
    assert e.value.code == F.FL_EMESH
    h.set_symmetry(2, Tw, vfold, pre, rot)
    h.assemble(0.4)
    with pytest.raises(F.FraclapError) as e:
        h.cluster_build()
    assert e.value.code == F.FL_EINVAL
    # switching off restores the full system
    h.set_symmetry(1, 0, vfold)
    n = h.assemble(0.4)
    assert n == len(mesh["verts"])
    h.close()
