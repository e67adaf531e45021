"""fl_matvec_noalloc (the allocation-free product) against fl_matvec, through
the C ABI: the same kernels and plan, so the results agree bit for bit, on
two calls in a row with the second system smaller; and the size limit is
refused before anything is launched."""
import pytest

torch = pytest.importorskip("torch")

from paper_1708_03912_amd import fraclap as F, meshgen as M

pytestmark = pytest.mark.gpu


def _product_pair(h, n, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.rand(n, dtype=torch.float64, generator=g).cuda()
    y_ref = torch.empty_like(x)
    y_na = torch.full_like(x, float("nan"))
    h.matvec(x, y_ref)
    h.matvec_noalloc(x, y_na)
    torch.cuda.synchronize()
    return y_ref, y_na


def test_noalloc_matches_matvec_two_calls_second_smaller():
    sizes = []
    for cells, s, seed in ((3000, 0.75, 1), (900, 0.25, 2)):
        h = F.Handle(0)
        h.set_mesh(M.disk_for_cells(cells, seed=2))
        n = h.assemble(s)
        sizes.append(n)
        y_ref, y_na = _product_pair(h, n, seed)
        print(f"noalloc: cells={cells} s={s} n={n}", flush=True)
        assert torch.isfinite(y_na).all()
        assert torch.equal(y_ref, y_na), float((y_ref - y_na).abs().max())
        h.close()
    assert sizes[1] < sizes[0]


def test_noalloc_refuses_too_large_system():
    h = F.Handle(0)
    h.set_mesh(M.disk_for_cells(40000, seed=2))
    n = h.assemble(0.75, F.make_opts(dof_mode="interior"))
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(F.FraclapError) as e:
        h.matvec_noalloc(x, y)
    assert e.value.code == F.FL_EINVAL and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert float(y.abs().max()) == 0.0  # nothing was launched
    h.close()
