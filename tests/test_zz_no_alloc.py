"""The allocation-free operator entry point (ibdl_apply_noalloc) against ibdl_apply,
through the C ABI: two calls in a row, the second with a smaller input, in both
precisions; calls beyond the scratch size are refused before any work."""
import numpy as np
import pytest

from paper_2203_12126_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2203_12126_amd import ibdl  # noqa: E402


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _plan(n, m, bc, prec, dim=2):
    if dim == 2:
        spec = dict(dim=2, n=n, shape="star", radius=0.3, bc=bc, alpha=7.0, m=m, c=1.0, seed=n)
    else:
        spec = dict(dim=3, n=n, shape="ellipsoid", axes=(0.3, 0.25, 0.2), bc=bc, alpha=7.0, m=m, c=1.0, seed=n)
    p = W.serve_instance(spec)
    return ibdl.Plan.from_problem(p, prec=prec), p.geom.m


@pytest.mark.parametrize("prec", [ibdl.FP64, ibdl.MIXED])
def test_noalloc_apply_equals_apply(prec):
    # first call: a larger plan and more right-hand sides; second: a smaller one
    for n, m, bc, nrhs, dim in [(512, 3000, W.NEUMANN, 4, 2), (64, 5000, W.DIRICHLET, 2, 3), (128, 1000, W.DIRICHLET, 1, 2)]:
        pl, mm = _plan(n, m, bc, prec, dim)
        q = T(W.random_density(mm, seed=n, nrhs=nrhs))
        ref = pl.apply(q)
        out = torch.full_like(ref, float("nan"))
        pl.apply_noalloc(q, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (n, dim, prec)
        # again on the same plan: the scratch keeps the last call's contents
        out2 = torch.full_like(ref, float("nan"))
        pl.apply_noalloc(q, out2)
        torch.cuda.synchronize()
        assert torch.equal(out2, ref)
        pl.close()


def test_noalloc_refuses_more_than_its_scratch():
    pl, mm = _plan(2048, 4000, W.DIRICHLET, ibdl.FP64)
    q = T(W.random_density(mm, seed=1, nrhs=8))
    out = torch.zeros_like(q)
    with pytest.raises(ibdl.IbdlError) as e:
        pl.apply_noalloc(q, out)
    assert e.value.status == ibdl.ERR_ARG and "scratch" in str(e.value)
    assert torch.count_nonzero(out) == 0
    # one right-hand side of the same plan fits
    pl.apply_noalloc(q[:1].contiguous(), out[:1])
    torch.cuda.synchronize()
    assert torch.equal(out[:1], pl.apply(q[:1].contiguous()))
    pl.close()
