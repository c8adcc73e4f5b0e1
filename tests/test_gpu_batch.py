"""Batched instances (one launch per stage and instance group): every instance
solved in the batch equals the same instance solved through its own plan
(bit-identical: the same kernels in the same reduction order), and matches the
FP64 oracle."""
import numpy as np
import pytest

from oracle import ibdl_oracle as O
from paper_2203_12126_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2203_12126_amd import ibdl  # noqa: E402


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def relerr(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def small_batch(count=7, seed=77, sizes=(64, 96, 128), prec=ibdl.MIXED, with_3d=True):
    """Instances of the ellipse batch recipe on small grids, plus (optionally) a
    3-D sphere instance, so the batch spans several (dim, n) groups and both bcs."""
    items = []
    for sp in W.config_batch(count=count, seed=seed, sizes=sizes):
        sp["nrhs"] = 1 + sp["nrhs"] % 3
        _, _, probs = W.batch_instance(sp)
        items.append(probs)
    if with_3d:
        items.append([W.table2_problem(16, 300) for _ in range(2)])
    inst = []
    for probs in items:
        p = probs[0]
        inst.append((p, len(probs)))
    batch = ibdl.Batch.from_problems(inst, prec=prec)
    data = [T(np.stack([q.data for q in probs])) for probs in items]
    g = [T(np.stack([q.g_tilde for q in probs])) for probs in items]
    return batch, items, data, g


@pytest.mark.parametrize("prec", [ibdl.MIXED, ibdl.FP64])
def test_batch_apply_equals_single(prec):
    batch, items, data, _ = small_batch(prec=prec)
    rng = np.random.default_rng(5)
    q = [T(rng.standard_normal(d.shape)) for d in data]
    out = batch.apply(q)
    for i, probs in enumerate(items):
        pl = ibdl.Plan.from_problem(probs[0], prec=prec)
        ref = pl.apply(q[i])
        assert torch.equal(out[i], ref), f"instance {i}"
        pl.close()
    batch.close()


def test_batch_solve_and_grid_equal_single():
    batch, items, data, g = small_batch()
    sol, info = batch.solve(data, g, tol=1e-8)
    vb = [d if items[i][0].bc == W.NEUMANN else None for i, d in enumerate(data)]
    u = batch.eval_grid(sol, vb=vb, g=g)
    r = 0
    for i, probs in enumerate(items):
        pl = ibdl.Plan.from_problem(probs[0], prec=ibdl.MIXED)
        s1, i1 = pl.solve(data[i], g[i], tol=1e-8)
        assert torch.equal(sol[i], s1), f"instance {i}"
        assert [x["iters"] for x in info[r:r + len(probs)]] == [x["iters"] for x in i1]
        assert all(x["status"] == ibdl.OK for x in info[r:r + len(probs)])
        u1 = pl.eval_grid(s1, vb=vb[i], g=g[i])
        assert torch.equal(u[i], u1), f"instance {i}"
        r += len(probs)
        pl.close()
    batch.close()


def test_batch_solutions_match_oracle():
    batch, items, data, g = small_batch(count=4, seed=91, with_3d=False)
    sol, info = batch.solve(data, g, tol=1e-10)
    for i, probs in enumerate(items):
        st = O.setup_from_problem(probs[0])
        ref, _ = O.solve(st, probs[0].data, probs[0].g_tilde, bc=probs[0].bc, tol=1e-13)
        assert relerr(sol[i][0].cpu().numpy(), ref.x) < 1e-6, f"instance {i}"
    batch.close()


def test_batch_argument_errors():
    batch, items, data, g = small_batch(count=3, with_3d=False)
    with pytest.raises(ValueError):
        batch.solve(data[:-1] + [None], g)
    o = ibdl.SolveOpts(1e-8, 50, 500, data[0].data_ptr(), 0)
    arr = ibdl._ptr_array(data, "data", batch._sizes())
    out = ibdl._ptr_array([torch.empty_like(d) for d in data], "sol", batch._sizes())
    import ctypes
    st = ibdl.lib().ibdl_batch_solve(batch._h, arr, None, ctypes.byref(o), out, None, None)
    assert st == ibdl.ERR_ARG and "x0" in ibdl.last_error()
    neu = [i for i, p in enumerate(items) if p[0].bc == W.NEUMANN]
    if neu:
        with pytest.raises(ibdl.IbdlError):
            batch.eval_grid(data, vb=None, g=g)
    batch.close()
