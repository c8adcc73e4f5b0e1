"""The row-pass shapes the tile autotuner chooses between (1, 2 or 4
right-hand sides per workgroup with several lines each, or one line of one
right-hand side) give bit-identical results, and the tuner records its
choices."""
import numpy as np
import pytest

from paper_2203_12126_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2203_12126_amd import ibdl  # noqa: E402


@pytest.mark.parametrize("dim,prec", [(2, ibdl.MIXED), (2, ibdl.FP64), (3, ibdl.MIXED)])
def test_row_block_variants_bit_identical(dim, prec):
    if dim == 2:
        p = W.config_star1024(m=1500, n=256, alpha=3.0, seed=9)
    else:
        p = W.table2_problem(32, 2000)
    ibdl.set_autotune(False)  # fixed rule: 4 rhs -> 4 per block, 2 -> 2, 1 -> 1
    try:
        pl = ibdl.Plan.from_problem(p, prec=prec)
        rng = np.random.default_rng(3)
        q = torch.as_tensor(rng.standard_normal((4, p.geom.m)), device="cuda")
        four = pl.apply(q)
        two = torch.cat([pl.apply(q[0:2].contiguous()), pl.apply(q[2:4].contiguous())])
        one = torch.cat([pl.apply(q[i:i + 1].contiguous()) for i in range(4)])
        assert torch.equal(four, two) and torch.equal(four, one)
        g = torch.as_tensor(np.stack([p.g_tilde.ravel()] * 4), device="cuda")
        u4 = pl.eval_grid(q, vb=q if p.bc == W.NEUMANN else None, g=g)
        u1 = torch.cat([pl.eval_grid(q[i:i + 1].contiguous(), vb=q[i:i + 1].contiguous() if p.bc == W.NEUMANN
                                     else None, g=g[i:i + 1].contiguous()) for i in range(4)])
        assert torch.equal(u4, u1)
        pl.close()
    finally:
        ibdl.set_autotune(True)


def test_autotuner_records_choices():
    ibdl.set_autotune(True)
    p = W.config_star1024(m=1500, n=192, alpha=1.0, seed=4)
    pl = ibdl.Plan.from_problem(p, prec=ibdl.MIXED)
    q = torch.as_tensor(np.random.default_rng(1).standard_normal((3, p.geom.m)), device="cuda")
    first = pl.apply(q)          # tunes: every variant runs
    second = pl.apply(q)         # uses the choice
    assert torch.equal(first, second)
    rep = ibdl.autotune_report()
    assert "n=192" in rep and "row_fwd" in rep and "row_inv" in rep
    pl.close()


def test_timing_on_a_pass_that_tunes():
    """A pass that tunes its row stages while stage timing is on still records
    every stage's events (the tuned stage runs once more under them)."""
    ibdl.set_autotune(True)  # clears the choices: the next pass tunes
    p = W.config_star1024(m=1500, n=128, alpha=1.0, seed=6)
    pl = ibdl.Plan.from_problem(p, prec=ibdl.MIXED)
    q = torch.as_tensor(np.random.default_rng(2).standard_normal((2, p.geom.m)), device="cuda")
    pl.set_timing(True)
    out = pl.apply(q)
    names = [nm for nm, ms, calls in pl.stage_times()]
    assert {"spread+fft_x", "fft_y+symbol", "ifft_x+interp", "finish"} <= set(names)
    assert torch.equal(out, pl.apply(q))
    pl.set_timing(False)
    pl.close()


@pytest.mark.parametrize("n", [192, 256])
@pytest.mark.parametrize("prec", [ibdl.MIXED, ibdl.FP64])
def test_every_row_shape_bit_identical(prec, n):
    """Each of the four row-block shapes, forced in turn, gives the same apply,
    grid solution and solve, bit for bit.  At n = 256 the blocks of 16 lines keep
    their LDS rows column-swizzled and the one-line shape keeps them plain; at
    n = 192 (21, 20 and 20 lines) all shapes use padded rows."""
    p = W.config_star1024(m=1500, n=n, alpha=2.0, seed=12)
    rng = np.random.default_rng(8)
    q = torch.as_tensor(rng.standard_normal((3, p.geom.m)), device="cuda")
    g = torch.as_tensor(np.stack([p.g_tilde.ravel()] * 3), device="cuda")
    outs = []
    try:
        for v in range(4):
            ibdl.set_autotune(force=v)
            pl = ibdl.Plan.from_problem(p, prec=prec)
            a = pl.apply(q)
            u = pl.eval_grid(q, g=g)
            s, _ = pl.solve(q, g, tol=1e-9)
            outs.append((a, u, s))
            pl.close()
    finally:
        ibdl.set_autotune(True)
    for v in range(1, 4):
        for x, y in zip(outs[0], outs[v]):
            assert torch.equal(x, y), f"shape {v}"


def test_autotune_mode_errors():
    assert ibdl.lib().ibdl_set_autotune(9) == ibdl.ERR_ARG
    ibdl.set_autotune(True)
