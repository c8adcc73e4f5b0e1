"""The seeded input generators: fast paths agree with the direct definitions."""
import numpy as np

from paper_2203_12126_amd import workloads as W


def test_separable_forcing_matches_direct_evaluation():
    specs = W.config_batch(count=8, sizes=(64, 96))
    for sp in specs[:3]:
        _, _, fast = W.batch_instance(sp, fast=True)
        _, _, slow = W.batch_instance(sp, fast=False)
        for a, b in zip(fast, slow):
            assert np.max(np.abs(a.g_tilde - b.g_tilde)) <= 1e-12 * np.max(np.abs(b.g_tilde))
            assert np.array_equal(a.data, b.data)


def test_batch_config_recipe():
    specs = W.config_batch()
    assert len(specs) == 512
    assert {s["n"] for s in specs} == {128, 192, 256, 384, 512}
    assert all(2 <= s["nrhs"] <= 8 for s in specs)
    assert all(1.0 <= s["alpha"] <= 1000.0 for s in specs)
    assert {s["bc"] for s in specs} == {W.DIRICHLET, W.NEUMANN}
    # points at spacing 0.75 h along the ellipse
    for s in specs[:20]:
        per = W.ellipse_perimeter(s["a"], s["b"])
        assert abs(per / s["m"] - 0.75 / s["n"]) < 0.01 / s["n"]


def test_serve_instances_match_direct_evaluation():
    specs = W.config_serve(count=60, sizes2=(64, 96), sizes3=(16, 24))
    two = [s for s in specs if s["dim"] == 2][:2]
    three = [s for s in specs if s["dim"] == 3][:2]
    assert two and three
    for sp in two + three:
        p = W.serve_instance(sp)
        sol = p.sol
        pts = np.stack([c.ravel() for c in p.grid.nodes()], axis=1)
        g = np.where(p.geom.inside(pts), sol.lap(pts) - p.alpha * sol.u(pts), 0.0).reshape(p.g_tilde.shape)
        assert np.max(np.abs(g - p.g_tilde)) <= 1e-11 * max(1.0, np.max(np.abs(g)))


def test_serve_config_recipe():
    specs = W.config_serve()
    assert len(specs) == 2000
    frac3 = np.mean([s["dim"] == 3 for s in specs])
    assert 0.17 < frac3 < 0.23
    for s in specs:
        lo, hi = (1000, 16000) if s["dim"] == 2 else (5000, 40000)
        assert lo <= s["m"] <= hi
        assert 1.0 <= s["alpha"] <= 1000.0
        if s["dim"] == 3:
            assert s["bc"] == W.DIRICHLET
    arr = np.array([s["arrival"] for s in specs])
    assert np.all(np.diff(arr) > 0)
    assert abs(np.mean(np.diff(arr)) - 1.0) < 0.1


def test_star_forcing_matches_direct_evaluation():
    p = W.config_star1024(m=300, n=64, alpha=3.0, seed=5)
    pts = np.stack([c.ravel() for c in p.grid.nodes()], axis=1)
    g = np.where(p.geom.inside(pts), p.sol.lap(pts) - 3.0 * p.sol.u(pts), 0.0).reshape(p.g_tilde.shape)
    assert np.max(np.abs(g - p.g_tilde)) <= 1e-11 * np.max(np.abs(g))
    pn = W.config_star1024(m=300, n=64, alpha=3.0, seed=5, bc=W.NEUMANN)
    assert np.allclose(pn.data, np.sum(pn.sol.grad(pn.geom.X) * pn.geom.normal, axis=1), rtol=0, atol=1e-13)
