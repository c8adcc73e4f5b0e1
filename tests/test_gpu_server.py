"""Serving loop: results alone vs in the mix, admission by memory footprint,
isolation of failing requests, the footprint as an upper bound."""
import time

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


def small_stream(count=40, seed=355):
    specs = W.config_serve(count=count, seed=seed, sizes2=(64, 96, 128), sizes3=(16, 24, 32))
    for s in specs:
        s["m"] = min(s["m"], 600 if s["dim"] == 2 else 1500)
    return specs


def alone(prob, prec):
    pl = ibdl.Plan.from_problem(prob, prec=prec)
    data = T(prob.data).reshape(1, -1)
    g = T(prob.g_tilde).reshape(1, -1)
    # a served request is a solve with its grid solution (V_b = data for Neumann)
    sol, u, info = pl.solve_grid(data, g, tol=1e-8)
    pl.close()
    return sol, u, info


def test_server_results_equal_alone():
    specs = small_stream()[:14]
    probs = [W.serve_instance(s) for s in specs]
    precs = [ibdl.MIXED if i % 3 else ibdl.FP64 for i in range(len(probs))]
    ref = [alone(p, pr) for p, pr in zip(probs, precs)]
    srv = ibdl.Server(max_slots=64, streams=4)
    tickets = []
    # a first wave, then more requests while the first is on the device
    for i in range(8):
        tickets.append(srv.submit_problem(probs[i], prec=precs[i]))
    t0 = time.perf_counter()
    while srv.stats()["cohorts"] < 1 and time.perf_counter() - t0 < 10.0:
        time.sleep(0.0005)  # the first wave is admitted (its plans are building or solving)
    for i in range(8, len(probs)):
        tickets.append(srv.submit_problem(probs[i], prec=precs[i]))
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(probs) and st["cohorts"] >= 2
    for i, (r, (sol, u, info)) in enumerate(zip(res, ref)):
        assert r["status"] == ibdl.OK
        assert torch.equal(r["sol"], sol), f"request {i} ({specs[i]['dim']}-D n={specs[i]['n']})"
        assert torch.equal(r["u"], u), f"request {i}"
        assert r["info"][0]["iters"] == info[0]["iters"]
        assert r["times"]["total_ms"] >= r["times"]["run_ms"] >= 0.0


def test_server_admission_by_footprint():
    specs = small_stream(count=12, seed=7)[:6]
    probs = [W.serve_instance(s) for s in specs]
    fps = [ibdl.Server.footprint(p.grid.dim, p.grid.n, p.geom.m, bc=p.bc) for p in probs]
    budget = max(fps) + 1
    srv = ibdl.Server(budget_bytes=budget, max_slots=64, streams=4)
    tickets = [srv.submit_problem(p) for p in probs]
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    # every pair of requests exceeds the budget, so they ran one at a time
    assert all(fps[i] + fps[j] > budget for i in range(len(fps)) for j in range(len(fps)) if i != j)
    assert st["peak_active"] == 1 and st["peak_in_use_bytes"] <= budget
    assert all(r["status"] == ibdl.OK for r in res)
    # a request larger than the whole budget is refused at submission
    big = W.serve_instance(dict(dim=2, n=512, shape="circle", radius=0.3, bc=W.DIRICHLET, alpha=1.0, m=8000,
                                c=1.0, seed=1))
    assert ibdl.Server.footprint(2, 512, 8000) > budget
    with pytest.raises(ibdl.IbdlError) as e:
        srv.submit_problem(big)
    assert e.value.status == ibdl.ERR_OOM
    srv.close()


def test_server_failing_request_is_isolated():
    specs = small_stream(count=10, seed=11)[:4]
    probs = [W.serve_instance(s) for s in specs]
    bad = probs[1]
    Xbad = bad.geom.X.copy()
    Xbad[3, 0] = np.nan
    srv = ibdl.Server(max_slots=64, streams=2)
    g = bad.grid
    tb = srv.submit(g.dim, g.n, tuple(g.lo), g.length, bad.alpha, T(Xbad), T(bad.geom.normal),
                    T(bad.geom.weight), T(bad.data).reshape(1, -1), T(bad.g_tilde).reshape(1, -1), bc=bad.bc)
    good = [srv.submit_problem(p) for i, p in enumerate(probs) if i != 1]
    rb = srv.wait(tb, raise_on_error=False)
    assert rb["status"] == ibdl.ERR_NUMERIC
    for t in good:
        assert srv.wait(t)["status"] == ibdl.OK
    assert srv.stats()["in_use_bytes"] == 0
    srv.close()


@pytest.mark.parametrize("dim,n,m,bc", [(2, 256, 2000, W.DIRICHLET), (2, 512, 6000, W.NEUMANN),
                                        (3, 64, 8000, W.DIRICHLET)])
def test_footprint_bounds_device_usage(dim, n, m, bc):
    if dim == 2:
        sp = dict(dim=2, n=n, shape="circle", radius=0.3, bc=bc, alpha=3.0, m=m, c=1.0, seed=5)
    else:
        sp = dict(dim=3, n=n, shape="sphere", axes=(0.3, 0.3, 0.3), bc=bc, alpha=3.0, m=m, c=1.0, seed=5)
    p = W.serve_instance(sp)
    data = T(p.data).reshape(1, -1)
    g = T(p.g_tilde).reshape(1, -1)
    sol = torch.empty_like(data)
    # the same solve once before measuring: what the runtime reserves once per
    # process (code objects, the scratch area of register-spilling kernels) is
    # not memory of the plan
    warm = ibdl.Plan.from_problem(p, prec=ibdl.MIXED)
    warm.solve(data, g, tol=1e-8, out=sol)
    warm.close()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    pl = ibdl.Plan.from_problem(p, prec=ibdl.MIXED)
    pl.solve(data, g, tol=1e-8, out=sol)
    torch.cuda.synchronize()
    used = free0 - torch.cuda.mem_get_info()[0]
    pl.close()
    fp = ibdl.footprint(dim, n, m, bc=bc, prec=ibdl.MIXED)
    assert used <= fp, (used, fp)
