"""The allocation-free coarse Poisson solve (cgp_poisson_solve_noalloc) against cgp_poisson_solve,
through the C ABI: two calls in a row on one GPU, the second on a smaller system, each within the
FP64 parity bar of the allocating solve on the same right-hand side; device memory unchanged by the
calls; the mesh's own solver still correct afterwards; sizes beyond the fixed array and unsupported
options rejected."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-test]", *a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1610_06993_amd as cgp
    cgp.lib()
    return torch, cgp


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _mesh(cgp, coarse):
    g = cgp.Mesh(coarse, 1)
    g.assemble(1.0, 1e-3, 1e-3)
    return g


def test_noalloc_solve_matches_allocating_solve(env):
    torch, cgp = env
    X0 = cgp._native
    meshes = [("cylinder 40000", W.cylinder_channel(40000, seed=2)), ("Taylor-Green 24x24", W.unit_square_tg(24))]
    built = [(name, _mesh(cgp, m)) for name, m in meshes]
    assert built[1][1].info["n_c"] < built[0][1].info["n_c"]
    opts = cgp.SolverOpts(tol=1e-13, max_iter=100000, x0_mode=X0.X0_ZERO)
    warm = cgp.SolverOpts(tol=1e-13, max_iter=100000, x0_mode=X0.X0_PREV)
    rng = np.random.default_rng(3)
    # every tensor, and every torch kernel the test uses, exists before the device's free memory is read:
    # between the two readings only the allocation-free calls run
    bufs = []
    for name, g in built:
        n = g.info["n_c"]
        t = dict(b=torch.from_numpy(rng.normal(size=n)).cuda(), x_ref=torch.zeros(n, dtype=torch.float64, device="cuda"),
                 x=torch.full((n,), 7.0, dtype=torch.float64, device="cuda"))
        t["ref_stats"] = g.poisson_solve(t["b"], t["x_ref"], opts)
        t["xw"] = t["x_ref"] * (1.0 + 1e-6)
        t["x2"] = torch.zeros_like(t["x_ref"])
        bufs.append(t)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    cold = [g.poisson_solve_noalloc(t["b"], t["x"], opts) for (name, g), t in zip(built, bufs)]
    warmed = [g.poisson_solve_noalloc(t["b"], t["xw"], warm) for (name, g), t in zip(built, bufs)]
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    _say(f"device free memory before / after the allocation-free calls: {free0} / {free1}")
    assert free1 == free0
    for (name, g), t, st, st2 in zip(built, bufs, cold, warmed):
        ref = t["x_ref"].cpu().numpy()
        e = rel(t["x"].cpu().numpy(), ref)
        _say(f"noalloc solve {name}, {g.info['n_c']} rows: rel err {e:.2e}, iterations {st['p_iters']} vs "
             f"{t['ref_stats']['p_iters']}; from a start 1e-6 off: {st2['p_iters']}")
        assert e <= 1e-10 and st["p_relres"] <= 1e-13
        assert rel(t["xw"].cpu().numpy(), ref) <= 1e-10 and st2["p_iters"] < st["p_iters"]
        # the mesh's own buffers are back in use and untouched
        g.poisson_solve(t["b"], t["x2"], opts)
        assert rel(t["x2"].cpu().numpy(), ref) <= 1e-10


def test_noalloc_rejects_what_it_does_not_serve(env):
    torch, cgp = env
    X0 = cgp._native
    g = _mesh(cgp, W.unit_square_tg(8))
    b = torch.ones(g.info["n_c"], dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    for o in (cgp.SolverOpts(precision=X0.PREC_FP32_IR), cgp.SolverOpts(x0_mode=X0.X0_POD_GALERKIN),
              cgp.SolverOpts(launch=X0.LAUNCH_PERSISTENT), cgp.SolverOpts(tol=0.0)):
        with pytest.raises(cgp.CGPError) as e:
            g.poisson_solve_noalloc(b, x, o)
        assert e.value.status == X0.E_ARG
    big = _mesh(cgp, W.cylinder_channel(560_000, seed=2))
    assert big.info["n_c"] > 262144
    bb = torch.ones(big.info["n_c"], dtype=torch.float64, device="cuda")
    with pytest.raises(cgp.CGPError) as e:
        big.poisson_solve_noalloc(bb, torch.zeros_like(bb), cgp.SolverOpts())
    assert e.value.status == X0.E_ARG and "262144" in str(e.value)
