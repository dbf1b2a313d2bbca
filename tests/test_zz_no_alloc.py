"""rte_steady_gmres_static (Krylov workspace in the library's static device
array: no device allocation) against rte_steady_gmres with a caller-owned
workspace, through the C-ABI: two calls in a row, the second on a smaller
problem, each compared with the caller-workspace solve of the same input
(Arnoldi steps, residual, full state); and the size limit."""
import numpy as np
import pytest

import rte_inputs as ri

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _solve(wl, static, restart, K):
    from paper_1801_06364_amd.rte import Solver
    s = Solver.from_workload(wl)
    if static:
        it, res = s.steady_gmres_static(tol=1e-11, restart=restart, max_iters=3000, steps_per_apply=K)
    else:
        it, res = s.steady_gmres(tol=1e-11, restart=restart, max_iters=3000, steps_per_apply=K)
    st = s.get_state()
    s.close()
    return it, res, st


def test_static_gmres_matches_caller_workspace(torch_cuda):
    from paper_1801_06364_amd import rte
    cap = int(rte.lib().rte_static_scratch_bytes())
    cases = [
        # (grid, restart, steps per operator application): the second call is
        # the smaller problem and reuses the static array the first one filled
        (32, 8, 20),
        (16, 24, 0),
    ]
    for n, restart, K in cases:
        wl = ri.workload("p5_steady", n=n, steps=0, precision="f64")
        need = int(rte.lib().rte_krylov_workspace_bytes(rte.make_config(
            wl.n, wl.N, rte.RTE_FP64, wl.dx, wl.c, wl.dt, wl.W, wl.mu0, wl.mu1)[0], restart))
        assert 0 < need <= cap
        print(f"\n[noalloc] p5_steady n={n} restart={restart} K={K} workspace {need / 2**20:.1f} MiB "
              f"of {cap / 2**20:.0f}", flush=True)
        it0, res0, st0 = _solve(wl, False, restart, K)
        it1, res1, st1 = _solve(wl, True, restart, K)
        err = float(np.linalg.norm(st1 - st0) / np.linalg.norm(st0))
        print(f"[noalloc] caller ws: {it0} steps, residual {res0:.3e}; static: {it1} steps, "
              f"residual {res1:.3e}; state rel-L2 {err:.2e}", flush=True)
        assert res0 <= 1e-11 and res1 <= 1e-11
        assert it1 == it0
        assert err <= 1e-12
        assert np.array_equal(st1, st0)   # same kernels, same order: bitwise


def test_static_gmres_refuses_workspace_beyond_the_array(torch_cuda):
    from paper_1801_06364_amd import rte
    from paper_1801_06364_amd.rte import Solver
    wl = ri.workload("p5_steady", n=32, steps=0, precision="f64")
    restart = 20
    cfg = rte.make_config(wl.n, wl.N, rte.RTE_FP64, wl.dx, wl.c, wl.dt, wl.W, wl.mu0, wl.mu1)[0]
    assert int(rte.lib().rte_krylov_workspace_bytes(cfg, restart)) > int(rte.lib().rte_static_scratch_bytes())
    s = Solver.from_workload(wl)
    u0 = s.get_state()
    with pytest.raises(rte.RteError) as ei:
        s.steady_gmres_static(tol=1e-8, restart=restart)
    assert ei.value.code == rte.RTE_ENOMEM
    assert np.array_equal(s.get_state(), u0)   # refused before touching the state
    s.close()
