"""Checkpoint / resume of a transient run (rte_snapshot / rte_restore) and
the restart of a run from a new state (rte_set_state)."""
import numpy as np
import pytest

import rte_inputs as ri
from oracle import pn

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, float).ravel()
    b = np.asarray(b, float).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _outputs(s):
    return {"state": s.get_state(), "phi_int": s.fluence(1), "readings": s.readings(),
            "residuals": s.residuals(), "steps": s.steps_done()}


@pytest.mark.parametrize("prec,n", [("f32", 32), ("f64", 48), ("f32", 128)])
def test_snapshot_destroy_restore_continues_bitwise(torch_cuda, prec, n):
    """Run k steps, snapshot, destroy the solver, create a fresh one from
    the same inputs, restore and run on: state, step count, integrated
    fluence, readings and residuals equal bitwise those of one
    uninterrupted run."""
    from paper_1801_06364_amd.rte import Solver
    total, cut = 9, 4
    print(f"\n[resume] p7_spheres n={n} {prec} {cut}+{total - cut} steps", flush=True)
    wl = ri.workload("p7_spheres", n=n, steps=total, precision=prec)
    s = Solver.from_workload(wl)
    s.step(total)
    ref = _outputs(s)
    s.close()
    s = Solver.from_workload(wl)
    s.step(cut)
    snap = s.snapshot()
    s.close()
    del s
    s = Solver.from_workload(wl)
    s.restore(snap)
    assert s.steps_done() == cut
    s.step(total - cut)
    got = _outputs(s)
    s.close()
    assert got["steps"] == total
    for k in ("state", "phi_int", "readings", "residuals"):
        assert np.array_equal(got[k], ref[k]), k


def test_restore_refuses_other_medium_or_short_input(torch_cuda):
    from paper_1801_06364_amd import rte
    wl = ri.workload("p7_spheres", n=16, steps=3, precision="f32")
    s = rte.Solver.from_workload(wl)
    s.step(2)
    snap = s.snapshot()
    mu_a = wl.mu_a.copy()
    mu_a[5, 5, 5] *= 1.5
    o = rte.Solver.from_workload(wl, mu_a=mu_a)
    with pytest.raises(rte.RteError) as e:
        o.restore(snap)
    assert e.value.code == rte.RTE_EINVAL
    with pytest.raises(rte.RteError) as e:
        s.restore(snap[:-8])
    assert e.value.code == rte.RTE_EINVAL
    bad = bytearray(snap)
    bad[0] ^= 0xFF
    with pytest.raises(rte.RteError) as e:
        s.restore(bytes(bad))
    assert e.value.code == rte.RTE_EINVAL
    s.restore(snap)
    assert s.steps_done() == 2
    o.close()
    s.close()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_set_state_on_a_handle_created_empty(torch_cuda, prec, tol):
    """A solver created with no initial state and no source, given a
    non-zero state by rte_set_state, steps on normally (the runaway-growth
    threshold follows the new state) and matches the oracle."""
    from paper_1801_06364_amd.rte import Solver
    n, steps = 32, 10
    wl = ri.workload("p7_spheres", n=n, steps=steps, precision=prec)
    psi = ri.gaussian_ic(n, wl.N, sigma=1.5)
    s = Solver.from_workload(wl, psi0=None, q=None)
    s.set_state(psi)
    s.step(steps)
    assert s.steps_done() == steps
    got = s.get_state()
    s.close()
    ref = pn.solve(wl.n, wl.N, wl.dx, wl.c, wl.dt, wl.mu_a, wl.mu_s, wl.g, psi, None, wl.W,
                   wl.mu0, wl.mu1, steps, det_index=wl.det_index)
    assert rel(got, ref["state"]) <= tol


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_flux_only_initial_state(torch_cuda, prec, tol):
    """An initial state with zero fluence and a non-zero flux (l = 1
    moments only) is a valid start: no false runaway stop, oracle parity."""
    from paper_1801_06364_amd.rte import Solver
    n, steps = 32, 10
    wl = ri.workload("p7_spheres", n=n, steps=steps, precision=prec)
    g = ri.gaussian_ic(n, wl.N, sigma=1.5)[0]
    psi = np.zeros((4, n, n, n))
    psi[1] = 0.3 * g
    psi[2] = -0.2 * g
    psi[3] = 0.5 * g
    s = Solver.from_workload(wl, psi0=psi, q=None, record_steps=steps)
    s.step(steps)
    assert s.steps_done() == steps
    got = s.get_state()
    fl = s.fluence()
    s.close()
    ref = pn.solve(wl.n, wl.N, wl.dx, wl.c, wl.dt, wl.mu_a, wl.mu_s, wl.g, psi, None, wl.W,
                   wl.mu0, wl.mu1, steps, det_index=wl.det_index)
    assert np.abs(ref["fluence"]).max() > 0
    assert rel(got, ref["state"]) <= tol
    assert rel(fl, ref["fluence"]) <= tol
