"""Time-dependent sources q(r) s(t) (rte_set_source_profile) against the
oracle's fourth-order variation-of-constants step, the Euler step of
eq. (11), graph replay and the adjoint."""
import os

import numpy as np
import pytest

import rte_inputs as ri
from oracle import pn

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def rel(a, b):
    a = np.asarray(a, float).ravel()
    b = np.asarray(b, float).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _pulse(dt, steps, delta_frac=0.7):
    """A Gaussian pulse in time, sampled every 0.7 dt (knots fall inside
    steps), peaking a third of the way through the run."""
    delta = delta_frac * dt
    t = delta * np.arange(int(steps * dt / delta) + 3)
    t_peak, width = steps * dt / 3, steps * dt / 6
    return np.exp(-0.5 * ((t - t_peak) / width) ** 2), delta


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name,n,steps", [("p5_steady", 16, 12), ("p5_steady", 32, 6),
                                          ("paper_pml_steady", 16, 10)])
def test_pulsed_source_matches_oracle(torch_cuda, name, n, steps, prec):
    """Heterogeneous medium, absorbing layer, collimated slab source (RK4)
    or the offset Gaussian source (Euler), driven by a pulse in time."""
    from paper_1801_06364_amd.rte import Solver
    wl = ri.workload(name, n=n, steps=steps, precision=prec)
    samples, delta = _pulse(wl.dt, steps)
    print(f"\n[source] {name} n={n} {wl.scheme} {prec}", flush=True)
    ref = pn.solve(wl.n, wl.N, wl.dx, wl.c, wl.dt, wl.mu_a, wl.mu_s, wl.g, wl.psi0, wl.q, wl.W,
                   wl.mu0, wl.mu1, steps, scheme=wl.scheme, q_profile=(samples, delta))
    s = Solver.from_workload(wl)
    s.set_source_profile(samples, delta, rows=steps)
    s.step(steps)
    st = s.get_state()
    err = rel(st, ref["state"])
    print(f"[source] rel err {err:.2e}", flush=True)
    assert err <= TOL[prec]
    assert rel(s.fluence(1), ref["phi_int"]) <= TOL[prec]
    s.close()


def test_rows_past_the_table_use_the_last_row(torch_cuda):
    """A table shorter than the run repeats its last row: a profile that ends
    at 1 and a 3-row table give the same state as the full-length table."""
    from paper_1801_06364_amd.rte import Solver
    wl = ri.workload("p5_steady", n=16, steps=8, precision="f64")
    samples = np.array([0.0, 1.0, 1.0])
    delta = 1.5 * wl.dt
    out = []
    for rows in (3, 8):
        s = Solver.from_workload(wl)
        s.set_source_profile(samples, delta, rows=rows)
        s.step(8)
        out.append(s.get_state())
        s.close()
    assert rel(out[0], out[1]) <= 1e-14


def test_profile_graph_replay_bitwise(torch_cuda):
    """The weights are read through the control block, so the captured step
    graph and plain launches give bitwise identical results."""
    from paper_1801_06364_amd.rte import Solver
    wl = ri.workload("p5_steady", n=16, steps=6, precision="f32")
    samples, delta = _pulse(wl.dt, 6)
    outs = []
    for env in ("0", "1"):
        os.environ["RTE_NO_GRAPH"] = env
        s = Solver.from_workload(wl, stream=torch_cuda.cuda.Stream())
        s.set_source_profile(samples, delta, rows=6)
        s.step(6)
        outs.append(s.get_state())
        s.close()
    os.environ.pop("RTE_NO_GRAPH", None)
    assert np.array_equal(outs[0], outs[1])


def test_adjoint_with_profile_matches_finite_differences(torch_cuda):
    """With a pulsed source the checkpointed recomputation uses each step's
    own weights: the adjoint gradient equals central differences of the
    GPU FP64 loss."""
    from paper_1801_06364_amd.rte import Solver
    wl = ri.workload("p5_steady", n=16, steps=6, precision="f64")
    wl.det_index = np.array([(8 * 16 + 8) * 16 + 8, (5 * 16 + 9) * 16 + 7], np.int64)
    samples, delta = _pulse(wl.dt, 6)

    def readings(mu_a, mu_s):
        s = Solver.from_workload(wl, mu_a=mu_a, mu_s=mu_s)
        s.set_source_profile(samples, delta, rows=6)
        s.step(6)
        r = s.readings()
        s.close()
        return r

    r = readings(wl.mu_a, wl.mu_s)
    s = Solver.from_workload(wl)
    s.set_source_profile(samples, delta, rows=6)
    s.forward_checkpointed(6, 2)
    ga, gs = s.adjoint(2.0 * r)
    s.close()
    for (z, y, x) in [(7, 8, 8), (6, 9, 7)]:
        for grad, which in ((ga, "a"), (gs, "s")):
            ma, ms = wl.mu_a.copy(), wl.mu_s.copy()
            base = ma if which == "a" else ms
            h = 1e-3 * base[z, y, x]
            base[z, y, x] += h
            Jp = float((readings(ma, ms) ** 2).sum())
            base[z, y, x] -= 2 * h
            Jm = float((readings(ma, ms) ** 2).sum())
            fd = (Jp - Jm) / (2 * h)
            assert abs(fd - grad[z, y, x]) <= 1e-5 * abs(fd) + 1e-15, (which, fd, grad[z, y, x])
