"""GPU discrete adjoint (rte_forward_checkpointed / rte_adjoint) against the
oracle's reverse-mode gradient, finite differences and itself."""
import numpy as np
import pytest

import rte_inputs as ri
from oracle import pn

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, float).ravel()
    b = np.asarray(b, float).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _problem(n=16, steps=8, prec="f64"):
    wl = ri.workload("p3_adjoint", n=n, steps=steps, precision=prec)
    tgt = ri.sphere_maps(n, wl.W, 5, seed=1005, radius=(1, max(1, n // 8)))
    return wl, tgt


def _readings(wl, mu_a, mu_s):
    from paper_1801_06364_amd.rte import Solver
    s = Solver.from_workload(wl, mu_a=mu_a, mu_s=mu_s)
    s.step(wl.steps)
    r = s.readings()
    s.close()
    return r


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_adjoint_matches_oracle(torch_cuda, prec, tol):
    """Same adjoint sources on both sides; gradient fields compared over the
    whole grid (FP64 <= 1e-10, FP32 <= 1e-4 relative L2)."""
    from paper_1801_06364_amd.rte import Solver
    wl, tgt = _problem(prec=prec)
    target = pn.solve(wl.n, wl.N, wl.dx, wl.c, wl.dt, tgt[0], tgt[1], tgt[2], wl.psi0, None, wl.W,
                      wl.mu0, wl.mu1, wl.steps, det_index=wl.det_index,
                      return_state=False)["readings"]
    ref = pn.solve(wl.n, wl.N, wl.dx, wl.c, wl.dt, wl.mu_a, wl.mu_s, wl.g, wl.psi0, None, wl.W,
                   wl.mu0, wl.mu1, wl.steps, det_index=wl.det_index, return_state=False)
    djdr = 2.0 * (ref["readings"] - target)
    ga_ref, gs_ref = pn.adjoint_gradient(wl.n, wl.N, wl.dx, wl.c, wl.dt, wl.mu_a, wl.mu_s, wl.g,
                                         wl.psi0, None, wl.W, wl.mu0, wl.mu1, wl.steps,
                                         wl.det_index, djdr)
    s = Solver.from_workload(wl)
    s.forward_checkpointed(wl.steps, 3)
    ga, gs = s.adjoint(djdr)
    assert s.steps_done() == wl.steps
    s.close()
    assert rel(ga, ga_ref) <= tol
    assert rel(gs, gs_ref) <= tol
    omega = pn.pml_depth(wl.n, wl.W) == 0
    assert np.all(ga[~omega] == 0.0) and np.all(gs[~omega] == 0.0)


def test_euler_adjoint_matches_oracle(torch_cuda):
    """Adjoint of the first-order step of eq. (11) on the GPU (FP64) against
    the oracle's reverse sweep."""
    from paper_1801_06364_amd.rte import Solver
    wl, _ = _problem(steps=7)
    wl.scheme = "euler"
    rng = np.random.default_rng(8)
    djdr = rng.standard_normal((wl.steps, wl.det_index.size))
    ga_ref, gs_ref = pn.adjoint_gradient(wl.n, wl.N, wl.dx, wl.c, wl.dt, wl.mu_a, wl.mu_s, wl.g,
                                         wl.psi0, None, wl.W, wl.mu0, wl.mu1, wl.steps,
                                         wl.det_index, djdr, scheme="euler")
    s = Solver.from_workload(wl)
    s.forward_checkpointed(wl.steps, 2)
    ga, gs = s.adjoint(djdr)
    s.close()
    assert rel(ga, ga_ref) <= 1e-10 and rel(gs, gs_ref) <= 1e-10


def test_checkpoint_interval_does_not_change_gradient(torch_cuda):
    """Recomputation from checkpoints replays the same kernels on the same
    data: the gradient is bitwise independent of the checkpoint interval."""
    from paper_1801_06364_amd.rte import Solver
    wl, _ = _problem(steps=9)
    rng = np.random.default_rng(0)
    djdr = rng.standard_normal((wl.steps, wl.det_index.size))
    out = []
    for every in (1, 3, 9, 4):
        s = Solver.from_workload(wl)
        s.forward_checkpointed(wl.steps, every)
        out.append(s.adjoint(djdr))
        s.close()
    for ga, gs in out[1:]:
        assert np.array_equal(ga, out[0][0]) and np.array_equal(gs, out[0][1])


def test_adjoint_matches_gpu_finite_differences(torch_cuda):
    """Central differences of the GPU FP64 forward loss at interior voxels."""
    from paper_1801_06364_amd.rte import Solver
    wl, tgt = _problem(n=16, steps=6)
    rng = np.random.default_rng(4)
    target = rng.uniform(0, 1e-3, (wl.steps, wl.det_index.size))
    r = _readings(wl, wl.mu_a, wl.mu_s)
    s = Solver.from_workload(wl)
    s.forward_checkpointed(wl.steps, 2)
    ga, gs = s.adjoint(2.0 * (r - target))
    s.close()
    for (z, y, x) in [(5, 6, 7), (8, 8, 8), (10, 4, 9)]:
        for grad, which in ((ga, "a"), (gs, "s")):
            ma, ms = wl.mu_a.copy(), wl.mu_s.copy()
            base = ma if which == "a" else ms
            # step large enough that dJ stands well above FP64 rounding of J,
            # small enough that the O(h^2) truncation stays below 1e-6
            h = 1e-3 * base[z, y, x]
            base[z, y, x] += h
            Jp = float(((_readings(wl, ma, ms) - target) ** 2).sum())
            base[z, y, x] -= 2 * h
            Jm = float(((_readings(wl, ma, ms) - target) ** 2).sum())
            fd = (Jp - Jm) / (2 * h)
            assert abs(fd - grad[z, y, x]) <= 1e-5 * abs(fd) + 1e-15, (which, fd, grad[z, y, x])


def test_autograd_function(torch_cuda):
    """torch.autograd through RteSolve gives the adjoint gradient."""
    torch = torch_cuda
    from paper_1801_06364_amd.autograd import rte_solve
    wl, _ = _problem(n=16, steps=5)
    prob = dict(n=wl.n, N=wl.N, dx=wl.dx, c=wl.c, dt=wl.dt, g=wl.g, psi0=wl.psi0, q=None, W=wl.W,
                mu0=wl.mu0, mu1=wl.mu1, precision="f64", det_index=wl.det_index, steps=wl.steps)
    mua = torch.tensor(wl.mu_a, dtype=torch.float64, device="cuda", requires_grad=True)
    mus = torch.tensor(wl.mu_s, dtype=torch.float64, device="cuda", requires_grad=True)
    r = rte_solve(mua, mus, prob)
    loss = (r ** 2).sum()
    loss.backward()
    rr = r.detach().cpu().numpy()
    ga_ref, gs_ref = pn.adjoint_gradient(wl.n, wl.N, wl.dx, wl.c, wl.dt, wl.mu_a, wl.mu_s, wl.g,
                                         wl.psi0, None, wl.W, wl.mu0, wl.mu1, wl.steps,
                                         wl.det_index, 2.0 * rr)
    assert rel(mua.grad.cpu().numpy(), ga_ref) <= 1e-10
    assert rel(mus.grad.cpu().numpy(), gs_ref) <= 1e-10


def test_full_size_adjoint_vs_finite_differences(torch_cuda):
    """The 96^3 / P_3 inclusion phantom (FP32 forward and adjoint, sqrt(T)
    checkpoints) against FP64 central differences at sampled voxels, on a
    shortened horizon; FP32 gradient against the FP64 GPU gradient."""
    from paper_1801_06364_amd.rte import Solver
    steps = 60
    wl, tgt = _problem(n=96, steps=steps, prec="f32")
    print("\n[adjoint] 96^3 P3 60 steps", flush=True)
    wl64 = ri.workload("p3_adjoint", n=96, steps=steps, precision="f64")
    target = _readings(ri.Workload("t", 96, 3, "f64", wl.dx, wl.c, wl.dt, wl.W, wl.mu0, wl.mu1, steps,
                                   tgt[0], tgt[1], tgt[2], wl.psi0, None, wl.det_index), tgt[0], tgt[1])
    r64 = _readings(wl64, wl.mu_a, wl.mu_s)
    djdr = 2.0 * (r64 - target)
    grads = {}
    for w in (wl, wl64):
        s = Solver.from_workload(w)
        s.forward_checkpointed(steps, 0)
        grads[w.precision] = s.adjoint(djdr)
        s.close()
    # FP32 against FP64 gradient: the reading A14 proposes (1e-4 relative L2)
    e32 = rel(grads["f32"][0], grads["f64"][0])
    print(f"[adjoint] FP32 vs FP64 gradient rel-L2 {e32:.2e}", flush=True)
    assert e32 <= 1e-4
    assert rel(grads["f32"][1], grads["f64"][1]) <= 1e-4
    rng = np.random.default_rng(5)
    omega = np.argwhere(pn.pml_depth(96, wl.W) == 0)
    ga = grads["f64"][0]
    # voxels where the gradient is not negligible (near the detectors' reach)
    cand = omega[rng.choice(len(omega), 4000, replace=False)]
    mags = np.array([abs(ga[tuple(v)]) for v in cand])
    pick = cand[np.argsort(mags)[-5:]]
    for v in pick:
        z, y, x = v
        ma = wl.mu_a.copy()
        h = 1e-4 * ma[z, y, x]
        ma[z, y, x] += h
        Jp = float(((_readings(wl64, ma, wl.mu_s) - target) ** 2).sum())
        ma[z, y, x] -= 2 * h
        Jm = float(((_readings(wl64, ma, wl.mu_s) - target) ** 2).sum())
        fd = (Jp - Jm) / (2 * h)
        assert abs(fd - ga[z, y, x]) <= 1e-4 * abs(fd), (v, fd, ga[z, y, x])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_device_medium_and_state_reproduce_host_creation(torch_cuda, prec):
    """A handle created with other maps, then given mu_a, mu_s and the
    initial state from device memory (loss maps rebuilt on the device),
    steps bitwise like a handle created from those maps on the host: state
    and readings (read back device to device)."""
    torch = torch_cuda
    from paper_1801_06364_amd.rte import Solver
    wl, tgt = _problem(n=16, steps=6, prec=prec)
    a = Solver.from_workload(wl)
    a.step(wl.steps)
    ref_state, ref_read = a.get_state(), a.readings()
    a.close()
    b = Solver.from_workload(wl, mu_a=tgt[0], mu_s=tgt[1])   # created with other maps
    b.set_medium_device(torch.tensor(wl.mu_a.ravel(), dtype=torch.float64, device="cuda"),
                        torch.tensor(wl.mu_s.ravel(), dtype=torch.float64, device="cuda"))
    b.step(3)                                                  # state and record are replaced next
    b.set_state_device(torch.tensor(wl.psi0.ravel(), dtype=torch.float64, device="cuda"))
    assert b.steps_done() == 0
    b.step(wl.steps)
    st, rd = b.get_state(), b.readings_device().cpu().numpy()
    b.close()
    assert np.array_equal(st, ref_state)
    assert np.array_equal(rd, ref_read)


def test_autograd_device_path_repeated_solves(torch_cuda):
    """Two solves with different maps through one device-resident problem:
    each gradient equals the host-path adjoint of its own maps (FP64,
    <= 1e-12) and the oracle's reverse mode (<= 1e-10)."""
    torch = torch_cuda
    from paper_1801_06364_amd.autograd import RteProblem, rte_solve
    from paper_1801_06364_amd.rte import Solver
    wl, tgt = _problem(n=16, steps=5)
    prob = RteProblem(wl.n, wl.N, wl.dx, wl.c, wl.dt, wl.g, psi0=wl.psi0, W=wl.W, mu0=wl.mu0, mu1=wl.mu1,
                      precision="f64", det_index=wl.det_index, steps=wl.steps, every=2)
    for ma, ms in ((wl.mu_a, wl.mu_s), (tgt[0], tgt[1])):
        mua = torch.tensor(ma, dtype=torch.float64, device="cuda", requires_grad=True)
        mus = torch.tensor(ms, dtype=torch.float64, device="cuda", requires_grad=True)
        r = rte_solve(mua, mus, prob)
        assert r.is_cuda
        (r ** 2).sum().backward()
        rr = r.detach().cpu().numpy()
        h = Solver.from_workload(wl, mu_a=ma, mu_s=ms)
        h.forward_checkpointed(wl.steps, 2)
        assert np.array_equal(h.readings(), rr)
        ga_h, gs_h = h.adjoint(2.0 * rr)
        h.close()
        assert mua.grad.is_cuda and mus.grad.is_cuda
        assert rel(mua.grad.cpu().numpy(), ga_h) <= 1e-12
        assert rel(mus.grad.cpu().numpy(), gs_h) <= 1e-12
        ga_ref, gs_ref = pn.adjoint_gradient(wl.n, wl.N, wl.dx, wl.c, wl.dt, ma, ms, wl.g, wl.psi0, None, wl.W,
                                             wl.mu0, wl.mu1, wl.steps, wl.det_index, 2.0 * rr)
        assert rel(mua.grad.cpu().numpy(), ga_ref) <= 1e-10
        assert rel(mus.grad.cpu().numpy(), gs_ref) <= 1e-10
    prob.close()
