"""Serving: continuous batching of heterogeneous solves on one GPU."""
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


def _trace(count=10, seed=11):
    return ri.serving_requests(count=count, seed=seed, sizes=(32, 48, 64), orders=(1, 3, 5),
                               steps=(20, 60))


class _Unstable:
    """A request whose time step is far beyond the stability limit."""

    def __init__(self, spec):
        self.__dict__.update(spec.__dict__)
        self._spec = spec

    def workload(self, precision="f32"):
        wl = self._spec.workload(precision)
        wl.dt *= 40.0
        return wl


def test_results_identical_alone_and_in_the_mix(torch_cuda):
    """Every request's fluence is bitwise the same when it runs alone and
    when it shares the GPU with others (all arriving at once)."""
    from paper_1801_06364_amd import serving
    specs = _trace()
    srv = serving.Server(budget_bytes=8 << 30, max_slots=6, keep_fluence=True)
    alone = srv.service_times(specs)
    rep = srv.serve(specs, [0.0] * len(specs))
    assert rep.peak_slots > 1
    for s in specs:
        a, b = alone[s.rid], rep.results[s.rid]
        assert a.ok and b.ok
        assert np.array_equal(a.fluence, b.fluence), s.rid


def test_admission_respects_memory_budget(torch_cuda):
    """With a budget that holds only one request at a time every request
    still completes, in arrival order, never above the budget."""
    from paper_1801_06364_amd import serving
    specs = _trace(count=5, seed=3)
    budget = max(serving.footprint(s) for s in specs)
    srv = serving.Server(budget_bytes=budget, max_slots=4)
    arr = [0.001 * i for i in range(len(specs))]
    rep = srv.serve(specs, arr)
    assert rep.peak_resident_bytes <= budget
    assert all(r.ok for r in rep.results.values())
    starts = [rep.results[s.rid].admitted for s in specs]
    assert starts == sorted(starts)


def test_poisoned_request_fails_alone(torch_cuda):
    """An unstable request is reported as failed; the others complete with
    the same results as alone."""
    from paper_1801_06364_amd import serving
    specs = _trace(count=6, seed=5)
    bad = _Unstable(specs[2])
    mix = specs[:2] + [bad] + specs[3:]
    srv = serving.Server(budget_bytes=8 << 30, max_slots=6, keep_fluence=True)
    alone = srv.service_times(specs)
    rep = srv.serve(mix, [0.0] * len(mix))
    assert not rep.results[bad.rid].ok
    for s in specs:
        if s.rid == bad.rid:
            continue
        assert rep.results[s.rid].ok
        assert np.array_equal(rep.results[s.rid].fluence, alone[s.rid].fluence)
