"""Host-side serving logic (no GPU): trace generation and FIFO replay."""
import pytest

import rte_inputs as ri


def _trace(count=10, seed=11):
    return ri.serving_requests(count=count, seed=seed, sizes=(32, 48, 64), orders=(1, 3, 5),
                               steps=(20, 60))


def test_trace_is_seeded_and_in_range():
    a, b = _trace(50, 4), _trace(50, 4)
    assert [(x.n, x.N, x.steps, x.nspheres, x.gap) for x in a] == \
        [(x.n, x.N, x.steps, x.nspheres, x.gap) for x in b]
    assert all(x.n in (32, 48, 64) and x.N in (1, 3, 5) and 20 <= x.steps <= 60 for x in a)
    full = ri.serving_requests()
    assert len(full) == 256 and {x.n for x in full} == {32, 48, 64, 96, 128}


def test_fifo_replay_queue_arithmetic():
    """The one-at-a-time replay is a first-come first-served queue."""
    from paper_1801_06364_amd import serving
    specs = _trace(count=3)
    alone = {s.rid: serving.Result(s.rid, 0.0, admitted=0.0, finished=t, ok=True)
             for s, t in zip(specs, (1.0, 2.0, 0.5))}
    rep = serving.fifo_replay(specs, [0.0, 0.5, 5.0], alone)
    lat = [rep.results[s.rid].latency for s in specs]
    assert lat == pytest.approx([1.0, 2.5, 0.5])
