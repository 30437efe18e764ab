"""Serving loop: each request's result is the same alone and in the mix.

Several simulations of different size and shear rate are admitted together
(own workspace, own stream) and advanced in interleaved chunks; the final
state and the whole sampled stress series of every request must equal, bit
for bit, those of the same request served alone.
"""
import numpy as np
import pytest

from paper_2109_11083_amd.serve import Server, sweep_trace

pytestmark = pytest.mark.gpu


def _trace(precision="fp64"):
    return sweep_trace(count=5, n_lo=1000, n_hi=6000, steps=300, seed=7, burst=True,
                       precision=precision)


@pytest.mark.parametrize("precision,graphs", [("fp64", True), ("mixed", True), ("fp64", False)])
def test_results_same_alone_and_in_the_mix(precision, graphs):
    trace = _trace(precision)
    mixed, summ = Server(max_active=5, chunk=100, keep_state=True, graphs=graphs).run(trace, realtime=False)
    print(f"mix: {summ}", flush=True)
    assert summ["requests"] == len(trace)
    for req in trace:
        alone, _ = Server(max_active=1, chunk=300, keep_state=True, graphs=False).run([req], realtime=False)
        a, m = alone[0], mixed[req.rid]
        assert a.rid == m.rid == req.rid
        assert np.array_equal(a.stress, m.stress), req.rid
        assert np.array_equal(a.state_x, m.state_x) and np.array_equal(a.state_u, m.state_u), req.rid
        assert np.isfinite(m.eta)


def test_admission_respects_the_hbm_budget():
    trace = _trace()
    from paper_2109_11083_amd.serve import footprint, request_params
    sizes = [footprint(request_params(r)[1], r) for r in trace]
    budget = max(sizes) + 1  # room for one request at a time (the largest)
    res, summ = Server(hbm_budget=budget, max_active=5, chunk=100).run(trace, realtime=False)
    # with room for one, no two requests overlap in time
    spans = sorted((r.admitted, r.done) for r in res)
    for (a0, d0), (a1, d1) in zip(spans, spans[1:]):
        assert a1 >= d0
    assert summ["requests"] == len(trace)
