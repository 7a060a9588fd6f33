"""Host logic of the serving loop (no GPU): seeded Poisson arrivals and the latency/throughput
summary."""
import numpy as np

from paper_2601_17164_amd import serve


def test_poisson_arrivals_are_seeded_increasing_and_at_rate():
    a = serve.poisson_arrivals(20.0, 20000, seed=7)
    b = serve.poisson_arrivals(20.0, 20000, seed=7)
    np.testing.assert_array_equal(a, b)
    assert np.all(np.diff(a) > 0) and a[0] > 0
    gaps = np.diff(np.concatenate([[0.0], a]))
    assert abs(gaps.mean() * 20.0 - 1.0) < 0.03          # mean gap 1/rate
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05    # exponential: coefficient of variation 1
    assert not np.array_equal(a, serve.poisson_arrivals(20.0, 20000, seed=8))


def test_summary_percentiles_and_throughput():
    res = [serve.Result(k, arrival=0.1 * k, admitted=0.1 * k, finished=0.1 * k + 0.001 * (k + 1),
                        n_traj=64, steps=1000 * (k + 1)) for k in range(100)]
    s = serve.summarize(res)
    lat = np.arange(1, 101, dtype=float)  # ms
    assert s["requests"] == 100
    assert abs(s["p50_ms"] - np.percentile(lat, 50)) < 1e-9
    assert abs(s["p99_ms"] - np.percentile(lat, 99)) < 1e-9
    assert abs(s["mean_ms"] - lat.mean()) < 1e-9
    span = res[-1].finished - res[0].arrival
    assert abs(s["span_s"] - span) < 1e-12
    assert abs(s["trajectory_steps_per_s"] - sum(r.steps for r in res) / span) < 1e-6
    s2 = serve.summarize(res, wall=20.0)
    assert s2["span_s"] == 20.0
