"""Host-side pieces of the request loop: the request trace and the hop."""
import numpy as np

from paper_2403_09158_amd import inputs, serve


def _replicas():
    rng = np.random.default_rng(5)
    out = []
    for n in (32, 48):
        L = n * inputs.H_VOXEL
        out.append((inputs.Problem(n, L, *inputs.CUBIC_FE), inputs.mixed_population(rng, 20, L, inputs.H_VOXEL)))
    return out


def test_trace_shape():
    reps = _replicas()
    reqs = serve.serving_requests(reps, 2000, rate_per_s=2000.0)
    t = np.array([r.t for r in reqs])
    assert np.all(np.diff(t) > 0)
    # Poisson arrivals at 2000/s: the mean gap is 0.5 ms within sampling error
    assert abs(np.mean(np.diff(t)) - 5e-4) < 5e-5
    upd = [r for r in reqs if r.op == "update"]
    assert 0.87 < len(upd) / len(reqs) < 0.93
    hops = {tuple(h) for h in inputs.HOPS111.tolist()}
    for r in upd:
        assert tuple(r.hop) in hops
        assert 0 <= r.idx < len(reps[r.replica][1])
    assert {r.op for r in reqs} == {"update", "solve"}
    assert {r.replica for r in reqs} == {0, 1}


def test_trace_is_reproducible():
    reps = _replicas()
    a = serve.serving_requests(reps, 100)
    b = serve.serving_requests(reps, 100)
    assert a == b


def test_moved_defect_is_a_whole_voxel_hop():
    reps = _replicas()
    prob, defs = reps[0]
    req = serve.Request(0, 0, 0.0, "update", idx=3, hop=(1, -1, 1))
    d = serve.moved_defect(defs, req, prob.h)
    assert np.allclose(d["c"] - defs[3]["c"], np.array([1, -1, 1]) * prob.h, rtol=0, atol=1e-12)
    for f in ("kind", "radius", "b", "normal", "thickness", "eig_v"):
        assert np.array_equal(d[f], defs[3][f])
    assert not np.shares_memory(d, defs)


def test_latency_split_by_grid():
    # four requests on two grid sizes; service = latency - wait per request
    lat = np.array([1.0, 3.0, 2.0, 6.0])
    wait = np.array([0.0, 1.0, 0.5, 4.0])
    st = serve.ServeStats(completed=4, wall_s=1.0, throughput=4.0, p50_ms=2.5, p99_ms=6.0, mean_ms=3.0, admissions=0,
                          evictions=0, latency_ms=lat, results={}, wait_ms=wait, grid=np.array([64, 240, 64, 240]))
    g = st.by_grid()
    assert sorted(g) == [64, 240]
    assert g[64]["requests"] == 2 and g[240]["requests"] == 2
    assert g[64]["p50_ms"] == 1.5 and g[240]["p50_ms"] == 4.5
    assert g[64]["service_p50_ms"] == 1.25 and g[240]["service_p50_ms"] == 2.0
    assert abs(g[240]["wait_p99_ms"] - (1.0 + 0.99 * 3.0)) < 1e-9
    assert abs(g[240]["p99_ms"] - (3.0 + 0.99 * 3.0)) < 1e-9
