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
