"""Strong guarantee under allocation failure (include/ec.h, error behaviour):
a call whose device allocation fails returns an error and leaves the state as
it was.  Allocations go through Python hooks that fail the j-th request;
every allocation point of each single-call operation is tried in turn, each
time on a fresh context and state.  A call that still succeeds (the failed
allocation served a cache the library rebuilds later) must give the same
results as an undisturbed run, and a failed one must succeed when repeated."""
import numpy as np
import pytest

from paper_2403_09158_amd import inputs

pytestmark = pytest.mark.gpu


class Hooks:
    """Torch-backed allocation hooks that fail request number fail_at."""

    def __init__(self):
        import torch

        self._alloc, self._delete = torch.cuda.caching_allocator_alloc, torch.cuda.caching_allocator_delete
        self.count = 0
        self.fail_at = None

    def alloc(self, nbytes):
        self.count += 1
        if self.fail_at is not None and self.count == self.fail_at:
            return None
        return self._alloc(nbytes)

    def free(self, ptr):
        self._delete(ptr)


def _case(n=32, seed=3):
    rng = np.random.default_rng(seed)
    L = n * inputs.H_VOXEL
    prob = inputs.Problem(n, L, *inputs.CUBIC_FE)
    small = inputs.mixed_population(rng, 6, L, L / n, r111=(0.4, 0.8), r100=(0.5, 0.8))
    big = inputs.mixed_population(rng, 40, L, L / n, r111=(0.4, 1.6), r100=(0.5, 1.6))
    return prob, small, big


def _grow(d, i):
    m = d[i].copy()
    m["c"] = m["c"] + 0.37
    m["radius"] = 1.8 * m["radius"]
    return m


PROB, SMALL, BIG = _case()

# (set-up on the state solved with SMALL, the one library call whose
# allocations fail, what the result is read from afterwards)
OPS = {
    "solve_larger_list": (None, lambda st: st.solve(BIG), lambda st, out: st.energies()),
    "update_growing_footprint": (
        None,
        lambda st: st.update(2, _grow(SMALL, 2), energies=False),
        lambda st, out: st.energies(),
    ),
    "energies_after_new_shape": (
        lambda st: st.update(1, _grow(SMALL, 1), energies=False),
        lambda st: st.energies(),
        lambda st, out: out,
    ),
    "jump_energies": (None, lambda st: st.jump_energies(inputs.glide_jumps(SMALL)), lambda st, out: out),
    "type_store": (None, lambda st: st.type_store(BIG[:1]), lambda st, out: st.type_energies(out, BIG["c"][:3])),
}


def _fresh(h, setup):
    from paper_2403_09158_amd import ec

    ctx = ec.Context(0, hooks=(h.alloc, h.free))
    st = ec.State(ctx, PROB)
    st.solve(SMALL)
    st.energies()
    if setup:
        setup(st)
    return ctx, st


@pytest.mark.parametrize("op", sorted(OPS))
def test_failed_allocation_leaves_state_unchanged(op):
    from paper_2403_09158_amd import ec

    setup, call, result = OPS[op]
    # undisturbed runs: the call's allocations and result, and the energies
    # of the state before the call
    h = Hooks()
    ctx, st = _fresh(h, setup)
    before = h.count
    out = call(st)
    n_alloc = h.count - before
    ref = np.array(result(st, out), copy=True)
    st.close()
    ctx.close()
    h = Hooks()
    ctx, st = _fresh(h, setup)
    E_pre = st.energies().copy()
    st.close()
    ctx.close()
    assert n_alloc > 0, "the call allocates nothing: nothing to inject"
    failed = 0
    for j in range(1, n_alloc + 1):
        h = Hooks()
        ctx, st = _fresh(h, setup)
        s0, f0 = st.field("sigma").copy(), [f.copy() for f in st.footprints()]
        h.fail_at = h.count + j
        try:
            out = call(st)
        except ec.EcError as e:
            assert e.status in (ec.EC_ERR_DEVICE, ec.EC_ERR_ADMIT), (j, e)
            failed += 1
            h.fail_at = None
            assert np.array_equal(st.field("sigma"), s0), (op, j)
            f1 = st.footprints()
            assert len(f1) == len(f0) and all(np.array_equal(a, b) for a, b in zip(f1, f0)), (op, j)
            assert np.array_equal(st.energies(), E_pre), (op, j)
            out = call(st)  # the state still works
        h.fail_at = None
        assert np.array_equal(np.asarray(result(st, out)), ref), (op, j)
        st.close()
        ctx.close()
    assert failed > 0
