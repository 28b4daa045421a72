"""OkMC time steps on the GPU (ec_okmc_step): steps against the oracle's steps
(the same random numbers), the step against the separate probe and selection
calls and against moving the chosen defects one by one, the Poisson gate at its
boundary, and the argument checks.

Tolerances: FP64 states to 1e-10 of the largest energy (normwise energy
tolerance); FP32 states to max(1e-4 |E_i|, 1e-5 eV) per defect.  The choices
are integers decided in FP64 on both sides and compared exactly."""
import numpy as np
import pytest

from oracle import energy as oenergy
from oracle import okmc as ookmc
from paper_2403_09158_amd import inputs

pytestmark = pytest.mark.gpu

KT, NU0 = 0.025852, 1.0e13


@pytest.fixture(scope="module")
def ctx():
    from paper_2403_09158_amd import ec

    return ec.Context()


def _population(seed, n, ndef, prec):
    rng = np.random.default_rng(inputs.SEED_BASE + seed)
    L = n * inputs.H_VOXEL
    prob = inputs.Problem(n, L, *inputs.CUBIC_FE, prec=prec)
    d = inputs.mixed_population(rng, ndef, L, inputs.H_VOXEL, r111=(0.4, 1.0), r100=(0.5, 1.0))
    J = np.concatenate([inputs.glide_jumps(d), np.tile(np.array([[[0, 1, 0]], [[0, 0, -1]]]).reshape(1, 2, 3), (ndef, 1, 1))], axis=1)
    Em = 0.1 + rng.uniform(0.0, 0.1, size=ndef)
    return rng, prob, d, J.astype(np.int32), Em


@pytest.mark.parametrize("n,ndef,steps", [(32, 8, 3), (48, 20, 2)])
def test_okmc_steps_match_oracle(ctx, n, ndef, steps):
    from paper_2403_09158_amd import ec

    rng, prob, d, J, Em = _population(810 + n, n, ndef, 0)
    st = ec.State(ctx, prob)
    st.solve(d)
    cur = d
    moved_any = False
    for step in range(steps):
        u = 1.0 - rng.uniform(size=ndef)
        xi = 1.0 - rng.uniform(size=ndef)
        choice, E = st.okmc_step(J, Em, NU0, KT, u, xi, energies=True)
        N, want_choice, cur, want_E = ookmc.okmc_step(prob, cur, J, Em, NU0, KT, 0.0, u, xi)
        assert np.array_equal(choice, want_choice), (step, choice, want_choice)
        assert np.abs(E - want_E).max() <= 1e-10 * np.abs(want_E).max(), step
        moved_any |= bool((choice >= 0).any())
    assert moved_any
    st.close()


def test_okmc_step_fp32_against_oracle(ctx):
    from paper_2403_09158_amd import ec

    rng, prob, d, J, Em = _population(830, 48, 20, 1)
    st = ec.State(ctx, prob)
    st.solve(d)
    u = 1.0 - rng.uniform(size=len(d))
    xi = 1.0 - rng.uniform(size=len(d))
    # the same state probed and selected by the separate calls
    st.jump_energies(J)
    _, sel = st.jump_select(Em, NU0, KT, xi)
    choice, E = st.okmc_step(J, Em, NU0, KT, u, xi, energies=True)
    dt = ookmc.time_step(Em, KT, NU0)
    N = ookmc.event_counts(ookmc.nominal_frequencies(Em, KT, NU0), dt, u)
    assert np.array_equal(choice, np.where(N > 0, sel, -1))
    from oracle import energy

    want = energy.energies_fast(prob, ookmc.move(prob, d, J, choice))
    assert np.all(np.abs(E - want) <= np.maximum(1e-4 * np.abs(want), 1e-5))
    st.close()


def test_okmc_step_equals_moving_the_chosen_defects(ctx):
    """The step's re-solve of the moved list against the chosen jumps made one
    by one with the incremental update on a second state."""
    from paper_2403_09158_amd import ec

    rng, prob, d, J, Em = _population(840, 48, 20, 0)
    a = ec.State(ctx, prob)
    b = ec.State(ctx, prob)
    a.solve(d)
    b.solve(d)
    u = 1.0 - rng.uniform(size=len(d))
    xi = 1.0 - rng.uniform(size=len(d))
    choice, Ea = a.okmc_step(J, Em, NU0, KT, u, xi, dt=1.0e-11, energies=True)
    assert (choice >= 0).sum() >= 3 and (choice < 0).sum() >= 1
    Eb = None
    for i in np.nonzero(choice >= 0)[0]:
        rec = d[i].copy()
        rec["c"] = rec["c"] + J[i, choice[i]].astype(np.float64) * prob.h
        Eb = b.update(int(i), rec)
    assert np.abs(Ea - Eb).max() <= 1e-10 * np.abs(Eb).max()
    a.close()
    b.close()


def test_poisson_gate_boundary_of_the_fixed_step(ctx):
    """Equal barriers and dt <= 0: every defect's P(N = 0) is 1/e exactly, so
    u just below it means no event and just above it one."""
    from paper_2403_09158_amd import ec

    rng, prob, d, J, _ = _population(850, 32, 8, 0)
    Em = np.full(len(d), 0.15)
    st = ec.State(ctx, prob)
    st.solve(d)
    p0 = np.exp(-1.0)
    u = np.where(np.arange(len(d)) % 2 == 0, p0 * (1 - 1e-9), p0 * (1 + 1e-9))
    choice = st.okmc_step(J, Em, NU0, KT, u, np.full(len(d), 0.5))
    assert np.all(choice[0::2] == -1) and np.all(choice[1::2] >= 0)
    st.close()


def test_okmc_step_argument_checks(ctx):
    from paper_2403_09158_amd import ec

    rng, prob, d, J, Em = _population(860, 32, 8, 0)
    st = ec.State(ctx, prob)
    with pytest.raises(ec.EcError) as ei:
        st.okmc_step(J[:0], Em[:0], NU0, KT, np.zeros(0), np.zeros(0))
    assert ei.value.status == ec.EC_ERR_STATE
    st.solve(d)
    E0 = st.energies().copy()
    good = np.full(8, 0.5)
    bad_u = good.copy()
    bad_u[3] = 0.0
    bad_Em = Em.copy()
    bad_Em[2] = np.inf
    bad_J = J.copy()
    bad_J[5, 1, 0] = 12
    for args, kw in (
        ((J, Em, NU0, KT, bad_u, good), {}),
        ((J, Em, NU0, KT, good, good + 0.6), {}),
        ((J, bad_Em, NU0, KT, good, good), {}),
        ((bad_J, Em, NU0, KT, good, good), {}),
        ((J, Em, NU0, 0.0, good, good), {}),
        ((J, Em, NU0, KT, good, good), {"dt": np.nan}),
    ):
        with pytest.raises(ec.EcError) as ei:
            st.okmc_step(*args, **kw)
        assert ei.value.status == ec.EC_ERR_ARG
    # nothing moved
    assert np.array_equal(st.energies(), E0)
    st.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_probe_after_step_reuses_cross_parts(ctx, prec):
    """The cross parts of the probe are kept across a step (footprints only
    translate): a repeated probe is bitwise the same, and the probe after a
    step matches a cold probe of a fresh state solved from the moved records."""
    from paper_2403_09158_amd import ec

    rng, prob, d, J, Em = _population(870, 48, 20, prec)
    a = ec.State(ctx, prob)
    a.solve(d)
    d1 = a.jump_energies(J).copy()
    assert np.array_equal(a.jump_energies(J), d1)
    u = 1.0 - rng.uniform(size=len(d))
    xi = 1.0 - rng.uniform(size=len(d))
    choice = a.okmc_step(J, Em, NU0, KT, u, xi)
    assert (choice >= 0).any()
    warm = a.jump_energies(J)
    b = ec.State(ctx, prob)
    b.solve(ookmc.move(prob, d, J, choice))
    cold = b.jump_energies(J)
    tol = 1e-10 if prec == 0 else 1e-6
    assert np.abs(warm - cold).max() <= tol * np.abs(cold).max()
    a.close()
    b.close()


def test_okmc_step_on_an_empty_list(ctx):
    from paper_2403_09158_amd import ec

    prob = inputs.Problem(32, 32 * inputs.H_VOXEL, *inputs.CUBIC_FE)
    st = ec.State(ctx, prob)
    st.solve(inputs.empty_defects(0))
    z = np.zeros(0)
    choice = st.okmc_step(np.zeros((0, 2, 3), dtype=np.int32), z, NU0, KT, z, z)
    assert choice.shape == (0,)
    st.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_okmc_step_with_one_acting_defect(ctx, prec):
    """A short step in which one defect acts (moved with the incremental
    update) against the oracle's step and a fresh solve."""
    from paper_2403_09158_amd import ec

    rng, prob, d, J, Em = _population(892, 48, 20, prec)
    u = 1.0 - rng.uniform(size=len(d))
    xi = 1.0 - rng.uniform(size=len(d))
    st = ec.State(ctx, prob)
    st.solve(d)
    choice, E = st.okmc_step(J, Em, NU0, KT, u, xi, dt=1.0e-12, energies=True)
    N, want_choice, moved, want_E = ookmc.okmc_step(prob.with_(prec=0), d, J, Em, NU0, KT, 1.0e-12, u, xi)
    assert (choice >= 0).sum() == 1
    if prec == 0:
        assert np.array_equal(choice, want_choice)
        assert np.abs(E - want_E).max() <= 1e-10 * np.abs(want_E).max()
    else:
        assert np.array_equal(choice >= 0, N > 0)
        want_E = oenergy.energies_fast(prob, ookmc.move(prob, d, J, choice))
        assert np.all(np.abs(E - want_E) <= np.maximum(1e-4 * np.abs(want_E), 1e-5))
    fresh = ec.State(ctx, prob)
    fresh.solve(ookmc.move(prob, d, J, choice))
    tol = 1e-10 if prec == 0 else 1e-6
    assert np.abs(E - fresh.energies()).max() <= tol * np.abs(E).max()
    # the probe after the step still reuses its cross parts (hops keep them)
    assert np.allclose(st.jump_energies(J), fresh.jump_energies(J), rtol=0, atol=tol * np.abs(E).max())
    st.close()
    fresh.close()
