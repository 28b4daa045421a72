"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: rasterisation bit-exact; fields relative L2 1e-12 (FP64) and 1e-5
(FP32 storage); energies normwise relative 1e-10 (FP64) and per defect
max(1e-4 |E|, 1e-5 eV) (FP32 storage).
"""
import numpy as np
import pytest

from helpers import energy_ok_fp32, energy_ok_fp64, rel_l2, rel_max, to6
from oracle import elastic, energy, raster, solve
from paper_2403_09158_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2403_09158_amd import ec

    return ec.Context()


def _state(ctx, prob):
    from paper_2403_09158_amd import ec

    return ec.State(ctx, prob)


def _mixed(n, ndef, seed, prec=0, bc=0):
    rng = np.random.default_rng(1000 + seed)
    L = n * inputs.H_VOXEL
    prob = inputs.Problem(n, L, *inputs.CUBIC_FE, prec=prec, bc=bc)
    rmax = min(1.6, 0.3 * L)
    d = inputs.mixed_population(rng, ndef, L, L / n, r111=(0.4, rmax), r100=(0.5, rmax))
    return prob, d


def _oracle_fields(prob, defs):
    fps, Es = raster.rasterise(prob, defs)
    es = raster.eigenstrain_field(prob.n, fps, Es)
    eps, sig, _ = solve.solve_field(elastic.stiffness_of(prob), prob.L, es, prob.bc)
    return fps, Es, to6(es), to6(eps), to6(sig)


# ------------------------------------------------------------------ rasteriser


@pytest.mark.parametrize("case", ["pair_32", "mixed24", "mixed32_wrap", "mixed48"])
def test_raster_bit_exact(ctx, case):
    if case == "pair_32":
        prob, d = inputs.pair_32()
    elif case == "mixed24":
        prob, d = _mixed(24, 12, 1)
    elif case == "mixed32_wrap":
        prob, d = _mixed(32, 30, 2)
        d["c"][:4] = 0.01  # centred near a corner: footprints wrap on all axes
    else:
        prob, d = _mixed(48, 60, 3)
    st = _state(ctx, prob)
    st.solve(d)
    got = st.footprints()
    want, Es = raster.rasterise(prob, d)
    assert len(got) == len(want)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    es = st.field("eps_star")
    ref = to6(raster.eigenstrain_field(prob.n, want, Es))
    assert np.max(np.abs(es - ref)) <= 2e-16 * max(1.0, np.max(np.abs(ref)))


def test_invalid_defect_rejected_state_unchanged(ctx):
    from paper_2403_09158_amd import ec

    prob, d = inputs.pair_32()
    st = _state(ctx, prob)
    st.solve(d)
    E0 = st.energies()
    bad = d.copy()
    bad[1]["radius"] = prob.L  # extent beyond half the cell
    with pytest.raises(ec.EcError) as ei:
        st.solve(bad)
    assert ei.value.status == ec.EC_ERR_ARG
    assert np.array_equal(st.energies(), E0)


def test_first_invalid_defect_of_a_long_list_is_reported(ctx):
    """Long lists are validated in parallel chunks; the error names the first
    invalid defect in list order and the state keeps its previous solve."""
    from paper_2403_09158_amd import ec

    prob, d = _mixed(48, 600, 11)
    st = _state(ctx, prob)
    st.solve(d)
    E0 = st.energies().copy()
    bad = d.copy()
    bad[517]["radius"] = -1.0
    bad[300]["radius"] = prob.L
    with pytest.raises(ec.EcError) as ei:
        st.solve(bad)
    assert ei.value.status == ec.EC_ERR_ARG
    assert "defect 300" in str(ei.value)
    assert np.array_equal(st.energies(), E0)
    st.close()


# --------------------------------------------------------------- single passes


@pytest.mark.parametrize("n", [8, 16, 24, 32, 48, 64, 96, 128, 160, 240, 256])
@pytest.mark.parametrize("prec", [0, 1])
def test_forward_transform(ctx, n, prec):
    rng = np.random.default_rng(n)
    prob = inputs.Problem(n, n * 0.3125, *inputs.CUBIC_FE, prec=prec)
    f = rng.normal(size=(6, n, n, n)) * 0.01
    st = _state(ctx, prob)
    got = st.debug_forward(f)
    want = solve.fft3(f)[..., : n // 2 + 1]
    tol = 1e-13 if prec == 0 else 2e-7
    assert rel_l2(got, want) < tol
    assert rel_max(got, want) < 10 * tol


@pytest.mark.parametrize("n", [8, 24, 48, 96, 160, 240, 256])
@pytest.mark.parametrize("prec", [0, 1])
def test_inverse_transform(ctx, n, prec):
    rng = np.random.default_rng(100 + n)
    prob = inputs.Problem(n, n * 0.3125, *inputs.CUBIC_FE, prec=prec)
    f = rng.normal(size=(6, n, n, n))
    spec = solve.fft3(f)[..., : n // 2 + 1]  # Hermitian half spectrum of a real field
    st = _state(ctx, prob)
    got = st.debug_inverse(spec)
    tol = 1e-13 if prec == 0 else 2e-7
    assert rel_l2(got, f) < tol
    assert rel_max(got, f) < 10 * tol


@pytest.mark.parametrize("n", [8, 16, 32])
@pytest.mark.parametrize("bc", [0, 1])
def test_green_step(ctx, n, bc):
    """sigma_hat = S(xi):eps*_hat on the half spectrum, against the oracle solve."""
    prob, d = _mixed(n, 6, n + bc, bc=bc)
    _, _, es6, _, sig6 = _oracle_fields(prob, d)
    st = _state(ctx, prob)
    spec_in = solve.fft3(es6)[..., : n // 2 + 1]
    got = st.debug_green(spec_in)
    want = solve.fft3(sig6)[..., : n // 2 + 1]
    if bc == 1:  # the kernel leaves xi = 0 at zero; the mean is added in FP64 afterwards
        want[:, 0, 0, 0] = 0.0
    assert rel_l2(got, want) < 1e-12


# ------------------------------------------------------------------ full solve


@pytest.mark.parametrize("n", [8, 16, 24, 32, 48, 64, 96, 128, 160, 240])
@pytest.mark.parametrize("prec", [0, 1])
def test_solve_fields_every_size(ctx, n, prec):
    """The whole solve (fused z pass included) at every supported length."""
    prob, d = _mixed(n, max(4, n // 8), 7 * n + prec, prec=prec)
    _, _, _, _, sig6 = _oracle_fields(prob, d)
    st = _state(ctx, prob)
    st.solve(d)
    tol = 1e-12 if prec == 0 else 1e-5
    sig = st.field("sigma")
    assert rel_l2(sig, sig6) < tol
    assert rel_max(sig, sig6) < 10 * tol
    st.close()



@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("bc", [0, 1])
def test_pair32_fields_and_energies(ctx, prec, bc):
    prob, d = inputs.pair_32()
    prob = prob.with_(prec=prec, bc=bc)
    _, _, _, eps6, sig6 = _oracle_fields(prob, d)
    Eo, _ = energy.energies_brute(prob, d)
    st = _state(ctx, prob)
    st.solve(d)
    E = st.energies()
    sig = st.field("sigma")
    eps = st.field("eps")
    tol = 1e-12 if prec == 0 else 1e-5
    assert rel_l2(sig, sig6) < tol and rel_max(sig, sig6) < 10 * tol
    assert rel_l2(eps, eps6) < tol and rel_max(eps, eps6) < 10 * tol
    if prec == 0:
        assert energy_ok_fp64(E, Eo)
    else:
        assert np.all(energy_ok_fp32(E, Eo))
    # reciprocity of a pair: E_1 = E_12 = E_21 = E_2
    if prec == 0:
        assert abs(E[0] - E[1]) <= 1e-10 * abs(E[0])
    else:
        assert abs(E[0] - E[1]) <= max(2e-4 * abs(E[0]), 2e-5)


@pytest.mark.parametrize("n,ndef,seed", [(24, 10, 4), (32, 25, 5), (48, 40, 6)])
@pytest.mark.parametrize("prec", [0, 1])
def test_mixed_energies(ctx, n, ndef, seed, prec):
    prob, d = _mixed(n, ndef, seed, prec=prec)
    Eo, parts = energy.energies_fast(prob, d, return_parts=True)
    st = _state(ctx, prob)
    st.solve(d)
    E = st.energies()
    if prec == 0:
        assert energy_ok_fp64(E, Eo)
        B = st.self_terms()
        assert np.max(np.abs(B - parts["B"])) <= 1e-10 * np.max(np.abs(parts["B"]))
    else:
        ok = energy_ok_fp32(E, Eo)
        assert np.all(ok), (np.abs(E - Eo)[~ok], Eo[~ok])


def test_mixed_energies_against_brute_force(ctx):
    prob, d = _mixed(24, 8, 11)
    Eb, _ = energy.energies_brute(prob, d)
    st = _state(ctx, prob)
    st.solve(d)
    assert energy_ok_fp64(st.energies(), Eb)


def test_repeat_solve_is_bitwise_deterministic(ctx):
    prob, d = _mixed(32, 30, 7, prec=1)
    st = _state(ctx, prob)
    st.solve(d)
    E1 = st.energies().copy()
    s1 = st.field("sigma")
    st.solve(d[::-1].copy())
    st.solve(d)
    assert np.array_equal(st.energies(), E1)
    assert np.array_equal(st.field("sigma"), s1)


# --------------------------------------------------------------- incremental update


@pytest.mark.parametrize("prec", [0, 1])
def test_hops_match_resolve_and_oracle(ctx, prec):
    prob, d = _mixed(32, 20, 8, prec=prec)
    rng = np.random.default_rng(9)
    st = _state(ctx, prob)
    st.solve(d)
    st.energies()
    cur = d.copy()
    for _ in range(12):
        i = int(rng.integers(0, len(cur)))
        hop = inputs.HOPS111[rng.integers(0, 8)]
        cur[i]["c"] = cur[i]["c"] + hop * prob.h
        E = st.update(i, cur[i])
    Eo = energy.energies_fast(prob, cur)
    ref = _state(ctx, prob)
    ref.solve(cur)
    Er = ref.energies()
    if prec == 0:
        assert energy_ok_fp64(E, Eo)
        assert energy_ok_fp64(E, Er)
        assert rel_l2(st.field("sigma"), ref.field("sigma")) < 1e-12
    else:
        assert np.all(energy_ok_fp32(E, Eo))
        assert np.all(energy_ok_fp32(E, Er))
    assert [np.array_equal(np.sort(a), b) for a, b in zip(st.footprints(), ref.footprints())] == [True] * len(cur)
    assert np.array_equal(st.field("eps_star"), ref.field("eps_star"))


@pytest.mark.parametrize("prec", [0, 1])
def test_update_drift_over_many_moves(ctx, prec):
    """400 incremental moves (hops and a few general moves) accumulated in the
    resident FP64 stress stay at the tolerance of a fresh solve of the final
    list."""
    prob, d = _mixed(64, 60, 12, prec=prec)
    rng = np.random.default_rng(13)
    st = _state(ctx, prob)
    st.solve(d)
    st.energies()
    cur = d.copy()
    for k in range(400):
        i = int(rng.integers(0, len(cur)))
        if k % 50 == 49:  # general move: off-grid shift and a new radius
            cur[i]["c"] = cur[i]["c"] + rng.uniform(-0.4, 0.4, 3)
            cur[i]["radius"] = cur[i]["radius"] * rng.uniform(0.8, 1.1)
        else:
            cur[i]["c"] = cur[i]["c"] + inputs.HOPS111[rng.integers(0, 8)] * prob.h
        st.update(i, cur[i], energies=(k % 100 == 99))
    E = st.energies()
    ref = _state(ctx, prob)
    ref.solve(cur)
    Er = ref.energies()
    if prec == 0:
        assert energy_ok_fp64(E, Er)
        assert rel_l2(st.field("sigma"), ref.field("sigma")) < 1e-12
    else:
        assert np.all(energy_ok_fp32(E, Er))
        assert rel_l2(st.field("sigma"), ref.field("sigma")) < 1e-5
    assert np.array_equal(st.field("eps_star"), ref.field("eps_star"))
    st.close()
    ref.close()


def test_general_move_matches_resolve(ctx):
    prob, d = _mixed(32, 15, 10)
    st = _state(ctx, prob)
    st.solve(d)
    cur = d.copy()
    cur[3]["c"] = cur[3]["c"] + np.array([0.37, -1.21, 0.05])  # not a whole-voxel move
    cur[3]["radius"] *= 1.3
    E = st.update(3, cur[3])
    Eo = energy.energies_fast(prob, cur)
    assert energy_ok_fp64(E, Eo)


def _move_kinds(d, prob):
    """Moves that change a defect's eigenstrain, not only its position: a
    reversed Burgers vector with the habit normal kept (E -> -E), a new
    sphere dilatation, a thicker slab, and a loop turned into a sphere."""
    loops = np.flatnonzero(d["kind"] == 0)
    spheres = np.flatnonzero(d["kind"] == 1)
    i, j, k = int(loops[0]), int(spheres[0]), int(loops[1])
    moves = []
    m = d[i].copy()
    m["b"] = -m["b"]
    moves.append((i, m))
    m = d[j].copy()
    m["eig_v"] = 2.5 * m["eig_v"]
    moves.append((j, m))
    m = d[k].copy()
    m["thickness"] = 2.0 * prob.h
    moves.append((k, m))
    m = d[i].copy()  # the reversed loop of the first move becomes a sphere
    m["kind"] = 1
    m["radius"] = 1.7 * prob.h
    m["eig_v"] = 0.011
    moves.append((i, m))
    return moves


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("bc", [0, 1])
def test_moves_that_change_the_eigenstrain(ctx, prec, bc):
    """ec_update_defect with a new eigenstrain (App. B: the old field out, the
    new one in): after every move the incremental state matches a fresh solve
    of the moved list and the oracle."""
    prob, d = _mixed(32, 16, 21, prec=prec, bc=bc)
    st = _state(ctx, prob)
    st.solve(d)
    cur = d.copy()
    for idx, rec in _move_kinds(d, prob):
        cur[idx] = rec
        E = st.update(idx, rec)
        ref = _state(ctx, prob)
        ref.solve(cur)
        Er = ref.energies()
        Eo = energy.energies_fast(prob, cur)
        assert np.array_equal(st.field("eps_star"), ref.field("eps_star"))
        if prec == 0:
            assert energy_ok_fp64(E, Eo)
            assert energy_ok_fp64(E, Er)
            assert rel_l2(st.field("sigma"), ref.field("sigma")) < 1e-12
        else:
            assert np.all(energy_ok_fp32(E, Eo))
            assert rel_l2(st.field("sigma"), ref.field("sigma")) < 1e-5
        ref.close()
    st.close()
