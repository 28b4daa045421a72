"""Pins of the jump oracle: the superposition form against the definition, a
jump of the defect record against the translated footprint, the identity jump,
the symmetry of the cross term, and closed forms of the biased frequencies and
the frequency-line selection."""
import numpy as np
import pytest

from oracle import elastic, energy, jumps, raster
from paper_2403_09158_amd import inputs


def _cell():
    """Three defects in a 32^3 cubic-Fe cell, one across the periodic boundary."""
    n = 32
    h = inputs.H_VOXEL
    L = n * h
    prob = inputs.Problem(n, L, *inputs.CUBIC_FE)
    b = 0.5 * inputs.A_FE * np.array([1.0, 1.0, 1.0])
    b2 = 0.5 * inputs.A_FE * np.array([1.0, -1.0, 1.0])
    d = np.concatenate(
        [
            inputs.loop(np.array([10.5, 12.5, 11.5]) * h, 2.6 * h, b, b),
            inputs.loop(np.array([21.2, 17.7, 19.4]) * h, 2.2 * h, b2, b2),
            inputs.sphere(np.array([31.5, 3.5, 16.5]) * h, 1.8 * h, 0.01),
        ]
    )
    return prob, d


JUMPS = [[(1, 1, 1), (-1, -1, -1), (0, 0, 0)], [(1, -1, 1), (-1, 1, -1), (2, 0, 0)], [(1, 0, 0), (0, -1, 0), (0, 0, 1)]]


@pytest.fixture(scope="module")
def cell():
    prob, d = _cell()
    fps, Es = raster.rasterise(prob, d)
    return prob, d, fps, Es


def test_superposition_form_matches_definition(cell):
    prob, _, fps, Es = cell
    brute = jumps.jump_energies_brute(prob, fps, Es, JUMPS)
    fast = jumps.jump_energies_fast(prob, fps, Es, JUMPS)
    scale = np.abs(brute).max()
    assert scale > 1e-6  # the jumps do change the energies
    assert np.abs(fast - brute).max() <= 1e-10 * scale


def test_identity_jump_changes_nothing(cell):
    prob, _, fps, Es = cell
    dE = jumps.jump_energies_fast(prob, fps, Es, [[(0, 0, 0)]] * len(fps))
    assert np.all(dE == 0.0)
    dEb = jumps.jump_energies_brute(prob, fps, Es, [[(0, 0, 0)]] * len(fps))
    assert np.all(dEb == 0.0)


def test_translated_footprint_is_the_moved_defect(cell):
    """Moving a defect record's centre by a whole voxel rasterises to the
    translated footprint, and the jump energy is the energy change of that move
    computed from scratch (one solve per defect, both configurations)."""
    prob, d, fps, Es = cell
    h = prob.L / prob.n
    E0, _ = energy.energies_brute(prob, d)
    for i, lam in ((0, (1, 1, 1)), (1, (-1, 1, -1)), (2, (1, 0, 0))):
        moved = d.copy()
        moved["c"][i] = moved["c"][i] + np.asarray(lam, dtype=np.float64) * h
        fps1, _ = raster.rasterise(prob, moved)
        assert np.array_equal(np.sort(fps1[i]), np.sort(jumps.shift_ids(fps[i], lam, prob.n)))
        E1, _ = energy.energies_brute(prob, moved)
        dE = jumps.jump_energies_brute(prob, fps, Es, [[lam]] * len(fps))[i, 0]
        assert abs(dE - (E1[i] - E0[i])) <= 1e-10 * max(abs(E0[i]), abs(dE), 1e-12)


def test_cross_term_symmetric_in_the_jump(cell):
    prob, _, fps, Es = cell
    C = elastic.stiffness_of(prob)
    D = energy.window_halfwidth(fps, prob.n) + 2
    G = energy.green_window(C, prob.L, prob.n, D)
    for ids, E in zip(fps, Es):
        for lam in ((1, 1, 1), (2, 0, -1)):
            a = jumps.cross_term(ids, E, lam, G, D, prob.n)
            b = jumps.cross_term(ids, E, tuple(-v for v in lam), G, D, prob.n)
            assert abs(a - b) <= 1e-12 * abs(a)
        # lam = 0 is the self-term sum
        h3c = (prob.L / prob.n) ** 3 * elastic.GPA_NM3_EV
        B = energy.self_term(ids, E, G, D, prob.n, h3c)
        assert abs(-h3c * jumps.cross_term(ids, E, (0, 0, 0), G, D, prob.n) - B) <= 1e-12 * abs(B)


def test_biased_frequencies_closed_forms():
    nu0, kT, Em = 1.0e13, 0.025, 0.3
    nu = jumps.jump_frequencies(np.zeros((2, 3)), [Em, Em], kT, nu0)
    assert np.allclose(nu, 0.5 * nu0 * np.exp(-Em / kT), rtol=1e-15, atol=0)
    dE = np.array([[0.04, -0.04, 0.0]])
    nu = jumps.jump_frequencies(dE, [Em], kT, nu0)
    # half the energy change raises (or lowers) the barrier
    assert np.isclose(nu[0, 0] / nu[0, 2], np.exp(-0.02 / kT), rtol=1e-14)
    assert np.isclose(nu[0, 1] / nu[0, 2], np.exp(0.02 / kT), rtol=1e-14)
    assert np.isclose(nu[0, 0] * nu[0, 1], nu[0, 2] ** 2, rtol=1e-14)


def test_frequency_line_selection():
    nu = np.array([[1.0, 1.0, 1.0, 1.0], [1.0, 2.0, 3.0, 4.0], [5.0, 0.0, 0.0, 0.0]])
    # equal frequencies: jump ceil(4 xi) - 1
    for xi, want in ((1e-12, 0), (0.25, 0), (0.2500001, 1), (0.5, 1), (0.75, 2), (0.76, 3), (1.0, 3)):
        assert jumps.select_jumps(nu[:1], [xi])[0] == want
    # R = 1, 3, 6, 10: boundaries at 0.1, 0.3, 0.6
    for xi, want in ((0.1, 0), (0.1000001, 1), (0.3, 1), (0.6, 2), (0.61, 3), (1.0, 3)):
        assert jumps.select_jumps(nu[1:2], [xi])[0] == want
    # zero-frequency jumps are never chosen
    assert all(jumps.select_jumps(nu[2:3], [xi])[0] == 0 for xi in (1e-9, 0.5, 1.0))
