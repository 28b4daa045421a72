"""Pins of the shift-theorem translation of stored type fields (oracle/shift.py;
Sec. 3.3, eq. shift).

* a whole-voxel offset is an exact cyclic shift of the voxel field (np.roll), so
  the phase's sign, the label set and the axis order are fixed;
* a sub-voxel offset of a single Fourier mode gives the closed form
  cos(xi . (x - d) + phi) (scale of xi = 2 pi k / L);
* at an even n's Nyquist bin the real-part reading gives cos(pi delta) times the
  mode (the two representatives averaged), a closed form of the reading;
* odd n: a translation by d then by -d is the identity;
* the energy of the translated type at whole-voxel offsets equals the plain
  definition with the defect rasterised there (and, with the moving defect in the
  field, the brute-force energy of the moved list).
"""
import numpy as np
import pytest

from oracle import elastic, energy, raster, shift, solve
from paper_2403_09158_amd import inputs


@pytest.mark.parametrize("n", [8, 9, 12])
def test_whole_voxel_offset_is_a_cyclic_shift(n):
    rng = np.random.default_rng(n)
    L = 2.5 * n
    f = rng.normal(size=(2, n, n, n))
    m = np.array([3, -2, 5])  # voxels along x, y, z
    got = shift.translate(f, m * (L / n), L)
    want = np.roll(f, shift=(m[2], m[1], m[0]), axis=(-3, -2, -1))
    assert np.max(np.abs(got - want)) < 1e-13


@pytest.mark.parametrize("n", [10, 11])
def test_sub_voxel_offset_of_one_mode(n):
    L = 3.7
    h = L / n
    k = np.array([2, -3, 1])  # (kx, ky, kz), all below n/2
    phi = 0.4
    z, y, x = np.meshgrid(*(h * np.arange(n),) * 3, indexing="ij")
    xi = 2.0 * np.pi * k / L
    f = np.cos(xi[0] * x + xi[1] * y + xi[2] * z + phi)
    d = np.array([0.31, -0.77, 0.123]) * h
    got = shift.translate(f, d, L)
    want = np.cos(xi[0] * (x - d[0]) + xi[1] * (y - d[1]) + xi[2] * (z - d[2]) + phi)
    assert np.max(np.abs(got - want)) < 1e-13


def test_even_nyquist_mode_reading():
    n, L = 8, 4.0
    h = L / n
    m = np.arange(n)
    f = np.broadcast_to(np.cos(np.pi * m)[None, None, :], (n, n, n)).copy()  # x Nyquist mode
    delta = 0.3
    got = shift.translate(f, [delta * h, 0.0, 0.0], L)
    assert np.max(np.abs(got - np.cos(np.pi * delta) * f)) < 1e-14


def test_odd_translation_round_trip():
    n, L = 9, 5.0
    rng = np.random.default_rng(3)
    f = rng.normal(size=(n, n, n))
    d = np.array([0.37, 1.91, -0.52])
    back = shift.translate(shift.translate(f, d, L), -d, L)
    assert np.max(np.abs(back - f)) < 1e-13


def _cell(n=16, bc=0, seed=5):
    rng = np.random.default_rng(seed)
    L = n * inputs.H_VOXEL
    prob = inputs.Problem(n, L, *inputs.CUBIC_FE, bc=bc)
    d = inputs.mixed_population(rng, 6, L, L / n, r111=(0.4, 1.0), r100=(0.5, 1.0))
    b = 0.5 * inputs.A_FE * np.array([1.0, -1.0, 1.0])
    proto = inputs.loop(np.array([0.41, 0.57, 0.33]) * L, 0.9, b, b)
    return prob, d, proto


def _field(prob, d):
    fps, Es = raster.rasterise(prob, d)
    es = raster.eigenstrain_field(prob.n, fps, Es)
    _, sig, _ = solve.solve_field(elastic.stiffness_of(prob), prob.L, es, prob.bc)
    return es, sig


@pytest.mark.parametrize("bc", [0, 1])
def test_type_energy_at_whole_voxels_equals_rasterised_defect(bc):
    prob, d, proto = _cell(bc=bc)
    _, sig = _field(prob, d)
    h = prob.h
    offs = np.array([[0, 0, 0], [1, 0, 0], [-3, 2, 5], [7, -8, 1]])
    X = proto["c"][0] + offs * h
    got = shift.type_energies(prob, proto, X, sig)
    h3c = h**3 * elastic.GPA_NM3_EV
    for p, Xp in enumerate(X):
        q = proto.copy()
        q["c"][0] = Xp
        fps, Es = raster.rasterise(prob, q)
        es = raster.eigenstrain_field(prob.n, fps, Es)
        want = -h3c * float(np.sum(es * sig))
        assert abs(got[p] - want) <= 1e-12 * max(1.0, abs(want))


def test_excluded_mover_equals_brute_force_of_the_moved_list():
    """The type defect is part of the field at X_excl; its energy after a
    whole-voxel move equals the brute-force E_i of the list with it moved."""
    prob, d, proto = _cell(seed=6)
    h = prob.h
    Xe = proto["c"][0] + np.array([2, 1, -1]) * h
    q = proto.copy()
    q["c"][0] = Xe
    full = np.concatenate([d, q])
    _, sig = _field(prob, full)
    hop = np.array([1, 1, 1]) * h
    got = shift.type_energies(prob, proto, [Xe, Xe + hop], sig, X_excl=Xe)
    E0, _ = energy.energies_brute(prob, full)
    moved = full.copy()
    moved["c"][-1] = Xe + hop
    E1, _ = energy.energies_brute(prob, moved)
    assert abs(got[0] - E0[-1]) <= 1e-11 * abs(E0[-1])
    assert abs(got[1] - E1[-1]) <= 1e-11 * abs(E1[-1])
