"""Pins of the dipole oracle: the total-field form against the definition, an
isolated defect, the approach of the dipole energy to the exact one as two
loops separate, and the centre-voxel rule."""
import numpy as np

from oracle import dipole, energy, raster
from paper_2403_09158_amd import inputs


def _cell():
    n = 32
    h = inputs.H_VOXEL
    prob = inputs.Problem(n, n * h, *inputs.CUBIC_FE)
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


def test_total_field_form_matches_definition():
    prob, d = _cell()
    fps, Es = raster.rasterise(prob, d)
    xc = dipole.centre_voxels(prob, d)
    brute = dipole.dipole_energies_brute(prob, fps, Es, xc)
    fast = dipole.dipole_energies_fast(prob, fps, Es, xc)
    assert np.abs(brute).max() > 1e-4
    assert np.abs(fast - brute).max() <= 1e-10 * np.abs(brute).max()


def test_isolated_defect_has_no_dipole_energy():
    prob, d = _cell()
    fps, Es = raster.rasterise(prob, d[:1])
    xc = dipole.centre_voxels(prob, d[:1])
    assert dipole.dipole_energies_brute(prob, fps, Es, xc)[0] == 0.0
    assert abs(dipole.dipole_energies_fast(prob, fps, Es, xc)[0]) <= 1e-12


def test_dipole_energy_approaches_exact_for_separating_loops():
    """Two coaxial 1/2[111] loops along [111] (R = 2 voxels): the ratio of the
    dipole energy to the exact pair energy moves towards 1 as they separate and
    is within 2.2 % of it at d/R = 15.6 (Sec. 2.1: the field of the other
    defect nearly constant over the loop)."""
    n = 128
    h = inputs.H_VOXEL
    prob = inputs.Problem(n, n * h, *inputs.CUBIC_FE)
    b = 0.5 * inputs.A_FE * np.array([1.0, 1.0, 1.0])
    c0 = np.array([0.5, 0.5, 0.5]) * h
    ratios = []
    for k in (9, 18):  # d/R = 7.8, 15.6
        d = np.concatenate([inputs.loop(c0, 2.0 * h, b, b), inputs.loop(c0 + k * h, 2.0 * h, b, b)])
        fps, Es = raster.rasterise(prob, d)
        xc = dipole.centre_voxels(prob, d)
        assert xc[1] == (k * n + k) * n + k
        Ed = dipole.dipole_energies_brute(prob, fps, Es, xc)
        Ex, _ = energy.energies_brute(prob, d)
        ratios.append(Ex[1] / Ed[1])
    assert abs(ratios[1] - 1.0) < abs(ratios[0] - 1.0), ratios
    assert abs(ratios[1] - 1.0) < 0.022, ratios


def test_centre_voxel_rule():
    n = 16
    h = inputs.H_VOXEL
    prob = inputs.Problem(n, n * h, *inputs.CUBIC_FE)
    b = 0.5 * inputs.A_FE * np.array([1.0, 1.0, 1.0])
    d = np.concatenate(
        [
            inputs.sphere(np.array([3.5, 4.5, 5.5]) * h, 1.5 * h, 0.01),  # a voxel centre
            inputs.sphere(np.array([4.0, 4.999, 5.0]) * h, 1.5 * h, 0.01),  # faces: floor
            inputs.loop(np.array([-0.25, 16.25, 7.5]) * h, 2.0 * h, b, b),  # wraps
        ]
    )
    xc = dipole.centre_voxels(prob, d)
    assert xc[0] == (5 * n + 4) * n + 3
    assert xc[1] == (5 * n + 4) * n + 4
    assert xc[2] == (7 * n + 0) * n + 15
