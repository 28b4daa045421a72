"""Pins of the dislocation-line oracle (field dislocation mechanics, Sec. 3.1):
the isotropic screw dislocation against its textbook stress spectrum (the
antiplane Poisson problem, sigma_hat_xz = i mu b xi_y rho_hat / xi^2,
sigma_hat_yz = -i mu b xi_x rho_hat / xi^2), the curl and divergence identities
of the incompatible distortion per frequency, the Burgers content of the spread
line, and the Volterra stresses of screw and edge lines near the core."""
import numpy as np

from oracle import dislocation as dl
from oracle import solve
from paper_2403_09158_amd import inputs

E_ISO, NU_ISO = 210.0, 0.29
MU = E_ISO / (2.0 * (1.0 + NU_ISO))


def _iso(n):
    h = inputs.H_VOXEL
    return inputs.Problem(n, n * h, *inputs.isotropic_C(E_ISO, NU_ISO))


def _non_nyquist(n):
    m = np.abs(solve.centred_labels(n)) != n // 2
    return m[:, None, None] & m[None, :, None] & m[None, None, :]


def _xi(prob):
    lab = solve.centred_labels(prob.n) * (2.0 * np.pi / prob.L)
    kz, ky, kx = np.meshgrid(lab, lab, lab, indexing="ij")
    return kx, ky, kz


def test_isotropic_screw_has_the_textbook_spectrum():
    prob = _iso(32)
    b = 0.25
    lines = [(np.array([13.3, 17.8, 0.0]) * prob.h, 2, 1, np.array([0.0, 0.0, b]))]
    sig = dl.dislocation_stress(prob, lines)
    rho = dl.nye_field(prob, lines)[2, 2] / b
    S, R = solve.fft3(sig), solve.fft3(rho)
    kx, ky, kz = _xi(prob)
    x2 = kx * kx + ky * ky + kz * kz
    x2[0, 0, 0] = 1.0
    want_xz = 1j * MU * b * ky * R / x2
    want_yz = -1j * MU * b * kx * R / x2
    M = _non_nyquist(prob.n)
    scale = np.abs(want_xz).max()
    assert np.abs(S[0, 2] - want_xz)[M].max() <= 1e-10 * scale
    assert np.abs(S[1, 2] - want_yz)[M].max() <= 1e-10 * scale
    for a, c in ((0, 0), (1, 1), (2, 2), (0, 1)):
        assert np.abs(S[a, c]).max() <= 1e-10 * scale


def test_incompatible_distortion_identities():
    """curl U = -alpha and div U = 0 per frequency for a mixed line (b not along t)."""
    prob = _iso(24)
    lines = [
        (np.array([7.3, 0.0, 11.6]) * prob.h, 1, -1, np.array([0.2, 0.05, -0.1])),
        (np.array([3.0, 20.2, 0.0]) * prob.h, 2, 1, np.array([0.0, 0.15, 0.1])),
    ]
    alpha = dl.nye_field(prob, lines)
    Uh = solve.fft3(dl.plastic_distortion(prob, alpha))
    Ah = solve.fft3(alpha)
    kx, ky, kz = _xi(prob)
    xi = np.stack([kx, ky, kz])
    M = _non_nyquist(prob.n).copy()
    M[0, 0, 0] = False
    # (curl U)_ij = e_jkl i xi_k U_il
    curl = np.einsum("jkl,kzyx,ilzyx->ijzyx", dl.LEVI, 1j * xi, Uh)
    scale = np.abs(Ah).max()
    assert np.abs(curl + Ah)[:, :, M].max() <= 1e-10 * scale
    div = np.einsum("jzyx,ijzyx->izyx", xi, Uh)
    assert np.abs(div)[:, M].max() <= 1e-10 * scale * np.abs(xi).max()


def test_spread_line_carries_one_burgers_vector():
    prob = _iso(16)
    b = np.array([0.1, -0.2, 0.3])
    for axis, sign in ((0, 1), (1, -1), (2, 1)):
        p = np.array([5.37, 9.81, 2.26]) * prob.h
        alpha = dl.nye_field(prob, [(p, axis, sign, b)])
        t = dl.line_direction(axis, sign)
        layer = [slice(None)] * 3
        layer[2 - axis] = 3  # one plane across the line
        tot = alpha[(slice(None), slice(None)) + tuple(layer)].sum(axis=(-2, -1)) * prob.h**2
        assert np.allclose(tot, np.outer(b, t), rtol=0, atol=1e-14)


def test_volterra_stresses_near_the_core():
    """Screw and edge lines in a 64^3 isotropic cell against the Volterra
    stresses of an isolated line, 3 to 6 voxels from the core (the periodic
    images and the spreading account for the few per cent left)."""
    prob = _iso(64)
    h = prob.h
    b = 0.25
    p = np.array([32.0, 32.0, 0.0]) * h
    s_screw = dl.dislocation_stress(prob, [(p, 2, 1, np.array([0.0, 0.0, b]))])
    s_edge = dl.dislocation_stress(prob, [(p, 2, 1, np.array([b, 0.0, 0.0]))])
    for r in (3, 4, 5, 6):
        ix, iy = 32 + r, 35  # a point off both axes
        x, y = (ix + 0.5) * h - p[0], (iy + 0.5) * h - p[1]
        r2 = x * x + y * y
        syz = MU * b / (2 * np.pi) * x / r2
        sxz = -MU * b / (2 * np.pi) * y / r2
        assert abs(s_screw[1, 2, 0, iy, ix] - syz) <= 0.08 * abs(syz)
        assert abs(s_screw[0, 2, 0, iy, ix] - sxz) <= 0.08 * abs(sxz) + 0.02 * abs(syz)
        k = MU * b / (2 * np.pi * (1 - NU_ISO))
        sxy = k * x * (x * x - y * y) / r2**2
        assert abs(s_edge[0, 1, 0, iy, ix] - sxy) <= 0.1 * abs(sxy) + 0.02 * k / np.sqrt(r2)
