"""Pins of the rotated-crystal stiffness (the cell axes of Sec. 4 along
[111], [-1-12], [1-10]): the textbook longitudinal modulus of a cubic crystal
along any direction, the rotation invariants, cubic symmetry operations and an
isotropic crystal leave C unchanged, and the solve with a rotated C keeps
equilibrium per frequency and the brute-force / fast-exact energy identity."""
import numpy as np

from oracle import elastic, energy, raster, solve
from paper_2403_09158_amd import inputs

C11, C12, C44 = inputs.CUBIC_FE


def _longitudinal(nv):
    """C'_nnnn of a cubic crystal along the unit direction n (cube coordinates):
    C11 - 2 (C11 - C12 - 2 C44) (n1^2 n2^2 + n2^2 n3^2 + n3^2 n1^2)."""
    n1, n2, n3 = nv
    return C11 - 2.0 * (C11 - C12 - 2.0 * C44) * (n1 * n1 * n2 * n2 + n2 * n2 * n3 * n3 + n3 * n3 * n1 * n1)


def _random_rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[2] = -q[2]
    return q


def test_longitudinal_moduli_of_the_papers_frame():
    A = np.array(inputs.FRAME_111).reshape(3, 3)
    Cr = elastic.rotate_stiffness(elastic.cubic_stiffness(C11, C12, C44), A)
    assert abs(Cr[0, 0, 0, 0] - (C11 + 2 * C12 + 4 * C44) / 3) < 1e-12 * C11  # along [111]
    assert abs(Cr[1, 1, 1, 1] - (C11 + C12 + 2 * C44) / 2) < 1e-12 * C11  # along <112>
    assert abs(Cr[2, 2, 2, 2] - (C11 + C12 + 2 * C44) / 2) < 1e-12 * C11  # along <110>
    rng = np.random.default_rng(inputs.SEED_BASE + 900)
    for _ in range(5):
        R = _random_rotation(rng)
        Cr = elastic.rotate_stiffness(elastic.cubic_stiffness(C11, C12, C44), R)
        for i in range(3):
            assert abs(Cr[i, i, i, i] - _longitudinal(R[i])) < 1e-10 * C11


def test_rotation_invariants_and_symmetry():
    C = elastic.cubic_stiffness(C11, C12, C44)
    rng = np.random.default_rng(inputs.SEED_BASE + 901)
    R = _random_rotation(rng)
    Cr = elastic.rotate_stiffness(C, R)
    assert abs(np.einsum("iijj->", Cr) - np.einsum("iijj->", C)) < 1e-10 * C11
    assert abs(np.einsum("ijij->", Cr) - np.einsum("ijij->", C)) < 1e-10 * C11
    # major and minor symmetries survive
    assert np.allclose(Cr, Cr.transpose(1, 0, 2, 3), atol=1e-12 * C11)
    assert np.allclose(Cr, Cr.transpose(2, 3, 0, 1), atol=1e-12 * C11)
    # a quarter turn about a cube axis is a symmetry of the cubic crystal
    Q = np.array([[0.0, 1.0, 0.0], [-1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    assert np.abs(elastic.rotate_stiffness(C, Q) - C).max() < 1e-12 * C11
    # an isotropic crystal has no orientation
    c11i, c12i, c44i = inputs.isotropic_C(210.0, 0.29)
    Ci = elastic.cubic_stiffness(c11i, c12i, c44i)
    assert np.abs(elastic.rotate_stiffness(Ci, R) - Ci).max() < 1e-12 * c11i


def _cell(n=16, frame=inputs.FRAME_111, Cs=inputs.CUBIC_FE):
    h = inputs.H_VOXEL
    prob = inputs.Problem(n, n * h, *Cs, frame=frame)
    bx = 0.5 * inputs.A_FE * np.sqrt(3.0) * np.array([1.0, 0.0, 0.0])  # 1/2[111] along the cell x axis
    d = np.concatenate(
        [
            inputs.loop(np.array([4.5, 5.5, 6.5]) * h, 2.2 * h, bx, bx),
            inputs.loop(np.array([11.2, 10.7, 9.4]) * h, 1.8 * h, 0.5 * inputs.A_FE * np.array([0.0, 0.0, 1.0]), np.array([0.0, 0.0, 1.0])),
            inputs.sphere(np.array([12.5, 3.5, 12.5]) * h, 1.6 * h, 0.01),
        ]
    )
    return prob, d


def test_isotropic_solve_is_orientation_free():
    Cs = inputs.isotropic_C(210.0, 0.29)
    p0, d = _cell(Cs=Cs, frame=())
    p1, _ = _cell(Cs=Cs)
    E0 = energy.energies_fast(p0, d)
    E1 = energy.energies_fast(p1, d)
    assert np.abs(E1 - E0).max() <= 1e-10 * np.abs(E0).max()


def test_rotated_solve_equilibrium_and_energy_identity():
    prob, d = _cell()
    C = elastic.stiffness_of(prob)
    assert abs(C[0, 0, 0, 0] - (C11 + 2 * C12 + 4 * C44) / 3) < 1e-12 * C11
    fps, Es = raster.rasterise(prob, d)
    es = raster.eigenstrain_field(prob.n, fps, Es)
    eps, sig, _ = solve.solve_field(C, prob.L, es, prob.bc)
    # equilibrium per frequency: xi_j sigma_hat_ij = 0 (labels of Sec. 3.4)
    n = prob.n
    sh = np.fft.fftn(sig, axes=(-3, -2, -1))
    k = np.fft.fftfreq(n, 1.0 / n)
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    xi = np.stack([kx, ky, kz])
    odd = (np.abs(kx) != n // 2) & (np.abs(ky) != n // 2) & (np.abs(kz) != n // 2)
    div = np.einsum("ij...,j...->i...", sh, xi)[:, odd]
    assert np.abs(div).max() <= 1e-10 * np.abs(sh).max() * n
    # the mean stress vanishes (bc 0)
    assert np.abs(sig.mean(axis=(-3, -2, -1))).max() <= 1e-12 * np.abs(sig).max()
    Eb, _ = energy.energies_brute(prob, d)
    Ef = energy.energies_fast(prob, d)
    assert np.abs(Ef - Eb).max() <= 1e-10 * np.abs(Eb).max()
    # the orientation matters for these defects
    E0 = energy.energies_fast(prob.with_(frame=()), d)
    assert np.abs(E0 - Ef).max() > 1e-3 * np.abs(Ef).max()
