"""Straight dislocation lines by field dislocation mechanics (oracle; test
infrastructure only).

Sec. 3.1, for dislocations that do not close into loops: the plastic
distortion U^p has an incompatible part fixed by the Nye tensor alpha (the net
Burgers vector density), curl U^p = -alpha with (curl A)_ij = e_jkl d_k A_il,
and a divergence-free incompatible part solves div grad U = curl alpha, which in
Fourier space reads

    U_hat_ij(xi) = -i xi_k / |xi|^2 e_jkl alpha_hat_il(xi),   xi != 0.

The compatible part is a constant that only closed loops carry.  The plastic
strain sym(U^p) then enters the Green solve as an eigenstrain (Sec. 3.2).

Readings: (i) a line is infinite and straight along a cell axis (the straight
dislocations of the paper's validation lie along cell axes of its rotated
frame); its Burgers vector density is spread, for every one-voxel subsegment,
to the grid points around the subsegment's midpoint with trilinear weights.
The midpoints lie on voxel-centre levels along the line, so the weights reduce
to the bilinear ones of the four grid points around the line in the
transverse plane; a unit weight carries the density 1 / h^2 (one Burgers
vector through one voxel face).  (ii) xi = 0: no plastic distortion (straight
lines have no compatible part).  (iii) Even n: the real part of the centred
full-complex solution, as in the Green step.
"""
from __future__ import annotations

import numpy as np

from .elastic import stiffness_of
from .solve import centred_labels, fft3, solve_field

# Levi-Civita symbol e_jkl
LEVI = np.zeros((3, 3, 3))
for _i, _j, _k in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
    LEVI[_i, _j, _k] = 1.0
    LEVI[_i, _k, _j] = -1.0


def line_direction(axis: int, sign: int) -> np.ndarray:
    t = np.zeros(3)
    t[axis] = float(sign)
    return t


def nye_field(problem, lines) -> np.ndarray:
    """alpha_ij(x) = b_i t_j rho(x) summed over the lines, shape (3, 3, n, n, n)
    [z, y, x].  A line is (p, axis, sign, b): a point p (nm) on it, the cell
    axis (0, 1, 2) it runs along, its sense (+1 / -1) and its Burgers vector
    (nm)."""
    n, h = problem.n, problem.L / problem.n
    alpha = np.zeros((3, 3, n, n, n))
    for p, axis, sign, b in lines:
        t = line_direction(axis, sign)
        a1, a2 = [a for a in range(3) if a != axis]
        u1 = float(p[a1]) / h - 0.5  # grid-index coordinates (voxel centres at integers)
        u2 = float(p[a2]) / h - 0.5
        f1, f2 = int(np.floor(u1)), int(np.floor(u2))
        for i1 in (f1, f1 + 1):
            for i2 in (f2, f2 + 1):
                w = (1.0 - abs(u1 - i1)) * (1.0 - abs(u2 - i2))
                if w == 0.0:
                    continue
                sl = [slice(None)] * 3  # array axes are (z, y, x) = cell axes (2, 1, 0)
                sl[2 - a1] = i1 % n
                sl[2 - a2] = i2 % n
                alpha[(slice(None), slice(None)) + tuple(sl)] += np.outer(b, t)[:, :, None] * (w / (h * h))
    return alpha


def plastic_distortion(problem, alpha) -> np.ndarray:
    """U^p (3, 3, n, n, n) from the Nye tensor by the Fourier solution above."""
    n, L = problem.n, problem.L
    ah = fft3(alpha)
    lab = centred_labels(n) * (2.0 * np.pi / L)
    kz, ky, kx = np.meshgrid(lab, lab, lab, indexing="ij")
    xi = np.stack([kx, ky, kz])  # (3, z, y, x)
    x2 = (xi * xi).sum(axis=0)
    x2[0, 0, 0] = 1.0
    # U_hat_ij = -i xi_k e_jkl alpha_hat_il / |xi|^2
    Uh = -1j * np.einsum("kzyx,jkl,ilzyx->ijzyx", xi, LEVI, ah) / x2
    Uh[:, :, 0, 0, 0] = 0.0
    return fft3(Uh, inverse=True).real


def dislocation_eigenstrain(problem, lines) -> np.ndarray:
    U = plastic_distortion(problem, nye_field(problem, lines))
    return 0.5 * (U + U.transpose(1, 0, 2, 3, 4))


def dislocation_stress(problem, lines, bc=None) -> np.ndarray:
    """sigma (3, 3, n, n, n) of the lines alone: the Green solve of sym(U^p)."""
    bc = problem.bc if bc is None else bc
    _, sig, _ = solve_field(stiffness_of(problem), problem.L, dislocation_eigenstrain(problem, lines), bc)
    return sig


def background_energies(problem, fps, Es, sig_d) -> np.ndarray:
    """Interaction energy of each defect with the lines' field,
    -h^3 c sum_{x in Omega_i} E_i : sigma_d(x) (the pair form of Sec. 2)."""
    from .elastic import GPA_NM3_EV

    h3c = (problem.L / problem.n) ** 3 * GPA_NM3_EV
    sf = sig_d.reshape(3, 3, -1)
    return np.array([-h3c * float(np.einsum("ij,ijx->", E, sf[:, :, ids])) for ids, E in zip(fps, Es)])
