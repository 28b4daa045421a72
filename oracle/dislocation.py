"""Dislocation lines and loops by field dislocation mechanics (oracle; test
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


# --------------------------------------------------------------- closed paths
#
# Sec. 3.1 for dislocations in any direction: a path is a closed polyline, a
# loop (the last vertex joined to the first) or a line through the periodic
# cell (the last vertex joined to the first shifted by a lattice vector of the
# cell).  Readings: (i) every segment is cut into the fewest equal pieces no
# longer than h, and each piece's Burgers vector density b (x) dl / h^3 is
# spread to the eight grid points around its midpoint with trilinear weights
# (the paper spreads every subsegment to the eight surrounding grid points);
# for a line along a cell axis this is the straight-line rule above.  (ii) With
# alpha = b (x) t, t along the vertex order, and curl U^p = -alpha, a loop's
# slipped area carries U^p = -b (x) n with n the right-hand normal of the vertex
# order (a loop running counterclockwise about n has the field of the slab
# eigenstrain -sym(b (x) n) of the defect records); the compatible part is the
# mean plastic distortion of the slipped areas, -b (x) A / V with
# A = 1/2 sum_j v_j x v_{j+1} the vector area of a loop (lines through the cell
# have none): it adds to U_hat at xi = 0 and only changes the mean stress under
# the zero-mean-strain condition.


def path_segments(path):
    """(start, vector) of every segment of a path (verts (k, 3), shift (3,))."""
    verts, shift = np.asarray(path[0], dtype=np.float64), np.asarray(path[1], dtype=np.float64)
    k = len(verts)
    out = []
    for j in range(k):
        a = verts[j]
        b = verts[j + 1] if j + 1 < k else verts[0] + shift
        out.append((a, b - a))
    return out


def path_nye_field(problem, paths) -> np.ndarray:
    """alpha_ij(x) (3, 3, n, n, n) [z, y, x] of closed paths (verts, shift, b)."""
    n, h = problem.n, problem.L / problem.n
    alpha = np.zeros((3, 3, n, n, n))
    for verts, shift, b in paths:
        b = np.asarray(b, dtype=np.float64)
        for a, d in path_segments((verts, shift)):
            m = max(1, int(np.ceil(np.linalg.norm(d) / h - 1e-12)))
            dl = d / m
            for q in range(m):
                mid = a + (q + 0.5) * dl
                u = mid / h - 0.5  # grid-index coordinates
                f = np.floor(u).astype(np.int64)
                for cz in (0, 1):
                    for cy in (0, 1):
                        for cx in (0, 1):
                            g = f + np.array([cx, cy, cz])
                            w = np.prod(1.0 - np.abs(u - g))
                            if w == 0.0:
                                continue
                            gx, gy, gz = (int(v) % n for v in g)
                            alpha[:, :, gz, gy, gx] += np.outer(b, dl) * (w / h**3)
    return alpha


def path_mean_distortion(problem, paths) -> np.ndarray:
    """<U^p> = -sum over loops of b (x) A / V (lines through the cell: none)."""
    V = problem.L**3
    U = np.zeros((3, 3))
    for verts, shift, b in paths:
        if np.any(np.asarray(shift) != 0.0):
            continue
        v = np.asarray(verts, dtype=np.float64)
        A = 0.5 * sum(np.cross(v[j], v[(j + 1) % len(v)]) for j in range(len(v)))
        U -= np.outer(b, A) / V
    return U


def path_stress(problem, paths, bc=None) -> np.ndarray:
    """sigma (3, 3, n, n, n) of the paths alone: sym(U^p) solved as an
    eigenstrain, U^p from the Nye tensor at xi != 0 and the mean distortion at
    xi = 0."""
    bc = problem.bc if bc is None else bc
    U = plastic_distortion(problem, path_nye_field(problem, paths))
    U = U + path_mean_distortion(problem, paths)[:, :, None, None, None]
    es = 0.5 * (U + U.transpose(1, 0, 2, 3, 4))
    _, sig, _ = solve_field(stiffness_of(problem), problem.L, es, bc)
    return sig
