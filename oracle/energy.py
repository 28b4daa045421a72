"""Per-defect interaction energies (oracle; test infrastructure only).

Sec. 2 gives the interaction energy of a defect with an external field in the
Betti-reciprocity form, an integral of sigma^ext : eps^{d,e}.  For periodic,
compatible total strains the integral of sigma^ext : eps^d vanishes (the
integration-by-parts argument of Appendix A, with u equal on opposite cell
faces), so the pair energy is written with the eigenstrain alone.  Reading used
throughout (the paper evaluates pairs and OkMC energy differences, never an
"all others" sum explicitly):

    E_ij = -h^3 c sum_x eps*_i(x) : sigma_j(x),      E_i = sum_{j != i} E_ij,

where sigma_j is the periodic stress of defect j alone, h^3 the voxel volume
and c = 1 GPa nm^3 in eV.  ``energies_brute`` is this definition, one solve per
defect.  ``energies_fast`` uses superposition (Sec. 3.3 and Appendix B: the
total field is the sum of the defects' fields):

    E_i = -h^3 c E_i : S_i - B_i,   S_i = sum_{x in Omega_i} sigma(x),
    B_i = -h^3 c sum_{x, y in Omega_i} E_i : G(x - y) : E_i,

with G the discrete periodic kernel sigma = G * eps* (response to a unit
symmetric eigenstrain impulse).  B_i is the self term of defect i.
"""
from __future__ import annotations

import numpy as np

from .elastic import GPA_NM3_EV, stiffness_of
from .raster import eigenstrain_field, rasterise
from .solve import solve_field

SYM_PAIRS = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


def voxel_coords(ids: np.ndarray, n: int) -> np.ndarray:
    """(k, 3) integer (x, y, z) voxel coordinates of linear ids (z n + y) n + x."""
    return np.stack([ids % n, (ids // n) % n, ids // (n * n)], axis=1)


def min_image(r: np.ndarray, n: int) -> np.ndarray:
    return (r + n // 2) % n - n // 2


def energies_brute(problem, defects, bc=None):
    """(E_i, E_ij) by one periodic solve per defect (the definition)."""
    fps, Es = rasterise(problem, defects)
    return energies_brute_fp(problem, fps, Es, bc)


def energies_brute_fp(problem, fps, Es, bc=None):
    """As ``energies_brute`` for given footprints (voxel id arrays) and tensors."""
    bc = problem.bc if bc is None else bc
    C = stiffness_of(problem)
    n, L = problem.n, problem.L
    h3c = (L / n) ** 3 * GPA_NM3_EV
    k = len(fps)
    Eij = np.zeros((k, k))
    for j in range(k):
        eps_j = eigenstrain_field(n, fps, Es, select=[j])
        _, sig_j, _ = solve_field(C, L, eps_j, bc)
        sf = sig_j.reshape(3, 3, -1)
        for i in range(k):
            Eij[i, j] = -h3c * float(np.einsum("ij,ijv->", Es[i], sf[:, :, fps[i]]))
    E = Eij.sum(axis=1) - np.diag(Eij)
    return E, Eij


def window_halfwidth(footprints, n: int) -> int:
    """Largest |component| of a minimum-image pair offset inside any footprint."""
    D = 0
    for ids in footprints:
        if len(ids) == 0:
            continue
        p = voxel_coords(ids, n)
        lo, hi = p.min(axis=0), p.max(axis=0)
        if np.any(hi - lo >= n // 2):
            # footprint wraps (or is wide): measure pair offsets explicitly
            r = min_image(p[:, None, :] - p[None, :, :], n)
            D = max(D, int(np.abs(r).max()))
        else:
            D = max(D, int((hi - lo).max()))
    return min(D, n // 2)


def green_window(C, L, n, D, bc=0):
    """G_ijkl(r) for r in [-D, D]^3, array (3, 3, 3, 3, 2D+1, 2D+1, 2D+1) [rz, ry, rx]."""
    W = 2 * D + 1
    G = np.zeros((3, 3, 3, 3, W, W, W))
    idx = np.arange(-D, D + 1) % n
    for k, l in SYM_PAIRS:
        U = np.zeros((3, 3))
        U[k, l] += 0.5
        U[l, k] += 0.5
        eps = np.zeros((3, 3, n, n, n))
        eps[:, :, 0, 0, 0] = U
        _, sig, _ = solve_field(C, L, eps, bc)
        win = sig[:, :, idx][:, :, :, idx][:, :, :, :, idx]
        G[:, :, k, l] = win
        G[:, :, l, k] = win
    return G


def self_term(ids, E, G, D, n, h3c):
    """B_i = -h^3 c sum over ordered pairs (x, y) in Omega_i of E:G(x - y):E."""
    if len(ids) == 0:
        return 0.0
    p = voxel_coords(ids, n)
    r = min_image(p[:, None, :] - p[None, :, :], n).reshape(-1, 3)
    W = 2 * D + 1
    flat = ((r[:, 2] + D) * W + (r[:, 1] + D)) * W + (r[:, 0] + D)
    u, cnt = np.unique(flat, return_counts=True)
    g = np.einsum("ij,ijklr,kl->r", E, G.reshape(3, 3, 3, 3, -1)[..., u], E)
    return -h3c * float(cnt @ g)


def energies_fast(problem, defects, bc=None, G=None, D=None, return_parts=False):
    """E_i from the total field and exact self terms (superposition)."""
    fps, Es = rasterise(problem, defects)
    return energies_fast_fp(problem, fps, Es, bc, G, D, return_parts)


def energies_fast_fp(problem, fps, Es, bc=None, G=None, D=None, return_parts=False):
    """As ``energies_fast`` for given footprints (voxel id arrays) and tensors."""
    bc = problem.bc if bc is None else bc
    C = stiffness_of(problem)
    n, L = problem.n, problem.L
    h3c = (L / n) ** 3 * GPA_NM3_EV
    eps_star = eigenstrain_field(n, fps, Es)
    _, sig, _ = solve_field(C, L, eps_star, bc)
    del eps_star
    sf = sig.reshape(3, 3, -1)
    S = [sf[:, :, ids].sum(axis=-1) for ids in fps]
    if G is None:
        D = window_halfwidth(fps, n)
        G = green_window(C, L, n, D, bc)
    B = np.array([self_term(ids, E, G, D, n, h3c) for ids, E in zip(fps, Es)])
    ES = np.array([float(np.einsum("ij,ij->", E, s)) for E, s in zip(Es, S)])
    E = -h3c * ES - B
    if return_parts:
        return E, {"S": S, "B": B, "sig": sig, "fps": fps, "Es": Es, "G": G, "D": D}
    return E
