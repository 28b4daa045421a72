"""Dipole-tensor interaction energies (oracle; test infrastructure only).

Sec. 2.1: when the field of the other defects is nearly constant over a
defect, the interaction integral is approximated by the dipole tensor of the
defect times that field at the defect's position,

    E_i^dip = -P_i : eps_others(X_i),   P_i = Omega_i C : mean(eps*_i),

which for a uniform eigenstrain E_i over m_i voxels of volume h^3 is

    E_i^dip = -h^3 c m_i E_i : sigma_others(X_i)

(C symmetric: (C:E):eps = E:(C:eps) = E:sigma), the exact energy of ``energy``
with the sum over the footprint replaced by m_i times the value at X_i.
Reading: the field is taken at the voxel that contains the defect centre
(quantised centre, floor to the voxel), the grid value the solver holds there.
"""
from __future__ import annotations

import numpy as np

from .elastic import GPA_NM3_EV, stiffness_of
from .energy import green_window, min_image, voxel_coords, window_halfwidth
from .raster import QSUB, eigenstrain_field, quantise
from .solve import solve_field


def centre_voxels(problem, defects) -> np.ndarray:
    """Linear id of the voxel containing each defect's (quantised) centre."""
    n = problem.n
    out = np.zeros(len(defects), dtype=np.int64)
    for i, d in enumerate(defects):
        cq = quantise(problem, d)["cq"]
        v = [int(c) // QSUB % n for c in cq]
        out[i] = (v[2] * n + v[1]) * n + v[0]
    return out


def dipole_energies_brute(problem, fps, Es, xc, bc=None):
    """E_i^dip from the definition: the field of every other defect from its own
    solve, summed and taken at the voxel xc[i]."""
    bc = problem.bc if bc is None else bc
    C = stiffness_of(problem)
    n, L = problem.n, problem.L
    h3c = (L / n) ** 3 * GPA_NM3_EV
    k = len(fps)
    sig = []
    for m in range(k):
        _, s_m, _ = solve_field(C, L, eigenstrain_field(n, fps, Es, select=[m]), bc)
        sig.append(s_m.reshape(3, 3, -1))
    out = np.zeros(k)
    for i in range(k):
        others = sum((sig[m][:, :, xc[i]] for m in range(k) if m != i), np.zeros((3, 3)))
        out[i] = -h3c * len(fps[i]) * float(np.einsum("ij,ij->", Es[i], others))
    return out


def dipole_energies_fast(problem, fps, Es, xc, bc=None, G=None, D=None):
    """E_i^dip from the total field and the defect's own field at xc[i]:
    sigma_others(xc) = sigma(xc) - sum_{y in Omega_i} G(xc - y) : E_i."""
    bc = problem.bc if bc is None else bc
    C = stiffness_of(problem)
    n, L = problem.n, problem.L
    h3c = (L / n) ** 3 * GPA_NM3_EV
    _, sig, _ = solve_field(C, L, eigenstrain_field(n, fps, Es), bc)
    sf = sig.reshape(3, 3, -1)
    if G is None:
        D = window_halfwidth(fps, n)
        G = green_window(C, L, n, D, bc)
    W = 2 * D + 1
    out = np.zeros(len(fps))
    for i, (ids, E) in enumerate(zip(fps, Es)):
        if len(ids) == 0:
            continue
        pc = voxel_coords(np.array([xc[i]]), n)[0]
        r = min_image(pc[None, :] - voxel_coords(np.asarray(ids, dtype=np.int64), n), n)
        if np.abs(r).max() > D:
            raise ValueError("window half-width too small for the centre offsets")
        flat = ((r[:, 2] + D) * W + (r[:, 1] + D)) * W + (r[:, 0] + D)
        own = np.einsum("ijklr,kl->ij", G.reshape(3, 3, 3, 3, -1)[..., flat], E)
        out[i] = -h3c * len(ids) * float(np.einsum("ij,ij->", E, sf[:, :, xc[i]] - own))
    return out
