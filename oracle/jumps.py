"""Jump-probe energies and biased jump selection (oracle; test infrastructure only).

The OkMC loop of App. B: for every candidate jump lambda_j of a moving defect
d_i, the defect's field is taken out of the total field and put back at
X_i + lambda_j, and the elastic energy of that configuration is compared with
the current one.  For a rigid whole-voxel translation the defect's own energy
is unchanged, so the difference is the change of d_i's interaction energy with
all the other defects (which stay where they are):

    dE_ij = E_i(X_i + lambda_j) - E_i(X_i),
    E_i(X) = -h^3 c sum_{k != i} sum_{x in Omega_i(X)} E_i : sigma_k(x)

(the pair energy of Sec. 2 in the eigenstrain form used by ``energy``).

Sec. 5 (biased jumps): the barrier of a jump is raised by half the energy
change (the saddle point halfway between the two positions), so

    nu_i^j = 1/2 nu_0 exp(-(E_m,i + dE_ij / 2) / (k_B T)),

the frequency line is R_k = sum_{j <= k} nu_i^j, and with xi in (0, 1] the
selected jump j is the one with R_{j-1} / R_tot < xi <= R_j / R_tot.

Jumps are whole-voxel offsets (integer vectors in voxel units), the moves of
the incremental update.
"""
from __future__ import annotations

import numpy as np

from .elastic import GPA_NM3_EV, stiffness_of
from .energy import green_window, min_image, voxel_coords, window_halfwidth
from .raster import eigenstrain_field
from .solve import solve_field


def shift_ids(ids: np.ndarray, lam, n: int) -> np.ndarray:
    """Voxel ids of a footprint translated by the integer vector lam (periodic)."""
    p = voxel_coords(np.asarray(ids, dtype=np.int64), n)
    q = (p + np.asarray(lam, dtype=np.int64)[None, :]) % n
    return (q[:, 2] * n + q[:, 1]) * n + q[:, 0]


def jump_energies_brute(problem, fps, Es, jumps, bc=None):
    """dE[i, j] from the definition: the field of every defect alone (one solve
    each; a jump of d_i leaves the others' fields unchanged), summed over the
    translated footprint of d_i.  jumps[i][j] is an integer voxel vector."""
    bc = problem.bc if bc is None else bc
    C = stiffness_of(problem)
    n, L = problem.n, problem.L
    h3c = (L / n) ** 3 * GPA_NM3_EV
    k = len(fps)
    sig = []
    for m in range(k):
        eps_m = eigenstrain_field(n, fps, Es, select=[m])
        _, s_m, _ = solve_field(C, L, eps_m, bc)
        sig.append(s_m.reshape(3, 3, -1))
    nj = len(jumps[0]) if k else 0
    dE = np.zeros((k, nj))
    for i in range(k):
        others = sum(sig[m] for m in range(k) if m != i) if k > 1 else np.zeros((3, 3, n**3))
        e0 = -h3c * float(np.einsum("ij,ijx->", Es[i], others[:, :, fps[i]]))
        for j, lam in enumerate(jumps[i]):
            ids = shift_ids(fps[i], lam, n)
            e1 = -h3c * float(np.einsum("ij,ijx->", Es[i], others[:, :, ids]))
            dE[i, j] = e1 - e0
    return dE


def cross_term(ids, E, lam, G, D, n):
    """sum over x in Omega + lam, y in Omega of E : G(x - y) : E (all ordered
    pairs; lam = 0 gives the self-term sum)."""
    if len(ids) == 0:
        return 0.0
    p = voxel_coords(np.asarray(ids, dtype=np.int64), n)
    r = min_image(p[:, None, :] + np.asarray(lam)[None, None, :] - p[None, :, :], n).reshape(-1, 3)
    if np.abs(r).max() > D:
        raise ValueError("window half-width too small for this jump")
    W = 2 * D + 1
    flat = ((r[:, 2] + D) * W + (r[:, 1] + D)) * W + (r[:, 0] + D)
    u, cnt = np.unique(flat, return_counts=True)
    g = np.einsum("ij,ijklr,kl->r", E, G.reshape(3, 3, 3, 3, -1)[..., u], E)
    return float(cnt @ g)


def jump_energies_fast(problem, fps, Es, jumps, bc=None, G=None, D=None):
    """dE[i, j] by superposition from the total field sigma and a window of the
    periodic kernel G (sigma = G * eps*):

        E_i(X + lam) = -h^3 c E_i : sum_{x in Omega_i + lam} (sigma - sigma_i)(x),
        sigma_i(x) = sum_{y in Omega_i} G(x - y) : E_i,

    so dE_ij = -h^3 c E_i : (S_i(lam) - S_i(0)) + h^3 c (X_i(lam) - X_i(0)) with
    S_i(lam) the sum of sigma over the translated footprint and X_i the
    ``cross_term``."""
    bc = problem.bc if bc is None else bc
    C = stiffness_of(problem)
    n, L = problem.n, problem.L
    h3c = (L / n) ** 3 * GPA_NM3_EV
    eps_star = eigenstrain_field(n, fps, Es)
    _, sig, _ = solve_field(C, L, eps_star, bc)
    sf = sig.reshape(3, 3, -1)
    if G is None:
        reach = max((int(np.abs(np.asarray(l)).max()) for js in jumps for l in js), default=0)
        D = min(window_halfwidth(fps, n) + reach, n // 2)
        G = green_window(C, L, n, D, bc)
    k = len(fps)
    nj = len(jumps[0]) if k else 0
    dE = np.zeros((k, nj))
    for i in range(k):
        S0 = sf[:, :, fps[i]].sum(axis=-1)
        X0 = cross_term(fps[i], Es[i], (0, 0, 0), G, D, n)
        for j, lam in enumerate(jumps[i]):
            S1 = sf[:, :, shift_ids(fps[i], lam, n)].sum(axis=-1)
            X1 = cross_term(fps[i], Es[i], lam, G, D, n)
            dE[i, j] = -h3c * float(np.einsum("ij,ij->", Es[i], S1 - S0)) + h3c * (X1 - X0)
    return dE


def jump_frequencies(dE, Em, kT, nu0):
    """nu[i, j] = 1/2 nu0 exp(-(Em_i + dE_ij / 2) / kT) (Sec. 5, biased forward
    frequency with the barrier raised halfway)."""
    dE = np.asarray(dE, dtype=np.float64)
    Em = np.broadcast_to(np.asarray(Em, dtype=np.float64).reshape(-1, 1), dE.shape)
    return 0.5 * nu0 * np.exp(-(Em + 0.5 * dE) / kT)


def select_jumps(nu, xi):
    """Index j per row with R_{j-1} / R_tot < xi <= R_j / R_tot on the frequency
    line R_k = sum_{j <= k} nu_j (xi in (0, 1]); -1 for a row with no jumps."""
    nu = np.asarray(nu, dtype=np.float64)
    out = np.full(nu.shape[0], -1, dtype=np.int64)
    for i in range(nu.shape[0]):
        if nu.shape[1] == 0:
            continue
        R = np.cumsum(nu[i])
        tot = R[-1]
        for j in range(nu.shape[1]):
            if xi[i] <= R[j] / tot:
                out[i] = j
                break
        else:
            out[i] = nu.shape[1] - 1
    return out
