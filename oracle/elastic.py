"""Stiffness tensors and the Green operator (oracle; test infrastructure only).

Sec. 3.2 of the paper: the strain of a periodic homogeneous medium carrying an
eigenstrain is the Green operator applied to C:eps* in Fourier space, and for a
general anisotropic C the operator is built from the inverse of the acoustic
tensor C_ijkl xi_j xi_l.  The printed formula repeats indices (garbled); the
reading used here is the standard symmetrised operator

    Gamma_ijkl(xi) = 1/4 (N_ik xi_j xi_l + N_jk xi_i xi_l + N_il xi_j xi_k + N_jl xi_i xi_k),
    N = K^-1,  K_ik = C_ijkl xi_j xi_l,

which follows from div(C:(eps - eps*)) = 0 with eps = sym grad u, and gives
eps_hat = +Gamma:(C:eps*_hat).  The isotropic closed form the paper cites
(Moulinec & Suquet 1994) is ``gamma_isotropic``; it pins the general form.
"""
from __future__ import annotations

import itertools
import numpy as np

# 1 GPa * nm^3 expressed in eV (1e-18 J / elementary charge).
GPA_NM3_EV = 1.0e-18 / 1.602176634e-19


def cubic_stiffness(C11: float, C12: float, C44: float) -> np.ndarray:
    """Full C_ijkl of a cubic crystal with cube axes along x, y, z."""
    C = np.zeros((3, 3, 3, 3))
    d = np.eye(3)
    for i, j, k, l in itertools.product(range(3), repeat=4):
        C[i, j, k, l] = (
            C12 * d[i, j] * d[k, l]
            + C44 * (d[i, k] * d[j, l] + d[i, l] * d[j, k])
            + (C11 - C12 - 2.0 * C44) * d[i, j] * d[k, l] * d[i, k]
        )
    return C


def isotropic_stiffness(lam: float, mu: float) -> np.ndarray:
    C = np.zeros((3, 3, 3, 3))
    d = np.eye(3)
    for i, j, k, l in itertools.product(range(3), repeat=4):
        C[i, j, k, l] = lam * d[i, j] * d[k, l] + mu * (d[i, k] * d[j, l] + d[i, l] * d[j, k])
    return C


def rotate_stiffness(C: np.ndarray, A) -> np.ndarray:
    """C in the cell frame of a rotated crystal, C'_ijkl = A_ip A_jq A_kr A_ls C_pqrs,
    where the rows of A are the cell axes as unit vectors in cube coordinates
    (Sec. 4 places x, y, z along [111], [-1-12] and [1-10])."""
    A = np.asarray(A, dtype=np.float64).reshape(3, 3)
    return np.einsum("ip,jq,kr,ls,pqrs->ijkl", A, A, A, A, C)


def stiffness_of(problem) -> np.ndarray:
    """The problem's stiffness in cell coordinates (rotated when it gives a frame)."""
    C = cubic_stiffness(problem.C11, problem.C12, problem.C44)
    frame = tuple(getattr(problem, "frame", ()) or ())
    if frame and any(v != 0.0 for v in frame):
        C = rotate_stiffness(C, frame)
    return C


def acoustic_tensor(C: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """K_ik = C_ijkl xi_j xi_l for xi of shape (..., 3)."""
    return np.einsum("ijkl,...j,...l->...ik", C, xi, xi)


def gamma_hat(C: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """Gamma_ijkl(xi) for xi != 0, shape (..., 3, 3, 3, 3)."""
    K = acoustic_tensor(C, xi)
    N = np.linalg.inv(K)
    t1 = np.einsum("...ik,...j,...l->...ijkl", N, xi, xi)
    t2 = np.einsum("...jk,...i,...l->...ijkl", N, xi, xi)
    t3 = np.einsum("...il,...j,...k->...ijkl", N, xi, xi)
    t4 = np.einsum("...jl,...i,...k->...ijkl", N, xi, xi)
    return 0.25 * (t1 + t2 + t3 + t4)


def gamma_isotropic(lam: float, mu: float, xi: np.ndarray) -> np.ndarray:
    """Moulinec-Suquet closed form of the isotropic Green operator, xi != 0."""
    d = np.eye(3)
    x2 = np.einsum("...i,...i->...", xi, xi)[..., None, None, None, None]
    a = (
        np.einsum("ki,...h,...j->...khij", d, xi, xi)
        + np.einsum("hi,...k,...j->...khij", d, xi, xi)
        + np.einsum("kj,...h,...i->...khij", d, xi, xi)
        + np.einsum("hj,...k,...i->...khij", d, xi, xi)
    )
    b = np.einsum("...i,...j,...k,...h->...khij", xi, xi, xi, xi)
    return a / (4.0 * mu * x2) - ((lam + mu) / (mu * (lam + 2.0 * mu))) * b / x2**2


def ddot(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """A_ij B_ij over the two leading tensor axes."""
    return np.einsum("ij...,ij...->...", A, B)
