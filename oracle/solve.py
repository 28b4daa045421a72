"""Periodic eigenstrain solve by FFT (oracle; test infrastructure only).

Sec. 3.2 / 3.4 of the paper, taken step by step in the paper's order:

1. tau = C:eps* (full 3x3x3x3 contraction);
2. tau_hat = DFT(tau) with full complex transforms (no real-to-complex
   shortcut), indexed by the centred labels of Sec. 3.4:  for even n the labels
   are -n/2 .. n/2-1, for odd n -(n-1)/2 .. (n-1)/2, and xi = 2 pi k / L;
3. eps_hat(xi) = Gamma(xi):tau_hat(xi) for xi != 0;
4. xi = 0 (the paper is silent on the macroscopic condition; reading): with
   ``bc=0`` eps_hat(0) = DFT(eps*)(0), i.e. <eps> = <eps*> and <sigma> = 0;
   with ``bc=1`` eps_hat(0) = 0 (no mean strain);
5. eps = Re(IDFT(eps_hat)).  Taking the real part of the full complex result is
   the literal reading of the centred labels for even n, where a Nyquist bin's
   Hermitian partner carries a different continuous direction;
6. sigma = C:(eps - eps*).

The forward DFT is unnormalised, the inverse scaled by 1/n^3 (numpy/scipy
convention; the paper does not fix one and results do not depend on it).
"""
from __future__ import annotations

import os
import numpy as np
import scipy.fft

from .elastic import gamma_hat

WORKERS = int(os.environ.get("ORACLE_FFT_WORKERS", "0")) or (os.cpu_count() or 1)


def centred_labels(n: int) -> np.ndarray:
    """Integer frequency labels of DFT bins 0..n-1 in the paper's centred convention."""
    m = np.arange(n)
    return np.where(m < (n + 1) // 2, m, m - n)


def fft3(f, inverse=False, workers=None):
    w = WORKERS if workers is None else workers
    if inverse:
        return scipy.fft.ifftn(f, axes=(-3, -2, -1), workers=w)
    return scipy.fft.fftn(f, axes=(-3, -2, -1), workers=w)


def apply_green(C, L, tau_hat, eps_star_dc, bc=0, planes=None):
    """eps_hat from tau_hat on the full complex spectrum, plane by plane in z
    (``planes``: optional subset of z planes to evaluate, for timing samples)."""
    n = tau_hat.shape[-1]
    lab = centred_labels(n)
    two_pi_L = 2.0 * np.pi / L
    ky, kx = np.meshgrid(lab, lab, indexing="ij")
    eps_hat = np.empty_like(tau_hat)
    for iz in range(n) if planes is None else planes:
        kz = lab[iz]
        xi = two_pi_L * np.stack([kx, ky, np.full_like(kx, kz)], axis=-1).astype(np.float64)
        zero = (kx == 0) & (ky == 0) & (kz == 0)
        xi_safe = np.where(zero[..., None], 1.0, xi)
        G = gamma_hat(C, xi_safe)  # (n, n, 3, 3, 3, 3) over (y, x)
        eps_hat[:, :, iz] = np.einsum("yxijkl,klyx->ijyx", G, tau_hat[:, :, iz])
        if kz == 0:
            eps_hat[:, :, iz, 0, 0] = eps_star_dc if bc == 0 else 0.0
    return eps_hat


def solve_field(C, L, eps_star, bc=0, return_hat=False):
    """(eps, sigma) for a (3, 3, n, n, n) eigenstrain field eps* in a periodic cell."""
    tau = np.einsum("ijkl,kl...->ij...", C, eps_star)
    tau_hat = fft3(tau)
    del tau
    dc = eps_star.sum(axis=(-3, -2, -1))  # DFT(eps*) at xi = 0
    eps_hat = apply_green(C, L, tau_hat, dc, bc)
    del tau_hat
    eps_c = fft3(eps_hat, inverse=True)
    eps = eps_c.real.copy()
    imag = float(np.max(np.abs(eps_c.imag)))
    del eps_c
    sig = np.einsum("ijkl,kl...->ij...", C, eps - eps_star)
    if return_hat:
        return eps, sig, imag, eps_hat
    return eps, sig, imag
