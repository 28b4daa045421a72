"""Stored defect-type fields translated by the shift theorem (oracle; test
infrastructure only).

Sec. 3.3: the field of a defect of a given type is computed once at a
reference position X0 and, for the defect at X, translated instead of solved
again; the translation is a phase factor on the stored Fourier transform
(eq. ``shift``, read as F[f(. - d)](xi) = exp(-i xi . d) F[f](xi), the printed
equation mixing x and xi).  The energy of the translated defect with a stress
field then follows the interaction-energy form of Sec. 3.3 (the eigenstrain of
the defect contracted with the others' stress, the reading used by the energy
module).

Readings:

* d = X - X0 is any real offset; whole-voxel offsets make the translation an
  exact cyclic shift of the voxel field, other offsets give its trigonometric
  interpolation (the discrete field is band limited to the grid's labels);
* labels are the centred ones of Sec. 3.4 (``solve.centred_labels``: -n/2 at an
  even n's Nyquist bin), the transform is the full complex one and the
  translated field is the real part of its inverse, as for the solve: at an
  even n's Nyquist bins this averages the phase over the two representatives
  -n/2 and +n/2 of every Nyquist component;
* the energy of a defect of type t at X with the field sigma is
  E = -h^3 c sum_x eps*_t(x - d) : sigma_others(x), where sigma_others is sigma
  minus, optionally, the type's own stress translated to X_excl (the moving
  defect itself, when sigma holds it at X_excl).

Every function takes the plain definition: a full 3-D transform, a phase per
bin, an inverse transform and a voxel sum.
"""
from __future__ import annotations

import numpy as np

from . import elastic, raster, solve


def translate(f: np.ndarray, d, L: float) -> np.ndarray:
    """f(x - d) for a real periodic field f[..., z, y, x] on a cube of side L."""
    n = f.shape[-1]
    lab = solve.centred_labels(n).astype(np.float64)
    two_pi_L = 2.0 * np.pi / L
    dx, dy, dz = (float(v) for v in d)
    ph = np.exp(
        -1j
        * two_pi_L
        * (lab[:, None, None] * dz + lab[None, :, None] * dy + lab[None, None, :] * dx)
    )
    fh = solve.fft3(f)
    return np.real(solve.fft3(fh * ph, inverse=True))


def type_fields(problem, proto):
    """(eps*_0, sigma_0, X0): the eigenstrain and stress of the prototype alone
    at its own centre X0, full (3, 3, n, n, n) tensors."""
    fps, Es = raster.rasterise(problem, proto)
    es0 = raster.eigenstrain_field(problem.n, fps, Es)
    _, sig0, _ = solve.solve_field(elastic.stiffness_of(problem), problem.L, es0, problem.bc)
    return es0, sig0, np.asarray(proto["c"][0], dtype=np.float64)


def type_energies(problem, proto, X, sigma, X_excl=None):
    """E_p for the prototype (a one-record defect array) translated to each
    position X[p] (nm), with the stress field sigma (3, 3, n, n, n)."""
    es0, sig0, X0 = type_fields(problem, proto)
    h3c = problem.h**3 * elastic.GPA_NM3_EV
    others = sigma
    if X_excl is not None:
        others = sigma - translate(sig0, np.asarray(X_excl, dtype=np.float64) - X0, problem.L)
    out = []
    for Xp in np.atleast_2d(np.asarray(X, dtype=np.float64)):
        esX = translate(es0, Xp - X0, problem.L)
        out.append(-h3c * float(np.sum(esX * others)))
    return np.array(out)
