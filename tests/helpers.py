"""Shared test helpers: layout conversions and tolerance checks (no method arithmetic)."""
import numpy as np

# 6-vector component order of the HIP path: xx, yy, zz, yz, xz, xy
PAIRS = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


def to6(t):
    """(3, 3, ...) symmetric tensor field -> (6, ...) tensor components."""
    return np.stack([t[i, j] for i, j in PAIRS])


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def rel_max(a, b):
    """Largest pointwise difference over the largest reference magnitude (a
    local error that a whole-field L2 norm would dilute)."""
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


def energy_ok_fp32(E, Eref):
    """Per-defect FP32 criterion: |E - Eref| <= max(1e-4 |Eref|, 1e-5 eV)."""
    return np.abs(E - Eref) <= np.maximum(1e-4 * np.abs(Eref), 1e-5)


def energy_ok_fp64(E, Eref, rtol=1e-10):
    """Normwise FP64 criterion: max |E - Eref| <= rtol * max |Eref|."""
    return float(np.max(np.abs(E - Eref))) <= rtol * float(np.max(np.abs(Eref)))
