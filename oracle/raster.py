"""Defects to eigenstrain fields on the periodic voxel grid (oracle; test infrastructure only).

Sec. 3.4: the cell is split into n^3 equal voxels with centres at
x_k = h (1/2 + m_k), h = L/n, and fields are sampled at voxel centres.
Sec. 3.1: a dislocation loop carries the eigenstrain sym(b x n)/e inside the
slab of thickness e obtained by extruding the loop area symmetrically along its
normal n (the paper's limit e -> 0 is taken at e = one voxel); point-defect
clusters carry a dilatational eigenstrain in a small region (read here as
eps* = v I inside a sphere).

Readings (the paper is silent on the discretisation of these shapes):

* membership is decided at voxel centres, in exact integer arithmetic on
  coordinates quantised to q = h/1024:  c_q = rint(c * s), s = (1024 n)/L,
  R2_q = rint((R s)^2), thickness e_q = rint(e s) (e = 0 means one voxel,
  e_q = 1024);
* the displacement d from the defect centre is the minimum image in
  [-L/2, L/2) per axis (periodic cell);
* the habit normal must be parallel to a small-integer lattice vector m
  (n_hat = m/|m|); slab: -e/2 <= d.n_hat < e/2 (half open); disk: in-plane
  distance <= R (closed); sphere: |d| <= R (closed);
* the loop eigenstrain is sym(b x n_hat)/e, not renormalised to the discrete
  footprint; the sphere eigenstrain is v I;
* the eigenstrain field is the sum of all defects' contributions (overlaps add).
"""
from __future__ import annotations

import math
import numpy as np

KIND_LOOP = 0
KIND_SPHERE = 1
QSUB = 1024  # quantisation steps per voxel edge


class DefectError(ValueError):
    pass


def lattice_normal(normal) -> np.ndarray:
    """Smallest integer vector parallel to ``normal`` (components up to 8)."""
    v = np.asarray(normal, dtype=np.float64)
    amax = float(np.max(np.abs(v)))
    if not np.isfinite(amax) or amax == 0.0:
        raise DefectError("zero or non-finite habit normal")
    a = v / amax
    for k in range(1, 9):
        w = a * k
        r = np.rint(w)
        if np.all(np.abs(w - r) < 1e-9):
            m = r.astype(np.int64)
            g = math.gcd(math.gcd(abs(int(m[0])), abs(int(m[1]))), abs(int(m[2])))
            return m // g
    raise DefectError("habit normal is not a small-integer lattice direction")


def quantise(problem, d):
    """Integer description of one defect record; raises DefectError if invalid."""
    n, L = problem.n, problem.L
    s = (1024.0 * n) / L
    Lq = QSUB * n
    kind = int(d["kind"])
    R = float(d["radius"])
    if not (R > 0.0) or not np.isfinite(R):
        raise DefectError("radius must be positive")
    cq = np.array([int(np.rint(float(ck) * s)) % Lq for ck in d["c"]], dtype=np.int64)
    Rs = R * s
    R2q = int(np.rint(Rs * Rs))
    out = {"kind": kind, "cq": cq, "R2q": R2q, "Lq": Lq, "n": n}
    if kind == KIND_LOOP:
        b = np.asarray(d["b"], dtype=np.float64)
        if float(b @ b) == 0.0:
            raise DefectError("zero Burgers vector")
        e = float(d["thickness"])
        if e < 0.0:
            raise DefectError("negative thickness")
        if e == 0.0:
            eq, e_nm = QSUB, L / n
        else:
            eq, e_nm = int(np.rint(e * s)), e
            if eq <= 0:
                raise DefectError("thickness below quantisation step")
        if R + 0.5 * e_nm >= 0.5 * L:
            raise DefectError("loop extent reaches half the cell")
        m = lattice_normal(d["normal"])
        out.update(m=m, eq=eq, e_nm=e_nm, b=b)
    elif kind == KIND_SPHERE:
        if R >= 0.5 * L:
            raise DefectError("sphere extent reaches half the cell")
        out.update(v=float(d["eig_v"]))
    else:
        raise DefectError("unknown defect kind")
    return out


def eigenstrain_tensor(qd) -> np.ndarray:
    """Constant 3x3 eigenstrain of one defect (Sec. 3.1)."""
    if qd["kind"] == KIND_SPHERE:
        return qd["v"] * np.eye(3)
    m = qd["m"].astype(np.float64)
    nhat = m / math.sqrt(float(m @ m))
    b = qd["b"]
    return (np.outer(b, nhat) + np.outer(nhat, b)) / (2.0 * qd["e_nm"])


def _axis_range(c, ext, n):
    # voxels m with |1024 m + 512 - c| <= ext (before wrapping), at most n of them
    lo = -((-(c - ext - 512)) // QSUB)
    hi = (c + ext - 512) // QSUB
    width = min(hi - lo + 1, n)
    return (np.arange(lo, lo + width) % n).astype(np.int64)


def footprint(qd) -> np.ndarray:
    """Sorted linear ids ((z n + y) n + x) of the voxels whose centre is inside."""
    n, Lq, cq, R2q = qd["n"], qd["Lq"], qd["cq"], qd["R2q"]
    ext = math.isqrt(R2q) + 1
    if qd["kind"] == KIND_LOOP:
        ext += (qd["eq"] + 1) // 2
    ax = [_axis_range(int(cq[k]), ext, n) for k in range(3)]
    mz, my, mx = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    mvox = [mx.ravel(), my.ravel(), mz.ravel()]
    dd = [((QSUB * mvox[k] + 512 - cq[k] + Lq // 2) % Lq) - Lq // 2 for k in range(3)]
    d2 = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]
    if qd["kind"] == KIND_SPHERE:
        inside = d2 <= R2q
    else:
        m = qd["m"]
        mm = int(m @ m)
        t = m[0] * dd[0] + m[1] * dd[1] + m[2] * dd[2]
        lim = qd["eq"] * qd["eq"] * mm
        slab = np.where(t >= 0, 4 * t * t < lim, 4 * t * t <= lim)
        disk = mm * d2 - t * t <= mm * R2q
        inside = slab & disk
    ids = (mvox[2] * n + mvox[1]) * n + mvox[0]
    return np.sort(ids[inside])


def rasterise(problem, defects):
    """(footprints, eigenstrain tensors) for every defect, in input order."""
    qds = [quantise(problem, d) for d in defects]
    return [footprint(q) for q in qds], [eigenstrain_tensor(q) for q in qds]


def eigenstrain_field(n, footprints, tensors, select=None) -> np.ndarray:
    """eps*(x) = sum_i E_i chi_i(x) as a (3, 3, n, n, n) [z, y, x] float64 field."""
    f = np.zeros((3, 3, n * n * n))
    idx = range(len(footprints)) if select is None else select
    for i in idx:
        f[:, :, footprints[i]] += tensors[i][:, :, None]
    return f.reshape(3, 3, n, n, n)
