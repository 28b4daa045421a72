"""Seeded synthetic workloads: problem descriptors and defect populations.

This module only draws random numbers and packs them into the record layout
that the C ABI (``include/ec.h``) takes.  It holds none of the method's
arithmetic: no quantisation, no membership tests, no eigenstrain, no Green
operator.  Both the FP64 oracle and the HIP path consume its output.

Workload recipes (defect populations in a cubic-iron-like crystal):

* ``pair_32``: 32^3 voxels, 10 nm box, isotropic E=210 GPa, nu=0.29; one
  dilatational sphere (R = 3 voxels, eps* = 0.01 I) at a voxel centre and one
  1/2[111] interstitial loop (a = 0.2866 nm, R = 4 voxels, (111) habit, one voxel
  thick) displaced by a seeded integer voxel offset of norm >= 8.
* ``loops_128``: 128^3, 40 nm, cubic C11/C12/C44 = 243/145/116 GPa; 200 1/2<111>
  loops, centres uniform, R ~ U[1, 4] nm, Burgers vector uniform over the four
  1/2<111> variants, habit normal parallel to b.
* ``mixed_256``: 256^3, 80 nm, same C; 2000 defects: 70 % 1/2<111> loops
  (R log-uniform in [0.5, 5] nm), 10 % <100> loops (b = a e_k, R ~ U[1, 6] nm),
  20 % dilatational spheres (R ~ U[1, 3] voxels, eps* = v I, v ~ U[0.005, 0.02]).
* ``serving_replicas``: n ~ U{64, 96, 128, 160, 240}, L = n h with
  h = 0.3125 nm, 50-1500 defects drawn as in mixed_256.
* ``mixed_512``: 512^3, 160 nm; 20000 defects as mixed_256 but 1/2<111> R
  log-uniform in [0.5, 8] nm and <100> R ~ U[1, 8] nm.
* ``glide_jumps``: the candidate jumps of the jump-probe workload, one voxel
  forward and back along each defect's Burgers-vector sign pattern.

Seeds: ``numpy.random.default_rng(240309158 + k)`` with k = 1, 2, 3, 5 for the
four fixed workloads above (pair_32 to mixed_512), 40 + r for serving replica r
and 400 for the serving arrivals.
"""
from __future__ import annotations

import dataclasses
import numpy as np

A_FE = 0.2866  # nm, bcc iron lattice parameter used for Burgers vectors
H_VOXEL = 0.3125  # nm, voxel edge shared by every workload below
SEED_BASE = 240309158

KIND_LOOP = 0
KIND_SPHERE = 1

# Layout-compatible with ``ec_defect`` in include/ec.h (104 bytes, 8-aligned).
DEFECT_DTYPE = np.dtype(
    [
        ("kind", "<i4"),
        ("_pad", "<i4"),
        ("c", "<f8", (3,)),
        ("radius", "<f8"),
        ("b", "<f8", (3,)),
        ("normal", "<f8", (3,)),
        ("thickness", "<f8"),
        ("eig_v", "<f8"),
    ],
    align=True,
)
assert DEFECT_DTYPE.itemsize == 104

# Layout-compatible with ``ec_line`` in include/ec.h (56 bytes): an infinite
# straight dislocation line along a cell axis.
LINE_DTYPE = np.dtype(
    [("p", "<f8", (3,)), ("axis", "<i4"), ("sense", "<i4"), ("b", "<f8", (3,))],
    align=True,
)
assert LINE_DTYPE.itemsize == 56


def line(p, axis, sense, b):
    rec = np.zeros(1, dtype=LINE_DTYPE)
    rec["p"] = p
    rec["axis"] = axis
    rec["sense"] = sense
    rec["b"] = b
    return rec


CUBIC_FE = (243.0, 145.0, 116.0)

# The four 1/2<111> Burgers-vector variants (b and -b describe the same loop).
B111 = np.array([[1, 1, 1], [-1, 1, 1], [1, -1, 1], [1, 1, -1]], dtype=np.float64)


@dataclasses.dataclass(frozen=True)
class Problem:
    """Periodic cubic cell of n^3 voxels and side L (nm), cubic stiffness (GPa)."""

    n: int
    L: float
    C11: float
    C12: float
    C44: float
    prec: int = 0  # 0 = FP64, 1 = FP32 storage
    bc: int = 0  # 0 = mean stress zero, 1 = mean strain zero
    nyq: int = 0  # 0 = paper-literal even-N Nyquist rule
    frame: tuple = ()  # 9 numbers, rows = cell axes in cube coordinates; () = cube axes

    @property
    def h(self) -> float:
        return self.L / self.n

    def with_(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def isotropic_C(E: float, nu: float):
    """(C11, C12, C44) of an isotropic solid from Young's modulus and Poisson ratio."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam + 2.0 * mu, lam, mu


def empty_defects(k: int) -> np.ndarray:
    return np.zeros(k, dtype=DEFECT_DTYPE)


def loop(c, radius, b, normal, thickness=0.0):
    d = empty_defects(1)
    d["kind"] = KIND_LOOP
    d["c"] = c
    d["radius"] = radius
    d["b"] = b
    d["normal"] = normal
    d["thickness"] = thickness
    return d


def sphere(c, radius, v):
    d = empty_defects(1)
    d["kind"] = KIND_SPHERE
    d["c"] = c
    d["radius"] = radius
    d["eig_v"] = v
    return d


def _rng(k: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + k)


def pair_32(seed_offset: int = 0):
    """Two defects in a 32^3 isotropic cell (plain FP64 case)."""
    rng = _rng(1 + seed_offset)
    n, L = 32, 10.0
    h = L / n
    prob = Problem(n, L, *isotropic_C(210.0, 0.29))
    centre = np.array([16.5, 16.5, 16.5]) * h  # a voxel centre
    while True:
        off = rng.integers(-10, 11, size=3)
        if off @ off >= 64:
            break
    b = 0.5 * A_FE * np.array([1.0, 1.0, 1.0])
    defs = np.concatenate(
        [
            sphere(centre, 3.0 * h, 0.01),
            loop(centre + off * h, 4.0 * h, b, b),
        ]
    )
    return prob, defs


def _loops111(rng, k, L, rmin, rmax, log_uniform):
    d = empty_defects(k)
    d["kind"] = KIND_LOOP
    d["c"] = rng.uniform(0.0, L, size=(k, 3))
    if log_uniform:
        d["radius"] = np.exp(rng.uniform(np.log(rmin), np.log(rmax), size=k))
    else:
        d["radius"] = rng.uniform(rmin, rmax, size=k)
    var = rng.integers(0, 4, size=k)
    b = 0.5 * A_FE * B111[var]
    d["b"] = b
    d["normal"] = b
    return d


def _loops100(rng, k, L, rmin, rmax):
    d = empty_defects(k)
    d["kind"] = KIND_LOOP
    d["c"] = rng.uniform(0.0, L, size=(k, 3))
    d["radius"] = rng.uniform(rmin, rmax, size=k)
    ax = rng.integers(0, 3, size=k)
    b = np.zeros((k, 3))
    b[np.arange(k), ax] = A_FE
    d["b"] = b
    d["normal"] = b
    return d


def _spheres(rng, k, L, h):
    d = empty_defects(k)
    d["kind"] = KIND_SPHERE
    d["c"] = rng.uniform(0.0, L, size=(k, 3))
    d["radius"] = rng.uniform(1.0, 3.0, size=k) * h
    d["eig_v"] = rng.uniform(0.005, 0.02, size=k)
    return d


def mixed_population(rng, ndef, L, h, r111=(0.5, 5.0), r100=(1.0, 6.0)):
    """70 % 1/2<111> loops, 10 % <100> loops, 20 % dilatational spheres, shuffled."""
    n111 = int(round(0.7 * ndef))
    n100 = int(round(0.1 * ndef))
    nsph = ndef - n111 - n100
    parts = [
        _loops111(rng, n111, L, r111[0], r111[1], log_uniform=True),
        _loops100(rng, n100, L, r100[0], r100[1]),
        _spheres(rng, nsph, L, h),
    ]
    d = np.concatenate(parts)
    return d[rng.permutation(ndef)]


def loops_128(prec: int = 0):
    rng = _rng(2)
    n, L = 128, 40.0
    prob = Problem(n, L, *CUBIC_FE, prec=prec)
    return prob, _loops111(rng, 200, L, 1.0, 4.0, log_uniform=False)


def paper_129(prec: int = 1):
    """The odd grid of the paper's simulations (Sec. 4: 129^3 voxels in a cube
    of 500 a0, cube axes here), with 300 defects mixed as in mixed_256 and
    loop radii of 1.5-6 nm (1.4-5.4 voxels)."""
    rng = _rng(129)
    n = 129
    L = 500.0 * A_FE
    prob = Problem(n, L, *CUBIC_FE, prec=prec)
    return prob, mixed_population(rng, 300, L, L / n, r111=(1.5, 6.0), r100=(2.0, 6.0))


def mixed_256(prec: int = 1):
    rng = _rng(3)
    n, L = 256, 80.0
    prob = Problem(n, L, *CUBIC_FE, prec=prec)
    return prob, mixed_population(rng, 2000, L, L / n)


def mixed_512(prec: int = 1):
    rng = _rng(5)
    n, L = 512, 160.0
    prob = Problem(n, L, *CUBIC_FE, prec=prec)
    return prob, mixed_population(rng, 20000, L, L / n, r111=(0.5, 8.0), r100=(1.0, 8.0))


def scaled_mixed(n: int, prec: int = 1, seed: int = 0):
    """The mixed_256 defect density and size mix in an n^3 cell with h = 0.3125 nm."""
    rng = np.random.default_rng(SEED_BASE + 300 + seed)
    L = n * H_VOXEL
    ndef = max(2, int(round(2000 * (n / 256.0) ** 3)))
    prob = Problem(n, L, *CUBIC_FE, prec=prec)
    r111 = (0.5, min(5.0, 0.4 * L))
    r100 = (1.0, min(6.0, 0.4 * L))
    return prob, mixed_population(rng, ndef, L, L / n, r111=r111, r100=r100)


REPLICA_SIZES = (64, 96, 128, 160, 240)


def serving_replicas(nrep: int = 64, prec: int = 1):
    """Per-replica (problem, defects) for the serving workload."""
    out = []
    for r in range(nrep):
        rng = np.random.default_rng(SEED_BASE + 40 + r)
        n = int(rng.choice(REPLICA_SIZES))
        L = n * H_VOXEL
        ndef = int(rng.integers(50, 1501))
        prob = Problem(n, L, *CUBIC_FE, prec=prec)
        out.append((prob, mixed_population(rng, ndef, L, H_VOXEL)))
    return out


# Crystal orientation of the paper's simulations (Sec. 4): cell x, y, z along
# [111], [-1-12], [1-10] (rows: unit vectors in cube coordinates).
FRAME_111 = tuple(
    np.concatenate(
        [
            np.array([1.0, 1.0, 1.0]) / np.sqrt(3.0),
            np.array([-1.0, -1.0, 2.0]) / np.sqrt(6.0),
            np.array([1.0, -1.0, 0.0]) / np.sqrt(2.0),
        ]
    ).tolist()
)


HOPS111 = np.array(
    [[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], dtype=np.int64
)


def serving_trace(nrep: int, nreq: int, rate_per_s: float = 2000.0, update_frac: float = 0.9):
    """Poisson arrival trace: (t_arrival, replica, op, defect_slot_draw, hop_index)."""
    rng = np.random.default_rng(SEED_BASE + 400)
    gaps = rng.exponential(1.0 / rate_per_s, size=nreq)
    t = np.cumsum(gaps)
    rep = rng.integers(0, nrep, size=nreq)
    is_update = rng.random(nreq) < update_frac
    draw = rng.random(nreq)
    hop = rng.integers(0, 8, size=nreq)
    return t, rep, is_update, draw, hop


def glide_jumps(defects) -> np.ndarray:
    """Candidate jumps of the jump-probe workload: per defect one voxel forward
    and back along the sign pattern of its Burgers vector (the glide direction
    of a loop: (+-1, +-1, +-1) for 1/2<111>, (+-1, 0, 0) and the like for
    <100>), along x for a sphere.  Shape (ndef, 2, 3), int32 voxel offsets."""
    d = np.asarray(defects)
    out = np.zeros((len(d), 2, 3), dtype=np.int32)
    for i, rec in enumerate(d):
        v = np.sign(np.round(rec["b"], 12)).astype(np.int32)
        if not v.any():
            v = np.array([1, 0, 0], dtype=np.int32)
        out[i, 0], out[i, 1] = v, -v
    return out
