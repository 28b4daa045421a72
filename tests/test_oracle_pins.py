"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test checks the oracle against a closed form, an identity of the
mathematics, a brute-force evaluation or a value printed in the paper, chosen
so that a dropped term, a wrong sign or index, or a transposed operand in the
oracle fails at least one of them.
"""
import itertools
import json
import math
import os
from decimal import ROUND_FLOOR, Decimal, getcontext

import numpy as np
import pytest

from oracle import elastic, energy, raster, solve
from paper_2403_09158_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(20240309)


def _rand_xi(k=50):
    return RNG.normal(size=(k, 3))


def _sym(a):
    return 0.5 * (a + np.swapaxes(a, 0, 1))


# ----------------------------------------------------------------------------- FFT


@pytest.mark.parametrize("n", [6, 8, 10, 12, 15])
def test_fft_matches_brute_force_dft(n):
    """The library FFT the oracle calls equals the DFT written as a plain sum."""
    f = RNG.normal(size=(n, n, n)) + 1j * RNG.normal(size=(n, n, n))
    m = np.arange(n)
    z, y, x = np.meshgrid(m, m, m, indexing="ij")
    pos = np.stack([z.ravel(), y.ravel(), x.ravel()], axis=1)
    phase = -2j * np.pi * (pos @ pos.T) / n  # k . x over every (k, x) pair
    F = (np.exp(phase) @ f.ravel()).reshape(n, n, n)
    got = solve.fft3(f)
    assert np.max(np.abs(got - F)) <= 1e-13 * np.max(np.abs(F)) * n
    back = solve.fft3(F, inverse=True)
    assert np.max(np.abs(back - f)) <= 1e-13 * np.max(np.abs(f)) * n


def test_centred_labels():
    assert list(solve.centred_labels(8)) == [0, 1, 2, 3, -4, -3, -2, -1]
    assert list(solve.centred_labels(7)) == [0, 1, 2, 3, -3, -2, -1]


# ---------------------------------------------------------------- Green operator


def test_gamma_general_equals_isotropic_closed_form():
    lam, mu = 112.4, 81.4
    xi = _rand_xi()
    a = elastic.gamma_hat(elastic.isotropic_stiffness(lam, mu), xi)
    b = elastic.gamma_isotropic(lam, mu, xi)
    assert np.max(np.abs(a - b)) < 1e-15


def test_table1_isotropisation_and_units():
    """Table 1: E_iso, nu_iso from C11, C12 at Zener ratio 1; dV = tr P / 3K."""
    g = json.load(open(os.path.join(GOLDEN, "table1_fe.json")))
    C11, C12 = g["C11_GPa"], g["C12_GPa"]
    C44 = 0.5 * (C11 - C12)
    E_iso = (C11 - C12) * (C11 + 2 * C12) / (C11 + C12)
    nu_iso = C12 / (C11 + C12)
    tol = g["printed_precision"]
    assert abs(E_iso - g["E_iso_GPa"]) <= tol["E_iso_GPa"]
    assert abs(nu_iso - g["nu_iso"]) <= tol["nu_iso"]
    # the cubic Green operator at Zener ratio 1 is the isotropic closed form
    lam = E_iso * nu_iso / ((1 + nu_iso) * (1 - 2 * nu_iso))
    mu = E_iso / (2 * (1 + nu_iso))
    xi = _rand_xi()
    a = elastic.gamma_hat(elastic.cubic_stiffness(C11, C12, C44), xi)
    b = elastic.gamma_isotropic(lam, mu, xi)
    assert np.max(np.abs(a - b)) < 1e-15
    # relaxation volume tr(P)/(3K): pins the GPa*volume -> eV constant
    P = g["P_eV"]
    trP = P["11"] + P["22"] + P["33"]
    K = (C11 + 2 * C12) / 3.0
    dV = trP / (3.0 * K * elastic.GPA_NM3_EV * 1e-3)  # eV / (eV per A^3)
    assert abs(dV / g["V_at_A3"] - g["dV_over_Vat"]) <= tol["dV_over_Vat"]


@pytest.mark.parametrize("Cs", [inputs.CUBIC_FE, (289.34, 152.34, 107.43), inputs.isotropic_C(210, 0.29)])
def test_gamma_projector_symmetry_degree0(Cs):
    C = elastic.cubic_stiffness(*Cs)
    xi = _rand_xi()
    G = elastic.gamma_hat(C, xi)
    GCG = np.einsum("...ijkl,klmn,...mnpq->...ijpq", G, C, G)
    tol = 1e-14 * np.max(np.abs(G))
    assert np.max(np.abs(GCG - G)) < tol
    assert np.max(np.abs(G - np.swapaxes(G, -4, -3))) < tol  # minor (ij)
    assert np.max(np.abs(G - np.swapaxes(G, -2, -1))) < tol  # minor (kl)
    assert np.max(np.abs(G - np.transpose(G, (0, 3, 4, 1, 2)))) < tol  # major
    assert np.max(np.abs(elastic.gamma_hat(C, -xi) - G)) < tol  # even
    assert np.max(np.abs(elastic.gamma_hat(C, 3.7 * xi) - G)) < tol  # degree 0


def test_gamma_solves_equilibrium_per_frequency():
    """xi_j C_ijkl (Gamma:tau)_kl = xi_j tau_ij for symmetric tau."""
    C = elastic.cubic_stiffness(*inputs.CUBIC_FE)
    xi = _rand_xi()
    tau = RNG.normal(size=(len(xi), 3, 3))
    tau = 0.5 * (tau + np.swapaxes(tau, 1, 2))
    eps = np.einsum("aijkl,akl->aij", elastic.gamma_hat(C, xi), tau)
    lhs = np.einsum("aj,ijkl,akl->ai", xi, C, eps)
    rhs = np.einsum("aj,aij->ai", xi, tau)
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(rhs))


# ------------------------------------------------------------------- the solve


def _random_field(n, k=12, seed=0):
    rng = np.random.default_rng(seed)
    f = np.zeros((3, 3, n, n, n))
    for _ in range(k):
        z, y, x = rng.integers(0, n, size=3)
        a = rng.normal(size=(3, 3)) * 0.01
        f[:, :, z, y, x] += 0.5 * (a + a.T)
    return f


def _xi_grid(n, L):
    lab = solve.centred_labels(n)
    kz, ky, kx = np.meshgrid(lab, lab, lab, indexing="ij")
    return 2 * np.pi / L * np.stack([kx, ky, kz], axis=0), (kx, ky, kz)


@pytest.mark.parametrize("n", [9, 10])
@pytest.mark.parametrize("bc", [0, 1])
def test_solve_invariants(n, bc):
    """Equilibrium, compatibility and the mean condition of the periodic solution."""
    L = 3.1
    C = elastic.cubic_stiffness(*inputs.CUBIC_FE)
    es = _random_field(n, seed=n + 10 * bc)
    eps, sig, imag = solve.solve_field(C, L, es, bc)
    xi, (kx, ky, kz) = _xi_grid(n, L)
    nyq = (n % 2 == 0) & ((np.abs(kx) == n // 2) | (np.abs(ky) == n // 2) | (np.abs(kz) == n // 2))
    ok = ~nyq if n % 2 == 0 else np.ones_like(kx, dtype=bool)
    sh = solve.fft3(sig)
    eh = solve.fft3(eps)
    div = np.einsum("jzyx,ijzyx->izyx", xi, sh)
    assert np.max(np.abs(div[:, ok])) < 1e-12 * np.max(np.abs(sh)) * np.max(np.abs(xi))
    lc = np.zeros((3, 3, 3))
    for i, j, k in itertools.permutations(range(3)):
        lc[i, j, k] = np.linalg.det(np.eye(3)[[i, j, k]])
    inc = np.einsum("ikm,jln,kzyx,lzyx,mnzyx->ijzyx", lc, lc, xi, xi, eh)
    assert np.max(np.abs(inc[:, :, ok])) < 1e-12 * np.max(np.abs(eh)) * np.max(np.abs(xi)) ** 2
    if bc == 0:
        assert np.max(np.abs(sig.mean(axis=(2, 3, 4)))) < 1e-14 * np.max(np.abs(sig))
    else:
        assert np.max(np.abs(eps.mean(axis=(2, 3, 4)))) < 1e-15 * np.max(np.abs(eps)) * n**3
    if n % 2 == 1:
        assert imag < 1e-13 * np.max(np.abs(eps))


def test_nyquist_reading_equals_two_representative_average():
    """Real part of the full-complex solve == half-spectrum solve with the
    Green operator averaged over the all-minus and all-plus Nyquist labels."""
    n, L = 8, 2.5
    C = elastic.cubic_stiffness(*inputs.CUBIC_FE)
    es = _random_field(n, k=20, seed=3)
    eps, _, imag = solve.solve_field(C, L, es, 0)
    assert imag > 1e-6 * np.max(np.abs(eps))  # the Nyquist bins do break Hermitian symmetry
    tau = np.einsum("ijkl,kl...->ij...", C, es)
    th = np.fft.rfftn(tau, axes=(2, 3, 4))
    lab = solve.centred_labels(n)
    out = np.zeros_like(th)
    for iz, iy, ix in itertools.product(range(n), range(n), range(n // 2 + 1)):
        k = np.array([ix, lab[iy], lab[iz]], dtype=float)
        if ix == 0 and lab[iy] == 0 and lab[iz] == 0:
            out[:, :, 0, 0, 0] = es.sum(axis=(2, 3, 4))
            continue
        isn = np.array([ix == n // 2, abs(lab[iy]) == n // 2, abs(lab[iz]) == n // 2])
        km, kp = k.copy(), k.copy()
        km[isn] = -n // 2
        kp[isn] = n // 2
        G = 0.5 * (elastic.gamma_hat(C, 2 * np.pi / L * km) + elastic.gamma_hat(C, 2 * np.pi / L * kp))
        out[:, :, iz, iy, ix] = np.einsum("ijkl,kl->ij", G, th[:, :, iz, iy, ix])
    e2 = np.fft.irfftn(out, s=(n, n, n), axes=(2, 3, 4))
    assert np.max(np.abs(e2 - eps)) < 1e-14 * np.max(np.abs(eps)) * 10


# --------------------------------------------------- isotropic dilatation closed forms


def _disjoint_sets(n, sizes, seed):
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n**3)
    out, o = [], 0
    for s in sizes:
        out.append(np.sort(perm[o : o + s]))
        o += s
    return out


@pytest.mark.parametrize("bc", [0, 1])
def test_isotropic_dilatation_closed_forms(bc):
    """Trace field, self energy and pair energy of dilatational inclusions of any shape."""
    Ey, nu = 210.0, 0.29
    n, L = 12, 4.0
    prob = inputs.Problem(n, L, *inputs.isotropic_C(Ey, nu), bc=bc)
    h = L / n
    V = L**3
    sets = _disjoint_sets(n, [17, 40, 5], seed=bc)
    es = [0.01, -0.02, 0.013]
    Es = [e * np.eye(3) for e in es]
    C = elastic.stiffness_of(prob)
    field = raster.eigenstrain_field(n, sets, Es)
    eps, sig, _ = solve.solve_field(C, L, field, bc)
    f = [len(s) / n**3 for s in sets]
    chi = [np.isin(np.arange(n**3), s).reshape(n, n, n) for s in sets]
    tr_mean = 3 * sum(e * fk for e, fk in zip(es, f)) if bc == 0 else 0.0
    expect = (1 + nu) / (1 - nu) * sum(e * (c - fk) for e, c, fk in zip(es, chi, f)) + tr_mean
    got = eps[0, 0] + eps[1, 1] + eps[2, 2]
    assert np.max(np.abs(got - expect)) < 1e-15 * 50
    Eb, Eij = energy.energies_brute_fp(prob, sets, Es, bc)
    c = elastic.GPA_NM3_EV
    for a in range(3):
        Va = len(sets[a]) * h**3
        fa = Va / V
        if bc == 0:
            w = Ey / (1 - nu) * es[a] ** 2 * Va * (1 - fa)
        else:
            w = Ey / (1 - nu) * es[a] ** 2 * Va * (1 + fa * (1 + nu) / (2 * (1 - 2 * nu)))
        assert abs(0.5 * Eij[a, a] - w * c) < 1e-12 * abs(w * c)  # W_self = B/2 = E_aa/2
        for b in range(3):
            if a == b:
                continue
            Vb = len(sets[b]) * h**3
            if bc == 0:
                p = -(2 * Ey / (1 - nu)) * es[a] * es[b] * Va * Vb / V
            else:
                p = Ey * (1 + nu) / ((1 - nu) * (1 - 2 * nu)) * es[a] * es[b] * Va * Vb / V
            assert abs(Eij[a, b] - p * c) < 1e-12 * abs(p * c)


def test_eshelby_sphere_interior_field():
    """Interior of a dilatational sphere in an isotropic medium: nearly uniform
    strain ((1+nu)/(3(1-nu))) e (1-f) + e f (mean-stress-zero cell); stress
    -(2E/(3(1-nu))) e (1-f) I.  Deviatoric part -> 0 with resolution (few %)."""
    Ey, nu, e = 210.0, 0.29, 0.01
    n = 48
    L = n * 0.3125
    prob = inputs.Problem(n, L, *inputs.isotropic_C(Ey, nu))
    h = L / n
    d = inputs.sphere(np.array([24.5, 24.5, 24.5]) * h, 8.0 * h, e)
    fps, Es = raster.rasterise(prob, d)
    eps, sig, _ = solve.solve_field(elastic.stiffness_of(prob), L, raster.eigenstrain_field(n, fps, Es))
    f = len(fps[0]) / n**3
    inner = energy.voxel_coords(fps[0], n)
    rr = np.linalg.norm(inner - 24, axis=1)
    core = fps[0][rr <= 5.0]
    ef = eps.reshape(3, 3, -1)[:, :, core]
    sf = sig.reshape(3, 3, -1)[:, :, core]
    e_in = (1 + nu) / (3 * (1 - nu)) * e * (1 - f) + e * f
    s_in = -(2 * Ey / (3 * (1 - nu))) * e * (1 - f)
    mean_e = ef.mean(axis=-1)
    mean_s = sf.mean(axis=-1)
    assert np.max(np.abs(mean_e - e_in * np.eye(3))) < 0.03 * e_in
    assert np.max(np.abs(mean_s - s_in * np.eye(3))) < 0.03 * abs(s_in)
    dev = ef - np.einsum("kkv->v", ef)[None, None] / 3 * np.eye(3)[:, :, None]
    assert np.sqrt(np.mean(dev**2)) < 0.05 * e_in  # staircase / Gibbs residue
    assert np.max(np.abs(dev)) < 0.10 * e_in


# --------------------------------------------------------------- energies


def _mixed_small(n=24, seed=0):
    rng = np.random.default_rng(seed)
    L = n * 0.3125
    h = L / n
    prob = inputs.Problem(n, L, *inputs.CUBIC_FE)
    b1 = 0.5 * inputs.A_FE * np.array([1.0, -1.0, 1.0])
    b2 = np.array([0.0, inputs.A_FE, 0.0])
    d = np.concatenate(
        [
            inputs.loop(rng.uniform(0, L, 3), 2.3 * h, b1, b1),
            inputs.loop(rng.uniform(0, L, 3), 3.1 * h, b2, b2),
            inputs.sphere(rng.uniform(0, L, 3), 1.7 * h, 0.012),
            inputs.loop(rng.uniform(0, L, 3), 1.9 * h, 0.5 * inputs.A_FE * np.array([1.0, 1, 1]), [1, 1, 1]),
        ]
    )
    # an overlapping pair
    d = np.concatenate([d, inputs.sphere(d[2]["c"] + 0.6 * h, 1.5 * h, 0.008)])
    return prob, d


@pytest.mark.parametrize("n", [24, 21])
@pytest.mark.parametrize("bc", [0, 1])
def test_brute_energies_equal_fast_exact(bc, n):
    """The windowed energies equal one solve per defect (the definition), also
    for an odd grid, whose minimum images and labels have no Nyquist case."""
    prob, d = _mixed_small(n=n)
    prob = prob.with_(bc=bc)
    Eb, Eij = energy.energies_brute(prob, d)
    Ef = energy.energies_fast(prob, d)
    assert np.max(np.abs(Eb - Ef)) <= 1e-11 * np.max(np.abs(Eb))
    # reciprocity of the pair energies (Betti)
    assert np.max(np.abs(Eij - Eij.T)) <= 1e-12 * np.max(np.abs(Eij))


def test_total_energy_identity():
    """-1/2 h^3 c sum eps*:sigma = sum_i B_i / 2 + 1/2 sum_i E_i."""
    prob, d = _mixed_small(seed=1)
    E, parts = energy.energies_fast(prob, d, return_parts=True)
    fps, Es = parts["fps"], parts["Es"]
    es = raster.eigenstrain_field(prob.n, fps, Es)
    h3c = prob.h**3 * elastic.GPA_NM3_EV
    W = -0.5 * h3c * float(np.sum(es * parts["sig"]))
    assert abs(W - (0.5 * parts["B"].sum() + 0.5 * E.sum())) < 1e-12 * abs(W)


def test_translation_and_axis_permutation_invariance():
    prob, d = _mixed_small(seed=2)
    E0 = energy.energies_fast(prob, d)
    d2 = d.copy()
    d2["c"] = d["c"] + np.array([5, -3, 11]) * prob.h  # integer voxel shift, wraps
    assert np.max(np.abs(energy.energies_fast(prob, d2) - E0)) < 1e-12 * np.max(np.abs(E0))
    d3 = d.copy()
    perm = [2, 0, 1]  # (x, y, z) -> (z, x, y): a symmetry of the cubic crystal
    for f in ("c", "b", "normal"):
        d3[f] = d[f][:, perm]
    assert np.max(np.abs(energy.energies_fast(prob, d3) - E0)) < 1e-12 * np.max(np.abs(E0))


@pytest.mark.slow
def test_dipole_limit_coaxial_111_loops():
    """E_12 -> -h^3 c |Omega_1| E_1 : sigma_2(X_1) as the separation grows (Sec. 2.1)."""
    n = 128
    L = n * 0.3125
    h = L / n
    prob = inputs.Problem(n, L, *inputs.CUBIC_FE)
    R = 2.0
    b = 0.5 * inputs.A_FE * np.array([1.0, 1.0, 1.0])
    c2 = np.array([0.5, 0.5, 0.5]) * h
    fps, Es = raster.rasterise(prob, inputs.loop(c2, R * h, b, b))
    _, sig, _ = solve.solve_field(elastic.stiffness_of(prob), L, raster.eigenstrain_field(n, fps, Es))
    sf = sig.reshape(3, 3, -1)
    h3c = h**3 * elastic.GPA_NM3_EV
    ratios = []
    for k in (5, 9, 14, 18):  # d/R = 4.3, 7.8, 12.1, 15.6 along [111]
        f1, E1 = raster.rasterise(prob, inputs.loop(c2 + k * h, R * h, b, b))
        E12 = -h3c * np.einsum("ij,ijv->", E1[0], sf[:, :, f1[0]])
        x1 = k + n * (k + n * k)
        Edip = -h3c * len(f1[0]) * np.einsum("ij,ij->", E1[0], sf[:, :, x1])
        ratios.append(E12 / Edip)
    assert all(b > a for a, b in zip(ratios, ratios[1:]))
    assert abs(ratios[2] - 1) < 0.035 and abs(ratios[3] - 1) < 0.022


# ------------------------------------------------------------------ rasteriser


def test_sphere_counts_are_lattice_ball_counts():
    g = json.load(open(os.path.join(GOLDEN, "lattice_ball_counts.json")))
    n = 40
    prob = inputs.Problem(n, n * 0.3125, *inputs.CUBIC_FE)
    h = prob.h
    for r, cnt in zip(g["r"], g["count"]):
        if r == 0:
            continue
        fps, _ = raster.rasterise(prob, inputs.sphere(np.array([7.5, 30.5, 19.5]) * h, r * h, 0.01))
        assert len(fps[0]) == cnt


def _brute_member(kind, c, R, m, e, n, vox):
    """Membership from the geometric definition in 60-digit decimal arithmetic."""
    getcontext().prec = 60
    L = Decimal(n)
    d = []
    for k in range(3):
        x = Decimal(int(vox[k])) + Decimal("0.5") - Decimal(c[k])
        x = x - L * ((x + L / 2) / L).to_integral_value(rounding=ROUND_FLOOR)  # in [-L/2, L/2)
        d.append(x)
    d2 = sum(x * x for x in d)
    Rd = Decimal(R)
    if kind == 1:
        return d2 <= Rd * Rd
    mn = Decimal(int(m[0] ** 2 + m[1] ** 2 + m[2] ** 2)).sqrt()
    s = sum(Decimal(int(m[k])) * d[k] for k in range(3)) / mn
    half = Decimal(e) / 2
    if not (-half <= s < half):
        return False
    return d2 - s * s <= Rd * Rd


@pytest.mark.parametrize("seed", range(4))
def test_raster_matches_geometric_definition(seed):
    """Integer-exact footprints == real-number geometry (h = 1, q-grid centres)."""
    rng = np.random.default_rng(seed)
    n = 12
    prob = inputs.Problem(n, float(n), *inputs.CUBIC_FE)  # h = 1 nm: q = 1/1024 exactly
    normals = [np.array([1, 1, 1]), np.array([1, -1, 1]), np.array([0, 0, 1]), np.array([1, 1, 0]), np.array([2, 1, 0])]
    for trial in range(6):
        c = rng.integers(0, n * 1024, size=3) / 1024.0
        R = rng.integers(1200, 3500) / 1024.0
        if trial % 3 == 2:
            d = inputs.sphere(c, R, 0.01)
            kind, m, e = 1, None, None
        else:
            m = normals[rng.integers(0, len(normals))]
            e = [1.0, 1.5, 0.75][trial % 3]
            d = inputs.loop(c, R, m * 0.3, m, thickness=e)
            kind = 0
        fps, _ = raster.rasterise(prob, d)
        box = np.arange(n)
        want = []
        for z, y, x in itertools.product(box, box, box):
            if _brute_member(kind, c, R, m, e, n, (x, y, z)):
                want.append((z * n + y) * n + x)
        assert list(fps[0]) == want


def test_raster_half_open_slab_and_wrap():
    n = 16
    prob = inputs.Problem(n, float(n), *inputs.CUBIC_FE)
    # <100> slab whose faces pass through voxel-centre planes x = 3.5 and 4.5:
    # the lower face is closed, the upper open -> only the x = 3 layer
    d = inputs.loop([4.0, 8.5, 8.5], 2.0, [1.0, 0, 0], [1, 0, 0])
    fps, _ = raster.rasterise(prob, d)
    xs = np.unique(energy.voxel_coords(fps[0], n)[:, 0])
    assert list(xs) == [3]
    # a sphere at a corner wraps: same shape as at the cell centre, shifted
    a, _ = raster.rasterise(prob, inputs.sphere([0.5, 0.5, 0.5], 2.5, 0.01))
    b, _ = raster.rasterise(prob, inputs.sphere([8.5, 8.5, 8.5], 2.5, 0.01))
    pa = energy.voxel_coords(a[0], n)
    pb = energy.voxel_coords(b[0], n)
    sa = sorted(map(tuple, (pa + 8) % n))
    assert sa == sorted(map(tuple, pb))


def test_raster_rejects_invalid_defects():
    prob = inputs.Problem(16, 5.0, *inputs.CUBIC_FE)
    bad = [
        inputs.sphere([1, 1, 1], 0.0, 0.01),
        inputs.sphere([1, 1, 1], 2.6, 0.01),
        inputs.loop([1, 1, 1], 1.0, [0, 0, 0], [1, 0, 0]),
        inputs.loop([1, 1, 1], 1.0, [1, 0, 0], [1, math.pi, 0]),
        inputs.loop([1, 1, 1], 2.4, [1, 0, 0], [1, 0, 0]),
    ]
    for d in bad:
        with pytest.raises(raster.DefectError):
            raster.rasterise(prob, d)


# ------------------------------------------------ loop eigenstrain amplitude (Sec. 2.1, 3.1)


@pytest.mark.parametrize(
    "family,R_vox,e_vox,n",
    [("100", 8.0, 1.0, 32), ("100", 12.5, 1.0, 32), ("100", 10.0, 2.0, 32), ("111", 8.0, math.sqrt(3.0), 32),
     ("111", 12.0, math.sqrt(3.0), 40)],
)
def test_loop_dipole_tensor_matches_the_paper(family, R_vox, e_vox, n):
    """The loop eigenstrain sym(b x n)/e of Sec. 3.1 has the dipole tensor the
    paper prints for a loop (Sec. 4.2): P = 1/2 C:(b x A + A x b), A = pi R^2 n
    its oriented area.  With <eps> = 0 (equal displacements on opposite cell
    faces) the paper's appendix gives P = -(integral of sigma over the cell), so
    the oracle's solve must return -h^3 sum_x sigma(x) = that P, up to the
    count of voxel centres in the discrete slab against its continuum volume
    (a few per cent here).  The <100> slabs hold one or two whole lattice
    planes; the (111) slab of thickness sqrt(3) h holds three planes of density
    1/(sqrt(3) h^2), i.e. sqrt(3) planes per h.  A dropped 1/2 of the symmetric
    part, a division by h instead of e or a sign error is off by a factor of 2,
    sqrt(3), 2 or -1 and fails."""
    h = inputs.H_VOXEL
    L = n * h
    prob = inputs.Problem(n, L, *inputs.CUBIC_FE, bc=1)
    if family == "100":
        b = inputs.A_FE * np.array([1.0, 0.0, 0.0])
        nrm = np.array([1.0, 0.0, 0.0])
    else:
        b = 0.5 * inputs.A_FE * np.array([1.0, 1.0, 1.0])
        nrm = np.array([1.0, 1.0, 1.0])
    c = (np.full(3, n // 2) + 0.5) * h  # a voxel centre: the slab planes sit symmetrically
    d = inputs.loop(c, R_vox * h, b, nrm, thickness=e_vox * h)
    fps, Es = raster.rasterise(prob, d)
    es = raster.eigenstrain_field(n, fps, Es)
    C = elastic.stiffness_of(prob)
    _, sig, _ = solve.solve_field(C, L, es, bc=1)
    P_num = -(h**3) * sig.sum(axis=(2, 3, 4))
    A = math.pi * (R_vox * h) ** 2 * nrm / np.linalg.norm(nrm)
    P_paper = 0.5 * np.einsum("ijkl,kl->ij", C, np.outer(b, A) + np.outer(A, b))
    assert np.linalg.norm(P_num - P_paper) <= 0.03 * np.linalg.norm(P_paper)
    assert np.allclose(P_num, P_num.T, rtol=0, atol=1e-12 * np.abs(P_num).max())
