"""Dislocation lines on the GPU (ec_set_dislocations): the stress of the lines
with defects against the oracle's superposition, the defects' energies in the
lines' field, the paper's rotated frame with an edge dislocation along [1-10],
hops through the incremental update, order independence and removal, and the
argument checks.

Tolerances: fields rel L2 1e-12 (FP64) / 1e-5 (FP32 storage of the defects'
spectra; the lines' stress is FP64 either way); energies 1e-10 of the largest
(FP64) / max(1e-4 |E_i|, 1e-5 eV) per defect (FP32)."""
import numpy as np
import pytest

from helpers import energy_ok_fp32, energy_ok_fp64, rel_l2, rel_max, to6
from oracle import dislocation as odl
from oracle import elastic, energy, raster, solve
from paper_2403_09158_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2403_09158_amd import ec

    return ec.Context()


def _case(prec=0, frame=(), n=32):
    h = inputs.H_VOXEL
    prob = inputs.Problem(n, n * h, *inputs.CUBIC_FE, prec=prec, frame=frame)
    bx = 0.5 * inputs.A_FE * np.sqrt(3.0) * np.array([1.0, 0.0, 0.0])
    d = np.concatenate(
        [
            inputs.loop(np.array([8.5, 10.5, 12.5]) * h, 3.2 * h, bx, bx),
            inputs.loop(np.array([21.2, 19.7, 18.4]) * h, 2.8 * h, 0.5 * inputs.A_FE * np.array([0.0, 0.0, 1.0]), np.array([0.0, 0.0, 1.0])),
            inputs.sphere(np.array([24.5, 3.5, 8.5]) * h, 1.9 * h, 0.012),
        ]
    )
    lines = np.concatenate(
        [
            inputs.line(np.array([15.3, 16.8, 0.0]) * h, 2, 1, bx),  # edge, along z
            inputs.line(np.array([4.0, 0.0, 26.6]) * h, 1, -1, np.array([0.0, 0.2, 0.0])),  # screw, along -y
        ]
    )
    return prob, d, lines


def _oracle_lines(lines):
    return [(np.array(l["p"]), int(l["axis"]), int(l["sense"]), np.array(l["b"])) for l in lines]


def _oracle(prob, d, lines):
    fps, Es = raster.rasterise(prob, d)
    es = raster.eigenstrain_field(prob.n, fps, Es)
    _, sig_def, _ = solve.solve_field(elastic.stiffness_of(prob), prob.L, es, prob.bc)
    sig_d = odl.dislocation_stress(prob, _oracle_lines(lines))
    E = energy.energies_fast(prob, d) + odl.background_energies(prob, fps, Es, sig_d)
    return to6(sig_def + sig_d), E


@pytest.mark.parametrize("frame", [(), inputs.FRAME_111], ids=["cube", "frame111"])
@pytest.mark.parametrize("prec", [0, 1])
def test_lines_and_defects_match_oracle(ctx, prec, frame):
    from paper_2403_09158_amd import ec

    prob, d, lines = _case(prec, frame)
    sig_o, E_o = _oracle(prob, d, lines)
    st = ec.State(ctx, prob)
    st.set_dislocations(lines)
    st.solve(d)
    E = st.energies()
    sig = st.field("sigma")
    tol = 1e-12 if prec == 0 else 1e-5
    assert rel_l2(sig, sig_o) < tol and rel_max(sig, sig_o) < 10 * tol
    if prec == 0:
        assert energy_ok_fp64(E, E_o)
    else:
        assert np.all(energy_ok_fp32(E, E_o))
    st.close()


@pytest.mark.parametrize("n", [48, 64])
def test_lines_at_larger_grids(ctx, n):
    """The direct inverse transforms of the lines' plane and the solve at 48
    and 64 (other transform plans than at 32), in the rotated frame, against
    the oracle."""
    from paper_2403_09158_amd import ec

    prob, d, lines = _case(0, inputs.FRAME_111, n=n)
    sig_o, E_o = _oracle(prob, d, lines)
    st = ec.State(ctx, prob)
    st.set_dislocations(lines)
    st.solve(d)
    sig = st.field("sigma")
    assert rel_l2(sig, sig_o) < 1e-12 and rel_max(sig, sig_o) < 1e-11
    assert energy_ok_fp64(st.energies(), E_o)
    st.close()


def test_order_removal_and_hops(ctx):
    from paper_2403_09158_amd import ec

    prob, d, lines = _case()
    a = ec.State(ctx, prob)
    a.solve(d)
    E_plain = a.energies().copy()
    a.set_dislocations(lines)  # after the solve
    b = ec.State(ctx, prob)
    b.set_dislocations(lines)  # before the solve
    b.solve(d)
    assert energy_ok_fp64(a.energies(), b.energies(), rtol=1e-12)
    # a hop with the lines present, against the oracle
    cur = d.copy()
    cur[0]["c"] = cur[0]["c"] + np.array([1.0, 0.0, -1.0]) * prob.h
    E = a.update(0, cur[0])
    _, E_o = _oracle(prob, cur, lines)
    assert energy_ok_fp64(E, E_o)
    # removing the lines restores the plain field
    b.set_dislocations(np.zeros(0, dtype=inputs.LINE_DTYPE))
    assert energy_ok_fp64(b.energies(), E_plain, rtol=1e-12)
    a.close()
    b.close()


def test_dislocation_argument_checks(ctx):
    from paper_2403_09158_amd import ec

    prob, d, lines = _case()
    st = ec.State(ctx, prob)
    st.solve(d)
    E0 = st.energies().copy()
    bad = []
    for field, value in (("axis", 3), ("sense", 0), ("b", (0.0, 0.0, 0.0)), ("p", (np.nan, 0.0, 0.0))):
        l = lines.copy()
        l[1][field] = value
        bad.append(l)
    bad.append(np.concatenate([lines] * 33))  # 66 lines
    for l in bad:
        with pytest.raises(ec.EcError) as ei:
            st.set_dislocations(l)
        assert ei.value.status == ec.EC_ERR_ARG
    assert np.array_equal(st.energies(), E0)
    st.close()


def test_lines_without_defects(ctx):
    """An empty defect list: the resident stress is the lines' stress alone."""
    from paper_2403_09158_amd import ec

    prob, _, lines = _case()
    st = ec.State(ctx, prob)
    st.set_dislocations(lines)
    st.solve(inputs.empty_defects(0))
    assert len(st.energies()) == 0
    sig_o = to6(odl.dislocation_stress(prob, _oracle_lines(lines)))
    assert rel_l2(st.field("sigma"), sig_o) < 1e-12
    st.close()


def test_lines_along_every_axis(ctx):
    """One line along each cell axis (mixed Burgers vectors), with defects."""
    from paper_2403_09158_amd import ec

    prob, d, _ = _case()
    h = prob.h
    lines = np.concatenate(
        [
            inputs.line(np.array([0.0, 9.3, 20.8]) * h, 0, 1, np.array([0.12, 0.05, -0.07])),
            inputs.line(np.array([27.1, 0.0, 5.6]) * h, 1, 1, np.array([-0.1, 0.15, 0.02])),
            inputs.line(np.array([3.4, 29.9, 0.0]) * h, 2, -1, np.array([0.0, 0.08, 0.2])),
        ]
    )
    sig_o, E_o = _oracle(prob, d, lines)
    st = ec.State(ctx, prob)
    st.set_dislocations(lines)
    st.solve(d)
    assert rel_l2(st.field("sigma"), sig_o) < 1e-12
    assert energy_ok_fp64(st.energies(), E_o)
    st.close()
