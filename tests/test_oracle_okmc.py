"""Pins of the OkMC step oracle: the paper's printed time step, the Poisson
event counts against the library inversion and the law's closed forms, the
uniform choice of an isolated defect, and the energies after a step against
the moved list computed from scratch."""
import json
import os

import numpy as np
from scipy import stats

from oracle import energy, jumps, okmc, raster
from paper_2403_09158_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_time_step_is_the_papers():
    g = json.load(open(os.path.join(GOLDEN, "okmc_time_step.json")))
    kT = g["kB_eV_per_K"] * g["T_K"]
    dt = okmc.time_step([g["Em_eV"], g["Em_eV"] + 0.05], kT, g["nu0_per_s"])
    assert abs(dt * 1e12 - g["dt_ps"]) <= g["printed_precision_ps"], dt
    # the fastest defect sets the step
    assert okmc.time_step([0.3, 0.1, 0.2], kT, 1e13) == okmc.time_step([0.1], kT, 1e13)


def test_event_counts_are_the_poisson_inversion():
    rng = np.random.default_rng(inputs.SEED_BASE + 800)
    mean = rng.uniform(0.0, 6.0, size=4000)
    u = 1.0 - rng.uniform(0.0, 1.0, size=4000)  # (0, 1]
    N = okmc.event_counts(mean, 1.0, u)
    assert np.array_equal(N, stats.poisson.ppf(u, mean).astype(np.int64))
    # the boundary of N = 0 is P(0) = exp(-nu dt) itself (u <= P(0): no event)
    m = 0.7
    p0 = np.exp(-m)
    assert okmc.event_counts([m], 1.0, [p0])[0] == 0
    assert okmc.event_counts([m], 1.0, [np.nextafter(p0, 1.0)])[0] == 1
    assert okmc.event_counts([0.0], 1.0, [1.0])[0] == 0


def test_event_count_statistics_of_the_fixed_step():
    """With dt = 1 / nu_max the fastest defect makes one event per step on
    average (Sec. 5); mean and variance 1, P(N = 0) = 1/e."""
    rng = np.random.default_rng(inputs.SEED_BASE + 801)
    k = 200000
    kT, nu0 = 0.025852, 1e13
    Em = np.full(k, 0.1)
    dt = okmc.time_step(Em, kT, nu0)
    N = okmc.event_counts(okmc.nominal_frequencies(Em, kT, nu0), dt, 1.0 - rng.uniform(size=k))
    se = 1.0 / np.sqrt(k)
    assert abs(N.mean() - 1.0) < 5 * se
    assert abs(N.var() - 1.0) < 5 * np.sqrt(2.0) * se
    assert abs((N == 0).mean() - np.exp(-1.0)) < 5 * se
    # a slower defect (barrier + kT) acts e times less often on average
    N2 = okmc.event_counts(okmc.nominal_frequencies(np.full(k, 0.1 + kT), kT, nu0), dt, 1.0 - rng.uniform(size=k))
    assert abs(N2.mean() - np.exp(-1.0)) < 5 * se


def _cell(n=32):
    h = inputs.H_VOXEL
    prob = inputs.Problem(n, n * h, *inputs.CUBIC_FE)
    b = 0.5 * inputs.A_FE * np.array([1.0, 1.0, 1.0])
    b2 = 0.5 * inputs.A_FE * np.array([1.0, -1.0, 1.0])
    d = np.concatenate(
        [
            inputs.loop(np.array([10.5, 12.5, 11.5]) * h, 2.6 * h, b, b),
            inputs.loop(np.array([21.2, 17.7, 19.4]) * h, 2.2 * h, b2, b2),
            inputs.sphere(np.array([31.5, 3.5, 16.5]) * h, 1.8 * h, 0.01),
        ]
    )
    return prob, d


J4 = [(1, 1, 1), (-1, -1, -1), (1, -1, 0), (0, 0, 2)]


def test_isolated_defect_chooses_uniformly():
    """Alone in the cell a defect has no interaction energy, every jump has the
    same frequency and the frequency line is split evenly."""
    prob, d = _cell()
    one = d[:1]
    for xi, want in ((0.1, 0), (0.25, 0), (0.26, 1), (0.7, 2), (1.0, 3)):
        N, choice, moved, E1 = okmc.okmc_step(prob, one, [J4], [0.1], 1e13, 0.025852, 0.0, [0.9], [xi])
        assert N[0] >= 1 and choice[0] == want
        assert np.allclose(moved["c"][0], one["c"][0] + np.asarray(J4[want]) * prob.h, rtol=0, atol=1e-12)
        assert E1[0] == 0.0 or abs(E1[0]) < 1e-12
    N, choice, moved, _ = okmc.okmc_step(prob, one, [J4], [0.1], 1e13, 0.025852, 0.0, [0.3], [0.5])
    assert N[0] == 0 and choice[0] == -1 and np.array_equal(moved["c"], one["c"])


def test_step_energies_are_those_of_the_moved_list():
    """All three defects act; the energies after the step equal the definition
    (one solve per defect) on the moved records, and a step in which one defect
    alone moves changes its energy by the probed dE of the chosen jump."""
    prob, d = _cell()
    J = [J4] * 3
    Em = [0.1, 0.12, 0.1]
    kT, nu0 = 0.025852, 1e13
    N, choice, moved, E1 = okmc.okmc_step(prob, d, J, Em, nu0, kT, 0.0, [0.999, 0.999, 0.999], [0.3, 0.6, 0.9])
    assert np.all(N > 0) and np.all(choice >= 0)
    Eb, _ = energy.energies_brute(prob, moved)
    assert np.abs(E1 - Eb).max() <= 1e-10 * np.abs(Eb).max()
    # one mover: its energy change is the probe's
    fps, Es = raster.rasterise(prob, d)
    dE = jumps.jump_energies_brute(prob, fps, Es, J)
    E0 = energy.energies_fast(prob, d)
    N, choice, _, E1 = okmc.okmc_step(prob, d, J, Em, nu0, kT, 0.0, [0.999, 1e-9, 1e-9], [0.6, 0.5, 0.5])
    assert choice[0] >= 0 and choice[1] == -1 and choice[2] == -1
    assert abs((E1[0] - E0[0]) - dE[0, choice[0]]) <= 1e-10 * np.abs(E0).max()
