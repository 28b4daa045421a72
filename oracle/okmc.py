"""One time step of the parallel OkMC loop (oracle; test infrastructure only).

Sec. 5 and App. B.  Every defect can act in every step.  The step is fixed
once, from the nominal frequencies nu_i = nu_0 exp(-E_m,i / (k_B T)) (the jump
frequency without elastic bias), as the inverse of the largest one, so that the
fastest defect makes one event per step on average.  In a step each defect
draws its number of events N_i from the Poisson law with mean nu_i dt.  A
defect with N_i > 0 evaluates the energy change of each of its candidate jumps
against the field of the current positions (the other defects all stay where
they are for this evaluation), turns them into biased frequencies and picks one
jump on its frequency line (``jumps``).  When every defect has been treated the
positions are updated and the total field is formed again for the new
positions; the clock advances by dt.

Readings: (i) a defect with N_i > 0 makes one jump in the step (the algorithm
selects a single jump per defect and step, whatever N_i is); (ii) the random
numbers are inputs: u_i in (0, 1] gives N_i by inversion of the Poisson
distribution function (the smallest N with u_i <= P(N_i <= N)), xi_i in (0, 1]
the jump on the frequency line; (iii) a jump moves the defect record's centre
by the jump vector times the voxel edge.
"""
from __future__ import annotations

import math

import numpy as np

from . import energy, jumps, raster


def nominal_frequencies(Em, kT, nu0) -> np.ndarray:
    """nu_i = nu_0 exp(-E_m,i / kT) (Sec. 5, the unbiased jump frequency)."""
    return nu0 * np.exp(-np.asarray(Em, dtype=np.float64) / kT)


def time_step(Em, kT, nu0) -> float:
    """dt = 1 / max_i nu_i (Sec. 5, the fixed time step)."""
    return 1.0 / float(nominal_frequencies(Em, kT, nu0).max())


def event_counts(nu, dt, u) -> np.ndarray:
    """N_i from the Poisson law P(N) = (nu dt)^N exp(-nu dt) / N! (Sec. 5) by
    inversion: the smallest N whose cumulative probability reaches u_i."""
    out = np.zeros(len(nu), dtype=np.int64)
    for i, (rate, ui) in enumerate(zip(np.asarray(nu, dtype=np.float64), u)):
        mean = rate * dt
        p = math.exp(-mean)  # P(N = 0)
        cdf = p
        k = 0
        while ui > cdf and k < 1000:
            k += 1
            p *= mean / k
            cdf += p
        out[i] = k
    return out


def move(problem, defects, jumps_, choice):
    """The defect records after the chosen jumps (choice -1: the defect stays)."""
    moved = np.array(defects, copy=True)
    h = problem.L / problem.n
    for i, j in enumerate(choice):
        if j >= 0:
            moved["c"][i] = moved["c"][i] + np.asarray(jumps_[i][j], dtype=np.float64) * h
    return moved


def okmc_step(problem, defects, jumps_, Em, nu0, kT, dt, u, xi):
    """One step: (N, choice, moved defects, energies after the step).

    dt <= 0 takes the fixed step of ``time_step``.  The energy changes come
    from the superposition form pinned against the definition in ``jumps``;
    the energies after the step are the exact ones of the moved list."""
    Em = np.broadcast_to(np.asarray(Em, dtype=np.float64), (len(defects),))
    if dt <= 0.0:
        dt = time_step(Em, kT, nu0)
    N = event_counts(nominal_frequencies(Em, kT, nu0), dt, u)
    fps, Es = raster.rasterise(problem, defects)
    dE = jumps.jump_energies_fast(problem, fps, Es, jumps_)
    nu = jumps.jump_frequencies(dE, Em, kT, nu0)
    sel = jumps.select_jumps(nu, xi)
    choice = np.where(N > 0, sel, -1)
    moved = move(problem, defects, jumps_, choice)
    E1 = energy.energies_fast(problem, moved)
    return N, choice, moved, E1
