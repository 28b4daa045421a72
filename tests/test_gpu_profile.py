"""Kernel timing through the C ABI (ec_profile_enable, ec_profile_select,
ec_profile_read): every family of a solve + energies is timed by default, a
family mask times only the named families (the benchmark times the fused z
pass alone in its timed steps), the algorithmic bytes per launch of the
z pass are those of a read and a write of the half spectrum, and a mask with
bits beyond the families is refused.  Timing does not change the results."""
import numpy as np
import pytest

from paper_2403_09158_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2403_09158_amd import ec

    return ec.Context()


def _timed(st, defs, families):
    st.profile(True, families)
    st.profile_read()
    st.solve(defs)
    E = st.energies()
    prof = st.profile_read()
    st.profile(False)
    return E, prof


@pytest.mark.parametrize("prec", [0, 1])
def test_family_selection(ctx, prec):
    from paper_2403_09158_amd import ec

    prob, defs = inputs.pair_32()
    prob = prob.with_(prec=prec)
    st = ec.State(ctx, prob)
    st.solve(defs)
    E0 = st.energies()
    E_all, p_all = _timed(st, defs, None)
    for fam in ("raster", "x_forward", "y_pass", "z_pass_green", "x_inverse_stress", "energy_reduce"):
        assert p_all[fam]["launches"] >= 1, (fam, p_all)
        assert p_all[fam]["ms"] > 0.0
    E_z, p_z = _timed(st, defs, ["z_pass_green"])
    assert p_z["z_pass_green"]["launches"] == p_all["z_pass_green"]["launches"]
    assert all(v["launches"] == 0 for k, v in p_z.items() if k != "z_pass_green"), p_z
    n = prob.n
    spec = 6 * n * n * (n // 2 + 1) * (16 if prec == 0 else 8)
    assert p_z["z_pass_green"]["bytes_per_launch"] == pytest.approx(2 * spec)
    # the events bracket the launches; they do not change what is computed
    assert np.array_equal(E_all, E0) and np.array_equal(E_z, E0)
    st.close()


def test_invalid_family_mask_is_refused(ctx):
    from paper_2403_09158_amd import ec

    prob, defs = inputs.pair_32()
    st = ec.State(ctx, prob)
    with pytest.raises(ec.EcError, match="family mask"):
        ec._check(ec.load().ec_profile_select(st.h, 1 << ec.NPROF))
    st.close()
