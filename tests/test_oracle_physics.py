"""Pins of the oracle's pointwise physics and of the operator that carries it,
against answers fixed outside the oracle (section 2.1 equation of state and
equations, section 4.1 isentropic vortex, section 4.4 speed of sound):

  * P' against the 50-digit difference P(Thetabar + Theta') - P(Thetabar) of
    the equation of state, over |Theta'/Thetabar| from 1e-12 to 0.9;
  * a hydrostatic atmosphere of another potential temperature, written as a
    perturbation of the background: R is its truncation error only, and shrinks
    like h^N (a misplaced or sign-flipped buoyancy leaves O(rho' g));
  * the isentropic vortex: R of the exact state against its exact time
    derivative (rigid translation) for all five variables at the design rate,
    and the solution error of SSP-RK3 steps at the design rate;
  * a manufactured state with every variable varying on the neutral background
    with gravity, walls and hanging faces: R against -div F + S formed by
    automatic differentiation of the fluxes written with the full pressure;
  * the speed of sound at 300 K read from a standing acoustic wave, against the
    paper's 347.3 m/s;
  * the Rusanov dissipation read back through the operator on two constant
    elements, against max(|u.n| + c) with c from the 50-digit equation of state.

The checks are functions so that ``test_oracle_mutations.py`` can run them on
an oracle with a planted mistake and show that they fail.
"""
import json
import math
import os

import pytest

from oracle import euler as eu
from tests import pins

HERE = os.path.dirname(__file__)

PPRIME_X = [s * v for v in (1e-12, 1e-9, 1e-6, 1e-4, 2.0 ** -7, 0.01, 0.1, 0.3, 0.5, 0.9) for s in (1.0, -1.0)]


def check_pprime(Thb=348.23, bound=2e-15):
    err = pins.pprime_relative_errors(Thb, PPRIME_X, eu.Phys())
    assert max(err) <= bound, (Thb, max(err))


def check_rebased_hydrostatic(N=4, nzs=(2, 4, 8)):
    r = [pins.rebased_hydrostatic(N, nz) for nz in nzs]
    for x in r:
        # U = 0 and a state continuous across every face: no mass or Theta flux at all
        assert x["R_max"][0] == 0.0 and x["R_max"][4] == 0.0, x["R_max"]
        # P' depends on z only: the horizontal derivatives are round-off of D 1 = 0
        for v in (1, 2):
            assert x["R_max"][v] <= 1e-12 * x["pprime_scale"] * 2.0 / x["h"], (v, x)
    rates = [math.log2(r[i]["R_max"][3] / r[i + 1]["R_max"][3]) for i in range(len(r) - 1)]
    assert min(rates) > N - 0.5, rates
    # the buoyancy balances -dP'/dz to truncation error (far below rho' g itself)
    assert r[-1]["R_max"][3] < 1e-6 * r[-1]["buoyancy_scale"], r[-1]


def check_vortex_rhs(N=4, ns=(8, 16, 32)):
    res = [pins.vortex_rhs_errors(N, n) for n in ns]
    for v in (0, 1, 2, 4):
        rates = [math.log2(res[i][0][v] / res[i + 1][0][v]) for i in range(len(ns) - 1)]
        assert rates[-1] > N - 0.5, (v, [r[0][v] for r in res], rates)
        assert res[-1][0][v] < 1e-3 * res[-1][1][v], (v, res[-1])
    # the vortex does not depend on z and has no w: R_w is round-off
    assert max(r[0][3] for r in res) < 1e-13


def check_vortex_solution(N=4, ns=(8, 16, 32), T=0.25):
    res = [pins.vortex_solution_errors(N, n, T) for n in ns]
    for v in (0, 1, 2, 4):
        rates = [math.log2(res[i][v] / res[i + 1][v]) for i in range(len(ns) - 1)]
        assert rates[-1] > N + 0.5, (v, [r[v] for r in res], rates)


def check_manufactured(N=4, ns=(2, 4, 8), amr=False):
    res = [pins.mms_rhs_errors(N, n, amr=amr) for n in ns]
    if amr:
        assert all(r[2] > 0 for r in res)
    for v in range(5):
        rates = [math.log2(res[i][0][v] / res[i + 1][0][v]) for i in range(len(ns) - 1)]
        assert rates[-1] > N - 0.5, (v, [r[0][v] for r in res], rates)
        assert res[-1][0][v] < 1e-2 * res[-1][1][v], (v, res[-1])


def paper_sound_speed():
    with open(os.path.join(HERE, "golden", "sound_speed.json")) as f:
        return json.load(f)["sound_speed_300K_m_per_s"]


def check_acoustic_speed():
    c = pins.acoustic_speed()
    # the paper prints one decimal
    assert abs(c - paper_sound_speed()) <= 0.05, c


RUSANOV_PHYS = eu.Phys(g=0.0, background=eu.BG_CONSTANT, rho0=1.2, Theta0=360.0)
# pairs of constant states with the same rho u; the larger wave speed is on the
# left in the first pair, on the right in the second (checked in the test)
RUSANOV_CASES = [((0.01, 40.0, 3.0, -1.0, 25.0), (-0.02, 40.0, -2.0, 0.5, -7.0)),
                 ((0.03, -30.0, 0.0, 0.0, -20.0), (0.0, -30.0, 1.0, 2.0, 30.0))]


def check_rusanov(N=4):
    for qL, qR in RUSANOV_CASES:
        lam = pins.rusanov_wave_speed(N, qL, qR, ph=RUSANOV_PHYS)
        want = pins.max_wave_speed_mp([qL, qR], RUSANOV_PHYS)
        assert abs(lam - want).max() <= 1e-13 * want, (lam.min(), lam.max(), want)


# ----------------------------------------------------------------------------- tests

@pytest.mark.parametrize("Thb", [1.0, 251.7, 348.23])
def test_pressure_perturbation_matches_eos_difference(Thb):
    check_pprime(Thb)


def test_background_pressure_is_the_eos_of_the_hydrostatic_profile():
    """Pbar = P0 (R Thetabar/P0)^gamma and equals the hydrostatic Exner form
    P0 (1 - g z/(cp theta0))^(cp/R) (section 4.3's neutral atmosphere)."""
    import mpmath as mp
    from oracle import forest as fo
    ph = eu.Phys()
    m = fo.build(fo.ForestDesc(3, 1, 1, 4, 0, (0.0, 0.0, 0.0), (500.0, 500.0, 8000.0)), None)
    op = eu.Operator(m, ph)
    _, _, Z = eu.node_xyz(m)
    rho_b, Th_b, P_b = (t.reshape(-1) for t in op.bg)
    z = Z.reshape(-1)
    with mp.workdps(50):
        for i in range(0, z.numel(), 7):
            eos = pins.eos_mp(float(Th_b[i]), ph)
            exner = 1 - mp.mpf(ph.g) * mp.mpf(float(z[i])) / (mp.mpf(ph.cp) * mp.mpf(ph.theta0))
            hyd = mp.mpf(ph.P0) * exner ** (mp.mpf(ph.cp) / (mp.mpf(ph.cp) - mp.mpf(ph.cv)))
            assert abs(mp.mpf(float(P_b[i])) - eos) <= 1e-15 * eos
            assert abs(mp.mpf(float(P_b[i])) - hyd) <= 1e-14 * hyd
            assert float(Th_b[i]) == float(rho_b[i]) * ph.theta0


def test_rebased_hydrostatic_state():
    check_rebased_hydrostatic()


def test_isentropic_vortex_rhs_design_order():
    check_vortex_rhs()


def test_isentropic_vortex_rhs_with_hanging_faces():
    """The same vortex on a mesh refined once around it (hanging faces on a
    ring): the error is at most that of the unrefined mesh."""
    e_amr, scale, nh = pins.vortex_rhs_errors(4, 16, amr=True)
    e_uni, _, _ = pins.vortex_rhs_errors(4, 16)
    assert nh > 0
    for v in (0, 1, 2, 4):
        assert e_amr[v] <= e_uni[v], (v, e_amr[v], e_uni[v])


def test_isentropic_vortex_solution_design_order():
    check_vortex_solution()


def test_manufactured_state_uniform():
    check_manufactured()


def test_manufactured_state_hanging_faces():
    check_manufactured(amr=True)


def test_acoustic_speed_matches_paper():
    check_acoustic_speed()


def test_rusanov_wave_speed_through_the_operator():
    # the two cases put the larger wave speed on different sides
    sides = []
    for qL, qR in RUSANOV_CASES:
        sides.append(pins.max_wave_speed_mp([qL], RUSANOV_PHYS) > pins.max_wave_speed_mp([qR], RUSANOV_PHYS))
    assert sides == [True, False]
    check_rusanov()
