"""Planted mistakes in the oracle, on the CPU: each plausible error in the
pointwise physics or the face terms must make at least one physics pin fail.

The mutants wrap or replace oracle functions for the duration of one test
(pytest's monkeypatch); the pins themselves are the checks of
``test_oracle_physics.py``.  A mutation that no pin caught would mean the
oracle could carry that mistake, and the library with it, through every
parity test.
"""
import pytest
import torch

from oracle import euler as eu
from tests import test_oracle_euler as oe
from tests import test_oracle_physics as phys

ORIG_PP = eu.pressure_perturbation
ORIG_FLUX = eu.flux_dir
ORIG_VOLUME = eu.Operator.volume
ORIG_INIT = eu.Operator.__init__


def check_conservation():
    oe.test_discrete_conservation((0, 0, 0))


def _buoyancy_sign(mp):
    def volume(self, q):
        R = ORIG_VOLUME(self, q).clone()
        R[3] = R[3] + 2.0 * q[0] * self.phys.g        # +rho' g instead of -rho' g
        return R
    mp.setattr(eu.Operator, "volume", volume)


def _buoyancy_on_v(mp):
    def volume(self, q):
        R = ORIG_VOLUME(self, q).clone()
        R[3] = R[3] + q[0] * self.phys.g                # removed from rho w ...
        R[2] = R[2] - q[0] * self.phys.g                # ... and put on rho v
        return R
    mp.setattr(eu.Operator, "volume", volume)


def _gamma_minus_one(mp):
    mp.setattr(eu, "pressure_perturbation", lambda Thp, Thb, Pb, gamma: ORIG_PP(Thp, Thb, Pb, gamma - 1.0))


def _pprime_over_full_theta(mp):
    # x = Theta'/(Thetabar + Theta') instead of Theta'/Thetabar
    mp.setattr(eu, "pressure_perturbation", lambda Thp, Thb, Pb, gamma: ORIG_PP(Thp, Thb + Thp, Pb, gamma))


def _theta_flux_perturbation_only(mp):
    def flux_dir(q, bg, ph, d):
        F = ORIG_FLUX(q, bg, ph, d).clone()
        rho = bg[0] + q[0]
        F[4] = F[4] - bg[1] * q[1 + d] / rho          # Theta' u instead of (Thetabar + Theta') u
        return F
    mp.setattr(eu, "flux_dir", flux_dir)


def _pressure_on_wrong_axis(mp):
    def flux_dir(q, bg, ph, d):
        F = ORIG_FLUX(q, bg, ph, d).clone()
        Pp = eu.pressure_perturbation(q[4], bg[1], bg[2], ph.gamma)
        F[1 + d] = F[1 + d] - Pp
        F[1 + (d + 1) % 3] = F[1 + (d + 1) % 3] + Pp
        return F
    mp.setattr(eu, "flux_dir", flux_dir)


def _rusanov_variant(speed="max", sign=1.0):
    def rusanov(qL, bgL, qR, bgR, ph, d, sgn):
        rhoL, uL, _, PL = eu.primitives(qL, bgL, ph)
        rhoR, uR, _, PR = eu.primitives(qR, bgR, ph)
        FL = eu.flux_dir(qL, bgL, ph, d) * sgn
        FR = eu.flux_dir(qR, bgR, ph, d) * sgn
        cL, cR = eu.sound_speed(rhoL, PL, ph.gamma), eu.sound_speed(rhoR, PR, ph.gamma)
        if speed == "c_only":
            lam = torch.maximum(cL, cR)
        elif speed == "mean":
            lam = 0.5 * (torch.abs(uL[d]) + cL + torch.abs(uR[d]) + cR)
        else:
            lam = torch.maximum(torch.abs(uL[d]) + cL, torch.abs(uR[d]) + cR)
        return 0.5 * (FL + FR) + sign * 0.5 * lam * (qL - qR)
    return rusanov


def _wave_speed_without_velocity(mp):
    mp.setattr(eu, "rusanov", _rusanov_variant("c_only"))


def _wave_speed_mean(mp):
    mp.setattr(eu, "rusanov", _rusanov_variant("mean"))


def _antidissipative_jump(mp):
    mp.setattr(eu, "rusanov", _rusanov_variant("max", -1.0))


def _lift_weight(mp):
    def init(self, *a, **k):
        ORIG_INIT(self, *a, **k)
        self.wN = 1.0 / (self.N * (self.N + 1))     # half the LGL end weight
    mp.setattr(eu.Operator, "__init__", init)


MUTATIONS = {
    "buoyancy_sign": (_buoyancy_sign, [phys.check_rebased_hydrostatic, phys.check_manufactured]),
    "buoyancy_on_v": (_buoyancy_on_v, [phys.check_rebased_hydrostatic, phys.check_manufactured]),
    "gamma_minus_one": (_gamma_minus_one, [phys.check_pprime, phys.check_acoustic_speed, phys.check_manufactured]),
    "pprime_over_full_theta": (_pprime_over_full_theta, [phys.check_pprime, phys.check_manufactured]),
    "theta_flux_perturbation_only": (_theta_flux_perturbation_only,
                                     [phys.check_acoustic_speed, phys.check_manufactured]),
    "pressure_on_wrong_axis": (_pressure_on_wrong_axis, [phys.check_rebased_hydrostatic, phys.check_manufactured,
                                                         phys.check_vortex_rhs]),
    "wave_speed_without_velocity": (_wave_speed_without_velocity, [phys.check_rusanov]),
    "wave_speed_mean": (_wave_speed_mean, [phys.check_rusanov]),
    "antidissipative_jump": (_antidissipative_jump, [phys.check_rusanov]),
    # a smooth state has O(h^(N+1)) jumps, so the manufactured state cannot see the
    # lift factor; the read-back dissipation and discrete conservation do
    "lift_weight": (_lift_weight, [phys.check_rusanov, check_conservation]),
}


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    patch, checks = MUTATIONS[name]
    patch(monkeypatch)
    for chk in checks:
        with pytest.raises(AssertionError):
            chk()


def test_unmutated_oracle_passes_the_same_checks():
    for chk in (phys.check_pprime, phys.check_rebased_hydrostatic, phys.check_manufactured,
                phys.check_acoustic_speed, phys.check_rusanov, check_conservation):
        chk()
