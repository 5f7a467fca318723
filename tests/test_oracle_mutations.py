"""Plant plausible mistakes in the oracle (on the CPU, by monkeypatching) and
check that the pins catch each one: a wrong coupling sign, a dropped damping
prefactor, a periodic instead of open exchange boundary, a transposed
demag-tensor component, a wrong Dormand-Prince weight, and in the memory
form's recursion swapped sin/cos, a flipped sign and a dropped e^{kappa t}."""
import math

import numpy as np
import pytest

from oracle import demag as D
from oracle import llg as L
from paper_2410_00966_amd import inputs as I

import os, sys
sys.path.insert(0, os.path.dirname(__file__))
import test_oracle_llg as T  # noqa: E402


def test_flipped_coupling_sign_breaks_polaritons(monkeypatch):
    orig = L.CavityLLG.cavity_rate

    def flipped(self, a, F, t):
        return orig(self, a, -F, t)
    monkeypatch.setattr(L.CavityLLG, "cavity_rate", flipped)
    with pytest.raises(AssertionError):
        T.test_dicke_normal_phase_polaritons(1.0, 0.3)


def test_dropped_damping_prefactor_breaks_kittel(monkeypatch):
    def torque(self, m, B):
        mxB = np.cross(m, B, axis=0)
        return -self.p.gamma * (mxB + self.p.alpha * np.cross(m, mxB, axis=0))
    monkeypatch.setattr(L.CavityLLG, "torque", torque)
    with pytest.raises(AssertionError):
        T.test_kittel_anisotropy_and_damping()


def test_periodic_exchange_breaks_cosine_mode(monkeypatch):
    def exchange(self, m):
        p = self.p
        lap = np.zeros_like(m)
        for axis, d in ((3, p.dx), (2, p.dy), (1, p.dz)):
            if m.shape[axis] > 1:
                lap += (np.roll(m, 1, axis) + np.roll(m, -1, axis)
                        - 2 * m) / (d * d)
        return 2 * p.aex / self.ms * lap
    monkeypatch.setattr(L.CavityLLG, "exchange", exchange)
    with pytest.raises(AssertionError):
        T.test_exchange_neumann_cosine_mode(3)


def test_swapped_tensor_component_breaks_aharoni(monkeypatch):
    orig = D.tensor_newell

    def swapped(X, Y, Z, dx, dy, dz):
        N = orig(X, Y, Z, dx, dy, dz)
        return N[[1, 0, 2, 3, 4, 5]]
    monkeypatch.setattr(D, "tensor_newell", swapped)
    import test_oracle_demag as TD
    with pytest.raises(AssertionError):
        TD.test_self_term_equals_aharoni_prism((2.0, 1.0, 0.5))


def test_wrong_dp_weight_breaks_order(monkeypatch):
    b5 = L.DP_B5.copy()
    b5[2] *= 1.001
    monkeypatch.setattr(L, "DP_B5", b5)
    with pytest.raises(AssertionError):
        T.test_dp45_local_error_order_five()


def _memory_pin():
    import test_oracle_memory as TM
    TM.test_coupled_memory_form_converges_at_first_order()


def test_memory_recursion_swapped_sin_cos(monkeypatch):
    def sums(prob, S, C, t, F, dt):
        e = math.exp(prob.kappa * t)
        return (S + e * math.cos(prob.wc * t) * F * dt,
                C + e * math.sin(prob.wc * t) * F * dt)
    monkeypatch.setattr(L, "memory_sums", sums)
    with pytest.raises(AssertionError):
        _memory_pin()


def test_memory_gamma_flipped_sign(monkeypatch):
    def gamma(prob, vh, S, C, t, x0, p0):
        ek = math.exp(-prob.kappa * t)
        return ek * (math.cos(prob.wc * t) * (x0 + 2.0 * vh * S)
                     - math.sin(prob.wc * t) * (p0 + 2.0 * vh * C))
    monkeypatch.setattr(L, "memory_gamma_value", gamma)
    with pytest.raises(AssertionError):
        _memory_pin()


def test_memory_sums_dropped_growth_factor(monkeypatch):
    def sums(prob, S, C, t, F, dt):
        return (S + math.sin(prob.wc * t) * F * dt,
                C + math.cos(prob.wc * t) * F * dt)
    monkeypatch.setattr(L, "memory_sums", sums)
    with pytest.raises(AssertionError):
        _memory_pin()


def _sinc_pin():
    import test_oracle_drive as TD
    TD.test_sinc_cavity_drive_closed_form(0.5)


def test_normalised_sinc_breaks_drive_pin(monkeypatch):
    def shape(kind, w, t):
        if kind == L.DRIVE_SINC:
            x = math.pi * w * t
            return 1.0 if x == 0.0 else math.sin(x) / x
        return 0.0 if kind == L.DRIVE_NONE else math.cos(w * t)
    monkeypatch.setattr(L, "drive_shape", shape)
    with pytest.raises(AssertionError):
        _sinc_pin()


def test_sinc_zero_at_origin_breaks_drive_pin(monkeypatch):
    def shape(kind, w, t):
        if kind == L.DRIVE_SINC:
            x = w * t
            return 0.0 if x == 0.0 else math.sin(x) / x
        return 0.0 if kind == L.DRIVE_NONE else math.cos(w * t)
    monkeypatch.setattr(L, "drive_shape", shape)
    with pytest.raises(AssertionError):
        _sinc_pin()


def test_ignored_drive_map_breaks_linear_response(monkeypatch):
    orig = L.CavityLLG.__init__

    def init(self, prob, demag="auto"):
        orig(self, prob, demag)
        if self.fdrive_cells is not None:   # drive along the first cell's
            self.fdrive_cells = self.fdrive_cells[:, :1, :1, :1] * np.ones(
                (1,) + self.shape)
    monkeypatch.setattr(L.CavityLLG, "__init__", init)
    import test_oracle_drive as TD
    with pytest.raises(AssertionError):
        TD.test_field_drive_map_linear_response()


def test_first_mode_only_field_breaks_multimode(monkeypatch):
    orig = L.CavityLLG.cavity_field

    def field(self, a):
        if self.multi:
            return self.mode_cells[0] * (2.0 * np.real(a[0]))
        return orig(self, a)
    monkeypatch.setattr(L.CavityLLG, "cavity_field", field)
    import test_oracle_multimode as TM
    with pytest.raises(AssertionError):
        TM.test_degenerate_modes_act_as_one_bright_mode()


def test_shared_coupling_sum_breaks_multimode_polaritons(monkeypatch):
    orig = L.CavityLLG.coupling_sum

    def coupling(self, m):
        F = orig(self, m)
        return np.full_like(F, F[0]) if self.multi else F
    monkeypatch.setattr(L.CavityLLG, "coupling_sum", coupling)
    import test_oracle_multimode as TM
    with pytest.raises(AssertionError):
        TM.test_multimode_polaritons((1.0, 1.6), (0.1, 0.2))


def test_mirrored_dmi_bonds_break_continuum_limit(monkeypatch):
    """e x z in place of z x e (the other chirality, in field and energy
    alike): the gradient pin still holds, the continuum pin does not."""
    def bonds(self):
        p = self.p
        z = np.array([0.0, 0.0, 1.0])
        out = []
        for axis, d, e in ((3, p.dx, np.array([1.0, 0.0, 0.0])),
                           (2, p.dy, np.array([0.0, 1.0, 0.0])),
                           (1, p.dz, np.array([0.0, 0.0, 1.0]))):
            out.append((axis, d, np.cross(e, z) / d, -e / d))
        return out
    monkeypatch.setattr(L.CavityLLG, "_dmi_bonds", bonds)
    import test_oracle_dmi as TD
    TD.test_field_is_energy_gradient(3e-3, 0.0)
    with pytest.raises(AssertionError):
        TD.test_continuum_limit_second_order(3e-3, 0.0)


def test_dmi_field_missing_factor_breaks_gradient_pin(monkeypatch):
    orig = L.CavityLLG.dmi

    def half(self, m):
        return 0.5 * orig(self, m)
    monkeypatch.setattr(L.CavityLLG, "dmi", half)
    import test_oracle_dmi as TD
    with pytest.raises(AssertionError):
        TD.test_field_is_energy_gradient(0.0, 2e-3)


def test_relax_dropping_anisotropy_breaks_stoner_wohlfarth(monkeypatch):
    """A relax whose copy of the problem loses the anisotropy lands at the
    field direction instead of the Stoner-Wohlfarth angle."""
    import dataclasses
    orig = dataclasses.replace

    def replace(obj, **kw):
        if "precession" in kw:
            kw["ku1"] = 0.0
        return orig(obj, **kw)
    monkeypatch.setattr(dataclasses, "replace", replace)
    import test_oracle_relax as TR
    with pytest.raises(AssertionError):
        TR.test_stoner_wohlfarth_equilibrium(0.05, 68.2, 10.0)


def test_thermal_variance_with_ll_prefactor_breaks_boltzmann(monkeypatch):
    """A thermal variance divided by 1 + alpha^2 (gamma of the LL form in
    place of the gyromagnetic ratio; here alpha = 1, a factor 2) misses the
    Langevin average."""
    orig = L.CavityLLG.thermal

    def thermal(self):
        return orig(self) * math.sqrt(1.0 + self.p.alpha ** 2)
    monkeypatch.setattr(L.CavityLLG, "thermal", thermal)
    import test_oracle_thermal as TT
    with pytest.raises(AssertionError):
        TT.test_boltzmann_equilibrium_langevin()
