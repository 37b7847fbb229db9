"""Pins of the closed forms used for units and properties (Eqs. 11, 12, 17, 26-29)."""
import math

import numpy as np
import pytest

R_GAS = 8.314462618


def test_knudsen_diffusivity_printed_value(orc):
    # Section 4.2 prints D_K,ref = 1.31e-5 (m^2/s) for d = 60 nm, T = 323 K, methane
    dk = orc.knudsen_diffusivity(60e-9, 323.0, 0.016043)
    assert dk == pytest.approx(1.31e-5, rel=5e-3)
    # linear in d, sqrt in T
    assert orc.knudsen_diffusivity(30e-9, 323.0) == pytest.approx(dk / 2, rel=1e-14)
    assert orc.knudsen_diffusivity(60e-9, 4 * 323.0) == pytest.approx(2 * dk, rel=1e-14)


@pytest.mark.parametrize("d,T,mu,P", [(20e-9, 323.0, 1.73e-5, 17236893.0),
                                      (60e-9, 400.0, 1.2e-5, 1e6), (5e-9, 300.0, 1e-5, 3e5)])
def test_eq28_coefficient(orc, d, T, mu, P):
    # Eqs. 11, 26, 27, 29 combine into f_c = 1 + 64/(3 pi) Kn with Kn = lambda / radius
    Dk = orc.knudsen_diffusivity(d, T)
    k = (d / 2) ** 2 / 8
    fc = orc.fc_dgm(Dk, mu, k, P)
    lam = orc.mean_free_path(mu, P, T)
    assert fc - 1 == pytest.approx(64 / (3 * math.pi) * lam / (d / 2), rel=1e-12)
    assert 64 / (3 * math.pi) == pytest.approx(6.7906, abs=1e-4)


def test_kozeny_carman(orc):
    assert orc.k_kozeny_carman(45e-9, 0.4) == pytest.approx(45e-9 ** 2 / 180 * 0.064 / 0.36,
                                                            rel=1e-14)


def test_tau_g_eq12(orc):
    # tau_g = tau_ref at d = d_ref, 1/2 at d = 0, linear in between
    assert orc.tau_g(40.0, 40.0, 1.0) == 1.0
    assert orc.tau_g(0.0, 40.0, 1.0) == 0.5
    d = np.array([1.0, 10.0, 20.0, 80.0])
    assert np.allclose(orc.tau_g(d, 40.0, 1.0), 0.5 + 0.5 * d / 40.0, rtol=1e-15)
