"""Pins of the oracle's MRT collision (Section 3.1, Eqs. 4-7, Appendix A).

* The inverse of Q implied by Q's orthogonal rows equals the inverse the paper prints
  (tests/golden/mrt_qinv_appendix_a.txt), except for the misprinted row 6.
* The collision conserves mass and adds exactly F to the momentum.
* With every rate set to 1/tau the MRT collision is the BGK collision (at rho = 1, where
  the incompressible equilibrium moments of Appendix A and Eq. 3 coincide).
* Eq. 7 relaxes every odd non-conserved moment at s_q = 8(2 tau - 1)/(8 tau - 1) and
  every even one at 1/tau: a two-relaxation-time scheme with (tau - 1/2)(1/s_q - 1/2) =
  3/16.  For that value the discrete slit with half-way bounce-back has the
  tau-independent permeability (H / n_y)(H^2 + 1/2)/12 (the BGK value has 8 (tau - 1/2)^2
  in place of 3/2).
* That two-relaxation-time form, written in velocity space from its own definition,
  gives the moment-space collision to rounding, also away from rho = 1 and with a force.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_1410_1921_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "mrt_qinv_appendix_a.txt")


def _printed_inverse():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 19 and all(len(r) == 19 for r in rows)
    return np.array([[float(Fraction(c)) for c in r] for r in rows])


def test_inverse_matches_the_printed_table(orc):
    q, qi = orc.mrt_matrices()
    assert np.allclose(q @ qi, np.eye(19), atol=1e-14)
    printed = _printed_inverse()
    rows = [i for i in range(19) if i != 6]
    assert np.allclose(qi[rows], printed[rows], rtol=0, atol=1e-15)
    # row 6: the printed -1/36, 1/36 in columns 11, 12 against -1/12, 1/12
    assert qi[6, 11] == pytest.approx(-1 / 12) and printed[6, 11] == pytest.approx(-1 / 36)
    other = [k for k in range(19) if k not in (11, 12)]
    assert np.allclose(qi[6, other], printed[6, other], atol=1e-15)


def test_rates_of_eq7(orc):
    tau = 0.9
    s = orc.mrt_rates(tau)
    sq = 8 * (2 * tau - 1) / (8 * tau - 1)
    assert [s[k] for k in (0, 3, 5, 7)] == [0, 0, 0, 0]
    assert np.allclose([s[k] for k in (1, 2, 9, 10, 11, 12, 13, 14, 15)], 1 / tau, rtol=1e-15)
    assert np.allclose([s[k] for k in (4, 6, 8, 16, 17, 18)], sq, rtol=1e-15)
    assert (tau - 0.5) * (1 / sq - 0.5) == pytest.approx(3 / 16, rel=1e-14)


def test_conservation(orc):
    rng = np.random.default_rng(3)
    e = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                  [1, 1, 0], [-1, 1, 0], [1, -1, 0], [-1, -1, 0], [1, 0, 1], [-1, 0, 1],
                  [1, 0, -1], [-1, 0, -1], [0, 1, 1], [0, -1, 1], [0, 1, -1], [0, -1, -1]], float)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    for _ in range(5):
        fin = w * (1 + 0.05 * rng.standard_normal(19))
        F = 1e-3 * rng.standard_normal(3)
        fout, mom = orc.collide19_mrt(fin, 0.77, F)
        assert fout.sum() == pytest.approx(fin.sum(), rel=1e-14)
        assert np.allclose(fout @ e, fin @ e + F, rtol=0, atol=1e-15)
        assert np.allclose(mom[1:], fin @ e + 0.5 * F, rtol=0, atol=1e-15)


def test_equal_rates_give_bgk(orc):
    rng = np.random.default_rng(4)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    for tau in (0.6, 0.8, 1.3):
        fin = w * (1 + 0.05 * rng.standard_normal(19))
        fin[0] += 1.0 - fin.sum()  # rho = 1: the incompressible and full equilibria agree
        F = 1e-4 * rng.standard_normal(3)
        a, _ = orc.collide19_mrt(fin, tau, F, rates=np.full(19, 1.0 / tau))
        b, _ = orc.collide19(fin, tau, F)
        assert np.allclose(a, b, rtol=0, atol=1e-15)


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.2])
@pytest.mark.parametrize("h", [6, 9])
def test_slit_permeability_is_viscosity_independent(orc, tau, h):
    m = W.slit(2, h + 2, 2, h, axis=1)
    r = orc.flow_solve(m, tau=tau, force=(1e-6, 0, 0), max_steps=400_000, check_every=100,
                       tol=1e-13, want_u=False, collision=orc.MRT)
    assert r["converged"]
    assert r["k_lattice"] == pytest.approx(h / (h + 2) * (h * h + 0.5) / 12, rel=1e-8)


@pytest.mark.parametrize("tau", [0.55, 0.8, 1.7])
def test_two_relaxation_time_form_is_the_same_collision(orc, tau):
    # the velocity-space TRT form (pairs of opposite velocities, even part at 1/tau, odd
    # part at s_q, incompressible equilibrium) against the moment-space MRT, away from
    # rho = 1 and with a force: the same operator, to rounding
    rng = np.random.default_rng(int(tau * 100))
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    for _ in range(6):
        fin = w * (0.9 + 0.25 * rng.random(19))
        F = 1e-3 * rng.standard_normal(3)
        a, ma = orc.collide19_mrt(fin, tau, F)
        b, mb = orc.collide19_trt(fin, tau, F)
        assert np.allclose(a, b, rtol=0, atol=2e-15)
        assert np.allclose(ma, mb, rtol=0, atol=1e-15)


def test_two_relaxation_time_form_in_a_solve(orc):
    m = W.blob_mask((7, 9, 11), 0.6, 5)
    kw = dict(tau=0.75, force=(1e-4, 2e-5, -3e-5), fixed_steps=200, check_every=50)
    a = orc.flow_solve(m, collision=orc.MRT, **kw)
    b = orc.flow_solve(m, collision=orc.TRT, **kw)
    assert np.abs(a["u"] - b["u"]).max() <= 1e-12 * np.abs(a["u"]).max()
    assert b["k_lattice"] == pytest.approx(a["k_lattice"], rel=1e-12)
