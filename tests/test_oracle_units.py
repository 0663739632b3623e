"""Pins of the oracle's unit layer and primitives against values fixed outside the oracle.

Eq.(1), Eq.(2), the b0 = a0 convention and the envelope of Eq.(3) are checked against
the numbers the paper prints (tests/golden/paper_examples.json) and against textbook
physics written from SI constants; Philox against numpy's independent implementation; ADK
against the hydrogen-like tunnelling rate of Landau & Lifshitz.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import units
from workloads import Cluster, Laser, Run
from workloads.species import SPECIES

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def test_eq1_ar40000_radius():
    """Sec. III: Ar_40000 with R_W = 2.4 A has R0 of about 82 A (Eq.(1) inverted)."""
    g = GOLDEN["ar40000_radius_angstrom"]
    r0_nm = g["value"] / 10.0
    n = units.n_atoms(r0_nm, g["rw_angstrom"])
    r0_from_n = g["rw_angstrom"] * g["n_atoms"] ** (1.0 / 3.0)
    assert abs(r0_from_n - g["value"]) < g["tolerance_angstrom"]
    assert abs(n - g["n_atoms"]) / g["n_atoms"] < 3 * g["tolerance_angstrom"] / g["value"]


def test_species_radii_match_paper():
    g = GOLDEN["wigner_seitz_radius_angstrom"]["value"]
    for sp, rw in g.items():
        assert SPECIES[sp]["rw_angstrom"] == rw


def test_eq2_against_si_definition():
    """Eq.(2) against a0 = eE/(m_e w c) with I = eps0 c E^2 / 2 (linear polarization).

    The paper's constant 1.366e18 follows from SI constants to 0.1 %; the printed a0 ~ 0.068
    at 1e16 W/cm^2, 800 nm must come out of the oracle's formula."""
    eps0 = 8.8541878128e-12
    lam = 0.8
    I_wm2 = 1e16 * 1e4
    E = math.sqrt(2.0 * I_wm2 / (eps0 * units.C_LIGHT))
    a0_si = units.E_CHARGE * E / (units.M_ELECTRON * units.omega(lam) * units.C_LIGHT)
    a0 = units.a0_from_intensity(1e16, lam)
    assert abs(a0 - a0_si) / a0_si < 2e-3
    g = GOLDEN["a0_at_1e16_800nm"]
    assert abs(units.a0_from_intensity(g["intensity_wcm2"], g["lambda_um"]) - g["value"]) < g["tolerance"]
    assert units.a0_from_intensity(GOLDEN["eq2_constant"]["value"], 1.0) == pytest.approx(1.0, rel=1e-15)


def test_coulomb_coupling_against_pair_energy():
    """kappa: two unit charges 1 nm apart hold e^2/(4 pi eps0 1 nm) = 1.439964548 eV."""
    lam = 0.8
    r_norm = units.nm_to_norm(1.0, lam)
    pe_ev = units.kappa(lam) / r_norm * units.MEC2_EV
    assert pe_ev == pytest.approx(1.439964548, rel=1e-8)


def test_field_and_rate_scales_against_photon_energy():
    """w t_au is the photon energy in Hartree: hc = 1239.84198 eV nm.  And the field unit:
    a0 = 1 at 800 nm is m_e w c/e = 4.0135e12 V/m, i.e. 7.805 atomic units."""
    lam = 0.8
    photon_hartree = 1239.841984 / (lam * 1000.0) / units.HARTREE_EV
    assert 1.0 / units.rate_scale(lam) == pytest.approx(photon_hartree, rel=1e-8)
    # In atomic units m_e = e = hbar = 1 and c = 1/alpha, so the field unit m_e w c / e is
    # (hbar w / E_h) / alpha atomic units of field.
    alpha = 7.2973525693e-3
    assert units.field_au_per_a0(lam) == pytest.approx(photon_hartree / alpha, rel=1e-8)


def test_philox_matches_numpy():
    """numpy's Philox (an independent Philox4x64-10) increments its 256-bit counter before
    producing each block of four words; block k of a generator started at counter c is
    Philox(key, c + k + 1)."""
    for key, ctr in [((5, 7), (0, 0, 0, 0)), ((0, 0), (0, 0, 0, 0)), ((2**64 - 1, 123), (9, 4, 2, 0)),
                     ((17, 2**63), (2**64 - 1, 0, 3, 0))]:
        g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
        raw = [int(v) for v in g.random_raw(8)]
        c0 = list(ctr)
        # counter + 1 with carry
        def inc(c):
            c = list(c)
            for k in range(4):
                c[k] = (c[k] + 1) % 2**64
                if c[k] != 0:
                    break
            return c
        c1 = inc(c0)
        c2 = inc(c1)
        assert oracle.philox4x64_10(key, c1) == raw[:4]
        assert oracle.philox4x64_10(key, c2) == raw[4:]


def test_u01_range():
    """0 < alpha <= 1 (Sec. II)."""
    assert oracle.u01(0) == 2.0**-53
    assert oracle.u01(2**64 - 1) == 1.0
    assert 0.0 < oracle.u01(2**63) <= 1.0


def test_adk_hydrogen_limit():
    """H-like ground state (Ip = 1/2, Zc = 1): the ADK rate reduces to the Landau-Lifshitz
    tunnelling rate w = (4/F) exp(-2/(3F)) in atomic units."""
    for F in [0.01, 0.03, 0.05, 0.1, 0.2, 0.5]:
        ref = 4.0 / F * math.exp(-2.0 / (3.0 * F))
        assert oracle.adk_rate(0.5, 1.0, F) == pytest.approx(ref, rel=1e-13)


def test_adk_hydrogenic_ion_scaling():
    """Hydrogen-like ion of charge Zc (Ip = Zc^2/2): w = 4 Zc^5 / F exp(-2 Zc^3 / (3F))."""
    for Zc in [2.0, 3.0, 5.0]:
        for F in [0.5, 2.0, 10.0]:
            ref = 4.0 * Zc**5 / F * math.exp(-2.0 * Zc**3 / (3.0 * F))
            assert oracle.adk_rate(Zc * Zc / 2.0, Zc, F) == pytest.approx(ref, rel=1e-12)


def test_adk_n_star_two():
    """n* = 2 (Zc = 2, Ip = 1/2): C^2 = 2^4 / (2 Gamma(4)) = 4/3, so
    w = (4/3)(1/2)(2/F)^3 exp(-2/(3F)) = (16/3) F^-3 exp(-2/(3F))."""
    for F in [0.02, 0.05, 0.1]:
        ref = 16.0 / 3.0 / F**3 * math.exp(-2.0 / (3.0 * F))
        assert oracle.adk_rate(0.5, 2.0, F) == pytest.approx(ref, rel=1e-12)


def test_adk_below_threshold_is_zero():
    assert oracle.adk_rate(1.0, 2.0, 0.0) == 0.0
    assert oracle.adk_rate(1.0, 2.0, 5e-7) == 0.0


def test_envelope_fwhm_readings():
    """Eq.(3) as printed: field envelope centred at 2 tau with constant 2.77 ~ 4 ln 2, so the
    field drops to one half at 2 tau +- tau/2; the intensity variant halves the exponent so
    the intensity (a^2) drops to one half there.  sin^2: zero at the ends, a0 mid-pulse."""
    c = Cluster(laser=Laser(envelope="gauss_field", fwhm_fs=30.0))
    p = oracle.make_params(c, Run())
    tau = p.tau
    assert oracle.envelope(p, 2 * tau) == pytest.approx(p.a0, rel=1e-15)
    assert oracle.envelope(p, 2 * tau + tau / 2) / p.a0 == pytest.approx(0.5, abs=1e-3)
    assert oracle.envelope(p, 2 * tau - tau / 2) / p.a0 == pytest.approx(0.5, abs=1e-3)
    c2 = Cluster(laser=Laser(envelope="gauss_intensity", fwhm_fs=30.0))
    p2 = oracle.make_params(c2, Run())
    assert (oracle.envelope(p2, 2 * tau + tau / 2) / p2.a0) ** 2 == pytest.approx(0.5, abs=1e-3)
    c3 = Cluster(laser=Laser(envelope="sin2", n_cycles=10))
    p3 = oracle.make_params(c3, Run())
    T = 20 * math.pi
    assert oracle.envelope(p3, 0.0) == 0.0
    assert oracle.envelope(p3, T / 2) == pytest.approx(p3.a0, rel=1e-15)
    assert oracle.envelope(p3, T + 1.0) == 0.0


def test_laser_components_linear():
    """Eqs.(4)-(9), linear polarization: only E_x and B_y, equal in these units (b0 = a0),
    both a(t) sin t in the dipole approximation; E x B points along +z for the plane wave."""
    c = Cluster(laser=Laser(envelope="flat"))
    p = oracle.make_params(c, Run())
    for t in [0.3, 1.0, 2.5, 4.0]:
        E, B = oracle.laser(p, t, 0.7)
        assert E[1] == 0.0 and E[2] == 0.0 and B[0] == 0.0 and B[2] == 0.0
        assert E[0] == pytest.approx(p.a0 * math.sin(t), rel=1e-14)
        assert B[1] == E[0]
    cp = Cluster(laser=Laser(envelope="flat", phase="plane_wave"))
    pp = oracle.make_params(cp, Run())
    E, B = oracle.laser(pp, 1.0, 0.4)
    assert E[0] == pytest.approx(pp.a0 * math.sin(0.6), rel=1e-14)
    assert np.cross(E, B)[2] >= 0.0


def test_laser_components_circular():
    """Eqs.(4)-(9), circular polarization (phi_E = 3 pi/2, phi_B = pi/2): E_x and B_y as in the
    linear case, E_y = a sin(t + 3 pi/2), B_x = a sin(t + pi/2); |E| = |B| = a(t) at every
    phase, E . B = 0 and E x B = a^2 z^ (the wave runs along +z)."""
    lin = oracle.make_params(Cluster(laser=Laser(envelope="flat")), Run())
    p = oracle.make_params(Cluster(laser=Laser(envelope="flat", polarization="circular")), Run())
    for t in [0.3, 1.0, 2.5, 4.0, 5.9]:
        E, B = oracle.laser(p, t)
        El, Bl = oracle.laser(lin, t)
        assert E[0] == El[0] and B[1] == Bl[1] and E[2] == 0.0 and B[2] == 0.0
        assert E[1] == pytest.approx(p.a0 * math.sin(t + 1.5 * math.pi), abs=1e-15 * p.a0)
        assert B[0] == pytest.approx(p.a0 * math.sin(t + 0.5 * math.pi), abs=1e-15 * p.a0)
        assert np.linalg.norm(E) == pytest.approx(p.a0, rel=1e-14)
        assert abs(E @ B) < 1e-15 * p.a0 ** 2
        assert np.cross(E, B) == pytest.approx([0.0, 0.0, p.a0 ** 2], rel=1e-13, abs=1e-18)


def test_exponential_integral_matches_scipy():
    """E1 from the series (x <= 1) and the continued fraction (x > 1) against scipy."""
    from scipy.special import exp1
    for x in np.concatenate([np.logspace(-8, 2.7, 300), [1.0, 1.0 + 1e-12, 0.999999]]):
        assert oracle.e1(x) == pytest.approx(float(exp1(x)), rel=2e-15)


def test_lotz_rate_is_the_maxwellian_average_of_the_cross_section():
    """The closed form 2 sqrt(2/(pi m_e)) a q E1(P/T) / (P sqrt T) against the average of the
    Lotz cross-section a q ln(E/P)/(E P) over a Maxwellian, integrated numerically with the
    electron speed from the SI constants (CODATA m_e, e)."""
    from scipy.integrate import quad
    me, ev = 9.1093837015e-31, 1.602176634e-19
    a, q = 4.5e-14, 5.0
    for P, T in [(27.63, 100.0), (27.63, 5.0), (143.46, 40.0), (12.13, 1000.0), (422.6, 30.0)]:
        def f(E):
            sigma = a * q * math.log(E / P) / (E * P)
            v = math.sqrt(2.0 * E * ev / me) * 100.0
            return sigma * v * 2.0 * math.sqrt(E / math.pi) * T ** -1.5 * math.exp(-E / T)
        val, err = quad(f, P, P + 60.0 * T, limit=400, epsabs=0.0, epsrel=1e-12)
        assert oracle.lotz_rate(a, q, P, T) == pytest.approx(val, rel=1e-9)
    assert oracle.lotz_rate(a, q, 27.63, 0.0) == 0.0 and oracle.lotz_rate(a, 0.0, 27.63, 50.0) == 0.0
