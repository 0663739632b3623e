"""Pins of the oracle's field sum, Boris mover, ionization and diagnostics.

Each test checks the oracle against something it does not compute itself: closed-form
solutions (two-body explosion, plane-wave figure-8 orbit, dipole-field invariants, the
uniform-sphere self energy), conservation laws (Newton's third law, the discrete Boris
energy identity, energy bookkeeping with second-order convergence), finite differences of
the potential, brute force at 50 digits, and Monte-Carlo statistics with a known survival
law.
"""
import dataclasses
import math

import mpmath
import numpy as np
import pytest

import oracle
from oracle import units
from workloads import Cluster, Laser, Run, initial_state, small_ar

mpmath.mp.dps = 50


def _rand_state(n, seed, scale=0.02):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-scale, scale, (n, 3))
    q = rng.choice([-1.0, 1.0, 2.0, 3.0], n) * 2.2e-8
    return x, q


@pytest.mark.parametrize("n", [2, 3, 7, 16])
def test_field_brute_force_50_digits(n):
    """K1: the FP64 direct sum equals the same sum carried out at 50 digits (mpmath) to a
    few ulp, for E and for the potential (self term excluded)."""
    x, q = _rand_state(n, n)
    eps2 = (7.854e-4) ** 2
    E, phi = oracle.coulomb_field(x, q, eps2)
    for i in range(n):
        ex = [mpmath.mpf(0)] * 3
        ph = mpmath.mpf(0)
        for j in range(n):
            if j == i:
                continue
            d = [mpmath.mpf(x[i, k]) - mpmath.mpf(x[j, k]) for k in range(3)]
            r2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2 + mpmath.mpf(eps2)
            s = mpmath.mpf(q[j]) / (r2 * mpmath.sqrt(r2))
            for k in range(3):
                ex[k] += s * d[k]
            ph += mpmath.mpf(q[j]) / mpmath.sqrt(r2)
        nrm = float(mpmath.sqrt(sum(v**2 for v in ex)))
        scale = sum(abs(q[j]) / ((np.sum((x[i] - x[j]) ** 2) + eps2)) for j in range(n) if j != i)
        for k in range(3):
            assert abs(E[i, k] - float(ex[k])) <= 8 * 2.0**-52 * scale + 1e-300
        pscale = sum(abs(q[j]) / math.sqrt(np.sum((x[i] - x[j]) ** 2) + eps2) for j in range(n) if j != i)
        assert abs(phi[i] - float(ph)) <= 8 * 2.0**-52 * pscale
        assert nrm >= 0.0


def test_field_is_minus_gradient_of_potential():
    """E = -grad phi: central differences of the oracle's potential at a displaced target
    reproduce its field (fixes the force law's sign and exponent against the potential's)."""
    x, q = _rand_state(12, 3)
    eps2 = (7.854e-4) ** 2
    E, _ = oracle.coulomb_field(x, q, eps2)
    h = 1e-6
    for i in [0, 5, 11]:
        g = np.zeros(3)
        for k in range(3):
            xp = x.copy()
            xm = x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            # potential at i from the others only (phi excludes the self term)
            _, pp = oracle.coulomb_field(xp, q, eps2)
            _, pm = oracle.coulomb_field(xm, q, eps2)
            g[k] = -(pp[i] - pm[i]) / (2 * h)
        assert np.allclose(g, E[i], rtol=1e-6, atol=1e-9 * np.abs(E[i]).max())


def test_field_coulomb_limit_and_softening_core():
    """One source of charge Q at the origin: far away the field is Q r / r^3 (Coulomb, with
    the kappa that test_coulomb_coupling pins); at the centre of the Plummer core the
    potential is Q / eps."""
    eps = 1e-3
    x = np.array([[0.0, 0.0, 0.0], [0.3, -0.4, 1.2]])
    q = np.array([2.0, 0.0])
    E, phi = oracle.coulomb_field(x, q, eps * eps)
    r = x[1]
    rn = np.linalg.norm(r)
    assert np.allclose(E[1], 2.0 * r / rn**3, rtol=1e-6)
    x2 = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    E2, phi2 = oracle.coulomb_field(x2, q, eps * eps)
    assert phi2[1] == pytest.approx(2.0 / eps, rel=1e-15)
    assert np.all(E2[1] == 0.0)


def _two_body(dt, t_end, eps_nm=0.0):
    lam = 0.8
    c = Cluster(species="Ar", r0_nm=1.0, n_ion=2, capacity=2, z_init=1, laser=Laser(envelope="flat"))
    run = Run(dt=dt, ionize=False, diag_every=0, softening_nm=eps_nm)
    p = oracle.make_params(c, run, weight=1.0, a0=0.0)
    d0 = 0.01
    x = np.array([[-d0 / 2, 0, 0], [d0 / 2, 0, 0]])
    sim = oracle.Sim(p, 2, x, np.zeros((2, 3)), np.array([1, 1], np.int8))
    sim.start()
    nst = int(round(t_end / dt))
    sim.run(nst)
    xs = sim.positions()
    return p, d0, xs[1, 0] - xs[0, 0], nst * dt


def _two_body_time_of_separation(p, d0, d):
    """Non-relativistic, unsoftened repulsion of two equal charges q from rest at d0:
    t(d) = sqrt(mu d0^3 / (2 kappa q^2)) [sqrt(s(s-1)) + ln(sqrt(s) + sqrt(s-1))], s = d/d0."""
    q = p.weight * 1.0
    m = p.weight * p.mass_ion
    mu = m / 2.0
    s = d / d0
    return math.sqrt(mu * d0**3 / (2.0 * p.kappa * q * q)) * (math.sqrt(s * (s - 1.0)) +
                                                             math.log(math.sqrt(s) + math.sqrt(s - 1.0)))


def test_two_body_coulomb_explosion_second_order():
    """K2: separation of a two-body Coulomb explosion vs the closed form; the error falls
    about 4x per halving of dt (second-order leap-frog)."""
    errs = []
    for dt in [0.8, 0.4, 0.2]:
        p, d0, d, t = _two_body(dt, 160.0)
        errs.append(abs(_two_body_time_of_separation(p, d0, d) - t))
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0
    assert errs[2] < 1e-3


def test_two_body_energy_relation_softened():
    """K2 (energy): exact relativistic relation for the softened pair,
    2 M (gamma - 1) = kappa q^2 [(d0^2+eps^2)^-1/2 - (d^2+eps^2)^-1/2], to O(dt^2)."""
    lam = 0.8
    eps = units.nm_to_norm(0.1, lam)
    out = []
    for dt in [0.4, 0.2]:
        c = Cluster(species="Ar", r0_nm=1.0, n_ion=2, capacity=2, laser=Laser(envelope="flat"))
        p = oracle.make_params(c, Run(dt=dt, ionize=False, diag_every=1, softening_nm=0.1), weight=1.0,
                               a0=0.0)
        d0 = 0.003
        x = np.array([[-d0 / 2, 0, 0], [d0 / 2, 0, 0]])
        sim = oracle.Sim(p, 2, x, np.zeros((2, 3)), np.array([1, 1], np.int8))
        sim.start()
        rec = sim.run(int(round(80.0 / dt)))
        # KE at integer time n from the averaged gamma (record 6) vs PE from separation at n
        r = rec[-1]
        xs = sim.positions()
        # separation at step n: undo the last drift using the record's time; use PE record instead
        pe = r[oracle.R_PE]
        pe0 = p.kappa / math.sqrt(d0 * d0 + eps * eps)
        out.append(abs(r[oracle.R_KE_BAR] + pe - pe0) / pe0)
    assert out[1] < out[0] / 3.0
    assert out[1] < 1e-6


def _figure8_closed_form(a, t_target, eta0=math.pi / 2):
    """Electron from rest in a plane wave A_x = a cos(eta), eta = t - z:
    x = a (sin eta - sin eta0), z = (a^2/2)[(eta - eta0)/2 + (sin 2eta - sin 2eta0)/4],
    t = eta + z; solve for eta by Newton."""
    def zf(eta):
        return 0.5 * a * a * ((eta - eta0) / 2.0 + (math.sin(2 * eta) - math.sin(2 * eta0)) / 4.0)

    eta = t_target
    for _ in range(100):
        f = eta + zf(eta) - t_target
        df = 1.0 + 0.5 * a * a * (0.5 + 0.5 * math.cos(2 * eta))
        eta -= f / df
    return a * (math.sin(eta) - math.sin(eta0)), zf(eta)


def _free_electron(phase, a, dt, t_run):
    c = Cluster(species="Ar", r0_nm=1.0, n_ion=0, capacity=1, laser=Laser(envelope="flat", phase=phase))
    run = Run(dt=dt, t0=math.pi / 2, ionize=False, diag_every=0)
    p = oracle.make_params(c, run, weight=1.0)
    p.a0 = a
    sim = oracle.Sim(p, 1, np.zeros((1, 3)), np.zeros((1, 3)), np.array([-1], np.int8))
    sim.start()
    nst = int(round(t_run / dt))
    sim.run(nst)
    return sim, math.pi / 2 + nst * dt


def test_plane_wave_figure8_second_order():
    """K3: free electron in a plane wave (flat envelope, psi = t - z) follows the closed-form
    figure-8 drift orbit; error ~dt^2."""
    a = 1.0
    errs = []
    for dt in [0.1, 0.05, 0.025]:
        sim, t = _free_electron("plane_wave", a, dt, 20.0)
        xe, ze = _figure8_closed_form(a, t)
        pos = sim.positions()[0]
        errs.append(math.hypot(pos[0] - xe, pos[2] - ze))
    for k in range(2):
        assert 3.6 < errs[k] / errs[k + 1] < 4.4
    assert errs[2] < 2.5e-3
    assert abs(sim.positions()[0][1]) == 0.0


def test_dipole_free_electron_invariants():
    """K4: in the dipole field E = a sin t x, B = a sin t y an electron from rest at t0 keeps
    gamma - p_z = 1 and p_x + p_x^3/6 = a (cos t - cos t0); both hold to O(dt^2)."""
    a = 0.7
    errs = []
    for dt in [0.1, 0.05]:
        sim, t = _free_electron("dipole", a, dt, 15.0)
        u = sim.momenta()[0]
        th = t - dt / 2  # momentum lives at the half step
        g = math.sqrt(1 + u @ u)
        e1 = abs(g - u[2] - 1.0)
        e2 = abs(u[0] + u[0] ** 3 / 6 - a * (math.cos(th) - math.cos(math.pi / 2)))
        errs.append(max(e1, e2))
    assert errs[0] / errs[1] > 3.0
    assert errs[1] < 5e-4


def _circular_orbit_error(a, dt, t_run, t0=0.3):
    """Electron started on the orbit u = a (cos t, sin t, 0) in the circularly polarized dipole
    field (flat envelope): max error of u at the last half step and of x at the last step
    against the closed form."""
    c = Cluster(species="Ar", r0_nm=1.0, n_ion=0, capacity=1,
                laser=Laser(envelope="flat", polarization="circular"))
    run = Run(dt=dt, t0=t0, ionize=False, diag_every=0)
    p = oracle.make_params(c, run, weight=1.0)
    p.a0 = a
    u0 = np.array([[a * math.cos(t0), a * math.sin(t0), 0.0]])
    sim = oracle.Sim(p, 1, np.zeros((1, 3)), u0, np.array([-1], np.int8))
    sim.start()
    nst = int(round(t_run / dt))
    sim.run(nst)
    t = t0 + nst * dt
    th = t - dt / 2
    g = math.sqrt(1.0 + a * a)
    ue = np.array([a * math.cos(th), a * math.sin(th), 0.0])
    xe = (a / g) * np.array([math.sin(t) - math.sin(t0), math.cos(t0) - math.cos(t), 0.0])
    return np.max(np.abs(sim.momenta()[0] - ue)), np.max(np.abs(sim.positions()[0] - xe))


@pytest.mark.parametrize("a", [0.3, 1.0, 3.0])
def test_circular_dipole_orbit_second_order(a):
    """Circular polarization (Eqs.(4)-(9) with phi_E = 3 pi/2, phi_B = pi/2): for an electron,
    u = a (cos t, sin t, 0) solves du/dt = -(E + v x B) exactly at any a, since du/dt = -E
    and v is parallel to B = a (cos t, sin t, 0), so gamma = sqrt(1 + a^2) stays constant and
    x = (a/gamma)(sin t - sin t0, cos t0 - cos t, 0).  The Boris orbit converges to it at
    second order in dt."""
    errs = [_circular_orbit_error(a, dt, 20.0) for dt in (0.1, 0.05, 0.025)]
    for k in range(2):
        for m in range(2):
            assert 3.6 < errs[k][m] / errs[k + 1][m] < 4.4
    assert errs[2][0] < 2e-4 * max(a, 1.0) and errs[2][1] < 1e-3


def _dipole_reference(a, u0, t0, t1):
    """Electron in the linearly polarized dipole field E = (a sin t, 0, 0), B = (0, a sin t, 0)
    from momentum u0 at the origin: du/dt = -(E + v x B), dx/dt = v, v = u / gamma, by an
    independent eighth-order Runge-Kutta integration at tight tolerance."""
    from scipy.integrate import solve_ivp

    def rhs(t, y):
        u = y[:3]
        g = math.sqrt(1.0 + u @ u)
        v = u / g
        f = a * math.sin(t)
        E = np.array([f, 0.0, 0.0])
        B = np.array([0.0, f, 0.0])
        return np.concatenate([-(E + np.cross(v, B)), v])

    out = solve_ivp(rhs, (t0, t1), np.concatenate([u0, np.zeros(3)]), method="DOP853", rtol=1e-13,
                    atol=1e-15, dense_output=True)
    return out.sol


def test_dipole_orbit_with_initial_momentum_second_order():
    """An electron that starts with momentum across the magnetic field (so the start's backward
    half kick has a v x B part) in the relativistic dipole field (a = 1): momenta at the last
    half step and positions at the last step against an independent high-order integration of
    the same equations of motion, converging at second order in dt (a first-order slip in the
    start or in the position update would show as a ratio near 2)."""
    a, t0 = 1.0, 0.3
    u0 = np.array([0.3, 0.2, 0.4])
    c = Cluster(species="Ar", r0_nm=1.0, n_ion=0, capacity=1, laser=Laser(envelope="flat"))
    errs = []
    for dt in (0.1, 0.05, 0.025):
        run = Run(dt=dt, t0=t0, ionize=False, diag_every=0)
        p = oracle.make_params(c, run, weight=1.0)
        p.a0 = a
        sim = oracle.Sim(p, 1, np.zeros((1, 3)), u0[None, :].copy(), np.array([-1], np.int8))
        sim.start()
        nst = int(round(10.0 / dt))
        sim.run(nst)
        t = t0 + nst * dt
        ref = _dipole_reference(a, u0, t0, t)
        eu = np.max(np.abs(sim.momenta()[0] - ref(t - dt / 2)[:3]))
        ex = np.max(np.abs(sim.positions()[0] - ref(t)[3:]))
        errs.append((eu, ex))
    for k in range(2):
        for m in range(2):
            assert 3.4 < errs[k][m] / errs[k + 1][m] < 4.6, (k, m, errs)
    assert errs[2][0] < 1e-3 and errs[2][1] < 1e-3


def test_ionization_survival_at_high_rate():
    """The check takes P = 1 - exp(-nu dt), not its first-order expansion: with the field set
    so that nu dt = 1 (circular polarization, flat envelope, so the rate is constant), one
    check leaves exp(-1) = 0.37 of the ions unionized (binomial count, 4.5 sigma)."""
    n_ion = 3000
    c = Cluster(species="Ar", r0_nm=20.0, n_ion=n_ion, capacity=3 * n_ion, z_init=1, z_max=2,
                laser=Laser(intensity_wcm2=1e15, envelope="flat", polarization="circular"))
    run = Run(dt=0.05, ionize=True, diag_every=0, seed=23)
    sim = oracle.Sim.from_workload(c, run, initial_state(c, 23))
    p = sim.p
    p.kappa = 0.0
    lo, hi = 1e-4, 10.0  # a0 with nu(a0) dt = 1, by bisection in log space
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if oracle.adk_rate(p.ip_au[1], 2.0, mid * p.field_au) * p.rate_scale * p.dt < 1.0:
            lo = mid
        else:
            hi = mid
    p.a0 = hi
    nu_dt = oracle.adk_rate(p.ip_au[1], 2.0, p.a0 * p.field_au) * p.rate_scale * p.dt
    assert abs(nu_dt - 1.0) < 1e-9
    sim.start()
    sim.run(1)
    surv = np.mean(sim.charges()[:n_ion] == 1)
    expect = math.exp(-1.0)
    sigma = math.sqrt(expect * (1 - expect) / n_ion)
    assert abs(surv - expect) < 4.5 * sigma, (surv, expect)


def test_ionization_survival_law_circular():
    """Circular polarization with a flat envelope keeps |E_L| = a0 at every phase, so the
    laser-only ADK rate nu is constant and an ion that may ionize once survives n checks with
    probability exp(-nu n dt) (binomial count, 4.5 sigma)."""
    n_ion = 3000
    c = Cluster(species="Ar", r0_nm=20.0, n_ion=n_ion, capacity=3 * n_ion, z_init=1, z_max=2,
                laser=Laser(intensity_wcm2=1e15, envelope="flat", polarization="circular"))
    run = Run(dt=0.05, ionize=True, diag_every=0, seed=22)
    sim = oracle.Sim.from_workload(c, run, initial_state(c, 22))
    sim.p.kappa = 0.0
    sim.start()
    nsteps = 40
    sim.run(nsteps)
    surv = np.mean(sim.charges()[:n_ion] == 1)
    p = sim.p
    nu = oracle.adk_rate(p.ip_au[1], 2.0, p.a0 * p.field_au) * p.rate_scale
    expect = math.exp(-nu * p.dt * nsteps)
    sigma = math.sqrt(expect * (1 - expect) / n_ion)
    assert 0.2 < expect < 0.8
    assert abs(surv - expect) < 4.5 * sigma


def _small_cluster(n_ion=100, seed=3, dt=0.05, ionize=False, intensity=1e17, diag_every=1,
                   envelope="flat"):
    c = Cluster(species="Ar", r0_nm=2.0, n_ion=n_ion, capacity=n_ion * 9, z_init=1, z_max=8,
                laser=Laser(intensity_wcm2=intensity, envelope=envelope))
    run = Run(dt=dt, ionize=ionize, diag_every=diag_every, seed=seed)
    st = initial_state(c, seed)
    return oracle.Sim.from_workload(c, run, st), c, run


def test_newton_third_law_and_momentum():
    """K5: sum_i w Z_i E_C,i vanishes to rounding, and with the laser off the total
    momentum stays at its start value."""
    sim, c, run = _small_cluster(intensity=1e16)
    sim.p.a0 = 0.0
    sim.start()
    rec = sim.run(50)
    for r in rec:
        assert np.linalg.norm(r[oracle.R_F:oracle.R_F + 3]) <= 1e-13 * r[oracle.R_FABS]
    p0 = rec[0][oracle.R_P:oracle.R_P + 3]
    p1 = rec[-1][oracle.R_P:oracle.R_P + 3]
    scale = np.sum(np.abs(sim.momenta()) * sim.p.mass_ion * sim.p.weight)
    assert np.linalg.norm(p1 - p0) <= 1e-12 * scale


def test_discrete_energy_identity():
    """K6: KE(n+1/2) - KE(-1/2) = W_L + W_C + spawn KE exactly up to rounding (the Boris
    energy split is exact), with ionization on."""
    sim, c, run = _small_cluster(ionize=True, intensity=3e17, diag_every=5)
    ke0 = sim.start()
    rec = sim.run(100)
    assert rec[-1][oracle.R_EVENTS] > 0
    for r in rec:
        lhs = r[oracle.R_KE_HALF] - ke0
        rhs = r[oracle.R_WL] + r[oracle.R_WC] + r[oracle.R_WSP]
        scale = abs(r[oracle.R_WL]) + abs(r[oracle.R_WC]) + r[oracle.R_WSP] + abs(ke0)
        assert abs(lhs - rhs) <= 1e-11 * scale


def _energy_drift(dt, t_end=3.0):
    sim, c, run = _small_cluster(n_ion=60, seed=11, dt=dt, intensity=1e17, diag_every=1)
    sim.start()
    rec = sim.run(int(round(t_end / dt)))
    # W_L at integer time n: mean of the cumulative values after pushes n-1 and n
    wl = rec[:, oracle.R_WL]
    wl_n = 0.5 * (wl[1:] + wl[:-1])
    etot = rec[1:, oracle.R_KE_BAR] + rec[1:, oracle.R_PE] - wl_n
    scale = np.max(np.abs(rec[1:, oracle.R_PE]))
    return np.max(np.abs(etot - etot[0])) / scale


def test_energy_bookkeeping_second_order():
    """K7: KE + PE - W_L is conserved to O(dt^2) with ionization off."""
    e = [_energy_drift(dt, t_end=1.0) for dt in (0.01, 0.005, 0.0025)]
    assert e[0] / e[1] > 3.5 and e[1] / e[2] > 3.5
    assert e[2] < 1e-4


def test_uniform_sphere_self_energy():
    """Ions uniform in a ball: E[1/|r_i - r_j|] = 6/(5 R) for two random points of a ball of
    radius R, so the pair energy is (3/5) kappa q^2 N (N-1) / R0 on average (the
    uniform-sphere energy whose 3/5 ratio the paper quotes for the deuterium case)."""
    n = 1500
    c = Cluster(species="D", r0_nm=5.0, n_ion=n, capacity=2 * n, z_init=1, laser=Laser(envelope="flat"))
    run = Run(ionize=False, diag_every=1, softening_nm=1e-4)
    st = initial_state(c, 4)
    # ions only
    st = {"x_nm": st["x_nm"][:n], "u": st["u"][:n], "Z": st["Z"][:n], "n_ion": n}
    sim = oracle.Sim.from_workload(c, run, st, weight=1.0)
    sim.p.a0 = 0.0
    _, phi = sim.field()
    pe = 0.5 * np.sum(phi)  # w = Z = 1
    r0 = units.nm_to_norm(5.0, 0.8)
    expect = 0.6 * sim.p.kappa * n * (n - 1) / r0
    assert pe == pytest.approx(expect, rel=0.02)


def test_uniform_sphere_explosion_three_fifths():
    """Pure Coulomb explosion of a uniform ion sphere expands self-similarly, so mean ion
    energy / maximum ion energy stays at 3/5 (the paper's D_8007 ratio, Sec. III)."""
    n = 800
    c = Cluster(species="D", r0_nm=3.0, n_ion=n, capacity=2 * n, z_init=1, laser=Laser(envelope="flat"))
    run = Run(dt=2.0, ionize=False, diag_every=0, softening_nm=0.01)
    st = initial_state(c, 9)
    st = {"x_nm": st["x_nm"][:n], "u": st["u"][:n], "Z": st["Z"][:n], "n_ion": n}
    sim = oracle.Sim.from_workload(c, run, st, weight=1.0)
    sim.p.a0 = 0.0
    sim.start()
    sim.run(1500)
    u = sim.momenta()
    g = np.sqrt(1 + np.sum(u * u, axis=1))
    ke = g - 1.0
    ratio = ke.mean() / np.quantile(ke, 0.995)
    assert ratio == pytest.approx(0.6, abs=0.03)


def test_ionization_survival_law():
    """K9: with the laser-only field, an ion that may ionize once survives n checks with
    probability exp(-sum_k nu_k dt) (P = 1 - exp(-nu dt) per step, alpha uniform in (0,1]).
    The count of surviving ions is binomial; test at 4.5 sigma."""
    n_ion = 3000
    c = Cluster(species="Ar", r0_nm=20.0, n_ion=n_ion, capacity=2 * n_ion + n_ion, z_init=1, z_max=2,
                laser=Laser(intensity_wcm2=1.25e15, envelope="flat"))
    run = Run(dt=0.05, ionize=True, diag_every=0, seed=21)
    st = initial_state(c, 21)
    sim = oracle.Sim.from_workload(c, run, st)
    sim.p.kappa = 0.0  # no Coulomb forces: ions must not move and the field is the laser's
    sim.start()
    nsteps = 40
    sim.run(nsteps)
    Z = sim.charges()[:n_ion]
    surv = np.mean(Z == 1)
    p = sim.p
    lam_sum = 0.0
    for k in range(nsteps):
        t = p.t0 + k * p.dt
        E, _ = oracle.laser(p, t)
        nu = oracle.adk_rate(p.ip_au[1], 2.0, abs(E[0]) * p.field_au) * p.rate_scale
        lam_sum += -math.log1p(-(-math.expm1(-nu * p.dt)))
    expect = math.exp(-lam_sum)
    sigma = math.sqrt(expect * (1 - expect) / n_ion)
    assert 0.2 < expect < 0.8
    assert abs(surv - expect) < 4.5 * sigma


def test_spawned_electrons_conserve_charge_and_sit_at_offset():
    """Each ionization adds one electron (charge conservation, total Z sum unchanged) placed
    at the offset distance from its parent ion with the parent's momentum; spawned
    electrons are appended in ascending parent order."""
    n_ion = 400
    c = Cluster(species="Ar", r0_nm=5.0, n_ion=n_ion, capacity=n_ion * 9, z_init=1, z_max=8,
                laser=Laser(intensity_wcm2=3e16, envelope="flat"))
    run = Run(dt=0.05, t0=math.pi / 2, ionize=True, diag_every=0, seed=2)
    st = initial_state(c, 2)
    sim = oracle.Sim.from_workload(c, run, st)
    sim.start()
    Z0 = sim.charges().copy()
    n0 = sim.N
    sim.run(1)
    n1 = sim.N
    Z1 = sim.charges()
    assert n1 > n0
    assert int(np.sum(Z1.astype(np.int64))) == int(np.sum(Z0.astype(np.int64)))
    parents = np.nonzero(Z1[:n_ion] != Z0[:n_ion])[0]
    assert len(parents) == n1 - n0
    x = sim.positions()
    u = sim.momenta()
    for k, ip in enumerate(parents):
        e = n0 + k
        assert Z1[e] == -1
        assert np.linalg.norm(x[e] - x[ip]) == pytest.approx(sim.p.delta, rel=1e-9)
        assert np.array_equal(u[e], u[ip])


def test_capacity_overflow_drops_spawns():
    """A full cluster drops further spawns (counted) and leaves the parent's charge as is."""
    n_ion = 50
    c = Cluster(species="Ar", r0_nm=3.0, n_ion=n_ion, capacity=n_ion * 2 + 3, z_init=1, z_max=8,
                laser=Laser(intensity_wcm2=1e18, envelope="flat"))
    run = Run(dt=0.05, t0=math.pi / 2, ionize=True, diag_every=1, seed=5)
    st = initial_state(c, 5)
    sim = oracle.Sim.from_workload(c, run, st)
    sim.start()
    sim.run(3)
    assert sim.N == c.capacity
    assert sim.counters[0] > 0
    Z = sim.charges()
    assert int(np.sum(Z.astype(np.int64))) == 0


def test_record_counts_consistent():
    """Record bookkeeping: ion and electron counts, charge histogram, mean charge and the
    absorbed energy per atom (laser work in eV over Eq.(1)'s atom count) agree with the
    state they describe."""
    c, run = small_ar()
    st = initial_state(c, run.seed)
    sim = oracle.Sim.from_workload(c, run, st)
    sim.start()
    rec = sim.run(30)
    r = rec[-1]
    Z = sim.charges()
    nion = np.sum(Z >= 0)
    assert r[oracle.R_NION] == nion and r[oracle.R_NEL] == np.sum(Z < 0)
    assert r[oracle.R_N] == sim.N
    assert np.sum(r[oracle.R_ZHIST:oracle.R_ZHIST + 17]) == nion
    zh = r[oracle.R_ZHIST:oracle.R_ZHIST + 17]
    assert r[oracle.R_MEANZ] == pytest.approx(np.sum(zh * np.arange(17)) / nion, rel=1e-14)
    natoms = units.n_atoms(c.r0_nm, 2.40)
    assert r[oracle.R_ABS_EV] == pytest.approx(r[oracle.R_WL] * units.MEC2_EV / natoms, rel=1e-14)
    assert r[oracle.R_T] == pytest.approx(run.t0 + r[oracle.R_STEP] * run.dt, rel=1e-15)


def _d_ion_u(ev):
    """Momentum u = gamma v of a deuteron with kinetic energy ev (50 digits)."""
    from workloads.species import SPECIES
    m = mpmath.mpf(SPECIES["D"]["mass_u"]) * mpmath.mpf(units.U_PER_ME)
    g = 1 + mpmath.mpf(ev) / (m * mpmath.mpf(units.MEC2_EV))
    return float(mpmath.sqrt(g * g - 1))


def test_detectors_free_streaming():
    """Ion detectors (Sec. III anisotropy study): with no forces every ion streams at its start
    momentum, so each one crossing the detector distance D is counted once, at its exact
    start energy, by the axes whose direction its path makes an angle below 30 degrees with;
    ions that never reach D and electrons are not counted.  Energies sit mid-bin."""
    c = Cluster(species="D", r0_nm=1.0, n_ion=8, capacity=9, z_init=1, laser=Laser(envelope="flat"))
    run = Run(dt=0.5, ionize=False, diag_every=0)
    deg = math.pi / 180
    # (direction, kinetic energy in eV, expected axes)
    ions = [((math.cos(29 * deg), math.sin(29 * deg), 0.0), 150.0, {0}),
            ((math.cos(31 * deg), -math.sin(31 * deg), 0.0), 3.1e3, set()),
            ((math.sin(29 * deg), -math.cos(29 * deg), 0.0), 47e3, {1}),
            ((0.0, math.sin(20 * deg), math.cos(20 * deg)), 830e3, {2}),
            ((-1.0, 0.0, 0.0), 2.2e6, {0}),
            ((0.0, 0.0, -1.0), 0.55, {2}),
            ((1 / math.sqrt(3), 1 / math.sqrt(3), 1 / math.sqrt(3)), 12e3, set())]
    x = np.zeros((9, 3))
    u = np.zeros((9, 3))
    Z = np.ones(9, np.int8)
    for i, (d, ev, _) in enumerate(ions):
        x[i] = 0.3e-3 * np.array(d)
        u[i] = _d_ion_u(ev) * np.array(d)
    x[7] = (0.0, 0.02, 0.0)          # ion at rest inside D: never reaches it
    x[8] = (0.001, 0.0, 0.0)         # electron moving out along x: not an ion
    u[8] = (0.05, 0.0, 0.0)
    Z[8] = -1
    p = oracle.make_params(c, run, weight=1.0)
    p.kappa = 0.0
    p.a0 = 0.0
    sim = oracle.Sim(p, 9, x, u, Z)
    D = 0.025
    sim.enable_detectors(D, 30.0)
    sim.start()
    sim.run(8000)  # the slowest ion (0.55 eV) needs about 7000 steps
    counts, edges = sim.iedf()
    assert counts[0].sum() == 7 and sim.det_seen[7] == 0 and sim.det_seen[8] == 0
    want = np.zeros((4, oracle.DET_SLOTS), np.int64)
    for d, ev, axes in ions:
        slot = int(np.searchsorted(edges, ev, side="right"))
        lo = edges[slot - 1] if slot > 0 else 0.0
        hi = edges[slot] if slot <= oracle.DET_BINS else np.inf
        assert lo * 1.02 < ev < hi / 1.02  # mid-bin: the slot does not depend on rounding
        want[0, slot] += 1
        for a in axes:
            want[a + 1, slot] += 1
    assert np.array_equal(counts, want)
    assert counts[0, 0] == 1 and counts[0, oracle.DET_BINS + 1] == 1  # underflow and overflow


def test_iedf_uniform_sphere_explosion():
    """A uniform sphere of ions explodes with shells in order: a shell starting at r0 that
    encloses N_enc ions has, on reaching the detectors at D = 9 R0, the kinetic energy
    kappa Z^2 w N_enc (1/r0 - 1/D) per real ion.  The detected histogram matches these
    energies of the same ions (Kolmogorov distance < 0.04), every ion is detected, and the
    per-axis counts match the solid-angle fraction 1 - cos 30 deg of an isotropic explosion."""
    n = 800
    c = Cluster(species="D", r0_nm=3.0, n_ion=n, capacity=2 * n, z_init=1, laser=Laser(envelope="flat"))
    run = Run(dt=2.0, ionize=False, diag_every=0, softening_nm=0.01)
    st = initial_state(c, 9)
    st = {"x_nm": st["x_nm"][:n], "u": st["u"][:n], "Z": st["Z"][:n], "n_ion": n}
    sim = oracle.Sim.from_workload(c, run, st)
    sim.p.a0 = 0.0
    x0 = sim.positions().copy()
    D = 9.0 * sim.r0_norm
    sim.enable_detectors(D, 30.0)
    sim.start()
    sim.run(3000)
    counts, edges = sim.iedf()
    assert counts[0].sum() == n
    r0 = np.linalg.norm(x0, axis=1)
    nenc = np.empty(n)
    nenc[np.argsort(r0)] = np.arange(n)
    p = sim.p
    e = p.kappa * p.weight * nenc * (1.0 / r0 - 1.0 / D) * p.mec2_ev
    pred = np.bincount(np.searchsorted(edges, e, side="right"), minlength=oracle.DET_SLOTS)
    ks = np.max(np.abs(np.cumsum(counts[0]) - np.cumsum(pred))) / n
    assert ks < 0.04
    f = 1.0 - math.cos(math.pi / 6)
    sigma = math.sqrt(f * (1 - f) / n)
    for a in range(3):
        assert abs(counts[a + 1].sum() / n - f) < 4.5 * sigma


def test_min_image_field_brute_force():
    """Periodic boundaries (Sec. II, cube of side L): the field and potential with every pair
    taken through the nearest of the 27 periodic copies of the partner, enumerated and
    summed at 50 digits, match the oracle's minimum-image sum."""
    rng = np.random.default_rng(17)
    n, L, eps = 12, 0.05, 1e-3
    x = rng.uniform(-L / 2, L / 2, (n, 3))
    q = rng.choice([-1.0, 1.0, 3.0], n) * 2.2e-8
    E, phi = oracle.coulomb_field(x, q, eps * eps, box=L)
    shifts = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    for i in range(n):
        acc = [mpmath.mpf(0)] * 4
        scale = mpmath.mpf(0)
        for j in range(n):
            if j == i:
                continue
            best = None
            for sh in shifts:
                d = [mpmath.mpf(x[i][k]) - mpmath.mpf(x[j][k]) - sh[k] * mpmath.mpf(L) for k in range(3)]
                r2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
                if best is None or r2 < best[0]:
                    best = (r2, d)
            r2, d = best
            s = r2 + mpmath.mpf(eps) ** 2
            inv = 1 / mpmath.sqrt(s)
            for k in range(3):
                acc[k] += mpmath.mpf(q[j]) * d[k] * inv ** 3
            acc[3] += mpmath.mpf(q[j]) * inv
            scale += abs(mpmath.mpf(q[j])) * inv ** 2
        for k in range(3):
            assert abs(E[i][k] - float(acc[k])) <= 1e-13 * float(scale)
        assert abs(phi[i] - float(acc[3])) <= 1e-13 * float(scale) * L


def _streaming_electron(boundary, t_switch, nsteps):
    c = Cluster(species="Ar", r0_nm=1.0, n_ion=0, capacity=1, laser=Laser(envelope="flat"))
    run = Run(dt=0.5, ionize=False, diag_every=0, boundary=boundary, box_r0=2.0, t_switch=t_switch)
    p = oracle.make_params(c, run, weight=1.0)
    p.a0 = 0.0
    u = np.array([0.3, 0.2, -0.1])
    x0 = np.array([0.004, -0.006, 0.002])
    sim = oracle.Sim(p, 1, x0[None, :], u[None, :], np.array([-1], np.int8))
    sim.start()
    sim.run(nsteps)
    v = u / math.sqrt(1.0 + u @ u)
    return sim.positions()[0], x0, v, p


@pytest.mark.parametrize("boundary", ["periodic", "mixed"])
def test_free_streaming_through_the_box(boundary):
    """A particle streaming freely leaves the periodic cube through one face and re-enters
    through the opposite one: after m periodic steps it sits at ((x0 + m dt v + L/2) mod L)
    - L/2; in the mixed mode the open steps after the switch then carry it on unwrapped."""
    nsteps = 400
    m = nsteps if boundary == "periodic" else 250
    pos, x0, v, p = _streaming_electron(boundary, (m - 0.5) * 0.5, nsteps)
    L = p.box
    assert L > 0 and nsteps * 0.5 * np.max(np.abs(v)) > 3 * L  # several crossings
    want = np.mod(x0 + m * p.dt * v + L / 2, L) - L / 2 + (nsteps - m) * p.dt * v
    assert np.max(np.abs(pos - want)) <= 1e-12 * L * nsteps


def test_periodic_momentum_newton3_and_box():
    """In a periodic cube barely wider than the cluster the minimum-image forces stay pairwise
    opposite: sum_i w Z_i E_C,i vanishes to rounding and, with the laser off, the total
    momentum stays at its start value; every particle stays inside the cube, spawned
    electrons included (ionization on)."""
    c = Cluster(species="Ar", r0_nm=2.0, n_ion=100, capacity=900, z_init=1, z_max=8,
                laser=Laser(intensity_wcm2=3e17, envelope="flat"))
    run = Run(dt=0.05, ionize=True, diag_every=1, seed=3, boundary="periodic", box_r0=2.5)
    sim = oracle.Sim.from_workload(c, run, initial_state(c, 3))
    sim.p.a0 = 0.0
    sim.start()
    rec = sim.run(60)
    for r in rec:
        assert np.linalg.norm(r[oracle.R_F:oracle.R_F + 3]) <= 1e-13 * r[oracle.R_FABS]
    p0, p1 = rec[0][oracle.R_P:oracle.R_P + 3], rec[-1][oracle.R_P:oracle.R_P + 3]
    scale = np.sum(np.abs(sim.momenta()) * sim.p.mass_ion * sim.p.weight)
    assert np.linalg.norm(p1 - p0) <= 1e-12 * scale
    L = sim.p.box
    assert np.all(np.abs(sim.positions()) <= L / 2)
    # the laser on: ionization spawns electrons; they and every other particle stay inside
    sim2 = oracle.Sim.from_workload(c, run, initial_state(c, 3))
    sim2.start()
    rec2 = sim2.run(60)
    assert rec2[-1][oracle.R_EVENTS] > 0 and sim2.N > 200
    assert np.all(np.abs(sim2.positions()) <= L / 2)
    lhs = rec2[-1][oracle.R_KE_HALF] - sim2.ke_start
    rhs = rec2[-1][oracle.R_WL] + rec2[-1][oracle.R_WC] + rec2[-1][oracle.R_WSP]
    assert abs(lhs - rhs) <= 1e-11 * (abs(rec2[-1][oracle.R_WL]) + abs(rec2[-1][oracle.R_WC]) + abs(sim2.ke_start))


def test_sampled_field_equals_full_sum():
    """The sampled evaluation (targets listed by index, used for the large-state checks) gives the
    full direct sum's values at those targets bit for bit, E and potential, including the first
    and last index and a repeated one."""
    x, q = _rand_state(300, 11)
    eps2 = (7.854e-4) ** 2
    E, phi = oracle.coulomb_field(x, q, eps2)
    idx = np.array([0, 299, 17, 17, 150, 3, 298, 42])
    Es, phis = oracle.coulomb_field_at(x, q, eps2, idx)
    assert np.array_equal(Es, E[idx]) and np.array_equal(phis, phi[idx])


def test_local_ofi_without_coulomb_coupling_is_laser_only():
    """With the Coulomb coupling switched off the local field at an ion is the laser's, so the
    LOCAL choice (|E_C + E_L|) must take exactly the laser-only decisions: identical charges,
    positions and records over a run with many ionizations (linear and circular polarization)."""
    for pol in ("linear_x", "circular"):
        c = Cluster(species="Ar", r0_nm=2.5, n_ion=400, capacity=4000, z_init=1, z_max=8,
                    laser=Laser(intensity_wcm2=2e16, envelope="flat", polarization=pol))
        out = []
        for ofi in ("laser_only", "local"):
            run = Run(dt=0.05, t0=math.pi / 2, ionize=True, ofi_field=ofi, diag_every=5, seed=4)
            sim = oracle.Sim.from_workload(c, run, initial_state(c, 4))
            sim.p.kappa = 0.0
            sim.start()
            rec = sim.run(60)
            out.append((sim.charges(), sim.positions(), rec))
        assert out[0][2][-1][oracle.R_EVENTS] > 50
        for a, b in zip(out[0], out[1]):
            assert np.array_equal(a, b)


def test_local_ofi_survival_law_around_frozen_sources():
    """LOCAL ionization is driven by |E_C + E_L| at the atom.  n neutral Ar atoms (Z = 0, may
    ionize once) each have one Ar+ source at distance d along +x; the pairs sit 1 c/w apart on a
    line, so the field of the other pairs changes E_C by under 1e-5 relative.  Before its
    ionization a neutral atom neither moves nor makes a field, so E_C at it is the softened
    Coulomb field of its source, -kappa w d / (d^2 + eps^2)^{3/2} x^, and with a flat laser from
    t = 0 (E_L = a sin t x^, a = E_C / 2) the atom survives n checks with probability
    exp(-dt sum_k nu(|E_C + a sin t_k|)).  Binomial count at 4.5 sigma; the laser-only field
    (a/2 here) and a flipped sign of E_L predict survivals many sigma away."""
    n = 3000
    d = 1.0e-3
    c = Cluster(species="Ar", r0_nm=2.5, n_ion=2 * n, capacity=4 * n, z_init=0, z_max=1,
                laser=Laser(intensity_wcm2=0.0, envelope="flat"))
    run = Run(dt=0.05, t0=0.0, ionize=True, ofi_field="local", diag_every=0, seed=8)
    x = np.zeros((2 * n, 3))
    x[:n, 0] = np.arange(n) * 1.0
    x[n:, 0] = x[:n, 0] + d
    Z = np.concatenate([np.zeros(n, np.int8), np.ones(n, np.int8)])
    p = oracle.make_params(c, run, weight=1.0)
    ec = p.kappa * 1.0 * d / (d * d + p.eps2) ** 1.5  # |E_C| at an atom, pointing along -x
    nsteps = 40
    ip = p.ip_au[0]

    def survival(fields):
        lam = sum(oracle.adk_rate(ip, 1.0, f * p.field_au) * p.rate_scale for f in fields) * p.dt
        return math.exp(-lam)
    ts = [k * run.dt for k in range(nsteps)]
    shape = [abs(-1.0 + 0.5 * math.sin(t)) for t in ts]  # |E_C + E_L| / |E_C| with a = |E_C| / 2
    # the weight (source strength) that makes the expected survival 1/2
    lo, hi = 0.1, 100.0
    for _ in range(200):
        w = math.sqrt(lo * hi)
        if survival([ec * w * f for f in shape]) > 0.5:
            lo = w
        else:
            hi = w
    p = oracle.make_params(c, run, weight=w)
    ec *= w
    p.a0 = 0.5 * ec
    sim = oracle.Sim(p, c.capacity, x, np.zeros_like(x), Z)
    sim.start()
    sim.run(nsteps)
    surv = np.mean(sim.charges()[:n] == 0)
    expect = survival([abs(-ec + p.a0 * math.sin(t)) for t in ts])
    sigma = math.sqrt(expect * (1 - expect) / n)
    assert 0.15 < expect < 0.85
    assert abs(surv - expect) < 4.5 * sigma, (surv, expect, sigma)
    for wrong in (survival([abs(p.a0 * math.sin(t)) for t in ts]),        # laser only
                  survival([abs(-ec - p.a0 * math.sin(t)) for t in ts])):  # E_C - E_L
        assert abs(wrong - expect) > 15 * sigma


def _philox_block(key, ctr):
    """Philox4x64-10 block at counter ctr from numpy's own implementation (which increments the
    counter before each block, so it starts one below)."""
    c = list(ctr)
    for k in range(4):  # counter - 1 with borrow
        c[k] = (c[k] - 1) % 2**64
        if c[k] != 2**64 - 1:
            break
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(c, dtype=np.uint64))
    return [int(v) for v in g.random_raw(4)]


def test_initial_placement_counters_and_geometry():
    """O1 initial placement (Sec. II: atoms at random inside R0, lumped into ion macroparticles,
    each with z_init electrons next to it).  The draws are numpy's Philox blocks at counter
    (i, 0, 0, 0) for ion i and (e, 0, 1, 0) for electron e; the ion radius is R0 u^{1/3}, the
    directions have polar cosine 2u - 1 and azimuth 2 pi u, the electrons sit at delta from
    their parent (ions first, then electrons by parent).  Values within a few ulp of R0."""
    seed, cl, n_ion, z_init = 3, 5, 64, 2
    r0, delta = 0.0196, 7.854e-5
    x, Z = oracle.init_cluster(seed, cl, n_ion, z_init, r0, delta)
    assert x.shape == (n_ion * 3, 3)
    assert np.all(Z[:n_ion] == z_init) and np.all(Z[n_ion:] == -1)
    u01 = lambda w: ((w >> 11) + 1) * 2.0**-53

    def direction(uc, up):
        ct = 2.0 * uc - 1.0
        st = math.sqrt(max(0.0, 1.0 - ct * ct))
        return np.array([st * math.cos(2 * math.pi * up), st * math.sin(2 * math.pi * up), ct])
    for i in range(n_ion):
        w = _philox_block((seed, cl), (i, 0, 0, 0))
        xi = r0 * u01(w[0]) ** (1.0 / 3.0) * direction(u01(w[1]), u01(w[2]))
        assert np.max(np.abs(x[i] - xi)) <= 8 * 2.0**-52 * r0
        for k in range(z_init):
            e = i * z_init + k
            we = _philox_block((seed, cl), (e, 0, 1, 0))
            xe = x[i] + delta * direction(u01(we[0]), u01(we[1]))
            assert np.max(np.abs(x[n_ion + e] - xe)) <= 8 * 2.0**-52 * r0


def test_initial_placement_distribution():
    """Uniform in the ball: (r/R0)^3, the polar cosine and the azimuth of the ions are uniform, and
    so are the polar cosine and azimuth of the electron offsets, whose length is delta
    (Kolmogorov-Smirnov, 20k ions; p > 1e-4); different clusters and seeds draw differently."""
    from scipy import stats
    n_ion = 20000
    r0, delta = 0.05, 1e-4
    x, Z = oracle.init_cluster(0, 0, n_ion, 1, r0, delta)
    ions = x[:n_ion]
    r = np.linalg.norm(ions, axis=1)
    assert r.max() <= r0 * (1 + 1e-15)
    off = x[n_ion:] - ions
    ln = np.linalg.norm(off, axis=1)
    assert np.max(np.abs(ln - delta)) <= 1e-9 * delta
    for sample, cdf in (((r / r0) ** 3, stats.uniform(0, 1).cdf), (ions[:, 2] / r, stats.uniform(-1, 2).cdf),
                        (np.arctan2(ions[:, 1], ions[:, 0]) % (2 * np.pi), stats.uniform(0, 2 * np.pi).cdf),
                        (off[:, 2] / ln, stats.uniform(-1, 2).cdf),
                        (np.arctan2(off[:, 1], off[:, 0]) % (2 * np.pi), stats.uniform(0, 2 * np.pi).cdf)):
        assert stats.kstest(sample, cdf).pvalue > 1e-4
    x1, _ = oracle.init_cluster(0, 1, 100, 1, r0, delta)
    x2, _ = oracle.init_cluster(1, 0, 100, 1, r0, delta)
    assert not np.array_equal(x1, x[:100]) and not np.array_equal(x2, x[:100])


def _ci_cloud(seed=31, n_ion=3000, n_e=2000, t_ev=100.0, surv=0.5, nsteps=40):
    """Ions Ar+ at rest within R0/4 and a cloud of electrons within R0/2 whose momenta all have
    the magnitude of kinetic energy 3 t_ev / 2 (temperature t_ev), no laser and no Coulomb
    coupling; spawned electrons land 2.5 R0 away, outside the sphere.  The weight is chosen so
    that the collisional rate gives survival `surv` after nsteps steps."""
    from scipy.integrate import quad
    from workloads.species import SPECIES
    r0_nm = 100.0
    c = Cluster(species="Ar", r0_nm=r0_nm, n_ion=n_ion, capacity=2 * n_ion + n_e, z_init=1, z_max=2,
                electron_offset_nm=2.5 * r0_nm, laser=Laser(intensity_wcm2=0.0, envelope="flat"))
    run = Run(dt=0.05, ionize=True, collisional=True, diag_every=0, seed=seed)
    me, ev = 9.1093837015e-31, 1.602176634e-19
    P = SPECIES["Ar"]["ip_ev"][1]
    q = SPECIES["Ar"]["outer_q"][1]

    def f(E):
        sigma = 4.5e-14 * q * math.log(E / P) / (E * P)
        return sigma * math.sqrt(2.0 * E * ev / me) * 100.0 * 2.0 * math.sqrt(E / math.pi) * t_ev ** -1.5 \
            * math.exp(-E / t_ev)
    sv = quad(f, P, P + 60 * t_ev, limit=400, epsrel=1e-12)[0]
    s_unit = 0.8e-6 / (2 * math.pi * units.C_LIGHT)
    nu = -math.log(surv) / (nsteps * run.dt * s_unit)
    vol = 4.0 / 3.0 * math.pi * (r0_nm * 1e-7) ** 3
    w = nu / sv * vol / n_e
    rng = np.random.default_rng(seed)

    def ball(n, r):
        v = rng.normal(size=(n, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        return v * (r * rng.random(n) ** (1 / 3))[:, None]
    r0 = units.nm_to_norm(r0_nm, 0.8)
    x = np.concatenate([ball(n_ion, r0 / 4), ball(n_e, r0 / 2)])
    g = 1.0 + 1.5 * t_ev / units.MEC2_EV
    u = np.concatenate([np.zeros((n_ion, 3)), ball(n_e, 1.0)])
    u[n_ion:] *= (math.sqrt(g * g - 1.0) / np.linalg.norm(u[n_ion:], axis=1))[:, None]
    Z = np.concatenate([np.ones(n_ion, np.int8), -np.ones(n_e, np.int8)])
    return c, run, x, u, Z, w, nu, s_unit


@pytest.mark.parametrize("t_ev", [10.0, 100.0])
def test_collisional_survival_law(t_ev):
    """With the collisional rate on and nothing else changing (frozen cloud), an Ar+ ion inside
    the sphere survives n steps with probability exp(-n_e <sigma v> n dt); <sigma v> here is the
    numerical Maxwellian average of the Lotz cross-section, n_e the cloud's real electrons per
    volume of the sphere.  Binomial count at 4.5 sigma.  At 10 eV (below the 27.6 eV binding
    energy) the rate changes steeply with the temperature, at 100 eV little."""
    c, run, x, u, Z, w, nu, s_unit = _ci_cloud(t_ev=t_ev)
    p = oracle.make_params(c, run, weight=w)
    p.kappa = 0.0
    sim = oracle.Sim(p, c.capacity, x, u, Z)
    sim.start()
    nsteps = 40
    sim.run(nsteps)
    n_ion = c.n_ion
    surv = np.mean(sim.charges()[:n_ion] == 1)
    expect = math.exp(-nu * nsteps * run.dt * s_unit)
    sigma = math.sqrt(expect * (1 - expect) / n_ion)
    assert 0.3 < expect < 0.7
    assert abs(surv - expect) < 4.5 * sigma
    # spawned electrons sit outside the sphere, so they did not change the estimate
    xs = sim.positions()[n_ion + 2000:]
    assert np.all(np.linalg.norm(xs, axis=1) > units.nm_to_norm(c.r0_nm, 0.8))
    # without the collisional term nothing ionizes (no laser)
    p0 = oracle.make_params(c, dataclasses.replace(run, collisional=False), weight=w)
    p0.kappa = 0.0
    sim0 = oracle.Sim(p0, c.capacity, x, u, Z)
    sim0.start()
    sim0.run(nsteps)
    assert np.all(sim0.charges()[:n_ion] == 1)


def test_native_build_takes_the_same_arithmetic(tmp_path):
    """The stronger CPU timing builds the oracle's source again with -O3 -march=native; with
    contraction and fast math still off it must reproduce the plain build bit for bit (the small
    argon run with ionization and diagnostics, 20 steps)."""
    c, run = small_ar()
    st = initial_state(c, run.seed)

    def states():
        s = oracle.Sim.from_workload(c, run, st)
        s.start()
        rec = s.run(20)
        return s.positions(), s.momenta(), s.charges(), rec

    ref = states()
    with oracle.library(oracle.build_native(str(tmp_path / "liblc_oracle_native.so"))):
        nat = states()
    for a, b in zip(ref, nat):
        assert np.array_equal(a, b)
