"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This module generates inputs only: cluster descriptions in physical units and the random
initial placement of atoms and electrons.  It holds none of the method's arithmetic (no unit
conversion, field, push or ionization code); both the oracle and the GPU library receive what
it produces and convert it themselves.

Recipe (the paper's workloads, Sec. II-III, made synthetic):
  * atoms of a species sit uniformly at random inside a sphere of radius R0 centred at the
    origin (the cluster geometry and random placement of Sec. II);
  * the number of real atoms follows Eq.(1) with the Wigner-Seitz radii the paper lists;
    the cluster is lumped into ``n_ion`` ion macroparticles, each standing for
    N_atoms / n_ion real ions with the same charge-to-mass ratio;
  * every ion starts with charge ``z_init`` and has ``z_init`` electron macroparticles placed
    at ``electron_offset_nm`` from it in an isotropic random direction, momenta zero;
  * particle order: all ions, then the initial electrons grouped by parent ion.
Random numbers come from numpy's Philox bit generator keyed by (seed, cluster index).
"""
from dataclasses import dataclass, field, replace
import math

import numpy as np

from .species import SPECIES


@dataclass(frozen=True)
class Laser:
    """Laser description in physical units."""
    lambda_um: float = 0.8
    intensity_wcm2: float = 1e16
    envelope: str = "gauss_field"     # gauss_field | gauss_intensity | sin2 | flat
    fwhm_fs: float = 30.0             # Gaussian envelopes
    n_cycles: float = 10.0            # sin2 envelope: total length in laser periods
    phase: str = "dipole"             # dipole | plane_wave (test mode)
    polarization: str = "linear_x"    # linear_x | circular (Eqs.(4)-(9))


@dataclass(frozen=True)
class Cluster:
    """One cluster in physical units."""
    species: str = "Ar"
    r0_nm: float = 2.5
    n_ion: int = 500
    capacity: int = 4500
    z_init: int = 1
    z_max: int = 8
    electron_offset_nm: float = 0.01
    laser: Laser = field(default_factory=Laser)
    n_steps: int = 200                # steps this cluster runs (ensembles retire early ones)


@dataclass(frozen=True)
class Run:
    """Integration settings shared by every cluster of a run."""
    dt: float = 0.05                  # in 1/w
    t0: float = 0.0
    softening_nm: float = 0.1
    ionize: bool = True
    ofi_field: str = "laser_only"     # laser_only | local
    diag_every: int = 10
    seed: int = 0
    boundary: str = "open"            # open | periodic | mixed (Sec. II)
    box_r0: float = 20.0              # side of the periodic cube in units of R0 (R_IC = 20 R0)
    t_switch: float = math.inf        # mixed: first time (1/w) with open boundaries
    collisional: bool = False         # add the collisional ionization rate (Sec. II)


def n_atoms_input(cluster):
    """Species radius and cluster radius, the inputs of Eq.(1) (the evaluation is each side's)."""
    return cluster.r0_nm, SPECIES[cluster.species]["rw_angstrom"]


def initial_state(cluster, seed, cluster_index=0):
    """Initial macroparticle arrays for one cluster.

    Returns a dict with positions ``x_nm`` (N0 x 3, float64, nm), momenta ``u`` (N0 x 3,
    zeros), charge numbers ``Z`` (int8, ions ``z_init``, electrons -1) and ``n_ion``.
    """
    rng = np.random.Generator(np.random.Philox(key=[int(seed), int(cluster_index)]))
    n = int(cluster.n_ion)
    u = rng.random((n, 3))
    r = cluster.r0_nm * np.cbrt(u[:, 0])
    ct = 2.0 * u[:, 1] - 1.0
    ph = 2.0 * math.pi * u[:, 2]
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ions = np.stack([r * st * np.cos(ph), r * st * np.sin(ph), r * ct], axis=1)
    ne = n * int(cluster.z_init)
    v = rng.random((ne, 2))
    ect = 2.0 * v[:, 0] - 1.0
    eph = 2.0 * math.pi * v[:, 1]
    est = np.sqrt(np.maximum(0.0, 1.0 - ect * ect))
    dirs = np.stack([est * np.cos(eph), est * np.sin(eph), ect], axis=1)
    parents = np.repeat(np.arange(n), int(cluster.z_init))
    electrons = ions[parents] + cluster.electron_offset_nm * dirs
    x = np.concatenate([ions, electrons], axis=0)
    Z = np.concatenate([np.full(n, cluster.z_init, np.int8), np.full(ne, -1, np.int8)])
    if x.shape[0] > cluster.capacity:
        raise ValueError("initial particle count exceeds the cluster capacity")
    return {"x_nm": np.ascontiguousarray(x), "u": np.zeros_like(x), "Z": Z, "n_ion": n}


# ----------------------------------------------------------------------------- workloads
# The five benchmark workloads.  Every one is synthetic: argon or xenon clusters at the
# paper's scales (Sec. III uses Ar, Xe and D clusters of a few nm with 1e15-1e17 W/cm^2
# pulses of 25-100 fs), seed 0 unless stated.

def small_ar():
    """Plain FP64 parity case: Ar, R0 = 2.5 nm, 500 Ar+ each with one electron at 0.01 nm,
    1e16 W/cm^2 at 800 nm, sin^2 envelope of 10 cycles, 200 steps of dt = 0.05."""
    laser = Laser(intensity_wcm2=1e16, envelope="sin2", n_cycles=10.0)
    c = Cluster(species="Ar", r0_nm=2.5, n_ion=500, capacity=4500, z_init=1, z_max=8, laser=laser,
                n_steps=200)
    return c, Run(dt=0.05, ionize=True, diag_every=10, seed=0)


def ar_20k():
    """Ar, R0 = 8 nm, 10k Ar+ + 10k electrons (20k macroparticles), 1e16 W/cm^2, 30 fs FWHM
    Gaussian, 4000 steps, charges frozen so the particle count stays 20k."""
    laser = Laser(intensity_wcm2=1e16, envelope="gauss_field", fwhm_fs=30.0)
    c = Cluster(species="Ar", r0_nm=8.0, n_ion=10000, capacity=20000, z_init=1, z_max=8, laser=laser,
                n_steps=4000)
    return c, Run(dt=0.05, ionize=False, diag_every=100, seed=0)


def xe_200k():
    """Xe, R0 = 20 nm, capacity 200k macroparticles (22,222 Xe+ + 22,222 electrons at the
    start, room for ionization up to Xe8+), 5e16 W/cm^2, 100 fs FWHM Gaussian, 10k steps."""
    laser = Laser(intensity_wcm2=5e16, envelope="gauss_field", fwhm_fs=100.0)
    c = Cluster(species="Xe", r0_nm=20.0, n_ion=22222, capacity=200000, z_init=1, z_max=8,
                laser=laser, n_steps=10000)
    return c, Run(dt=0.05, ionize=True, diag_every=100, seed=0)


def ar_anisotropy(n_ion=5000, n_steps=60000):
    """The anisotropy study of Sec. III made synthetic: Ar cluster of R0 = 8.2 nm (about 40,000
    atoms by Eq.(1) with R_W = 2.4 A) lumped into n_ion Ar+ macro-ions and as many electrons,
    capacity for Ar8+, 806 nm, 8e15 W/cm^2, 100 fs FWHM Gaussian, linear polarization along x,
    detectors at 9 R0 with 30 degree acceptance (set by the caller)."""
    laser = Laser(lambda_um=0.806, intensity_wcm2=8e15, envelope="gauss_field", fwhm_fs=100.0)
    c = Cluster(species="Ar", r0_nm=8.2, n_ion=n_ion, capacity=9 * n_ion, z_init=1, z_max=8, laser=laser,
                n_steps=n_steps)
    return c, Run(dt=0.05, ionize=True, diag_every=1000, seed=0)


def ensemble(n_clusters=256, seed=0, cap_lo=1000, cap_hi=16000, steps_per_fwhm=None,
             lambda_um=0.8, dt=0.05, capacity_rule="random"):
    """Batched ensemble of uneven clusters.

    Cluster c draws (numpy Philox keyed by (seed, 1_000_000 + c)): species Ar or Xe with
    probability 1/2; capacity log-uniform in [cap_lo, cap_hi]; R0 uniform in [2, 10] nm;
    intensity log-uniform in [1e15, 1e17] W/cm^2; FWHM uniform in [20, 100] fs.  Ion count
    min(capacity // 9, floor(N_atoms)) so that each ion can reach Xe8+/Ar8+ within capacity
    and no macroparticle stands for less than one atom.  Each cluster runs until
    t_end = 4 FWHM (the Gaussian peak sits at 2 FWHM); steps_per_fwhm overrides that length.
    capacity_rule "radius" replaces the random capacity by one fixed by the radius,
    cap_lo (cap_hi / cap_lo)^((R0 - 2 nm) / 8 nm) (log-linear over the same range), so that the
    lumping N_atoms / n_ion is a function of the cluster's species and size; every other draw is
    unchanged.
    """
    out = []
    for c in range(n_clusters):
        rng = np.random.Generator(np.random.Philox(key=[int(seed), 1_000_000 + c]))
        species = "Ar" if rng.random() < 0.5 else "Xe"
        cap = int(round(math.exp(rng.uniform(math.log(cap_lo), math.log(cap_hi)))))
        r0 = float(rng.uniform(2.0, 10.0))
        inten = float(math.exp(rng.uniform(math.log(1e15), math.log(1e17))))
        fwhm = float(rng.uniform(20.0, 100.0))
        if capacity_rule == "radius":
            cap = int(round(cap_lo * (cap_hi / cap_lo) ** ((r0 - 2.0) / 8.0)))
        elif capacity_rule != "random":
            raise ValueError("capacity_rule must be random or radius")
        rw = SPECIES[species]["rw_angstrom"]
        n_atoms_floor = int(math.floor((r0 * 10.0 / rw) ** 3))
        n_ion = max(1, min(cap // 9, n_atoms_floor))
        # t_end = 4 FWHM; 1 fs = 2 pi c / lambda * 1e-15 rad of laser phase
        w_fs = 2.0 * math.pi * 299792458.0 / (lambda_um * 1e-6) * 1e-15
        steps = int(math.ceil(4.0 * fwhm * w_fs / dt)) if steps_per_fwhm is None else int(
            math.ceil(4.0 * steps_per_fwhm))
        laser = Laser(lambda_um=lambda_um, intensity_wcm2=inten, envelope="gauss_field", fwhm_fs=fwhm)
        out.append(Cluster(species=species, r0_nm=r0, n_ion=n_ion, capacity=cap, z_init=1, z_max=8,
                           laser=laser, n_steps=steps))
    return out


def surrogate_inputs(n_points, seed, lo=None, hi=None):
    """Surrogate query points (R0 nm, N_atoms proxy via species, intensity, FWHM) drawn like
    the ensemble's clusters; returns an (n, 4) float64 array of
    (R0_nm, rw_angstrom, intensity_wcm2, fwhm_fs)."""
    rng = np.random.Generator(np.random.Philox(key=[int(seed), 7]))
    sp = rng.random(n_points) < 0.5
    rw = np.where(sp, SPECIES["Ar"]["rw_angstrom"], SPECIES["Xe"]["rw_angstrom"])
    r0 = rng.uniform(2.0, 10.0, n_points)
    inten = np.exp(rng.uniform(math.log(1e15), math.log(1e17), n_points))
    fwhm = rng.uniform(20.0, 100.0, n_points)
    return np.stack([r0, rw, inten, fwhm], axis=1)


__all__ = ["Laser", "Cluster", "Run", "SPECIES", "initial_state", "small_ar", "ar_20k", "xe_200k",
           "ensemble", "surrogate_inputs", "replace"]
