"""Unit conversions and physical constants of the oracle (test infrastructure only).

The paper's model (Sec. II) works in dimensionless units: electric field a0 = eE/(m_e w c),
magnetic field b0 = eB/(m_e w), time in 1/w and length in 1/k = c/w.  This module turns
the physical workload description (nm, W/cm^2, fs, eV, u) into those units.  It is written
independently of the GPU library's host code; a test compares the two.

Constants are CODATA 2018 values.
"""
import math

C_LIGHT = 299792458.0                 # m/s
R_ELECTRON = 2.8179403262e-15         # classical electron radius, m
MEC2_EV = 510998.95000                # electron rest energy, eV
E_CHARGE = 1.602176634e-19            # C
M_ELECTRON = 9.1093837015e-31         # kg
FIELD_AU = 5.14220674763e11           # atomic unit of electric field, V/m
TIME_AU = 2.4188843265857e-17         # atomic unit of time, s
HARTREE_EV = 27.211386245988          # eV
U_PER_ME = 1822.888486209             # atomic mass unit in electron masses

# Eq.(2): a0 = sqrt(I0 lambda^2 / 1.366e18), I0 in W/cm^2, lambda in micrometres.
EQ2_CONSTANT = 1.366e18


def wavenumber(lambda_um):
    """k = 2 pi / lambda in 1/m."""
    return 2.0 * math.pi / (lambda_um * 1e-6)


def omega(lambda_um):
    """Laser angular frequency w = c k in rad/s."""
    return C_LIGHT * wavenumber(lambda_um)


def nm_to_norm(length_nm, lambda_um):
    """Length in nm -> units of c/w (multiply by k)."""
    return length_nm * 1e-9 * wavenumber(lambda_um)


def fs_to_norm(time_fs, lambda_um):
    """Time in fs -> units of 1/w."""
    return time_fs * 1e-15 * omega(lambda_um)


def a0_from_intensity(intensity_wcm2, lambda_um):
    """Eq.(2): dimensionless peak field from intensity and wavelength."""
    return math.sqrt(intensity_wcm2 * lambda_um * lambda_um / EQ2_CONSTANT)


def kappa(lambda_um):
    """Coulomb coupling in the dimensionless units.

    The field of charge Q e at distance r is Q e / (4 pi eps0 r^2).  Scaling by
    e/(m_e w c) and writing r = r'/k gives Q r_e k / r'^2 with r_e = e^2/(4 pi eps0 m_e c^2),
    so a charge Q produces kappa Q / r'^2 with kappa = r_e k; the pair potential energy in
    m_e c^2 units is kappa Q_i Q_j / r'.
    """
    return R_ELECTRON * wavenumber(lambda_um)


def field_au_per_a0(lambda_um):
    """Atomic units of electric field per unit of a0: (m_e w c / e) / E_au."""
    return M_ELECTRON * omega(lambda_um) * C_LIGHT / E_CHARGE / FIELD_AU


def rate_scale(lambda_um):
    """A rate in inverse atomic time units expressed per 1/w: 1 / (w t_au)."""
    return 1.0 / (omega(lambda_um) * TIME_AU)


def n_atoms(r0_nm, rw_angstrom):
    """Eq.(1): N_atoms = (R0 / R_W)^3, unrounded."""
    return (r0_nm * 10.0 / rw_angstrom) ** 3


def ev_to_hartree(e_ev):
    return e_ev / HARTREE_EV
