"""Species data: problem input, not method.

``rw_angstrom``: Wigner-Seitz radii the paper lists for D, Ne, Ar and Xe clusters (Sec. II,
after Eq.(1)).  ``mass_u``: standard atomic weights (IUPAC; deuterium's isotopic mass).
``ip_ev[k]``: ionization energy of the charge state k -> k+1 in eV (NIST Atomic Spectra
Database ground-state values; the paper uses ADK rates but does not list them).
"""

SPECIES = {
    "D": {
        "rw_angstrom": 1.70,
        "mass_u": 2.01410177812,
        "ip_ev": [13.6026],
    },
    "Ne": {
        "rw_angstrom": 2.02,
        "mass_u": 20.1797,
        "ip_ev": [21.564540, 40.96297, 63.4233, 97.1900, 126.247, 157.934, 207.271, 239.0970,
                  1195.8078, 1362.1991],
    },
    "Ar": {
        "rw_angstrom": 2.40,
        "mass_u": 39.948,
        "ip_ev": [15.7596117, 27.62967, 40.735, 59.58, 74.84, 91.290, 124.41, 143.4567, 422.60,
                  478.69],
    },
    "Xe": {
        "rw_angstrom": 2.73,
        "mass_u": 131.293,
        "ip_ev": [12.1298437, 20.975, 31.05, 42.20, 54.1, 66.703, 91.6, 105.9759, 179.84, 202.0],
    },
}
