"""Species data: problem input, not method.

``rw_angstrom``: Wigner-Seitz radii the paper lists for D, Ne, Ar and Xe clusters (Sec. II,
after Eq.(1)).  ``mass_u``: standard atomic weights (IUPAC; deuterium's isotopic mass).
``ip_ev[k]``: ionization energy of the charge state k -> k+1 in eV (NIST Atomic Spectra
Database ground-state values; the paper uses ADK rates but does not list them).
``outer_q[k]``: electrons in the outermost occupied subshell of the ground state of charge
state k (the subshell the next ionization empties), from the ground-state configurations
(D 1s; Ne 2p6 2s2 1s2; Ar 3p6 3s2 2p6; Xe 5p6 5s2 4d10).
"""

SPECIES = {
    "D": {
        "rw_angstrom": 1.70,
        "mass_u": 2.01410177812,
        "ip_ev": [13.6026],
        "outer_q": [1],
    },
    "Ne": {
        "rw_angstrom": 2.02,
        "mass_u": 20.1797,
        "ip_ev": [21.564540, 40.96297, 63.4233, 97.1900, 126.247, 157.934, 207.271, 239.0970,
                  1195.8078, 1362.1991],
        "outer_q": [6, 5, 4, 3, 2, 1, 2, 1, 2, 1],
    },
    "Ar": {
        "rw_angstrom": 2.40,
        "mass_u": 39.948,
        "ip_ev": [15.7596117, 27.62967, 40.735, 59.58, 74.84, 91.290, 124.41, 143.4567, 422.60,
                  478.69],
        "outer_q": [6, 5, 4, 3, 2, 1, 2, 1, 6, 5],
    },
    "Xe": {
        "rw_angstrom": 2.73,
        "mass_u": 131.293,
        "ip_ev": [12.1298437, 20.975, 31.05, 42.20, 54.1, 66.703, 91.6, 105.9759, 179.84, 202.0],
        "outer_q": [6, 5, 4, 3, 2, 1, 2, 1, 10, 9],
    },
}
