"""Unit conversions (CODATA 2018) between spectroscopic units and atomic units.

Every quantity handed to the propagator or to the oracle is in atomic units:
energies in hartree, lengths in bohr, masses in electron masses, time in
hbar/E_h.  The paper quotes energies in cm^-1, lengths in bohr or angstrom
(Section III), which these factors translate.
"""

HARTREE_PER_CM = 1.0 / 219474.6313705      # 1 cm^-1 in hartree
BOHR_PER_ANG = 1.0 / 0.529177210903         # 1 angstrom in bohr
ANG2_PER_BOHR2 = 0.529177210903 ** 2        # 1 bohr^2 in angstrom^2
ME_PER_AMU = 1822.888486209                 # 1 unified atomic mass unit in m_e
FS_PER_AU_TIME = 2.4188843265857e-2         # 1 a.u. of time in femtoseconds


def cm_to_hartree(x):
    return x * HARTREE_PER_CM


def hartree_to_cm(x):
    return x / HARTREE_PER_CM


def ang_to_bohr(x):
    return x * BOHR_PER_ANG


def bohr_to_ang(x):
    return x / BOHR_PER_ANG


def amu_to_me(x):
    return x * ME_PER_AMU
