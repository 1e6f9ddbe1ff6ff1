"""Inputs of the coupling-matrix builder (Section II, Eqs. 1-3 and 12-13).

An asymmetric-top rotor (states j1, tau1 with the coefficients b_k of Eq. 1)
combined with a linear rotor (j2) into coupled states |j1 tau1 j2 j m> (Eq. 3),
and a potential given by its expansion coefficients v_{l1 mu1 l2 l}(R) on a radial
grid (Eq. 12).  These are inputs only: the matrix elements themselves are
computed by the builder (and, independently, by the oracle).

Defaults follow the paper's system where it states numbers: H2O rotational
constants, para-H2 (even j2), expansion terms up to l1 = 9, mu1 = 6, l2 = 6,
l = 11, and a 63-point radial grid from 3 to 30 bohr with logarithmic spacing
(Section III).  The expansion coefficients are synthetic (the paper's potential
is not available): a repulsive exponential and an attractive R^-6 tail per term,
with amplitudes that fall off with the term's angular order.
"""
from dataclasses import dataclass, field
import math

import numpy as np

from . import units as U
from .angular import asymmetric_top_states, jx_block
from .systems import SEED_BASE, System

H2O_ABC_CM = (27.88, 14.51, 9.28)
H2_B_CM = 60.853


@dataclass
class CouplingBasis:
    j: np.ndarray          # [N] total angular momentum of each channel
    m: np.ndarray          # [N] its projection
    rot1: np.ndarray       # [N] index of the rotor-1 state (j1, tau1)
    j2: np.ndarray         # [N] linear-rotor angular momentum
    rot1_j: np.ndarray     # [n1] j1 of each rotor-1 state
    rot1_tau: np.ndarray   # [n1] tau1 (-j1 .. j1, ascending energy)
    b: np.ndarray          # [n1, 2*j1max+1] b_k at column k + j1 (zeros elsewhere)
    E: np.ndarray          # [N] channel energies, hartree
    jx_row: np.ndarray     # Coriolis J_x within each (j1 tau1 j2 j) level, over m
    jx_col: np.ndarray
    jx_val: np.ndarray
    level_of_channel: np.ndarray
    n_levels: int

    @property
    def N(self):
        return int(self.j.shape[0])

    @property
    def j1(self):
        return self.rot1_j[self.rot1]


@dataclass
class Expansion:
    lam1: np.ndarray       # [T]
    mu1: np.ndarray        # [T]
    lam2: np.ndarray       # [T]
    lam: np.ndarray        # [T]
    R_grid: np.ndarray     # [K] bohr
    v: np.ndarray          # [T, K] hartree

    @property
    def T(self):
        return int(self.lam1.shape[0])

    @property
    def K(self):
        return int(self.R_grid.shape[0])


def top_rotor_basis(j1max=2, j2_values=(0, 2), rot=H2O_ABC_CM, B2_cm=H2_B_CM, jmax=None,
                    m_values=None, rot1_states=None, order="level", e_max_cm=None,
                    tau_parity=None):
    """Channels |j1 tau1 j2 j m> for j1 <= j1max (every tau1, or only the (j1, tau1)
    pairs in rot1_states, or only tau1 of the given parity), j2 in j2_values, rotational
    energy below e_max_cm if given, |j1 - j2| <= j <= j1 + j2 (and j <= jmax),
    m = -j..j (or the given m only).  order="level": by level (j1, tau1, j2, j), then
    m; order="m": by m, then level (each m block contiguous)."""
    rot1_j, rot1_tau, rot1_E, bl = [], [], [], []
    for j1 in range(j1max + 1):
        E1, b1 = asymmetric_top_states(j1, *rot)
        for t in range(2 * j1 + 1):
            if rot1_states is not None and (j1, t - j1) not in rot1_states:
                continue
            if tau_parity is not None and (t - j1) % 2 != tau_parity:
                continue
            row = np.zeros(2 * j1max + 1)
            row[:2 * j1 + 1] = b1[t]
            rot1_j.append(j1)
            rot1_tau.append(t - j1)
            rot1_E.append(E1[t])
            bl.append(row)
    j, m, r1, j2, E, lev = [], [], [], [], [], []
    jr, jc, jv = [], [], []
    n_lev = 0
    for r in range(len(rot1_j)):
        for jb in j2_values:
            if e_max_cm is not None and rot1_E[r] + B2_cm * jb * (jb + 1) >= e_max_cm:
                continue
            for jt in range(abs(rot1_j[r] - jb), rot1_j[r] + jb + 1):
                if jmax is not None and jt > jmax:
                    continue
                ms = [x for x in range(-jt, jt + 1) if m_values is None or x in m_values]
                if not ms:
                    continue
                off = len(j)
                for x in ms:
                    j.append(jt); m.append(x); r1.append(r); j2.append(jb)
                    E.append(rot1_E[r] + B2_cm * jb * (jb + 1))
                    lev.append(n_lev)
                if m_values is None:
                    rr, cc, vv = jx_block(jt)
                    jr += [off + a for a in rr]; jc += [off + a for a in cc]; jv += vv
                n_lev += 1
    i32 = lambda a: np.array(a, np.int32)
    j, m, r1, j2, E, lev, jr, jc = (np.array(a) for a in (j, m, r1, j2, E, lev, jr, jc))
    if order == "m":
        p = np.lexsort((lev, m))               # new position -> old channel
        inv = np.empty_like(p)
        inv[p] = np.arange(p.size)
        j, m, r1, j2, E, lev = (a[p] for a in (j, m, r1, j2, E, lev))
        jr, jc = inv[jr.astype(np.int64)] if jr.size else jr, inv[jc.astype(np.int64)] if jc.size else jc
    return CouplingBasis(i32(j), i32(m), i32(r1), i32(j2), i32(rot1_j), i32(rot1_tau),
                         np.array(bl), U.cm_to_hartree(np.array(E, np.float64)), i32(jr), i32(jc),
                         np.array(jv, np.float64), i32(lev), n_lev)


def expansion_terms(l1max=9, mu1max=6, l2max=6, lmax=11, even_mu1=True, even_l2=True):
    """(l1, mu1, l2, l) with 0 <= mu1 <= l1, |l1 - l2| <= l <= l1 + l2, l <= lmax.
    even_mu1: the C2v symmetry of the top (H2O); even_l2: a homonuclear linear rotor.
    Terms with mu1 = 0 and l1 + l2 + l odd vanish identically (Eq. 13) and are left out."""
    out = []
    for l1 in range(l1max + 1):
        for mu1 in range(0, min(l1, mu1max) + 1):
            if even_mu1 and mu1 % 2:
                continue
            for l2 in range(l2max + 1):
                if even_l2 and l2 % 2:
                    continue
                for l in range(abs(l1 - l2), min(l1 + l2, lmax) + 1):
                    if mu1 == 0 and (l1 + l2 + l) % 2:
                        continue
                    out.append((l1, mu1, l2, l))
    return out


def log_grid(K=63, R_min=3.0, R_max=30.0):
    """K points from R_min to R_max bohr, denser at short range (Section III)."""
    return np.exp(np.linspace(math.log(R_min), math.log(R_max), K))


def synthetic_expansion(terms, R_grid, seed=0):
    """v_t(R) = a_t exp(-beta_t (R - 5)) - c_t (5/R)^6 in cm^-1 (then hartree), with
    a_t, c_t drawn at random and scaled by 1/(1 + l1 + l2) (the isotropic term is the
    largest: a = 200, c = 100 cm^-1)."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 6, seed]))
    T = len(terms)
    v = np.zeros((T, len(R_grid)))
    for t, (l1, mu1, l2, l) in enumerate(terms):
        if (l1, mu1, l2, l) == (0, 0, 0, 0):
            a, c, beta = 200.0, 100.0, 1.6
        else:
            sc = 1.0 / (1.0 + l1 + l2)
            a, c = 60.0 * sc * rng.standard_normal(), 20.0 * sc * rng.standard_normal()
            beta = 1.2 + 0.6 * rng.random()
        v[t] = a * np.exp(-beta * (R_grid - 5.0)) - c * (5.0 / R_grid) ** 6
    arr = lambda k: np.array([x[k] for x in terms], np.int32)
    return Expansion(arr(0), arr(1), arr(2), arr(3), np.asarray(R_grid, np.float64),
                     U.cm_to_hartree(v))


def system_from_tables(basis, R_grid, M, mu_amu=1.8, name="top_rotor"):
    """A propagatable system from built tables M [K, N, N] (host array or device tensor)."""
    return System(name=name, R_grid=np.asarray(R_grid, np.float64), E=basis.E, M=M,
                  jx_row=basis.jx_row, jx_col=basis.jx_col, jx_val=basis.jx_val,
                  mu=U.amu_to_me(mu_amu), level_of_channel=basis.level_of_channel,
                  n_levels=basis.n_levels)


# Screening threshold for the paper-size build with this module's synthetic
# expansion.  The paper keeps |M| > 1 cm^-1 of its ab-initio potential (14.6 M of
# about 0.5 B elements); the synthetic potential is about twenty times weaker at
# the screening distances (its isotropic well is a few cm^-1 deep against some
# 200 cm^-1 for H2O + H2), so the threshold is scaled with it: 0.05 cm^-1 keeps a
# number of elements of the paper's order.
PAPER_SCALE_DROP_CM = 0.05
PAPER_SCREEN_R = (6.03, 7.11)        # bohr, Section III


def para_h2o_para_h2_basis(e_max_cm=8000.0, j1max=28, j2max=10, order="m"):
    """Section III's p-H2O + p-H2 basis: para-H2O (tau1 = kA - kC even) up to j1 = 28,
    para-H2 (even j2) up to 10, rotational energy below 8000 cm^-1, all j and m (rigid
    rotors with the H2O and H2 constants: 1034 levels, 206,350 states)."""
    return top_rotor_basis(j1max, tuple(range(0, j2max + 1, 2)), order=order,
                           e_max_cm=e_max_cm, tau_parity=0)


# the levels j1_{kA kC} of Section II's check of Eq. 18, as (j1, tau1 = kA - kC)
PAPER_CHECK_ROT1 = [(0, 0), (1, 0), (2, -2), (2, 0), (2, 2), (3, -2), (3, 0)]


def paper_check_basis():
    """The 14 (j1_{kA kC}, j2) combinations of Section II's check (j2 = 0, 2), all j, m."""
    return top_rotor_basis(3, (0, 2), rot1_states=PAPER_CHECK_ROT1)


def select_terms(terms, n, seed=0):
    """n of the terms (the isotropic one always), drawn without replacement."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 6, 1000 + seed]))
    iso = [i for i, t in enumerate(terms) if t == (0, 0, 0, 0)]
    rest = [i for i in range(len(terms)) if i not in iso]
    pick = sorted(iso + list(rng.choice(rest, size=n - len(iso), replace=False)))
    return [terms[i] for i in pick]


def config6(j1max=6, j2_values=(0, 2, 4), K=63, n_terms=83, seed=0):
    """Coupling-builder workload: H2O-like top, j1 <= 6 (every tau1) + para-H2, j2 <= 4,
    all j and m, channels ordered by m; 83 expansion terms drawn from the ranges of
    Section II's potential (l1 <= 9, mu1 <= 6, l2 <= 6, l <= 11); 63 log-spaced radial
    points from 3 to 30 bohr (Section III)."""
    basis = top_rotor_basis(j1max, j2_values, order="m")
    terms = select_terms(expansion_terms(), n_terms, seed)
    return basis, synthetic_expansion(terms, log_grid(K), seed)
