"""Seeded synthetic collision systems and trajectory batches.

The paper's own workload (H2O + H2 with its ab-initio potential and coupling
matrices, Section III) is not available, so these generators build systems of
the same shape: channel energies, a coupling matrix tabulated on an R grid
(Section III: tabulated then cubic-splined), a Coriolis operator (Section II,
Eq. 5) and Monte-Carlo initial conditions (Section III: random impact
parameters).  They produce inputs only; none of the propagation arithmetic is
here, so the oracle and the GPU library can both consume them.

All arrays returned are in atomic units (hartree, bohr, m_e).  Five stock
configurations are provided:

  1  rigid-rotor diatom + atom, |j m>, j <= 6 (N = 49), Legendre potential
     expanded with exact Gaunt coefficients, 64 trajectories, RK4 2000 steps
  2  asymmetric top (A/B/C = 27/14.5/9.3 cm^-1) + atom, |j tau m>, j <= 8
     (N = 969), random smooth Hermitian complex tables, 4096 trajectories
  3  uneven mix of the systems of 1, 2 and 4, log-uniform energies, DP5
  4  product of two linear rotors, |j1 m1 j2 m2>, j1, j2 <= 3 (N = 256),
     potential linear in 96 expansion coefficients (adjoint workload)
  5  N = 4096 random Hermitian tables (binned-MFMA workload)
"""
from dataclasses import dataclass, field
import math

import numpy as np

from . import units as U
from .angular import (asymmetric_top_levels, gaunt, jx_block,
                      legendre_matrix_element, clebsch_gordan)

SEED_BASE = 231202322


def _streams(cfg_index, n=3):
    ss = np.random.SeedSequence(SEED_BASE + cfg_index)
    return [np.random.default_rng(s) for s in ss.spawn(n)]


@dataclass
class System:
    name: str
    R_grid: np.ndarray            # [K] bohr, strictly increasing
    E: np.ndarray                 # [N] hartree
    M: np.ndarray                 # [K, N, N] hartree, real symmetric or complex Hermitian per k
    jx_row: np.ndarray            # Coriolis J_x in coordinate form (real symmetric)
    jx_col: np.ndarray
    jx_val: np.ndarray
    mu: float                     # reduced mass, m_e
    level_of_channel: np.ndarray  # [N] non-degenerate level index of each channel
    n_levels: int
    labels: dict = field(default_factory=dict)
    # optional parametric form M(R_k) = sum_p theta_p radial_p(R_k) G_{gidx_p}
    param_radial: np.ndarray = None   # [P, K] hartree
    param_G_index: np.ndarray = None  # [P]
    G: np.ndarray = None              # [nG, N, N] real symmetric, dimensionless
    theta: np.ndarray = None          # [P]

    @property
    def N(self):
        return int(self.E.shape[0])

    @property
    def K(self):
        return int(self.R_grid.shape[0])

    @property
    def is_complex(self):
        return np.iscomplexobj(self.M)


@dataclass
class Batch:
    system_index: np.ndarray   # [B] int32, index into the system list
    init_channel: np.ndarray   # [B] int32
    E_coll: np.ndarray         # [B] hartree, translational energy at R0
    b: np.ndarray              # [B] bohr
    R0: np.ndarray             # [B] bohr
    dt: np.ndarray             # [B] a.u. of time (RK4 step or DP5 initial-step hint)
    n_steps: np.ndarray        # [B] int64 (RK4 step count)
    b_max: float               # bohr, the Monte-Carlo sampling range of b
    init_level: np.ndarray = None   # [B] level of the initial channel

    @property
    def B(self):
        return int(self.system_index.shape[0])

    def subset(self, idx):
        idx = np.asarray(idx)
        return Batch(self.system_index[idx].copy(), self.init_channel[idx].copy(),
                     self.E_coll[idx].copy(), self.b[idx].copy(), self.R0[idx].copy(),
                     self.dt[idx].copy(), self.n_steps[idx].copy(), self.b_max,
                     None if self.init_level is None else self.init_level[idx].copy())


def uniform_grid_bohr(r_min_ang=2.0, r_max_ang=20.0, K=200):
    return U.ang_to_bohr(np.linspace(r_min_ang, r_max_ang, K))


def collision_time(R0, E_coll, mu):
    """Time for a free particle to go in from R0 and back out: 2 R0 / v0 (a.u.)."""
    return 2.0 * R0 / np.sqrt(2.0 * E_coll / mu)


# ---------------------------------------------------------------------------
# radial potentials


def _legendre_potential_params(rng, lam_max=4):
    """A_l e^{-alpha_l R} - C_l / R^6 (R in angstrom, cm^-1), seeded."""
    a0 = rng.uniform(2.8, 3.4)
    A0 = 1000.0 * math.exp(3.0 * a0) * rng.uniform(0.8, 1.25)
    C0 = rng.uniform(5e4, 2e5)
    alpha = [a0]; A = [A0]; C = [C0]
    for _ in range(1, lam_max + 1):
        alpha.append(a0 * rng.uniform(1.0, 1.2))
        A.append(A0 * rng.uniform(-0.2, 0.2))
        C.append(C0 * rng.uniform(-0.3, 0.3))
    return np.array(A), np.array(alpha), np.array(C)


def _v_lambda_cm(params, R_ang):
    A, alpha, C = params
    R = np.asarray(R_ang)[None, :]
    return A[:, None] * np.exp(-alpha[:, None] * R) - C[:, None] / R ** 6


def _check_turning_point(v_cm, R_ang, U_cm, r_min_ang=2.5):
    """The repulsive wall must stop a head-on collision before r_min_ang."""
    inside = R_ang <= r_min_ang
    if not np.all(v_cm[inside] > U_cm):
        raise AssertionError("synthetic wall too soft: turning point below %.2f A" % r_min_ang)


# ---------------------------------------------------------------------------
# system 1: rigid-rotor diatom + atom


def rotor_atom_system(jmax=6, K=200, B_cm=2.0, mu_amu=4.0, cfg_index=1, with_coriolis=True,
                      R_ang=None):
    """R_ang: the radial grid in angstrom (default K points uniform on 2-20 A)."""
    rng_pot, _, _ = _streams(cfg_index)
    params = _legendre_potential_params(rng_pot, lam_max=4)
    R_ang = np.linspace(2.0, 20.0, K) if R_ang is None else np.asarray(R_ang, np.float64)
    V = _v_lambda_cm(params, R_ang)                     # [5, K]
    chans = [(j, m) for j in range(jmax + 1) for m in range(-j, j + 1)]
    N = len(chans)
    E = np.array([B_cm * j * (j + 1) for j, _ in chans])
    # angular factors <j'' m | P_lam | j' m>, symmetric by construction
    ang = np.zeros((5, N, N))
    for a, (j2, m2) in enumerate(chans):
        for b_, (j1, m1) in enumerate(chans):
            if m1 != m2 or b_ < a:
                continue
            for lam in range(5):
                val = legendre_matrix_element(j2, j1, lam, m1)
                ang[lam, a, b_] = val
                ang[lam, b_, a] = val
    M_cm = np.einsum("lk,lab->kab", V, ang)
    jr, jc, jv = [], [], []
    if with_coriolis:
        off = 0
        for j in range(jmax + 1):
            r, c, v = jx_block(j)
            jr += [off + x for x in r]; jc += [off + x for x in c]; jv += v
            off += 2 * j + 1
    levels = np.array([j for j, _ in chans], dtype=np.int32)
    return System(
        name="rotor_atom_j%d" % jmax,
        R_grid=U.ang_to_bohr(R_ang), E=U.cm_to_hartree(E), M=U.cm_to_hartree(M_cm),
        jx_row=np.array(jr, np.int32), jx_col=np.array(jc, np.int32),
        jx_val=np.array(jv, np.float64), mu=U.amu_to_me(mu_amu),
        level_of_channel=levels, n_levels=jmax + 1,
        labels={"j": np.array([c[0] for c in chans]), "m": np.array([c[1] for c in chans]),
                "V_lambda_cm": V, "R_ang": R_ang, "potential_params": params})


# ---------------------------------------------------------------------------
# Gaussian-process random Hermitian tables (systems 2 and 5)


def gp_factors(rng, N, Q=32, length_ang=1.0, workers=0):
    """Random-Fourier-feature factors of a squared-exponential GP: (omega, phase, H).

    workers > 0: each H_q is drawn from a generator of its own (seeded from rng)
    on a pool of that many threads -- other values than the serial draw, for
    sizes where one stream would take a minute."""
    omega = rng.standard_normal(Q) / length_ang
    phase = rng.uniform(0.0, 2.0 * math.pi, Q)
    if workers <= 0:
        X = (rng.standard_normal((Q, N, N)) + 1j * rng.standard_normal((Q, N, N))) / math.sqrt(2.0)
        H = (X + np.conj(np.swapaxes(X, 1, 2))) / math.sqrt(2.0)   # entry std 1, Hermitian
        return omega, phase, H
    from concurrent.futures import ThreadPoolExecutor
    seeds = rng.integers(0, 2 ** 63 - 1, Q)
    H = np.empty((Q, N, N), np.complex128)

    def one(q):
        g = np.random.default_rng(int(seeds[q]))
        X = np.empty((N, N), np.complex128)
        X.real = g.standard_normal((N, N))
        X.imag = g.standard_normal((N, N))
        X /= math.sqrt(2.0)
        H[q] = (X + X.conj().T) / math.sqrt(2.0)

    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(one, range(Q)))
    return omega, phase, H


def gp_basis(omega, phase, R_ang):
    Q = omega.shape[0]
    return math.sqrt(2.0 / Q) * np.cos(np.outer(R_ang, omega) + phase[None, :])   # [K, Q]


def gp_tables_cm(omega, phase, H, R_ang, s_cm, v_iso_cm):
    """M(R_k) = V_iso(R_k) I + s e^{-(R_k - 3 A)/1 A} G(R_k), exactly Hermitian."""
    K = R_ang.shape[0]
    Q, N, _ = H.shape
    phi = gp_basis(omega, phase, R_ang) * (s_cm * np.exp(-(R_ang - 3.0)))[:, None]
    # real and imaginary parts in one product over the interleaved storage
    Hv = np.ascontiguousarray(H).view(np.float64).reshape(Q, 2 * N * N)
    M = (phi @ Hv).view(np.complex128).reshape(K, N, N)
    for k in range(K):
        Mk = M[k]
        M[k] = 0.5 * (Mk + Mk.conj().T)
        M[k].flat[:: N + 1] += v_iso_cm[k]
    return M


def top_atom_system(jmax=8, K=200, rot=(27.0, 14.5, 9.3), s_cm=5.0, mu_amu=3.275,
                    cfg_index=2, Q=32):
    rng_pot, rng_tab, _ = _streams(cfg_index)
    params = _legendre_potential_params(rng_pot, lam_max=0)
    R_ang = np.linspace(2.0, 20.0, K)
    v_iso = _v_lambda_cm(params, R_ang)[0]
    chans, E = [], []
    for j in range(jmax + 1):
        lev = asymmetric_top_levels(j, *rot)
        for tau_i, e in enumerate(lev):
            for m in range(-j, j + 1):
                chans.append((j, tau_i - j, m))
                E.append(e)
    N = len(chans)
    omega, phase, H = gp_factors(rng_tab, N, Q=Q)
    M_cm = gp_tables_cm(omega, phase, H, R_ang, s_cm, v_iso)
    del H
    jr, jc, jv = [], [], []
    off = 0
    for j in range(jmax + 1):
        for _ in range(2 * j + 1):
            r, c, v = jx_block(j)
            jr += [off + x for x in r]; jc += [off + x for x in c]; jv += v
            off += 2 * j + 1
    level_ids = {}
    levels = np.array([level_ids.setdefault((j, t), len(level_ids)) for j, t, _ in chans],
                      np.int32)
    return System(
        name="top_atom_j%d" % jmax,
        R_grid=U.ang_to_bohr(R_ang), E=U.cm_to_hartree(np.array(E)), M=U.cm_to_hartree(M_cm),
        jx_row=np.array(jr, np.int32), jx_col=np.array(jc, np.int32),
        jx_val=np.array(jv, np.float64), mu=U.amu_to_me(mu_amu),
        level_of_channel=levels, n_levels=len(level_ids),
        labels={"j": np.array([c[0] for c in chans]), "tau": np.array([c[1] for c in chans]),
                "m": np.array([c[2] for c in chans]), "V_iso_cm": v_iso, "R_ang": R_ang})


# ---------------------------------------------------------------------------
# system 4: two linear rotors, potential linear in 96 coefficients

ANGULAR_TERMS = [(0, 0, 0), (1, 0, 1), (0, 1, 1), (1, 1, 0), (1, 1, 2), (2, 0, 2),
                 (0, 2, 2), (2, 1, 1), (2, 1, 3), (1, 2, 1), (1, 2, 3), (2, 2, 0)]


def _bipolar_matrix(chans, l1, l2, lam):
    """4 pi <j1'' m1'' j2'' m2''| sum_mu C(l1 mu l2 -mu|lam 0) Y_{l1 mu}(1) Y_{l2 -mu}(2) |...>."""
    N = len(chans)
    G = np.zeros((N, N))
    for a, (j1b, m1b, j2b, m2b) in enumerate(chans):
        for b_, (j1a, m1a, j2a, m2a) in enumerate(chans):
            mu_ = m1b - m1a
            if m2b - m2a != -mu_ or abs(mu_) > min(l1, l2):
                continue
            cg = clebsch_gordan(l1, mu_, l2, -mu_, lam, 0)
            if cg == 0.0:
                continue
            G[a, b_] = 4.0 * math.pi * cg * gaunt(j1b, m1b, l1, mu_, j1a, m1a) \
                * gaunt(j2b, m2b, l2, -mu_, j2a, m2a)
    return G


def rotor_rotor_system(jmax=3, K=200, B1_cm=2.0, B2_cm=1.5, mu_amu=8.0, cfg_index=4,
                       theta=None):
    rng_pot, _, _ = _streams(cfg_index)
    R_ang = np.linspace(2.0, 20.0, K)
    chans, E, lev = [], [], []
    level_ids = {}
    for j1 in range(jmax + 1):
        for j2 in range(jmax + 1):
            lid = level_ids.setdefault((j1, j2), len(level_ids))
            for m1 in range(-j1, j1 + 1):
                for m2 in range(-j2, j2 + 1):
                    chans.append((j1, m1, j2, m2))
                    E.append(B1_cm * j1 * (j1 + 1) + B2_cm * j2 * (j2 + 1))
                    lev.append(lid)
    N = len(chans)
    G = np.stack([_bipolar_matrix(chans, *t) for t in ANGULAR_TERMS])
    G = 0.5 * (G + np.swapaxes(G, 1, 2))
    # radial functions g_c(R): 7 exponentials and one dispersion term
    g = [np.exp(-(1.25 ** c) * (R_ang - 3.0)) for c in range(7)]
    g.append(-(3.0 / R_ang) ** 6)
    g = np.stack(g)                                      # [8, K]
    scale = np.array([100.0] + [30.0] * (len(ANGULAR_TERMS) - 1))
    if theta is None:
        theta = rng_pot.standard_normal((len(ANGULAR_TERMS), 8))
        theta[0, 6] = 5.0                                # repulsive wall of the isotropic term
    theta = np.asarray(theta, np.float64).reshape(len(ANGULAR_TERMS), 8)
    radial = (scale[:, None, None] * g[None, :, :]).reshape(-1, K)   # [96, K] cm^-1
    gidx = np.repeat(np.arange(len(ANGULAR_TERMS)), 8).astype(np.int32)
    V_t = (theta.reshape(-1)[:, None] * radial).reshape(len(ANGULAR_TERMS), 8, K).sum(1)
    M_cm = np.einsum("tk,tab->kab", V_t, G)
    # Coriolis J_x = j1x + j2x in the product basis
    index = {c: i for i, c in enumerate(chans)}
    jr, jc, jv = [], [], []
    for i, (j1, m1, j2, m2) in enumerate(chans):
        for dm in (-1, 1):
            if abs(m1 + dm) <= j1:
                mm = m1 + dm
                jr.append(i); jc.append(index[(j1, mm, j2, m2)])
                jv.append(0.5 * math.sqrt(j1 * (j1 + 1) - m1 * mm))
            if abs(m2 + dm) <= j2:
                mm = m2 + dm
                jr.append(i); jc.append(index[(j1, m1, j2, mm)])
                jv.append(0.5 * math.sqrt(j2 * (j2 + 1) - m2 * mm))
    return System(
        name="rotor_rotor_j%d" % jmax,
        R_grid=U.ang_to_bohr(R_ang), E=U.cm_to_hartree(np.array(E)), M=U.cm_to_hartree(M_cm),
        jx_row=np.array(jr, np.int32), jx_col=np.array(jc, np.int32),
        jx_val=np.array(jv, np.float64), mu=U.amu_to_me(mu_amu),
        level_of_channel=np.array(lev, np.int32), n_levels=len(level_ids),
        labels={"chans": chans, "R_ang": R_ang, "V_t_cm": V_t},
        param_radial=U.cm_to_hartree(radial), param_G_index=gidx, G=G,
        theta=theta.reshape(-1).copy())


def parametric_tables(system, theta):
    """M(R_k) = sum_p theta_p radial_p(R_k) G_{gidx_p} for a new coefficient vector."""
    theta = np.asarray(theta, np.float64)
    nG = system.G.shape[0]
    Vt = np.zeros((nG, system.K))
    for p in range(theta.shape[0]):
        Vt[system.param_G_index[p]] += theta[p] * system.param_radial[p]
    return np.einsum("tk,tab->kab", Vt, system.G)


# ---------------------------------------------------------------------------
# system 5: large random Hermitian tables


def large_random_system(N=4096, K=200, s_cm=2.0, mu_amu=9.0, cfg_index=5, Q=32,
                        E_span_cm=2000.0, build_tables=True, dtype=np.complex128, workers=16,
                        R_ang=None):
    """N random Hermitian channels (the N = 4096 workload); the GP factors are
    drawn on `workers` threads (0: one serial stream).  R_ang: the radial grid in
    angstrom (default K points uniform on 2-20 A)."""
    rng_pot, rng_tab, _ = _streams(cfg_index)
    params = _legendre_potential_params(rng_pot, lam_max=0)
    R_ang = np.linspace(2.0, 20.0, K) if R_ang is None else np.asarray(R_ang, np.float64)
    v_iso = _v_lambda_cm(params, R_ang)[0]
    E = np.sort(rng_pot.uniform(0.0, 1.0, N)) * E_span_cm
    omega, phase, H = gp_factors(rng_tab, N, Q=Q, workers=workers)
    sysm = System(
        name="random_N%d" % N, R_grid=U.ang_to_bohr(R_ang), E=U.cm_to_hartree(E),
        M=None, jx_row=np.zeros(0, np.int32), jx_col=np.zeros(0, np.int32),
        jx_val=np.zeros(0), mu=U.amu_to_me(mu_amu),
        level_of_channel=np.arange(N, dtype=np.int32), n_levels=N,
        labels={"R_ang": R_ang, "V_iso_cm": v_iso, "gp": (omega, phase, H), "s_cm": s_cm})
    if build_tables:
        sysm.M = U.cm_to_hartree(gp_tables_cm(omega, phase, H, R_ang, s_cm, v_iso)).astype(dtype)
    return sysm


def gp_tables_device(system, device):
    """The tables of a large random system built on a GPU with torch (hartree,
    complex128 [K, N, N]): the same construction as gp_tables_cm, for sizes whose
    tables do not fit comfortably in host memory."""
    import torch
    omega, phase, H = system.labels["gp"]
    R_ang = system.labels["R_ang"]
    s_cm = system.labels["s_cm"]
    v_iso = system.labels["V_iso_cm"]
    K = R_ang.shape[0]
    Q, N, _ = H.shape
    phi = gp_basis(omega, phase, R_ang) * (s_cm * np.exp(-(R_ang - 3.0)))[:, None]
    phi_t = torch.as_tensor(U.cm_to_hartree(phi), dtype=torch.float64, device=device)
    Hd = torch.as_tensor(H, device=device).reshape(Q, N * N)
    M = torch.empty((K, N, N), dtype=torch.complex128, device=device)
    Mr = torch.view_as_real(M).view(K, N * N, 2)
    Mr[:, :, 0] = phi_t @ Hd.real
    Mr[:, :, 1] = phi_t @ Hd.imag
    del Hd
    diag = torch.as_tensor(U.cm_to_hartree(v_iso), dtype=torch.float64, device=device)
    for k in range(K):
        Mk = M[k]
        Mk.copy_(0.5 * (Mk + Mk.conj().transpose(0, 1).contiguous()))
        Mk.diagonal().real.add_(diag[k])
    return M


def gp_rank_factors(system):
    """The generator's factors of a random-table system: phi [K, Q] and v_iso [K]
    in cm^-1 on its grid, the H_q [Q, N, N] and the cm^-1 -> hartree scale, so that
    M(R_k) = scale (sum_q phi[k, q] H_q + v_iso[k] 1)."""
    omega, phase, H = system.labels["gp"]
    R_ang = system.labels["R_ang"]
    phi = gp_basis(omega, phase, R_ang) * (system.labels["s_cm"] * np.exp(-(R_ang - 3.0)))[:, None]
    return phi, np.asarray(system.labels["V_iso_cm"], np.float64), H, U.cm_to_hartree(1.0)


def gp_knot_tables(system, ks):
    """Tables of a large random system at selected knots only (hartree, complex128)."""
    omega, phase, H = system.labels["gp"]
    R_ang = system.labels["R_ang"][np.asarray(ks)]
    v_iso = system.labels["V_iso_cm"][np.asarray(ks)]
    return U.cm_to_hartree(gp_tables_cm(omega, phase, H, R_ang, system.labels["s_cm"], v_iso))


# ---------------------------------------------------------------------------
# trajectory batches


def mc_batch(system, n_traj, U_cm, b_max_ang, init_channels, rng, n_steps=None, dt=None,
             system_index=0, R0_bohr=None):
    """Monte-Carlo initial conditions: b ~ U(0, b_max), initial channel uniform over a set."""
    U_cm = np.broadcast_to(np.asarray(U_cm, np.float64), (n_traj,)).copy()
    E_coll = U.cm_to_hartree(U_cm)
    b = U.ang_to_bohr(rng.uniform(0.0, b_max_ang, n_traj))
    ch = np.asarray(init_channels)[rng.integers(0, len(init_channels), n_traj)].astype(np.int32)
    R0 = np.full(n_traj, system.R_grid[-1] if R0_bohr is None else R0_bohr)
    T = collision_time(R0, E_coll, system.mu)
    if dt is None:
        dt = T / n_steps
        steps = np.full(n_traj, n_steps, np.int64)
    else:
        dt = np.full(n_traj, float(dt))
        steps = np.ceil(T / dt).astype(np.int64) if n_steps is None else \
            np.full(n_traj, n_steps, np.int64)
    return Batch(np.full(n_traj, system_index, np.int32), ch, E_coll, b, R0,
                 np.asarray(dt, np.float64), steps, U.ang_to_bohr(b_max_ang),
                 system.level_of_channel[ch].astype(np.int32))


def config1(n_traj=64, n_steps=2000, jmax=6, K=200):
    """Rotor + atom, N = 49, U = 500 cm^-1, b in 0-10 A, j' = 2 with random m'."""
    sysm = rotor_atom_system(jmax=jmax, K=K)
    _, _, rng = _streams(1)
    init = np.where(sysm.labels["j"] == min(2, jmax))[0]
    batch = mc_batch(sysm, n_traj, 500.0, 10.0, init, rng, n_steps=n_steps)
    return [sysm], batch


def config2(n_traj=4096, jmax=8, K=200, full_collision=True, window_steps=None, dt=12.0):
    """Asymmetric top + atom, N = 969.

    full_collision=True: every trajectory starts at the grid end and runs T(U)/dt steps.
    full_collision=False: a mid-collision population for throughput measurement,
    R0 ~ U(4, 19.5) A, every trajectory advancing window_steps steps.
    """
    sysm = top_atom_system(jmax=jmax, K=K)
    _, _, rng = _streams(2)
    init = np.where(sysm.labels["j"] <= 2)[0]
    if full_collision:
        U_cm = rng.uniform(100.0, 2000.0, n_traj)
        batch = mc_batch(sysm, n_traj, U_cm, 12.0, init, rng, dt=dt)
    else:
        U_cm = rng.uniform(100.0, 2000.0, n_traj)
        R0_ang = rng.uniform(4.0, 19.5, n_traj)
        b_ang = rng.uniform(0.0, 1.0, n_traj) * np.minimum(12.0, 0.9 * R0_ang)
        ch = init[rng.integers(0, len(init), n_traj)].astype(np.int32)
        batch = Batch(np.zeros(n_traj, np.int32), ch, U.cm_to_hartree(U_cm),
                      U.ang_to_bohr(b_ang), U.ang_to_bohr(R0_ang), np.full(n_traj, dt),
                      np.full(n_traj, window_steps or 10, np.int64), U.ang_to_bohr(12.0),
                      sysm.level_of_channel[ch].astype(np.int32))
    return [sysm], batch


def config4(n_traj=1024, n_steps=4096, jmax=3, K=200, theta=None):
    """Rotor + rotor, N = 256, potential linear in 96 coefficients."""
    sysm = rotor_rotor_system(jmax=jmax, K=K, theta=theta)
    _, _, rng = _streams(4)
    chans = sysm.labels["chans"]
    j0 = min(1, jmax)
    init = np.array([i for i, c in enumerate(chans) if c[0] == j0 and c[2] == j0])
    batch = mc_batch(sysm, n_traj, 500.0, 10.0, init, rng, n_steps=n_steps)
    return [sysm], batch


def config3(n_traj=20000, split=(0.6, 0.3, 0.1), jmax=(6, 3, 8), K=200):
    """Uneven mix of three systems with log-uniform energies (adaptive DP5)."""
    systems = [rotor_atom_system(jmax=jmax[0], K=K, cfg_index=1),
               rotor_rotor_system(jmax=jmax[1], K=K, cfg_index=4),
               top_atom_system(jmax=jmax[2], K=K, cfg_index=2)]
    _, _, rng = _streams(3)
    counts = [int(round(f * n_traj)) for f in split]
    counts[-1] = n_traj - sum(counts[:-1])
    bmax = [10.0, 10.0, 12.0]
    parts = []
    for si, (s, c) in enumerate(zip(systems, counts)):
        if c == 0:
            continue
        U_cm = np.exp(rng.uniform(math.log(10.0), math.log(5000.0), c))
        if si == 0:
            init = np.where(s.labels["j"] == min(2, jmax[0]))[0]
        elif si == 1:
            init = np.array([i for i, ch in enumerate(s.labels["chans"])
                             if ch[0] == min(1, jmax[1]) and ch[2] == min(1, jmax[1])])
        else:
            init = np.where(s.labels["j"] <= 2)[0]
        bt = mc_batch(s, c, U_cm, bmax[si], init, rng, n_steps=1000, system_index=si)
        parts.append(bt)
    cat = lambda f: np.concatenate([getattr(p, f) for p in parts])
    batch = Batch(cat("system_index"), cat("init_channel"), cat("E_coll"), cat("b"),
                  cat("R0"), cat("dt"), cat("n_steps"), U.ang_to_bohr(12.0),
                  cat("init_level"))
    perm = rng.permutation(batch.B)
    return systems, batch.subset(perm)


def config5(n_traj=512, n_steps=10000, N=4096, K=200, build_tables=True, dtype=np.complex128):
    sysm = large_random_system(N=N, K=K, build_tables=build_tables, dtype=dtype)
    _, _, rng = _streams(5)
    init = np.arange(min(16, N))
    batch = mc_batch(sysm, n_traj, 1000.0, 12.0, init, rng, n_steps=n_steps)
    return [sysm], batch
