"""GPU parity of the cross-section post-processing (Section III, Eqs. 19-20, rates).

* Eq. 19 ratios and Eq. 20 symmetrised cross sections against the oracle (zeros
  included, where the ratio is NaN);
* rate coefficients against the oracle (scipy spline and adaptive quadrature) at
  the paper's ten collision energies and temperatures from 5 to 2000 K, with level
  energies of the paper's H2O + H2 check basis: relative 1e-10; thresholds above
  the first and above the last energy; detailed balance of the GPU rates;
* the whole chain on one system -- propagation at three energies, Monte-Carlo cross
  sections, symmetrisation, rates -- against the oracle's chain.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import postproc as PP
from synth import systems as S
from synth import units as U_

pytestmark = pytest.mark.gpu

KB_HARTREE = 3.166811563e-6          # Boltzmann constant, hartree per kelvin
PAPER_U_CM = [20.0, 41.28, 84.0, 170.47, 346.41, 703.89, 1430.0, 2906.3, 5906.0, 12000.0]


def say(msg):
    print("[gpu] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context()
    yield c
    c.synchronize()
    c.close()


def test_symmetrize_matches_oracle(ctx):
    rng = np.random.default_rng(11)
    nE, L = 10, 30
    g = rng.integers(1, 40, L).astype(float)
    sigma = rng.random((nE, L, L)) * 50.0
    sigma[rng.random((nE, L, L)) < 0.1] = 0.0
    say("Eq. 19/20 on %d energies x %d levels" % (nE, L))
    sym, ratio = ctx.xs_symmetrize(sigma, g)
    assert np.max(np.abs(sym - PP.symmetrize(sigma, g))) <= 1e-15 * np.max(np.abs(sym))
    r_o = PP.reversibility_ratio(sigma, g)
    assert np.array_equal(np.isnan(ratio), np.isnan(r_o))
    nz = ~np.isnan(r_o) & (r_o != 0.0)
    assert np.max(np.abs(ratio[nz] - r_o[nz]) / np.abs(r_o[nz])) < 1e-15
    assert np.all(ratio[r_o == 0.0] == 0.0)


def paper_levels():
    """Level energies and degeneracies of the (j1_{kA kC}, j2) levels of Section II's check."""
    from synth import coupling as CP
    b = CP.paper_check_basis()
    E, g = [], []
    for lev in range(b.n_levels):
        n = int(np.where(b.level_of_channel == lev)[0][0])
        E.append(b.E[n])
        g.append(int(np.sum(b.level_of_channel == lev)))
    return np.array(E), np.array(g, float)


def compare_rates(k, k_o):
    tiny = 1e-290
    big = np.abs(k_o) > tiny
    rel = np.abs(k[big] - k_o[big]) / np.abs(k_o[big])
    assert np.all(np.abs(k[~big]) <= 1e-280)
    return float(rel.max())


def test_rates_match_oracle(ctx):
    rng = np.random.default_rng(12)
    E, g = paper_levels()
    L = E.shape[0]
    U = U_.cm_to_hartree(np.array(PAPER_U_CM))
    # smooth positive cross sections: A_if (U/U_1)^p exp(-U/U_c)
    A = rng.random((L, L)) * 30.0
    p = 0.2 + 0.6 * rng.random((L, L))
    Uc = U_.cm_to_hartree(3000.0 + 6000.0 * rng.random((L, L)))
    sigma = A[None] * (U[:, None, None] / U[0]) ** p[None] * np.exp(-U[:, None, None] / Uc[None])
    sym = PP.symmetrize(sigma, g)
    T = np.array([5.0, 20.0, 100.0, 300.0, 1000.0, 2000.0])
    beta = KB_HARTREE * T
    mu = U_.amu_to_me(1.8)
    say("rates: %d levels, %d energies, %d temperatures" % (L, U.size, T.size))
    k = ctx.rate_coefficients(U, sym, E, g, mu, beta)
    pairs = [tuple(x) for x in rng.integers(0, L, (120, 2))]
    k_o = PP.rate_coefficients(U, sym, E, g, mu, beta, pairs=pairs)
    k_s = np.stack([k[:, i, f] for i, f in pairs], axis=1)
    rel = compare_rates(k_s, k_o)
    say("  %d sampled transitions: max relative difference %.2e" % (len(pairs), rel))
    assert rel < 1e-10
    for t, b in enumerate(beta):
        lhs = g[:, None] * k[t] * np.exp(-(E - E.min()) / b)[:, None]
        ok = np.abs(lhs) > 1e-250
        assert np.max(np.abs(lhs - lhs.T)[ok] / np.abs(lhs)[ok]) < 1e-12


def test_rates_with_thresholds_beyond_the_energies(ctx):
    """Level gaps that put the threshold |dE|/2 above the first and above the last
    computed energy."""
    U = np.array([0.001, 0.002, 0.004, 0.008])
    E = np.array([0.0, 0.004, 0.03])          # thresholds 0.002, 0.015, 0.013
    g = np.array([1.0, 3.0, 5.0])
    rng = np.random.default_rng(13)
    sym = PP.symmetrize(rng.random((U.size, 3, 3)) * 10, g)
    beta = np.array([0.0005, 0.003, 0.02])
    k = ctx.rate_coefficients(U, sym, E, g, 1000.0, beta)
    k_o = PP.rate_coefficients(U, sym, E, g, 1000.0, beta)
    assert compare_rates(k, k_o) < 1e-10


def test_whole_chain_against_the_oracle_chain(ctx):
    """Propagation at three energies -> cross sections -> Eq. 20 -> rates."""
    sysm = S.rotor_atom_system(jmax=3, K=200)
    rng = np.random.default_rng(14)
    U_cm = [200.0, 500.0, 1200.0]
    n_levels = sysm.n_levels
    init = np.arange(sysm.N)                              # every channel, every level
    sig_g, sig_o = [], []
    sid = ctx.load_system(sysm)
    for e, u in enumerate(U_cm):
        b = S.mc_batch(sysm, 48, u, 8.0, init, np.random.default_rng(100 + e), n_steps=600)
        g_run = ctx.run_host([sid] * b.B, [sysm.N] * b.B, init_channel=b.init_channel,
                             E_coll=b.E_coll, b=b.b, R0=b.R0, dt=b.dt, n_steps=b.n_steps,
                             schedule="gemv")
        import torch
        P = torch.as_tensor(g_run["P"].reshape(b.B, sysm.N), device=ctx.device)
        sig_g.append(ctx.cross_sections(P, b.b, b.init_level, sysm.level_of_channel, n_levels,
                                        b.b_max).cpu().numpy())
        o = oracle.OracleSystem(sysm).propagate(b)
        sig_o.append(oracle.cross_sections(b.init_level, b.b, o["P"], sysm.level_of_channel,
                                           n_levels, b.b_max))
    ctx.free_system(sid)
    sig_g, sig_o = np.array(sig_g), np.array(sig_o)
    g = np.bincount(sysm.level_of_channel).astype(float)
    E = np.array([sysm.E[np.where(sysm.level_of_channel == l)[0][0]] for l in range(n_levels)])
    U = U_.cm_to_hartree(np.array(U_cm))
    sym_g, _ = ctx.xs_symmetrize(sig_g, g)
    beta = KB_HARTREE * np.array([50.0, 300.0, 1000.0])
    k_g = ctx.rate_coefficients(U, sym_g, E, g, sysm.mu, beta)
    k_o = PP.rate_coefficients(U, PP.symmetrize(sig_o, g), E, g, sysm.mu, beta)
    rel = np.max(np.abs(k_g - k_o)) / np.max(np.abs(k_o))
    say("chain: %d levels, max difference of the rates %.2e of the largest" % (n_levels, rel))
    assert rel < 1e-8
