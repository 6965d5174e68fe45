"""Statistical pins of the oracle against what the paper fixes.

* Diffusion (2.3, eqs. 1-2; 3.1; appendix): the mean-squared displacement
  grows as 6 D t.  Checked for nearly lone walkers (the paper's own check,
  one molecule per walk) and at 1 % occupancy.
* First-order reactions (2.4.1; closed form of 3.2.1):
  [A_t] = [A_0] exp(-k t), [B_t] = [A_0](1 - exp(-k t)), at the paper's three
  rate constants 0.135, 1.35 and 13.5 1/s, for both laws.
* Reversible reactions (3.2.2): B + C <-> A started from A alone settles
  where the mean association flux equals the mean dissociation flux,
  k_f <N_B N_C> / V = k_b <N_A> (the law of mass action at equilibrium).
* Second-order reactions (2.4.2, eq. 6): with p = k / (6 sqrt2 (DA+DB) r) the
  reaction-limited rate is the mass-action rate k (checked at the paper's
  k_f = 0.027 1/(nM s), D = 10 um^2/s, r = 5 nm where p = 0.053); in the
  diffusion-limited limit (p clamped to 1) the rate approaches
  k_max / G(0), k_max = 6 sqrt2 (DA+DB) r, with G(0) the lattice Green's
  function at the origin, computed here from the oracle's stencil.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle

MODES = [oracle.MODE_C, oracle.MODE_S]


def voxel_volume(rv):
    return 4.0 * math.sqrt(2.0) * rv ** 3


def msd_slope_ratio(n_mol, events, seed, mode, dims=(64, 64, 64), rv=4.4e-9, D=1e-12,
                    max_lag=10):
    """time-averaged MSD over lags 1..max_lag from unwrapped integer
    displacements, least-squares slope through the origin, divided by 6D"""
    o = oracle.Oracle(dims, rv, seed)
    o.add_species(D)
    o.place_uniform(1, n_mol)
    traj = []
    for _ in range(events):
        o.run(1, mode)
        s = o.state(with_occ=False)
        traj.append(np.stack([s["dx"], s["dy"], s["dz"]]).astype(np.float64))
    traj = np.array(traj)
    tau = 2.0 * rv * rv / (3.0 * D)
    lags = np.arange(1, max_lag + 1)
    msd = []
    for lag in lags:
        d = traj[lag:] - traj[:-lag]
        r2 = rv ** 2 * (d[:, 0] ** 2 + d[:, 1] ** 2 / 3.0 + 8.0 * d[:, 2] ** 2 / 3.0)
        msd.append(r2.mean())
    t = lags * tau
    slope = float((np.array(msd) * t).sum() / (t * t).sum())
    return slope / (6.0 * D)


@pytest.mark.parametrize("mode", MODES)
def test_msd_lone_walkers_is_6Dt(mode):
    # 300 walkers on 262,144 voxels: occupancy 0.1 %, effectively free walks
    r = [msd_slope_ratio(300, 1500, seed, mode) for seed in (1, 2)]
    assert abs(np.mean(r) - 1.0) < 0.02, r


def test_msd_at_one_percent_occupancy():
    # the 64^3, 1 % occupancy workload; exclusion lowers the tracer slope
    # slightly (about 1 %), still within 2 % of 6 D
    r = msd_slope_ratio(2621, 1000, 1, oracle.MODE_C)
    assert abs(r - 1.0) < 0.02, r
    assert r < 1.0


def first_order_ratios(k, mode, n0, seed, t_end, events=150, rv=5e-9):
    """Immobile A -> B + C on 64^3 with a single mobile 'clock' molecule that
    sets the diffusion-event interval; first-order reactions are applied once
    per diffusion event (2.2) over the elapsed interval."""
    o = oracle.Oracle((64, 64, 64), rv, seed)
    tau_clock = t_end / events
    Dz = 2.0 * rv * rv / (3.0 * tau_clock)
    Z = o.add_species(Dz)
    A = o.add_species(0.0)
    B = o.add_species(0.0)
    Cc = o.add_species(0.0)
    o.add_reaction((A,), (B, Cc), k)
    o.place_uniform(Z, 1)
    o.place_uniform(A, n0)
    out = []
    for _ in range(events):
        o.run(1, mode)
        t = o.L.orc_time(o.h)
        na, nb, nc = o.species_count(A), o.species_count(B), o.species_count(Cc)
        out.append((t, na, nb, nc))
    return np.array(out)


@pytest.mark.parametrize("k", [0.135, 1.35, 13.5])
@pytest.mark.parametrize("mode", MODES)
def test_first_order_closed_form(k, mode):
    n0 = 30000
    res = first_order_ratios(k, mode, n0, seed=int(k * 1000) + mode, t_end=1.5 / k)
    t, na, nb, nc = res.T
    decay = np.exp(-k * t)
    assert np.all(np.abs(na / (n0 * decay) - 1.0) < 0.05)
    late = t > 0.3 / k
    assert np.all(np.abs(nb[late] / (n0 * (1.0 - decay[late])) - 1.0) < 0.05)
    assert np.array_equal(nb, nc)  # no placement failures in the dilute regime


@pytest.mark.parametrize("mode", MODES)
def test_first_order_with_mobile_reactant(mode):
    # the paper's setting: A, B, C all diffusing at D = 10 um^2/s, r = 5 nm,
    # k = 13.5 1/s (the validation lattice is smaller, same dilution order)
    rv, D, k, n0 = 5e-9, 10e-12, 13.5, 3000
    o = oracle.Oracle((64, 64, 64), rv, 21 + mode)
    A = o.add_species(D)
    B = o.add_species(D)
    Cc = o.add_species(D)
    o.add_reaction((A,), (B, Cc), k)
    o.place_uniform(A, n0)
    tau = 2.0 * rv * rv / (3.0 * D)
    events = int(0.03 / tau)
    o.run(events, mode)
    t = o.L.orc_time(o.h)
    exp_a = n0 * math.exp(-k * t)
    assert abs(o.species_count(A) / exp_a - 1.0) < 0.05
    assert abs(o.species_count(B) / (n0 - exp_a) - 1.0) < 0.05


def second_order_inverse(k, DA, DB, rv, n0, events, seed, mode, dims):
    o = oracle.Oracle(dims, rv, seed)
    A = o.add_species(DA)
    B = o.add_species(DB)
    Cc = o.add_species(DA)
    o.add_reaction((A, B), (Cc,), k)
    o.place_uniform(A, n0)
    o.place_uniform(B, n0)
    ts, inv = [], []
    for _ in range(events):
        o.run(1, mode)
        ts.append(o.L.orc_time(o.h))
        inv.append(1.0 / o.species_count(A) - 1.0 / n0)
    V = dims[0] * dims[1] * dims[2] * voxel_volume(rv)
    return np.array(ts), np.array(inv), V


@pytest.mark.parametrize("mode", MODES)
def test_second_order_reaction_limited_rate_is_mass_action(mode):
    # A + B -> C with N_A = N_B: 1/N_A(t) - 1/N_0 = k_eff t / V
    kf = 0.027 * 1e9 * 1e-3 / 6.02214076e23   # 0.027 1/(nM s) in m^3/s
    rv, D = 5e-9, 10e-12
    p = kf / (6 * math.sqrt(2) * 2 * D * rv)
    assert 0.05 < p < 0.06
    ratios = []
    for seed in range(10):
        t, inv, V = second_order_inverse(kf, D, D, rv, 2000, 1000, 100 + seed + 50 * mode,
                                         mode, (64, 64, 64))
        ratios.append(float((inv * t).sum() / (t * t).sum()) * V / kf)
    assert abs(np.mean(ratios) - 1.0) < 0.05, ratios


def green_origin(dims=(64, 64, 64), steps=600):
    """G(0) = sum_n P(walker at its start after n steps), from powers of the
    transition matrix built from the oracle's stencil; the n^(-3/2) tail
    beyond `steps` is added from the last half of the computed terms."""
    nb = oracle.neighbour_table(dims)
    nv = nb.shape[0]
    P = sp.csr_matrix((np.full(nv * 12, 1.0 / 12.0), (nb.ravel(), np.repeat(np.arange(nv), 12))),
                      shape=(nv, nv))
    p = np.zeros(nv)
    p[0] = 1.0
    terms = []
    for _ in range(steps):
        terms.append(p[0])
        p = P @ p
    terms = np.array(terms)
    n = np.arange(steps)
    c = float(np.mean(terms[steps // 2:] * n[steps // 2:] ** 1.5))
    return float(terms.sum() + 2.0 * c / math.sqrt(steps))


def test_green_function_of_the_hcp_walk():
    g = green_origin()
    # return probability F = 1 - 1/G(0) of a 12-neighbour close-packed walk
    assert 1.33 < g < 1.36


@pytest.mark.parametrize("mode", MODES)
def test_second_order_diffusion_limited_rate(mode):
    DA, DB, rv = 1e-12, 0.5e-12, 4.4e-9
    kmax = 6 * math.sqrt(2) * (DA + DB) * rv
    g0 = green_origin()
    ratios = []
    for seed in range(3):
        t, inv, V = second_order_inverse(1e-18, DA, DB, rv, 8000, 300, 200 + seed + 50 * mode,
                                         mode, (96, 96, 96))
        sel = t > t[60]  # past the initial transient
        A = np.vstack([t[sel], np.ones(sel.sum())]).T
        slope = np.linalg.lstsq(A, inv[sel], rcond=None)[0][0]
        ratios.append(slope * V / kmax)
    assert abs(np.mean(ratios) * g0 - 1.0) < 0.05, (ratios, 1 / g0)


@pytest.mark.parametrize("mode", MODES)
def test_first_order_coarse_interval_keeps_exponential_law(mode):
    # K dt = 0.5 per event: a linearised firing probability (K dt) or a
    # one-reaction-per-event reading would be far off exp(-k t)
    k, n0 = 1.35, 30000
    res = first_order_ratios(k, mode, n0, seed=31 + mode, t_end=6 * 0.5 / k, events=6)
    t, na, nb, nc = res.T
    assert np.all(np.abs(na / (n0 * np.exp(-k * t)) - 1.0) < 0.05)


@pytest.mark.parametrize("mode", MODES)
def test_first_order_branching_follows_rate_constants(mode):
    # A -> B (k1) and A -> C (k2): fraction of B among products = k1/(k1+k2)
    # (2.4.1, eq. 5)
    rv = 5e-9
    o = oracle.Oracle((64, 64, 64), rv, 41 + mode)
    tau_clock = 1e-3
    Z = o.add_species(2.0 * rv * rv / (3.0 * tau_clock))
    A = o.add_species(0.0)
    B = o.add_species(0.0)
    Cc = o.add_species(0.0)
    k1, k2 = 30.0, 90.0
    o.add_reaction((A,), (B,), k1)
    o.add_reaction((A,), (Cc,), k2)
    o.place_uniform(Z, 1)
    o.place_uniform(A, 20000)
    o.run(60, mode)
    nb, nc = o.species_count(B), o.species_count(Cc)
    assert nb + nc > 15000
    frac = nb / (nb + nc)
    assert abs(frac - k1 / (k1 + k2)) < 0.02


@pytest.mark.parametrize("mode", MODES)
def test_reversible_reaction_settles_at_mass_action_equilibrium(mode):
    """The reversible check of 3.2.2, B + C <-> A with D = 10 um^2/s and
    r = 5 nm, started from A alone (the text's initial numbers 0, 0, 64,000
    for A, B, C could not react at all; the figure's caption has A
    dissociating, so A starts at 64,000), scaled to 400 molecules on 40^3
    voxels with k_b = 1 / (600 tau) and k_f = k_b V / 200 (p = 0.27), so that
    equilibrium falls at N_A = N_B = 200 and is reached within a few hundred
    events.  The spatial model has no closed form in time (the paper compares
    with its serial program), but its equilibrium does: the mean fluxes
    balance, k_f <N_B N_C> / V = k_b <N_A>, because a dissociation places C
    on a uniformly chosen vacant neighbour and the walk leaves B-C pair
    placements uniform (the 12 contact states of a pair then react at the
    summed rate p (1/tau_B + 1/tau_C) / 12 each, which eq. 6 makes
    k_f / V per pair).  Averaged over 50,000 events (about 80 relaxation
    times; spread of the mean below 1 %), at 0.6 % occupancy (crowding
    shifts it by about that much)."""
    rv, D, dims, n0 = 5e-9, 10e-12, (40, 40, 40), 400
    V = dims[0] * dims[1] * dims[2] * voxel_volume(rv)
    tau = 2.0 * rv * rv / (3.0 * D)
    kb = 1.0 / (600.0 * tau)
    kf = kb * V / (n0 / 2)
    o = oracle.Oracle(dims, rv, 31 + mode)
    for _ in range(3):
        o.add_species(D)                  # A, B, C
    o.add_reaction((2, 3), (1,), kf)      # B + C -> A
    o.add_reaction((1,), (2, 3), kb)      # A -> B + C
    o.place_uniform(1, n0)
    o.run(2000, mode)
    na, nbc = [], []
    for _ in range(1000):
        o.run(50, mode)
        sp_count = np.bincount(o.state(with_occ=False)["species"], minlength=4)
        assert sp_count[2] == sp_count[3] and sp_count[1] + sp_count[2] == n0
        na.append(sp_count[1])
        nbc.append(sp_count[2] * sp_count[3])
    ratio = kf * np.mean(nbc) / (V * kb * np.mean(na))
    assert abs(ratio - 1.0) < 0.04, ratio
