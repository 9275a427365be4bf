"""Pins of the oracle's event-level steps (CPU only): cross-section weights,
hit-or-miss unweighting, and the event-by-event choice of a helicity and a
leading colour flow.

The pins are closed forms and properties that do not retype the oracle's
formulas:
  - the e+e- -> mu+mu- (photon only) and g g -> t t~ (Combridge) total cross
    sections, in pb, from the weights' sums, within the Monte Carlo error that
    the same sums give;
  - that error against the scatter of independent runs;
  - unweighted e+e- -> mu+mu- events distributed as 1 + cos^2(theta), and an
    acceptance equal to <w>/w_ref;
  - the helicity choice for e+e- -> mu+mu- against the per-helicity closed
    form (u^2 for equal e-/mu- helicities, t^2 for opposite ones, with the Z
    couplings);
  - the colour choice for g g -> t t~ against the relation
    (t - m^2) A(1,2) = (u - m^2) A(2,1) between its two colour-ordered
    amplitudes (so the two flows' weights are in the ratio
    (u - m^2)^2 : (t - m^2)^2), and for more gluons against Bose symmetry
    (relabelling two final gluons permutes the flows);
  - choice frequencies on a uniform grid of random numbers against the
    weights.
"""
import math

import numpy as np
import pytest

ALPHA = 1.0 / 132.5
SW2 = 0.2222
MZ, WZ = 91.188, 2.441
MT = 173.0
GEV2PB = 0.3893793721e9  # (hbar c)^2 in GeV^2 pb (PDG)


def mdot(a, b):
    return a[..., 0] * b[..., 0] - a[..., 1] * b[..., 1] - a[..., 2] * b[..., 2] - a[..., 3] * b[..., 3]


def masses_for(pdg):
    return [MT if abs(x) == 6 else 0.0 for x in pdg[2:]]


def _sigma(st, n):
    mean = st[0] / n
    err = math.sqrt(max(st[1] / n - mean * mean, 0.0) / (n - 1))
    return mean, err


def test_cross_section_ee_photon(oracle_mod):
    P = oracle_mod.Process(oracle_mod.PROCESSES["ee_mumu"], z_enabled=0)
    n = 60000
    mom, wgt = oracle_mod.rambo([0.0, 0.0], 500.0, 17, 0, n)
    w, st = oracle_mod.event_weights(wgt, P.me(mom, nthreads=8), 500.0)
    sigma, err = _sigma(st, n)
    s = 500.0 ** 2
    exact = 4 * math.pi * ALPHA ** 2 / (3 * s) * GEV2PB
    assert abs(sigma - exact) < 4 * err, (sigma, exact, err)
    assert err < 2e-3 * exact
    assert st[2] == w.max() and np.all(w > 0)


def test_weight_sums_exactly_rounded(oracle_mod):
    """Heavy-tailed weights: the sums equal the exactly rounded sums."""
    rng = np.random.default_rng(4)
    n = 200000
    wgt = np.exp(rng.normal(-12.0, 0.5, n))
    me = np.exp(rng.normal(-20.0, 3.0, n))
    w, st = oracle_mod.event_weights(wgt, me, 1500.0)
    assert abs(st[0] / math.fsum(w.tolist()) - 1.0) <= 2.3e-16
    assert abs(st[1] / math.fsum((w * w).tolist()) - 1.0) <= 4.5e-16  # w*w rounded once more in fsum's input
    assert st[2] == w.max()


def test_cross_section_gg_tt_combridge(oracle_mod):
    P = oracle_mod.Process(oracle_mod.PROCESSES["gg_tt"])
    n = 40000
    mom, wgt = oracle_mod.rambo([MT, MT], 1500.0, 23, 0, n)
    _, st = oracle_mod.event_weights(wgt, P.me(mom, nthreads=8), 1500.0)
    sigma, err = _sigma(st, n)
    s = 1500.0 ** 2
    rho = 4 * MT * MT / s
    beta = math.sqrt(1 - rho)
    exact = (math.pi * 0.118 ** 2 / (3 * s)) * ((1 + rho + rho ** 2 / 16) * math.log((1 + beta) / (1 - beta))
                                                 - beta * (7 / 4 + 31 * rho / 16)) * GEV2PB
    assert abs(sigma - exact) < 4 * err, (sigma, exact, err)


def test_error_estimate_matches_scatter(oracle_mod):
    """The error from sum w and sum w^2 predicts the spread of independent runs."""
    P = oracle_mod.Process(oracle_mod.PROCESSES["gg_tt"])
    n, runs = 2000, 40
    sig, errs = [], []
    for k in range(runs):
        mom, wgt = oracle_mod.rambo([MT, MT], 1500.0, 1000 + k, 0, n)
        _, st = oracle_mod.event_weights(wgt, P.me(mom, nthreads=8), 1500.0)
        a, b = _sigma(st, n)
        sig.append(a)
        errs.append(b)
    spread = np.std(sig, ddof=1)
    predicted = np.sqrt(np.mean(np.square(errs)))
    # the sample standard deviation of 40 runs is known to about 11%
    assert 0.7 < spread / predicted < 1.3, (spread, predicted)


def test_unweighting_acceptance_and_shape(oracle_mod):
    P = oracle_mod.Process(oracle_mod.PROCESSES["ee_mumu"], z_enabled=0)
    n = 60000
    mom, wgt = oracle_mod.rambo([0.0, 0.0], 500.0, 31, 0, n)
    w, st = oracle_mod.event_weights(wgt, P.me(mom, nthreads=8), 500.0)
    r = np.random.default_rng(3).random(n)
    idx = oracle_mod.unweight(w, r, st[2])
    assert np.all(np.diff(idx) > 0)
    # acceptance <w>/w_max = <1 + c^2> / 2 = 2/3 for the photon-only process
    acc = len(idx) / n
    assert abs(acc - 2 / 3) < 4 * math.sqrt(acc * (1 - acc) / n)
    # kept events follow (3/8)(1 + c^2) in c = cos(theta between e- and mu-)
    p1, p4 = mom[idx, 1], mom[idx, 3]
    c = (p1[:, 1:] * p4[:, 1:]).sum(1) / (np.linalg.norm(p1[:, 1:], axis=1) * np.linalg.norm(p4[:, 1:], axis=1))
    edges = np.linspace(-1, 1, 11)
    counts, _ = np.histogram(c, edges)
    cdf = lambda x: (3 * x + x ** 3) / 8
    expect = len(idx) * (cdf(edges[1:]) - cdf(edges[:-1]))
    chi2 = ((counts - expect) ** 2 / expect).sum()
    assert chi2 < 30, chi2  # 9 degrees of freedom; a flat distribution gives ~500


def test_unweighting_special_cases(oracle_mod):
    w = np.array([0.0, 1.0, 2.0, 2.0, 0.5])
    r = np.array([1e-300, 0.999999999, 0.999999999, 0.5, 0.25])
    # w_ref = 2: a zero weight never survives; r * 2 < w decides the rest,
    # strictly (event 4 has r * 2 == w and is dropped)
    assert oracle_mod.unweight(w, r, 2.0).tolist() == [2, 3]
    # every event at the reference weight survives (r < 1)
    assert oracle_mod.unweight(np.full(5, 3.0), r, 3.0).tolist() == [0, 1, 2, 3, 4]
    assert oracle_mod.unweight(np.zeros(0), np.zeros(0), 1.0).tolist() == []


def _ee_helicity_weights(p, z):
    """Closed-form per-helicity |M_h|^2 (up to a common factor) in code order."""
    s = mdot(p[0] + p[1], p[0] + p[1])
    t = -2 * mdot(p[0], p[2])
    u = -2 * mdot(p[0], p[3])
    cw2 = 1 - SW2
    gl, gr = -0.5 + SW2, SW2
    zf = (lambda gi, gj: gi * gj / (SW2 * cw2 * (s - MZ ** 2 + 1j * MZ * WZ))) if z else (lambda gi, gj: 0.0)
    A = {k: 1 / s + zf(*g) for k, g in {"LL": (gl, gl), "RR": (gr, gr), "LR": (gl, gr), "RL": (gr, gl)}.items()}
    wts = np.zeros(16)
    wts[0b1010] = abs(A["LL"]) ** 2 * u ** 2
    wts[0b0101] = abs(A["RR"]) ** 2 * u ** 2
    wts[0b1001] = abs(A["LR"]) ** 2 * t ** 2
    wts[0b0110] = abs(A["RL"]) ** 2 * t ** 2
    return wts


@pytest.mark.parametrize("z", [0, 1])
def test_helicity_choice_ee_closed_form(oracle_mod, z):
    P = oracle_mod.Process(oracle_mod.PROCESSES["ee_mumu"], z_enabled=z)
    mom, _ = oracle_mod.rambo([0.0, 0.0], 500.0, 5, 0, 12)
    grid = (np.arange(97) + 0.5) / 97
    for p in mom:
        cum = np.cumsum(_ee_helicity_weights(p, z))
        cum /= cum[-1]
        for r in grid:
            h, col, margin = P.select(p, r, 0.5)
            assert col == 0
            k = int(np.searchsorted(cum, r, side="right"))
            if abs(cum[k] - r) > 1e-9 and (k == 0 or abs(cum[k - 1] - r) > 1e-9):
                assert h == k, (r, h, k)


def test_colour_choice_gg_tt_ordered_amplitudes(oracle_mod):
    """Flow 0 = (T^a1 T^a2) and flow 1 = (T^a2 T^a1) carry weights in the ratio
    (u - m^2)^2 : (t - m^2)^2 with t = (p1 - p3)^2, u = (p1 - p4)^2."""
    P = oracle_mod.Process(oracle_mod.PROCESSES["gg_tt"])
    mom, _ = oracle_mod.rambo([MT, MT], 1500.0, 9, 0, 20)
    for p in mom:
        t = mdot(p[0] - p[2], p[0] - p[2]) - MT * MT
        u = mdot(p[0] - p[3], p[0] - p[3]) - MT * MT
        f0 = u * u / (u * u + t * t)
        for r in (f0 * (1 - 1e-9), f0 * (1 + 1e-9)):
            _, col, _ = P.select(p, 0.5, r)
            assert col == (0 if r < f0 else 1), (r, f0)


@pytest.mark.parametrize("name", ["gg_ttg", "gg_ttgg"])
def test_colour_choice_bose_symmetry(oracle_mod, name):
    """Exchanging the momenta of two gluons exchanges their labels in
    every flow: the boundary between consecutive flows moves accordingly, so
    the choice frequencies on a grid map onto each other."""
    P = oracle_mod.Process(oracle_mod.PROCESSES[name])
    _, _, basis = P.colour_matrix()
    basis = [tuple(b) for b in basis.tolist()]
    # two gluons of the same side: the initial pair for one final gluon
    a, b = (0, 1) if name == "gg_ttg" else (4, 5)
    swap = {a: b, b: a}
    perm = [basis.index(tuple(swap.get(l, l) for l in f)) for f in basis]
    mom, _ = oracle_mod.rambo(masses_for(oracle_mod.PROCESSES[name]), 1500.0, 4, 0, 3)
    grid = (np.arange(400) + 0.5) / 400
    for p in mom:
        q = p.copy()
        q[[a, b]] = p[[b, a]]
        f = np.zeros(len(basis))
        g = np.zeros(len(basis))
        for r in grid:
            f[P.select(p, 0.5, r)[1]] += 1
            g[P.select(q, 0.5, r)[1]] += 1
        # flow s at p has the weight of flow perm[s] at q; each count is its
        # weight times the grid size to within one grid step at either end
        assert np.abs(f - g[perm]).max() <= 2, (f, g[perm])
        assert np.abs(f - g).max() > 2  # the exchange does move weight between flows


def test_choice_frequencies_follow_weights(oracle_mod):
    """On a uniform grid of r the helicity frequencies equal |M_h|^2 / |M|^2."""
    P = oracle_mod.Process(oracle_mod.PROCESSES["gg_ttg"])
    mom, _ = oracle_mod.rambo([MT, MT, 0.0], 1500.0, 8, 0, 2)
    K = 4000
    grid = (np.arange(K) + 0.5) / K
    for p in mom:
        wts = P.me_hel(p)
        cnt = np.zeros(len(wts))
        for r in grid:
            cnt[P.select(p, r, 0.5)[0]] += 1
        np.testing.assert_allclose(cnt / K, wts / wts.sum(), atol=1.0 / K + 1e-12)
