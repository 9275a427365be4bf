"""Pins of the oracle's |M|^2 (CPU only).

e+e- -> mu+mu- (s-channel photon + Z) and g g -> t t~ against per-event closed
forms and total cross sections; g g -> t t~ + 1..3 gluons against gauge
invariance, Lorentz invariance, Bose symmetry, the brute-force colour sum,
the diagram and colour-flow counts, the published colour matrices and the
soft-gluon limit of the colour-ordered amplitudes.
"""
import math
import os
from itertools import permutations

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
MT = 173.0
SEED = 230318244


def mdot(a, b):
    return a[..., 0] * b[..., 0] - a[..., 1] * b[..., 1] - a[..., 2] * b[..., 2] - a[..., 3] * b[..., 3]


def masses_for(pdg):
    return [MT if abs(x) == 6 else 0.0 for x in pdg[2:]]


@pytest.fixture(scope="module")
def procs(oracle_mod):
    return {name: oracle_mod.Process(pdg) for name, pdg in oracle_mod.PROCESSES.items()}


def two_body(n, sqrt_s, m, seed=1):
    """Exactly on-shell 2 -> 2 kinematics from random angles: RAMBO's conformal
    boost can leave momenta off shell by ~1e-12 relative for nearly collinear
    pairs, which is too coarse for a 1e-13 closed-form pin."""
    rng = np.random.default_rng(seed)
    cost = rng.uniform(-1, 1, n)
    phi = rng.uniform(0, 2 * np.pi, n)
    e = sqrt_s / 2
    pa = math.sqrt(e * e - m * m)
    sint = np.sqrt(1 - cost ** 2)
    mom = np.zeros((n, 4, 4))
    mom[:, 0] = [e, 0, 0, e]
    mom[:, 1] = [e, 0, 0, -e]
    k = np.stack([np.full(n, e), pa * sint * np.cos(phi), pa * sint * np.sin(phi), pa * cost], axis=1)
    mom[:, 2] = k
    mom[:, 3] = k * np.array([1, -1, -1, -1])
    return mom


def events(oracle_mod, name, n, first=0, sqrt_s=None):
    pdg = oracle_mod.PROCESSES[name]
    if sqrt_s is None:
        sqrt_s = 500.0 if name == "ee_mumu" else 1500.0
    return oracle_mod.rambo(masses_for(pdg), sqrt_s, SEED, first, n)


# ----------------------------------------------------------------- e+e- -> mu+mu-
ALPHA = 1.0 / 132.5
SW2 = 0.2222
MZ, WZ = 91.188, 2.441


def ee_amplitudes(s):
    cw2 = 1 - SW2
    gl, gr = -0.5 + SW2, SW2
    a = lambda gi, gj: 1 / s + gi * gj / (SW2 * cw2 * (s - MZ ** 2 + 1j * MZ * WZ))
    return {"LL": a(gl, gl), "RR": a(gr, gr), "LR": a(gl, gr), "RL": a(gr, gl)}


def test_ee_closed_form_per_event(procs, oracle_mod):
    mom = two_body(200, 500.0, 0.0)
    me = procs["ee_mumu"].me(mom)
    s = 500.0 ** 2
    e4 = (4 * math.pi * ALPHA) ** 2
    t = -2 * mdot(mom[:, 0], mom[:, 2])  # massless legs: (p1 - p3)^2 = -2 p1.p3
    u = -2 * mdot(mom[:, 0], mom[:, 3])
    A = ee_amplitudes(s)
    ref = e4 * ((abs(A["LL"]) ** 2 + abs(A["RR"]) ** 2) * u ** 2 + (abs(A["LR"]) ** 2 + abs(A["RL"]) ** 2) * t ** 2)
    np.testing.assert_allclose(me, ref, rtol=1e-13)


def test_ee_per_helicity(procs, oracle_mod):
    mom = two_body(5, 500.0, 0.0)
    s = 500.0 ** 2
    e4 = (4 * math.pi * ALPHA) ** 2
    A = ee_amplitudes(s)
    for p in mom:
        hel = procs["ee_mumu"].me_hel(p)
        t = -2 * mdot(p[0], p[2])
        u = -2 * mdot(p[0], p[3])
        # helicity index: bit (3 - leg) set for helicity +1; legs e+ e- mu+ mu-
        expect = np.zeros(16)
        expect[0b1010] = e4 * abs(A["LL"]) ** 2 * u ** 2  # e-_L, mu-_L
        expect[0b0101] = e4 * abs(A["RR"]) ** 2 * u ** 2  # e-_R, mu-_R
        expect[0b1001] = e4 * abs(A["LR"]) ** 2 * t ** 2  # e-_L, mu-_R
        expect[0b0110] = e4 * abs(A["RL"]) ** 2 * t ** 2  # e-_R, mu-_L
        np.testing.assert_allclose(hel, expect, rtol=1e-13, atol=0)
        assert np.count_nonzero(hel) == 4  # the other twelve vanish exactly


def test_ee_photon_only(oracle_mod):
    P = oracle_mod.Process(oracle_mod.PROCESSES["ee_mumu"], z_enabled=0)
    mom = two_body(400, 500.0, 0.0)
    me = P.me(mom)
    s = 500.0 ** 2
    e4 = (4 * math.pi * ALPHA) ** 2
    t = -2 * mdot(mom[:, 0], mom[:, 2])  # massless legs: (p1 - p3)^2 = -2 p1.p3
    u = -2 * mdot(mom[:, 0], mom[:, 3])
    np.testing.assert_allclose(me, 2 * e4 * (t ** 2 + u ** 2) / s ** 2, rtol=1e-13)
    mom, w = events(oracle_mod, "ee_mumu", 20000)
    me = P.me(mom)
    # total cross section 4 pi alpha^2 / (3 s), Monte Carlo with RAMBO weights
    f = w * me / (2 * s)
    sigma, err = f.mean(), f.std() / math.sqrt(len(f))
    assert abs(sigma - 4 * math.pi * ALPHA ** 2 / (3 * s)) < 4 * err


# -------------------------------------------------------------------- g g -> t t~
def esw(p):
    s = mdot(p[:, 0] + p[:, 1], p[:, 0] + p[:, 1])
    gs4 = (4 * math.pi * 0.118) ** 2
    t1 = 2 * mdot(p[:, 0], p[:, 2]) / s
    t2 = 2 * mdot(p[:, 1], p[:, 2]) / s
    rho = 4 * MT * MT / s
    return gs4 * (1 / (6 * t1 * t2) - 3 / 8) * (t1 ** 2 + t2 ** 2 + rho - rho ** 2 / (4 * t1 * t2))


def test_ggtt_closed_form(procs, oracle_mod):
    mom = two_body(400, 1500.0, MT)
    np.testing.assert_allclose(procs["gg_tt"].me(mom), esw(mom), rtol=1e-13)


def test_ggtt_total_cross_section(procs, oracle_mod):
    # Combridge: sigma = pi as^2/(3s) [(1 + rho + rho^2/16) ln((1+b)/(1-b)) - b (7/4 + 31 rho/16)]
    mom, w = events(oracle_mod, "gg_tt", 20000)
    me = procs["gg_tt"].me(mom)
    s = 1500.0 ** 2
    rho = 4 * MT * MT / s
    beta = math.sqrt(1 - rho)
    sig = (math.pi * 0.118 ** 2 / (3 * s)) * ((1 + rho + rho ** 2 / 16) * math.log((1 + beta) / (1 - beta))
                                               - beta * (7 / 4 + 31 * rho / 16))
    f = w * me / (2 * s)
    assert abs(f.mean() - sig) < 4 * f.std() / math.sqrt(len(f))


# ------------------------------------------------------------------ multi-gluon
COUNTS = {"gg_tt": (3, 2, 16), "gg_ttg": (16, 6, 32), "gg_ttgg": (123, 24, 64), "gg_ttggg": (1240, 120, 128)}


@pytest.mark.parametrize("name", list(COUNTS))
def test_counts(procs, name):
    P = procs[name]
    assert (P.n_diagrams, P.n_colour, P.n_hel) == COUNTS[name]


def _golden_rows():
    rows = {}
    with open(os.path.join(HERE, "golden", "colour_matrices.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x) for x in line.split()]
            rows[v[0]] = (v[1], sorted(v[2:]))
    return rows


@pytest.mark.parametrize("name,k", [("gg_tt", 2), ("gg_ttg", 3), ("gg_ttgg", 4), ("gg_ttggg", 5)])
def test_colour_matrix(procs, name, k):
    C, den, basis = procs[name].colour_matrix()
    n = math.factorial(k)
    assert C.shape == (n, n) and basis.shape == (n, k)
    assert np.array_equal(C, C.T)
    # diagonal N C_F^k
    np.testing.assert_allclose(np.diag(C) / den, 3 * (4 / 3) ** k, rtol=1e-15)
    np.linalg.cholesky(C.astype(float))  # positive definite
    golden = _golden_rows()
    if k in golden:
        gden, grow = golden[k]
        assert den == gden
        for r in range(n):
            assert sorted(C[r].tolist()) == grow


def test_colour_matrix_recursion(procs):
    """Orderings that share their first (or last) gluon: summing that gluon's
    colour gives C_F times the entry of the k-1 gluon matrix."""
    for name, sub in (("gg_ttggg", "gg_ttgg"), ("gg_ttgg", "gg_ttg")):
        C, den, basis = procs[name].colour_matrix()
        Cs, dens, bs = procs[sub].colour_matrix()
        legs_sub = sorted(bs[0].tolist())
        index = {tuple(b): i for i, b in enumerate(bs.tolist())}
        checked = 0
        for a in range(len(basis)):
            for b in range(len(basis)):
                sa, sb = list(basis[a]), list(basis[b])
                for pos in (0, -1):
                    if sa[pos] != sb[pos]:
                        continue
                    g = sa[pos]
                    ra = [x for x in sa if x != g]
                    rb = [x for x in sb if x != g]
                    # relabel the remaining gluon legs onto the smaller process
                    rest = sorted(ra)
                    mp = dict(zip(rest, legs_sub))
                    ia = index[tuple(mp[x] for x in ra)]
                    ib = index[tuple(mp[x] for x in rb)]
                    assert C[a, b] * dens * 3 == Cs[ia, ib] * den * 4
                    checked += 1
        assert checked > len(basis)


@pytest.mark.parametrize("name,n", [("gg_tt", 8), ("gg_ttg", 8), ("gg_ttgg", 1)])
def test_brute_force_colour_sum(procs, oracle_mod, name, n):
    mom, _ = events(oracle_mod, name, n)
    P = procs[name]
    np.testing.assert_allclose(P.me(mom, colour_mode=1), P.me(mom), rtol=1e-12)


GAUGE_CASES = [("gg_ttg", 3, None), ("gg_ttgg", 2, None), ("gg_ttggg", 1, [0, 6])]


@pytest.mark.parametrize("name,n,legs", GAUGE_CASES)
def test_gauge_invariance(procs, oracle_mod, name, n, legs):
    mom, _ = events(oracle_mod, name, n)
    P = procs[name]
    gl = [i for i, x in enumerate(P.pdg) if x == 21] if legs is None else legs
    for p in mom:
        for leg in gl:
            rep, ref = P.gauge(p, leg)
            assert rep <= 1e-11 * p[leg][0] * ref


def boost(mom, beta_vec):
    b2 = beta_vec @ beta_vec
    g = 1 / math.sqrt(1 - b2)
    out = np.empty_like(mom)
    bp = mom[..., 1:] @ beta_vec
    out[..., 0] = g * (mom[..., 0] + bp)
    out[..., 1:] = mom[..., 1:] + ((g - 1) * bp / b2 + g * mom[..., 0])[..., None] * beta_vec
    return out


@pytest.mark.parametrize("name,n", [("gg_tt", 20), ("gg_ttg", 10), ("gg_ttgg", 2), ("gg_ttggg", 1),
                                    ("ee_mumu", 20)])
def test_lorentz_invariance(procs, oracle_mod, name, n):
    mom, _ = events(oracle_mod, name, n)
    rng = np.random.default_rng(3)
    d = rng.normal(size=3)
    bvec = 0.9 * d / np.linalg.norm(d)
    P = procs[name]
    np.testing.assert_allclose(P.me(boost(mom, bvec)), P.me(mom), rtol=1e-12)


@pytest.mark.parametrize("name,n", [("gg_tt", 10), ("gg_ttg", 10), ("gg_ttgg", 2), ("gg_ttggg", 1)])
def test_bose_symmetry(procs, oracle_mod, name, n):
    mom, _ = events(oracle_mod, name, n)
    P = procs[name]
    ref = P.me(mom)
    swapped = mom.copy()
    swapped[:, [0, 1]] = mom[:, [1, 0]]
    np.testing.assert_allclose(P.me(swapped), ref, rtol=1e-12)
    fin = list(range(4, P.n_ext))
    if len(fin) > 1:
        for perm in list(permutations(fin))[1:3]:
            pm = mom.copy()
            pm[:, fin] = mom[:, list(perm)]
            np.testing.assert_allclose(P.me(pm), ref, rtol=1e-12)


@pytest.mark.parametrize("name,n", [("gg_tt", 10), ("gg_ttg", 5), ("gg_ttgg", 2)])
def test_long_double_agrees(procs, oracle_mod, name, n):
    mom, _ = events(oracle_mod, name, n)
    P = procs[name]
    np.testing.assert_allclose(P.me(mom, precision=1), P.me(mom), rtol=1e-12)


@pytest.mark.parametrize("name,power", [("gg_tt", 2), ("gg_ttg", 3), ("gg_ttgg", 4)])
def test_coupling_power(oracle_mod, name, power):
    mom, _ = events(oracle_mod, name, 3)
    a = oracle_mod.Process(oracle_mod.PROCESSES[name], alpha_s=0.118).me(mom)
    b = oracle_mod.Process(oracle_mod.PROCESSES[name], alpha_s=0.236).me(mom)
    np.testing.assert_allclose(b / a, 2.0 ** power, rtol=1e-13)


def test_unsupported_process(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.Process([21, 21, 5, -5])
    with pytest.raises(ValueError):
        oracle_mod.Process([21, 21, 6, -6], wt=1.5)


# --------------------------------------------------------------- soft-gluon limit
def _boost_to(p, beta_vec):
    b2 = beta_vec @ beta_vec
    g = 1.0 / math.sqrt(1.0 - b2)
    bp = beta_vec @ p[1:]
    out = np.empty(4)
    out[0] = g * (p[0] + bp)
    out[1:] = p[1:] + ((g - 1) * bp / b2 + g * p[0]) * beta_vec
    return out


def _recoil(final, masses, P_target):
    """Final-state momenta (given in the frame where they sum to (M, 0)) mapped
    onto total momentum P_target: three-momenta rescaled by a common factor so
    that the energies sum to the new invariant mass, then boosted."""
    M_new = math.sqrt(mdot(P_target, P_target))
    p2 = np.sum(final[:, 1:] ** 2, axis=1)
    lo, hi = 0.0, 1.0
    for _ in range(200):
        lam = 0.5 * (lo + hi)
        if np.sum(np.sqrt(masses ** 2 + lam * lam * p2)) > M_new:
            hi = lam
        else:
            lo = lam
    q = np.concatenate([np.sqrt(masses ** 2 + lam * lam * p2)[:, None], lam * final[:, 1:]], axis=1)
    return np.array([_boost_to(x, P_target[1:] / P_target[0]) for x in q])


@pytest.mark.parametrize("hard_name,soft_leg,delta,tol,n_hel", [
    ("gg_tt", 4, 1e-7, 1e-5, None),
    ("gg_ttg", 5, 1e-7, 1e-5, None),
    ("gg_ttgg", 6, 1e-6, 2e-3, 12),
    ("gg_ttgg", 4, 1e-6, 2e-3, 6),
])
def test_soft_gluon_limit(procs, oracle_mod, hard_name, soft_leg, delta, tol, n_hel):
    """Soft-gluon factorisation of the colour-ordered amplitudes: when the
    energy of a final-state gluon k goes to zero, the flow (T^a1 ... T^am)_ij
    whose ordering has k between neighbours a and b (the top quark before the
    first gluon, the antitop after the last) tends to -g_s (eps*.p_a/k.p_a -
    eps*.p_b/k.p_b) times the flow of the process without k, in the same order,
    for every helicity (eikonal quark and gluon vertices, whose i g_s times the
    propagator's i gives -g_s).  This ties each process with one more gluon,
    g g -> t t~ g g g included, to the one below it, and so down to the g g ->
    t t~ closed form; the deviation is O(k / sqrt(s))."""
    names = list(oracle_mod.PROCESSES)
    soft_name = names[names.index(hard_name) + 1]
    H, S = procs[hard_name], procs[soft_name]
    n = S.n_ext
    sqrt_s = 1500.0
    hard_ev, _ = events(oracle_mod, hard_name, 1, first=5)
    hard_ev = hard_ev[0]
    rng = np.random.default_rng(17)
    u = rng.normal(size=3)
    k = delta * sqrt_s * np.concatenate([[1.0], u / np.linalg.norm(u)])
    masses = np.array([MT, MT] + [0.0] * (H.n_ext - 4))
    final = _recoil(hard_ev[2:], masses, hard_ev[0] + hard_ev[1] - k)
    hard_legs = [leg for leg in range(n) if leg != soft_leg]  # hard leg i is soft-event leg hard_legs[i]
    mom = np.zeros((n, 4))
    mom[soft_leg] = k
    mom[hard_legs] = np.concatenate([hard_ev[:2], final])
    basis_s = [tuple(b) for b in S.colour_matrix()[2].tolist()]
    index_h = {tuple(b): i for i, b in enumerate(H.colour_matrix()[2].tolist())}
    gs = math.sqrt(4 * math.pi * 0.118)
    flows_h = [H.flows(hard_ev, h) for h in range(H.n_hel)]
    scale = max(np.max(np.abs(J)) for J in flows_h)
    hels = [h for h in range(H.n_hel) if np.max(np.abs(flows_h[h])) > 1e-8 * scale]
    if n_hel is not None:
        hels = list(rng.choice(hels, n_hel, replace=False))
    checked = 0
    for h in hels:
        for lam in (-1, 1):
            code = (1 << (n - 1 - soft_leg)) if lam > 0 else 0
            for i, leg in enumerate(hard_legs):
                if (h >> (H.n_ext - 1 - i)) & 1:
                    code |= 1 << (n - 1 - leg)
            J = S.flows(mom, code)
            eps = np.conj(oracle_mod.external("eps", k, 0.0, lam))
            for s, order in enumerate(basis_s):
                j = order.index(soft_leg)
                a = 2 if j == 0 else order[j - 1]
                b = 3 if j == len(order) - 1 else order[j + 1]
                eik = mdot(eps, mom[a]) / mdot(k, mom[a]) - mdot(eps, mom[b]) / mdot(k, mom[b])
                hard_order = tuple(hard_legs.index(x) for x in order if x != soft_leg)
                pred = -gs * eik * flows_h[h][index_h[hard_order]]
                assert abs(J[s] - pred) <= tol * abs(eik) * scale * gs, (h, lam, order, J[s], pred)
                checked += 1
    assert checked >= 2 * len(hels) * len(basis_s)


# ------------------------------------------------ condition number of |M|^2
def test_condition_ee_closed_form(procs, oracle_mod):
    """e+e- -> mu+mu-: per helicity one photon and one Z diagram, so
    kappa = sum_ij X_ij (|A_gamma| + |A_Z,ij|)^2 / sum_ij X_ij |A_ij|^2 with
    X = u^2 for equal and t^2 for opposite lepton helicities; the photon alone
    has kappa = 1."""
    mom = two_body(50, 500.0, 0.0)
    s = 500.0 ** 2
    cw2 = 1 - SW2
    gl, gr = -0.5 + SW2, SW2
    D = s - MZ ** 2 + 1j * MZ * WZ
    A = ee_amplitudes(s)
    za = lambda gi, gj: abs(gi * gj / (SW2 * cw2 * D))
    P0 = oracle_mod.Process(oracle_mod.PROCESSES["ee_mumu"], z_enabled=0)
    for p in mom:
        t = -2 * mdot(p[0], p[2])
        u = -2 * mdot(p[0], p[3])
        num = (u ** 2 * ((1 / s + za(gl, gl)) ** 2 + (1 / s + za(gr, gr)) ** 2)
               + t ** 2 * ((1 / s + za(gl, gr)) ** 2 + (1 / s + za(gr, gl)) ** 2))
        den = (u ** 2 * (abs(A["LL"]) ** 2 + abs(A["RR"]) ** 2) + t ** 2 * (abs(A["LR"]) ** 2 + abs(A["RL"]) ** 2))
        assert procs["ee_mumu"].condition(p) == pytest.approx(num / den, rel=1e-13)
        assert P0.condition(p) == pytest.approx(1.0, rel=1e-15)


@pytest.mark.parametrize("name,n", [("gg_tt", 50), ("gg_ttg", 20), ("gg_ttgg", 4)])
def test_condition_invariances(procs, oracle_mod, name, n):
    """kappa >= 1 (triangle inequality); independent of alpha_s (every
    diagram carries the same power of g_s); unchanged when two final-state
    gluons are exchanged (the amplitudes are permuted)."""
    mom, _ = events(oracle_mod, name, n)
    P = procs[name]
    P2 = oracle_mod.Process(oracle_mod.PROCESSES[name], alpha_s=0.2)
    for p in mom:
        k = P.condition(p)
        assert k >= 1.0 - 1e-15
        assert P2.condition(p) == pytest.approx(k, rel=1e-13)
        if P.n_ext >= 6:
            q = p.copy()
            q[[4, 5]] = p[[5, 4]]
            assert P.condition(q) == pytest.approx(k, rel=1e-12)


def test_condition_bounds_fp64_rounding(procs, oracle_mod):
    """The bound the GPU parity tests use for ill-conditioned events holds
    for the oracle's own FP64 evaluation: |double / long double - 1| is
    within 512 u kappa on the worst-rounded events of a sample."""
    P = procs["gg_ttgg"]
    mom, _ = events(oracle_mod, "gg_ttgg", 1500)
    d = P.me(mom, nthreads=8)
    ld = P.me(mom, precision=1, nthreads=8)
    rel = np.abs(d / ld - 1.0)
    u = 2.0 ** -53
    idx = np.argsort(rel)[-20:]  # the worst-rounded events
    for i in idx:
        k = P.condition(mom[i])
        assert rel[i] <= 512 * u * k, (i, rel[i], k)
