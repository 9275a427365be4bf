"""Pins of the oracle's random numbers and RAMBO phase space (CPU only).

Philox4x32-10 is pinned to the published known-answer vectors; RAMBO to
momentum conservation, mass shells, the closed-form massless weight, the exact
two-body phase-space volume and isotropy.
"""
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers(oracle_mod):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert oracle_mod.philox4x32_10(ctr, key) == out


def test_uniforms_open_interval_and_uniform(oracle_mod):
    u = np.array([oracle_mod.uniform_pair(7, e, b) for e in range(2000) for b in range(4)]).ravel()
    assert np.all(u > 0) and np.all(u < 1)
    hist, _ = np.histogram(u, bins=20, range=(0, 1))
    expected = u.size / 20
    chi2 = float(np.sum((hist - expected) ** 2 / expected))
    assert chi2 < 45.3  # 19 dof, p = 0.001


def _mdot(a, b):
    return a[..., 0] * b[..., 0] - a[..., 1] * b[..., 1] - a[..., 2] * b[..., 2] - a[..., 3] * b[..., 3]


@pytest.mark.parametrize("masses,sqrt_s", [([0.0, 0.0], 500.0), ([173.0, 173.0], 1500.0),
                                           ([173.0, 173.0, 0.0], 1500.0),
                                           ([173.0, 173.0, 0.0, 0.0], 1500.0),
                                           ([173.0, 173.0, 0.0, 0.0, 0.0], 1500.0)])
def test_rambo_conservation_and_shell(oracle_mod, masses, sqrt_s):
    mom, w = oracle_mod.rambo(masses, sqrt_s, 230318244, 0, 500)
    tot_out = mom[:, 2:, :].sum(axis=1)
    tot_in = mom[:, :2, :].sum(axis=1)
    assert np.max(np.abs(tot_out - tot_in)) < 1e-13 * sqrt_s * 10
    for i, m in enumerate(masses):
        p = mom[:, 2 + i, :]
        m2 = _mdot(p, p)
        assert np.max(np.abs(m2 - m * m)) < 1e-12 * sqrt_s ** 2
        assert np.all(p[:, 0] > 0)
    np.testing.assert_allclose(mom[:, 0], [[sqrt_s / 2, 0, 0, sqrt_s / 2]] * len(mom))
    np.testing.assert_allclose(mom[:, 1], [[sqrt_s / 2, 0, 0, -sqrt_s / 2]] * len(mom))
    assert np.all(w > 0)


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_rambo_massless_weight_closed_form(oracle_mod, n):
    sqrt_s = 1000.0
    s = sqrt_s ** 2
    _, w = oracle_mod.rambo([0.0] * n, sqrt_s, 11, 0, 20)
    expect = ((math.pi / 2) ** (n - 1) * s ** (n - 2) / (math.factorial(n - 1) * math.factorial(n - 2))
              * (2 * math.pi) ** (4 - 3 * n))
    np.testing.assert_allclose(w, expect, rtol=1e-13)


def test_rambo_two_body_massive_volume(oracle_mod):
    # Exact two-body phase space: beta / (8 pi), beta = sqrt(1 - 4 m^2 / s).
    m, sqrt_s = 173.0, 1500.0
    _, w = oracle_mod.rambo([m, m], sqrt_s, 3, 0, 50)
    beta = math.sqrt(1 - 4 * m * m / sqrt_s ** 2)
    np.testing.assert_allclose(w, beta / (8 * math.pi), rtol=1e-13)


def test_rambo_two_body_isotropic(oracle_mod):
    mom, _ = oracle_mod.rambo([173.0, 173.0], 1500.0, 5, 0, 20000)
    p = mom[:, 2, 1:]
    cost = p[:, 2] / np.linalg.norm(p, axis=1)
    hist, _ = np.histogram(cost, bins=20, range=(-1, 1))
    expected = len(cost) / 20
    chi2 = float(np.sum((hist - expected) ** 2 / expected))
    assert chi2 < 45.3


def test_rambo_event_counter_prefix(oracle_mod):
    a, wa = oracle_mod.rambo([173.0, 173.0, 0.0, 0.0], 1500.0, 230318244, 0, 40)
    b, wb = oracle_mod.rambo([173.0, 173.0, 0.0, 0.0], 1500.0, 230318244, 17, 10)
    np.testing.assert_array_equal(a[17:27], b)
    np.testing.assert_array_equal(wa[17:27], wb)


# --- Massive weights for n >= 3: the phase-space volume by nested two-body
# decays.  With the (2 pi)^(4-3n) convention the n-body volume obeys
#   Phi_n(s; m_1, rest) = int dM^2 / (2 pi) Phi_2(s; m_1, M) Phi_(n-1)(M^2; rest),
#   Phi_2(s; m_a, m_b) = lambda^(1/2)(s, m_a^2, m_b^2) / (8 pi s),
# over (sum of rest)^2 <= M^2 <= (sqrt(s) - m_1)^2.  This shares nothing with
# RAMBO's momenta, its conformal step or its massive rescaling, so the mean
# RAMBO weight (the Monte Carlo estimate of the same volume) pins the whole
# massive weight, including its n-dependence.

_GL_X, _GL_W = np.polynomial.legendre.leggauss(48)


def _phi2(s, ma, mb):
    lam = (s - (ma + mb) ** 2) * (s - (ma - mb) ** 2)
    return np.sqrt(np.maximum(lam, 0.0)) / (8.0 * math.pi * s)


def _phase_space_volume(s, masses):
    """Phi_n(s) by nested Gauss-Legendre quadrature.  The substitution
    M^2 = lo + (hi - lo) sin^2(theta) absorbs the square-root behaviour of the
    two-body factors at both ends, so the rule converges quickly."""
    s = np.asarray(s, dtype=np.float64)
    if len(masses) == 2:
        return _phi2(s, masses[0], masses[1])
    m1, rest = masses[0], list(masses[1:])
    lo = np.full(s.shape, float(sum(rest)) ** 2)
    hi = (np.sqrt(s) - m1) ** 2
    theta = (_GL_X + 1.0) * (math.pi / 4.0)   # [0, pi/2]
    wts = _GL_W * (math.pi / 4.0)
    span = (hi - lo)[..., None]
    m2 = lo[..., None] + span * np.sin(theta) ** 2
    jac = span * np.sin(2.0 * theta)
    f = _phi2(s[..., None], m1, np.sqrt(m2)) * _phase_space_volume(m2, rest) * jac / (2.0 * math.pi)
    return np.sum(f * wts, axis=-1)


@pytest.mark.parametrize("n", [3, 4, 5])
def test_nested_two_body_volume_massless_closed_form(n):
    """The quadrature itself against the closed-form massless volume."""
    s = 1500.0 ** 2
    expect = ((math.pi / 2) ** (n - 1) * s ** (n - 2) / (math.factorial(n - 1) * math.factorial(n - 2))
              * (2 * math.pi) ** (4 - 3 * n))
    got = float(_phase_space_volume(np.array(s), [0.0] * n))
    assert abs(got / expect - 1.0) < 1e-12, (got, expect)


def test_nested_two_body_volume_two_body_massive():
    m, sqrt_s = 173.0, 1500.0
    beta = math.sqrt(1 - 4 * m * m / sqrt_s ** 2)
    got = float(_phase_space_volume(np.array(sqrt_s ** 2), [m, m]))
    assert abs(got * 8 * math.pi / beta - 1.0) < 1e-14


@pytest.mark.parametrize("masses", [[173.0, 173.0, 0.0], [173.0, 173.0, 0.0, 0.0],
                                    [173.0, 173.0, 0.0, 0.0, 0.0]])
def test_rambo_massive_weight_matches_nested_volume(oracle_mod, masses):
    """g g -> t t~ + 1..3 g at 1500 GeV: the mean RAMBO weight over 1e5 events
    equals the nested two-body volume within 4 Monte Carlo standard errors.
    The same test rejects a massive weight with the rescaling factor to the
    power n-1 instead of 2n-3 (the two agree at n = 2): xi is recovered from
    the event as sum |k_i| / sqrt(s), and the mean of w * xi^(2-n) must lie far
    outside the error band."""
    sqrt_s, n = 1500.0, len(masses)
    # the gluons split off first: Phi_n(s; 0, [rest]) down to Phi_2(t, t~)
    order = sorted(masses)
    vol = float(_phase_space_volume(np.array(sqrt_s ** 2), order))
    mom, w = oracle_mod.rambo(masses, sqrt_s, 230318244, 0, 100000)
    mean, err = w.mean(), w.std(ddof=1) / math.sqrt(len(w))
    assert abs(mean - vol) < 4.0 * err, (mean, vol, err, (mean - vol) / err)
    assert err < 0.01 * vol
    kmod = np.linalg.norm(mom[:, 2:, 1:], axis=2).sum(axis=1)
    xi = kmod / sqrt_s
    assert np.all((xi > 0) & (xi < 1))
    wrong = w * xi ** (2 - n)
    assert abs(wrong.mean() - vol) > 10.0 * err
