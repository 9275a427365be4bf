"""Pins of the oracle's external states: Dirac equations, completeness
relations, normalisation, helicity eigenvalues and transversality, checked
with gamma matrices built independently here (chiral representation)."""
import numpy as np
import pytest

s0 = np.eye(2, dtype=complex)
sx = np.array([[0, 1], [1, 0]], dtype=complex)
sy = np.array([[0, -1j], [1j, 0]], dtype=complex)
sz = np.array([[1, 0], [0, -1]], dtype=complex)
Z2 = np.zeros((2, 2), dtype=complex)
G = [np.block([[Z2, s0], [s0, Z2]])] + [np.block([[Z2, s], [-s, Z2]]) for s in (sx, sy, sz)]
METRIC = np.diag([1.0, -1.0, -1.0, -1.0])


def pslash(p):
    return G[0] * p[0] - G[1] * p[1] - G[2] * p[2] - G[3] * p[3]


def test_clifford_algebra():
    for m in range(4):
        for n in range(4):
            anti = G[m] @ G[n] + G[n] @ G[m]
            np.testing.assert_allclose(anti, 2 * METRIC[m, n] * np.eye(4), atol=1e-15)


def _momenta(mass, rng):
    out = []
    for _ in range(12):
        v = rng.normal(size=3) * 300
        out.append(np.array([np.sqrt(v @ v + mass * mass), *v]))
    pabs = 400.0  # along the axes, including -z
    for d in ([0, 0, 1], [0, 0, -1], [1, 0, 0], [0, 1, 0]):
        v = pabs * np.array(d, dtype=float)
        out.append(np.array([np.sqrt(v @ v + mass * mass), *v]))
    return out


@pytest.mark.parametrize("mass", [0.0, 173.0])
def test_dirac_equations_and_completeness(oracle_mod, mass):
    rng = np.random.default_rng(1)
    for p in _momenta(mass, rng):
        ps = pslash(p)
        sum_u = np.zeros((4, 4), dtype=complex)
        sum_v = np.zeros((4, 4), dtype=complex)
        scale = p[0]
        for lam in (-1, 1):
            u = oracle_mod.external("u", p, mass, lam)
            v = oracle_mod.external("v", p, mass, lam)
            ub = oracle_mod.external("ubar", p, mass, lam)
            vb = oracle_mod.external("vbar", p, mass, lam)
            np.testing.assert_allclose((ps - mass * np.eye(4)) @ u, 0, atol=1e-13 * scale ** 1.5)
            np.testing.assert_allclose((ps + mass * np.eye(4)) @ v, 0, atol=1e-13 * scale ** 1.5)
            np.testing.assert_allclose(ub @ (ps - mass * np.eye(4)), 0, atol=1e-13 * scale ** 1.5)
            np.testing.assert_allclose(vb @ (ps + mass * np.eye(4)), 0, atol=1e-13 * scale ** 1.5)
            np.testing.assert_allclose(ub, u.conj() @ G[0], atol=1e-15 * scale)
            np.testing.assert_allclose(ub @ u, 2 * mass, atol=1e-12 * scale)
            np.testing.assert_allclose(vb @ v, -2 * mass, atol=1e-12 * scale)
            # helicity: (Sigma . phat) u = lam u, antiparticle v: (Sigma . phat) v = -lam v
            ph = p[1:] / np.linalg.norm(p[1:])
            sig = ph[0] * sx + ph[1] * sy + ph[2] * sz
            Sig = np.block([[sig, Z2], [Z2, sig]])
            np.testing.assert_allclose(Sig @ u, lam * u, atol=1e-13 * scale ** 0.5)
            np.testing.assert_allclose(Sig @ v, -lam * v, atol=1e-13 * scale ** 0.5)
            sum_u += np.outer(u, ub)
            sum_v += np.outer(v, vb)
        np.testing.assert_allclose(sum_u, ps + mass * np.eye(4), atol=1e-12 * scale)
        np.testing.assert_allclose(sum_v, ps - mass * np.eye(4), atol=1e-12 * scale)


def test_polarisation_vectors(oracle_mod):
    rng = np.random.default_rng(2)
    for p in _momenta(0.0, rng):
        k = p
        eps = {lam: oracle_mod.external("eps", k, 0.0, lam) for lam in (-1, 1)}
        khat = k[1:] / np.linalg.norm(k[1:])
        proj = np.zeros((3, 3), dtype=complex)
        for lam, e in eps.items():
            md = lambda a, b: a[0] * b[0] - a[1:] @ b[1:]
            assert abs(md(e, k)) < 1e-12 * k[0]
            np.testing.assert_allclose(md(e, e.conj()), -1.0, atol=1e-14)
            assert abs(e[0]) == 0.0
            # helicity: (S . khat) eps = lam eps with (S_k)_ij = -i eps_kij
            Sk = np.zeros((3, 3), dtype=complex)
            lc = np.zeros((3, 3, 3))
            lc[0, 1, 2] = lc[1, 2, 0] = lc[2, 0, 1] = 1
            lc[0, 2, 1] = lc[2, 1, 0] = lc[1, 0, 2] = -1
            for a in range(3):
                Sk += khat[a] * (-1j) * lc[a]
            np.testing.assert_allclose(Sk @ e[1:], lam * e[1:], atol=1e-14)
            proj += np.outer(e[1:], e[1:].conj())
        np.testing.assert_allclose(proj, np.eye(3) - np.outer(khat, khat), atol=1e-14)
        md = lambda a, b: a[0] * b[0] - a[1:] @ b[1:]
        assert abs(md(eps[1], eps[-1].conj())) < 1e-14
