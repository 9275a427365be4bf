"""GPU parity of the event-level steps (through the C ABI) against the oracle:
cross-section weights and their sums, hit-or-miss unweighting, and the
per-event choice of a helicity and a leading colour flow.

Inputs are seeded synthetic arrays or the oracle's own RAMBO events copied to
the device; nothing the GPU computes is handed to the oracle.

Tolerances:
  - weights w = (wgt * me) * k: the same two roundings on both sides, so
    bitwise equal;
  - sum w and sum w^2 (positive terms): the GPU's fixed-order tree (at most 16
    sequential terms per lane, then a depth-18 tree) is within 34 u of the
    exact sum, the oracle's long-double sum within n 2^-64, so both within
    1e-13 relative of each other; max w exactly;
  - unweighting: bitwise equal index lists;
  - helicity / colour choice in FP64: equal wherever the oracle's threshold is
    more than 1e-9 (relative to the total) away from a running-sum boundary:
    the GPU's per-helicity values agree with the oracle's to 1e-12, so only
    such near-ties can flip.  Reduced precision: equal beyond a 1e-4 margin.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SEED = 230318244
CASES = {  # name -> (events, sqrt(s))
    "ee_mumu": (4096, 500.0),
    "gg_tt": (4096, 1500.0),
    "gg_ttg": (1024, 1500.0),
    "gg_ttgg": (192, 1500.0),
    "gg_ttggg": (40, 1500.0),
}


def _torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def M():
    _torch()
    import paper_2303_18244_amd as M

    return M


def _masses(pdg):
    return [173.0 if abs(x) == 6 else 0.0 for x in pdg[2:]]


def _dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _synthetic(n, seed):
    """Phase-space weights and |M|^2 spanning several decades, as in flat
    RAMBO samples of multi-gluon processes."""
    rng = np.random.default_rng(seed)
    wgt = np.exp(rng.normal(-12.0, 0.5, n))
    me = np.exp(rng.normal(-20.0, 3.0, n))
    return wgt, me


@pytest.mark.parametrize("n", [0, 1, 4095, 4096 * 16 * 3 + 77, 524288, 3_000_001])
def test_event_weights_match_oracle(M, oracle_mod, n):
    torch = _torch()
    wgt, me = _synthetic(n, 11 + n % 97)
    sqrt_s = 1500.0
    w_o, st_o = oracle_mod.event_weights(wgt, me, sqrt_s)
    w, st = M.event_weights(sqrt_s, _dev(wgt), _dev(me), nevt=n)
    st = st.cpu().numpy()
    if n == 0:
        assert np.all(st == 0.0)
        return
    assert np.array_equal(w.cpu().numpy(), w_o)
    assert abs(st[0] / st_o[0] - 1.0) <= 1e-13, (st, st_o)
    assert abs(st[1] / st_o[1] - 1.0) <= 1e-13, (st, st_o)
    assert st[2] == st_o[2]
    # deterministic: the same inputs give the same bits
    _, st2 = M.event_weights(sqrt_s, _dev(wgt), _dev(me), nevt=n, want_weights=False)
    assert np.array_equal(st2.cpu().numpy(), st)


def test_cross_section_chain(M, oracle_mod):
    """g g -> t t~ on the oracle's events: GPU |M|^2 and weights against the
    oracle's, and the Monte Carlo estimate of sigma."""
    torch = _torch()
    name, n, sqrt_s = "gg_tt", 65536, 1500.0
    host, wgt = oracle_mod.rambo(_masses(oracle_mod.PROCESSES[name]), sqrt_s, SEED, 0, n)
    O = oracle_mod.Process(oracle_mod.PROCESSES[name])
    _, st_o = oracle_mod.event_weights(wgt, O.me(host, nthreads=16), sqrt_s)
    P = M.Process(M.PROCESSES[name])
    me = P.matrix_element(_dev(host.transpose(1, 2, 0)))
    _, st = M.event_weights(sqrt_s, _dev(wgt), me)
    st = st.cpu().numpy()
    np.testing.assert_allclose(st, st_o, rtol=1e-12)


@pytest.mark.parametrize("n", [0, 1, 2047, 2048, 2049, 2048 * 7 + 5, 524288, 4_194_307])
def test_unweight_matches_oracle(M, oracle_mod, n):
    torch = _torch()
    wgt, me = _synthetic(n, 5 + n % 89)
    w = wgt * me
    r = np.random.default_rng(n).random(n)
    w_ref = float(w.max()) if n else 1.0
    ref = oracle_mod.unweight(w, r, w_ref)
    idx = M.unweight(_dev(w), _dev(r), _dev(np.array([w_ref])), nevt=n)
    assert np.array_equal(idx.cpu().numpy(), ref)


def test_unweight_edge_cases(M, oracle_mod):
    torch = _torch()
    n = 5000
    rng = np.random.default_rng(2)
    # exact ties: r * w_ref == w (dyadic values) are dropped on both sides
    r = rng.integers(1, 8, n) / 8.0
    w = rng.integers(0, 9, n).astype(np.float64)
    ref = oracle_mod.unweight(w, r, 8.0)
    got = M.unweight(_dev(w), _dev(r), _dev(np.array([8.0]))).cpu().numpy()
    assert np.array_equal(got, ref)
    assert len(ref) < n
    # every weight at the reference: all kept; all zero: none
    ones = np.full(n, 3.0)
    assert M.unweight(_dev(ones), _dev(r), _dev(np.array([3.0]))).numel() == n
    assert M.unweight(_dev(np.zeros(n)), _dev(r), _dev(np.array([3.0]))).numel() == 0
    # w_ref read on the device from the weight sums
    wgt, me = _synthetic(n, 3)
    w, st = M.event_weights(1500.0, _dev(wgt), _dev(me))
    w_o, st_o = oracle_mod.event_weights(wgt, me, 1500.0)
    got = M.unweight(w, _dev(r), st[2:]).cpu().numpy()
    assert np.array_equal(got, oracle_mod.unweight(w_o, r, st_o[2]))


def _compare_choices(got_hel, got_col, host, r_hel, r_col, O, margin_min):
    n_checked = 0
    for e in range(len(host)):
        h, c, margin = O.select(host[e], float(r_hel[e]), float(r_col[e]))
        if margin[0] > margin_min:
            assert got_hel[e] == h, (e, got_hel[e], h, margin)
            n_checked += 1
        if margin[1] > margin_min:
            assert got_col[e] == c, (e, got_col[e], c, margin)
    return n_checked


@pytest.mark.parametrize("name", list(CASES))
def test_select_fp64_matches_oracle(M, oracle_mod, name):
    torch = _torch()
    n, sqrt_s = CASES[name]
    P = M.Process(M.PROCESSES[name])
    O = oracle_mod.Process(oracle_mod.PROCESSES[name])
    if O.n_colour > 1:  # both sides order the flows the same way
        assert [list(b) for b in O.colour_matrix()[2].tolist()] == P.colour_matrix()[2]
    host, _ = oracle_mod.rambo(_masses(P.pdg), sqrt_s, SEED, 0, n)
    rng = np.random.default_rng(77)
    r_hel, r_col = rng.random(n), rng.random(n)
    mom = _dev(host.transpose(1, 2, 0))
    me, hel, col = P.select(mom, _dev(r_hel), _dev(r_col))
    me, hel, col = me.cpu().numpy(), hel.cpu().numpy(), col.cpu().numpy()
    # the |M|^2 it returns is that of mgme_matrix_element
    np.testing.assert_allclose(me, P.matrix_element(mom).cpu().numpy(), rtol=1e-14, atol=0)
    assert _compare_choices(hel, col, host, r_hel, r_col, O, 1e-9) >= n - 2
    good = set(P.good_helicities())
    assert set(hel.tolist()) <= good
    assert col.min() >= 0 and col.max() < O.n_colour


def test_denominator_table_same_bits(M, oracle_mod):
    """g g -> t t~ g g in FP64: the plain kernel and the selection kernel
    (which also writes every helicity's value and the flow weights) take the
    momentum sums and denominators from the same per-event rows and add the
    event's lane sums in the same order; the |M|^2 of both must agree bit for
    bit."""
    torch = _torch()
    n, sqrt_s = 1000, 1500.0
    P = M.Process(M.PROCESSES["gg_ttgg"])
    host, _ = oracle_mod.rambo(_masses(P.pdg), sqrt_s, SEED, 7, n)
    mom = _dev(host.transpose(1, 2, 0))
    r = _dev(np.random.default_rng(5).random(n))
    me_sel, _, _ = P.select(mom, r, r)
    assert torch.equal(me_sel, P.matrix_element(mom))


@pytest.mark.parametrize("name", ["gg_ttg", "gg_ttgg", "gg_ttggg"])
@pytest.mark.parametrize("prec", [1, 2, 3])
def test_select_reduced_precision(M, oracle_mod, name, prec):
    torch = _torch()
    n, sqrt_s = CASES[name]
    P = M.Process(M.PROCESSES[name])
    O = oracle_mod.Process(oracle_mod.PROCESSES[name])
    host, _ = oracle_mod.rambo(_masses(P.pdg), sqrt_s, SEED, 0, n)
    rng = np.random.default_rng(78)
    r_hel, r_col = rng.random(n), rng.random(n)
    mom = _dev(host.transpose(1, 2, 0))
    me, hel, col = P.select(mom, _dev(r_hel), _dev(r_col), precision=prec)
    # same arithmetic as mgme_matrix_element (a separate instantiation of the
    # same code for the fused processes)
    np.testing.assert_allclose(me.cpu().numpy(), P.matrix_element(mom, precision=prec).cpu().numpy(), rtol=1e-6)
    _compare_choices(hel.cpu().numpy(), col.cpu().numpy(), host, r_hel, r_col, O, 1e-4)


def test_select_across_sub_batches(M, oracle_mod):
    """g g -> t t~ g g g: a batch over five staging sub-batches; events on both
    sides of every boundary against the oracle (offsets of the random numbers
    and outputs)."""
    torch = _torch()
    name, sqrt_s = "gg_ttggg", 1500.0
    n = 65536 + 100  # four and a bit staging sub-batches of at most 16384 events
    P = M.Process(M.PROCESSES[name])
    O = oracle_mod.Process(oracle_mod.PROCESSES[name])
    host, _ = oracle_mod.rambo(_masses(P.pdg), sqrt_s, SEED, 0, n)
    rng = np.random.default_rng(79)
    r_hel, r_col = rng.random(n), rng.random(n)
    me, hel, col = P.select(_dev(host.transpose(1, 2, 0)), _dev(r_hel), _dev(r_col))
    hel, col = hel.cpu().numpy(), col.cpu().numpy()
    edges = [b + d for b in (16384, 32768, 49152, 65536) for d in (-1, 0)]
    idx = np.array([0, 1] + edges + [65537, n - 1] + list(np.random.default_rng(3).choice(n, 10, replace=False)))
    assert _compare_choices(hel[idx], col[idx], host[idx], r_hel[idx], r_col[idx], O, 1e-9) >= len(idx) - 1
