"""GPU parity of the HIP path (through the C ABI) against the oracle.

Tolerances: FP64 |M|^2 per event within 1e-12 relative (an event outside it
is re-evaluated by the long-double oracle and must be within 1e-12 of that,
or within 512 u kappa with kappa the event's condition number: fp64_check.py);
FP32 diagrams: the batch mean and the per-event median within 1e-5
relative (the paper's cross-section criterion for reduced precision),
per-event p99 and maximum printed.  RAMBO momenta within 1e-12 sqrt(s):
the conformal boost amplifies rounding for nearly collinear pairs, so host
and device libm results agree only to that level.
"""
import math
import os

import numpy as np
import pytest
from fp64_check import check

pytestmark = pytest.mark.gpu

SEED = 230318244
NTHREADS = max(1, min(16, os.cpu_count() or 1))

# name -> (events checked against the oracle, full configuration size, sqrt(s))
CASES = {
    "ee_mumu": (16384, 16384, 500.0),
    "gg_tt": (8192, 524288, 1500.0),
    "gg_ttg": (2048, 65536, 1500.0),
    "gg_ttgg": (389, 524288, 1500.0),
    "gg_ttggg": (67, 65536, 1500.0),
}


def _torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def lib_procs():
    _torch()
    import paper_2303_18244_amd as M

    out = {}
    for name, pdg in M.PROCESSES.items():
        try:
            out[name] = M.Process(pdg)
        except M.MgmeError as e:
            if e.code == M.MGME_EUNSUPPORTED:
                continue
            raise
    return out


@pytest.fixture(scope="module")
def oracle_procs(oracle_mod):
    return {name: oracle_mod.Process(pdg) for name, pdg in oracle_mod.PROCESSES.items()}


def _proc(lib_procs, name):
    if name not in lib_procs:
        pytest.skip(f"{name} not compiled into libmgme.so")
    return lib_procs[name]


def _host(mom, nevt):
    """[n_ext, 4, ld] device tensor -> [nevt, n_ext, 4] host array."""
    return mom[:, :, :nevt].cpu().numpy().transpose(2, 0, 1).copy()


_EVENTS = {}


def _events(oracle_mod, name, n, seed=SEED):
    """The oracle's RAMBO events (seed, events 0..n-1) as the common input of
    both sides: ([n, n_ext, 4] host array, [n_ext, 4, n] device tensor).
    Nothing computed by the GPU path is ever handed to the oracle."""
    torch = _torch()
    key = (name, n, seed)
    if key not in _EVENTS:
        pdg = oracle_mod.PROCESSES[name]
        host, _ = oracle_mod.rambo(_masses(pdg), CASES[name][2], seed, 0, n)
        dev = torch.from_numpy(np.ascontiguousarray(host.transpose(1, 2, 0))).to("cuda")
        _EVENTS.clear()  # keep at most one batch resident
        _EVENTS[key] = (host, dev)
    return _EVENTS[key]


def _masses(pdg):
    return [173.0 if abs(x) == 6 else 0.0 for x in pdg[2:]]


def _check_fp64(gpu, mom_host, oproc):
    """The rule of fp64_check.py: per event within 1e-12 of the oracle's
    double value, or, for an ill-conditioned event, within 512 u kappa of the
    long-double oracle (both evaluated for the outliers only)."""
    ref = oproc.me(mom_host, nthreads=NTHREADS)
    rel, _, _ = check(gpu, ref, lambda idx: oproc.me(mom_host[idx], precision=1, nthreads=NTHREADS),
                      lambda idx: np.array([oproc.condition(mom_host[i]) for i in idx]))
    return rel


@pytest.mark.parametrize("name", list(CASES))
def test_rambo_matches_oracle(lib_procs, oracle_mod, name):
    torch = _torch()
    P = _proc(lib_procs, name)
    n, _, sq = CASES[name]
    n = min(n, 4096)
    mom, wgt = P.rambo(sq, SEED, 0, n)
    torch.cuda.synchronize()
    om, ow = oracle_mod.rambo(_masses(P.pdg), sq, SEED, 0, n)
    dp = np.abs(_host(mom, n) - om).max()
    assert dp <= 1e-12 * sq, dp
    np.testing.assert_allclose(wgt.cpu().numpy()[:n], ow, rtol=1e-11)


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_matches_oracle(lib_procs, oracle_procs, oracle_mod, name):
    torch = _torch()
    P = _proc(lib_procs, name)
    n, _, sq = CASES[name]
    host, mom = _events(oracle_mod, name, n)
    me = P.matrix_element(mom).cpu().numpy()
    rel = _check_fp64(me, host, oracle_procs[name])
    print(f"{name} FP64 vs oracle on {n} events: max rel {rel.max():.2e}, median {np.median(rel):.2e}")


@pytest.mark.parametrize("name", list(CASES))
def test_fp32_accuracy(lib_procs, oracle_procs, oracle_mod, name):
    torch = _torch()
    P = _proc(lib_procs, name)
    n, _, sq = CASES[name]
    host, mom = _events(oracle_mod, name, n)
    me = P.matrix_element(mom, precision=1).cpu().numpy()
    ref = oracle_procs[name].me(host, nthreads=NTHREADS)
    rel = np.abs(me / ref - 1.0)
    mean_rel = abs(me.mean() / ref.mean() - 1.0)
    print(f"{name} FP32 vs oracle on {n} events: batch-mean {mean_rel:.2e}, median {np.median(rel):.2e}, "
          f"p99 {np.quantile(rel, 0.99):.2e}, max {rel.max():.2e}")
    assert mean_rel <= 1e-5
    assert np.median(rel) <= 1e-5


@pytest.mark.parametrize("name", list(CASES))
def test_mixed_accuracy(lib_procs, oracle_procs, oracle_mod, name):
    """Single-precision diagrams with the 16-bit matrix-core colour sum."""
    torch = _torch()
    import paper_2303_18244_amd as M

    P = _proc(lib_procs, name)
    n, _, sq = CASES[name]
    host, mom = _events(oracle_mod, name, n)
    me = P.matrix_element(mom, precision=M.MIXED).cpu().numpy()
    ref = oracle_procs[name].me(host, nthreads=NTHREADS)
    rel = np.abs(me / ref - 1.0)
    mean_rel = abs(me.mean() / ref.mean() - 1.0)
    print(f"{name} mixed vs oracle on {n} events: batch-mean {mean_rel:.2e}, median {np.median(rel):.2e}, "
          f"p99 {np.quantile(rel, 0.99):.2e}, max {rel.max():.2e}")
    assert mean_rel <= 1e-5
    assert np.median(rel) <= 1e-5


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_diagrams_fp32_colour_accuracy(lib_procs, oracle_procs, oracle_mod, name):
    """The paper's mixed mode: double-precision diagrams, single-precision
    colour algebra (section 3).  Same criterion as the other reduced-precision
    modes; the error comes from the colour quadratic form alone, so it is also
    bounded per event by the float rounding of that form."""
    torch = _torch()
    import paper_2303_18244_amd as M

    P = _proc(lib_procs, name)
    n, _, sq = CASES[name]
    host, mom = _events(oracle_mod, name, n)
    me = P.matrix_element(mom, precision=M.FP64_FP32COLOUR).cpu().numpy()
    ref = oracle_procs[name].me(host, nthreads=NTHREADS)
    rel = np.abs(me / ref - 1.0)
    mean_rel = abs(me.mean() / ref.mean() - 1.0)
    print(f"{name} FP64 diagrams + FP32 colour vs oracle on {n} events: batch-mean {mean_rel:.2e}, "
          f"median {np.median(rel):.2e}, p99 {np.quantile(rel, 0.99):.2e}, max {rel.max():.2e}")
    assert mean_rel <= 1e-5
    assert np.median(rel) <= 1e-5


@pytest.mark.parametrize("name", list(CASES))
def test_full_size_sampled(lib_procs, oracle_procs, oracle_mod, name):
    """The configuration's full batch in one launch (the benchmark's launch):
    sampled events against the oracle, and the leading events bitwise equal
    to a small batch (no dependence on the batch size or on the launch grid).
    RAMBO at the full size on sampled events against the oracle's."""
    torch = _torch()
    P = _proc(lib_procs, name)
    n_small, n_full, sq = CASES[name]
    host, mom = _events(oracle_mod, name, n_full)
    me = P.matrix_element(mom).cpu().numpy()
    rng = np.random.default_rng(5)
    k = 24 if name == "gg_ttggg" else 96
    idx = np.unique(np.concatenate([rng.choice(n_full, k, replace=False), [0, n_full - 1]]))
    _check_fp64(me[idx], host[idx], oracle_procs[name])
    me_small = P.matrix_element(mom[:, :, :333].contiguous()).cpu().numpy()
    assert np.array_equal(me_small, me[:333])
    assert np.all(np.isfinite(me)) and np.all(me > 0)
    gmom, gw = P.rambo(sq, SEED, 0, n_full)
    gsel = gmom[:, :, idx].cpu().numpy().transpose(2, 0, 1)
    for j, e in enumerate(idx):
        om, ow = oracle_mod.rambo(_masses(P.pdg), sq, SEED, int(e), 1)
        assert np.abs(gsel[j] - om[0]).max() <= 1e-12 * sq
        assert abs(gw[int(e)].item() / ow[0] - 1.0) <= 1e-11


@pytest.mark.parametrize("name", list(CASES))
def test_good_helicities_match_oracle(lib_procs, oracle_procs, oracle_mod, name):
    """Good helicities = helicities with a non-zero FP64 contribution on at
    least one of 64 calibration events (seed 1); per-helicity values agree."""
    torch = _torch()
    P = _proc(lib_procs, name)
    host, mom = _events(oracle_mod, name, 64, seed=1)
    O = oracle_procs[name]
    step = 1 if P.n_ext < 7 else 16
    per = np.array([O.me_hel(host[e]) for e in range(0, 64, step)])
    expected = [h for h in range(1 << P.n_ext) if np.any(per[:, h] != 0.0)]
    if P.n_ext < 7:
        assert P.good_helicities() == expected
    if name == "ee_mumu":
        assert len(expected) == 4
    gpu = P.matrix_element_per_helicity(mom).cpu().numpy()  # [n_hel, 64]
    for j, e in enumerate(range(0, 64, step)):
        # helicities that vanish analytically come out as rounding noise far
        # below the others; compare them on the scale of the event's total
        np.testing.assert_allclose(gpu[:, e], per[j], rtol=1e-11, atol=1e-13 * per[j].max())
    # the masked sum equals the sum over every helicity
    me = P.matrix_element(mom).cpu().numpy()
    np.testing.assert_allclose(me, gpu.sum(axis=0), rtol=1e-13)


@pytest.mark.parametrize("name", ["gg_ttg", "gg_ttgg"])
def test_invariances_on_gpu(lib_procs, name):
    """Lorentz boost (beta = 0.9) and Bose symmetry of final gluons."""
    torch = _torch()
    P = _proc(lib_procs, name)
    n, _, sq = CASES[name]
    mom, _ = P.rambo(sq, SEED, 0, n)
    ref = P.matrix_element(mom).cpu().numpy()
    h = mom.cpu().numpy()  # [n_ext, 4, n]
    beta = np.array([0.3, -0.5, 0.6])
    beta *= 0.9 / np.linalg.norm(beta)
    g = 1 / math.sqrt(1 - beta @ beta)
    e, p = h[:, 0, :], h[:, 1:, :]
    bp = np.einsum("k,ikn->in", beta, p)
    hb = np.empty_like(h)
    hb[:, 0, :] = g * (e + bp)
    hb[:, 1:, :] = p + ((g - 1) * bp / (beta @ beta) + g * e)[:, None, :] * beta[None, :, None]
    boosted = P.matrix_element(torch.from_numpy(hb).cuda()).cpu().numpy()
    np.testing.assert_allclose(boosted, ref, rtol=1e-11)
    if P.n_ext >= 6:
        hs = h.copy()
        hs[[4, 5]] = h[[5, 4]]
        np.testing.assert_allclose(P.matrix_element(torch.from_numpy(hs).cuda()).cpu().numpy(), ref, rtol=1e-12)
    hs = h.copy()
    hs[[0, 1]] = h[[1, 0]]
    np.testing.assert_allclose(P.matrix_element(torch.from_numpy(hs).cuda()).cpu().numpy(), ref, rtol=1e-12)


def test_determinism_and_ragged_edges(lib_procs):
    torch = _torch()
    import paper_2303_18244_amd as M

    P = _proc(lib_procs, "gg_ttgg")
    mom, _ = P.rambo(1500.0, SEED, 0, 1000)
    a = P.matrix_element(mom).cpu().numpy()
    b = P.matrix_element(mom).cpu().numpy()
    assert np.array_equal(a, b)
    # one event, and a padded leading dimension
    one = P.matrix_element(mom[:, :, :1].contiguous()).cpu().numpy()
    assert one[0] == a[0]
    padded = torch.zeros((P.n_ext, 4, 1024), dtype=torch.float64, device="cuda")
    padded[:, :, :1000] = mom
    out = torch.full((1024,), -7.0, dtype=torch.float64, device="cuda")
    P.matrix_element(padded, nevt=1000, out=out)
    o = out.cpu().numpy()
    assert np.array_equal(o[:1000], a) and np.all(o[1000:] == -7.0)
    # empty batch is a no-op
    out0 = torch.full((4,), -3.0, dtype=torch.float64, device="cuda")
    P.matrix_element(padded, nevt=0, out=out0)
    assert np.all(out0.cpu().numpy() == -3.0)
    with pytest.raises(M.MgmeError) as ei:
        P.matrix_element(mom, precision=7)
    assert ei.value.code == M.MGME_EINVAL


@pytest.mark.parametrize("name", ["gg_ttgg", "gg_ttggg"])
@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_staging_edges(lib_procs, name, prec):
    """Ragged batch sizes and a padded leading dimension give the same
    per-event values as one small batch; for the staged process a batch of
    65836 events spans five sub-batches of the staging buffers (at most 16384
    events each), and the events on both sides of the last boundary equal a
    small batch's."""
    torch = _torch()
    P = _proc(lib_procs, name)
    n = 200
    mom, _ = P.rambo(1500.0, SEED, 0, n)
    a = P.matrix_element(mom, precision=prec).cpu().numpy()
    for m in (1, 63, 65, 131):
        b = P.matrix_element(mom[:, :, :m].contiguous(), precision=prec).cpu().numpy()
        np.testing.assert_array_equal(b, a[:m])
    if name == "gg_ttggg":
        big, _ = P.rambo(1500.0, SEED, 0, 65536 + 300)
        whole = P.matrix_element(big, precision=prec).cpu().numpy()
        np.testing.assert_array_equal(whole[:n], a)
        edge = P.matrix_element(big[:, :, 65400:].contiguous(), precision=prec).cpu().numpy()
        np.testing.assert_array_equal(whole[65400:], edge)
        assert np.all(np.isfinite(whole)) and np.all(whole > 0)
    padded = torch.zeros((P.n_ext, 4, 256), dtype=torch.float64, device="cuda")
    padded[:, :, :n] = mom
    out = torch.full((256,), -5.0, dtype=torch.float64, device="cuda")
    P.matrix_element(padded, nevt=n, precision=prec, out=out)
    o = out.cpu().numpy()
    np.testing.assert_array_equal(o[:n], a)
    assert np.all(o[n:] == -5.0)


def test_colour_matrix_export_matches_oracle(lib_procs, oracle_procs):
    _torch()
    for name in ("gg_tt", "gg_ttg", "gg_ttgg"):
        num, den, basis = _proc(lib_procs, name).colour_matrix()
        Co, oden, obasis = oracle_procs[name].colour_matrix()
        idx = {tuple(b): i for i, b in enumerate(obasis.tolist())}
        for i, bi in enumerate(basis):
            for j, bj in enumerate(basis):
                assert num[i][j] * oden == Co[idx[tuple(bi)], idx[tuple(bj)]] * den


def test_huge_batch_runs_in_parts(lib_procs):
    """A fused batch above 2^28 events (more than 2^31 lanes at eight lanes
    per event) runs as consecutive launches; events on both sides of the
    part boundary equal a small batch's, bit for bit.  g g -> t t~ with
    2^28 + 96 events: 34 GB of momenta."""
    torch = _torch()
    free, _ = torch.cuda.mem_get_info()
    if free < 48 << 30:
        pytest.skip("needs 48 GB of free device memory")
    P = _proc(lib_procs, "gg_tt")
    n = (1 << 28) + 96
    mom, _ = P.rambo(1500.0, SEED, 0, n)
    for prec in (0, 1):
        me = P.matrix_element(mom, precision=prec)
        lo = (1 << 28) - 64
        part = P.matrix_element(mom[:, :, lo:].contiguous(), precision=prec)
        assert torch.equal(me[lo:], part)
        assert bool(torch.isfinite(me).all()) and bool((me > 0).all())
        del me, part
    del mom
    torch.cuda.empty_cache()
