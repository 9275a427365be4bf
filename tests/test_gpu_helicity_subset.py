"""A helicity sum restricted to a subset (mgme_set_helicities) against the
oracle's per-helicity values.

The fused kernels give an event eight lanes (four for e+e- -> mu+mu-), lane
k taking the helicities k, k+8, ...; the subsets here are not multiples of
that, so in the last step some of an event's lanes have no helicity left and
every mode must drop their values.  The staged process takes one helicity
per wave and skips waves past the list.  Oracle inputs are its own RAMBO
events; FP64 sums agree within 1e-11 relative (sums of non-negative
per-helicity terms, each within the oracle tolerance of the full sum).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SEED = 230318244

# name -> (events, sqrt(s), subset as positions in the good-helicity list)
CASES = {
    "ee_mumu": (512, 500.0, [0, 1, 3]),
    "gg_tt": (256, 1500.0, [0, 3, 5, 6, 9]),
    "gg_ttg": (128, 1500.0, [1, 2, 4, 8, 16, 30, 31]),
    "gg_ttgg": (48, 1500.0, [0, 5, 9, 12, 17, 33, 40, 51, 60, 62, 63]),
    "gg_ttggg": (6, 1500.0, [3, 17, 64, 100, 127]),
}


def _masses(pdg):
    return [173.0 if abs(x) == 6 else 0.0 for x in pdg[2:]]


@pytest.mark.parametrize("name", list(CASES))
def test_restricted_helicity_sum(name, oracle_mod):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_18244_amd as M

    n, sqrt_s, pos = CASES[name]
    pdg = M.PROCESSES[name]
    P = M.Process(pdg)
    O = oracle_mod.Process(oracle_mod.PROCESSES[name])
    good = P.good_helicities()
    subset = [good[i] for i in pos]
    host, _ = oracle_mod.rambo(_masses(pdg), sqrt_s, SEED, 0, n)
    mom = torch.from_numpy(np.ascontiguousarray(host.transpose(1, 2, 0))).to("cuda")

    full = P.matrix_element(mom).clone()
    P.set_helicities(subset)
    assert P.good_helicities() == subset and P.info["n_good_hel"] == len(subset)

    me64 = P.matrix_element(mom)
    per_hel = np.array([O.me_hel(host[e]) for e in range(n)])  # [n, n_hel], oracle
    ref = per_hel[:, subset].sum(axis=1)
    np.testing.assert_allclose(me64.cpu().numpy(), ref, rtol=1e-11, atol=0)

    # the same helicities from the per-helicity call (every configuration)
    rows = P.matrix_element_per_helicity(mom).cpu().numpy()
    np.testing.assert_allclose(me64.cpu().numpy(), rows[subset].sum(axis=0), rtol=1e-13)

    # reduced precisions sum the same subset
    for prec in (M.FP32, M.MIXED, M.FP64_FP32COLOUR):
        me = P.matrix_element(mom, precision=prec).cpu().numpy()
        assert abs(me.sum() / ref.sum() - 1.0) < 1e-5, prec
        assert np.median(np.abs(me / ref - 1.0)) < 1e-5, prec

    # the helicity choice picks only from the subset; |M|^2 is the same sum
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    r_hel = torch.rand(n, dtype=torch.float64, device="cuda", generator=g)
    r_col = torch.rand(n, dtype=torch.float64, device="cuda", generator=g)
    me_s, hel, _ = P.select(mom, r_hel, r_col)
    assert set(hel.cpu().numpy().tolist()) <= set(subset)
    np.testing.assert_allclose(me_s.cpu().numpy(), ref, rtol=1e-11)

    # restoring the good helicities gives the original values bit for bit
    P.set_helicities(None)
    assert P.good_helicities() == good
    assert torch.equal(P.matrix_element(mom), full)
    P.close()


def test_set_helicities_rejects_bad_lists():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_18244_amd as M

    P = M.Process(M.PROCESSES["gg_tt"])
    good = P.good_helicities()
    for bad in ([3, 3], [5, 2], [-1], [16], list(range(17))):
        with pytest.raises(M.MgmeError) as e:
            P.set_helicities(bad)
        assert e.value.code == M.MGME_EINVAL
        assert P.good_helicities() == good  # unchanged
    P.close()
