"""mgme_matrix_element_noalloc against mgme_matrix_element (through the C
ABI): the same bits on two calls in a row, the second with a smaller batch,
for fused and staged processes in every precision.  The no-allocation call
stages in a fixed array, so its sub-batches are smaller than those of the
allocating call; every event's |M|^2 must not depend on that."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SEED = 230318244

# process -> (first batch, second smaller batch); the staged process spans
# several 512-event FP64 (1024-event FP32 and mixed) sub-batches with a
# ragged tail; the fused processes take no workspace at all.
CASES = {
    "gg_tt": (5000, 333),
    "gg_ttgg": (23000, 10500),
    "gg_ttggg": (1700, 600),
}


@pytest.fixture(scope="module")
def procs():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_18244_amd as M

    return {name: M.Process(M.PROCESSES[name]) for name in CASES}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_noalloc_equals_allocating_call(procs, name, prec):
    import torch

    P = procs[name]
    n1, n2 = CASES[name]
    print(f"no-alloc: {name} precision {prec}, batches {n1} then {n2}", flush=True)
    mom, _ = P.rambo(1500.0, SEED, 0, n1)
    ref = P.matrix_element(mom, precision=prec).cpu().numpy()
    out = torch.full((n1,), -1.0, dtype=torch.float64, device="cuda")
    P.matrix_element_noalloc(mom, precision=prec, out=out)
    a = out.cpu().numpy()
    np.testing.assert_array_equal(a, ref)
    # second call, smaller batch, offset into the same momenta (padded ld)
    out2 = torch.full((n2 + 7,), -2.0, dtype=torch.float64, device="cuda")
    P.matrix_element_noalloc(mom, nevt=n2, precision=prec, out=out2)
    b = out2.cpu().numpy()
    np.testing.assert_array_equal(b[:n2], ref[:n2])
    assert np.all(b[n2:] == -2.0)
    assert np.all(np.isfinite(a)) and np.all(a > 0)


def test_noalloc_rejects_bad_arguments(procs):
    import paper_2303_18244_amd as M

    L = M.lib()
    P = procs["gg_ttgg"]
    assert L.mgme_matrix_element_noalloc(None, None, 10, 10, 0, None, None) == M.MGME_EINVAL
    assert L.mgme_matrix_element_noalloc(P._h, None, 10, 10, 7, None, None) == M.MGME_EINVAL
    assert L.mgme_matrix_element_noalloc(P._h, None, -1, 10, 0, None, None) == M.MGME_EINVAL
    assert L.mgme_matrix_element_noalloc(P._h, None, 0, 0, 0, None, None) == M.MGME_OK
