"""Serving loop scheduler on the CPU, with the library's test double in
place of the device: admission by workspace budget, slot limit, arrival
order with pass-over, completion of every request, latency accounting."""
import os
import time

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2303_18244_amd", "libmgme.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libmgme.so not built")


def test_slots_budget_and_latency():
    import paper_2303_18244_amd as M

    # 2 us per event, 1 kB of workspace per event, 3 slots, 5 MB budget
    S = M.Server(n_slots=3, hbm_budget_bytes=5_000_000, fake_ns_per_event=2000.0, fake_bytes_per_event=1000)
    sizes = [1000, 4000, 2000, 500, 3000, 1500, 800, 2500]
    t0 = time.perf_counter()
    ids = [S.submit(None, nevt=n) for n in sizes]
    lats = [S.wait(i) for i in ids]
    wall = time.perf_counter() - t0
    st = S.stats()
    S.close()
    assert st["completed"] == len(sizes) and st["failed"] == 0 and st["events"] == sum(sizes)
    # the requests overlap (the scheduler's own count), within the slot limit
    assert 2 <= st["max_concurrent"] <= 3
    assert st["peak_workspace_bytes"] <= 5_000_000
    # every request lasts at least its scripted duration; overlapped, the
    # whole batch takes less than the same requests one after another (a
    # loose wall-clock bound, so that host scheduling jitter cannot fail it)
    for n, lat in zip(sizes, lats):
        assert lat >= n * 2000e-6 * 0.99
    assert wall < sum(sizes) * 2000e-9
    assert st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]


def test_large_request_runs_alone_and_small_ones_pass_it():
    import paper_2303_18244_amd as M

    S = M.Server(n_slots=4, hbm_budget_bytes=1_000_000, fake_ns_per_event=1000.0, fake_bytes_per_event=1000)
    a = S.submit(None, nevt=600)       # 0.6 MB
    big = S.submit(None, nevt=5000)    # 5 MB: larger than the budget, must run alone
    small = S.submit(None, nevt=300)   # fits beside the first, passes the big one
    S.wait(a)
    S.wait(small)
    S.wait(big)
    st = S.stats()
    S.close()
    assert st["completed"] == 3
    assert st["peak_workspace_bytes"] == 5_000_000  # the big request alone


def test_bad_arguments():
    import paper_2303_18244_amd as M

    with pytest.raises(M.MgmeError):
        M.Server(n_slots=0, fake_ns_per_event=1.0)
    S = M.Server(n_slots=1, fake_ns_per_event=1.0)
    with pytest.raises(M.MgmeError):
        S.submit(None, nevt=0)
    with pytest.raises(M.MgmeError):
        S.wait(12345)
    S.close()
