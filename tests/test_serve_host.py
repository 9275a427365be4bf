"""Serving loop scheduler on the CPU, with the library's test double in
place of the device: admission by footprint budget, slot limit, arrival
order with bounded pass-over, splitting of oversize requests, a failing
request surfacing as its own error, latency accounting."""
import os
import threading
import time

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2303_18244_amd", "libmgme.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libmgme.so not built")


def test_slots_budget_and_latency():
    import paper_2303_18244_amd as M

    # 2 us per event, 1 kB of footprint per event, 3 slots, 5 MB budget
    S = M.Server(n_slots=3, hbm_budget_bytes=5_000_000, fake_ns_per_event=2000.0, fake_bytes_per_event=1000)
    sizes = [1000, 4000, 2000, 500, 3000, 1500, 800, 2500]
    t0 = time.perf_counter()
    ids = [S.submit(None, nevt=n) for n in sizes]
    lats = [S.wait(i) for i in ids]
    wall = time.perf_counter() - t0
    st = S.stats()
    S.close()
    assert st["completed"] == len(sizes) and st["failed"] == 0 and st["events"] == sum(sizes)
    assert st["split_requests"] == 0 and st["budget_bytes"] == 5_000_000
    # the requests overlap (the scheduler's own count), within the slot limit
    assert 2 <= st["max_concurrent"] <= 3
    assert st["peak_footprint_bytes"] <= 5_000_000
    # every request lasts at least its scripted duration; overlapped, the
    # whole batch takes less than the same requests one after another (a
    # loose wall-clock bound, so that host scheduling jitter cannot fail it)
    for n, lat in zip(sizes, lats):
        assert lat >= n * 2000e-6 * 0.99
    assert wall < sum(sizes) * 2000e-9
    assert st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]


def test_oversize_request_is_split_and_small_ones_pass_it():
    import paper_2303_18244_amd as M

    S = M.Server(n_slots=4, hbm_budget_bytes=1_000_000, fake_ns_per_event=1000.0, fake_bytes_per_event=1000)
    a = S.submit(None, nevt=600)       # 0.6 MB
    big = S.submit(None, nevt=5000)    # 5 MB: larger than the budget, split into parts of 640 events
    small = S.submit(None, nevt=300)   # fits beside the first, may pass the big one's parts
    S.wait(a)
    S.wait(small)
    lat_big = S.wait(big)
    st = S.stats()
    S.close()
    assert st["completed"] == 3 and st["events"] == 5900 and st["split_requests"] == 1
    assert st["peak_footprint_bytes"] <= 1_000_000
    # eight parts (7 x 640 + 520 events); two parts exceed the budget, so
    # they run one after another
    assert lat_big >= 5000 * 1000e-6 * 0.99


def test_part_of_64_events_that_does_not_fit_runs_alone():
    import paper_2303_18244_amd as M

    S = M.Server(n_slots=2, hbm_budget_bytes=10_000, fake_ns_per_event=10.0, fake_bytes_per_event=1000)
    r = S.submit(None, nevt=200)  # parts of 64 events (64 kB each) exceed the 10 kB budget: run alone
    S.wait(r)
    st = S.stats()
    S.close()
    assert st["completed"] == 1 and st["split_requests"] == 1 and st["max_concurrent"] == 1


def _starvation_run(max_pass_over):
    """Small requests (30 units of a 100 budget, 50 ms each; three fit at
    once) keep arriving every 8 ms for 1 s, faster than they are served; a
    large request (90 units) fits only when no small one runs.  The first
    three small requests start 15 ms apart, so that completions never
    coincide and the running set never empties by chance.  Returns the large
    request's latency in ms."""
    import paper_2303_18244_amd as M

    S = M.Server(n_slots=4, hbm_budget_bytes=100, fake_ns_per_event=50e6 / 30, fake_bytes_per_event=1,
                 max_pass_over=max_pass_over)
    # footprint = nevt units; a small request lasts 50 ms, the large one 150 ms
    small = []
    for _ in range(3):
        small.append(S.submit(None, nevt=30))
        time.sleep(0.015)
    big = S.submit(None, nevt=90)
    stop = time.perf_counter() + 1.0
    while time.perf_counter() < stop:
        small.append(S.submit(None, nevt=30))
        time.sleep(0.008)
    lat = S.wait(big)
    for r in small:
        S.wait(r)
    S.close()
    return lat


def test_bounded_pass_over_prevents_starvation():
    aged = _starvation_run(max_pass_over=4)
    starved = _starvation_run(max_pass_over=1_000_000)
    # with the bound the large request waits for a few pass-overs and the
    # running small requests to drain; without it, for the whole arrival stream
    assert aged < 600.0, aged
    assert starved > 1000.0, starved


def test_failing_request_surfaces_alone_and_queue_keeps_moving():
    import paper_2303_18244_amd as M

    S = M.Server(n_slots=2, fake_ns_per_event=1000.0, fake_bytes_per_event=0, fake_fail_nevt=777)
    sizes = [500, 777, 400, 300, 777, 200]
    ids = [S.submit(None, nevt=n) for n in sizes]
    codes = []
    for i in ids:
        try:
            S.wait(i)
            codes.append(M.MGME_OK)
        except M.MgmeError as e:
            codes.append(e.code)
    S.drain()
    st = S.stats()
    S.close()
    assert codes == [M.MGME_EDEVICE if n == 777 else M.MGME_OK for n in sizes]
    assert st["failed"] == 2 and st["completed"] == 4 and st["events"] == 1400


def test_failing_part_fails_the_whole_request():
    import paper_2303_18244_amd as M

    # 1000 events at 1 B per event against a 500 B budget: parts of 256, 256, 256 and 232 (fails)
    S = M.Server(n_slots=2, hbm_budget_bytes=500, fake_ns_per_event=100.0, fake_bytes_per_event=1,
                 fake_fail_nevt=232)
    r = S.submit(None, nevt=1000)
    ok = S.submit(None, nevt=100)
    with pytest.raises(M.MgmeError) as ei:
        S.wait(r)
    assert ei.value.code == M.MGME_EDEVICE
    S.wait(ok)
    st = S.stats()
    S.close()
    assert st["failed"] == 1 and st["completed"] == 1 and st["split_requests"] == 1


def test_concurrent_submitters():
    """Several host threads submitting and waiting at once (the scheduler's
    lock discipline; the sanitizer build runs the same pattern)."""
    import paper_2303_18244_amd as M

    S = M.Server(n_slots=3, hbm_budget_bytes=50_000, fake_ns_per_event=200.0, fake_bytes_per_event=10)
    errors = []

    def worker(k):
        try:
            for j in range(20):
                S.wait(S.submit(None, nevt=100 + 37 * ((k * 20 + j) % 50)))
        except Exception as e:  # noqa: BLE001
            errors.append(e)

    th = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    st = S.stats()
    S.close()
    assert not errors and st["completed"] == 80 and st["peak_footprint_bytes"] <= 50_000


def test_bad_arguments():
    import paper_2303_18244_amd as M

    with pytest.raises(M.MgmeError):
        M.Server(n_slots=0, fake_ns_per_event=1.0)
    with pytest.raises(M.MgmeError):
        M.Server(n_slots=1, max_pass_over=-1, fake_ns_per_event=1.0)
    S = M.Server(n_slots=1, fake_ns_per_event=1.0)
    with pytest.raises(M.MgmeError):
        S.submit(None, nevt=0)
    with pytest.raises(M.MgmeError):
        S.wait(12345)
    S.close()
