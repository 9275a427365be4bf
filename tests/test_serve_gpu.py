"""Serving loop on the GPU: requests of different processes, sizes and
precisions run concurrently, and each result equals the same request run
alone (bitwise: every request runs the kernels of a standalone call)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_mix_equals_alone():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_18244_amd as M

    procs = {name: M.Process(pdg) for name, pdg in M.PROCESSES.items()}
    plan = [("gg_tt", 5000, M.FP64), ("gg_ttgg", 3000, M.MIXED), ("gg_ttggg", 300, M.FP64),
            ("gg_ttg", 20000, M.FP32), ("gg_ttgg", 7001, M.FP64), ("gg_ttggg", 197, M.MIXED),
            ("ee_mumu", 4000, M.FP64), ("gg_ttg", 1500, M.MIXED), ("gg_tt", 65536, M.FP32),
            ("gg_ttgg", 1024, M.FP32), ("gg_ttgg", 2000, M.FP64_FP32COLOUR)]
    inputs, refs = [], []
    for k, (name, n, prec) in enumerate(plan):
        P = procs[name]
        sq = 500.0 if name == "ee_mumu" else 1500.0
        mom, _ = P.rambo(sq, 1000 + k, 0, n)
        inputs.append(mom)
        refs.append(P.matrix_element(mom, precision=prec).clone())
    torch.cuda.synchronize()
    S = M.Server(n_slots=4, hbm_budget_bytes=24 << 30)
    outs, ids = [], []
    for (name, n, prec), mom in zip(plan, inputs):
        out = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
        outs.append(out)
        ids.append(S.submit(procs[name], mom, precision=prec, out=out))
    lat = [S.wait(i) for i in ids]
    st = S.stats()
    S.close()
    assert st["completed"] == len(plan) and st["failed"] == 0
    assert st["max_concurrent"] >= 2
    for (name, n, prec), out, ref in zip(plan, outs, refs):
        assert torch.equal(out, ref), (name, n, prec)
    print(f"served {len(plan)} requests, latency p50 {st['p50_ms']:.2f} ms p99 {st['p99_ms']:.2f} ms, "
          f"max concurrent {st['max_concurrent']}")
