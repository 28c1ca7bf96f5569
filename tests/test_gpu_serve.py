"""Serving on the GPU: a stream of requests of mixed sizes arrives while
others run; the workspace budget makes some wait; every request finishes and
a sample of them equals the same simulation run alone, bitwise."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_served_stream_identity_and_queueing():
    import torch

    from paper_1812_05711_amd.lbm_ec import Simulation, batch_workspace_bytes, make_params
    from paper_1812_05711_amd.serve import BatchBackend, make_requests, serve

    reqs = make_requests(24, rate=400.0, seed=7, steps=300, sizes=(64, 128), weights=(0.5, 0.5))
    biggest = max(reqs, key=lambda r: r["params"]["nx"] * r["params"]["ny"])
    one = batch_workspace_bytes([make_params(**biggest["params"])], 8, 1) - batch_workspace_bytes([], 8, 1)
    budget = batch_workspace_bytes([], 8, 1) + 3 * one
    sample = {0, 5, 11, 23}
    be = BatchBackend(budget, max_slots=8, keep=sample)
    records, summary = serve(reqs, be, chunk=50, max_wall=300.0)
    be.close()
    assert sorted(r["id"] for r in records) == list(range(24))
    assert summary["max_queue"] > 0
    for rid in sample:
        req = reqs[rid]
        sim = Simulation(device="cuda:0", **req["params"])
        sim.step(req["steps"])
        ref = {k: v.cpu().numpy() for k, v in sim.fields().items()}
        torch.cuda.synchronize()
        sim.close()
        for k in ref:
            assert np.array_equal(be.kept[rid][k], ref[k]), (rid, k)
