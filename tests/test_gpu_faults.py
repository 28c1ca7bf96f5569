"""Failure detection on the GPU path, forced from the host (a NaN written
into one population through the test hooks, no kernel is made to fault):
the health check flags the poisoned instance, and in a batch only the
poisoned slot; the other slots still equal their runs alone, bitwise, and
the serving backend reports the poisoned request as unhealthy."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

BASE = dict(T=200.0, C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8, Lambda=0.25, Lambda_g=1e-6, noise_amp=1e-3,
            seed=181205711)


def test_single_instance_health_check():
    from paper_1812_05711_amd.lbm_ec import Simulation

    sim = Simulation(device="cuda:0", **dict(BASE, nx=32, ny=20))
    sim.step(5)
    st, ok = sim.stats()
    assert ok and st["bad"] == 0
    sim.debug_poison()
    sim.step(3)
    st, ok = sim.stats()
    assert not ok and st["bad"] > 0
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_f64math"])
def test_poisoned_slot_is_flagged_alone(precision):
    from paper_1812_05711_amd.lbm_ec import Batch, Simulation, batch_workspace_bytes, make_params

    kws = [dict(BASE, nx=24, ny=16, instance_id=i, T=150.0 + 20 * i) for i in range(3)]
    ps = [make_params(precision=precision, **kw) for kw in kws]
    b = Batch(4, batch_workspace_bytes(ps, 3, 8) + (1 << 20), precision=precision, emit_every=10, hist_rows=8)
    slots = [b.admit(30, **kw) for kw in kws]
    b.step(10)
    b.debug_poison(slots[1])
    b.step(20)
    assert sorted(b.poll()) == sorted(slots)
    for i, s in enumerate(slots):
        h = b.history(s)
        last = h[h[:, 0] > 0][-1]
        assert last[0] == 30
        if i == 1:
            assert last[5] > 0
        else:
            assert last[5] == 0
            got = {k: v.cpu().numpy() for k, v in b.fields(s).items()}
            sim = Simulation(device="cuda:0", precision=precision, **kws[i])
            sim.step(30)
            ref = {k: v.cpu().numpy() for k, v in sim.fields().items()}
            sim.close()
            for k in ref:
                assert np.array_equal(got[k], ref[k]), (i, k)
    b.close()


def test_serving_backend_reports_unhealthy_request():
    from paper_1812_05711_amd.serve import BatchBackend, make_requests

    reqs = make_requests(2, rate=50.0, steps=40)
    be = BatchBackend(1 << 30, max_slots=4, precision=reqs[0]["params"]["precision"])
    slots = [be.admit(r) for r in reqs]
    be.step(10)
    be.batch.debug_poison(slots[0])
    be.step(40)
    done = be.poll()
    assert sorted(done) == sorted(slots)
    flags = [be.finish(s, r)["healthy"] for s, r in zip(slots, reqs)]
    assert flags == [False, True]
    be.close()
