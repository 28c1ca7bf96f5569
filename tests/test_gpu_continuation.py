"""Continuation at another T through the C ABI (lbm_ec_set_T,
lbm_ec_batch_set_T) against the oracle's, and the collector current (the
cathode current of Ne_0, section V.2) of lbm_ec_stats and of the batch
history.

A schedule is a list of (steps, T): run the steps, then continue at T (None:
no change).  Both sides run the same schedule; the oracle's reading of a
change is pinned in test_oracle_continuation.py.  Tolerances as in the
parity tests: 1e-11 relative for FP64 storage, 1e-5 for FP32 storage; the
electrode currents, sums over a row of post-collision populations, 1e-10
relative (FP64) and 1e-4 (FP32 storage).
"""

import numpy as np
import pytest

from gpu_util import errors

pytestmark = pytest.mark.gpu

BASE = dict(T=200.0, C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8, Lambda=0.25, Lambda_g=1e-6,
            noise_amp=1e-3, seed=181205711)
TOL = {"fp64": 1e-11, "fp32_f64math": 1e-5, "fp32": 1e-5}
TOL_CUR = {"fp64": 1e-10, "fp32_f64math": 1e-4, "fp32": 1e-4}

SCHEDULES = [
    [(30, 150.0), (30, None)],
    [(0, 260.0), (40, None)],                  # at the first state
    [(20, 150.0), (0, 180.0), (25, None)],     # two changes with no step between
    [(15, 170.0), (15, 140.0), (15, None)],
]


def _oracle(kw, schedule):
    from oracle import Oracle, Params

    o = Oracle(Params(**kw))
    for n, T in schedule:
        o.step(n)
        if T is not None:
            o.set_T(T)
    return o


def _gpu(kw, schedule, precision):
    import torch

    from paper_1812_05711_amd.lbm_ec import Simulation

    sim = Simulation(device="cuda:0", precision=precision, **kw)
    for n, T in schedule:
        sim.step(n)
        if T is not None:
            sim.set_T(T)
    f = {k: v.cpu().numpy() for k, v in sim.fields().items()}
    st, _ = sim.stats()
    torch.cuda.synchronize()
    f["steps"] = sim.steps_done()
    sim.close()
    return f, st


@pytest.mark.parametrize("precision", ["fp64", "fp32_f64math", "fp32"])
@pytest.mark.parametrize("sched", range(len(SCHEDULES)))
@pytest.mark.parametrize("nx,ny", [(24, 20), (61, 50), (5, 1027)])
def test_set_T_matches_oracle(nx, ny, sched, precision):
    schedule = SCHEDULES[sched]
    kw = dict(BASE, nx=nx, ny=ny)
    print("set_T", nx, ny, precision, schedule, flush=True)
    o = _oracle(kw, schedule)
    g, st = _gpu(kw, schedule, precision)
    assert g["steps"] == sum(n for n, _ in schedule)
    e = errors(g, o.fields())
    print({k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    for k in ("rho", "rho_m1", "u", "rho_c", "phi"):
        assert e[k] <= TOL[precision], (k, e)
    inj, col = o.electrode_currents()
    assert abs(st["q_injector"] - inj) <= TOL_CUR[precision] * abs(inj), (st["q_injector"], inj)
    assert abs(-st["q_collector"] - col) <= TOL_CUR[precision] * abs(col), (st["q_collector"], col)


def test_refused_T_changes_nothing():
    import torch

    from paper_1812_05711_amd.lbm_ec import EINVAL, LbmEcError, Simulation

    kw = dict(BASE, nx=24, ny=20)
    runs = []
    for refuse in (False, True):
        sim = Simulation(device="cuda:0", precision="fp64", **kw)
        sim.step(10)
        if refuse:
            for bad in (-1.0, 0.0, float("nan"), float("inf")):
                with pytest.raises(LbmEcError) as ei:
                    sim.set_T(bad)
                assert ei.value.code == EINVAL
        sim.step(10)
        runs.append({k: v.cpu().numpy() for k, v in sim.fields().items()})
        torch.cuda.synchronize()
        sim.close()
    for k in runs[0]:
        assert np.array_equal(runs[0][k], runs[1][k]), k


@pytest.mark.parametrize("precision", ["fp64", "fp32_f64math"])
def test_batch_set_T_equals_alone_bitwise(precision):
    import torch

    from paper_1812_05711_amd.lbm_ec import HIST_CURRENT, Batch, Simulation, batch_workspace_bytes, make_params

    kwa = dict(BASE, nx=40, ny=30, instance_id=1)
    kwb = dict(BASE, nx=24, ny=20, instance_id=2, T=230.0)
    ps = [make_params(precision=precision, **kw) for kw in (kwa, kwb)]
    b = Batch(4, batch_workspace_bytes(ps, 4, 16) + (1 << 20), precision=precision, emit_every=10, hist_rows=16)
    sa, sb = b.admit(60, **kwa), b.admit(60, **kwb)
    b.step(25)
    b.set_T(sa, 150.0)
    b.step(35)
    assert set(b.poll()) == {sa, sb}
    got = {s: {k: v.cpu().numpy() for k, v in b.fields(s).items()} for s in (sa, sb)}
    hist = b.history(sa)

    alone = {}
    for s, kw, sched in ((sa, kwa, [(25, 150.0), (35, None)]), (sb, kwb, [(60, None)])):
        sim = Simulation(device="cuda:0", precision=precision, **kw)
        for n, T in sched:
            sim.step(n)
            if T is not None:
                sim.set_T(T)
        alone[s] = {k: v.cpu().numpy() for k, v in sim.fields().items()}
        if s == sa:
            st, _ = sim.stats()
        torch.cuda.synchronize()
        sim.close()
    for s in (sa, sb):
        for k in alone[s]:
            assert np.array_equal(got[s][k], alone[s][k]), (precision, s, k)
    # the last history row is the final step: its collector current is the
    # one lbm_ec_stats reports for the same state
    last = hist[hist[:, 0] == 60]
    assert len(last) == 1
    assert last[0, HIST_CURRENT] == pytest.approx(-st["q_collector"], rel=1e-12)
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_f64math"])
def test_fields_right_after_a_change(precision):
    """lbm_ec_fields between lbm_ec_set_T and the next step: the charge keeps
    its nondimensional value, the velocity its lattice value (u / u0 scales
    by u0_old / u0_new = T_old / T_new), the density its departure from the
    reference row."""
    import torch

    from paper_1812_05711_amd.lbm_ec import Simulation

    sim = Simulation(device="cuda:0", precision=precision, **dict(BASE, nx=24, ny=20))
    sim.step(15)
    before = {k: v.cpu().numpy() for k, v in sim.fields().items()}
    sim.set_T(150.0)
    after = {k: v.cpu().numpy() for k, v in sim.fields().items()}
    torch.cuda.synchronize()
    sim.close()
    np.testing.assert_allclose(after["rho_c"], before["rho_c"], rtol=1e-12, atol=0)
    for k in ("ux", "uy"):
        np.testing.assert_allclose(after[k], before[k] * (200.0 / 150.0), rtol=1e-12,
                                   atol=1e-12 * np.abs(before[k]).max())
