"""Batched execution: every slot of a mixed batch computes exactly what the
same simulation computes alone through lbm_ec_step (bitwise), slots stop at
their own step counts, admission respects the workspace, and a slot admitted
while others run is unaffected by them."""

import numpy as np
import pytest

from gpu_util import errors, oracle_fields

pytestmark = pytest.mark.gpu

BASE = dict(T=200.0, C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8, Lambda=0.25, Lambda_g=1e-6, noise_amp=1e-3,
            seed=181205711)
MIX = [
    (dict(BASE, nx=24, ny=10, T=150.0, instance_id=1), 30),
    (dict(BASE, nx=61, ny=20, T=250.0, instance_id=2), 45),
    (dict(BASE, nx=16, ny=40, C=1.0, instance_id=3), 17),
    (dict(BASE, nx=80, ny=64, T=120.0, C=100.0, instance_id=4), 60),
    (dict(BASE, nx=122, ny=100, instance_id=5, init_mode="eq29"), 33),
]


def _alone(kw, n, precision):
    import torch

    from paper_1812_05711_amd.lbm_ec import Simulation

    sim = Simulation(device="cuda:0", precision=precision, **kw)
    sim.step(n)
    f = {k: v.cpu().numpy() for k, v in sim.fields().items()}
    torch.cuda.synchronize()
    sim.close()
    return f


def _batch(precision, max_slots=8, extra=1 << 20):
    from paper_1812_05711_amd.lbm_ec import Batch, batch_workspace_bytes, make_params

    ps = [make_params(precision=precision, **kw) for kw, _ in MIX]
    ws = batch_workspace_bytes(ps, max_slots, 64) + extra
    return Batch(max_slots, ws, precision=precision, emit_every=10, hist_rows=64)


@pytest.mark.parametrize("precision", ["fp64", "fp32_f64math", "fp32"])
def test_mix_equals_alone_bitwise(precision):
    b = _batch(precision)
    slots = [b.admit(n, **kw) for kw, n in MIX]
    assert None not in slots
    b.step(7)
    # a late arrival joins while the others run
    late_kw, late_n = dict(BASE, nx=40, ny=33, T=300.0, instance_id=9), 25
    late = b.admit(late_n, **late_kw)
    assert late is not None
    b.step(100)
    done = set(b.poll())
    assert done == set(slots + [late])
    for (kw, n), s in list(zip(MIX, slots)) + [((late_kw, late_n), late)]:
        assert b.steps_done(s) == n
        got = {k: v.cpu().numpy() for k, v in b.fields(s).items()}
        ref = _alone(kw, n, precision)
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (precision, kw["nx"], kw["ny"], k)
    b.close()


def test_batch_slot_matches_oracle():
    b = _batch("fp64")
    kw, n = MIX[1]
    s = b.admit(n, **kw)
    other = b.admit(MIX[3][1], **MIX[3][0])
    b.step(200)
    assert set(b.poll()) == {s, other}
    got = {k: v.cpu().numpy() for k, v in b.fields(s).items()}
    e = errors(got, oracle_fields(kw, n))
    assert max(e["rho"], e["rho_m1"], e["u"], e["rho_c"], e["phi"]) <= 1e-11, e
    b.close()


def test_history_rows_match_fields():
    b = _batch("fp64")
    kw, n = MIX[3]
    s = b.admit(n, **kw)
    b.step(n)
    b.poll()
    h = b.history(s)
    steps = h[:, 0]
    assert list(steps[: n // 10]) == [10.0 * (r + 1) for r in range(n // 10)]
    f = b.fields(s)
    import math

    from oracle import Params, lattice_constants

    u0 = lattice_constants(Params(**kw)).u0
    uy = f["uy"].cpu().numpy() * u0
    row = n // 10 - 1  # n = 60 is a multiple of 10
    assert math.isclose(h[row, 1], float(np.sqrt(np.mean(uy * uy))), rel_tol=1e-12)
    a1 = float(np.max(np.abs(np.fft.fft(uy, axis=1)[:, 1])) / uy.shape[1])
    assert math.isclose(h[row, 4], a1, rel_tol=1e-9)
    # a negative row count is refused
    import ctypes

    from paper_1812_05711_amd.lbm_ec import EINVAL, HIST_COLS, lib

    buf = (ctypes.c_double * HIST_COLS)()
    assert lib().lbm_ec_batch_history(b._h, int(s), buf, -1) == EINVAL
    b.close()


def test_admission_respects_workspace_and_reuse():
    from paper_1812_05711_amd.lbm_ec import Batch, batch_workspace_bytes, make_params

    kw = dict(BASE, nx=64, ny=32)
    one = batch_workspace_bytes([make_params(**kw)], 4, 8) - batch_workspace_bytes([], 4, 8)
    ws = batch_workspace_bytes([], 4, 8) + 2 * one + 1024
    b = Batch(4, ws, precision="fp64", emit_every=0, hist_rows=8)
    a = b.admit(5, **kw)
    c = b.admit(5, **dict(kw, instance_id=1))
    assert a is not None and c is not None
    assert b.admit(5, **dict(kw, instance_id=2)) is None  # workspace full: EBUSY
    b.step(5)
    assert set(b.poll()) == {a, c}
    b.release(a)
    d = b.admit(7, **dict(kw, instance_id=2))
    assert d is not None
    assert b.steps_done(d) == 0  # a reused slot starts from its own state
    b.step(7)
    assert b.poll() == [d]
    got = {k: v.cpu().numpy() for k, v in b.fields(d).items()}
    ref = _alone(dict(kw, instance_id=2), 7, "fp64")
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k
    b.close()


def test_many_slots_equal_alone_bitwise():
    """More slots than a wave has lanes (the block-to-slot search then runs on
    two levels): 150 small slots of varied shapes and step counts, including
    shapes whose chunk solves and interface systems have no blocks; a sample
    across the whole slot range equals the same simulations run alone."""
    from paper_1812_05711_amd.lbm_ec import Batch, batch_workspace_bytes, make_params

    kws = []
    for i in range(150):
        nx = (2, 3, 8, 12, 17, 24)[i % 6]
        ny = (6, 10, 16, 40, 70)[i % 5]
        kws.append((dict(BASE, nx=nx, ny=ny, T=150.0 + i % 50, instance_id=i), 5 + i % 7))
    ps = [make_params(precision="fp64", **kw) for kw, _ in kws]
    ws = batch_workspace_bytes(ps, len(ps), 4) + (1 << 20)
    b = Batch(len(ps), ws, precision="fp64", emit_every=0, hist_rows=4)
    slots = [b.admit(n, **kw) for kw, n in kws]
    assert None not in slots
    b.step(20)
    assert set(b.poll()) == set(slots)
    for i in (0, 1, 63, 64, 65, 100, 127, 128, 149):
        kw, n = kws[i]
        assert b.steps_done(slots[i]) == n
        got = {k: v.cpu().numpy() for k, v in b.fields(slots[i]).items()}
        ref = _alone(kw, n, "fp64")
        for k in ref:
            assert np.all(np.isfinite(ref[k])), (i, k)
            assert np.array_equal(got[k], ref[k]), (i, kw["nx"], kw["ny"], k)
    b.close()


def test_empty_batch_and_refused_arguments():
    """Stepping and polling an empty batch does nothing; a precision other
    than the batch's, a non-positive step count, more slots than the limit
    and a release of a free slot are refused with EINVAL."""
    from paper_1812_05711_amd.lbm_ec import EINVAL, Batch, LbmEcError, batch_workspace_bytes

    b = Batch(4, batch_workspace_bytes([], 4, 8) + (1 << 20), precision="fp64", emit_every=0, hist_rows=8)
    b.step(10)
    assert b.poll() == []
    kw = dict(BASE, nx=16, ny=12)
    for bad in (dict(kw, precision="fp32"), dict(kw, nx=0)):
        with pytest.raises(LbmEcError) as ei:
            b.admit(5, **bad)
        assert ei.value.code == EINVAL
    with pytest.raises(LbmEcError) as ei:
        b.admit(0, **kw)
    assert ei.value.code == EINVAL
    with pytest.raises(LbmEcError) as ei:
        b.release(2)
    assert ei.value.code == EINVAL
    b.close()
    with pytest.raises(LbmEcError) as ei:
        Batch(5000, 1 << 20, precision="fp64")
    assert ei.value.code == EINVAL


def test_one_column_slots_equal_alone_bitwise():
    """Channels of one and two columns (no y solves: their y-solve launch
    ranges are empty) between wider slots, as the hydrostatic companions of a
    hysteresis run use them."""
    from paper_1812_05711_amd.lbm_ec import Batch, batch_workspace_bytes, make_params

    kws = [dict(BASE, nx=24, ny=20, instance_id=1),
           dict(BASE, nx=1, ny=25, noise_amp=0.0),
           dict(BASE, nx=2, ny=16, instance_id=2),
           dict(BASE, nx=31, ny=25, instance_id=3, init_mode="eq29"),
           dict(BASE, nx=1, ny=50, T=140.0)]
    ps = [make_params(precision="fp64", **kw) for kw in kws]
    b = Batch(8, batch_workspace_bytes(ps, 8, 16) + (1 << 20), precision="fp64", emit_every=10, hist_rows=16)
    slots = [b.admit(40, **kw) for kw in kws]
    b.step(40)
    assert sorted(b.poll()) == sorted(slots)
    for kw, s in zip(kws, slots):
        got = {k: v.cpu().numpy() for k, v in b.fields(s).items()}
        ref = _alone(kw, 40, "fp64")
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (kw["nx"], kw["ny"], k)
    b.close()
