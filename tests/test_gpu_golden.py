"""Parity at the full 1024 x 840 single-instance configuration (T = 300,
C = 10, M = 10, Fe = 4000, noise 1e-3, 10000 steps) and at the 4096 x 4096
bandwidth configuration (T = 500, noise 1e-4) after a 100-step prefix (its
full 1000 steps: test_gpu_zfull_4096x4096.py), against oracle fields stored by
tests/golden/make_oracle_golden.py (oracle only) on a strided subsample that
includes the rows next to both electrodes and the periodic-wrap column
nx - 1, normalised by the oracle's full-grid max |X|.

Gated fields: rho, rho - 1 (normalised by its own max |rho - 1|, so that the
hydrostatic density departure is held to the same relative tolerance), u as
a vector field, rho_c and phi.  FP64 storage must match to 1e-11 and
FP32-deviation storage to 1e-5 on every field.  FP32-deviation storage with
FP32 collision arithmetic meets 1e-5 on rho, rho - 1, rho_c and phi; its
velocity is held only to a regression bound (the precision notes of the
design document give the measured level and the experiments on its cause)."""

import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "oracle_cfg1.npz")
KW = dict(nx=1024, ny=840, T=300.0, C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8, Lambda=0.25,
          Lambda_g=1e-6, noise_amp=1e-3, seed=181205711)
GOLDEN2 = os.path.join(HERE, "golden", "oracle_cfg2.npz")
KW2 = dict(nx=4096, ny=4096, T=500.0, C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8, Lambda=0.25,
           Lambda_g=1e-6, noise_amp=1e-4, seed=181205711)
SCALARS = ("rho", "rho_m1", "rho_c", "phi")


def _golden(path, what, case):
    if not os.path.exists(path):
        pytest.skip(f"oracle golden for {what} not generated yet (tests/golden/make_oracle_golden.py {case})")
    return np.load(path)


def _snapshots(gold):
    return sorted(int(k[4:]) for k in gold.files if k.startswith("rho_") and k[4:].isdigit())


def _errors(gold, f, step):
    rows, cols = gold["rows"], gold["cols"]
    e = {}
    for k in ("rho", "rho_m1", "ux", "uy", "rho_c", "phi"):
        if f"{k}_{step}" not in gold.files:
            continue
        got = f[k][np.ix_(rows, cols)]
        e[k] = float(np.max(np.abs(got - gold[f"{k}_{step}"])) / gold[f"max_{k}_{step}"])
    du = np.hypot(f["ux"][np.ix_(rows, cols)] - gold[f"ux_{step}"], f["uy"][np.ix_(rows, cols)] - gold[f"uy_{step}"])
    e["u"] = float(np.max(du) / gold[f"max_u_{step}"])
    return e


def _run(precision, snaps, kw, tuning=None):
    import torch

    from paper_1812_05711_amd.lbm_ec import Simulation

    sim = Simulation(device="cuda:0", precision=precision, **kw)
    if tuning is not None:
        sim.set_tuning(*tuning)
    out = {}
    for s in snaps:
        sim.step(s - sim.steps_done())
        out[s] = {k: v.cpu().numpy() for k, v in sim.fields().items()}
    torch.cuda.synchronize()
    sim.close()
    return out


def _gate(gold, res, snaps, precision, tol, gate_u=True):
    for s in snaps:
        e = _errors(gold, res[s], s)
        print(precision, s, {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
        for k in SCALARS:
            if k in e:
                assert e[k] <= tol, (precision, s, k, e)
        if gate_u:
            assert e["u"] <= tol, (precision, s, e)
    return e


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32_f64math", 1e-5), ("fp32", 1e-5)])
def test_cfg1_against_oracle(precision, tol):
    gold = _golden(GOLDEN, "1024 x 840", "cfg1")
    snaps = _snapshots(gold)
    res = _run(precision, snaps, KW)
    _gate(gold, res, snaps, precision, tol, gate_u=precision != "fp32")


def test_cfg1_fp32_arithmetic_velocity_regression_bound():
    """Not a parity test: FP32 storage with FP32 collision arithmetic misses
    the 1e-5 gate on u (8.3e-5 of max |u| after 10000 steps; the design notes
    give the experiments that place the error in the fluid collision's FP32
    arithmetic as a whole).  FP32 storage meets the gate with FP64 collision
    arithmetic (test_cfg1_against_oracle[fp32_f64math]).  This bound, about
    twice the measured level, only catches a regression of the FP32-arithmetic
    mode (test_cfg1_fp32_arithmetic_velocity_gate is the gate itself, marked as
    an expected failure)."""
    gold = _golden(GOLDEN, "1024 x 840", "cfg1")
    snaps = _snapshots(gold)
    res = _run("fp32", snaps, KW)
    e = _gate(gold, res, snaps, "fp32", 1e-5, gate_u=False)
    assert e["u"] <= 2e-4, e


@pytest.mark.xfail(strict=True, reason="FP32 collision arithmetic misses the 1e-5 gate on u after 10000 "
                   "steps; the precision notes of the design document give the measured level and the "
                   "experiments on its cause (strict: a pass would mean the gate is met and this mark goes)")
def test_cfg1_fp32_arithmetic_velocity_gate():
    """The parity gate on u for FP32 storage with FP32 collision arithmetic,
    expected to fail until that mode meets it."""
    gold = _golden(GOLDEN, "1024 x 840", "cfg1")
    if 10000 not in _snapshots(gold):
        pytest.skip("1024 x 840 oracle golden has no step 10000 yet")
    res = _run("fp32", [10000], KW)
    _gate(gold, res, [10000], "fp32", 1e-5, gate_u=True)


def _cfg2(step):
    gold = _golden(GOLDEN2, "4096 x 4096", "cfg2")
    if step not in _snapshots(gold):
        pytest.skip(f"4096 x 4096 oracle golden has no step {step} yet")
    return gold


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32_f64math", 1e-5), ("fp32", 1e-5)])
def test_cfg2_prefix_against_oracle(precision, tol):
    """4096 x 4096 after 100 steps (FP64 storage runs x-tiled collide tiles
    at this row length): every field within the precision's tolerance."""
    gold = _cfg2(100)
    res = _run(precision, [100], KW2)
    _gate(gold, res, [100], precision, tol, gate_u=True)
