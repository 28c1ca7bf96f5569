"""Parity at the full 1024 x 840 single-instance configuration (T = 300,
C = 10, M = 10, Fe = 4000, noise 1e-3, 10000 steps) and on a 100-step
prefix of the 4096 x 4096 bandwidth configuration (T = 500, noise 1e-4),
against oracle fields stored by tests/golden/make_oracle_golden.py (oracle
only) on a strided subsample, normalised by the oracle's full-grid max |X|.

FP64 storage must match to 1e-11 and FP32-deviation storage with FP64
collision arithmetic to 1e-5 on every field.  FP32-deviation storage with
FP32 collision arithmetic meets 1e-5 on rho, rho_c and phi; its velocity
error is bounded here at the measured level (see the precision notes in the
design document)."""

import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "oracle_cfg1.npz")
KW = dict(nx=1024, ny=840, T=300.0, C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8, Lambda=0.25,
          Lambda_g=1e-6, noise_amp=1e-3, seed=181205711)
GOLDEN2 = os.path.join(HERE, "golden", "oracle_cfg2_prefix.npz")
KW2 = dict(nx=4096, ny=4096, T=500.0, C=10.0, M=10.0, Fe=4000.0, tau_plus=0.8, Lambda=0.25,
           Lambda_g=1e-6, noise_amp=1e-4, seed=181205711)


def _golden(path=GOLDEN, what="1024 x 840", case="cfg1"):
    if not os.path.exists(path):
        pytest.skip(f"oracle golden for {what} not generated yet (tests/golden/make_oracle_golden.py {case})")
    return np.load(path)


def _errors(gold, f, step):
    rows, cols = gold["rows"], gold["cols"]
    e = {}
    for k in ("rho", "ux", "uy", "rho_c", "phi"):
        got = f[k][np.ix_(rows, cols)]
        e[k] = float(np.max(np.abs(got - gold[f"{k}_{step}"])) / gold[f"max_{k}_{step}"])
    du = np.hypot(f["ux"][np.ix_(rows, cols)] - gold[f"ux_{step}"], f["uy"][np.ix_(rows, cols)] - gold[f"uy_{step}"])
    e["u"] = float(np.max(du) / gold[f"max_u_{step}"])
    return e


def _run(precision, snaps, kw=KW):
    import torch

    from paper_1812_05711_amd.lbm_ec import Simulation

    sim = Simulation(device="cuda:0", precision=precision, **kw)
    out = {}
    for s in snaps:
        sim.step(s - sim.steps_done())
        out[s] = {k: v.cpu().numpy() for k, v in sim.fields().items()}
    torch.cuda.synchronize()
    sim.close()
    return out


@pytest.mark.parametrize("precision,tol,utol", [("fp64", 1e-11, 1e-11), ("fp32_f64math", 1e-5, 1e-5),
                                                ("fp32", 1e-5, 3e-4)])
def test_cfg1_against_oracle(precision, tol, utol):
    gold = _golden()
    snaps = [int(k.split("_")[1]) for k in gold.files if k.startswith("rho_") and k[4:].isdigit()]
    res = _run(precision, sorted(snaps))
    for s in sorted(snaps):
        e = _errors(gold, res[s], s)
        print(precision, s, {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
        for k in ("rho", "rho_c", "phi"):
            assert e[k] <= tol, (precision, s, k, e)
        assert e["u"] <= utol, (precision, s, e)


@pytest.mark.parametrize("precision", ["fp32_f64math", "fp32"])
def test_cfg2_prefix_against_oracle(precision):
    """4096 x 4096 (FP32 storage; FP64 storage is limited to nx <= 2048),
    100 steps: every field within 1e-5 (the FP32-arithmetic velocity drift of
    the long runs has not built up after 100 steps)."""
    gold = _golden(GOLDEN2, "4096 x 4096", "cfg2_prefix")
    res = _run(precision, [100], KW2)
    e = _errors(gold, res[100], 100)
    print(precision, 100, {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    for k in ("rho", "rho_c", "phi", "u"):
        assert e[k] <= 1e-5, (precision, k, e)
