"""Parity of the 4096 x 4096 bandwidth workload (T = 500, C = 10, M = 10,
Fe = 4000, noise 1e-4) after its stated 1000 steps, against the oracle's
fields at step 1000 stored by tests/golden/make_oracle_golden.py (oracle
only; a strided subsample with the rows next to both electrodes and the
periodic-wrap column, normalised by the oracle's full-grid max |X|), in the
launch shapes the benchmark's autotuner picks.  The helpers and the gates are
those of test_gpu_golden.py (this file is collected after it: the run of
1000 steps at this size is the longest single case)."""

import pytest

from test_gpu_golden import KW2, _cfg2, _gate, _run

pytestmark = pytest.mark.gpu


def _bench_tuning(precision, kw):
    """The launch shapes bench.py times: its autotuner run on a throwaway
    instance of the same workload."""
    import torch

    from paper_1812_05711_amd import autotune
    from paper_1812_05711_amd.lbm_ec import Simulation

    sim = Simulation(device="cuda:0", precision=precision, **kw)
    tuning, _ = autotune.tune_single(sim, steps=8)
    torch.cuda.synchronize()
    sim.close()
    return tuning


@pytest.mark.parametrize("precision,tol", [("fp32_f64math", 1e-5), ("fp64", 1e-11)])
def test_cfg2_full_against_oracle(precision, tol):
    """4096 x 4096 after the workload's 1000 steps, in the precision mode the
    benchmark times and in FP64, each in the launch shapes the benchmark's
    autotuner picks: every field within the precision's tolerance."""
    gold = _cfg2(1000)
    tuning = _bench_tuning(precision, KW2)
    print(precision, "launch shapes", tuning, flush=True)
    res = _run(precision, [1000], KW2, tuning)
    _gate(gold, res, [1000], precision, tol, gate_u=True)
