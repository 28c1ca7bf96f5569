"""Autotuner for the launch shapes of the time step (they never change
results): threads per x-transform block, threads per collide tile and, for
rows wider than 512, columns per collide tile (whole rows or tiles of 1024 or
512 columns that recompute their halo columns).

Candidates are timed with events on the batch's stream, on a throwaway batch
of the same composition (so the real run is not advanced), and the best is
cached in a JSON file keyed by the precision and the multiset of grid shapes.
"""

import hashlib
import json
import os

FFT_THREADS = (64, 128, 256, 512)
COLLIDE_SHAPES = ((64, 1), (128, 1), (256, 1), (512, 1), (1024, 1))
TILE_WIDTHS = (0, 1024, 512)  # 0: the library's default width
BATCH_TILE_WIDTHS = (0, 128, 64)  # batches: whole rows, or narrower tiles for more blocks per slot
DEFAULT = (256, 256, 1)


def cache_path():
    return os.environ.get("LBM_EC_TUNING_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "lbm_ec_tuning.json"))


def signature(configs):
    shapes = sorted((c["nx"], c["ny"]) for c in configs)
    key = json.dumps([configs[0].get("precision", "fp64"), shapes])
    return hashlib.sha256(key.encode()).hexdigest()[:24]


def _load():
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except Exception:
        return {}


def _store(cache):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, path)
    except OSError:
        pass


BATCH_REPS = 2  # timings per candidate (the best one counts): single short timings picked noise


def _time_batch(b, steps, reps=BATCH_REPS):
    import torch

    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    b.step(8)  # capture and warm up
    best = float("inf")
    for _ in range(reps):
        start.record(b.stream)
        b.step(steps)
        end.record(b.stream)
        end.synchronize()
        best = min(best, start.elapsed_time(end) / steps)
    return best


def tune_batch(configs, device="cuda:0", steps=64, use_cache=True):
    """Best (fft_threads, collide_bx, collide_by, collide_tw) for this batch
    composition: the transform threads, then the collide block shape, then
    the collide tile width (each at the best of the earlier ones)."""
    from .sweep import make_batch

    sig = signature(configs)
    cache = _load() if use_cache else {}
    if sig in cache:
        return tuple(cache[sig]["tuning"])
    # enough steps for every candidate; the throwaway batch is never polled
    n_cand = len(FFT_THREADS) + len(COLLIDE_SHAPES) + len(BATCH_TILE_WIDTHS)
    b, _ = make_batch(configs, steps=(BATCH_REPS * steps + 8) * n_cand + 8, emit_every=0, device=device)
    best_fft, best_t = DEFAULT[0], float("inf")
    for ft in FFT_THREADS:
        b.set_tuning(ft, DEFAULT[1], DEFAULT[2])
        try:
            t = _time_batch(b, steps)
        except Exception:  # a transform block too small for the widest slot
            continue
        if t < best_t:
            best_fft, best_t = ft, t
    best_shape, best_t = DEFAULT[1:], float("inf")
    for bx, by in COLLIDE_SHAPES:
        b.set_tuning(best_fft, bx, by)
        t = _time_batch(b, steps)
        if t < best_t:
            best_shape, best_t = (bx, by), t
    best_tw = 0
    for tw in BATCH_TILE_WIDTHS[1:]:
        b.set_tuning(best_fft, best_shape[0], best_shape[1], tw)
        t = _time_batch(b, steps)
        if t < best_t:
            best_tw, best_t = tw, t
    b.close()
    tuning = (best_fft, best_shape[0], best_shape[1], best_tw)
    cache[sig] = {"tuning": list(tuning), "ms_per_step": best_t}
    if use_cache:
        _store(cache)
    return tuning


def tune_single(sim, steps=16):
    """Best launch shapes (fft_threads, collide_bx, collide_by, collide_tw)
    for one simulation (advances it by the timing steps).  Shapes the library
    refuses (a transform block too small for the row) are skipped."""
    import torch

    from .lbm_ec import LbmEcError

    widths = [w for w in TILE_WIDTHS if w == 0 or w < sim.nx]
    best, best_t = DEFAULT + (0,), float("inf")
    for ft in FFT_THREADS:
        for (bx, by), tw in [(s, w) for s in COLLIDE_SHAPES for w in widths]:
            try:
                sim.set_tuning(ft, bx, by, tw)
            except LbmEcError:
                continue
            sim.step(2)
            start = torch.cuda.Event(enable_timing=True)
            end = torch.cuda.Event(enable_timing=True)
            start.record(sim.stream)
            sim.step(steps)
            end.record(sim.stream)
            end.synchronize()
            t = start.elapsed_time(end) / steps
            if t < best_t:
                best, best_t = (ft, bx, by, tw), t
    sim.set_tuning(*best)
    return best, best_t
