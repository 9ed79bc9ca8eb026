"""Launch-schedule tuner for the transform passes.

For a given operator shape (d, M), batch size and precision, times candidate
schedules with fl_profile_apply (HIP events around each kernel) and keeps the
fastest.  The passes are timed separately, so each pass group is tuned on its
own: the axis-0 pair (first and last pass share E_first, W_first), the
middle pass (E_mid, LPB_mid) and, in 3D, the axis-1 pair (E_c2c, W_c2c).
Results are cached in a JSON file (FL_SCHEDULE_CACHE, default
~/.cache/fl_schedules.json) keyed by d, M, precision and batch size.
"""

import json
import os

KEYS = ["e_first", "e_mid", "e_c2c", "w_first", "w_c2c", "lpb_mid"]


def cache_path():
    return os.environ.get("FL_SCHEDULE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "fl_schedules.json"))


def _load():
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except Exception:
        return {}


def _store(db):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(db, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def key(op, nrhs, fp32):
    return f"d{op.d}-M{op.M}-{'f32' if fp32 else 'f64'}-r{nrhs}"


def _lds_ok(M, E, W, fp32):
    return W * (M // E) <= 512 and W * 2 * (M + M // E) * (4 if fp32 else 8) <= 159 * 1024


def candidates(M, fp32):
    out = []
    for E in (8, 16, 32):
        if E > M:
            continue
        for W in (1, 2, 4, 8, 16):
            if _lds_ok(M, E, W, fp32):
                out.append((E, W))
    return out


def tune(op, nrhs, fp32, reps=10, use_cache=True, verbose=False):
    """Choose and apply the fastest schedule; returns (schedule dict, ms per pass)."""
    import torch
    db = _load() if use_cache else {}
    k = key(op, nrhs, fp32)
    if k in db:
        sch = db[k]["schedule"]
        op.set_schedule(fp32, **sch)
        return sch, db[k]["ms"]
    dt = torch.float32 if fp32 else torch.float64
    u = torch.randn(nrhs * op.nd, dtype=dt, device="cuda")
    y = torch.empty_like(u)
    base = op.get_schedule(fp32)
    cands = candidates(op.M, fp32)
    groups = [("e_first", "w_first", [0, -1])]
    if op.d >= 2:
        groups.append(("e_mid", "lpb_mid", [1 if op.d == 2 else 2]))
    if op.d == 3:
        groups.append(("e_c2c", "w_c2c", [1, 3]))
    if op.d == 1:
        groups = [("e_mid", "lpb_mid", [0])]
        cands = [(E, 1) for E in (8, 16, 32) if E <= op.M]
    best = dict(base)
    for ek, wk, idx in groups:
        results = []
        for E, W in cands:
            trial = dict(best)
            trial[ek], trial[wk] = E, W
            try:
                op.set_schedule(fp32, **trial)
                op.profile_apply(u, out=y, reps=2)          # warm
                ms = op.profile_apply(u, out=y, reps=reps)
            except Exception as exc:  # schedule rejected
                if verbose:
                    print("skip", trial, exc)
                continue
            t = sum(ms[i] for i in idx)
            results.append((t, E, W))
            if verbose:
                print(ek, E, wk, W, f"{t * 1e3:.1f} us")
        if results:
            t, E, W = min(results)
            best[ek], best[wk] = E, W
    op.set_schedule(fp32, **best)
    ms = op.profile_apply(u, out=y, reps=reps)
    if use_cache:
        db = _load()
        db[k] = {"schedule": best, "ms": ms}
        _store(db)
    return best, ms
