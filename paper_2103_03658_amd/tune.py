"""Launch-schedule tuner for the transform passes.

For a given operator shape (d, M), batch size and precision, times candidate
schedules with fl_profile_apply (HIP events around each kernel) and keeps the
fastest.  The passes are timed separately, so each pass group is tuned on its
own: the axis-0 pair (first and last pass share E_first, W_first), the
middle pass (E_mid, LPB_mid) and, in 3D, the axis-1 pair (E_c2c, W_c2c).
The preconditioner's passes (fl_profile_precond) get a schedule of their own
the same way.  Results are cached in a JSON file (FL_SCHEDULE_CACHE, default
~/.cache/fl_schedules.json) keyed by d, M, precision, batch size and
preconditioner kind.
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
    pc = getattr(op, "precond_kind", 2)
    ms = "x".join(str(m) for m in getattr(op, "Ms", (op.M,) * op.d))
    return f"d{op.d}-M{ms}-{'f32' if fp32 else 'f64'}-r{nrhs}-pc{pc}"


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


def _tune_passes(op, u, y, fp32, reps, verbose, precond):
    """Tune one schedule (the product's, or the preconditioner's) group by
    group; the candidates within 25% of the fastest are timed in a second
    round and their best time kept, so that one slow measurement (clock ramp,
    a neighbour's traffic) does not decide."""
    setter = lambda **kw: op.set_schedule(fp32, precond=precond, **kw)
    prof = op.profile_precond if precond else op.profile_apply
    best = dict(op.get_schedule(fp32, precond=precond))
    cands = candidates(op.M, fp32)
    groups = [("e_first", "w_first", [0, -1])]
    if op.d >= 2:
        groups.append(("e_mid", "lpb_mid", [1 if op.d == 2 else 2]))
    if op.d == 3:
        groups.append(("e_c2c", "w_c2c", [1, 3]))
    if op.d == 1:
        groups = [("e_mid", "lpb_mid", [0])]
        cands = [(E, 1) for E in (8, 16, 32) if E <= op.M]
    for ek, wk, idx in groups:
        times = {}
        for rnd in range(2):
            cut = 1.25 * min(times.values()) if times else None
            for E, W in cands:
                if rnd and ((E, W) not in times or times[(E, W)] > cut):
                    continue
                trial = dict(best)
                trial[ek], trial[wk] = E, W
                try:
                    setter(**trial)
                    if rnd == 0:
                        prof(u, out=y, reps=2)          # warm
                    ms = prof(u, out=y, reps=reps)
                except Exception as exc:  # schedule rejected
                    if verbose:
                        print("skip", trial, exc)
                    continue
                t = sum(ms[i] for i in idx)
                times[(E, W)] = min(t, times.get((E, W), t))
                if verbose:
                    print("pc" if precond else "A", ek, E, wk, W, f"{t * 1e3:.1f} us")
        if times:
            (E, W), _ = min(times.items(), key=lambda kv: kv[1])
            best[ek], best[wk] = E, W
    setter(**best)
    return best, prof(u, out=y, reps=reps)


def tune(op, nrhs, fp32, reps=10, use_cache=True, verbose=False):
    """Choose and apply the fastest schedules of the product's passes and,
    unless the operator runs plain CG, of its preconditioner's passes.
    Returns (schedule dict, ms per pass) of the product."""
    import torch
    db = _load() if use_cache else {}
    k = key(op, nrhs, fp32)
    pc = getattr(op, "precond_kind", 2)
    if k in db:
        ent = db[k]
        op.set_schedule(fp32, **ent["schedule"])
        if pc and "precond_schedule" in ent:
            op.set_schedule(fp32, precond=True, **ent["precond_schedule"])
        return ent["schedule"], ent["ms"]
    dt = torch.float32 if fp32 else torch.float64
    u = torch.randn(nrhs * op.nd, dtype=dt, device="cuda")
    y = torch.empty_like(u)
    best, ms = _tune_passes(op, u, y, fp32, reps, verbose, False)
    ent = {"schedule": best, "ms": ms}
    if pc:
        bp, mp = _tune_passes(op, u, y, fp32, reps, verbose, True)
        ent.update(precond_schedule=bp, precond_ms=mp)
    if use_cache:
        db = _load()
        db[k] = ent
        _store(db)
    return best, ms
