"""Persistent cache of autotuned repulsion tables (fl_autotune).

A table depends on the device, the library build, the error bound and the
sizes it was measured at, so those form the key.  The cache is one JSON file:
``$FA2LAY_TUNE_CACHE`` if set, else ``~/.cache/fa2lay/tuning.json``.  Writes
go to a temporary file that is then renamed over the old one, so a reader
never sees a partial file.  Plain file handling: the measurement itself runs
in the library.
"""
from __future__ import annotations

import json
import os
import tempfile

ENV = "FA2LAY_TUNE_CACHE"


def cache_path() -> str:
    return os.environ.get(ENV) or os.path.join(os.path.expanduser("~"), ".cache", "fa2lay", "tuning.json")


def make_key(device: dict, version: str, max_rel_err: float, sizes) -> str:
    sz = ",".join(str(int(s)) for s in sizes)
    return (f"{device.get('name', '?')}|{device.get('arch', '?')}|cu{device.get('cus', '?')}|{version}|"
            f"err{max_rel_err:.3e}|{sz}")


def load_all(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return {}
    return data if isinstance(data, dict) else {}


def lookup(key: str, path: str | None = None) -> dict | None:
    e = load_all(path).get(key)
    if not isinstance(e, dict) or "tuning" not in e:
        return None
    t = e["tuning"]
    ok = all(k in t for k in ("fmm_min_nodes", "bucket_max", "p", "leaf_size"))
    return e if ok else None


def store(key: str, entry: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    data = load_all(path)
    data[key] = entry
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(os.path.abspath(path)), suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def device_identity(device_index: int = 0) -> dict:
    import torch
    pr = torch.cuda.get_device_properties(device_index)
    return {"name": pr.name, "arch": getattr(pr, "gcnArchName", "?"), "cus": pr.multi_processor_count}


def tuned(ctx, x, y, deg, sizes, max_rel_err: float = 1e-3, reps: int = 3, path: str | None = None,
          retune: bool = False) -> tuple[dict, bool]:
    """The tuning table for this device and bound: from the cache when present
    (unless ``retune``), else measured by ``ctx.autotune`` and stored.  The
    table is installed in ``ctx``.  Returns (table, came_from_cache)."""
    from . import fa2lay
    key = make_key(device_identity(ctx.device.index or 0), fa2lay.version(), max_rel_err, sizes)
    if not retune:
        e = lookup(key, path)
        if e is not None:
            ctx.set_tuning(e["tuning"])
            return e["tuning"], True
    table, samples = ctx.autotune(x, y, deg, sizes, max_rel_err, reps)
    store(key, {"tuning": table, "samples": samples, "reps": reps}, path)
    return table, False
