"""Persistent cache of autotuned schedules, one JSON file.

An entry maps a system's signature to the schedule the autotuner picked for
it.  The signature covers what the choice depends on: the device, the
library build (a digest of the shared object, so a rebuilt kernel never
inherits an old pick) and the system's shape (atoms and box length of every
box, and every box's parameters).  Writes replace the file atomically, so a
reader never sees a half-written cache.
"""

from __future__ import annotations

import hashlib
import json
import os
import tempfile
from typing import Optional, Sequence

VERSION = 1

# tmd_info fields that make up a schedule, as tmd_set_schedule takes them
SCHEDULE_KEYS = ("block_threads", "lds_atoms", "block_edge", "block_parts", "lanes_per_atom", "build_threads",
                 "build_lanes", "half_list", "layout")

_PARAM_FIELDS = ("epsilon", "sigma", "mass", "cutoff", "skin", "dt", "rebuild_every", "max_neighbors")

_digests: dict = {}


def file_digest(path: str) -> str:
    """SHA-256 prefix of a file's bytes (memoised per path and mtime)."""
    st = os.stat(path)
    k = (path, st.st_mtime_ns, st.st_size)
    if k not in _digests:
        h = hashlib.sha256()
        with open(path, "rb") as f:
            for block in iter(lambda: f.read(1 << 20), b""):
                h.update(block)
        _digests[k] = h.hexdigest()[:16]
    return _digests[k]


def system_key(device: str, library: str, box_atoms: Sequence[int], box_lengths: Sequence[float],
               params: Sequence, for_adjoint: bool = False) -> str:
    """Signature of a system: device name, library digest, per-box atom
    counts, box lengths (exact, as repr), parameters, and whether the
    schedule is for the adjoint."""
    sig = {
        "adjoint": bool(for_adjoint),
        "device": device,
        "library": library,
        "atoms": [int(n) for n in box_atoms],
        "lengths": [repr(float(v)) for v in box_lengths],
        "params": [[repr(getattr(p, f)) for f in _PARAM_FIELDS] for p in params],
    }
    return hashlib.sha256(json.dumps(sig, sort_keys=True).encode()).hexdigest()[:32]


def load(path: str) -> dict:
    """The cache's entries; an absent, unreadable or other-version file is empty."""
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return {}
    if not isinstance(data, dict) or data.get("version") != VERSION or not isinstance(data.get("entries"), dict):
        return {}
    return data["entries"]


def lookup(path: str, key: str) -> Optional[dict]:
    e = load(path).get(key)
    if not isinstance(e, dict) or any(not isinstance(e.get(k), int) for k in SCHEDULE_KEYS):
        return None
    return {k: e[k] for k in SCHEDULE_KEYS}


def store(path: str, key: str, schedule: dict) -> None:
    entries = load(path)
    entries[key] = {k: int(schedule[k]) for k in SCHEDULE_KEYS}
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(prefix=".tune_cache.", suffix=".json", dir=d)
    try:
        with os.fdopen(fd, "w") as f:
            json.dump({"version": VERSION, "entries": entries}, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except BaseException:
        if os.path.exists(tmp):
            os.unlink(tmp)
        raise
