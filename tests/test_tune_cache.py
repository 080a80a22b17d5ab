"""The autotuner's schedule cache (host only): signatures and the JSON file."""

import json
import os

from paper_2009_07400_amd import tune_cache
from paper_2009_07400_amd.system import make_params

SCHED = {"block_threads": 640, "lds_atoms": 3328, "block_edge": 3, "block_parts": 1, "lanes_per_atom": 1,
         "build_threads": 512, "build_lanes": 1, "half_list": 0, "layout": 0}


def _key(**over):
    a = dict(device="AMD Instinct MI355X", library="0123456789abcdef", box_atoms=[4000, 256],
             box_lengths=[16.79596, 6.7183], params=[make_params(), make_params(epsilon=1.05)])
    adj = over.pop("for_adjoint", False)
    a.update(over)
    return tune_cache.system_key(a["device"], a["library"], a["box_atoms"], a["box_lengths"], a["params"], adj)


def test_key_is_stable_and_covers_every_input():
    k = _key()
    assert k == _key()
    changed = [_key(device="other"), _key(library="fedcba9876543210"), _key(box_atoms=[4000, 257]),
               _key(box_lengths=[16.79596, 6.7183000000000002e0 + 1e-12]),
               _key(params=[make_params(), make_params(epsilon=1.0500000001)]),
               _key(params=[make_params(), make_params(epsilon=1.05, max_neighbors=160)]),
               _key(box_atoms=[256, 4000], box_lengths=[6.7183, 16.79596]), _key(for_adjoint=True)]
    assert len({k, *changed}) == len(changed) + 1


def test_store_lookup_round_trip(tmp_path):
    p = str(tmp_path / "sub" / "tune.json")
    assert tune_cache.lookup(p, "k") is None
    tune_cache.store(p, "k", dict(SCHED, extra=7))
    assert tune_cache.lookup(p, "k") == SCHED
    tune_cache.store(p, "k2", dict(SCHED, block_edge=2))
    assert tune_cache.lookup(p, "k") == SCHED and tune_cache.lookup(p, "k2")["block_edge"] == 2
    # no temporary files left beside the cache
    assert sorted(os.listdir(tmp_path / "sub")) == ["tune.json"]
    data = json.load(open(p))
    assert data["version"] == tune_cache.VERSION and set(data["entries"]) == {"k", "k2"}


def test_unreadable_or_foreign_files_are_empty(tmp_path):
    p = tmp_path / "tune.json"
    p.write_text("{not json")
    assert tune_cache.load(str(p)) == {}
    p.write_text(json.dumps({"version": tune_cache.VERSION + 1, "entries": {"k": SCHED}}))
    assert tune_cache.lookup(str(p), "k") is None
    p.write_text(json.dumps({"version": tune_cache.VERSION, "entries": {"k": dict(SCHED, block_edge="3")}}))
    assert tune_cache.lookup(str(p), "k") is None
    # a store over a foreign file starts a fresh cache
    tune_cache.store(str(p), "k", SCHED)
    assert tune_cache.lookup(str(p), "k") == SCHED


def test_file_digest_tracks_content(tmp_path):
    p = tmp_path / "lib.so"
    p.write_bytes(b"a" * 10)
    d1 = tune_cache.file_digest(str(p))
    assert d1 == tune_cache.file_digest(str(p)) and len(d1) == 16
    p.write_bytes(b"b" * 11)
    assert tune_cache.file_digest(str(p)) != d1
