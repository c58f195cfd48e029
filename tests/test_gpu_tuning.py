"""The autotuner's cache on disk (hs_context_load_tuning / _save_tuning and
HS_TUNE_CACHE): JSON entries keyed by the gfx architecture and the batch's
size class, read back into a fresh context so that an autotuned plan takes
the stored shape without timing candidates; malformed files are refused
with the cache unchanged."""
import json
import os

import numpy as np
import pytest
import torch

from paper_2505_06703_amd import hs
from paper_2505_06703_amd import workloads as wl

pytestmark = pytest.mark.gpu


def batch():
    return wl.heterogeneous(num_characters=200, seed=12)


def test_save_then_load_gives_the_stored_shape(tmp_path):
    b = batch()
    a = hs.Context(0)
    tuned = hs.Plan(b.offsets, b.parents, ctx=a, autotune=True)
    path = tmp_path / "tune.json"
    a.save_tuning(path)
    data = json.loads(path.read_text())
    assert data["version"] == 1 and len(data["entries"]) == 1
    (key, shape), = data["entries"].items()
    assert key.startswith("gfx950|")
    assert set(shape) == {"tile_cap", "waves", "grid_per_cu", "chain_units", "queue_waves"}
    assert tuned.info["tile_joints"] == shape["tile_cap"]
    # an unusual but valid shape under the same key: a fresh context that
    # loads it must build exactly that shape instead of timing candidates
    data["entries"][key] = {"tile_cap": 2048, "waves": 8, "grid_per_cu": 0, "chain_units": 0, "queue_waves": 2}
    path.write_text(json.dumps(data))
    c = hs.Context(0)
    c.load_tuning(path)
    p = hs.Plan(b.offsets, b.parents, ctx=c, autotune=True)
    assert p.info["tile_joints"] == 2048 and p.info["waves_per_tile"] == 2
    assert p.info["schedule"] == hs.HS_SCHED_QUEUE
    # the resident workgroups looping over the tiles (grid_per_cu > 0)
    data["entries"][key]["grid_per_cu"] = 1
    path.write_text(json.dumps(data))
    d = hs.Context(0)
    d.load_tuning(path)
    p2 = hs.Plan(b.offsets, b.parents, ctx=d, autotune=True)
    assert p.info["grid"] == p.info["num_tiles"]  # grid_per_cu 0: one workgroup per tile
    assert p2.info["grid"] == min(p2.info["num_tiles"], torch.cuda.get_device_properties(0).multi_processor_count)
    q, t, s = (torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0") for x in (b.quat, b.trans, b.scale))
    G1, _ = hs.hs_scan_forward(p, q, t, s)
    G2, _ = hs.hs_scan_forward(p2, q, t, s)
    torch.cuda.synchronize()
    assert torch.equal(G1, G2)  # the same tiles, whichever workgroup takes them
    tuned.close(), p.close(), p2.close()
    a.close(), c.close(), d.close()


def test_missing_and_malformed_files(tmp_path):
    c = hs.Context(0)
    c.load_tuning(tmp_path / "absent.json")  # nothing tuned yet: fine
    for text in ("", "{", '{"entries": {"k": {"waves": 8}}}', '{"entries": {"k": {"tile_cap": 100, "waves": 8}}}',
                 '{"entries": {"k": {"tile_cap": 1024, "waves": 3}}}', '{"entries": []}', "[1, 2]",
                 '{"entries": {"k": {"tile_cap": 1024, "waves": 8}}} trailing'):
        bad = tmp_path / "bad.json"
        bad.write_text(text)
        with pytest.raises(hs.HSError) as ei:
            c.load_tuning(bad)
        assert ei.value.status == hs.HS_ERR_INVALID_ARG, text
    out = tmp_path / "empty.json"
    c.save_tuning(out)  # the refused files left the cache empty
    assert json.loads(out.read_text()) == {"version": 1, "entries": {}}
    # unknown members are skipped
    ok = tmp_path / "ok.json"
    ok.write_text('{"version": 1, "note": {"a": [1, {"b": "x"}]}, "entries": '
                  '{"gfx950|x": {"tile_cap": 1024, "waves": 8, "extra": "y"}}}')
    c.load_tuning(ok)
    c.save_tuning(out)
    assert json.loads(out.read_text())["entries"] == {
        "gfx950|x": {"tile_cap": 1024, "waves": 8, "grid_per_cu": 0, "chain_units": 0, "queue_waves": 0}}
    c.close()


def test_environment_variable_persists_every_tuning(tmp_path, monkeypatch):
    path = tmp_path / "env_tune.json"
    monkeypatch.setenv("HS_TUNE_CACHE", str(path))
    c = hs.Context(0)
    b = batch()
    p = hs.Plan(b.offsets, b.parents, ctx=c, autotune=True)
    assert path.exists()
    entries = json.loads(path.read_text())["entries"]
    assert len(entries) == 1 and next(iter(entries.values()))["tile_cap"] == p.info["tile_joints"]
    p.close()
    c.close()
    c2 = hs.Context(0)  # loads the file at creation
    out = tmp_path / "copy.json"
    c2.save_tuning(out)
    assert json.loads(out.read_text())["entries"] == entries
    c2.close()
