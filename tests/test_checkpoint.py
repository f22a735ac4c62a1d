"""The sweep's per-map checkpoint file (CPU): records reload, a line cut short
by a crash is dropped and cut off the file, and appending continues cleanly."""
import json

from paper_1810_09784_amd.sweep import Checkpoint


def test_checkpoint_round_trip_and_torn_last_line(tmp_path):
    path = str(tmp_path / "sweep.jsonl")
    ck = Checkpoint(path)
    assert ck.done == {}
    recs = [{"key": [2.0 + 0.5 * i, 2.0, 100.0, 164.0, 5], "candidates": [[1, 2, 3, 0, 4.5]], "map_crc32": i}
            for i in range(3)]
    for r in recs:
        ck.write(r)
    with open(path, "a") as f:
        f.write('{"key": [9.0, 2.0, 100.0, 1')  # a record torn by a crash
    ck2 = Checkpoint(path)
    assert set(ck2.done) == {Checkpoint.key(*r["key"]) for r in recs}
    assert ck2.done[Checkpoint.key(2.5, 2, 100, 164, 5)]["map_crc32"] == 1
    with open(path) as f:
        assert f.read().endswith("}\n")  # the torn tail is gone
    ck2.write({"key": [9.0, 2.0, 100.0, 164.0, 5], "candidates": []})
    with open(path) as f:
        lines = [json.loads(x) for x in f.read().splitlines()]
    assert len(lines) == 4 and lines[-1]["key"][0] == 9.0
    # a garbled line stops the reload there (later lines are not trusted either)
    with open(path, "a") as f:
        f.write("not json\n")
        f.write(json.dumps({"key": [10.0, 2.0, 100.0, 164.0, 5]}) + "\n")
    ck3 = Checkpoint(path)
    assert len(ck3.done) == 4
