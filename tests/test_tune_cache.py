"""The autotuner's cache of walk launch shapes through the C ABI, without a GPU:
bh_tune_cache_load / save / clear / size on JSON files (round trip, merge, refusal of
malformed or missing files with the cache unchanged).  The cache's reader and writer are
host code; the timing itself is covered by the GPU tests."""
import json

import pytest

bh = pytest.importorskip("paper_1109_5190_amd")


def _entry(device="gfx950:256", n_log2=20, sims_log2=0, theta=0.5, precision="fp32", shape=4, ms=2.77):
    return dict(device=device, n_log2=n_log2, sims_log2=sims_log2, theta=theta, precision=precision,
                shape=shape, ms=ms)


def _write(path, entries, **top):
    doc = {"format": "bh-tune-cache", "version": 1, "entries": entries}
    doc.update(top)
    path.write_text(json.dumps(doc))


@pytest.fixture()
def clean():
    bh.tune_cache_clear()
    yield
    bh.tune_cache_clear()


def test_round_trip_and_merge(tmp_path, clean):
    a = tmp_path / "a.json"
    ents = [_entry(), _entry(n_log2=24, sims_log2=9, theta=0.53, precision="mixed", shape=1 | bh.WALK_PERSISTENT,
                             ms=48.7),
            _entry(device="gfx942:304", precision="fp64", shape=8, ms=4.1)]
    _write(a, ents)
    bh.tune_cache_load(a)
    assert bh.tune_cache_size() == 3
    b = tmp_path / "b.json"
    bh.tune_cache_save(b)
    doc = json.loads(b.read_text())
    assert doc["format"] == "bh-tune-cache" and doc["version"] == 1
    key = lambda e: (e["device"], e["n_log2"], e["sims_log2"], round(e["theta"], 2), e["precision"])
    got = {key(e): (e["shape"], e["ms"]) for e in doc["entries"]}
    assert got == {key(e): (e["shape"], pytest.approx(e["ms"], rel=1e-5)) for e in ents}
    # equal keys are replaced, new ones added
    _write(a, [_entry(shape=2, ms=2.5), _entry(n_log2=21)])
    bh.tune_cache_load(a)
    assert bh.tune_cache_size() == 4
    bh.tune_cache_save(b)
    got = {key(e): e["shape"] for e in json.loads(b.read_text())["entries"]}
    assert got[("gfx950:256", 20, 0, 0.5, "fp32")] == 2
    bh.tune_cache_clear()
    assert bh.tune_cache_size() == 0


@pytest.mark.parametrize("bad", [
    "", "{", "[]", "not json",
    json.dumps({"format": "bh-tune-cache", "version": 2, "entries": []}),
    json.dumps({"format": "bh-tune-cache", "version": 1, "entries": [_entry(shape=3)]}),
    json.dumps({"format": "bh-tune-cache", "version": 1, "entries": [_entry(shape=0x204)]}),
    json.dumps({"format": "bh-tune-cache", "version": 1, "entries": [_entry(shape=-4)]}),
    json.dumps({"format": "bh-tune-cache", "version": 1, "entries": [_entry(shape=-1e300)]}),
    json.dumps({"format": "bh-tune-cache", "version": 1, "entries": [_entry(precision="bf16")]}),
    json.dumps({"format": "bh-tune-cache", "version": 1, "entries": [_entry(ms=-1.0)]}),
    json.dumps({"format": "bh-tune-cache", "version": 1, "entries": [{**_entry(), "extra": 1}]}),
    json.dumps({"format": "bh-tune-cache", "version": 1, "entries": [_entry(), "x"]}),
])
def test_malformed_files_are_refused_whole(tmp_path, clean, bad):
    good = tmp_path / "good.json"
    _write(good, [_entry()])
    bh.tune_cache_load(good)
    p = tmp_path / "bad.json"
    p.write_text(bad)
    with pytest.raises(bh.BHError) as ei:
        bh.tune_cache_load(p)
    assert ei.value.status == bh.E_IO
    assert bh.tune_cache_size() == 1


def test_missing_and_unwritable_paths(tmp_path, clean):
    with pytest.raises(bh.BHError) as ei:
        bh.tune_cache_load(tmp_path / "absent.json")
    assert ei.value.status == bh.E_IO
    with pytest.raises(bh.BHError) as ei:
        bh.tune_cache_save(tmp_path / "no_such_dir" / "c.json")
    assert ei.value.status == bh.E_IO
    assert bh.lib().bh_tune_cache_load(None) == bh.E_INVAL
