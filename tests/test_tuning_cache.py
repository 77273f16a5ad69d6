"""Host logic of the autotuner's persistent cache (paper_1807_08848_amd.tuning):
a miss runs the (native) tuner once and stores its choice under the device and
problem signature; a hit sets the stored shapes without tuning.  The problem is
a stand-in object here, so no device is needed."""
import json

import pytest


class _Desc:
    def __init__(self, n_cells):
        self.kind, self.n_cells, self.M, self.n_samples, self.rank = 0, n_cells, 4, 10, 6
        self.precision, self.n_vel = 1, 0
        self.overlap = [8] * 16


class _Layout:
    n_patches = 16


class _FakeProblem:
    def __init__(self, n_cells=128):
        self.desc = _Desc(n_cells)
        self.values = {}
        self.autotune_calls = 0

    def layout(self):
        return _Layout()

    def set_tuning(self, k, v):
        self.values[k] = v

    def get_tuning(self, k):
        return self.values.get(k, 0)

    def autotune(self, stage, reps):
        from paper_1807_08848_amd import msrs
        self.autotune_calls += 1
        if stage == msrs.TUNE_STAGE_OFFLINE:
            self.values[msrs.TUNE_SWEEP_COLS] = 32
            return [(0, 16, 3.0), (0, 32, 2.0), (0, 64, 2.5)]
        self.values[msrs.TUNE_RECON_BATCH] = 16
        self.values[msrs.TUNE_APPLY_BATCH] = 8
        return [(102, 1608, 1.0)]


def test_cache_miss_tunes_and_hit_reuses(tmp_path):
    from paper_1807_08848_amd import msrs, tuning
    path = str(tmp_path / "tuning.json")
    pr = _FakeProblem()
    r1 = tuning.tune(pr, msrs.TUNE_STAGE_OFFLINE, path=path)
    assert r1["source"] == "tuned" and r1["values"] == {"sweep_cols": 32} and pr.autotune_calls == 1
    db = json.load(open(path))
    assert len(db) == 1
    pr2 = _FakeProblem()
    r2 = tuning.tune(pr2, msrs.TUNE_STAGE_OFFLINE, path=path)
    assert r2["source"] == "cache" and pr2.autotune_calls == 0
    assert pr2.values == {msrs.TUNE_SWEEP_COLS: 32}
    # another stage and another problem shape are separate entries
    r3 = tuning.tune(pr2, msrs.TUNE_STAGE_ONLINE, path=path)
    assert r3["source"] == "tuned" and r3["values"] == {"recon_batch": 16, "apply_batch": 8}
    pr3 = _FakeProblem(n_cells=256)
    assert tuning.tune(pr3, msrs.TUNE_STAGE_OFFLINE, path=path)["source"] == "tuned"
    assert len(json.load(open(path))) == 3
    # force re-tunes a cached entry
    assert tuning.tune(pr2, msrs.TUNE_STAGE_OFFLINE, path=path, force=True)["source"] == "tuned"


def test_unwritable_cache_still_tunes(tmp_path):
    from paper_1807_08848_amd import msrs, tuning
    bad = str(tmp_path / "file_not_dir")
    open(bad, "w").write("x")
    pr = _FakeProblem()
    r = tuning.tune(pr, msrs.TUNE_STAGE_OFFLINE, path=bad + "/tuning.json")
    assert r["source"] == "tuned" and pr.values


def test_signature_depends_on_shape():
    from paper_1807_08848_amd import msrs, tuning
    a, b = _FakeProblem(128), _FakeProblem(256)
    assert tuning.signature(a, msrs.TUNE_STAGE_OFFLINE) != tuning.signature(b, msrs.TUNE_STAGE_OFFLINE)
    assert tuning.signature(a, msrs.TUNE_STAGE_OFFLINE) != tuning.signature(a, msrs.TUNE_STAGE_ONLINE)
