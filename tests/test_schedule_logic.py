"""Host-side rules of the launch schedules and of the autotuner's JSON cache
(no GPU: lm_schedule_candidates, lm_set_schedule and lm_get_schedule touch no
device; the cache is plain JSON)."""

import json
import os

import pytest

SIZES = (64, 128, 192, 256, 384, 512, 1024)


@pytest.fixture(scope="module")
def L():
    import paper_2208_02682_amd as lib
    from paper_2208_02682_amd.lagmean import LIB_PATH
    if not os.path.exists(LIB_PATH):
        from paper_2208_02682_amd.build import build
        build(verbose=False)
    yield lib
    for n in SIZES:
        for p in ("fp32", "fp64"):
            lib.set_schedule(n, p, 0, 1)
            lib.set_schedule(n, p, 0, 1, batched=True)


def _usable(n, w, cplx_bytes):
    # the rule stated in include/lagmean.h, from first principles: E values per
    # lane (12 for n = 3 * 2^k, else 16), base width 8 columns unless a transform
    # has fewer than 8 lanes (then 64 / lanes), whole wavefronts of at most 1024
    # threads, LDS (padded column buffers) within 160 KiB
    E = 12 if n % 3 == 0 else 16
    lanes = n // E
    base = 8 if lanes >= 8 else 64 // lanes
    C = {-1: base // 2, 0: base, 1: base * 2}[w]
    threads = C * lanes
    col = (n + n // 16 + 1) | 1
    return C >= 1 and threads >= 64 and threads % 64 == 0 and threads <= 1024 and C * col * cplx_bytes <= 160 * 1024


def test_candidates_follow_the_stated_rule(L):
    for n in SIZES:
        for p, cb in (("fp32", 8), ("fp64", 16)):
            c = L.schedule_candidates(n, p)
            assert c[0] == (0, 1, 1), (n, p)                   # the default first
            assert len(set(c)) == len(c)
            want = [(w, x, st) for st in (1, 2) for w in (0, -1, 1) if _usable(n, w, cb) for x in (1, 0)]
            assert c == want, (n, p, c)
    # the cases the rule singles out
    assert (1, 1, 1) not in L.schedule_candidates(1024, "fp64")  # 16 float64 columns need 278 KB of LDS
    assert (-1, 1, 1) not in L.schedule_candidates(64, "fp32")   # half a wavefront
    assert len(L.schedule_candidates(1024, "fp32")) == 12


def test_set_get_and_refusals(L):
    from paper_2208_02682_amd import LagMeanError
    assert L.get_schedule(256, "fp32") == (0, 1, 1)
    L.set_schedule(256, "fp32", -1, 0)
    assert L.get_schedule(256, "fp32") == (-1, 0, 1)
    L.set_schedule(256, "fp32", -1, 0, 2)
    assert L.get_schedule(256, "fp32") == (-1, 0, 2)
    assert L.get_schedule(256, "fp64") == (0, 1, 1)            # per precision
    with pytest.raises(LagMeanError) as e:
        L.set_schedule(1024, "fp64", 1, 1)
    assert e.value.status == -1
    with pytest.raises(LagMeanError) as e:
        L.set_schedule(256, "fp32", 0, 2)
    assert e.value.status == -1
    with pytest.raises(LagMeanError) as e:
        L.set_schedule(100, "fp32", 0, 1)
    assert e.value.status == -6
    with pytest.raises(LagMeanError) as e:
        L.set_schedule(256, "fp32", 0, 1, 3)
    assert e.value.status == -1
    L.set_schedule(256, "fp32", 0, 1)
    # the batched launches' table is separate, and takes one stream only
    L.set_schedule(256, "fp32", 1, 0, batched=True)
    assert L.get_schedule(256, "fp32", batched=True) == (1, 0, 1) and L.get_schedule(256, "fp32") == (0, 1, 1)
    with pytest.raises(LagMeanError):
        L.set_schedule(1024, "fp64", 1, 1, batched=True)
    with pytest.raises(LagMeanError):
        L.set_schedule(256, "fp32", 0, 1, 2, batched=True)
    L.set_schedule(256, "fp32", 0, 1, batched=True)
    lib = L.load_library()
    assert lib.lm_schedule_candidates(256, 1, None, 1, None) == -1   # cap > 0 with no array
    assert lib.lm_autotune(None, 8, 3, None, None, 0, None) == -1
    assert lib.lm_batch_autotune(None, 4, 3, None) == -1


def test_json_cache_round_trip_and_merge(L, tmp_path):
    from paper_2208_02682_amd import autotune as at
    path = str(tmp_path / "s.json")
    t1 = [{"n": 256, "precision": "fp32", "best": (-1, 0, 2), "ms": {(0, 1, 1): 0.2, (0, 0, 1): 0.21,
                                                                    (-1, 1, 1): 0.19, (-1, 0, 2): 0.18,
                                                                    (1, 1, 1): 0.25, (1, 0, 1): 0.26}}]
    t2 = [{"n": 512, "precision": "fp64", "best": (0, 0, 1), "ms": {(0, 1, 1): 1.0, (0, 0, 1): 0.9}}]
    at.merge_save(path, "gfx950", t1)
    at.merge_save(path, "gfx950", t2)                          # keeps the 256 entry
    doc = json.load(open(path))
    assert doc["arch"] == "gfx950" and [(e["n"], e["precision"]) for e in doc["entries"]] == [(256, "fp32"),
                                                                                             (512, "fp64")]
    assert doc["entries"][0]["ms_per_step"]["-1,0,2"] == 0.18
    assert L.load_schedules(path, "gfx942") == 0               # another architecture: nothing applied
    assert L.get_schedule(256, "fp32") == (0, 1, 1)
    assert L.load_schedules(path, "gfx950") == 2
    assert L.get_schedule(256, "fp32") == (-1, 0, 2) and L.get_schedule(512, "fp64") == (0, 0, 1)
    # a re-tune of one entry replaces it; batched entries are kept apart
    at.merge_save(path, "gfx950", [dict(t1[0], best=(0, 1, 1))])
    at.merge_save(path, "gfx950", [{"context": "batched", "n": 256, "precision": "fp32", "best": (1, 1, 1)}])
    got = {(e["context"], e["n"], e["precision"]): (e["col_tile"], e["xcd_order"], e["streams"])
           for e in json.load(open(path))["entries"]}
    assert got == {("single", 256, "fp32"): (0, 1, 1), ("single", 512, "fp64"): (0, 0, 1),
                   ("batched", 256, "fp32"): (1, 1, 1)}
    assert L.load_schedules(path, "gfx950") == 3
    assert L.get_schedule(256, "fp32", batched=True) == (1, 1, 1) and L.get_schedule(256, "fp32") == (0, 1, 1)
    # entries written before the streams field existed read as one stream
    doc = json.load(open(path))
    for e in doc["entries"]:
        e.pop("streams")
    json.dump(doc, open(path, "w"))
    assert L.load_schedules(path, "gfx950") == 3 and L.get_schedule(512, "fp64") == (0, 0, 1)


def test_shipped_cache_is_well_formed(L):
    from paper_2208_02682_amd import autotune as at
    path = at.cache_path("gfx950")
    if not os.path.exists(path):
        pytest.skip("no shipped cache")
    doc = json.load(open(path))
    assert doc["format"] == 1 and doc["arch"] == "gfx950"
    for e in doc["entries"]:
        assert e.get("context", "single") in ("single", "batched")
        key = (e["col_tile"], e["xcd_order"], e.get("streams", 1))
        assert key in L.schedule_candidates(e["n"], e["precision"])
        # the chosen schedule is the fastest measured one (where times were recorded)
        if e["ms_per_step"]:
            best = min(e["ms_per_step"], key=e["ms_per_step"].get)
            assert best in (",".join(str(x) for x in key), ",".join(str(x) for x in key[:2]))
