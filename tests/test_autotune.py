"""Host logic of the autotuner: shape classes, candidate sets, the JSON cache
(CPU only; the measurements themselves run in the GPU tests)."""

import json

from paper_2208_08410_amd import autotune as T


def test_dense_class_buckets_and_sides():
    assert T.dense_class(200000, 4096, "bf16x3") == "dense/bf16x3/R/d4096/K262144"
    assert T.dense_class(150000, 4000, "bf16x3") == T.dense_class(200000, 4096, "bf16x3")
    assert T.dense_class(300, 1000, "fp32") == "dense/fp32/L/d512/K1024"
    # the printed branch (m > n) sends a square problem to the left Gram
    assert T.dense_class(500, 500, "fp32", branch=1).startswith("dense/fp32/L/")
    assert T.dense_class(500, 500, "fp32", branch=0).startswith("dense/fp32/R/")


def test_batch_class():
    assert T.batch_class([(1000, 100), (50, 3000)]) == "batch/c2/d128"
    assert T.batch_class([(10, 10)] * 33) == "batch/c64/d16"


def test_gram_candidates_are_valid_tunings():
    c = T.gram_candidates("bf16x3", 4096, 200000, 256)
    assert {t for t, _ in c} == {128, 256}
    assert all(0 <= s <= 4096 for _, s in c)
    assert (256, 0) in c and (128, 0) in c
    # FP32 has one tile size; chunk counts never exceed K / 256
    c = T.gram_candidates("fp32", 512, 1024, 256)
    assert {t for t, _ in c} == {0}
    assert max(s for _, s in c) <= 4


def test_power_candidates_keep_four_rows_per_workgroup():
    assert T.power_candidates(4096, 256) == [0, 64, 128, 192]
    assert T.power_candidates(300, 256) == [0, 64]
    assert T.power_candidates(16, 256) == [0]


class FakeCtx:
    num_cu = 256


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tuning.json")
    t = T.Tuner(FakeCtx(), path)
    assert t.lookup("dense/bf16x3/R/d4096/K262144") is None
    t._record("dense/bf16x3/R/d4096/K262144", {"gram_tile": 256, "gram_chunks": 0, "power_blocks": 0}, 12.5, [])
    t.save()
    data = json.load(open(path))
    assert data["dense/bf16x3/R/d4096/K262144"]["tuning"]["gram_tile"] == 256
    t2 = T.Tuner(FakeCtx(), path)
    assert t2.lookup("dense/bf16x3/R/d4096/K262144") == {"gram_tile": 256, "gram_chunks": 0, "power_blocks": 0}


def test_gram_unit_candidates_and_class_table(tmp_path):
    """Per-class batched Gram units: both tile edges, chunk lengths up to
    twice the class's longest contraction; the stored classes come back as
    the group_tile / group_kchunk_cls tuning arrays (0 for untuned classes)."""
    import paper_2208_08410_amd as P
    c = T.gram_unit_candidates(300)
    assert c == [(64, 512), (128, 512)]
    c = T.gram_unit_candidates(65536)
    assert {t for t, _ in c} == {64, 128} and max(kc for _, kc in c) == 8192
    assert T.gram_unit_key(3) == "gram_unit/c3"
    t = T.Tuner(FakeCtx(), str(tmp_path / "t.json"))
    empty = t.class_tuning()
    assert empty == {"group_tile": [0] * P.GRAM_CLASSES, "group_kchunk_cls": [0] * P.GRAM_CLASSES}
    t._record(T.gram_unit_key(1), {"group_tile": 64, "group_kchunk": 1024}, 1.0, [])
    t._record(T.gram_unit_key(5), {"group_tile": 128, "group_kchunk": 4096}, 1.0, [])
    ct = t.class_tuning()
    assert ct["group_tile"][1] == 64 and ct["group_kchunk_cls"][1] == 1024
    assert ct["group_tile"][5] == 128 and ct["group_kchunk_cls"][5] == 4096
    assert sum(1 for v in ct["group_tile"] if v) == 2
