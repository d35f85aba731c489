"""CPU checks of the tuning table's host side: key validation, the JSON cache
(read and written per architecture) and the report.  No device work."""

import json

import pytest

import paper_1705_04601_amd as P


@pytest.fixture(autouse=True)
def _fresh_table():
    P.h2_tune_clear()
    yield
    P.h2_tune_clear()


def test_set_get_and_clear():
    assert P.h2_tune_get("gemm.f32.solve.a1b0.m3") is None
    P.h2_tune_set("gemm.f32.solve.a1b0.m3", 3)
    P.h2_tune_set("schur.split_k", 1024)
    assert P.h2_tune_get("gemm.f32.solve.a1b0.m3") == 3
    assert P.h2_tune_get("schur.split_k") == 1024
    P.h2_tune_clear()
    assert P.h2_tune_get("gemm.f32.solve.a1b0.m3") is None


@pytest.mark.parametrize("key,value", [
    ("gemm.f32.solve.a1b0.m3", 6),      # no seventh variant
    ("gemm.f64.solve.a1b0.m3", 3),      # 64 x 64 is not built for the FP64 solve
    ("gemm.f64.matvec.a1b2.m3", 4),     # no fifth matvec variant
    ("gemm.f32.solve.a0b0.m3", 0),      # no solve kernel for this layout
    ("gemm.f32.solver.a1b0.m3", 0),     # unknown role
    ("gemm.f32.solve.a1b0.m4", 0),      # unknown bucket
    ("gemm.f16.solve.a1b0.m3", 0),      # unknown precision
    ("schur.split_k", 8),               # below range
    ("schur.key_z", 2),
    ("schur.split_big", -1),
    ("solve.transpose", 2),
    ("no.such.key", 1),
])
def test_rejects_bad_entries(key, value):
    with pytest.raises(P.H2Error) as e:
        P.h2_tune_set(key, value)
    assert e.value.code == P.H2_EINVAL


def test_save_load_round_trip_keeps_other_architectures(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"gfx999": {"schur.split_k": 256}}))
    P.h2_tune_set("gemm.f32.factor.a0b0.m1", 2)
    P.h2_tune_set("schur.key_z", 1)
    P.h2_tune_save(str(path))
    data = json.loads(path.read_text())
    assert data["gfx999"] == {"schur.split_k": 256}
    mine = [v for k, v in data.items() if k != "gfx999"]
    assert mine == [{"gemm.f32.factor.a0b0.m1": 2, "schur.key_z": 1}]
    P.h2_tune_clear()
    P.h2_tune_load(str(path))
    assert P.h2_tune_get("gemm.f32.factor.a0b0.m1") == 2
    assert P.h2_tune_report()["source"] == str(path)


@pytest.mark.parametrize("text", ['{"x": {"schur.split_k": "a"}}', '{"x": [1]}', '{', '{"x": {}} trailing'])
def test_malformed_cache_is_an_error(tmp_path, text):
    path = tmp_path / "bad.json"
    path.write_text(text)
    with pytest.raises(P.H2Error):
        P.h2_tune_load(str(path))


def test_cache_naming_an_unbuilt_variant_is_an_error(tmp_path):
    arch = P.h2_tune_report()["arch"]
    path = tmp_path / "t.json"
    path.write_text(json.dumps({arch: {"gemm.f64.solve.a1b1.m3": 3}}))
    with pytest.raises(P.H2Error):
        P.h2_tune_load(str(path))


def test_report_shape():
    rep = P.h2_tune_report()
    assert set(rep) == {"arch", "source", "used"} and rep["source"] == "defaults"
