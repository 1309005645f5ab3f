"""Host logic of the counter store (no GPU): the copy-kernel scaling of
FETCH_SIZE / WRITE_SIZE, the step-level byte sum, the EK instruction count, and
the source-hash gating that keeps stale counters out of the bench line.  The
counter databases are small SQLite files with the columns of rocprofv3's
counters_collection table."""
import json
import sqlite3

import pytest

from paper_1607_04572_amd import counters as C


def make_db(path, rows):
    """rows: (kernel_name, dispatch_id, counter_name, value); several rows of one
    dispatch are the counter's instances (summed per dispatch)."""
    c = sqlite3.connect(path)
    c.execute("create table counters_collection (kernel_name text, dispatch_id integer, counter_name text, "
              "value real)")
    c.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    c.commit()
    c.close()
    return str(path)


@pytest.fixture
def store(tmp_path, monkeypatch):
    monkeypatch.setattr(C, "STORE", str(tmp_path / "counters.json"))
    monkeypatch.setattr(C, "VALU_STORE", str(tmp_path / "counters_valu.json"))
    return tmp_path


def test_traffic_scaling_and_step_sum(store, tmp_path):
    copy = "ek::k_copy16(float4*, float4 const*, long)"
    lb = "void ek::k_lb<float, true>(ek::Sim<float>)"
    ek = "void ek::k_ek32<2, 32, 8>(ek::Sim<float>, int, int, int, int)"
    diag = "void ek::k_diag_stage1<float>(ek::Sim<float>)"  # not a step kernel
    # FETCH_SIZE of the 1024 MiB copy reads half its bytes, in two instances;
    # the LB kernel's two dispatches average to 700000 KiB
    fetch = make_db(tmp_path / "f.db", [
        (copy, 1, "FETCH_SIZE", 262144.0), (copy, 1, "FETCH_SIZE", 262144.0),
        (lb, 2, "FETCH_SIZE", 600000.0), (lb, 3, "FETCH_SIZE", 800000.0),
        (ek, 4, "FETCH_SIZE", 400000.0), (diag, 5, "FETCH_SIZE", 900000.0)])
    write = make_db(tmp_path / "w.db", [
        (copy, 1, "WRITE_SIZE", 1048576.0), (lb, 2, "WRITE_SIZE", 1400000.0), (lb, 3, "WRITE_SIZE", 1400000.0),
        (ek, 4, "WRITE_SIZE", 300000.0), (diag, 5, "WRITE_SIZE", 100.0)])
    out = C.main(fetch, write, 1024)
    assert out["fetch_scale"] == pytest.approx(2.0)
    assert out["write_scale"] == pytest.approx(1.0)
    assert out["traffic_bytes_per_launch"] == pytest.approx((700000.0 * 2 + 1400000.0) * 1024)
    # the step sum takes the step's kernels only (LB and EK here), not the diagnostics or the copy
    assert out["step_bytes"] == pytest.approx((700000.0 * 2 + 1400000.0 + 400000.0 * 2 + 300000.0) * 1024)
    assert C.stored_traffic()["traffic_bytes_per_launch"] == out["traffic_bytes_per_launch"]
    assert C.stored_step_bytes() == out["step_bytes"]
    # counters taken with other sources are not reported
    d = json.loads(open(C.STORE).read())
    d["source_sha256"] = "0" * 64
    d["all_sources_sha256"] = "0" * 64
    open(C.STORE, "w").write(json.dumps(d))
    assert C.stored_traffic() is None
    assert C.stored_step_bytes() is None


def test_ek_valu_store_and_gating(store, tmp_path):
    ek = "void ek::k_ek32<2, 32, 8>(ek::Sim<float>, int, int, int, int)"
    sq = make_db(tmp_path / "sq.db", [
        (ek, 1, "SQ_INSTS_VALU", 7.0e7), (ek, 1, "SQ_INSTS_VALU", 7.5e7), (ek, 1, "SQ_WAVES", 3072.0),
        (ek, 2, "SQ_INSTS_VALU", 1.45e8), (ek, 2, "SQ_WAVES", 3072.0)])
    out = C.store_valu(sq)
    assert out["valu_per_launch"] == pytest.approx(1.45e8)
    assert out["waves_per_launch"] == pytest.approx(3072.0)
    assert C.stored_valu()["valu_per_launch"] == pytest.approx(1.45e8)
    d = json.loads(open(C.VALU_STORE).read())
    d["source_sha256"] = "0" * 64
    open(C.VALU_STORE, "w").write(json.dumps(d))
    assert C.stored_valu() is None


def test_missing_kernel_is_an_error(store, tmp_path):
    sq = make_db(tmp_path / "sq.db", [("void ek::k_lb<float, true>(ek::Sim<float>)", 1, "SQ_INSTS_VALU", 1.0)])
    with pytest.raises(KeyError):
        C.store_valu(sq)
