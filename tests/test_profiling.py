"""Host logic of the profile summaries on a synthetic counter database laid
out like rocprofv3's (counters_collection: kernel_name, counter_name, value,
duration in ns)."""
import os
import sqlite3

from paper_2505_21404_amd import profiling as PR


def _db(tmp_path, rows):
    d = tmp_path / "run"
    d.mkdir()
    path = d / "x_results.db"
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, counter_name text, "
                "value real, duration real)")
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    con.commit()
    con.close()
    return str(tmp_path)


def test_counters_summary_busy_fraction(tmp_path):
    k = "void dngd::(anonymous namespace)::gram_bf16_kernel<3, 16>(long, long)"
    # two dispatches: busy = 0.5 * 1024 SIMDs * (GUI / 8 XCDs)
    rows = []
    for gui in (8000.0, 16000.0):
        rows += [(k, "GRBM_GUI_ACTIVE", gui, 1000.0),
                 (k, "SQ_VALU_MFMA_BUSY_CYCLES", 0.5 * 1024 * gui / 8, 1000.0)]
    rows += [("dngd::other_kernel(int)", "GRBM_GUI_ACTIVE", 1.0, 5.0)]
    text = PR.counters_summary(_db(tmp_path, rows), ["gram_bf16"], "cmd", "title")
    assert "kernel: gram_bf16_kernel<3, 16>" in text
    assert "mfma_busy_frac: 0.500" in text
    assert "other_kernel" not in text


def test_traffic_summary_scaling(tmp_path):
    k = "void dngd::gemv_t_partial_kernel<float>(long)"
    cp = "__amd_rocclr_copyBuffer"
    base = tmp_path
    dirs = {}
    for name, rows in {
        "fetch": [(k, "FETCH_SIZE", 1000.0, 2000.0)],
        "write": [(k, "WRITE_SIZE", 10.0, 2000.0)],
        "cfetch": [(cp, "FETCH_SIZE", 512.0, 1.0)],
        "cwrite": [(cp, "WRITE_SIZE", 1024.0, 1.0)],
    }.items():
        p = base / name
        p.mkdir()
        dirs[name] = _db(p, rows)
    src = base / "k.hip"
    src.write_text("kernel source")
    text = PR.traffic_summary("gemv_t_partial", str(src), dirs["fetch"], dirs["write"],
                              dirs["cfetch"], dirs["cwrite"], 1024 * 1024, "a ;; b", "t",
                              copy_kernel="copyBuffer")
    rec = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line
               and not line.startswith(" "))
    # a 1 MiB copy read 512 KiB of FETCH_SIZE (factor 2) and 1024 KiB of WRITE_SIZE (1)
    assert rec["fetch_scale"] == "2.0000" and rec["write_scale"] == "1.0000"
    assert float(rec["traffic_bytes_per_dispatch"]) == 1000 * 1024 * 2 + 10 * 1024
    assert rec["source_sha256"] == PR.sha256_file(str(src))
    # a record whose source changed is stale
    out = base / "rec.txt"
    out.write_text(text.replace(f"source: {rec['source']}", f"source: {os.path.relpath(src, base)}"))
    assert PR.read_traffic(str(out), str(base)) is not None
    src.write_text("changed")
    assert PR.read_traffic(str(out), str(base)) is None
