"""CPU: the bench's summaries of rocprofv3 result databases (kernel trace,
counter runs and the HBM traffic entry), on small synthetic databases laid out
as rocprofv3 writes them (a `kernels` view and a `pmc_events` table)."""
import json
import os
import sqlite3
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, HERE)
import bench  # noqa: E402


def _db(path, rows, pmc=()):
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, start integer, end integer, dispatch_id integer)")
    con.execute("create table pmc_events (dispatch_id integer, counter_name text, counter_value real)")
    con.executemany("insert into kernels values (?, ?, ?, ?)", rows)
    con.executemany("insert into pmc_events values (?, ?, ?)", pmc)
    con.commit()
    con.close()


def _update_rows():
    """A static run, then two updates of (merge, sweep, modularity scan), then
    a static run on the final graph; times in ns."""
    rows, t, d = [], 0, 0

    def k(name, dur):
        nonlocal t, d
        rows.append((name, t, t + dur, d))
        t += dur + 1000
        d += 1

    k("lk::k_mod_edges(...)", 5_000_000)          # static run before the stream
    for _ in range(2):
        k("lk::k_batch_apply_old(lk::BatchArgs)", 10_000_000)
        k("void lk::k_refine_async<4, 512, true>(lk::RefineArgs)", 40_000_000)
        k("void lk::k_move_async<4, 512, true>(lk::MoveArgs)", 20_000_000)
        k("void lk::k_mod_intra<double>(long const*, ...)", 4_000_000)
    k("void lk::k_mod_intra<float>(long const*, ...)", 30_000_000)  # static run after the stream
    k("MulFunctor calibration", 1_000_000)
    return rows


def test_update_window_ends_at_the_last_updates_modularity_scan(tmp_path):
    db = str(tmp_path / "t.db")
    _db(db, _update_rows())
    rows = bench._trace_rows(db)
    a, b, nup = bench._update_window(rows)
    assert nup == 2
    names = [r[0] for r in rows if a <= r[1] < b]
    assert names[0].startswith("lk::k_batch_apply_old") and len(names) == 8
    assert "k_mod_intra<float>" not in "".join(names)
    md = bench.summarize_trace(db, "cmd")
    assert "Dynamic updates: 2" in md
    refine = [l for l in md.splitlines() if "k_refine_async" in l][0]
    assert "| 40.00 | 1.0 | 40000.0 |" in refine


def test_traffic_entry_scales_by_the_calibration_kernel(tmp_path):
    rows = _update_rows()
    ids = {r[0].split("(")[0]: r[3] for r in rows}
    refine = [r[3] for r in rows if "k_refine_async" in r[0]]
    cal = ids["MulFunctor calibration"]
    # the calibration's 1 GiB read counted as 0.5 GiB, written as 1 GiB
    fetch = [(d, "FETCH_SIZE", 1000.0) for d in refine] + [(cal, "FETCH_SIZE", (1 << 30) / 2048.0)]
    write = [(d, "WRITE_SIZE", 500.0) for d in refine] + [(cal, "WRITE_SIZE", (1 << 30) / 1024.0)]
    fdb, wdb = str(tmp_path / "f.db"), str(tmp_path / "w.db")
    _db(fdb, rows, fetch)
    _db(wdb, rows, write)
    e = bench.traffic_from_pmc(fdb, wdb, "void lk::k_refine_async", "key")
    assert e["fetch_launches"] == 2 and e["write_launches"] == 2
    assert e["fetch_factor"] == pytest.approx(2.0) and e["write_factor"] == pytest.approx(1.0)
    assert e["bytes_per_launch"] == int(1000 * 1024 * 2.0 + 500 * 1024 * 1.0)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(HERE, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
    assert r.stdout.strip() == "" or json.loads(r.stdout) is None
