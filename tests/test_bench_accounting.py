"""The benchmark's byte accounting (CPU): the algorithmic bytes bench.py divides by each kernel's time are
the ones the committed counter summaries list, the counter tables parse while their kernel hash is
current, and a run on more than one GPU is refused with a message."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

PACK_NODES, PACK_CELLS = 53_686_166, 512 ** 3
CHANNEL_NODES = 256 * 256 * 254


def _profile_rows(workload):
    """{label: (algorithmic bytes, kernel hash)} of profiles/counters_<workload>.md."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.md")
    rows, h = {}, None
    for line in open(path):
        if line.startswith("kernel_source_hash:"):
            h = line.split(":", 1)[1].strip()
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 8 and cells[0].startswith(workload + "/"):
            rows[cells[0]] = int(float(cells[6]))
    return rows, h


def test_channel_kernel_bytes_match_the_counter_summary():
    rows, _ = _profile_rows("channel256")
    assert rows
    for label, alg in rows.items():
        _, scheme, layout, prec, name = label.split("/")
        assert bench.kernel_bytes(name, "direct", prec, CHANNEL_NODES) == alg, label


def test_pack_kernel_bytes_match_the_counter_summary():
    """FP64 pack: neighbour ids (and the esoteric twist's table) by rank, as the library runs it."""
    rows, _ = _profile_rows("pack512")
    assert rows
    for label, alg in rows.items():
        _, scheme, layout, prec, name = label.split("/")
        if name in ("ts_collide", "ts_stream"):
            continue   # timed together as ts_step
        b = bench.kernel_bytes(name, "indirect", prec, PACK_NODES, rank=True, cells=PACK_CELLS, et_rank=True)
        assert b == alg, label
    step = rows["pack512/ts/soa/f64/ts_step"]
    assert bench.kernel_bytes("ts_step", "indirect", "f64", PACK_NODES, rank=True, cells=PACK_CELLS) == step


def test_kernel_bytes_forms():
    """Each PDF read and written once; IDX 72 B or 4 B of cell_of plus the words once; ET table 28 B or
    4 B plus fluid and ghost words."""
    n, c = 1000, 4096
    assert bench.kernel_bytes("aa_even", "direct", "f64", n) == 304 * n
    assert bench.kernel_bytes("aa_odd", "indirect", "f64", n) == (304 + 72) * n
    assert bench.kernel_bytes("aa_odd", "indirect", "f32", n, rank=True, cells=c) == (152 + 4) * n + 8 * (c // 32)
    assert bench.kernel_bytes("aa_even", "indirect", "f64", n, rank=True, cells=c) == 304 * n
    assert bench.kernel_bytes("ts_step", "indirect", "f64", n) == (608 + 72) * n
    assert bench.kernel_bytes("et_odd", "indirect", "f64", n) == (304 + 28) * n
    assert bench.kernel_bytes("et_odd", "indirect", "f64", n, rank=True, cells=c, et_rank=True) == \
        (304 + 4) * n + 16 * (c // 32)


@pytest.mark.parametrize("workload", ["channel256", "pack512"])
def test_counter_tables_parse_while_current(workload):
    """While a summary carries the current kernel hash the bench reads every row of it; once the kernels
    change it reads none (its traffic is then reported as unknown)."""
    rows, h = _profile_rows(workload)
    table = bench.counter_table(workload)
    if h != bench.kernel_hash():
        assert table == {}
        pytest.skip(f"counters_{workload}.md was taken on kernels {h}, these hash to {bench.kernel_hash()}")
    assert set(table) >= set(rows)
    assert all(v > 0 for v in table.values())


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)


def test_channel_table_rows_pick_their_storage_order(monkeypatch):
    """The FP64 AA row that carries the headline's counters runs plain SoA (block 0) whatever the
    library's default is; the blocked row and every other row run the library's default (no option)."""
    calls = []
    monkeypatch.setattr(bench, "channel_grid", lambda P, torch, n, scheme, layout, prec="f64", block=None:
                        calls.append((scheme, layout, prec, block)))
    for scheme, layout, prec in bench.CHANNEL_SET:
        bench.table_grid(None, None, 256, scheme, layout, prec)
    assert len(calls) == len(bench.CHANNEL_SET)
    assert ("aa", "soa", "f64", 0) in calls
    assert ("aa", "soa", "f64", None) in calls          # the row "aa/soa_blocked"
    assert sum(1 for c in calls if c[3] == 0) == 1
    assert ("aa", "soa_blocked", "f64") in bench.CHANNEL_SET
    # the headline is measured on the grid of that same row
    import inspect
    assert 'table_grid(P, torch, n, "aa", "soa", "f64")' in inspect.getsource(bench.main)
