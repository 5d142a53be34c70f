"""Host-side checks of bench.py: every name its functions read is defined (a deleted
helper fails here, not on the GPU), and more than one GPU is refused with a message."""
import ast
import builtins
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def _undefined_names(src: str):
    tree = ast.parse(src)
    module_names = set(dir(builtins))
    for node in tree.body:
        if isinstance(node, (ast.FunctionDef, ast.ClassDef)):
            module_names.add(node.name)
        elif isinstance(node, (ast.Import, ast.ImportFrom)):
            module_names.update((a.asname or a.name).split(".")[0] for a in node.names)
        elif isinstance(node, ast.Assign):
            module_names.update(t.id for t in node.targets if isinstance(t, ast.Name))
    missing = []
    # each top-level function with everything nested in it (closures see enclosing locals)
    for fn in tree.body:
        if not isinstance(fn, ast.FunctionDef):
            continue
        local = set()
        for n in ast.walk(fn):
            if isinstance(n, ast.Name) and isinstance(n.ctx, (ast.Store, ast.Del)):
                local.add(n.id)
            elif isinstance(n, ast.arg):
                local.add(n.arg)
            elif isinstance(n, (ast.Import, ast.ImportFrom)):
                local.update((a.asname or a.name).split(".")[0] for a in n.names)
            elif isinstance(n, ast.FunctionDef) and n is not fn:
                local.add(n.name)
            elif isinstance(n, ast.comprehension):
                local.update(t.id for t in ast.walk(n.target) if isinstance(t, ast.Name))
            elif isinstance(n, ast.ExceptHandler) and n.name:
                local.add(n.name)
        for n in ast.walk(fn):
            if isinstance(n, ast.Name) and isinstance(n.ctx, ast.Load):
                if n.id not in local and n.id not in module_names:
                    missing.append((getattr(fn, "name", "<lambda>"), n.id))
    return missing


def test_bench_reads_no_undefined_name():
    assert _undefined_names(open(BENCH).read()) == []


def test_undefined_name_checker_catches_a_deleted_helper():
    assert ("main", "helper") in _undefined_names("def main():\n    return helper(1)\n")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_traffic_only_for_the_counted_source_and_tiles(monkeypatch):
    """`roofline.traffic` comes from the committed counter summary only while the
    dedispersion sources hash to the recorded value and every beam runs the recorded
    tile shape; otherwise it is null."""
    import re
    sys.path.insert(0, ROOT)
    import bench
    text = open(os.path.join(ROOT, "profiles", "dedisp_c3_hbm_counters.md")).read()
    m = re.search(r"^counters: workload=c3 kernel=k_dedisp tiles=(\d+),(\d+),(\d+),(\d+),(\d+) grid=\d+ "
                  r"fetch_bytes=(\d+) write_bytes=(\d+) dedisp_src_sha256=([0-9a-f]{64})$", text, re.M)
    assert m, "the summary carries one machine-readable counters line"
    dw, j, nw, cc, nbuf = (int(m.group(i)) for i in range(1, 6))
    tiles = [{"dm_per_wave": dw, "time_groups": j, "waves": nw, "chan_chunk": cc, "buffers": nbuf}] * 2
    want = {"fetch_bytes": int(m.group(6)), "write_bytes": int(m.group(7))}
    monkeypatch.setattr(bench, "dedisp_source_hash", lambda: m.group(8))
    assert bench.counter_traffic("c3", tiles) == want
    assert bench.counter_traffic("c3", tiles[:1] + [dict(tiles[0], chan_chunk=cc // 2)]) is None
    assert bench.counter_traffic("c3", tiles[:1] + [dict(tiles[0], buffers=3 - nbuf)]) is None
    assert bench.counter_traffic("c4", tiles) is None          # no summary for that workload
    monkeypatch.setattr(bench, "dedisp_source_hash", lambda: "0" * 64)
    assert bench.counter_traffic("c3", tiles) is None
    # the counted bytes are at least the launch's algorithmic bytes (blocks read once,
    # DM transforms written once)
    assert want["fetch_bytes"] >= 24 * 4096 * 26305 and want["write_bytes"] >= 24 * 2048 * 16639 * 4
