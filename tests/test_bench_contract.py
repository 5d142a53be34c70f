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
