"""bench.py's command-line contract that needs no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_every_workload_prints_one_json_line():
    # static check of bench.py: top-level functions are defined once, and each
    # bench_* entry point ends by printing its JSON object
    import ast
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    names = [f.name for f in tree.body if isinstance(f, ast.FunctionDef)]
    assert len(names) == len(set(names)), sorted(n for n in names if names.count(n) > 1)
    for f in tree.body:
        if isinstance(f, ast.FunctionDef) and f.name.startswith("bench_"):
            last = f.body[-1]
            assert isinstance(last, ast.Expr) and isinstance(last.value, ast.Call), f.name
            call = last.value
            assert getattr(call.func, "id", None) == "print", f.name
            inner = call.args[0]
            assert isinstance(inner, ast.Call) and getattr(inner.func, "attr", None) == "dumps", f.name
