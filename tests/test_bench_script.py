"""CPU checks of bench.py: it parses, every module-level function it calls
exists, and the GPU-count guard exits with a message (no device needed)."""
import ast
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_every_called_function_is_defined_or_imported():
    tree = ast.parse(open(BENCH).read())
    defined = {n.name for n in ast.walk(tree)
               if isinstance(n, (ast.FunctionDef, ast.ClassDef))}
    imported = set()
    for n in ast.walk(tree):
        if isinstance(n, ast.ImportFrom) or isinstance(n, ast.Import):
            imported |= {a.asname or a.name.split(".")[0] for a in n.names}
    assigned = {t.id for n in ast.walk(tree) if isinstance(n, ast.Assign)
                for t in n.targets if isinstance(t, ast.Name)}
    import builtins
    called = {n.func.id for n in ast.walk(tree)
              if isinstance(n, ast.Call) and isinstance(n.func, ast.Name)}
    missing = sorted(c for c in called if c not in defined | imported
                     | assigned and not hasattr(builtins, c))
    assert not missing, missing
    for name in ("bench_batched", "bench_wire", "bench_adjoint",
                 "cpu_baseline", "counted_traffic", "kernel_bytes", "main"):
        assert name in defined, name


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
