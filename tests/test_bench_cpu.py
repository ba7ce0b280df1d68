"""bench.py's command-line contract on the CPU: more than one GPU is refused
with a message before anything touches a device, and the kernel-source hash
that guards the committed HBM-traffic counters is stable and content-based."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_kernel_source_hash_is_stable():
    sys.path.insert(0, ROOT)
    import bench
    a = bench.kernel_source_hash()
    b = bench.kernel_source_hash()
    assert a == b and len(a) == 64


def _names_bound(node):
    """Names a function (or module) binds: arguments, assignments, loop and
    comprehension targets, imports, nested definitions."""
    import ast
    out = set()
    for n in ast.walk(node):
        if isinstance(n, ast.arg):
            out.add(n.arg)
        elif isinstance(n, ast.Name) and isinstance(n.ctx, (ast.Store, ast.Del)):
            out.add(n.id)
        elif isinstance(n, (ast.FunctionDef, ast.AsyncFunctionDef, ast.ClassDef)):
            out.add(n.name)
        elif isinstance(n, (ast.Import, ast.ImportFrom)):
            for a in n.names:
                out.add((a.asname or a.name).split(".")[0])
        elif isinstance(n, ast.ExceptHandler) and n.name:
            out.add(n.name)
    return out


def test_every_called_name_in_bench_is_defined():
    """Each bare-name call in bench.py resolves to a builtin, a module-level
    name or a name its function binds: the legs the default run takes only on
    a GPU cannot call a helper that no longer exists."""
    import ast
    import builtins
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    known = set(dir(builtins)) | _names_bound(tree)
    missing = sorted({n.func.id for n in ast.walk(tree)
                      if isinstance(n, ast.Call) and isinstance(n.func, ast.Name) and n.func.id not in known})
    assert not missing, missing
