"""The product path has no fallback: without the built library the binding, and
everything above it, refuses to import."""
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_binding_refuses_to_import_without_the_library(tmp_path):
    pkg = tmp_path / "paper_1604_03570_amd"
    pkg.mkdir()
    src = os.path.join(ROOT, "paper_1604_03570_amd")
    for name in os.listdir(src):
        if name.endswith(".py"):
            shutil.copy(os.path.join(src, name), pkg / name)
    shutil.copytree(os.path.join(ROOT, "include"), tmp_path / "include")
    for mod in ("boxtile", "serve"):
        r = subprocess.run([sys.executable, "-c", f"import paper_1604_03570_amd.{mod}"], cwd=tmp_path,
                           capture_output=True, text=True, timeout=120)
        assert r.returncode != 0, mod
        assert "ImportError" in r.stderr and "libboxtile.so is missing" in r.stderr, r.stderr[-500:]
