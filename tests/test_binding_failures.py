"""The product path has one compute route, the HIP library, and says so when it cannot take it
(no GPU needed):

* a missing library raises VsError at load time instead of falling back to anything;
* host tensors handed to an entry point are refused before the library is called;
* nothing in the package imports the oracle, and the HIP library neither links the oracle's
  library nor exports any of its symbols.
"""
import ast
import os
import subprocess

import pytest
import torch

from paper_1701_03572_amd import vstab as V

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1701_03572_amd")
LIB = os.path.join(PKG, "libvstab.so")


def test_missing_library_raises(monkeypatch):
    monkeypatch.setattr(V, "_lib", None)
    with pytest.raises(V.VsError, match="not built"):
        V.load(os.path.join(ROOT, "no_such_dir", "libvstab.so"))


def test_host_tensors_are_refused_before_the_call():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    f = torch.zeros((1, 32, 32), dtype=torch.uint8)
    m = torch.zeros((1, 6), dtype=torch.float64)
    with pytest.raises(V.VsError, match="device tensor"):
        V.vs_warp_frame(f, 32 * 32, 32, 32, 32, m, 6, f.clone(), 32 * 32, 32, 1, 0, stream=0)


def test_package_never_imports_the_oracle():
    for name in sorted(os.listdir(PKG)):
        if not name.endswith(".py"):
            continue
        tree = ast.parse(open(os.path.join(PKG, name)).read())
        for node in ast.walk(tree):
            if isinstance(node, ast.Import):
                mods = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom):
                mods = [node.module or ""]
            else:
                continue
            assert not any(m == "oracle" or m.startswith("oracle.") for m in mods), (name, mods)


def test_hip_library_does_not_link_the_oracle():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    deps = subprocess.run(["readelf", "-d", LIB], capture_output=True, text=True, check=True).stdout
    assert "vs_oracle" not in deps
    syms = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = [line.split()[-1] for line in syms.splitlines() if line.strip()]
    assert not [s for s in exported if s.startswith("vso_")]
    assert "vs_track_lk" in exported
