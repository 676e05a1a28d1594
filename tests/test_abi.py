"""The C-ABI library loads and exports every symbol its header declares (no
compute calls: this runs without a GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kd.h")
LIB = os.path.join(ROOT, "paper_0905_1744_amd", "libkmerdecomp.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(LIB):
        from paper_0905_1744_amd import build
        build.build()
    return LIB


def test_header_declares_the_four_calls():
    names = _declared()
    for n in ("kmer_count", "kmer_similarity", "kmer_rank", "sample_partition",
              "kd_ctx_create", "kd_ctx_destroy", "kd_set_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol(built):
    out = subprocess.run(["nm", "-D", "--defined-only", built], capture_output=True, text=True,
                         check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing


def test_library_loads_with_torch_runtime(built):
    import torch  # noqa: F401  (the binding shares torch's HIP runtime)
    import paper_0905_1744_amd as kd
    L = kd.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert L.kd_strerror(-2) == b"residue outside the 20 standard amino acids"
    maps = open("/proc/self/maps").read()
    hip = {l.split()[-1] for l in maps.splitlines() if "libamdhip64" in l}
    assert len(hip) == 1, hip


def test_binding_refuses_missing_library(monkeypatch, tmp_path):
    import paper_0905_1744_amd as kd
    monkeypatch.setattr(kd, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(kd, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        kd.lib()
