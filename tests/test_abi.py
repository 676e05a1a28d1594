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


def test_binding_structs_match_the_header(tmp_path):
    """Every struct the ctypes binding passes through the ABI has the size and
    field offsets the C compiler gives the header's declaration."""
    import ctypes
    import paper_0905_1744_amd as kdm
    pairs = {"kd_server_opts": kdm.ServerOpts, "kd_job": kdm.Job, "kd_done": kdm.Done,
             "kd_server_stage": kdm.ServerStage,
             "kd_psp_pair": kdm.PspPair}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "kd.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                           text=True).stdout.splitlines())
    for cname, py in pairs.items():
        assert int(got[f"{cname} size"]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname} {f}"]) == getattr(py, f).offset, (cname, f)
