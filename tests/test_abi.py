"""The C ABI library loads on a machine without a GPU and exports every entry point that
include/gi.h declares; the ctypes mirrors of the structs have the C layout."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gi.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gi_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2310_19855_amd import gi
    L = gi.lib()
    names = _declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert b"gfx950" in L.gi_version()


def test_struct_layout_matches_header(tmp_path):
    from paper_2310_19855_amd import gi
    prog = tmp_path / "layout.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "gi.h"\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(gi_config), sizeof(gi_frame),'
                    ' offsetof(gi_config, cell_scale), offsetof(gi_config, mlp_batch_log2),'
                    ' offsetof(gi_config, scene_max), offsetof(gi_frame, up), offsetof(gi_config, upscale));'
                    ' return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(prog), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [C.sizeof(gi.Config), C.sizeof(gi.Frame), gi.Config.cell_scale.offset,
            gi.Config.mlp_batch_log2.offset, gi.Config.scene_max.offset, gi.Frame.up.offset,
            gi.Config.upscale.offset]
    assert got == want


def test_create_without_gpu_fails_cleanly():
    from paper_2310_19855_amd import gi
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("GPU present")
    except ImportError:
        pass
    with pytest.raises(gi.GIError):
        gi.Context(width=64, height=64)


def test_missing_library_is_an_error(monkeypatch, tmp_path):
    from paper_2310_19855_amd import gi
    monkeypatch.setattr(gi, "_lib", None)
    monkeypatch.setattr(gi, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(gi.GIError, match="missing"):
        gi.lib()
