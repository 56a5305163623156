"""The C-ABI library loads and exports every entry point include/rlc.h
declares (no compute: these run without a GPU)."""
import ctypes
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rlc.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rlc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_method_calls():
    names = _declared()
    for must in ("rlc_build_light_tree", "rlc_sample", "rlc_shade", "rlc_learn", "rlc_adapt_cuts",
                 "rlc_frame", "rlc_set_occluders"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1911_10217_amd import rlc
    if not os.path.exists(rlc.LIB_PATH):
        pytest.skip("librlc.so not built")
    lib = ctypes.CDLL(rlc.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares exactly the header's entry points
    assert sorted(rlc.EXPORTS) == _declared()


def test_config_struct_layout_matches_header():
    # field order and sizes of rlc_config as declared in the header
    from paper_1911_10217_amd import rlc
    text = open(HEADER).read()
    body = text[text.index("typedef struct rlc_config"):text.index("} rlc_config;")]
    fields = re.findall(r"^\s*(?:uint32_t|uint64_t|float)\s+(\w+)", body, flags=re.M)
    assert [f[0] for f in rlc.rlc_config._fields_] == fields
    # offsets and size as a C compiler lays the header's struct out
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        pytest.skip("no C compiler")
    d = tempfile.mkdtemp()
    try:
        src = os.path.join(d, "layout.c")
        with open(src, "w") as f:
            f.write('#include <stddef.h>\n#include <stdio.h>\n#include "rlc.h"\nint main(void) {\n')
            f.write('    printf("%zu\\n", sizeof(rlc_config));\n')
            for n in fields:
                f.write('    printf("%%zu\\n", offsetof(rlc_config, %s));\n' % n)
            f.write("    return 0;\n}\n")
        exe = os.path.join(d, "layout")
        subprocess.check_call([cc, "-I", os.path.dirname(HEADER), "-o", exe, src])
        got = [int(v) for v in subprocess.check_output([exe]).split()]
    finally:
        shutil.rmtree(d, ignore_errors=True)
    assert got[0] == ctypes.sizeof(rlc.rlc_config)
    assert got[1:] == [getattr(rlc.rlc_config, n).offset for n in fields]


def test_no_gpu_means_loud_failure():
    import torch
    from paper_1911_10217_amd import rlc, scenes
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        rlc.Context(scenes.params_for())
