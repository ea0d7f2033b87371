"""CPU checks of the C-ABI library: it loads, exports every function that
include/dicod.h declares, and the binding's structures match the header's
layout (compiled with gcc against the header).  No compute call is made."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dicod.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dicod_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dicod_init", "dicod_set_dictionary", "dicod_solve", "dicod_submit",
                     "dicod_poll", "dicod_last_error", "dicod_finalize"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_1705_10087_amd as d
    L = d.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, f"libdicod.so lacks {missing}"


def test_library_has_gfx950_code_and_no_cpu_fallback_symbols():
    import paper_1705_10087_amd as d
    out = subprocess.run(["nm", "-D", "--defined-only", d.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    assert "oracle_" not in out          # the product never links the oracle
    blob = open(d.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


@pytest.mark.parametrize("struct,cname", [("dicod_config", "dicod_config"),
                                          ("dicod_stats", "dicod_stats"),
                                          ("dicod_tune_entry", "dicod_tune_entry")])
def test_struct_layout_matches_header(tmp_path, struct, cname):
    import paper_1705_10087_amd as d
    cls = getattr(d, struct)
    fields = [f for f, _ in cls._fields_]
    cfields = [("lambda" if f == "lambda_" else f) for f in fields]
    prog = ["#include <stdio.h>", "#include <stddef.h>", '#include "dicod.h"',
            "int main(void){", f'printf("%zu\\n", sizeof({cname}));']
    prog += [f'printf("%zu\\n", offsetof({cname}, {f}));' for f in cfields]
    prog += ["return 0;}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(prog))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    vals = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert vals[0] == ctypes.sizeof(cls)
    for f, off in zip(fields, vals[1:]):
        assert getattr(cls, f).offset == off, f


def test_trace_record_layout(tmp_path):
    import paper_1705_10087_amd as d
    src = tmp_path / "tr.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "dicod.h"\n'
                   'int main(void){printf("%zu %zu %zu\\n", sizeof(dicod_trace_rec),'
                   ' offsetof(dicod_trace_rec, t0), offsetof(dicod_trace_rec, delta));}')
    exe = tmp_path / "tr"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    size, off_t0, off_d = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert size == d.TRACE_DTYPE.itemsize
    assert off_t0 == d.TRACE_DTYPE.fields["t0"][1]
    assert off_d == d.TRACE_DTYPE.fields["delta"][1]


def test_config_defaults_and_init_error_without_device():
    import torch
    import paper_1705_10087_amd as d
    cfg = d.dicod_config_init()
    assert cfg.precision == d.DICOD_PREC_FP32 and cfg.update_cap == -1
    if not torch.cuda.is_available():
        with pytest.raises(d.DicodError) as e:
            d.dicod_init(cfg)
        assert e.value.code == d.DICOD_EDEVICE
    bad = d.dicod_config_init(precision=7)
    with pytest.raises(d.DicodError):
        d.dicod_init(bad)
