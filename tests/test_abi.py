"""Host-side checks of the C-ABI library (no GPU calls)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1612_03310_amd import native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mithra.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mithra_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_functions():
    assert _declared_functions() == sorted(native.ABI_FUNCTIONS)


def test_library_loads_and_exports_every_declared_symbol():
    if not os.path.exists(native.LIB_PATH):
        pytest.fail("libmithra.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(native.LIB_PATH)
    missing = [f for f in _declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_struct_layouts_match_the_header():
    # sizes implied by the C declarations (natural alignment on x86-64)
    assert ctypes.sizeof(native.Mesh) == 3 * 4 + 4 + 3 * 8 + 3 * 8 + 8 + 8 + 4 + 4 + 3 * 4 + 4
    assert ctypes.sizeof(native.Undulator) == 40
    assert ctypes.sizeof(native.Seed) == 8 * 8 + 4 + 4
    assert ctypes.sizeof(native.Beam) == 4 + 4 + 2 * 8 + 3 * 8
    assert ctypes.sizeof(native.DiagCfg) == 28 + 12
    assert ctypes.sizeof(native.DiagRow) == 8 * 14 + 4 + 4 + 3 * 8 + 3 * 8 + 3 * 8 + 2 * 8
    assert ctypes.sizeof(native.Info) == 7 * 8 + 3 * 8 + 3 * 4 + 4 + 3 * 4 + 4


def test_last_error_is_empty_string_before_any_failure():
    lib = native.load_library()
    assert isinstance(lib.mithra_last_error(), bytes)


def test_null_arguments_are_rejected_without_a_device():
    lib = native.load_library()
    assert lib.mithra_create(None, None, 0, None, None) == native.EINVAL
    assert lib.mithra_run(None, 1) == native.EINVAL
    assert b"NULL" in lib.mithra_last_error()
    assert lib.mithra_set_allocator(ctypes.c_void_p(1), None, None) == native.EINVAL


def test_allocator_callbacks_outlive_every_simulation():
    """Each simulation keeps the allocator function pointers it was created
    with; installing the hook again must not replace (and free) the callback
    objects an existing simulation still calls."""
    native.use_torch_allocator(True)
    first = list(native._hooks)
    native.use_torch_allocator(True)
    native.use_torch_allocator(False)
    native.use_torch_allocator(True)
    assert len(native._hooks) == 2
    assert native._hooks[0] is first[0] and native._hooks[1] is first[1]


def test_struct_field_offsets_match_the_header(tmp_path):
    """Every field of every struct the binding passes sits where a C compiler
    puts it (gcc on include/mithra.h, offsetof), not only the sizes."""
    structs = {"mithra_mesh": native.Mesh, "mithra_undulator": native.Undulator,
               "mithra_seed": native.Seed, "mithra_beam": native.Beam,
               "mithra_diag_cfg": native.DiagCfg, "mithra_diag_row": native.DiagRow,
               "mithra_info": native.Info}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mithra.h"', 'int main(void) {']
    for cname, cls in structs.items():
        lines.append('printf("%%s %%zu\\n", "%s", sizeof(%s));' % (cname, cname))
        for fname, _ in cls._fields_:
            lines.append('printf("%%s.%%s %%zu\\n", "%s", "%s", offsetof(%s, %s));'
                         % (cname, fname, cname, fname))
    lines.append('return 0; }')
    src = tmp_path / "offsets.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "offsets"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)])
    out = dict(line.rsplit(" ", 1) for line in subprocess.check_output([str(exe)]).decode().split("\n")
               if line)
    for cname, cls in structs.items():
        assert int(out[cname]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(out["%s.%s" % (cname, fname)]) == getattr(cls, fname).offset, (cname, fname)
