"""The C ABI library loads, exports every symbol include/surfgn.h declares,
and its argument checks answer without touching a GPU."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "surfgn.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:sgn_status|const char\*)\s+(sgn_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def sg():
    from paper_1910_01997_amd import surfgn
    if not os.path.exists(surfgn.LIB_PATH):
        from paper_1910_01997_amd import build
        build.build()
    surfgn.lib()
    return surfgn


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["sgn_create", "sgn_destroy", "sgn_init_from_neighbours", "sgn_optimize_keyframe",
              "sgn_render_inverse_depth", "sgn_optimize_batch", "sgn_autotune", "sgn_quantize"]:
        assert n in names


def test_library_exports_every_declared_symbol(sg):
    L = sg.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert sorted(sg.EXPORTED) == _declared()
    out = subprocess.run(["nm", "-D", "--defined-only", sg.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (sgn_\w+)", out))
    assert set(_declared()) <= exported


def test_library_is_built_for_gfx950(sg):
    out = subprocess.run(["/opt/rocm/bin/roc-obj-ls", sg.LIB_PATH], capture_output=True, text=True)
    if out.returncode != 0:
        pytest.skip("roc-obj-ls unavailable")
    assert "gfx950" in out.stdout


def test_status_strings_and_version(sg):
    assert sg.sgn_status_str(0) == "ok"
    assert sg.sgn_status_str(-1) == "invalid argument"
    assert "gfx950" in sg.sgn_version()


def test_null_arguments_are_rejected_synchronously(sg):
    L = sg.lib()
    assert L.sgn_optimize_keyframe(None, None, None, None, None) == sg.SGN_E_INVALID
    assert L.sgn_render_inverse_depth(None, None, None, None, None) == sg.SGN_E_INVALID
    assert L.sgn_optimize_batch(None, None, 0, None, None) == sg.SGN_E_INVALID
    assert L.sgn_init_from_neighbours(None, None, None, None, None) == sg.SGN_E_INVALID
    assert L.sgn_quantize(None, None, 0, None) == sg.SGN_E_INVALID
    ms = C.c_float()
    assert L.sgn_last_kernel_ms(None, C.byref(ms)) == sg.SGN_E_INVALID
    assert L.sgn_create(None, 0, None) == sg.SGN_E_INVALID
    assert "null" in sg.sgn_last_error()
    assert L.sgn_destroy(None) == sg.SGN_OK


def test_create_without_a_gpu_fails_cleanly(sg):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    st = sg.lib().sgn_create(C.byref(h), 0, None)
    assert st in (sg.SGN_E_DEVICE, sg.SGN_E_INVALID)
    assert h.value is None


def test_binding_refuses_to_run_without_the_library(tmp_path, monkeypatch):
    from paper_1910_01997_amd import surfgn
    monkeypatch.setattr(surfgn, "_lib", None)
    monkeypatch.setattr(surfgn, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        surfgn.lib()


def test_struct_layouts_match_the_header():
    """Compile a probe against the header and compare struct sizes/offsets
    with the ctypes mirrors."""
    from paper_1910_01997_amd import surfgn as s
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "surfgn.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(sgn_intrinsics), sizeof(sgn_pose),
         sizeof(sgn_image), sizeof(sgn_keyframe), sizeof(sgn_surfels), sizeof(sgn_params),
         sizeof(sgn_plan), sizeof(sgn_batch_item), sizeof(sgn_device_props));
  printf("%zu %zu %zu %zu\n", offsetof(sgn_keyframe, K), offsetof(sgn_keyframe, patch),
         offsetof(sgn_batch_item, is_new), offsetof(sgn_device_props, name));
  return 0;
}
'''
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    sizes = [int(v) for v in out[0].split()]
    offs = [int(v) for v in out[1].split()]
    mine = [C.sizeof(t) for t in (s.sgn_intrinsics, s.sgn_pose, s.sgn_image, s.sgn_keyframe,
                                  s.sgn_surfels, s.sgn_params, s.sgn_plan, s.sgn_batch_item,
                                  s.sgn_device_props)]
    assert sizes == mine
    assert offs == [s.sgn_keyframe.K.offset, s.sgn_keyframe.patch.offset,
                    s.sgn_batch_item.is_new.offset, s.sgn_device_props.name.offset]
