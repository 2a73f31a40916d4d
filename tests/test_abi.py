"""The C ABI: the library loads without a GPU, exports every symbol that
include/vmfmm.h declares, and its host-only entry points validate their
arguments (no device work)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "vmfmm.h")).read()
    decl = r"^(?:vm_status|void|const char \*)\s*(vm_[a-z0-9_]+)\s*\("
    return sorted(set(re.findall(decl, text, flags=re.M)))


def test_every_declared_symbol_is_exported():
    from paper_1110_2921_amd import _lib
    lib = _lib.load()
    names = _declared()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(_lib.EXPORTS) == names


def test_host_entry_points_validate_arguments():
    from paper_1110_2921_amd import _lib
    lib = _lib.load()
    out = np.zeros((121, 121))
    assert lib.vm_debug_operator(0, 10, 316, out.ctypes.data) == _lib.VM_EINVAL
    assert lib.vm_debug_operator(1, 10, 8, out.ctypes.data) == _lib.VM_EINVAL
    assert lib.vm_debug_operator(3, 10, 0, out.ctypes.data) == _lib.VM_EINVAL
    assert lib.vm_debug_operator(7, 10, 0, out.ctypes.data) == _lib.VM_EINVAL
    assert lib.vm_debug_operator(0, 0, 0, out.ctypes.data) == _lib.VM_EINVAL
    assert lib.vm_debug_operator(0, 19, 0, out.ctypes.data) == _lib.VM_EINVAL   # VM_MAX_P = 18
    assert lib.vm_debug_operator(0, 10, 0, None) == _lib.VM_EINVAL
    cnt = ctypes.c_int()
    src = np.zeros(189, np.int32)
    d = np.zeros((189, 3), np.int8)
    assert lib.vm_debug_list(1, 0, 0, src.ctypes.data, d.ctypes.data, d.ctypes.data,
                             ctypes.byref(cnt)) == _lib.VM_EINVAL       # free space needs level >= 2
    assert lib.vm_debug_list(2, 1, 64, src.ctypes.data, d.ctypes.data, d.ctypes.data,
                             ctypes.byref(cnt)) == _lib.VM_EINVAL       # key out of range
    assert lib.vm_fmm_eval(None, 10, None, None, 1.0, 4, 2, None, None, None, None) == _lib.VM_EINVAL
    assert lib.vm_set_timing(None, 1) == _lib.VM_EINVAL


def test_offset_table_is_the_oracles():
    import paper_1110_2921_amd as vm
    from oracle import tree as T
    offs = [tuple(map(int, d)) for d in vm.debug_offsets()]
    assert offs == T.all_offsets()


@pytest.mark.parametrize("p", [1, 3, 10, 18])     # 18 = VM_MAX_P
def test_operator_generation_is_finite(p):
    import paper_1110_2921_amd as vm
    for kind, idx in ((0, 0), (0, 315), (1, 7), (2, 3), (3, 2)):
        m = vm.debug_operator(kind, p, idx)
        assert np.all(np.isfinite(m))
        assert np.abs(m).max() > 0


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library there is no fallback: loading it, and so
    creating a context, raises."""
    import paper_1110_2921_amd as vm
    from paper_1110_2921_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libvmfmm.so"))
    monkeypatch.setattr(_lib, "_LIB", None)
    with pytest.raises(ImportError):
        _lib.load()
    with pytest.raises(ImportError):
        vm.FMM(0)
