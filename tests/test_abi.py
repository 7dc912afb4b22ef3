"""Host-only checks of the C ABI: the library loads, exports every symbol
include/scc.h declares, and sizes workspaces (no GPU calls)."""
import ctypes
import os
import re

import pytest

from paper_2403_01007_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in ("scc.h", "scc_learn.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        names |= set(re.findall(r"\b(scc_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_and_binding_agree():
    assert sorted(binding.EXPORTED_SYMBOLS) == _declared()


def test_library_exports_every_declared_symbol():
    lib = binding.load_library()
    for name in _declared():
        assert hasattr(lib, name), name


@pytest.mark.parametrize("dims", [(2, 3, 10, 2), (4, 12, 48, 2), (10, 90, 300, 3)])
def test_workspace_bytes(dims):
    n = binding.workspace_bytes(*dims)
    o, v, nj, ns = dims
    nov = o * v
    assert n > 8 * (nov * nov + nj * (o + v) ** 2)


def test_workspace_bytes_rejects_bad_dims():
    lib = binding.load_library()
    d = binding.Dims(0, 3, 10, 2)
    n = ctypes.c_size_t(0)
    assert lib.scc_workspace_bytes(ctypes.byref(d), None, ctypes.byref(n)) == -1
