"""CPU-side checks of the C ABI library: it loads and exports every symbol
declared in include/fds.h (no compute calls without a GPU), and the binding
refuses to run without it."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fds.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(fds_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("fds_build", "fds_solve", "fds_rhs_plane", "fds_destroy", "fds_size", "fds_entries"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import ctypes
    import paper_2411_18026_amd as m
    if not os.path.exists(m.lib_path()):
        pytest.skip("library not built")
    L = ctypes.CDLL(m.lib_path())
    for n in _declared():
        assert hasattr(L, n), n
    assert set(m.EXPORTS) <= set(_declared())


def test_strerror_without_gpu():
    import paper_2411_18026_amd as m
    if not os.path.exists(m.lib_path()):
        pytest.skip("library not built")
    L = m.load()
    assert L.fds_strerror(0) == b"ok"
    assert L.fds_strerror(5) == b"singular pivot"


def test_options_defaults_without_gpu():
    import paper_2411_18026_amd as m
    if not os.path.exists(m.lib_path()):
        pytest.skip("library not built")
    o = m._options()
    assert (o.leaf_nodes, o.n_proxy, o.root_level, o.proxy_ratio, o.use_alpha) == (64, 64, 1, 1.5, 0)
