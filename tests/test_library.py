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
    assert (o.precision, o.ir_max_iter, o.ir_rtol, o.ir_dtol) == (m.PREC_FP64, 10, 1e-8, 1e-6)


def test_binding_structs_match_the_header(tmp_path):
    """ctypes mirrors of fds_options / fds_stats have the C layout (sizes and
    field offsets from a C program compiled against include/fds.h)."""
    import ctypes
    import shutil
    import subprocess
    import paper_2411_18026_amd as m
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    fields = {"fds_options": [f for f, _ in m._Options._fields_],
              "fds_stats": [f for f, _ in m._Stats._fields_]}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "fds.h"', "int main(void) {"]
    for t, fs in fields.items():
        lines.append(f'printf("{t} %zu\\n", sizeof({t}));')
        for f in fs:
            lines.append(f'printf("{t}.{f} %zu\\n", offsetof({t}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "abi"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True, check=True)
               .stdout.splitlines())
    for t, cls in (("fds_options", m._Options), ("fds_stats", m._Stats)):
        assert int(out[t]) == ctypes.sizeof(cls), t
        for f, _ in cls._fields_:
            assert int(out[f"{t}.{f}"]) == getattr(cls, f).offset, (t, f)
