"""The C ABI library loads and exports every entry point include/bfs.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header="bfs.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bfs_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("bfs_create_graph_csr", "bfs_create_graph_dcsc", "bfs_run", "bfs_run_multi", "bfs_block_td",
                     "bfs_block_bu", "bfs_workspace_bytes", "bfs_destroy_graph", "bfs_status_string"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_1705_04590_amd as bfs
    lib = bfs.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in bfs.EXPORTED, name


def test_library_exports_every_server_symbol():
    import paper_1705_04590_amd as bfs
    lib = bfs.lib()
    names = declared_functions("bfs_serve.h")
    assert "bfs_server_submit" in names and "bfs_server_replay" in names
    for name in names:
        assert hasattr(lib, name), name


def test_server_options_defaults_need_no_gpu():
    from paper_1705_04590_amd import serve
    o = serve.bfs_server_opts_default()
    assert (o.slots, o.max_batch, o.want_parent) == (4, 64, 0)
    assert o.opts.alpha == 15.0 and o.hbm_budget == 8 << 30


def test_host_side_defaults_and_strings():
    import paper_1705_04590_amd as bfs
    o = bfs.bfs_opts_default()
    assert (o.dir, o.parent_mode, o.alpha, o.beta, o.timing) == (bfs.BFS_DIR_DO, bfs.BFS_PARENT_ANY, 15.0, 18.0, 0)
    assert bfs.bfs_status_string(0) == "ok"
    assert "workspace" in bfs.bfs_status_string(7)


def test_host_argument_errors_need_no_gpu():
    import paper_1705_04590_amd as bfs
    lib = bfs.lib()
    h = ctypes.c_void_p()
    assert lib.bfs_create_graph_csr(-1, 1, 8, 1, 0, 0, None, ctypes.byref(h)) == 1
    assert "n=-1" in bfs.bfs_last_error()
    assert lib.bfs_create_graph_csr(4, 1, 3, 1, 0, 0, None, ctypes.byref(h)) == 1
    assert lib.bfs_create_graph_csr(4, None, 8, 1, 0, 0, None, ctypes.byref(h)) == 1
    assert lib.bfs_create_graph_csr(4, 1, 4, 1, 1 << 31, 0, None, ctypes.byref(h)) == 1
    assert lib.bfs_create_graph_csr(4, 1, 8, 1, 0, 0x80, None, ctypes.byref(h)) == 1
    assert lib.bfs_run(None, 0, None, 1, 1, 1, 0, None, None) == 1
    assert lib.bfs_workspace_bytes(None, 1) == 0
    assert lib.bfs_create_graph_dcsc(0, 4, 0, 0, 0, None, None, None, 0, None, None, None, 0, 0, None,
                                     ctypes.byref(h)) == 1


def test_binding_structs_match_the_headers(tmp_path):
    """The Python binding's ctypes structures have the sizes and field offsets
    that the C headers give them (checked with gcc; no GPU)."""
    import shutil
    import subprocess

    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    import paper_1705_04590_amd as bfs
    from paper_1705_04590_amd import serve

    structs = {"bfs_opts": bfs.bfs_opts, "bfs_stats": bfs.bfs_stats,
               "bfs_server_opts": serve.bfs_server_opts, "bfs_server_stats": serve.bfs_server_stats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bfs_serve.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} . %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c11", "-Wall", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        name, field, value = line.split()
        got[(name, field)] = int(value)
    for name, cls in structs.items():
        assert got[(name, ".")] == ctypes.sizeof(cls), f"sizeof({name})"
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, f"offsetof({name}, {field})"
