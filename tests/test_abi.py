"""The C ABI without a GPU: the built library loads, exports every function
include/bfs.h declares, and rejects bad arguments before any device call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bfs.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1408_1605_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_1408_1605_amd import build
        build.build()
    return binding


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(bfs_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_parses():
    names = declared_functions()
    assert "bfs_run" in names and "bfs_run_batch" in names and "bfs_submit" in names
    assert len(names) >= 15


def test_every_declared_symbol_is_exported(lib):
    so = ctypes.CDLL(lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(so, name), name
    assert sorted(declared_functions()) == sorted(lib.EXPORTS)


def test_exported_symbols_are_c_linkage(lib):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", lib.LIB_PATH], capture_output=True,
                         text=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in declared_functions():
        assert name in syms, name  # unmangled


def test_version_and_error_string(lib):
    assert lib.bfs_version() >= 100
    assert isinstance(lib.bfs_last_error(), str)


def test_workspace_bytes(lib):
    a = lib.bfs_workspace_bytes(1 << 16, 1 << 20)
    b = lib.bfs_workspace_bytes(1 << 16, 1 << 20, lib.BFS_WS_BATCH)
    c = lib.bfs_workspace_bytes(1 << 16, 1 << 20, lib.BFS_DEGREE_ORDER)
    assert b >= a + 3 * 8 * (1 << 16)
    # rank, orig, row offsets, two column copies, ten row prefix skip counts,
    # level and parent by internal id
    assert c >= a + 64 * (1 << 16) + 8 * (1 << 20)
    assert a % 256 == 0
    # scale 26 stays well inside 288 GB of HBM
    big = lib.bfs_workspace_bytes(1 << 26, 2_110_000_000, lib.BFS_DEGREE_ORDER | lib.BFS_WS_BATCH)
    assert big < 32e9


@pytest.mark.parametrize("V,nnz,flags", [(0, 5, 0), (-3, 5, 0), (10, -1, 0), (10, 5, 0x80)])
def test_workspace_bytes_rejects(lib, V, nnz, flags):
    with pytest.raises(lib.BFSError) as e:
        lib.bfs_workspace_bytes(V, nnz, flags)
    assert e.value.code == lib.BFS_ERR_INVALID


def test_graph_create_argument_checks(lib):
    so = lib.load()
    h = ctypes.c_void_p(0)
    # NULL out-pointer, NULL offsets, NULL workspace, misaligned workspace
    assert so.bfs_graph_create(None, 10, 5, 1, 1, 256, 1 << 30, 0, None) == lib.BFS_ERR_INVALID
    assert so.bfs_graph_create(ctypes.byref(h), 10, 5, None, 1, 256, 1 << 30, 0, None) == lib.BFS_ERR_INVALID
    assert so.bfs_graph_create(ctypes.byref(h), 10, 5, 8, None, 256, 1 << 30, 0, None) == lib.BFS_ERR_INVALID
    assert so.bfs_graph_create(ctypes.byref(h), 10, 5, 8, 8, None, 1 << 30, 0, None) == lib.BFS_ERR_INVALID
    assert so.bfs_graph_create(ctypes.byref(h), 10, 5, 8, 8, 257, 1 << 30, 0, None) == lib.BFS_ERR_INVALID
    # workspace too small is reported before any device call
    assert so.bfs_graph_create(ctypes.byref(h), 10, 5, 8, 8, 256, 16, 0, None) == lib.BFS_ERR_WORKSPACE
    assert "workspace" in lib.bfs_last_error()


def test_no_device_reported(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    so = lib.load()
    h = ctypes.c_void_p(0)
    code = so.bfs_graph_create(ctypes.byref(h), 10, 5, 8, 8, 256, 1 << 30, 0, None)
    assert code == lib.BFS_ERR_NO_DEVICE


def test_null_handles(lib):
    so = lib.load()
    assert so.bfs_graph_destroy(None) == lib.BFS_OK
    assert so.bfs_run(None, 0, 8, None, None, None) == lib.BFS_ERR_INVALID
    roots = (ctypes.c_int32 * 1)(0)
    assert so.bfs_run_batch(None, roots, 1, 8, None, None) == lib.BFS_ERR_INVALID
    assert so.bfs_set_option(None, 1, 4) == lib.BFS_ERR_INVALID
    assert so.bfs_server_create(None, 256, 1 << 20, None) == lib.BFS_ERR_INVALID
    assert so.bfs_server_destroy(None) == lib.BFS_OK
    t = ctypes.c_uint64(0)
    assert so.bfs_submit(None, 0, 0, ctypes.byref(t)) == lib.BFS_ERR_INVALID
    assert so.bfs_poll(None, 1, None, None) == lib.BFS_ERR_INVALID
    assert so.bfs_server_drain(None) == lib.BFS_ERR_INVALID


def test_binding_has_no_cpu_fallback(lib, monkeypatch):
    """Without the built library the binding raises; nothing computes on the CPU."""
    import importlib
    from paper_1408_1605_amd import binding
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(ImportError):
        binding.load(os.path.join(ROOT, "does_not_exist.so"))
    importlib.reload(binding)


def test_package_does_not_import_oracle():
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r); import paper_1408_1605_amd; "
            "print('oracle' in sys.modules)") % ROOT
    out = subprocess.check_output([sys.executable, "-c", code], text=True).strip()
    assert out == "False"
    src = os.path.join(ROOT, "paper_1408_1605_amd")
    for dirpath, _, files in os.walk(src):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "bfs_oracle" not in text, f


def test_binding_structs_match_header(tmp_path):
    """Every ctypes struct of the binding has the C header's field offsets,
    field sizes and total size (gcc compiles a probe against include/bfs.h)."""
    import shutil
    import subprocess
    from paper_1408_1605_amd import binding
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    structs = [binding.bfs_stats, binding.bfs_server_config, binding.bfs_timing,
               binding.bfs_server_stats, binding.bfs_grid2d_stats]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "bfs.h"', 'int main(void) {']
    for S in structs:
        n = S.__name__
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (n, n))
        for f, _ in S._fields_:
            lines.append('printf("%s.%s %%zu %%zu\\n", offsetof(%s, %s), sizeof(((%s*)0)->%s));'
                         % (n, f, n, f, n, f))
    lines += ["return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    subprocess.run([gcc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict(l.split(" ", 1) for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                     text=True).stdout.splitlines())
    for S in structs:
        n = S.__name__
        assert int(got[n]) == ctypes.sizeof(S), n
        for f, _ in S._fields_:
            off, size = (int(x) for x in got["%s.%s" % (n, f)].split())
            desc = getattr(S, f)
            assert (off, size) == (desc.offset, desc.size), (n, f)


def test_noalloc_size_limit(lib):
    """bfs_run_noalloc's scratch is the plain workspace layout inside a
    32 MiB static array: the sizes its declaration promises fit, and an
    oversize input is refused before any device call."""
    limit = 32 << 20
    assert lib.bfs_workspace_bytes(524288, 1 << 28, 0) <= limit
    for V, nnz in [(1, 0), (1000, 10**6), (1 << 19, 1 << 24)]:
        assert lib.bfs_workspace_bytes(V, nnz, 0) <= 32.25 * V + nnz / 64 + 2.2e6
    so = lib.load()
    code = so.bfs_run_noalloc(1 << 22, 1 << 26, 256, 256, 0, 256, None, None, None)
    assert code == lib.BFS_ERR_WORKSPACE
    assert "static array" in lib.bfs_last_error()
    # argument checks come first
    assert so.bfs_run_noalloc(0, 0, 256, 256, 0, 256, None, None, None) == lib.BFS_ERR_INVALID
    assert so.bfs_run_noalloc(10, 5, None, 256, 0, 256, None, None, None) == lib.BFS_ERR_INVALID
    assert so.bfs_run_noalloc(10, 5, 256, 256, 10, 256, None, None, None) == lib.BFS_ERR_INVALID


def test_binding_constants_match_header(lib):
    # every BFS_* integer macro of the header has the same value in the
    # binding (status codes, flags, option keys)
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    defs = dict(re.findall(r"^\s*#define\s+(BFS_[A-Z0-9_]+)\s+(-?(?:0x)?[0-9a-fA-F]+)u?\s*$", text,
                           flags=re.M))
    assert "BFS_OPT_CLAIM_MODE" in defs and "BFS_ERR_TICKET" in defs
    for name, val in defs.items():
        assert hasattr(lib, name), name
        assert getattr(lib, name) == int(val, 0), name
