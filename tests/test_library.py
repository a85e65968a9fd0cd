"""Host-side checks of the HIP library that need no GPU: the shared library
loads and exports every entry point include/bdl.h declares, and the header
and binding agree on constants and the node layout."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bdl.h")
HEADERS = [os.path.join(ROOT, "include", h) for h in ("bdl.h", "bdl_server.h")]
LIB = os.path.join(ROOT, "paper_2112_06188_amd", "libbdl.so")


def _declared():
    src = "".join(open(h).read() for h in HEADERS)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(bdl_[a-z_]+)\s*\(", src))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2112_06188_amd import build_lib
        build_lib.build()
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    names = _declared()
    assert {"bdl_create", "bdl_insert", "bdl_erase", "bdl_knn", "bdl_destroy"} <= names
    for n in sorted(names):
        assert hasattr(lib, n), f"libbdl.so does not export {n}"
    import paper_2112_06188_amd as pkg
    assert set(pkg.EXPORTS) == names


def test_header_constants_match_binding():
    import paper_2112_06188_amd as pkg
    src = open(HEADER).read()
    consts = dict(re.findall(r"#define (BDL_[A-Z_]+) \(?(-?\w+)\)?", src))
    assert int(consts["BDL_OK"]) == pkg.BDL_OK
    assert int(consts["BDL_EINVAL"]) == pkg.BDL_EINVAL
    assert int(consts["BDL_ENOMEM"]) == pkg.BDL_ENOMEM
    assert int(consts["BDL_EHIP"]) == pkg.BDL_EHIP
    assert int(consts["BDL_MAX_DIM"]) == pkg.MAX_DIM
    assert int(consts["BDL_MAX_K"]) == pkg.MAX_K
    assert int(consts["BDL_INVALID_ID"].rstrip("u"), 16) == pkg.INVALID_ID


def test_node_export_layout_matches_oracle_layout():
    import oracle
    import paper_2112_06188_amd as pkg
    assert pkg.NODE_DTYPE.itemsize == 176
    assert pkg.NODE_DTYPE.names == oracle.NODE_DTYPE.names
    for f in pkg.NODE_DTYPE.names:
        assert pkg.NODE_DTYPE.fields[f][1] == oracle.NODE_DTYPE.fields[f][1]


def test_binding_fails_loudly_without_gpu():
    import torch
    import paper_2112_06188_amd as pkg
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        pkg.Tree(3)


def test_create_rejects_bad_config_before_touching_the_gpu(lib):
    """Argument errors are detected on the host (no device call needed)."""
    import paper_2112_06188_amd as pkg
    L = pkg.load_library()
    h = ctypes.c_void_p()
    for cfg in (pkg.Config(0, 16, 1024, 100, 0, 0), pkg.Config(17, 16, 1024, 100, 0, 0),
                pkg.Config(3, 0, 1024, 100, 0, 0), pkg.Config(3, 16, 0, 100, 0, 0),
                pkg.Config(3, 16, 1024, 0, 0, 0)):
        assert L.bdl_create(ctypes.byref(cfg), None, ctypes.byref(h)) == pkg.BDL_EINVAL
        assert L.bdl_last_error()
    assert L.bdl_insert(None, None, None, 5) == pkg.BDL_EINVAL
    assert L.bdl_knn(None, None, 5, 3, None, None) == pkg.BDL_EINVAL


def test_veb_key_host_matches_treecheck_formula():
    """The vEB index the GPU layout sorts by (a header-only helper) agrees with
    the independent formula of the tests, checked through a tiny host build
    of the same header."""
    import subprocess
    import tempfile
    from treecheck import veb_key
    src = r'''
#define __HIP_PLATFORM_AMD__ 1
#include <cstdio>
#include <cstdint>
#include "bdl_common.hpp"
int main() {
  for (int H = 1; H <= 12; ++H)
    for (int dep = 0; dep < H; ++dep)
      for (uint64_t p = 0; p < (1ull << dep); ++p)
        std::printf("%d %d %llu %llu\n", H, dep, (unsigned long long)p,
                    (unsigned long long)bdl::veb_key(H, dep, p));
  const int Hs[] = {33, 40, 57, 64};
  for (int H : Hs) {
    uint64_t paths[] = {0ull, 1ull, 0x5555ull, 0x123456789abcull};
    for (uint64_t p : paths) {
      int dep = H - 1;
      uint64_t pp = dep >= 64 ? p : (p & ((1ull << dep) - 1));
      std::printf("%d %d %llu %llu\n", H, dep, (unsigned long long)pp,
                  (unsigned long long)bdl::veb_key(H, dep, pp));
    }
  }
}
'''
    with tempfile.TemporaryDirectory() as td:
        cpp = os.path.join(td, "k.cpp")
        exe = os.path.join(td, "k")
        open(cpp, "w").write(src)
        r = subprocess.run(["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-arch=gfx950", "-O1",
                            "-I", os.path.join(ROOT, "paper_2112_06188_amd", "csrc"), cpp,
                            "-o", exe], capture_output=True, text=True)
        if r.returncode != 0:
            pytest.skip(f"host build of the header helper failed: {r.stderr[-400:]}")
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    for line in out.strip().splitlines():
        H, dep, p, k = (int(x) for x in line.split())
        assert k == veb_key(H, dep, p), (H, dep, p)


def test_abi_struct_layouts_match_header():
    """The ctypes mirrors of the structs in bdl.h have the C compiler's sizes
    and field offsets (a host C build of the header prints them)."""
    import subprocess
    import tempfile
    import paper_2112_06188_amd as pkg
    structs = {"bdl_config": pkg.Config, "bdl_profile_t": pkg.Profile,
               "bdl_knn_request": pkg.KnnRequest, "bdl_knn_shape": pkg.KnnShape,
               "bdl_server_config": pkg.ServerConfig, "bdl_request": pkg.Request,
               "bdl_completion": pkg.Completion}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bdl_server.h"',
             "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "l.c")
        exe = os.path.join(td, "l")
        open(c, "w").write("\n".join(lines) + "\n")
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe],
                       check=True, capture_output=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    seen = 0
    for line in out.strip().splitlines():
        cname, field, val = line.split()
        py = structs[cname]
        want = ctypes.sizeof(py) if field == "sizeof" else getattr(py, field).offset
        assert int(val) == want, (cname, field)
        seen += 1
    assert seen == sum(len(p._fields_) + 1 for p in structs.values())


def test_shape_table_rejects_bad_rows_on_the_host(lib):
    import paper_2112_06188_amd as pkg
    L = pkg.load_library()
    assert L.bdl_set_knn_shapes(None, None, 0) == pkg.BDL_EINVAL
    assert L.bdl_set_param(None, pkg.PARAM_PERSISTENT, 1) == pkg.BDL_EINVAL


def test_server_rejects_bad_arguments_on_the_host(lib):
    import paper_2112_06188_amd as pkg
    L = pkg.load_library()
    h = ctypes.c_void_p()
    cfg = pkg.ServerConfig(1, 16, 64, 2, 1 << 20, 0)
    assert L.bdl_server_create(None, ctypes.byref(cfg), ctypes.byref(h)) == pkg.BDL_EINVAL
    assert L.bdl_server_submit(None, None, None) == pkg.BDL_EINVAL
    assert L.bdl_server_drain(None) == pkg.BDL_EINVAL
