"""CPU-side checks of the C ABI: the library loads and exports every function
include/fsc.h declares, and the binding names match (no GPU calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2310_10939_amd", "libfsc.so")
HDR = os.path.join(ROOT, "include", "fsc.h")


def declared_functions():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fsc_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["fsc_create", "fsc_destroy", "fsc_embed", "fsc_cluster", "fsc_kmeans", "fsc_ari", "fsc_nmi",
                 "fsc_cluster_batched", "fsc_autotune", "fsc_tuning_set", "fsc_timing_enable",
                 "fsc_timing_read", "fsc_last_error", "fsc_version"]:
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfsc.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (fsc_\w+)", out))
    assert exported == set(declared_functions())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfsc.so not built")
def test_binding_covers_the_exports_and_needs_no_gpu_to_load():
    from paper_2310_10939_amd import fsc
    assert set(fsc.EXPORTS) == set(declared_functions())
    assert fsc.version() == (1, 0)
    # the message is per thread: a thread that made no call has none, whatever
    # tests ran before this one
    import threading
    seen = []
    th = threading.Thread(target=lambda: seen.append(fsc._lib.fsc_last_error()))
    th.start()
    th.join()
    assert seen == [b""]


def test_struct_layouts_match_header(tmp_path):
    """Every field offset and struct size of the binding's ctypes mirrors
    equals what a C compiler makes of include/fsc.h."""
    from paper_2310_10939_amd import fsc
    structs = {"fsc_csr": fsc.Csr, "fsc_opts": fsc.Opts, "fsc_tuning": fsc.Tuning}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "fsc.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)
