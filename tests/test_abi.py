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


def test_struct_layouts_match_header():
    from paper_2310_10939_amd import fsc
    # int64 n, nnz, 3 pointers, int32 dtype (+pad) ; opts: 4 int32, 3 pointers, int32 (+pad)
    assert ctypes.sizeof(fsc.Csr) == 8 * 5 + 8
    assert ctypes.sizeof(fsc.Opts) == 4 * 4 + 8 * 3 + 8
    assert ctypes.sizeof(fsc.Tuning) == 6 * 4
