"""CPU checks of the C ABI: the library loads and exports every function that
include/*.h declares; host-side argument errors are returned without a device."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"\b(superdc_[a-z0-9_]+)\s*\(", src):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_four_calls():
    names = declared_functions()
    for n in ("superdc_secular_solve", "superdc_loewner", "superdc_cauchy_apply",
              "superdc_secular_backward"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2108_04209_amd import native
    lib = native.load_library()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_no_device_or_bad_args_fail_cleanly():
    """Without a GPU the context cannot be created; NULL arguments are rejected."""
    from paper_2108_04209_amd import native
    lib = native.load_library()
    assert lib.superdc_create(None) == -1
    assert lib.superdc_batch_create(None, 1, None, None) == -1
    assert lib.superdc_secular_solve(None, None, None, None, None, None, None, None, None, None,
                                     None, None) == -1
    assert lib.superdc_deflate(None, None, None, None, None, 1e-10, None, None, None, None,
                               None, None, None, None, None, None) == -1
    assert lib.superdc_deflate_expand(None, None, None, None, None, None, None, 0, 1, None, 1,
                                      None, 1, None) == -1
    assert lib.superdc_batch_copy_rows(None, None, None, None, 1, None, 1, None, 1, None,
                                       None) == -1
    assert lib.superdc_hss_divide(None, None, None, None, None, None, 1, None, None, None,
                                  None) == -1
    o = native.default_opts()
    assert o.stop_c == 1.0 and o.max_iter == 40 and o.persistent == 1
    assert lib.superdc_strerror(-4) == b"no gfx950 device"


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU may be present")
def test_create_without_device():
    from paper_2108_04209_amd import native
    h = ctypes.c_void_p()
    rc = native.load_library().superdc_create(ctypes.byref(h))
    assert rc == -4
