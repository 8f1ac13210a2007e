"""C-ABI checks that need no GPU: the library loads, exports what include/kohler.h declares, and the
host-side argument checks answer without touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kohler.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\w[\w\s\*]*?\b(kohler_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1707_05062_amd import _lib
    return _lib.load()


def test_header_declares_expected_api():
    from paper_1707_05062_amd import _lib
    assert declared_functions() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strerror(lib):
    for st in (0, -1, -2, -3, -4, -5, -6, -7):
        assert lib.kohler_strerror(st)
    assert lib.kohler_strerror(12345) == b"unknown status"


def test_host_argument_checks_without_device(lib):
    from paper_1707_05062_amd import _lib
    # NULL out-pointer and NULL contexts are rejected before any HIP call
    assert lib.kohler_create(None, 0) == _lib.E_ARG
    i64 = ctypes.c_int64(0)
    i32 = ctypes.c_int32(0)
    d = ctypes.c_double(0)
    st = lib.kohler_curve(None, ctypes.c_void_p(1), 1, 4, 4, 4, 256, 4, ctypes.byref(i64),
                          ctypes.byref(i64), ctypes.byref(d), None, 0, ctypes.byref(i32), ctypes.byref(i32))
    assert st == _lib.E_ARG
    st = lib.kohler_curve_async(None, ctypes.c_void_p(1), 1, 4, 4, 4, 256, 4, *([ctypes.c_void_p(8)] * 4),
                                0, *([ctypes.c_void_p(8)] * 3), None)
    assert st == _lib.E_ARG
    pl = _lib.Plan()
    assert lib.kohler_get_plan(None, 1, 4, 4, 256, 4, ctypes.byref(pl)) == _lib.E_ARG
    assert lib.kohler_set_plan(None, 1, 256, 4, ctypes.byref(pl)) == _lib.E_ARG
    lib.kohler_destroy(None)  # no-op


def test_header_constants_match_binding():
    from paper_1707_05062_amd import _lib
    text = open(HEADER).read()
    m = re.search(r"#define KOHLER_MAX_M_U16 (\d+)", text)
    assert int(m.group(1)) == _lib.MAX_M_U16
    for name, val in [("KOHLER_OK", 0), ("KOHLER_E_ARG", -1), ("KOHLER_E_RANGE", -2),
                      ("KOHLER_E_CAPACITY", -3), ("KOHLER_E_NOMEM", -4), ("KOHLER_E_DEVICE", -5),
                      ("KOHLER_E_BUSY", -6), ("KOHLER_E_CANCELED", -7), ("KOHLER_U8", 1),
                      ("KOHLER_U16", 2)]:
        assert re.search(rf"{name}\s*=\s*{val}\b", text), name


def test_serving_and_tuning_argument_checks_without_device(lib):
    from paper_1707_05062_amd import _lib
    cfg = _lib.ServerConfig(1, 256, 4, 4, 1, 4, 16, 16, 1, 0, 1 << 28)
    h = ctypes.c_void_p()
    assert lib.kohler_server_create(None, ctypes.byref(cfg), ctypes.byref(h)) == _lib.E_ARG
    assert lib.kohler_server_create(None, ctypes.byref(cfg), None) == _lib.E_ARG
    t = ctypes.c_uint64(0)
    assert lib.kohler_server_submit(None, ctypes.c_void_p(1), 4, 4, 4, ctypes.byref(t)) == _lib.E_ARG
    assert lib.kohler_server_poll(None, 1) == _lib.E_ARG
    assert lib.kohler_server_wait(None, 1, None, None, None, None, 0, None) == _lib.E_ARG
    assert lib.kohler_server_cancel(None, 1) == _lib.E_ARG
    assert lib.kohler_server_pause(None, 1) == _lib.E_ARG
    assert lib.kohler_server_stats(None, None) == _lib.E_ARG
    lib.kohler_server_destroy(None)  # no-op
    pl = _lib.Plan()
    us = ctypes.c_double(0)
    assert lib.kohler_autotune(None, 1, None, None, None, None, 1, 256, 4, 5, ctypes.byref(pl),
                               ctypes.byref(us)) == _lib.E_ARG


def test_segmentation_consumers_reject_null_context(lib):
    from paper_1707_05062_amd import _lib
    v = ctypes.c_void_p(16)
    assert lib.kohler_segment(None, v, 1, 4, 4, 4, 256, v, v, 4, v, 1, 4, None) == _lib.E_ARG
    assert lib.kohler_class_stats(None, v, 1, 4, 4, 4, 256, v, v, 4, v, v, v, None) == _lib.E_ARG
    assert lib.kohler_mean_image(None, v, 1, 4, 4, 4, 256, v, v, 4, v, v, 4, None) == _lib.E_ARG
    assert lib.kohler_top_thresholds(None, v, v, 256, v, v, 4, 2, v, v, None) == _lib.E_ARG
    text = open(HEADER).read()
    assert re.search(r"#define KOHLER_MAX_CLASS_THRESHOLDS (\d+)", text)


def _c_struct_fields(name):
    """(type, field) pairs of a typedef struct in the header, in order."""
    text = open(HEADER).read()
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), text, flags=re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ty, names = decl.split(None, 1)
        out += [(ty, n.strip()) for n in names.split(",")]
    return out


@pytest.mark.parametrize("cname,pyname", [("kohler_plan", "Plan"), ("kohler_server_config", "ServerConfig"),
                                          ("kohler_request_info", "RequestInfo"),
                                          ("kohler_server_counters", "ServerCounters")])
def test_struct_layouts_match_header(cname, pyname):
    from paper_1707_05062_amd import _lib
    fields = _c_struct_fields(cname)
    py = getattr(_lib, pyname)
    assert [n for _, n in fields] == [n for n, _ in py._fields_]
    sizes = {"int32_t": 4, "int64_t": 8}
    for (ty, n), (pn, pty) in zip(fields, py._fields_):
        assert sizes[ty] == ctypes.sizeof(pty), (cname, n)
