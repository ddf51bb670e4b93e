"""CPU-only checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad arguments on the host before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tucker.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tucker_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_five_entry_points():
    names = _declared_functions()
    for n in ("tucker_sketch", "tucker_shifted_power", "tucker_core", "tucker_rthosvd", "tucker_rsthosvd"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2506_04840_amd import _lib
    for name in _declared_functions():
        assert hasattr(_lib.lib, name), name
        assert name in _lib.SIGNATURES, name


def test_info_struct_layout(tmp_path):
    """The binding's tucker_info matches the C header's: size and the offset of
    every field, as gcc lays the struct out."""
    import subprocess
    from paper_2506_04840_amd import _lib
    fields = [f[0] for f in _lib.Info._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "tucker.h"\nint main(void) {\n'
                   '  printf("%zu\\n", sizeof(tucker_info));\n'
                   + "".join('  printf("%%zu\\n", offsetof(tucker_info, %s));\n' % f for f in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(root, "include"), "-I/opt/rocm/include",
                        str(src), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got[0] == _lib.INFO_BYTES
    assert got[1:] == [getattr(_lib.Info, f).offset for f in fields]


def _ws(dims, ranks, p, q, prec, seq):
    from paper_2506_04840_amd import _lib
    return _lib.workspace_bytes(dims, ranks, p, q, prec, seq)


def test_workspace_query_and_validation():
    from paper_2506_04840_amd import _lib
    assert _ws((60, 60, 60), (10, 10, 10), 5, 1, _lib.FP64, False) > 0
    assert _ws((1000, 1000, 1000), (50, 50, 50), 10, 3, _lib.FP32, True) > 4e8
    # infeasible Tucker rank: r_3 = 32 > r_1 r_2 = 16 in ST
    assert _ws((40, 40, 40), (4, 4, 32), 2, 1, _lib.FP32, True) == 0
    # rank above the mode size, negative p, q too large, l too wide, bad order
    assert _ws((10, 10, 10), (11, 2, 2), 2, 1, _lib.FP32, True) == 0
    assert _ws((10, 10, 10), (2, 2, 2), -1, 1, _lib.FP32, True) == 0
    assert _ws((10, 10, 10), (2, 2, 2), 1, 17, _lib.FP32, True) == 0
    assert _ws((100, 100, 100), (60, 60, 60), 10, 1, _lib.FP32, True) == 0
    assert _ws((3,) * 9, (1,) * 9, 1, 1, _lib.FP32, True) == 0


def test_error_codes_before_any_launch():
    from paper_2506_04840_amd import _lib
    s = _lib._shape((10, 10, 10))
    r = (ctypes.c_int64 * 3)(2, 2, 2)
    rc = _lib.lib.tucker_rsthosvd(ctypes.byref(s), None, r, 2, 1, 0, 1, 1, None, None, None, None, 0, None)
    assert rc == -1
    assert "null" in _lib.lib.tucker_status_string(rc).decode()
    big = (ctypes.c_int64 * 3)(60, 60, 60)
    s2 = _lib._shape((100, 100, 100))
    rc = _lib.lib.tucker_rsthosvd(ctypes.byref(s2), ctypes.c_void_p(16), big, 10, 1, 0, 1, 1, ctypes.c_void_p(16),
                                  None, None, None, 0, None)
    assert rc == -4
    # workspace too small is reported as such
    rc = _lib.lib.tucker_sketch(ctypes.byref(s), 0, ctypes.c_void_p(16), 4, 1, 1, ctypes.c_void_p(16),
                                ctypes.c_void_p(16), 8, None)
    assert rc == -2
    # l above n
    rc = _lib.lib.tucker_sketch(ctypes.byref(s), 0, ctypes.c_void_p(16), 11, 1, 1, ctypes.c_void_p(16),
                                ctypes.c_void_p(16), 1 << 30, None)
    assert rc == -1
    rc = _lib.lib.tucker_core(ctypes.byref(s), 3, ctypes.c_void_p(16), ctypes.c_void_p(16), 2, 1,
                              ctypes.c_void_p(16), None)
    assert rc == -1
    rc = _lib.lib.tucker_orth(10, 11, ctypes.c_void_p(16), 0, ctypes.c_void_p(16), ctypes.c_void_p(16),
                              ctypes.c_void_p(16), 1 << 20, None)
    assert rc == -1
    rc = _lib.lib.tucker_fill_gaussian(1, 9, 0, 10, 10, 0, ctypes.c_void_p(16), None)
    assert rc == -1


def test_noalloc_entry_point_rejects_on_the_host():
    """tucker_rsthosvd_noalloc checks its arguments and the static scratch's
    size before it touches a device (nothing here needs a GPU)."""
    from paper_2506_04840_amd import _lib
    hdr = open(HEADER).read()
    m = re.search(r"#define TUCKER_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", hdr)
    assert m and int(m.group(1)) << int(m.group(2)) == _lib.NOALLOC_SCRATCH_BYTES
    s = _lib._shape((1000, 1000, 1000))
    r = (ctypes.c_int64 * 3)(50, 50, 50)
    assert _lib.workspace_bytes((1000,) * 3, (50,) * 3, 10, 3, _lib.FP32, True) > _lib.NOALLOC_SCRATCH_BYTES
    u = (ctypes.c_void_p * 3)(16, 16, 16)
    rc = _lib.lib.tucker_rsthosvd_noalloc(ctypes.byref(s), ctypes.c_void_p(16), r, 10, 3, 0, 1, _lib.FP32,
                                          ctypes.c_void_p(16), u, None, None)
    assert rc == -2
    assert "static scratch" in _lib.lib.tucker_status_string(rc).decode()
    bad = (ctypes.c_int64 * 3)(50, 50, 1001)
    rc = _lib.lib.tucker_rsthosvd_noalloc(ctypes.byref(s), ctypes.c_void_p(16), bad, 10, 3, 0, 1, _lib.FP32,
                                          ctypes.c_void_p(16), u, None, None)
    assert rc == -1
    rc = _lib.lib.tucker_rsthosvd_noalloc(None, None, r, 10, 3, 0, 1, _lib.FP32, None, None, None, None)
    assert rc == -1


def test_pve_entry_point_validates_on_the_host():
    """Algorithm 4's entry point rejects a bad q_max, tol or q_used before any
    device work."""
    import math
    from paper_2506_04840_amd import _lib
    L = _lib.lib
    s = _lib._shape((10, 10, 10))
    r = (ctypes.c_int64 * 3)(2, 2, 2)
    qu = (ctypes.c_int32 * 3)()
    p16 = ctypes.c_void_p(16)
    u = (ctypes.c_void_p * 3)(16, 16, 16)
    args = lambda qmax, tol, q: (ctypes.byref(s), p16, r, 2, qmax, ctypes.c_double(tol), 0, 1, 1, p16, u, None, q,
                                 p16, 1 << 30, None)
    assert L.tucker_rsthosvd_pve(*args(0, 0.5, qu)) == -1
    assert L.tucker_rsthosvd_pve(*args(_lib.MAX_Q_PVE + 1, 0.5, qu)) == -1
    assert L.tucker_rsthosvd_pve(*args(5, -0.1, qu)) == -1
    assert L.tucker_rsthosvd_pve(*args(5, math.nan, qu)) == -1
    assert L.tucker_rsthosvd_pve(*args(5, 0.5, None)) == -1
    assert "q_max" in L.tucker_status_string(L.tucker_rsthosvd_pve(*args(0, 0.5, qu))).decode()
    # the T-HOSVD form checks the same
    assert L.tucker_rthosvd_pve(*args(0, 0.5, qu)) == -1
    assert L.tucker_rthosvd_pve(*args(5, math.nan, qu)) == -1
    assert L.tucker_rthosvd_pve(*args(5, 0.5, None)) == -1


def test_processing_order_options_on_the_host():
    """The processing-order option: the workspace query follows the order
    (ST-HOSVD's intermediate sizes change with it, T-HOSVD's do not), and an
    order that is not a permutation, an unknown kind or nonzero reserved fields
    are rejected before any device work."""
    from paper_2506_04840_amd import _lib
    ws = lambda seq, **kw: _lib.workspace_bytes((60, 12, 40), (5, 6, 4), 4, 1, _lib.FP32, seq, _lib.make_options(**kw))
    nat = _lib.workspace_bytes((60, 12, 40), (5, 6, 4), 4, 1, _lib.FP32, True)
    assert nat > 0 and ws(True) == nat and ws(True, order=(0, 1, 2)) == nat
    assert ws(True, order="decreasing") == ws(True, order=(0, 2, 1))
    assert ws(True, order=(1, 2, 0)) > nat   # mode 1 first sketches a 12 x 2400 unfolding
    tn = _lib.workspace_bytes((60, 12, 40), (5, 6, 4), 4, 1, _lib.FP32, False)
    assert ws(False, order=(2, 1, 0)) == tn
    for kw in ({"order": (0, 0, 1)}, {"order": (0, 1, 3)}, {"order": (0, 1)}, {"order": (0, 1, 2, 3)}):
        assert ws(True, **kw) == 0, kw
    bad = _lib.make_options()
    bad.order_kind = 7
    assert _lib.workspace_bytes((60, 12, 40), (5, 6, 4), 4, 1, _lib.FP32, True, bad) == 0
    bad = _lib.make_options()
    bad.reserved[3] = 1
    assert _lib.workspace_bytes((60, 12, 40), (5, 6, 4), 4, 1, _lib.FP32, True, bad) == 0
    bad = _lib.make_options()
    bad.fp32_products = 2
    assert _lib.workspace_bytes((60, 12, 40), (5, 6, 4), 4, 1, _lib.FP32, True, bad) == 0
    native = _lib.make_options(fp32_products="native")
    assert _lib.workspace_bytes((60, 12, 40), (5, 6, 4), 4, 1, _lib.FP32, True, native) == nat
    L = _lib.lib
    s = _lib._shape((60, 12, 40))
    r = (ctypes.c_int64 * 3)(5, 6, 4)
    u = (ctypes.c_void_p * 3)(16, 16, 16)
    p16 = ctypes.c_void_p(16)
    opt = _lib.make_options(order=(2, 2, 0))
    rc = L.tucker_rsthosvd_ex(ctypes.byref(s), p16, r, 4, 1, 0, 1, 1, ctypes.byref(opt), p16, u, None, p16, 1 << 40,
                              None)
    assert rc == -1 and "permutation" in L.tucker_status_string(rc).decode()


def test_holistic_option_on_the_host():
    """The holistic variants size their own workspace (Q_k at width l_k, the
    small tensor and its HOSVD), reject a bad flag, and reject ranks that no
    unfolding of the small tensor can carry (T-HOSVD, p = 0: l = r, so mode 2's
    unfolding of the 1 x 1 x 3 tensor has rank 1)."""
    from paper_2506_04840_amd import _lib
    dims, ranks = (60, 12, 40), (5, 6, 4)
    plain = _lib.workspace_bytes(dims, ranks, 4, 1, _lib.FP32, True)
    hol = _lib.workspace_bytes(dims, ranks, 4, 1, _lib.FP32, True, _lib.make_options(holistic=True))
    assert hol > plain > 0
    # T-HOSVD: sequential modes (no per-mode scratch copies), plus the holistic buffers
    assert _lib.workspace_bytes(dims, ranks, 4, 1, _lib.FP32, False, _lib.make_options(holistic=True)) > 0
    bad = _lib.make_options()
    bad.holistic = 2
    assert _lib.workspace_bytes(dims, ranks, 4, 1, _lib.FP32, True, bad) == 0
    assert _lib.workspace_bytes((10, 10, 10), (1, 1, 3), 0, 1, _lib.FP64, False) > 0
    assert _lib.workspace_bytes((10, 10, 10), (1, 1, 3), 0, 1, _lib.FP64, False,
                                _lib.make_options(holistic=True)) == 0


def test_empty_and_oversized_shapes_rejected():
    """A zero-size mode, order 0 and order above TUCKER_MAX_ORDER are rejected by
    the workspace query (and by the solves, which share the plan)."""
    from paper_2506_04840_amd import _lib
    assert _lib.workspace_bytes((10, 0, 10), (2, 1, 2), 4, 1, _lib.FP64, True) == 0
    assert _lib.workspace_bytes((), (), 4, 1, _lib.FP64, True) == 0
    assert _lib.workspace_bytes((2,) * 9, (1,) * 9, 0, 1, _lib.FP64, True) == 0
    assert _lib.workspace_bytes((2,) * 8, (1,) * 8, 0, 1, _lib.FP64, True) > 0
    s = _lib._shape((10, 0, 10))
    r = (ctypes.c_int64 * 3)(2, 1, 2)
    u = (ctypes.c_void_p * 3)(16, 16, 16)
    rc = _lib.lib.tucker_rsthosvd(ctypes.byref(s), ctypes.c_void_p(16), r, 2, 1, 0, 1, 1, ctypes.c_void_p(16), u,
                                  None, ctypes.c_void_p(16), 1 << 30, None)
    assert rc == -1


def test_python_binding_rejects_host_tensors():
    import torch
    from paper_2506_04840_amd import _lib
    with pytest.raises(ValueError):
        _lib._dev(torch.zeros(3), "X")


def _fake_item(dims, ranks, seed=1):
    from paper_2506_04840_amd import _lib
    it = _lib.BatchItem()
    it.shape = _lib._shape(dims)
    for k, r in enumerate(ranks):
        it.ranks[k] = r
    it.seed = seed
    it.A, it.G = 4096, 8192
    for k in range(len(dims)):
        it.U[k] = 12288 + 4096 * k
    it.info = None
    return it


def test_batch_plan_on_the_host():
    """tucker_batch_plan is host-only: it validates, carves the workspace and
    writes the plan without touching device memory (fake addresses here)."""
    from paper_2506_04840_amd import _lib
    L = _lib.lib
    cap, d, q, p = 8, 3, 1, 8
    nplan = L.tucker_batch_plan_bytes(cap, d, q)
    ntab = L.tucker_batch_table_bytes(cap, d, q)
    assert nplan > ntab > 0
    assert L.tucker_batch_plan_bytes(0, d, q) == 0 and L.tucker_batch_plan_bytes(cap, 9, q) == 0
    items = (_lib.BatchItem * cap)(*[_fake_item((40 + i, 50, 33 + 2 * i), (10 - i, 6, 4 + i)) for i in range(3)])
    need = ntab + sum(L.tucker_batch_item_bytes(ctypes.byref(items[i]), p, q) for i in range(3))
    plan = ctypes.create_string_buffer(nplan)
    ws = ctypes.c_void_p(1 << 40)
    ok = L.tucker_batch_plan(cap, d, 48, 3, items, p, q, 0, ws, need, plan, nplan)
    assert ok == 0, L.tucker_status_string(ok)
    # an empty batch plans too (the launch sequence is the same)
    assert L.tucker_batch_plan(cap, d, 48, 0, items, p, q, 0, ws, need, plan, nplan) == 0
    # workspace one byte short, plan buffer short, lclass too narrow, bad lclass, order mismatch
    assert L.tucker_batch_plan(cap, d, 48, 3, items, p, q, 0, ws, need - 1, plan, nplan) == -2
    assert L.tucker_batch_plan(cap, d, 48, 3, items, p, q, 0, ws, need, plan, nplan - 1) == -2
    assert L.tucker_batch_plan(cap, d, 16, 3, items, p, q, 0, ws, need, plan, nplan) == -4
    assert L.tucker_batch_plan(cap, d, 40, 3, items, p, q, 0, ws, need, plan, nplan) == -1
    n4 = L.tucker_batch_plan_bytes(cap, 4, q)
    plan4 = ctypes.create_string_buffer(n4)
    assert L.tucker_batch_plan(cap, 4, 48, 3, items, p, q, 0, ws, 1 << 30, plan4, n4) == -1
    assert L.tucker_batch_plan(cap, d, 48, cap + 1, items, p, q, 0, ws, need, plan, nplan) == -1
    # infeasible rank inside a batch is rejected like in tucker_rsthosvd
    bad = (_lib.BatchItem * 1)(_fake_item((40, 40, 40), (4, 4, 32)))
    assert L.tucker_batch_plan(cap, d, 48, 1, bad, p, q, 0, ws, 1 << 30, plan, nplan) == -1


def test_serving_width_class_choice():
    """A request goes to the smallest width class holding every sketch width
    min(r_k + p, n_k); wider than 64 is refused."""
    import types

    import torch

    from paper_2506_04840_amd import serve
    srv = types.SimpleNamespace(p=8, classes=serve.BatchServer.CLASSES)

    def key(dims, ranks):
        j = serve.Job(0, torch.zeros(dims), ranks, 1, 0.0)
        return serve.BatchServer.key_of(srv, j)

    assert key((40, 50, 60), (4, 5, 8)) == (3, 16)
    assert key((40, 50, 60), (4, 9, 8)) == (3, 32)
    assert key((12, 50, 60), (10, 20, 24)) == (3, 32)    # min(10 + 8, 12) = 12, 28, 32
    assert key((40, 50, 60), (4, 30, 8)) == (3, 48)
    assert key((100, 90, 80, 70), (50, 2, 2, 2)) == (4, 64)
    with pytest.raises(ValueError):
        key((100, 90, 80), (60, 2, 2))
