"""Host-side checks of the C ABI: exports, planner outputs, error codes.

No GPU is needed: planning, pair lists and footprints are host computations,
and argument errors are reported before any device call.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2201_06620_amd as rn
from workloads import configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    with open(os.path.join(ROOT, "include", "rn.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(rn_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = rn.lib()
    declared = header_functions()
    assert len(declared) >= 14
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(rn.EXPORTS) == sorted(declared)


def test_status_strings():
    for code in range(8):
        assert rn.lib().rn_status_str(code)


def test_plan_config1():
    p = configs.config1()
    cd, cg, ws, fl = rn.plan_block_tensordot(p.a.dims, p.a.grid, p.b.dims, p.b.grid,
                                             p.axes_a, p.axes_b, "fp64")
    assert cd == [2] * 16
    assert cg == [2, 2, 2] + [1] * 13
    assert fl == 8.0 * 2 ** 8 * 2 ** 8 * 2 ** 8
    # Both operands need a relayout into the GEMM layout (complex128).
    assert ws >= 2 * (2 ** 16) * 16


def test_pairs_config1():
    # A splits free axes 0-2, B splits contracted axes 0-2: after refinement
    # every C block couples 8 pairs; A's block is fixed by the C block and B's
    # block runs over its 8 stored blocks in the pairing order.
    p = configs.config1()
    for cb in range(8):
        pairs = rn.block_pairs(p.a.dims, p.a.grid, p.b.dims, p.b.grid, p.axes_a, p.axes_b, cb)
        assert len(pairs) == 8
        assert all(a == cb for a, _ in pairs)
        assert sorted(b for _, b in pairs) == list(range(8))


def test_pairs_match_brute_force():
    # Brute force over all block coordinates: pair (ia, ib) belongs to C block
    # c when their free coordinates match c's and their contracted
    # coordinates agree on the refined grid.
    da, ga = [2, 4, 2, 2], [2, 2, 1, 2]
    db, gb = [4, 2, 2], [4, 1, 2]
    axa, axb = [1, 3], [0, 2]
    cgrid = [2, 1]           # A free axes 0, 2 ; B free axis 1
    cgrid += [1]
    pairs = {}
    for c in range(int(np.prod(cgrid))):
        pairs[c] = rn.block_pairs(da, ga, db, gb, axa, axb, c)
    # Refined contracted grid: lcm(2, 4) = 4 on pair 0, lcm(2, 2) = 2 on pair 1.
    for c, lst in pairs.items():
        assert len(lst) == 4 * 2
        ca0, ca2, cb1 = np.unravel_index(c, cgrid)
        for p, (ia, ib) in enumerate(lst):
            r0, r1 = np.unravel_index(p, (4, 2))
            a_coord = np.unravel_index(ia, ga)
            b_coord = np.unravel_index(ib, gb)
            assert a_coord[0] == ca0 and a_coord[2] == ca2 and b_coord[1] == cb1
            assert a_coord[1] == r0 // 2 and a_coord[3] == r1
            assert b_coord[0] == r0 and b_coord[2] == r1


def test_footprint_equations_weak_scaling_shapes():
    # Section V.A shapes: blocks m_b = n_b = 2^14, k_b = 2^13 (complex64).
    for bk in (2, 4, 8, 16, 32):
        bm, bn = 8, 6
        e1, e2 = rn.block_footprint([2 ** 14 * bm, 2 ** 13 * bk], [bm, bk],
                                    [2 ** 14 * 8, 2 ** 13 * bk], [8, bk], [1], [1])
        assert e2 == 2 ** 13 * 2 ** 15 + 2 ** 28 == 2 ** 29        # 4 GiB complex64
        assert e1 == bk * 2 ** 13 * 2 ** 15 + 2 ** 28 == (bk + 1) * 2 ** 28
    # Capacity statement of Section II.C: order 33 fits 100 GB, order 34 not.
    assert (2 ** 33) * 8 < 100e9 < (2 ** 34) * 8


@pytest.mark.parametrize("kw,status", [
    (dict(axes_a=[0], axes_b=[5]), 1),                       # axis out of range
    (dict(axes_a=[0, 0], axes_b=[0, 1]), 1),                 # repeated axis
    (dict(dims_b=[4, 2, 2]), 2),                             # paired dims differ
    (dict(grid_a=[4, 1, 1]), 3),                             # grid above dim
    (dict(dims_a=[3, 2, 2], dims_b=[3, 2, 2]), 7),           # not a power of two
    (dict(grid_a=[1, 1, 1], dims_a=[2, 2, 2], mode="fp32_4m", dtype=2), 1),  # dtype/mode
    (dict(grid_a=[1, 1, 3], dims_a=[2, 2, 4], dims_b=[2, 2, 4]), 7),  # grid not a power of 2
    (dict(dims_a=[0, 2, 2]), 2),                             # empty axis
    (dict(dims_a=[2] * 21, grid_a=[1] * 21, dims_b=[2] * 21, grid_b=[1] * 21,
          axes_a=[], axes_b=[]), 7),                         # output above 2^40 entries
])
def test_plan_error_codes(kw, status):
    args = dict(dims_a=[2, 2, 2], grid_a=[1, 1, 1], dims_b=[2, 2, 2], grid_b=[1, 1, 1],
                axes_a=[0], axes_b=[0], mode="fp64", dtype=None)
    args.update(kw)
    dt = args.pop("dtype")
    mode = args.pop("mode")
    if dt is not None:
        A = rn.descriptor(args["dims_a"], args["grid_a"], dt)
        B = rn.descriptor(args["dims_b"], args["grid_b"], dt)
        aa = np.array(args["axes_a"], dtype=np.int32)
        bb = np.array(args["axes_b"], dtype=np.int32)
        st = rn.lib().rn_block_tensordot_plan(None, ctypes.byref(A), ctypes.byref(B), len(aa),
                                              aa.ctypes.data, bb.ctypes.data,
                                              rn.mode_id(mode), None, None, None)
        assert st == status
        return
    with pytest.raises(rn.RnError) as e:
        rn.plan_block_tensordot(args["dims_a"], args["grid_a"], args["dims_b"], args["grid_b"],
                                args["axes_a"], args["axes_b"], mode)
    assert e.value.status == status


def test_block_tensordot_rejects_null_handle():
    # Argument errors come back as status codes without touching a device.
    lib = rn.lib()
    A = rn.descriptor([2] * 4, None, rn.C128, 0x1000)
    B = rn.descriptor([2] * 4, None, rn.C128, 0x2000)
    axa = np.array([3, 1], dtype=np.int32)
    axb = np.array([0, 2], dtype=np.int32)
    C = rn.RnTensor()
    ws = ctypes.c_size_t()
    assert lib.rn_block_tensordot_plan(None, ctypes.byref(A), ctypes.byref(B), 2,
                                       axa.ctypes.data, axb.ctypes.data, 0, ctypes.byref(C),
                                       ctypes.byref(ws), None) == 0
    assert ws.value > 0
    C.data = 0x3000
    st = lib.rn_block_tensordot(None, ctypes.byref(A), ctypes.byref(B), 2, axa.ctypes.data,
                                axb.ctypes.data, ctypes.byref(C), 0, None, 0, None)
    assert st == 1  # RN_ERR_INVALID
    assert b"handle" in lib.rn_last_error()
    assert lib.rn_set_option(None, 1, 4) == 1
    v = ctypes.c_int64()
    assert lib.rn_get_option(None, 1, ctypes.byref(v)) == 1


def test_network_plan_config2_host():
    w = configs.config2()
    lib = rn.lib()
    n = len(w.network.tensors)
    Ts = (rn.RnTensor * n)()
    keep = []
    lab = (ctypes.c_void_p * n)()
    for i, l in enumerate(w.network.labels):
        Ts[i] = rn.descriptor([2] * len(l), None, rn.C128, 0x1000 + i)
        a = np.array(l, dtype=np.int32)
        keep.append(a)
        lab[i] = a.ctypes.data
    path = np.array([x for st in w.path for x in st], dtype=np.int32)
    sl = np.array(w.sliced, dtype=np.int32)
    ws, fl, mr = ctypes.c_size_t(), ctypes.c_double(), ctypes.c_int32()
    st = lib.rn_contract_network_plan(None, n, Ts, lab, len(w.path), path.ctypes.data, len(sl),
                                      sl.ctypes.data, 0, ctypes.byref(ws), ctypes.byref(fl),
                                      ctypes.byref(mr))
    assert st == 0, lib.rn_last_error()
    assert mr.value == w.meta["max_rank"]
    assert ws.value > 0 and fl.value > 0
    # A bad path is rejected.
    bad = path.copy()
    bad[1] = bad[0]
    st = lib.rn_contract_network_plan(None, n, Ts, lab, len(w.path), bad.ctypes.data, len(sl),
                                      sl.ctypes.data, 0, ctypes.byref(ws), ctypes.byref(fl),
                                      ctypes.byref(mr))
    assert st == 1


def test_batch_plan_empty_and_invalid_counts():
    # An empty batch plans to nothing (no flops, no workspace);
    # a negative count, or a positive one without descriptors, is refused.
    L = rn.lib()
    ws, fl = ctypes.c_size_t(), ctypes.c_double(-1.0)
    assert L.rn_block_tensordot_batch_plan(None, 0, None, None, None, None, None, 1, None,
                                           ctypes.byref(ws), ctypes.byref(fl)) == 0
    assert fl.value == 0.0 and ws.value == 0
    for n in (-1, 2):
        assert L.rn_block_tensordot_batch_plan(None, n, None, None, None, None, None, 1, None,
                                               ctypes.byref(ws), ctypes.byref(fl)) == 1
        assert b"batch" in L.rn_last_error()


def test_missing_library_fails_loudly():
    # No CPU fallback: without the built HIP library every entry point of the
    # binding raises instead of computing anything.
    import subprocess
    import sys
    code = ("import paper_2201_06620_amd as rn\n"
            "rn.LIB_PATH = '/nonexistent/librosnet.so'\n"
            "try:\n"
            "    rn.plan_block_tensordot([2, 2], None, [2, 2], None, [1], [0], 'fp64')\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n")
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       timeout=300, cwd=root)
    assert r.returncode == 0 and "raised:" in r.stdout and "no CPU fallback" in r.stdout
