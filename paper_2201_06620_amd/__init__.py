"""Python binding of the MI355X block tensor contraction library (librosnet.so).

Argument marshalling only: every step of the contraction runs in the HIP
kernels behind the C ABI declared in include/rn.h.  PyTorch supplies device
memory and the current stream; there is no CPU fallback, and loading fails
loudly when the built library is missing.

Operand tensors are torch complex tensors on a GPU holding the stored
(block-major) buffer; their logical dims and grid are passed separately.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librosnet.so")
RN_MAX_RANK = 64
RN_MAX_SLICED = 15

MODES = {"fp64": 0, "fp32_4m": 1, "fp32_3m": 2, "bf16x3": 3}
C64, C128 = 1, 2
STATUS = {0: "RN_OK", 1: "RN_ERR_INVALID", 2: "RN_ERR_SHAPE", 3: "RN_ERR_GRID",
          4: "RN_ERR_WORKSPACE", 5: "RN_ERR_OOM", 6: "RN_ERR_HIP", 7: "RN_ERR_UNSUPPORTED"}

EXPORTS = ["rn_create", "rn_destroy", "rn_status_str", "rn_last_error",
           "rn_block_tensordot_plan", "rn_block_tensordot", "rn_block_pairs",
           "rn_block_footprint", "rn_block_tensordot_batch_plan", "rn_block_tensordot_batch",
           "rn_contract_network_plan", "rn_contract_network", "rn_norm2", "rn_sum_c128",
           "rn_profile_enable", "rn_profile_read", "rn_autotune_batch", "rn_tune_save",
           "rn_tune_load", "rn_tune_clear", "rn_tile_count", "rn_set_graphs", "rn_server_create",
           "rn_server_submit", "rn_server_poll", "rn_server_wait", "rn_server_stats",
           "rn_server_destroy", "rn_set_option", "rn_get_option",
           "rn_block_tensordot_streamed_plan", "rn_block_tensordot_streamed",
           "rn_block_tensordot_noalloc", "rn_server_set_admission", "rn_network_prepare",
           "rn_network_execute", "rn_network_release"]

# Handle options (rn_option).
OPTIONS = {"graphs": 0, "pair_split_threshold": 1, "split_footprint": 2, "slice_sum": 3,
           "batched_slice_bits": 4, "network_footprint": 5}


class RnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class RnResult(ctypes.Structure):
    _fields_ = [("amp", ctypes.c_double * 2), ("latency_s", ctypes.c_double),
                ("queue_s", ctypes.c_double), ("run_s", ctypes.c_double),
                ("footprint_bytes", ctypes.c_double), ("status", ctypes.c_int32),
                ("start_s", ctypes.c_double), ("done_s", ctypes.c_double)]


class RnTensor(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("dims", ctypes.c_int64 * RN_MAX_RANK), ("grid", ctypes.c_int32 * RN_MAX_RANK),
                ("data", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python paper_2201_06620_amd/build.py` (no CPU fallback exists)")
        # PyTorch brings its own HIP runtime; load it first so that the
        # library binds to that same runtime instead of a second copy.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        p, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        T = ctypes.POINTER(RnTensor)
        pp = ctypes.POINTER(ctypes.c_void_p)
        L.rn_create.argtypes = [ctypes.POINTER(p), ctypes.c_int]
        L.rn_destroy.argtypes = [p]
        L.rn_status_str.argtypes = [ctypes.c_int]
        L.rn_status_str.restype = ctypes.c_char_p
        L.rn_last_error.argtypes = []
        L.rn_last_error.restype = ctypes.c_char_p
        L.rn_block_tensordot_plan.argtypes = [p, T, T, i32, p, p, ctypes.c_int, T,
                                              ctypes.POINTER(sz), ctypes.POINTER(ctypes.c_double)]
        L.rn_block_tensordot.argtypes = [p, T, T, i32, p, p, T, ctypes.c_int, p, sz, p]
        L.rn_block_tensordot_noalloc.argtypes = [p, T, T, i32, p, p, T, ctypes.c_int, p]
        L.rn_block_pairs.argtypes = [p, T, T, i32, p, p, i64, p, i64, ctypes.POINTER(i64)]
        L.rn_block_footprint.argtypes = [T, T, i32, p, p, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]
        L.rn_block_tensordot_batch_plan.argtypes = [p, i32, T, T, p, pp, pp, ctypes.c_int, T,
                                                    ctypes.POINTER(sz),
                                                    ctypes.POINTER(ctypes.c_double)]
        L.rn_block_tensordot_batch.argtypes = [p, i32, T, T, p, pp, pp, T, ctypes.c_int, p, sz, p]
        L.rn_contract_network_plan.argtypes = [p, i32, T, pp, i32, p, i32, p, ctypes.c_int,
                                               ctypes.POINTER(sz), ctypes.POINTER(ctypes.c_double),
                                               ctypes.POINTER(i32)]
        L.rn_contract_network.argtypes = [p, i32, T, pp, i32, p, i32, p, ctypes.c_int, p, sz, p,
                                          p, p]
        L.rn_network_prepare.argtypes = [p, i32, T, pp, i32, p, i32, p, ctypes.c_int,
                                         ctypes.POINTER(p), ctypes.POINTER(sz)]
        L.rn_network_execute.argtypes = [p, p, sz, p, p, p]
        L.rn_network_release.argtypes = [p]
        L.rn_norm2.argtypes = [p, T, p, p]
        L.rn_sum_c128.argtypes = [p, i64, p, p, p]
        L.rn_profile_enable.argtypes = [p, ctypes.c_int]
        L.rn_autotune_batch.argtypes = [p, i32, T, T, p, pp, pp, T, ctypes.c_int, p, sz, p]
        L.rn_tune_save.argtypes = [p, ctypes.c_char_p]
        L.rn_tune_load.argtypes = [p, ctypes.c_char_p]
        L.rn_tune_clear.argtypes = [p]
        L.rn_tile_count.argtypes = [ctypes.c_int]
        L.rn_set_graphs.argtypes = [p, ctypes.c_int]
        L.rn_set_option.argtypes = [p, ctypes.c_int, i64]
        L.rn_block_tensordot_streamed_plan.argtypes = [p, T, T, i32, p, p, ctypes.c_int, T,
                                                       ctypes.POINTER(sz),
                                                       ctypes.POINTER(ctypes.c_double),
                                                       ctypes.POINTER(ctypes.c_double)]
        L.rn_block_tensordot_streamed.argtypes = [p, T, T, i32, p, p, T, ctypes.c_int, p, sz, p]
        L.rn_get_option.argtypes = [p, ctypes.c_int, ctypes.POINTER(i64)]
        L.rn_server_create.argtypes = [ctypes.c_int, sz, i32, ctypes.POINTER(p)]
        L.rn_server_submit.argtypes = [p, i32, T, pp, i32, p, i32, p, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_uint64)]
        L.rn_server_set_admission.argtypes = [p, i32, i32]
        L.rn_server_poll.argtypes = [p, ctypes.c_uint64, ctypes.POINTER(i32),
                                     ctypes.POINTER(RnResult)]
        L.rn_server_wait.argtypes = [p, ctypes.c_uint64, ctypes.POINTER(RnResult)]
        L.rn_server_stats.argtypes = [p, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                      ctypes.POINTER(i64), ctypes.POINTER(sz)]
        L.rn_server_destroy.argtypes = [p]
        L.rn_profile_read.argtypes = [p, p, p]
        for name in EXPORTS:
            getattr(L, name).restype = getattr(L, name).restype if name in (
                "rn_status_str", "rn_last_error") else ctypes.c_int
        _lib = L
    return _lib


def check(status: int, what: str = "") -> None:
    if status != 0:
        msg = lib().rn_last_error().decode()
        raise RnError(status, f"{what}: {msg}" if what else msg)


def descriptor(dims, grid=None, dtype=C128, data=None) -> RnTensor:
    t = RnTensor()
    dims = [int(d) for d in dims]
    if len(dims) > RN_MAX_RANK:
        raise ValueError("rank above RN_MAX_RANK")
    grid = [1] * len(dims) if grid is None else [int(g) for g in grid]
    t.rank = len(dims)
    t.dtype = dtype
    for j, (d, g) in enumerate(zip(dims, grid)):
        t.dims[j] = d
        t.grid[j] = g
    t.data = data
    return t


def _arr32(x):
    a = np.ascontiguousarray(np.asarray(list(x), dtype=np.int32).reshape(-1))
    return a, (a.ctypes.data if a.size else None)


def _axes(axes_a, axes_b):
    """Paired contracted axes as int32 arrays and their pointers; the library
    reads k = len(axes_a) entries of each, so the lengths must agree."""
    aa, pa = _arr32(axes_a)
    ab, pb = _arr32(axes_b)
    if len(aa) != len(ab):
        raise RnError(1, f"{len(aa)} axes of A paired with {len(ab)} axes of B")
    return aa, pa, ab, pb


def _check_tensor(t, name, dtype=None, numel=None, min_numel=None, device=None, on_gpu=True):
    """Raise RnError(RN_ERR_INVALID) unless t is a contiguous torch tensor of
    this dtype and element count on GPU `device` (every check is made before
    a pointer is handed to the library, so a wrong buffer never reaches a
    kernel)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise RnError(1, f"{name}: expected a torch tensor, got {type(t).__name__}")
    if dtype is not None and t.dtype != dtype:
        raise RnError(1, f"{name}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise RnError(1, f"{name}: not contiguous")
    if numel is not None and t.numel() != numel:
        raise RnError(1, f"{name}: {t.numel()} elements, expected {numel}")
    if min_numel is not None and t.numel() < min_numel:
        raise RnError(1, f"{name}: {t.numel()} elements, at least {min_numel} needed")
    if not on_gpu:
        return
    if not t.is_cuda:
        raise RnError(1, f"{name}: not on the GPU")
    if device is not None and t.device.index != device:
        raise RnError(1, f"{name}: on cuda:{t.device.index}, the handle is on cuda:{device}")


def _numel(dims) -> int:
    return math.prod(int(d) for d in dims)


def _torch_dtype(mode):
    import torch
    return torch.complex128 if dtype_of_mode(mode) == C128 else torch.complex64


def tile_count(mode) -> int:
    """Number of GEMM tile shapes of a mode (the autotuner's candidates)."""
    return int(lib().rn_tile_count(mode_id(mode)))


def mode_id(mode) -> int:
    return MODES[mode] if isinstance(mode, str) else int(mode)


def dtype_of_mode(mode) -> int:
    return C128 if mode_id(mode) == 0 else C64


# ------------------------------------------------------------- host-only

def plan_block_tensordot(dims_a, grid_a, dims_b, grid_b, axes_a, axes_b, mode="fp64"):
    """(C dims, C grid, workspace bytes, useful flops) of a block tensordot."""
    dt = dtype_of_mode(mode)
    A, B, C = descriptor(dims_a, grid_a, dt), descriptor(dims_b, grid_b, dt), RnTensor()
    aa, pa, ab, pb = _axes(axes_a, axes_b)
    ws, fl = ctypes.c_size_t(), ctypes.c_double()
    check(lib().rn_block_tensordot_plan(None, ctypes.byref(A), ctypes.byref(B), len(aa), pa, pb,
                                        mode_id(mode), ctypes.byref(C), ctypes.byref(ws),
                                        ctypes.byref(fl)), "plan")
    return ([C.dims[j] for j in range(C.rank)], [C.grid[j] for j in range(C.rank)],
            ws.value, fl.value)


def block_pairs(dims_a, grid_a, dims_b, grid_b, axes_a, axes_b, cblock, dtype=C128):
    """Coupled (A block, B block) pairs of one C block, in K-loop order."""
    A, B = descriptor(dims_a, grid_a, dtype), descriptor(dims_b, grid_b, dtype)
    aa, pa, ab, pb = _axes(axes_a, axes_b)
    n = ctypes.c_int64()
    check(lib().rn_block_pairs(None, ctypes.byref(A), ctypes.byref(B), len(aa), pa, pb, cblock,
                               None, 0, ctypes.byref(n)), "pairs")
    out = np.zeros(2 * max(n.value, 1), dtype=np.int64)
    check(lib().rn_block_pairs(None, ctypes.byref(A), ctypes.byref(B), len(aa), pa, pb, cblock,
                               out.ctypes.data, n.value, ctypes.byref(n)), "pairs")
    return [(int(out[2 * i]), int(out[2 * i + 1])) for i in range(n.value)]


def block_footprint(dims_a, grid_a, dims_b, grid_b, axes_a, axes_b, dtype=C64):
    """(Eq. 1, Eq. 2) element counts of Section IV.A for this contraction."""
    A, B = descriptor(dims_a, grid_a, dtype), descriptor(dims_b, grid_b, dtype)
    aa, pa, ab, pb = _axes(axes_a, axes_b)
    e1, e2 = ctypes.c_double(), ctypes.c_double()
    check(lib().rn_block_footprint(ctypes.byref(A), ctypes.byref(B), len(aa), pa, pb,
                                   ctypes.byref(e1), ctypes.byref(e2)), "footprint")
    return e1.value, e2.value


def plan_batch_workspace(ctx, problems, mode="fp32_4m"):
    """Workspace bytes of rn_block_tensordot_batch for these problems."""
    n = len(problems)
    dt = dtype_of_mode(mode)
    As, Bs = (RnTensor * n)(), (RnTensor * n)()
    ks = np.zeros(max(n, 1), dtype=np.int32)
    keep = []
    pa_arr = (ctypes.c_void_p * max(n, 1))()
    pb_arr = (ctypes.c_void_p * max(n, 1))()
    for i, (a, da, ga, b, db, gb, axa, axb) in enumerate(problems):
        As[i] = descriptor(da, ga, dt, None)
        Bs[i] = descriptor(db, gb, dt, None)
        x, px, y, py = _axes(axa, axb)
        keep += [x, y]
        ks[i] = len(x)
        pa_arr[i] = px
        pb_arr[i] = py
    ws_n = ctypes.c_size_t()
    check(lib().rn_block_tensordot_batch_plan(ctx.h if ctx else None, n, As, Bs, ks.ctypes.data,
                                              pa_arr, pb_arr, mode_id(mode), None,
                                              ctypes.byref(ws_n), None), "batch plan")
    return ws_n.value


# ------------------------------------------------------------- GPU calls

class Context:
    """One library handle bound to a HIP device (torch device index)."""

    def __init__(self, device: int = 0):
        import torch  # noqa: F401  (device memory and streams come from torch)
        self.device = device
        h = ctypes.c_void_p()
        check(lib().rn_create(ctypes.byref(h), device), "rn_create")
        self.h = h
        # Block tensordot plans by shape (see _td_plan).
        self._plans = {}

    def close(self):
        if self.h:
            lib().rn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers -----------------------------------------------------------
    @staticmethod
    def _stream():
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def _workspace(self, nbytes, workspace=None):
        import torch
        if nbytes == 0:
            return None, 0
        if workspace is not None:
            _check_tensor(workspace, "workspace", device=self.device)
            if workspace.numel() * workspace.element_size() < nbytes:
                raise RnError(4, "workspace too small")
            return workspace.data_ptr(), workspace.numel() * workspace.element_size()
        ws = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{self.device}")
        self._last_ws = ws
        return ws.data_ptr(), nbytes

    # -- block tensordot -----------------------------------------------------
    def _td_plan(self, dims_a, grid_a, dims_b, grid_b, axes_a, axes_b, mode):
        """The descriptors (without data), axis arrays, C shape and workspace
        size of one block tensordot shape under this handle, planned on the
        first call with that shape and reused after it: a repeated call then
        costs the tensor checks and one library call.  The plan depends on
        the shapes, the mode and the handle's split options; set_option
        clears the cache."""
        key = (tuple(dims_a), None if grid_a is None else tuple(grid_a), tuple(dims_b),
               None if grid_b is None else tuple(grid_b), tuple(axes_a), tuple(axes_b), mode)
        e = self._plans.get(key)
        if e is not None:
            return e
        dt = dtype_of_mode(mode)
        A, B, C = descriptor(dims_a, grid_a, dt), descriptor(dims_b, grid_b, dt), RnTensor()
        aa, pa, ab, pb = _axes(axes_a, axes_b)
        ws, fl = ctypes.c_size_t(), ctypes.c_double()
        check(lib().rn_block_tensordot_plan(self.h, ctypes.byref(A), ctypes.byref(B), len(aa),
                                            pa, pb, mode_id(mode), ctypes.byref(C),
                                            ctypes.byref(ws), ctypes.byref(fl)), "plan")
        cdims = [C.dims[j] for j in range(C.rank)]
        cgrid = [C.grid[j] for j in range(C.rank)]
        e = {"A": bytes(A), "B": bytes(B), "C": bytes(C), "aa": aa, "ab": ab, "pa": pa, "pb": pb,
             "k": len(aa),
             "cdims": cdims, "cgrid": cgrid, "n": _numel(cdims), "ws": ws.value,
             "flops": fl.value, "na": _numel(dims_a), "nb": _numel(dims_b),
             "want": _torch_dtype(mode), "mode": mode_id(mode)}
        if len(self._plans) >= 1024:
            self._plans.clear()
        self._plans[key] = e
        return e

    def plan_block_tensordot(self, dims_a, grid_a, dims_b, grid_b, axes_a, axes_b,
                             mode="fp64"):
        """As the module-level plan, under this handle's options (split policy)."""
        dt = dtype_of_mode(mode)
        A, B, C = descriptor(dims_a, grid_a, dt), descriptor(dims_b, grid_b, dt), RnTensor()
        aa, pa, bb, pb = _axes(axes_a, axes_b)
        ws, fl = ctypes.c_size_t(), ctypes.c_double()
        check(lib().rn_block_tensordot_plan(self.h, ctypes.byref(A), ctypes.byref(B), len(aa),
                                            pa, pb, mode_id(mode), ctypes.byref(C),
                                            ctypes.byref(ws), ctypes.byref(fl)), "plan")
        return ([C.dims[j] for j in range(C.rank)], [C.grid[j] for j in range(C.rank)],
                ws.value, fl.value)

    def block_tensordot(self, a, dims_a, grid_a, b, dims_b, grid_b, axes_a, axes_b,
                        mode="fp64", out=None, workspace=None):
        """C (stored block-major, flat torch tensor), C dims, C grid."""
        import torch
        e = self._td_plan(dims_a, grid_a, dims_b, grid_b, axes_a, axes_b, mode)
        want = e["want"]
        _check_tensor(a, "a", want, e["na"], device=self.device)
        _check_tensor(b, "b", want, e["nb"], device=self.device)
        if out is None:
            out = torch.empty(e["n"], dtype=want, device=a.device)
        _check_tensor(out, "out", want, e["n"], device=self.device)
        op = out.data_ptr()
        if op == a.data_ptr() or op == b.data_ptr():
            raise RnError(1, "out aliases an operand")
        A = RnTensor.from_buffer_copy(e["A"])
        B = RnTensor.from_buffer_copy(e["B"])
        C = RnTensor.from_buffer_copy(e["C"])
        A.data, B.data, C.data = a.data_ptr(), b.data_ptr(), op
        wp, wn = self._workspace(e["ws"], workspace)
        check(lib().rn_block_tensordot(self.h, ctypes.byref(A), ctypes.byref(B), e["k"],
                                       e["pa"], e["pb"], ctypes.byref(C),
                                       e["mode"], wp, wn, self._stream()), "block_tensordot")
        return out, list(e["cdims"]), list(e["cgrid"])

    def block_tensordot_noalloc(self, a, dims_a, grid_a, b, dims_b, grid_b, axes_a, axes_b,
                                mode="fp64", out=None):
        """As block_tensordot through rn_block_tensordot_noalloc: the library's
        fixed device scratch array is the workspace (nothing is allocated
        when `out` is given)."""
        import torch
        e = self._td_plan(dims_a, grid_a, dims_b, grid_b, axes_a, axes_b, mode)
        want = e["want"]
        _check_tensor(a, "a", want, e["na"], device=self.device)
        _check_tensor(b, "b", want, e["nb"], device=self.device)
        if out is None:
            out = torch.empty(e["n"], dtype=want, device=a.device)
        _check_tensor(out, "out", want, e["n"], device=self.device)
        A = RnTensor.from_buffer_copy(e["A"])
        B = RnTensor.from_buffer_copy(e["B"])
        C = RnTensor.from_buffer_copy(e["C"])
        A.data, B.data, C.data = a.data_ptr(), b.data_ptr(), out.data_ptr()
        check(lib().rn_block_tensordot_noalloc(self.h, ctypes.byref(A), ctypes.byref(B), e["k"],
                                               e["pa"], e["pb"], ctypes.byref(C), e["mode"],
                                               self._stream()), "block_tensordot_noalloc")
        return out, list(e["cdims"]), list(e["cgrid"])

    def plan_streamed(self, dims_a, grid_a, dims_b, grid_b, axes_a, axes_b, mode="fp64"):
        """(C dims, C grid, workspace bytes, useful flops, host-to-device bytes)."""
        dt = dtype_of_mode(mode)
        A, B, C = descriptor(dims_a, grid_a, dt), descriptor(dims_b, grid_b, dt), RnTensor()
        aa, pa, bb, pb = _axes(axes_a, axes_b)
        ws, fl, hd = ctypes.c_size_t(), ctypes.c_double(), ctypes.c_double()
        check(lib().rn_block_tensordot_streamed_plan(
            self.h, ctypes.byref(A), ctypes.byref(B), len(aa), pa, pb, mode_id(mode),
            ctypes.byref(C), ctypes.byref(ws), ctypes.byref(fl), ctypes.byref(hd)),
            "streamed plan")
        return ([C.dims[j] for j in range(C.rank)], [C.grid[j] for j in range(C.rank)],
                ws.value, fl.value, hd.value)

    def block_tensordot_streamed(self, a_host, dims_a, grid_a, b_host, dims_b, grid_b, axes_a,
                                 axes_b, mode="fp64", out=None, workspace=None):
        """Operands in (pinned) host memory, C on the device; returns C, dims, grid.

        Queued on the current stream; a_host and b_host must stay alive and
        unchanged until that stream has passed this call.
        """
        import torch
        dt = dtype_of_mode(mode)
        want = torch.complex128 if dt == C128 else torch.complex64
        for t in (a_host, b_host):
            if t.is_cuda or t.dtype != want or not t.is_contiguous():
                raise ValueError("streamed operands: contiguous host tensors of the mode's dtype")
        cd, cg, ws_n, _, _ = self.plan_streamed(dims_a, grid_a, dims_b, grid_b, axes_a, axes_b,
                                                 mode)
        n = int(np.prod(cd, dtype=np.int64)) if cd else 1
        if a_host.numel() != _numel(dims_a) or b_host.numel() != _numel(dims_b):
            raise RnError(1, "streamed operands: element count does not match dims")
        if out is None:
            out = torch.empty(n, dtype=want, device=torch.device("cuda", self.device))
        _check_tensor(out, "out", want, n, device=self.device)
        A = descriptor(dims_a, grid_a, dt, a_host.data_ptr())
        B = descriptor(dims_b, grid_b, dt, b_host.data_ptr())
        C = descriptor(cd, cg, dt, out.data_ptr())
        aa, pa, bb, pb = _axes(axes_a, axes_b)
        wp, wn = self._workspace(ws_n, workspace)
        check(lib().rn_block_tensordot_streamed(self.h, ctypes.byref(A), ctypes.byref(B), len(aa),
                                                pa, pb, ctypes.byref(C), mode_id(mode), wp, wn,
                                                self._stream()), "streamed tensordot")
        return out, cd, cg

    def block_tensordot_batch(self, problems, mode="fp32_4m", outs=None, workspace=None,
                              autotune=False):
        """problems: list of (a, dims_a, grid_a, b, dims_b, grid_b, axes_a, axes_b).

        autotune=True first times the tile shapes of every untuned problem
        shape (synchronously), then runs the batch with the chosen tiles.
        Returns ([(C, dims, grid)], useful flops)."""
        pb = PreparedBatch(self, problems, mode, outs, workspace, own_workspace=False)
        if autotune:
            pb.autotune()
        pb.run()
        return pb.results, pb.flops

    def prepare_batch(self, problems, mode="fp32_4m", outs=None, workspace=None):
        """A batch call with its descriptors, plan and outputs built once, for
        repeated calls on the same tensors (values may change in place)."""
        return PreparedBatch(self, problems, mode, outs, workspace)

    def set_graphs(self, on: bool) -> None:
        check(lib().rn_set_graphs(self.h, 1 if on else 0), "set_graphs")

    def set_option(self, name: str, value: int) -> None:
        """Handle option by name: graphs, pair_split_threshold, split_footprint, slice_sum."""
        self._plans.clear()
        check(lib().rn_set_option(self.h, OPTIONS[name], int(value)), f"set_option {name}")

    def get_option(self, name: str) -> int:
        v = ctypes.c_int64()
        check(lib().rn_get_option(self.h, OPTIONS[name], ctypes.byref(v)), f"get_option {name}")
        return v.value

    def tune_save(self, path: str) -> None:
        check(lib().rn_tune_save(self.h, path.encode()), "tune_save")

    def tune_load(self, path: str) -> None:
        check(lib().rn_tune_load(self.h, path.encode()), "tune_load")

    def tune_clear(self) -> None:
        check(lib().rn_tune_clear(self.h), "tune_clear")

    # -- networks ------------------------------------------------------------
    def _net_args(self, tensors, labels, mode):
        n = len(tensors)
        if len(labels) != n:
            raise RnError(1, f"{n} tensors but {len(labels)} label lists")
        dt = dtype_of_mode(mode)
        want = _torch_dtype(mode)
        Ts = (RnTensor * n)()
        lab_arr = (ctypes.c_void_p * n)()
        keep = []
        for i, (t, l) in enumerate(zip(tensors, labels)):
            if len(l) > 62:
                raise RnError(1, f"tensor {i}: rank {len(l)} too large")
            _check_tensor(t, f"tensor {i}", want, 1 << len(l), device=self.device)
            Ts[i] = descriptor([2] * len(l), None, dt, t.data_ptr())
            x, px = _arr32(l)
            keep.append(x)
            lab_arr[i] = px
        return Ts, lab_arr, keep

    def contract_network_plan(self, tensors, labels, path, sliced, mode="fp64"):
        Ts, lab_arr, keep = self._net_args(tensors, labels, mode)
        pth, pp = _arr32([x for st in path for x in st])
        sl, ps = _arr32(sliced)
        ws_n, fl, mr = ctypes.c_size_t(), ctypes.c_double(), ctypes.c_int32()
        check(lib().rn_contract_network_plan(self.h, len(tensors), Ts, lab_arr, len(path), pp,
                                             len(sl), ps, mode_id(mode), ctypes.byref(ws_n),
                                             ctypes.byref(fl), ctypes.byref(mr)), "network plan")
        return ws_n.value, fl.value, mr.value

    def contract_network(self, tensors, labels, path, sliced=(), mode="fp64", amp=None,
                         slices=None, workspace=None):
        """Amplitude (device tensor of 2 doubles, re and im) of a sliced network."""
        import torch
        Ts, lab_arr, keep = self._net_args(tensors, labels, mode)
        pth, pp = _arr32([x for st in path for x in st])
        sl, ps = _arr32(sliced)
        ws_n, fl, mr = ctypes.c_size_t(), ctypes.c_double(), ctypes.c_int32()
        check(lib().rn_contract_network_plan(self.h, len(tensors), Ts, lab_arr, len(path), pp,
                                             len(sl), ps, mode_id(mode), ctypes.byref(ws_n),
                                             ctypes.byref(fl), ctypes.byref(mr)), "network plan")
        dev = tensors[0].device
        if amp is None:
            amp = torch.zeros(2, dtype=torch.float64, device=dev)
        _check_amp_slices(amp, slices, len(sliced), self.device)
        wp, wn = self._workspace(ws_n.value, workspace)
        check(lib().rn_contract_network(self.h, len(tensors), Ts, lab_arr, len(path), pp,
                                        len(sl), ps, mode_id(mode), wp, wn, self._stream(),
                                        amp.data_ptr(),
                                        slices.data_ptr() if slices is not None else None),
              "contract_network")
        return amp

    def prepare_network(self, tensors, labels, path, sliced=(), mode="fp64"):
        """A network call with its argument arrays built once (for repeated
        amplitudes of one circuit: same tensors, new values written in place)."""
        return PreparedNetwork(self, tensors, labels, path, sliced, mode)

    # -- kernel timing -------------------------------------------------------
    KERNEL_CLASSES = ("permute", "gemm", "splitk_reduce", "fp64_reduce")

    def profile(self, on: bool = True) -> None:
        check(lib().rn_profile_enable(self.h, 1 if on else 0), "profile")

    def profile_read(self):
        """{class: (total ms, launches)} since the last read; clears the record."""
        ms = np.zeros(4, dtype=np.float64)
        cnt = np.zeros(4, dtype=np.int64)
        check(lib().rn_profile_read(self.h, ms.ctypes.data, cnt.ctypes.data), "profile_read")
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(self.KERNEL_CLASSES)}

    # -- reductions ----------------------------------------------------------
    def norm2(self, t, dims=None):
        import torch
        dt = C128 if t.dtype == torch.complex128 else C64
        dims = [t.numel()] if dims is None else dims
        T = descriptor(dims, None, dt, t.data_ptr())
        out = torch.zeros(1, dtype=torch.float64, device=t.device)
        check(lib().rn_norm2(self.h, ctypes.byref(T), out.data_ptr(), self._stream()), "norm2")
        return out

    def sum_c128(self, vals):
        import torch
        out = torch.zeros(2, dtype=torch.float64, device=vals.device)
        check(lib().rn_sum_c128(self.h, vals.numel(), vals.data_ptr(), out.data_ptr(),
                                self._stream()), "sum_c128")
        return out


def _check_amp_slices(amp, slices, nsliced, device):
    import torch
    checks = [(amp, "amp", 2)] + ([(slices, "slices", 2 << nsliced)] if slices is not None else [])
    for on_gpu in (False, True):   # every size check before any device check
        for t, name, need in checks:
            _check_tensor(t, name, torch.float64, min_numel=need, device=device, on_gpu=on_gpu)


class Server:
    """Amplitude server (rn_server_*): submit networks with host tensors,
    collect amplitudes and latencies.  All GPU work runs in the library's
    worker thread."""

    def __init__(self, device: int = 0, hbm_budget: int = 8 << 30, max_active: int = 4):
        s = ctypes.c_void_p()
        check(lib().rn_server_create(device, hbm_budget, max_active, ctypes.byref(s)),
              "rn_server_create")
        self.s = s

    def submit(self, tensors, labels, path, sliced=(), mode="fp64") -> int:
        """tensors: numpy complex arrays (complex128 for fp64, complex64 otherwise)."""
        dt = dtype_of_mode(mode)
        want = np.complex128 if dt == C128 else np.complex64
        n = len(tensors)
        Ts = (RnTensor * n)()
        lab = (ctypes.c_void_p * n)()
        keep = []
        if len(labels) != n:
            raise RnError(1, f"{n} tensors but {len(labels)} label lists")
        for i, (t, l) in enumerate(zip(tensors, labels)):
            a = np.ascontiguousarray(np.asarray(t).reshape(-1), dtype=want)
            if len(l) > 62 or a.size != (1 << len(l)):
                raise RnError(1, f"tensor {i}: {a.size} elements for {len(l)} labels")
            keep.append(a)
            Ts[i] = descriptor([2] * len(l), None, dt, a.ctypes.data)
            x, px = _arr32(l)
            keep.append(x)
            lab[i] = px
        pth, pp = _arr32([x for st in path for x in st])
        sl, ps = _arr32(sliced)
        tk = ctypes.c_uint64()
        check(lib().rn_server_submit(self.s, n, Ts, lab, len(path), pp, len(sl), ps,
                                     mode_id(mode), ctypes.byref(tk)), "submit")
        return tk.value

    @staticmethod
    def _res(r):
        return {"amp": complex(r.amp[0], r.amp[1]), "latency_s": r.latency_s,
                "queue_s": r.queue_s, "run_s": r.run_s, "footprint": r.footprint_bytes,
                "status": r.status, "start_s": r.start_s, "done_s": r.done_s}

    def set_admission(self, policy: str = "smallest", max_overtakes: int = 8) -> None:
        """Admission order: "fifo" (arrival order) or "smallest" (fewest
        planned flops first, a request overtaken max_overtakes times next)."""
        check(lib().rn_server_set_admission(self.s, {"fifo": 0, "smallest": 1}[policy],
                                            int(max_overtakes)), "set_admission")

    def poll(self, ticket):
        d = ctypes.c_int32()
        r = RnResult()
        check(lib().rn_server_poll(self.s, ticket, ctypes.byref(d), ctypes.byref(r)), "poll")
        return self._res(r) if d.value else None

    def wait(self, ticket):
        r = RnResult()
        check(lib().rn_server_wait(self.s, ticket, ctypes.byref(r)), "wait")
        return self._res(r)

    def stats(self):
        q, a, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        b = ctypes.c_size_t()
        check(lib().rn_server_stats(self.s, ctypes.byref(q), ctypes.byref(a), ctypes.byref(c),
                                    ctypes.byref(b)), "stats")
        return {"queued": q.value, "active": a.value, "completed": c.value,
                "bytes_in_use": b.value}

    def close(self):
        if self.s:
            lib().rn_server_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PreparedBatch:
    """Argument arrays, plan and outputs of one batch of block tensordots,
    kept for repeated calls.

    The operand tensors (and `outs`, if given) must stay alive and keep
    their storage; their contents may change between calls.  A repeated
    call on the same stream replays the batch's HIP graph.
    """

    def __init__(self, ctx, problems, mode, outs=None, workspace=None, own_workspace=True):
        import torch
        self.ctx = ctx
        self.mode = mode
        self.problems = list(problems)
        n = self.n = len(self.problems)
        dt = dtype_of_mode(mode)
        want = torch.complex128 if dt == C128 else torch.complex64
        self.As, self.Bs, self.Cs = (RnTensor * n)(), (RnTensor * n)(), (RnTensor * n)()
        self.ks = np.zeros(max(n, 1), dtype=np.int32)
        self._keep = []
        self.pa = (ctypes.c_void_p * max(n, 1))()
        self.pb = (ctypes.c_void_p * max(n, 1))()
        if outs is not None and len(outs) != n:
            raise RnError(1, f"{n} problems but {len(outs)} outputs")
        for i, (a, da, ga, b, db, gb, axa, axb) in enumerate(self.problems):
            _check_tensor(a, f"problem {i} a", want, _numel(da), device=ctx.device)
            _check_tensor(b, f"problem {i} b", want, _numel(db), device=ctx.device)
            self.As[i] = descriptor(da, ga, dt, a.data_ptr())
            self.Bs[i] = descriptor(db, gb, dt, b.data_ptr())
            x, px, y, py = _axes(axa, axb)
            self._keep += [x, y]
            self.ks[i] = len(x)
            self.pa[i] = px
            self.pb[i] = py
        ws_n, fl = ctypes.c_size_t(), ctypes.c_double()
        check(lib().rn_block_tensordot_batch_plan(ctx.h, n, self.As, self.Bs, self.ks.ctypes.data,
                                                  self.pa, self.pb, mode_id(mode), self.Cs,
                                                  ctypes.byref(ws_n), ctypes.byref(fl)),
              "batch plan")
        self.flops = fl.value
        self.results = []
        for i in range(n):
            cd = [self.Cs[i].dims[j] for j in range(self.Cs[i].rank)]
            cg = [self.Cs[i].grid[j] for j in range(self.Cs[i].rank)]
            nc = int(np.prod(cd, dtype=np.int64)) if cd else 1
            o = outs[i] if outs is not None else torch.empty(
                nc, dtype=want, device=self.problems[i][0].device)
            _check_tensor(o, f"problem {i} out", want, nc, device=ctx.device)
            self.Cs[i].data = o.data_ptr()
            self.results.append((o, cd, cg))
        self.outputs = [o for o, _, _ in self.results]
        if own_workspace and ws_n.value > 0 and workspace is None:
            workspace = torch.empty(ws_n.value, dtype=torch.uint8, device=f"cuda:{ctx.device}")
        self.workspace = workspace  # kept alive with the plan (else the handle's last one)
        self.wp, self.wn = ctx._workspace(ws_n.value, workspace)

    def autotune(self):
        """Time the tile shapes of every untuned problem shape, then each tile
        group of the batch (synchronous); the outputs' contents afterwards are
        unspecified until the next run()."""
        check(lib().rn_autotune_batch(self.ctx.h, self.n, self.As, self.Bs, self.ks.ctypes.data,
                                      self.pa, self.pb, self.Cs, mode_id(self.mode), self.wp,
                                      self.wn, self.ctx._stream()), "autotune")

    def run(self):
        """Enqueue the batch on the current stream; returns the outputs."""
        check(lib().rn_block_tensordot_batch(self.ctx.h, self.n, self.As, self.Bs,
                                             self.ks.ctypes.data, self.pa, self.pb, self.Cs,
                                             mode_id(self.mode), self.wp, self.wn,
                                             self.ctx._stream()), "batch")
        return self.outputs


class PreparedNetwork:
    """A network call prepared once (rn_network_prepare: descriptors copied,
    planned and hashed), for repeated amplitudes of one circuit.

    The tensors passed in must stay alive and keep their storage; their
    contents may change between calls.
    """

    def __init__(self, ctx, tensors, labels, path, sliced, mode):
        self.ctx = ctx
        self.tensors = list(tensors)
        self.mode = mode
        Ts, lab_arr, keep = ctx._net_args(self.tensors, labels, mode)
        _, pp = _arr32([x for st in path for x in st])
        sl, ps = _arr32(sliced)
        self.nsliced = len(sl)
        prep, ws_n = ctypes.c_void_p(), ctypes.c_size_t()
        check(lib().rn_network_prepare(ctx.h, len(self.tensors), Ts, lab_arr, len(path), pp,
                                       len(sl), ps, mode_id(mode), ctypes.byref(prep),
                                       ctypes.byref(ws_n)), "network prepare")
        self.prep = prep
        self.ws_bytes = ws_n.value
        fl, mr = ctypes.c_double(), ctypes.c_int32()
        check(lib().rn_contract_network_plan(ctx.h, len(self.tensors), Ts, lab_arr, len(path),
                                             pp, len(sl), ps, mode_id(mode), None,
                                             ctypes.byref(fl), ctypes.byref(mr)), "network plan")
        self.flops, self.max_rank = fl.value, mr.value
        import torch
        dev = self.tensors[0].device
        self.workspace = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=dev)
        self._ws = ctypes.c_void_p(self.workspace.data_ptr())

    def run(self, amp=None, slices=None, stream=None):
        """Amplitude (device tensor of 2 doubles) on `stream` (a torch stream;
        default: the current stream)."""
        import torch
        if amp is None:
            amp = torch.zeros(2, dtype=torch.float64, device=self.tensors[0].device)
        _check_amp_slices(amp, slices, self.nsliced, self.ctx.device)
        sp = self.ctx._stream() if stream is None else ctypes.c_void_p(stream.cuda_stream)
        check(lib().rn_network_execute(self.prep, self._ws, self.ws_bytes, sp,
                                       amp.data_ptr(),
                                       slices.data_ptr() if slices is not None else None),
              "network execute")
        return amp

    def __del__(self):
        prep = getattr(self, "prep", None)
        if prep is not None and prep.value and _lib is not None:
            _lib.rn_network_release(prep)
            self.prep = None
