"""Oracle: plain, slow CPU reference (complex128) for block tensor contraction.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the library's product
path never does.  The arithmetic lives in ``oracle.c`` (plain loops, FP64,
no FMA contraction); this module only marshals numpy arrays.

Functions and the passage each follows:
  permute              index permutation (transpose), the reshuffle inside a
                       pairwise contraction (Section II.A)
  tensordot            pairwise contraction, A's free axes then B's
                       (Section II.A; tensordot semantics of the commutative
                       task of Section III)
  tensordot_entries    the same definition evaluated at chosen outputs only
  to_blocked /
  from_blocked         uniform-grid block layout (Section II.C)
  block_tensordot      the four steps of block tensor contraction (Section II.C)
  statevector          2^n state tensor evolved gate by gate (Section II.A)
  contract_network     sliced network contraction on a path, slices summed in
                       FP64 (Sections II.A, II.B)
  contract_network_slices  the value of chosen single slices (one projection
                       each, Section II.B)
  norm2                sum of squared magnitudes in FP64
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_SO_OMP = os.path.join(_HERE, "liboracle_omp.so")
_lib = None
_lib_omp = None

ERRORS = {1: "invalid argument", 2: "shape mismatch", 3: "grid does not divide dims",
          5: "out of memory"}


class OracleError(RuntimeError):
    pass


def build(force: bool = False, openmp: bool = False) -> str:
    """Compile the oracle (gcc, -O2 -ffp-contract=off, no fast-math).  The
    OpenMP build (a second library, for the CPU baseline) runs the output
    blocks of block_tensordot on several threads, each block summed in the
    same order as the single-threaded build, so the results are identical."""
    so = _SO_OMP if openmp else _SO
    if force or not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(_SRC):
        tmp = so + ".tmp%d" % os.getpid()
        extra = ["-fopenmp", "-DORC_OPENMP"] if openmp else []
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall"] + extra + [_SRC, "-o", tmp])
        os.replace(tmp, so)
    return so


def _L():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        p, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        lib.orc_permute.argtypes = [p, i32, p, p, p]
        lib.orc_tensordot.argtypes = [p, i32, p, p, i32, p, i32, p, p, p]
        lib.orc_tensordot_entries.argtypes = [p, i32, p, p, i32, p, i32, p, p, i64, p, p]
        lib.orc_to_blocked.argtypes = [p, i32, p, p, p]
        lib.orc_from_blocked.argtypes = [p, i32, p, p, p]
        lib.orc_block_tensordot.argtypes = [p, i32, p, p, p, i32, p, p, i32, p, p, p, p]
        lib.orc_statevector.argtypes = [i32, i32, p, p, p, p]
        lib.orc_norm2.argtypes = [p, i64]
        lib.orc_norm2.restype = ctypes.c_double
        lib.orc_contract_network.argtypes = [i32, p, p, p, i32, p, i32, p, p, i64, p, p]
        lib.orc_contract_network_range.argtypes = [i32, p, p, p, i32, p, i32, p, i64, i64, p,
                                                   i64, p, p]
        _lib = lib
    return _lib


def _c128(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.complex128)


def _i64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.int64).reshape(-1))


def _i32(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32).reshape(-1))


def _check(rc: int, what: str) -> None:
    if rc:
        raise OracleError(f"{what}: {ERRORS.get(rc, rc)}")


def _ptr(a: np.ndarray):
    return a.ctypes.data if a.size else None


def permute(t: np.ndarray, perm) -> np.ndarray:
    t = _c128(t)
    perm = _i32(perm)
    dims = _i64(t.shape)
    out = np.empty(tuple(t.shape[p] for p in perm) if t.ndim else (), dtype=np.complex128)
    _check(_L().orc_permute(_ptr(t) or t.ctypes.data, t.ndim, _ptr(dims), _ptr(perm),
                            out.ctypes.data), "permute")
    return out


def _out_shape(da, db, axes_a, axes_b):
    fa = [j for j in range(len(da)) if j not in set(axes_a)]
    fb = [j for j in range(len(db)) if j not in set(axes_b)]
    return tuple(da[j] for j in fa) + tuple(db[j] for j in fb)


def tensordot(a: np.ndarray, b: np.ndarray, axes_a, axes_b) -> np.ndarray:
    a, b = _c128(a), _c128(b)
    axa, axb = _i32(axes_a), _i32(axes_b)
    if axa.size != axb.size:
        raise OracleError("tensordot: axes lists differ in length")
    da, db = _i64(a.shape), _i64(b.shape)
    if any(not (0 <= x < a.ndim) for x in axa) or any(not (0 <= x < b.ndim) for x in axb):
        raise OracleError("tensordot: invalid argument")
    out = np.empty(_out_shape(a.shape, b.shape, list(axa), list(axb)), dtype=np.complex128)
    _check(_L().orc_tensordot(a.ctypes.data, a.ndim, _ptr(da), b.ctypes.data, b.ndim,
                              _ptr(db), axa.size, _ptr(axa), _ptr(axb), out.ctypes.data),
           "tensordot")
    return out


def tensordot_entries(a: np.ndarray, b: np.ndarray, axes_a, axes_b, flat_idx) -> np.ndarray:
    """C.flat[flat_idx] of tensordot(a, b), each entry summed on its own."""
    a, b = _c128(a), _c128(b)
    axa, axb = _i32(axes_a), _i32(axes_b)
    da, db = _i64(a.shape), _i64(b.shape)
    idx = _i64(flat_idx)
    out = np.empty(idx.size, dtype=np.complex128)
    _check(_L().orc_tensordot_entries(a.ctypes.data, a.ndim, _ptr(da), b.ctypes.data, b.ndim,
                                      _ptr(db), axa.size, _ptr(axa), _ptr(axb), idx.size,
                                      _ptr(idx), _ptr(out)), "tensordot_entries")
    return out


def to_blocked(dense: np.ndarray, grid) -> np.ndarray:
    """Flat block-major buffer of a dense tensor on the given uniform grid."""
    dense = _c128(dense)
    dims, g = _i64(dense.shape), _i32(grid)
    out = np.empty(dense.size, dtype=np.complex128)
    _check(_L().orc_to_blocked(dense.ctypes.data, dense.ndim, _ptr(dims), _ptr(g),
                               out.ctypes.data), "to_blocked")
    return out


def from_blocked(blocked: np.ndarray, dims, grid) -> np.ndarray:
    blocked = _c128(blocked).reshape(-1)
    d, g = _i64(dims), _i32(grid)
    out = np.empty(tuple(int(x) for x in dims), dtype=np.complex128)
    _check(_L().orc_from_blocked(blocked.ctypes.data, d.size, _ptr(d), _ptr(g),
                                 out.ctypes.data), "from_blocked")
    return out


def _L_omp():
    global _lib_omp
    if _lib_omp is None:
        lib = ctypes.CDLL(build(openmp=True))
        p, i32 = ctypes.c_void_p, ctypes.c_int32
        lib.orc_block_tensordot.argtypes = [p, i32, p, p, p, i32, p, p, i32, p, p, p, p]
        _lib_omp = lib
    return _lib_omp


def block_tensordot(a_blocked, dims_a, grid_a, b_blocked, dims_b, grid_b, axes_a, axes_b,
                    openmp=False):
    """(C block-major buffer, C dims, C grid) by the four steps of Section II.C
    (openmp: output blocks on several threads, OMP_NUM_THREADS, same result)."""
    ab, bb = _c128(a_blocked).reshape(-1), _c128(b_blocked).reshape(-1)
    da, ga, db, gb = _i64(dims_a), _i32(grid_a), _i64(dims_b), _i32(grid_b)
    axa, axb = _i32(axes_a), _i32(axes_b)
    cdims = _out_shape(list(da), list(db), list(axa), list(axb))
    out = np.empty(int(np.prod(cdims, dtype=np.int64)), dtype=np.complex128)
    gc = np.zeros(max(1, len(cdims)), dtype=np.int32)
    lib = _L_omp() if openmp else _L()
    _check(lib.orc_block_tensordot(ab.ctypes.data, da.size, _ptr(da), _ptr(ga), bb.ctypes.data,
                                    db.size, _ptr(db), _ptr(gb), axa.size, _ptr(axa), _ptr(axb),
                                    out.ctypes.data, gc.ctypes.data), "block_tensordot")
    return out, list(cdims), [int(x) for x in gc[:len(cdims)]]


def statevector(circuit) -> np.ndarray:
    """U|0...0> for a workloads.circuits.Circuit (qubit 0 = most significant)."""
    nq = _i32([len(g.qubits) for g in circuit.gates])
    qs = _i32([q for g in circuit.gates for q in g.qubits])
    mats = _c128(np.concatenate([np.asarray(g.matrix).reshape(-1) for g in circuit.gates])
                 if circuit.gates else np.zeros(1))
    psi = np.empty(1 << circuit.n, dtype=np.complex128)
    _check(_L().orc_statevector(circuit.n, nq.size, _ptr(nq), _ptr(qs), mats.ctypes.data,
                                psi.ctypes.data), "statevector")
    return psi


def norm2(x: np.ndarray) -> float:
    x = _c128(x).reshape(-1)
    return float(_L().orc_norm2(x.ctypes.data, x.size))


def contract_network(tensors, labels, path, sliced=()):
    """(summed final tensor, its labels) of a sliced contraction on a path."""
    ranks = _i32([len(l) for l in labels])
    for t, l in zip(tensors, labels):
        if np.asarray(t).size != (1 << len(l)):
            raise OracleError("contract_network: every dim must be 2")
    flat_l = _i32([x for l in labels for x in l] or [0])
    data = _c128(np.concatenate([_c128(t).reshape(-1) for t in tensors]))
    p = _i32([x for st in path for x in st] or [0])
    sl = _i32(list(sliced) or [0])
    # Largest intermediate bounds the output; open legs only survive to the end.
    nopen = sum(1 for x in set(flat_l.tolist()) if flat_l.tolist().count(x) == 1)
    cap = 2 * (1 << nopen)
    out = np.zeros(cap // 2, dtype=np.complex128)
    orank = np.zeros(1, dtype=np.int32)
    olab = np.zeros(64, dtype=np.int32)
    _check(_L().orc_contract_network(len(tensors), ranks.ctypes.data, flat_l.ctypes.data,
                                     data.ctypes.data, len(path), p.ctypes.data, len(sliced),
                                     sl.ctypes.data, out.ctypes.data, cap, orank.ctypes.data,
                                     olab.ctypes.data), "contract_network")
    r = int(orank[0])
    return out[:1 << r].reshape((2,) * r), [int(x) for x in olab[:r]]


def contract_network_slices(tensors, labels, path, sliced, which):
    """Scalar value of each slice s in `which` (slice s fixes sliced[i] to bit
    nsliced-1-i of s) of a network that closes to a scalar."""
    ranks = _i32([len(l) for l in labels])
    for t, l in zip(tensors, labels):
        if np.asarray(t).size != (1 << len(l)):
            raise OracleError("contract_network_slices: every dim must be 2")
    flat_l = _i32([x for l in labels for x in l] or [0])
    data = _c128(np.concatenate([_c128(t).reshape(-1) for t in tensors]))
    p = _i32([x for st in path for x in st] or [0])
    sl = _i32(list(sliced) or [0])
    res = []
    for s in which:
        out = np.zeros(1, dtype=np.complex128)
        orank = np.zeros(1, dtype=np.int32)
        olab = np.zeros(64, dtype=np.int32)
        _check(_L().orc_contract_network_range(len(tensors), ranks.ctypes.data,
                                               flat_l.ctypes.data, data.ctypes.data, len(path),
                                               p.ctypes.data, len(sliced), sl.ctypes.data,
                                               int(s), int(s) + 1, out.ctypes.data, 2,
                                               orank.ctypes.data, olab.ctypes.data),
               "contract_network_slices")
        if orank[0] != 0:
            raise OracleError("contract_network_slices: the network has open labels")
        res.append(complex(out[0]))
    return np.asarray(res, dtype=np.complex128)
