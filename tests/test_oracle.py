"""Pins for the CPU oracle: it is checked against things other than itself.

Each test names what fixes the expected value: a library routine the oracle
does not use (numpy), a closed form, an invariant, an exactly representable
case, or brute force on tiny inputs.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from workloads import circuits, configs, paths, rng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def cn(seed, shape):
    n = int(np.prod(shape, dtype=np.int64))
    return rng.complex_normal(seed, n).reshape(shape)


def gi(seed, shape, lo=-8, hi=8):
    n = int(np.prod(shape, dtype=np.int64))
    return rng.gaussian_integers(seed, n, lo, hi).reshape(shape)


def rel_err(x, ref):
    return np.linalg.norm((x - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300)


# ---------------------------------------------------------------- generators

def test_splitmix64_reference_vector():
    with open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) as f:
        ref = [int(l) for l in f if l.strip() and not l.startswith("#")]
    got = [int(x) for x in rng.splitmix64_block(1234567, 0, len(ref))]
    assert got == ref
    s = rng.SplitMix64(1234567)
    assert [s.next_u64() for _ in ref] == ref
    out = np.empty(len(ref), dtype=np.uint64)
    rng._native().wl_splitmix64(1234567, 0, len(ref), out.ctypes.data)
    assert [int(x) for x in out] == ref


def test_complex_normal_moments_and_bulk_agreement():
    x = rng.complex_normal(99, 1 << 18)
    assert abs(x.mean()) < 0.01
    assert abs(np.mean(x.real ** 2) - 0.5) < 0.01
    assert abs(np.mean(x.imag ** 2) - 0.5) < 0.01
    assert abs(np.mean(x.real * x.imag)) < 0.01
    y = rng.complex_normal_numpy(99, 1 << 12)
    assert np.abs(x[:1 << 12] - y).max() < 1e-14
    g = rng.gaussian_integers(3, 4096)
    assert np.array_equal(g, rng.gaussian_integers_numpy(3, 4096))
    assert g.real.min() == -8 and g.real.max() == 8


# ------------------------------------------------------------------- permute

def test_permute_hand_transpose():
    t = np.array([[1, 2, 3], [4, 5, 6]], dtype=np.complex128) * (1 + 2j)
    out = oracle.permute(t, [1, 0])
    assert out.shape == (3, 2)
    assert np.array_equal(out, np.array([[1, 4], [2, 5], [3, 6]]) * (1 + 2j))


@pytest.mark.parametrize("shape", [(2, 3, 4), (2,) * 7, (1, 4, 1, 2, 3), (5,)])
def test_permute_matches_numpy_transpose_and_inverts(shape):
    t = cn(11, shape)
    r = rng.SplitMix64(len(shape))
    for _ in range(4):
        perm = r.permutation(len(shape))
        out = oracle.permute(t, perm)
        assert np.array_equal(out, np.transpose(t, perm))
        inv = list(np.argsort(perm))
        assert np.array_equal(oracle.permute(out, inv), t)


def test_permute_dims2_is_bit_permutation():
    # For all-2 dims, output linear index bits are a permutation of the input's.
    r = 6
    t = np.arange(1 << r).astype(np.complex128).reshape((2,) * r)
    perm = [3, 0, 5, 1, 4, 2]
    out = oracle.permute(t, perm).reshape(-1)
    for o in range(1 << r):
        src = 0
        for j in range(r):
            bit = (o >> (r - 1 - j)) & 1
            src |= bit << (r - 1 - perm[j])
        assert out[o] == src


def test_permute_rejects_bad_perm():
    with pytest.raises(oracle.OracleError):
        oracle.permute(cn(1, (2, 2)), [0, 0])


# ----------------------------------------------------------------- tensordot

def naive_matmul(a, b):
    m, k = a.shape
    _, n = b.shape
    c = np.zeros((m, n), dtype=np.complex128)
    for i in range(m):
        for j in range(n):
            s = 0j
            for p in range(k):
                s += a[i, p] * b[p, j]
            c[i, j] = s
    return c


def test_tensordot_reduces_to_matmul():
    # Textbook case: A's last k axes against B's first k axes, in order.
    a = cn(21, (2, 3, 2, 2))
    b = cn(22, (2, 2, 5))
    c = oracle.tensordot(a, b, [2, 3], [0, 1])
    ref = naive_matmul(a.reshape(6, 4), b.reshape(4, 5)).reshape(2, 3, 5)
    assert rel_err(c, ref) < 1e-14


@pytest.mark.parametrize("case", range(6))
def test_tensordot_matches_numpy(case):
    r = rng.SplitMix64(100 + case)
    ra, rb = r.randint(1, 6), r.randint(1, 6)
    k = r.randint(0, min(ra, rb))
    axa, axb = r.sample(ra, k), r.sample(rb, k)
    da = [r.randint(1, 3) for _ in range(ra)]
    db = [r.randint(1, 3) for _ in range(rb)]
    for i in range(k):
        db[axb[i]] = da[axa[i]]
    a, b = cn(200 + case, da), cn(300 + case, db)
    c = oracle.tensordot(a, b, axa, axb)
    ref = np.tensordot(a, b, (axa, axb))
    assert c.shape == ref.shape
    assert rel_err(c, ref) < 1e-14


def test_tensordot_outer_and_full():
    a, b = cn(31, (2, 3)), cn(32, (4,))
    assert rel_err(oracle.tensordot(a, b, [], []), np.multiply.outer(a, b)) < 1e-15
    x, y = cn(33, (2, 3, 2)), cn(34, (3, 2, 2))
    full = oracle.tensordot(x, y, [0, 1, 2], [2, 0, 1])
    assert full.shape == ()
    ref = np.sum(x * np.transpose(y, (2, 0, 1)))
    assert abs(full - ref) < 1e-14 * abs(ref) + 1e-15


def test_tensordot_with_delta_is_permutation():
    # Contracting with identity matrices on chosen axes only relabels them.
    a = cn(41, (2, 2, 2))
    eye = np.eye(2, dtype=np.complex128)
    c = oracle.tensordot(a, eye, [0], [1])       # C[j,k,x] = A[x,j,k]
    assert np.array_equal(c, np.transpose(a, (1, 2, 0)))


def test_tensordot_gaussian_integers_exact():
    # Integer inputs: every partial sum is exact, so the result is the same
    # bits whatever the summation order (numpy sums in its own order).
    a, b = gi(51, (2,) * 9), gi(52, (2,) * 8)
    axa, axb = [8, 2, 5, 0], [1, 7, 3, 4]
    c = oracle.tensordot(a, b, axa, axb)
    ref = np.tensordot(a, b, (axa, axb))
    assert np.array_equal(c, ref)


def test_tensordot_worked_example_ijk_ikm():
    # Figure 1's contraction A_ijk B_ikm -> C_jm with values whose sums have
    # a closed form: A = (1 + i) * (j + 1), B = (m + 1) - i*k*1j.
    A = np.zeros((2, 3, 2), dtype=np.complex128)
    B = np.zeros((2, 2, 4), dtype=np.complex128)
    for i, j, k in itertools.product(range(2), range(3), range(2)):
        A[i, j, k] = (1 + 1j) * (j + 1)
    for i, k, m in itertools.product(range(2), range(2), range(4)):
        B[i, k, m] = (m + 1) - 1j * i * k
    C = oracle.tensordot(A, B, [0, 2], [0, 1])
    for j in range(3):
        for m in range(4):
            # sum over (i,k) of (m+1) - i*k*1j = 4(m+1) - 1j
            expect = (1 + 1j) * (j + 1) * (4 * (m + 1) - 1j)
            assert C[j, m] == expect


def test_tensordot_entries_equal_full():
    a, b = cn(61, (2,) * 10), cn(62, (2,) * 9)
    axa, axb = [9, 1, 4], [0, 8, 5]
    c = oracle.tensordot(a, b, axa, axb).reshape(-1)
    idx = np.array([0, 1, 77, 1000, c.size - 1])
    e = oracle.tensordot_entries(a, b, axa, axb, idx)
    assert np.array_equal(e, c[idx])
    with pytest.raises(oracle.OracleError):
        oracle.tensordot_entries(a, b, axa, axb, [c.size])


def test_tensordot_rejects_bad_axes():
    a, b = cn(1, (2, 3)), cn(2, (2, 2))
    with pytest.raises(oracle.OracleError):
        oracle.tensordot(a, b, [1], [0])          # 3 vs 2
    with pytest.raises(oracle.OracleError):
        oracle.tensordot(a, b, [0, 0], [0, 1])    # repeated axis


# ------------------------------------------------------------- block layout

def numpy_blocked(dense, grid):
    # Independent construction: split each axis into (grid, extent), move all
    # grid axes to the front, flatten.
    shp = []
    for d, g in zip(dense.shape, grid):
        shp += [g, d // g]
    r = dense.ndim
    t = dense.reshape(shp).transpose(list(range(0, 2 * r, 2)) + list(range(1, 2 * r, 2)))
    return t.reshape(-1)


@pytest.mark.parametrize("shape,grid", [((2,) * 6, [2, 2, 1, 1, 2, 1]),
                                        ((4, 6, 2), [2, 3, 1]), ((8,), [4])])
def test_blocked_layout(shape, grid):
    d = cn(71, shape)
    b = oracle.to_blocked(d, grid)
    assert np.array_equal(b, numpy_blocked(d, grid))
    assert np.array_equal(oracle.from_blocked(b, shape, grid), d)
    with pytest.raises(oracle.OracleError):
        oracle.to_blocked(d, [3] * len(shape))


# ------------------------------------------------------- block tensordot

def blocked_vs_unblocked(ra, rb, axa, axb, ga, gb, seed, integer=False):
    gen = gi if integer else cn
    A, B = gen(seed, (2,) * ra), gen(seed + 1, (2,) * rb)
    cb, cd, cg = oracle.block_tensordot(oracle.to_blocked(A, ga), [2] * ra, ga,
                                        oracle.to_blocked(B, gb), [2] * rb, gb, axa, axb)
    C = oracle.from_blocked(cb, cd, cg)
    return C, np.tensordot(A, B, (axa, axb)), cg


def test_block_tensordot_config1_refinement():
    p = configs.config1()
    cb, cd, cg = oracle.block_tensordot(p.a.data, p.a.dims, p.a.grid, p.b.data, p.b.dims,
                                        p.b.grid, p.axes_a, p.axes_b)
    assert cg == [2, 2, 2] + [1] * 13
    A = oracle.from_blocked(p.a.data, p.a.dims, p.a.grid)
    B = oracle.from_blocked(p.b.data, p.b.dims, p.b.grid)
    ref = np.tensordot(A, B, (p.axes_a, p.axes_b))
    assert rel_err(oracle.from_blocked(cb, cd, cg), ref) < 1e-14


@pytest.mark.parametrize("integer", [False, True])
def test_block_tensordot_equivalence(integer):
    # Mismatched grids on contracted pairs, split free axes, odd pairing order.
    ga = [2, 1, 2, 2, 1, 2, 1]
    gb = [1, 2, 2, 1, 2, 1]
    C, ref, cg = blocked_vs_unblocked(7, 6, [2, 6, 0], [4, 1, 3], ga, gb, 81, integer)
    assert cg == [1, 2, 1, 2] + [1, 2, 1]   # A free axes 1,3,4,5 then B free 0,2,5
    if integer:
        assert np.array_equal(C, ref)
    else:
        assert rel_err(C, ref) < 1e-14


def test_block_tensordot_openmp_build_identical():
    # The CPU-baseline build runs output blocks on several threads; each block
    # is summed in the same order, so the results are the same bits.
    for p in (configs.config1(), configs.make_problem(
            10, 9, [1, 7, 4], [8, 0, 3], [2, 2, 1, 1, 2, 1, 1, 2, 1, 1],
            [1, 2, 2, 1, 1, 1, 1, 1, 2], 515)):
        args = (p.a.data, p.a.dims, p.a.grid, p.b.data, p.b.dims, p.b.grid, p.axes_a, p.axes_b)
        serial = oracle.block_tensordot(*args)
        threaded = oracle.block_tensordot(*args, openmp=True)
        assert np.array_equal(serial[0], threaded[0]) and serial[1:] == threaded[1:]


def test_block_tensordot_outer_and_scalar():
    C, ref, _ = blocked_vs_unblocked(3, 2, [], [], [2, 1, 2], [2, 2], 91)
    assert rel_err(C, ref) < 1e-15
    C, ref, cg = blocked_vs_unblocked(3, 3, [0, 1, 2], [2, 0, 1], [2, 2, 1], [1, 2, 2], 92)
    assert cg == [] and C.shape == ()
    assert abs(C - ref) < 1e-14 * abs(ref)


def test_tensordot_rank_above_32_matches_numpy():
    # Rank 40 x rank 34 -> rank 50 with dims 1, 2 and 4 in a seeded order
    # (Section V: tensors past 32 axes); numpy 2 handles 64 axes.
    rs = np.random.default_rng(4034)
    kd = [2, 2, 4] + [1] * 9
    pa, pb = rs.permutation(40), rs.permutation(34)
    da, db = [0] * 40, [0] * 34
    for i, d in enumerate(kd + [2, 2, 2, 4] + [1] * 24):
        da[pa[i]] = d
    for i, d in enumerate(kd + [2, 2, 4, 2] + [1] * 18):
        db[pb[i]] = d
    axa, axb = [int(x) for x in pa[:12]], [int(x) for x in pb[:12]]
    a = rs.normal(size=da) + 1j * rs.normal(size=da)
    b = rs.normal(size=db) + 1j * rs.normal(size=db)
    got = oracle.tensordot(a, b, axa, axb)
    ref = np.tensordot(a, b, (axa, axb))
    assert got.shape == ref.shape and got.ndim == 50
    assert rel_err(got, ref) < 1e-14


# -------------------------------------------------------------- statevector

def dense_unitary(circ):
    # Independent: full 2^n x 2^n matrix from Kronecker products.
    n = circ.n
    U = np.eye(1 << n, dtype=np.complex128)
    for g in circ.gates:
        if len(g.qubits) == 1:
            (q,) = g.qubits
            op = np.kron(np.kron(np.eye(1 << q), g.matrix), np.eye(1 << (n - 1 - q)))
        else:
            a, b = g.qubits
            # Move qubits a,b next to each other via a permutation matrix.
            perm = [a, b] + [x for x in range(n) if x not in (a, b)]
            P = np.zeros((1 << n, 1 << n))
            for i in range(1 << n):
                bits = [(i >> (n - 1 - x)) & 1 for x in range(n)]
                j = 0
                for x in perm:
                    j = 2 * j + bits[x]
                P[j, i] = 1
            op = P.T @ np.kron(g.matrix, np.eye(1 << (n - 2))) @ P
        U = op @ U
    return U


def test_statevector_vs_dense_unitary():
    circ = circuits.random_circuit(2, 2, 3, seed=5)
    psi = oracle.statevector(circ)
    ref = dense_unitary(circ)[:, 0]
    assert np.abs(psi - ref).max() < 1e-14


def test_statevector_ghz_closed_form():
    for n in (2, 5, 9):
        psi = oracle.statevector(circuits.ghz_circuit(n))
        ref = np.zeros(1 << n, dtype=np.complex128)
        ref[0] = ref[-1] = 1 / math.sqrt(2)
        assert np.abs(psi - ref).max() < 1e-15


def test_statevector_cnot_orientation():
    # CNOT(control=q0, target=q1) on |10> gives |11>; on |01> leaves |01>.
    c = circuits.Circuit(2, [circuits.Gate((0,), np.array([[0, 1], [1, 0]])),
                             circuits.Gate((0, 1), circuits.CNOT)])
    psi = oracle.statevector(c)
    assert psi[3] == 1 and np.count_nonzero(psi) == 1
    c = circuits.Circuit(2, [circuits.Gate((1,), np.array([[0, 1], [1, 0]])),
                             circuits.Gate((0, 1), circuits.CNOT)])
    psi = oracle.statevector(c)
    assert psi[1] == 1 and np.count_nonzero(psi) == 1


def test_statevector_norm_and_gate_unitarity():
    for m in circuits.ONE_QUBIT_SET + (circuits.FSIM,):
        assert np.abs(m @ m.conj().T - np.eye(m.shape[0])).max() < 1e-15
    psi = oracle.statevector(circuits.random_circuit(3, 4, 8, seed=7))
    assert abs(oracle.norm2(psi) - 1.0) < 1e-13


def test_norm2_matches_numpy():
    x = cn(5, (1000,))
    assert abs(oracle.norm2(x) - np.sum(np.abs(x) ** 2)) < 1e-12


# ----------------------------------------------------------------- networks

def full_state_by_network(circ, path_seed=1, sliced_count=0):
    net = circuits.circuit_network(circ, None)
    path = paths.greedy_path(net.labels, path_seed, restarts=2)
    sliced = []
    if sliced_count:
        sliced = paths.greedy_slices(net.labels, path, 3, n_slices=sliced_count)
    out, labels = oracle.contract_network(net.tensors, net.labels, path, sliced)
    order = [labels.index(l) for l in net.open_labels]
    return np.transpose(out, order).reshape(-1)


@pytest.mark.parametrize("rows,cols,cycles", [(2, 3, 4), (3, 4, 5)])
def test_network_all_amplitudes_vs_statevector(rows, cols, cycles):
    circ = circuits.random_circuit(rows, cols, cycles, seed=rows * 10 + cols)
    psi = oracle.statevector(circ)
    got = full_state_by_network(circ)
    assert np.abs(got - psi).max() < 1e-13
    assert abs(np.sum(np.abs(got) ** 2) - 1.0) < 1e-12


def test_network_slices_sum_to_unsliced_and_paths_agree():
    circ = circuits.random_circuit(3, 3, 6, seed=8)
    a = full_state_by_network(circ, path_seed=1)
    b = full_state_by_network(circ, path_seed=2, sliced_count=3)
    assert np.abs(a - b).max() < 1e-13


def test_network_ghz():
    for n in (3, 6):
        circ = circuits.ghz_circuit(n)
        for bits, expect in (([0] * n, 1 / math.sqrt(2)), ([1] * n, 1 / math.sqrt(2)),
                             ([1] + [0] * (n - 1), 0.0)):
            net = circuits.circuit_network(circ, bits)
            path = paths.greedy_path(net.labels, 4, restarts=1)
            amp, labels = oracle.contract_network(net.tensors, net.labels, path)
            assert labels == [] and abs(complex(amp) - expect) < 1e-15


def test_network_config2_amplitude_vs_statevector():
    w = configs.config2()
    assert len(w.sliced) == 4
    amp, _ = oracle.contract_network(w.network.tensors, w.network.labels, w.path, w.sliced)
    psi = oracle.statevector(w.circuit)
    x = int("".join(map(str, w.bitstring)), 2)
    assert abs(complex(amp) - psi[x]) < 1e-12 * max(abs(psi[x]), 2 ** -10)


def test_network_single_slices_are_projections_and_sum_to_the_sliced_result():
    # One slice of Section II.B is the network with each sliced bond fixed to
    # one basis value: checked against an independent projection (numpy
    # indexing of every tensor carrying the bond, the bond dropped from its
    # labels) contracted without slicing; the FP64 sum of all single slices
    # in ascending s is the sliced result bit for bit.  Slice s fixes
    # sliced[i] to bit nsliced-1-i of s (first sliced label most significant).
    w = configs.config2()
    net, path, sliced = w.network, w.path, w.sliced
    S = len(sliced)
    vals = oracle.contract_network_slices(net.tensors, net.labels, path, sliced,
                                          range(1 << S))
    total, _ = oracle.contract_network(net.tensors, net.labels, path, sliced)
    acc = 0j
    for v in vals:
        acc += v
    assert complex(total) == acc
    for s in (0, 5, (1 << S) - 1):
        fix = {lab: (s >> (S - 1 - i)) & 1 for i, lab in enumerate(sliced)}
        ts, ls = [], []
        for t, l in zip(net.tensors, net.labels):
            t = np.asarray(t).reshape((2,) * len(l))
            keep = []
            for j, lab in enumerate(l):
                if lab in fix:
                    t = np.take(t, fix[lab], axis=len(keep))
                else:
                    keep.append(lab)
            ts.append(np.ascontiguousarray(t))
            ls.append(keep)
        proj, labels = oracle.contract_network(ts, ls, path)
        assert labels == [] and complex(proj) == vals[s], s


def test_network_rejects_bad_path():
    circ = circuits.ghz_circuit(2)
    net = circuits.circuit_network(circ, [0, 0])
    bad = [(0, 0)] * (len(net.tensors) - 1)
    with pytest.raises(oracle.OracleError):
        oracle.contract_network(net.tensors, net.labels, bad)


# ------------------------------------------------------------ path helpers

def test_greedy_path_is_valid_and_slices_reduce_rank():
    w = configs.config2()
    n = len(w.network.tensors)
    live = set(range(n))
    for s, (a, b) in enumerate(w.path):
        assert a in live and b in live and a != b
        live -= {a, b}
        live.add(n + s)
    assert live == {n + len(w.path) - 1}
    r0, f0, _ = paths.path_stats(w.network.labels, w.path)
    r1, f1, _ = paths.path_stats(w.network.labels, w.path, w.sliced)
    assert r1 < r0 and f1 <= f0
