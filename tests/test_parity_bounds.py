"""CPU checks of the parity machinery the GPU tests rely on.

The element-wise bounds of tests/parity.py are checked against simulations
of each mode's arithmetic in numpy (float32 products and sums, the bf16
hi/lo split done on the bits), and shown to reject planted mistakes: one
output off by 4e-4 relative, and a split-BF16 product that drops a cross
term.  The exact-split inputs (odd nine-bit integers against units) are
shown to make every mode's arithmetic exact while a dropped cross term is
not.  Also pins the bulk generators of those inputs to their numpy form.
"""
import numpy as np
import pytest

import parity
from workloads import rng

M, N = 24, 20


def bf16_round(x):
    """Nearest bfloat16 (ties to even) of float32 values, as float32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32)


def split(x):
    hi = bf16_round(x)
    lo = bf16_round((x - hi).astype(np.float32))
    return hi, lo


def sim(mode, a, b, drop=None):
    """C = a @ b (complex, M x K times K x N) in the arithmetic of `mode`;
    drop = "lohi" or "hilo" leaves out that cross term of split BF16."""
    if mode == "fp64":
        return a @ b
    a, b = a.astype(np.complex64), b.astype(np.complex64)
    ar, ai, br, bi = (np.ascontiguousarray(v, dtype=np.float32)
                      for v in (a.real, a.imag, b.real, b.imag))
    f = np.float32
    if mode == "fp32_4m":
        re = (ar @ br).astype(f) - (ai @ bi).astype(f)
        im = (ar @ bi).astype(f) + (ai @ br).astype(f)
    elif mode == "fp32_3m":
        t1, t2 = (ar @ br).astype(f), (ai @ bi).astype(f)
        t3 = ((ar + ai).astype(f) @ (br + bi).astype(f)).astype(f)
        re, im = t1 - t2, (t3 - t1) - t2
    else:
        (arh, arl), (aih, ail), (brh, brl), (bih, bil) = map(split, (ar, ai, br, bi))

        def prod(xh, xl, yh, yl):
            s = (xh @ yh).astype(f)
            if drop != "lohi":
                s = s + (xl @ yh).astype(f)
            if drop != "hilo":
                s = s + (xh @ yl).astype(f)
            return s

        if mode == "bf16x3_3m":  # Gauss form on planar splits of re, im, re + im
            (sah, sal), (sbh, sbl) = split((ar + ai).astype(f)), split((br + bi).astype(f))
            t1, t2 = prod(arh, arl, brh, brl), prod(aih, ail, bih, bil)
            t3 = prod(sah, sal, sbh, sbl)
            re, im = t1 - t2, (t3 - t1) - t2
        else:
            re = prod(arh, arl, brh, brl) - prod(aih, ail, bih, bil)
            im = prod(arh, arl, bih, bil) + prod(aih, ail, brh, brl)
    return re.astype(np.float64) + 1j * im.astype(np.float64)


def normal(seed, shape):
    return rng.complex_normal(seed, int(np.prod(shape))).reshape(shape)


@pytest.mark.parametrize("mode", ["fp64", "fp32_4m", "fp32_3m", "bf16x3", "bf16x3_3m"])
@pytest.mark.parametrize("K", [1, 16, 1024])
def test_simulated_arithmetic_within_bound(mode, K):
    # "bf16x3" simulates the 4M split form, "bf16x3_3m" the Gauss split form;
    # each is held to its own form's bound and to the mode's (the larger).
    a, b = normal(11 + K, (M, K)), normal(12 + K, (K, N))
    ref = a @ b
    absprod = np.abs(a) @ np.abs(b)
    own = {"bf16x3": "bf16x3_4m"}.get(mode, mode)
    r = parity.check(sim(mode, a, b), ref, absprod, K, own, "simulated")
    assert r["higham"] <= r["higham_bound"]
    if mode.startswith("bf16"):
        parity.check(sim(mode, a, b), ref, absprod, K, "bf16x3", "simulated")


def test_bound_constants():
    # Large-K limits of g / (K u): 2 sqrt 2 for 4M, sqrt 10 for Gauss,
    # 6 sqrt 2 (1 + 2^-8)^2 (1 + 2^-7) for split BF16 (plus the split term).
    K = 1 << 14
    u = 2.0 ** -24
    assert abs(parity.bound_factor("fp32_4m", K) / (K * u) / (2 * np.sqrt(2)) - 1) < 3e-3
    assert abs(parity.bound_factor("fp32_3m", K) / (K * u) / np.sqrt(10) - 1) < 3e-3
    g = parity.bound_factor("bf16x3_4m", K) / (K * u)
    assert 6 * np.sqrt(2) < g < 6 * np.sqrt(2) * 1.03 + 3 * np.sqrt(2) * 256 / K + 0.01
    # Gauss split form: dRe -> 2 E, dIm -> 4 E with E -> 3 K u m_s, so
    # sqrt(6^2 + 12^2) m_s (plus the split term); the mode takes the larger
    # of the two forms.
    m_s = (1 + 2.0 ** -8) ** 2 * (1 + 2.0 ** -7)
    g3 = parity.bound_factor("bf16x3_3m", K) / (K * u)
    assert np.hypot(6, 12) * m_s < g3 < np.hypot(6, 12) * m_s * 1.01 + 20 * 256 / K
    assert parity.bound_factor("bf16x3", K) == max(parity.bound_factor("bf16x3_4m", K),
                                                   parity.bound_factor("bf16x3_3m", K))


def test_planted_single_entry_error_fails():
    a, b = normal(21, (M, 4096)), normal(22, (4096, N))
    ref = a @ b
    got = sim("fp32_4m", a, b)
    parity.check(got, ref, np.abs(a) @ np.abs(b), 4096, "fp32_4m")
    got[3, 5] += 4e-4 * abs(ref[3, 5])
    with pytest.raises(AssertionError):
        parity.check(got, ref, np.abs(a) @ np.abs(b), 4096, "fp32_4m")


def test_planted_dropped_cross_term_fails_bound_at_small_k():
    a, b = normal(31, (M, 64)), normal(32, (64, N))
    ref = a @ b
    with pytest.raises(AssertionError):
        parity.check(sim("bf16x3", a, b, drop="hilo"), ref, np.abs(a) @ np.abs(b), 64,
                     "bf16x3")


@pytest.mark.parametrize("order", [("wide", "unit"), ("unit", "wide")])
def test_exact_split_inputs(order):
    K = 4096
    gen = {"wide": rng.wide_odd_integers, "unit": rng.unit_values}
    a = gen[order[0]](41, M * K).reshape(M, K)
    b = gen[order[1]](42, K * N).reshape(K, N)
    ref = a @ b
    wide = a if order[0] == "wide" else b
    assert np.all(bf16_round(wide.real.astype(np.float32)) != wide.real)  # lo != 0
    for mode in ("fp64", "fp32_4m", "fp32_3m", "bf16x3", "bf16x3_3m"):
        assert np.array_equal(sim(mode, a, b), ref), mode
    # The cross term that multiplies the wide operand's low part is needed
    # for exactness (so a kernel that drops it fails); the other one
    # multiplies zeros here, which is why both orders are tested.
    needed, idle = ("lohi", "hilo") if order[0] == "wide" else ("hilo", "lohi")
    assert not np.array_equal(sim("bf16x3", a, b, drop=needed), ref)
    assert np.array_equal(sim("bf16x3", a, b, drop=idle), ref)


def test_exact_split_generators_native_matches_numpy():
    for n in (1, 5, 4097):
        assert np.array_equal(rng.wide_odd_integers(77, n), rng.wide_odd_integers_numpy(77, n))
        assert np.array_equal(rng.unit_values(78, n), rng.unit_values_numpy(78, n))
    w = rng.wide_odd_integers(79, 10000)
    for part in (w.real, w.imag):
        m = np.abs(part)
        assert m.min() >= 257 and m.max() <= 511 and np.all(m % 2 == 1)
        assert (part < 0).any() and (part > 0).any()
    u = rng.unit_values(80, 10000)
    assert set(np.unique(u).tolist()) == {0, 1, -1, 1j, -1j}
