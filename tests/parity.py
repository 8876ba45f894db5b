"""Element-wise parity bounds shared by the GPU tests (test infrastructure).

A GPU result C is compared with the oracle's C_ref (complex128, computed on
the original complex128 inputs) three ways:

  e_F   = ||C - C_ref||_F / ||C_ref||_F over the compared entries,
  e_max = max |C - C_ref| / max |C_ref|,
both below the mode's tolerance (1e-12 FP64, 1e-5 FP32, 1e-3 split BF16),
and, entry by entry, the a-priori rounding-error bound of the mode's
arithmetic,

  |C_ij - C_ref,ij| <= g(mode, K) * (|A| |B|)_ij,

where (|A||B|)_ij = sum_k |a_ik| |b_kj| is the same contraction taken on the
entries' magnitudes (computed by the oracle) and K is the number of complex
terms per output.  The reported Higham ratio is
|C_ij - C_ref,ij| / (K u (|A||B|)_ij), u the unit roundoff of the mode's
accumulation format (2^-53 FP64, 2^-24 otherwise); the bound is that ratio
<= g / (K u).

g follows the arithmetic of each mode (Higham, "Accuracy and Stability of
Numerical Algorithms", 2nd ed., Section 3.1: a real dot product of n terms
evaluated in any order, every product and sum rounded once,
has error <= gamma_n sum |x_i y_i| with gamma_n = n u / (1 - n u)):

  4M:    each real part of C is a real dot product of 2K terms whose
         magnitudes add up to at most (|A||B|)_ij, so
         |dC| <= sqrt(2) gamma_2K (|A||B|)_ij.
  Gauss (3M): T1 = Ar.Br, T2 = Ai.Bi (K terms each), T3 = (Ar+Ai).(Br+Bi)
         with the two sums rounded first (K terms, each |.| <= 2|a||b|),
         Re = T1 - T2, Im = (T3 - T1) - T2:
         |dRe| <= (gamma_K + u (1 + gamma_K)) S,
         |dIm| <= (2 gamma_(K+2) + gamma_K + 7.01 u (1 + gamma_(K+2))) S,
         S = (|A||B|)_ij, and |dC| <= sqrt(dRe^2 + dIm^2).
  split BF16x3: x = hi + lo + e with hi = bf16(x), lo = bf16(x - hi),
         |e| <= 2^-16 |x|; the dropped lo*lo and the split residues leave
         each real product off by at most e_s |x||y|,
         e_s = 2 * 2^-16 + 2^-32 + 2^-16 (1 + 2^-8)^2; the three exact
         bf16 products of each of the 2K real products (6K terms, their
         magnitudes at most m_s |x||y|, m_s = (1 + 2^-8)^2 (1 + 2^-7)) are
         summed in FP32: |dC| <= sqrt(2) (e_s + m_s gamma_6K) S.
  split BF16x3, Gauss form (the planar tile): T1 = Ar.Br, T2 = Ai.Bi and
         T3 = sa.sb with sa = fl(Ar + Ai), sb = fl(Br + Bi), each a split
         product of K terms (3K exact bf16 products summed in FP32), so
         |dT1|, |dT2| <= E S with E = e_s + m_s gamma_3K, and, since
         sum (|ar| + |ai|)(|br| + |bi|) <= 2 S and the two sums add
         (2u + u^2) relative, |dT3| <= 2 E3 S with
         E3 = E (1 + u)^2 + 2u + u^2; Re = T1 - T2 and Im = (T3 - T1) - T2
         add their roundings:
         |dRe| <= 2 E S + 2u (1 + E) S,
         |dIm| <= (2 E3 + 2 E) S + u (7 + 4 E3 + 3 E) (1 + u)^2 S.
         The split-BF16 mode may run either form, so its bound is the larger.
  FP32 and split-BF16 modes take the complex128 inputs rounded once to
  complex64 (relative u per part): that adds (2u + u^2) S and scales the
  bounds above by (1 + u)^2.  FP64 mode may run the 4M or the Gauss tile, so
  its bound is the larger of the two.
"""
from __future__ import annotations

import math

import numpy as np

TOL = {"fp64": 1e-12, "fp32_4m": 1e-5, "fp32_3m": 1e-5, "bf16x3": 1e-3, "bf16x3_4m": 1e-3,
       "bf16x3_3m": 1e-3}
UNIT = {"fp64": 2.0 ** -53, "fp32_4m": 2.0 ** -24, "fp32_3m": 2.0 ** -24, "bf16x3": 2.0 ** -24,
        "bf16x3_4m": 2.0 ** -24, "bf16x3_3m": 2.0 ** -24}


def _gamma(n: float, u: float) -> float:
    return n * u / (1.0 - n * u)


def _bound_4m(K: int, u: float) -> float:
    return math.sqrt(2.0) * _gamma(2 * K, u)


def _bound_gauss(K: int, u: float) -> float:
    g_k, g_k2 = _gamma(K, u), _gamma(K + 2, u)
    d_re = g_k + u * (1.0 + g_k)
    d_im = 2.0 * g_k2 + g_k + 7.01 * u * (1.0 + g_k2)
    return math.hypot(d_re, d_im)


def _bound_bf16x3(K: int, u: float) -> float:
    b = 2.0 ** -8
    e_s = 2.0 * b * b + b ** 4 + b * b * (1.0 + b) ** 2
    m_s = (1.0 + b) ** 2 * (1.0 + 2.0 * b)
    return math.sqrt(2.0) * (e_s + m_s * _gamma(6 * K, u))


def _bound_bf16x3_gauss(K: int, u: float) -> float:
    b = 2.0 ** -8
    e_s = 2.0 * b * b + b ** 4 + b * b * (1.0 + b) ** 2
    m_s = (1.0 + b) ** 2 * (1.0 + 2.0 * b)
    e = e_s + m_s * _gamma(3 * K, u)
    e3 = e * (1.0 + u) ** 2 + 2.0 * u + u * u
    d_re = 2.0 * e + 2.0 * u * (1.0 + e)
    d_im = 2.0 * e3 + 2.0 * e + u * (7.0 + 4.0 * e3 + 3.0 * e) * (1.0 + u) ** 2
    return math.hypot(d_re, d_im)


def bound_factor(mode: str, K: int) -> float:
    """g(mode, K): |dC_ij| <= g * (|A||B|)_ij for K complex terms per output."""
    K = max(int(K), 1)
    u = UNIT[mode]
    if mode == "fp64":
        return max(_bound_4m(K, u), _bound_gauss(K, u))
    if mode == "fp32_4m":
        g = _bound_4m(K, u)
    elif mode == "fp32_3m":
        g = _bound_gauss(K, u)
    elif mode == "bf16x3_4m":  # one form alone (simulations)
        g = _bound_bf16x3(K, u)
    elif mode == "bf16x3_3m":
        g = _bound_bf16x3_gauss(K, u)
    else:
        g = max(_bound_bf16x3(K, u), _bound_bf16x3_gauss(K, u))
    return g * (1.0 + u) ** 2 + 2.0 * u + u * u


def abs_product_blocked(p) -> np.ndarray:
    """(|A||B|) of a configs.Problem in C's block-major order (oracle)."""
    import oracle
    ref, _, _ = oracle.block_tensordot(np.abs(p.a.data), p.a.dims, p.a.grid, np.abs(p.b.data),
                                       p.b.dims, p.b.grid, p.axes_a, p.axes_b)
    return ref.real


def abs_product_entries(a, b, axes_a, axes_b, idx) -> np.ndarray:
    """(|A||B|) at flat output indices idx of tensordot(a, b) (oracle)."""
    import oracle
    return oracle.tensordot_entries(np.abs(a), np.abs(b), axes_a, axes_b, idx).real


def contracted_size(dims_a, axes_a) -> int:
    return int(np.prod([dims_a[j] for j in axes_a], dtype=np.int64)) if len(axes_a) else 1


def report(got, ref, absprod, K, mode) -> dict:
    """e_F, e_max, the largest Higham ratio and its bound (no assertion)."""
    got = np.asarray(got, dtype=np.complex128).reshape(-1)
    ref = np.asarray(ref, dtype=np.complex128).reshape(-1)
    absprod = np.asarray(absprod, dtype=np.float64).reshape(-1)
    d = np.abs(got - ref)
    nref = np.linalg.norm(ref)
    e_f = float(np.linalg.norm(got - ref) / nref) if nref > 0 else float(np.linalg.norm(got))
    mref = float(np.max(np.abs(ref))) if ref.size else 0.0
    e_max = float(d.max() / mref) if mref > 0 else float(d.max() if d.size else 0.0)
    u = UNIT[mode]
    g = bound_factor(mode, K)
    scale = max(int(K), 1) * u * absprod
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(scale > 0, d / np.where(scale > 0, scale, 1.0),
                         np.where(d > 0, np.inf, 0.0))
    worst = int(np.argmax(ratio)) if ratio.size else 0
    return {"e_F": e_f, "e_max": e_max, "higham": float(ratio.max()) if ratio.size else 0.0,
            "higham_bound": g / (max(int(K), 1) * u), "worst_index": worst,
            "over_bound": int(np.count_nonzero(d > g * absprod))}


def check(got, ref, absprod, K, mode, what: str = "") -> dict:
    """Assert e_F and e_max below the mode's tolerance and every entry within
    its a-priori bound; returns the report."""
    r = report(got, ref, absprod, K, mode)
    tag = f"{what} {mode} K={K}".strip()
    print(f"  {tag}: e_F={r['e_F']:.3e} e_max={r['e_max']:.3e} "
          f"higham={r['higham']:.3e} (bound {r['higham_bound']:.3g})", flush=True)
    assert r["e_F"] < TOL[mode], (tag, "e_F", r)
    assert r["e_max"] < TOL[mode], (tag, "e_max", r)
    assert r["over_bound"] == 0, (tag, "entries over the rounding bound", r)
    return r
