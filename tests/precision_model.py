"""Host model of each precision form's operand rounding (test code).

The GPU path contracts with rounded operands: 2 theta'_j as FP32, as BF16
limbs, or as two BF16 limbs and a scaled FP8 one in the forward, the backward weights S_ki = u_k / s * sin(E_ki) as FP32,
BF16 limbs, a BF16 limb plus a row-scaled FP8 limb, or 8-bit fixed-point
limbs. Feeding the same rounded operands
through the FP64 oracle gives the result the arithmetic itself defines, so a
tolerance can be tied to the form: the gap between this emulation and the
exact oracle is the form's representation error, and the gap between the GPU
and this emulation is the kernels' own (accumulation order, FP32 sums).

Written from the definitions (round to nearest even on the bit patterns, the
reduction of theta by whole multiples of pi); it shares nothing with the HIP
sources.
"""
import numpy as np

import oracle

# fixed-point scale of the 16-bit backward weights: |S_ki| <= sigma_k maps to
# at most 32639 = 127 * 256 + 127, the largest value two signed 8-bit limbs
# (hi in [-127, 127], lo in [-128, 127]) hold with hi = floor((N + 128) / 256)
I8X2_MAX = 32639.0
# the third theta limb of split3_bf16 holds E4M3(rest * 2^LO8_EXP)
LO8_EXP = 20


def bf16_rne(x):
    """Round float32 values to the nearest BF16 (ties to even), returned as
    float64."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def e4m3_rne(y):
    """Round to the nearest OCP FP8 E4M3 value (ties to even), for |y| within
    its range (at most 448): 4 significant bits, exponent bias 7, subnormal
    spacing 2^-9. Written from the format's definition."""
    y = np.asarray(y, dtype=np.float64)
    a = np.abs(y)
    _, x = np.frexp(a)                     # a = f 2^x, f in [0.5, 1)
    e = np.maximum(x - 1, -6)              # binade, clamped to the subnormal one
    quantum = np.ldexp(1.0, e - 3)
    r = np.rint(a / quantum) * quantum
    assert np.all(r <= 448.0), "outside the E4M3 range"
    return np.copysign(r, y)


def fp16_row_exponent(bound):
    """Per-row scale exponent e_k of the FP16 + FP8 weights: with
    bound_k = f 2^x, f in [1/2, 1) (frexp), e_k = 15 - x puts bound_k 2^e_k in
    [2^14, 2^15), clamped to [-120, 120]; 0 for a zero or non-finite bound."""
    bound = np.asarray(bound, dtype=np.float64)
    ok = np.isfinite(bound) & (bound > 0)
    _, x = np.frexp(np.where(ok, bound, 1.0))
    return np.where(ok, np.clip(15 - x, -120, 120), 0)


def two_theta_reduced(theta):
    """2 theta' with theta' = theta - pi * rint(theta / pi) in FP64 (a shift
    by pi is a global phase of the gate, so results do not change)."""
    theta = np.asarray(theta, dtype=np.float64)
    return 2.0 * (theta - np.pi * np.rint(theta / np.pi))


def bf16_limbs(t, k):
    """k BF16 limbs of t: each the RNE of the FP32 rounding of what the
    previous ones left (the first of t itself)."""
    out = np.zeros_like(t)
    for _ in range(k):
        out = out + bf16_rne((t - out).astype(np.float32))
    return out


def theta_represented(prec, theta):
    """The angles whose doubles the form contracts with exactly: theta~ with
    2 theta~_j equal to the kernel's representation of 2 theta'_j."""
    t = two_theta_reduced(theta)
    if prec in ("fp32", "sparse_fp32"):
        r = t.astype(np.float32).astype(np.float64)
    elif prec in ("split_bf16", "split_bf16_fp8"):
        r = bf16_limbs(t, 2)
    elif prec == "split3_bf16":
        # hi and mid BF16, then the rest as E4M3 of rest * 2^20 (from FP32)
        hm = bf16_limbs(t, 2)
        rest = (t - hm) * 2.0 ** LO8_EXP
        r = hm + e4m3_rne(rest.astype(np.float32).astype(np.float64)) * 2.0 ** -LO8_EXP
    else:
        raise ValueError(prec)
    return r / 2.0


def weights_represented(prec, S, bound):
    """The backward weights as the form holds them; bound[k] >= |S[k, :]| is
    the per-observable bound the fixed-point form scales by."""
    S = np.asarray(S, dtype=np.float64)
    if prec in ("fp32", "sparse_fp32"):
        return S.astype(np.float32).astype(np.float64)
    if prec == "split_bf16":
        return bf16_limbs(S.astype(np.float32).astype(np.float64), 2)
    if prec == "split_bf16_fp8":
        # x = S 2^e_k (exact), FP16 limb rn(x), FP8 limb rn_e4m3(x - rn(x))
        e = fp16_row_exponent(bound)[:, None]
        x = np.ldexp(S.astype(np.float32).astype(np.float64), e)
        hi = x.astype(np.float16).astype(np.float64)
        return np.ldexp(hi + e4m3_rne(x - hi), -e)
    if prec == "split3_bf16":
        q = np.where(bound > 0, bound / I8X2_MAX, 0.0)[:, None]
        N = np.rint(np.divide(S, q, out=np.zeros_like(S), where=q > 0))
        return N * q
    raise ValueError(prec)


def grad_emulated(n, gates, theta, ops01, samples01, u, prec=None):
    """dL/dtheta for L = sum_k u_k mean_k with the operands of form `prec`
    (None: exact FP64): phases from the oracle at the represented angles,
    S_ki = u_k / s sin(E_ki) rounded as the form holds it, then
    -2 sum_k C_kj (S B)_kj with B_ij = (-1)^{z_i . g_j} (the reverse pass of
    eq. Emat, Fig. 3)."""
    u = np.asarray(u, dtype=np.float64)
    s = samples01.shape[0]
    th = theta if prec is None else theta_represented(prec, theta)
    _, _, ph = oracle.expval(n, gates, th, ops01, samples01, phases=True)
    S = (u[:, None] / s) * np.sin(ph)
    if prec is not None:
        S = weights_represented(prec, S, np.abs(u) / s)
    C = oracle.parity(n, ops01, gates).astype(np.float64)
    B = 1.0 - 2.0 * oracle.parity(n, samples01, gates).astype(np.float64)
    return -2.0 * (C * (S @ B)).sum(axis=0)
