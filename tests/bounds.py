"""Rounding-error bounds behind the tolerances of the GPU parity tests.

A dot product of n terms computed in a precision with unit roundoff u
satisfies |fl(x.y) - x.y| <= gamma_n |x|.|y|, gamma_n = n u / (1 - n u)
(Higham, Accuracy and Stability of Numerical Algorithms, Sec. 3.1).  The
kernels accumulate:

  * FP64: every term in FP64.
  * FP32 (the chi and NAF-metric SYRK, the NAF transform): in FP32 within
    blocks of 256 rows, then in FP64 across blocks; the error of an entry is
    at most (gamma_256(u32) + gamma_nb(u64)) times the sum of |terms|.
  * FP32 (the B.W.B contraction): the product with W^ in FP32 over all N
    terms, the row dot product in FP64.
  * BF16x3: each product as hi*hi + hi*lo + lo*hi of BF16 parts.  With
    round-to-nearest splits |x - hi| <= 2^-9 |x| and |x - hi - lo| <=
    2^-18 |x|, so the omitted lo*lo and the split residuals cost at most
    3 * 2^-18 |x y| per product, on top of the accumulation: the SYRK sums
    256 rows in the MFMA accumulators and adds each block into a second
    FP32 sum (blocked summation: gamma_{256 + nb}(u32)), the split-K slices
    in FP64.

Inputs rounded from FP64 to FP32 before the call add u32 per factor (3 u32
for a quadratic form x^T A x with x and A both rounded).
"""
import numpy as np

U64 = 2.0 ** -53
U32 = 2.0 ** -24
SPLIT3 = 3 * 2.0 ** -18


def gamma(n, u):
    return n * u / (1.0 - n * u)


def syrk_coeff(prec, rows, block=256):
    """Per-entry coefficient c of the blocked SYRK: |dK| <= c (|R|^T |R|)."""
    nb = max(1, -(-rows // block)) + 16          # blocks plus the split-K partial sums
    if prec == "fp64":
        return gamma(rows + 16, U64)
    if prec == "bf16x3":
        return gamma(block + nb, U32) + SPLIT3
    return gamma(block, U32) + gamma(nb, U64)


def quadform_coeff(prec, N, rounded_inputs):
    """Per-entry coefficient c of W_r = R_r^T W^ R_r from the B.W.B kernel:
    |dW_r| <= c (|R_r|^T |W^| |R_r|)."""
    if prec == "fp64":
        return gamma(N + 4, U64)
    c = gamma(N, U32) + gamma(2 * N // 64 + 4, U64)
    if prec == "bf16x3":
        c += SPLIT3
    if rounded_inputs:
        c += 3 * U32
    return c


def quadform_scale(R_rows, What):
    """S[j][r] = |R_r|^T |W^_j| |R_r| for rows R_rows [rows][N] and What [F][N][N]."""
    A = np.abs(R_rows)
    return np.stack([np.einsum("rp,pq,rq->r", A, np.abs(Wj), A, optimize=True)
                     for Wj in What])


def assert_quadform_close(W_gpu, W_ref, R_rows, What, prec, rounded_inputs):
    """Every W_nm entry within the bound of its own row and frequency."""
    F = What.shape[0]
    Wg = np.asarray(W_gpu).reshape(F, -1)
    Wr = np.asarray(W_ref).reshape(F, -1)
    S = quadform_scale(R_rows, What)
    c = quadform_coeff(prec, What.shape[-1], rounded_inputs)
    ratio = np.abs(Wg - Wr) / (c * S + 1e-300)
    worst = np.unravel_index(np.argmax(ratio), ratio.shape)
    assert ratio.max() <= 1.0, (f"W_nm entry (freq {worst[0]}, row {worst[1]}) off by "
                                f"{ratio.max():.2f} x its bound (c = {c:.2e})")
    return float(ratio.max())
