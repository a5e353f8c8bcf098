"""Elementwise error bounds of the grouped packed product's passes, shared by
the batch parity tests."""
import numpy as np


U32 = 2.0 ** -24     # unit roundoff of FP32


def product_bound(mat, unit, Zabs, Xabs):
    """Elementwise bound on |(T x)_i - (T_oracle x)_i| for the grouped product,
    from the arithmetic of each pass, with S_i = sum_j |T_ij| |x_j| (oracle
    magnitudes) and e64 = 1e-12 max|T| sum_j |x_j| for the difference between
    the library's and the oracle's FP64 fills:
      fp64, fp64_mfma   e64 (FP64 tiles and accumulation, vector units or
                 FP64 matrix cores);
      fp32       sqrt(2) u S_i + e64 (each FP32 entry is the FP64 entry rounded:
                 re and im each within u relative; FP64 accumulation);
      fp32_mfma  (2 sqrt(2) u + 5 sqrt(n) u) S_i + e64: entries and vector
                 entries rounded to FP32, and the FP32 accumulation of n = 2 x 64
                 x unit real terms per output within a unit, taken with the
                 probabilistic bound lambda sqrt(n) u (Higham and Mary, 2019) at
                 lambda = 5; the units' partial sums are added in FP64.
    Zabs (N x N) and Xabs (R x N) are |T_oracle| and |X|; returns R x N."""
    S = Xabs @ Zabs.T
    e64 = 1e-12 * Zabs.max() * Xabs.sum(axis=1, keepdims=True)
    if mat in ("fp64", "fp64_mfma"):
        return e64 + 0 * S
    if mat == "fp32":
        return np.sqrt(2) * U32 * S + e64
    n = 2 * 64 * unit
    return (2 * np.sqrt(2) + 5 * np.sqrt(n)) * U32 * S + e64
