"""Element-wise error bounds for the mixed-precision kernels (FP16-stored
links and prolongators, FP32 vectors, operators and arithmetic), used by the
GPU parity tests.

The reference is the oracle's FP64 product on the SAME FP32-rounded input, so
the bound only has to cover what the kernel itself rounds:
  * an FP16-stored complex value z carries |dz| <= 2^-11 |z| (each component
    rounds to nearest with unit roundoff 2^-11);
  * an FP32-stored value 2^-24 |z|;
  * FP32 accumulation of K products adds at most K * 2^-24 times the sum of
    the absolute values of the terms (the usual gamma_K bound), doubled for
    the three-product complex multiplication of the MFMA kernels, whose
    imaginary part combines (|a_r| + |a_i|)(|b_r| + |b_i|) <= 2 |a| |b|.
Each output i is compared with c * T_i, T_i = (|M| |v|)_i the sum of the
absolute values of its terms."""
import numpy as np
import scipy.sparse as sp

U16 = 2.0 ** -11
U32 = 2.0 ** -24


def fp16_coef(nterms):
    """Per-term coefficient for FP16-stored operator values, FP32 arithmetic."""
    return U16 + 4.0 * (nterms + 4) * U32


def fp32_coef(nterms):
    """Per-term coefficient for FP32-stored operator values and FP32 MFMA/SIMT
    accumulation over nterms products."""
    return 4.0 * (nterms + 4) * U32


def abs_terms(M, v):
    """(|M| |v|) for a sparse or dense operator M and vectors v [nrhs][n]."""
    Ma = abs(M) if sp.issparse(M) else np.abs(M)
    return (Ma @ np.abs(v).T).T


def rounded(v, dtype=np.complex64):
    """The FP32 input the kernel sees, widened back for the reference."""
    return np.asarray(v).astype(dtype).astype(np.complex128)


def check_elementwise(got, ref, terms, c, what=""):
    """|got - ref| <= c * terms for every element; returns max err / bound."""
    err = np.abs(np.asarray(got).astype(np.complex128) - ref)
    bound = c * terms
    ratio = float(np.max(err / np.maximum(bound, 1e-300)))
    assert ratio <= 1.0, "%s: max |err| / bound = %.3g" % (what, ratio)
    return ratio
