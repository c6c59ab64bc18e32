"""Helpers for the GPU parity tests: device upload and the FP tolerance checks.

The FP gates (stated for the fp16 mode): relative Frobenius error per channel
<= 2e-3 against the FP64 oracle, and, per element,
    |gpu - oracle| <= 2 * gamma(2K) * sum_k |w_k| |x_k|,
    gamma(n) = n u / (1 - n u),  u = 2^-24,
the classical worst-case bound for a recursive sum of 2K real products in fp32
(the products of two fp16 values are exact in fp32), doubled as margin for the
matrix unit's internal summation order.
"""
import sys

import numpy as np

U32 = 2.0 ** -24
REL_FRO_F16 = 2e-3


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.view(dtype)
    return t.to("cuda:0")


def words_to_dev(w):
    import torch
    return torch.from_numpy(np.ascontiguousarray(w).view(np.int32)).to("cuda:0")


def gamma(n):
    return n * U32 / (1.0 - n * U32)


def c_planar_to_complex(C):
    """[batch, 2, M, N] fp32 planar -> complex128."""
    C = np.asarray(C, np.float64)
    return C[:, 0] + 1j * C[:, 1]


def c_inter_to_complex(C):
    C = np.asarray(C, np.float64)
    return C[..., 0] + 1j * C[..., 1]


def check_fp_full(got, ref, absdot, K, rel=REL_FRO_F16):
    """got, ref complex [batch, M, N]; absdot real [batch, M, N] (sum |w||x|)."""
    for c in range(ref.shape[0]):
        num = np.linalg.norm(got[c] - ref[c])
        den = np.linalg.norm(ref[c])
        assert num <= rel * den + 1e-30, "channel %d: rel Frobenius %.3e" % (c, num / max(den, 1e-300))
    bound = 2.0 * gamma(2 * K) * absdot
    err = np.maximum(np.abs(got.real - ref.real), np.abs(got.imag - ref.imag))
    bad = err > bound
    assert not bad.any(), "elementwise bound violated at %d entries, worst %.3e vs %.3e" % (
        int(bad.sum()), float(err[bad].max()), float(bound[bad][np.argmax(err[bad])]))


def check_fp_entries(got, ref, absdot, K, rel=REL_FRO_F16):
    num = np.linalg.norm(got - ref)
    den = np.linalg.norm(ref)
    assert num <= rel * den, "sampled rel Frobenius %.3e" % (num / den)
    bound = 2.0 * gamma(2 * K) * absdot
    err = np.maximum(np.abs(got.real - ref.real), np.abs(got.imag - ref.imag))
    assert np.all(err <= bound), "elementwise bound violated: worst ratio %.3f" % float(np.max(err / bound))


def rel_fro(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
