"""Half-precision storage codec of the mixed-precision form (FP64 reference).

The paper does not fix a precision.  The mixed form stores spinors as IEEE
binary16 values of x / s with one FP32 scale s per site (s = the largest
absolute real or imaginary part over the site's components), and links as
binary16 without a scale (SU(3) entries are bounded by 1).  Rounding is
round-to-nearest-even (NumPy's float64 -> float16 conversion).  A decoded value
is half * s, so the round-trip error is at most 2^-11 * s per real component.
"""
from __future__ import annotations

import numpy as np


def encode_spinor(v, axis_sites=0):
    """v: complex (n_sites, ...) -> (half array of the reals (n_sites, 2*m), float32 scales)."""
    v = np.asarray(v)
    n = v.shape[axis_sites]
    re = np.stack([v.real, v.imag], axis=-1).reshape(n, -1)
    s = np.abs(re).max(axis=1)
    s32 = s.astype(np.float32)
    safe = np.where(s32 > 0, s32.astype(np.float64), 1.0)
    h = (re / safe[:, None]).astype(np.float16)
    return h, s32


def decode_spinor(h, s32, shape):
    re = h.astype(np.float64) * s32.astype(np.float64)[:, None]
    re = re.reshape(re.shape[0], -1, 2)
    return (re[..., 0] + 1j * re[..., 1]).reshape(shape)


def encode_links(U):
    """U complex -> half reals (same layout with a trailing re/im axis)."""
    U = np.asarray(U)
    return np.stack([U.real, U.imag], axis=-1).astype(np.float16)


def decode_links(h):
    h = h.astype(np.float64)
    return h[..., 0] + 1j * h[..., 1]
