"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws random numbers and packs them into the canonical layouts;
it holds none of the solver's arithmetic (no stencil, no Krylov step, no
multigrid, no network).  The paper's physical 128x64^3 ensemble is not
available, so every workload is a synthetic stand-in with the same operator
parameters and the lattice shapes listed in ``CONFIGS``.

Canonical layouts (the C-ABI uses the same ones):

* lattice dims ``(T, Lz, Ly, Lx)``; site index ``s = ((t*Lz + z)*Ly + y)*Lx + x``;
  parity ``(t + z + y + x) mod 2``.  Direction ``mu = 0`` is time, ``1`` is x,
  ``2`` is y, ``3`` is z.
* gauge links ``U[s][mu][row][col]`` complex128, ``U_mu(x)`` connects x to x+mu.
* odd-site doublet spinor ``psi[h][flavour][spin][colour]`` complex128 with
  half index ``h = s >> 1`` over the odd sites (lexicographic order of the odd
  sites), shape ``(V/2, 2, 4, 3)``.
"""
from __future__ import annotations

import os

import numpy as np

KAPPA = 0.1275
MUBAR = 0.1408
EPSBAR = 0.1521


def geometric_shifts(n: int, smallest: float) -> np.ndarray:
    """n shifts sigma_k = smallest**(k/(n-1)), k=0..n-1, descending from 1."""
    k = np.arange(n, dtype=np.float64)
    return smallest ** (k / (n - 1))


CONFIGS = {
    # name: dims (T, Lz, Ly, Lx), gauge seed, rhs seed, shifts
    "c1": dict(dims=(4, 4, 4, 4), gauge_seed=11, rhs_seed=21, amp=0.3,
               shifts=geometric_shifts(10, 1e-4)),
    "c2": dict(dims=(32, 16, 16, 16), gauge_seed=12, rhs_seed=22, amp=0.3,
               shifts=geometric_shifts(12, 1e-5)),
    "c3": dict(dims=(48, 24, 24, 24), gauge_seed=13, rhs_seed=23, amp=0.3,
               shifts=geometric_shifts(12, 1e-5)),
    "c4": dict(dims=(64, 32, 32, 32), gauge_seed=14, rhs_seed=24, amp=0.3,
               shifts=geometric_shifts(12, 1e-5)),
    "c5": dict(dims=(96, 48, 48, 48), gauge_seed=15, rhs_seed=25, amp=0.3,
               shifts=geometric_shifts(12, 1e-5)),
}

# Gell-Mann matrices lambda_1..lambda_8 (generators of su(3) are lambda_a/2).
_GM = np.zeros((8, 3, 3), dtype=np.complex128)
_GM[0][0, 1] = _GM[0][1, 0] = 1
_GM[1][0, 1] = -1j
_GM[1][1, 0] = 1j
_GM[2][0, 0] = 1
_GM[2][1, 1] = -1
_GM[3][0, 2] = _GM[3][2, 0] = 1
_GM[4][0, 2] = -1j
_GM[4][2, 0] = 1j
_GM[5][1, 2] = _GM[5][2, 1] = 1
_GM[6][1, 2] = -1j
_GM[6][2, 1] = 1j
_GM[7][0, 0] = _GM[7][1, 1] = 1 / np.sqrt(3)
_GM[7][2, 2] = -2 / np.sqrt(3)


def volume(dims) -> int:
    return int(np.prod(dims))


def _exp_i_amp_h(h: np.ndarray, amp: float) -> np.ndarray:
    """exp(i*amp*H) for H = sum_a h_a lambda_a / 2, one link per row of h (n x 8)."""
    H = np.einsum("na,aij->nij", h, _GM) * 0.5
    w, vec = np.linalg.eigh(H)
    ph = np.exp(1j * amp * w)
    return np.einsum("nij,nj,nkj->nik", vec, ph, vec.conj())


def gauge_field(dims, seed: int, amp: float = 0.3, chunk: int = 1 << 20, workers: int | None = None) -> np.ndarray:
    """U = exp(i*amp*H) per link, H = sum_a h_a lambda_a / 2, h_a ~ N(0,1) iid.

    Returns complex128 array of shape (V, 4, 3, 3).  The exponential is taken
    through the eigendecomposition of the Hermitian H, so U is unitary with
    unit determinant to rounding.  Generated in chunks of links so that large
    lattices fit in host memory.  The normal deviates are always drawn in link
    order from one generator.  With ``workers`` > 1 the exponentials of the
    chunks are taken by that many forked processes, which gives the same array
    as the serial loop; call it so only before the process has touched a GPU.
    """
    V = volume(dims)
    n = 4 * V
    rng = np.random.default_rng(seed)
    out = np.empty((n, 3, 3), dtype=np.complex128)
    n_chunks = (n + chunk - 1) // chunk
    if n_chunks <= 2 or not workers or workers <= 1:
        for lo in range(0, n, chunk):
            hi = min(n, lo + chunk)
            out[lo:hi] = _exp_i_amp_h(rng.standard_normal((hi - lo, 8)), amp)
        return out.reshape(V, 4, 3, 3)
    import concurrent.futures as cf
    import multiprocessing as mp

    with cf.ProcessPoolExecutor(max_workers=min(workers, os.cpu_count() or 1),
                                mp_context=mp.get_context("fork")) as ex:
        pending = []
        for lo in range(0, n, chunk):
            hi = min(n, lo + chunk)
            pending.append((lo, hi, ex.submit(_exp_i_amp_h, rng.standard_normal((hi - lo, 8)), amp)))
            while len(pending) > 2 * workers:
                a, b_, f = pending.pop(0)
                out[a:b_] = f.result()
        for a, b_, f in pending:
            out[a:b_] = f.result()
    return out.reshape(V, 4, 3, 3)


def gaussian_spinor(dims, seed: int, sites: str = "odd") -> np.ndarray:
    """Doublet spinor with Re and Im iid N(0,1).

    sites="odd": shape (V/2, 2, 4, 3) on the odd sites; "full": (V, 2, 4, 3).
    """
    V = volume(dims)
    n = V // 2 if sites == "odd" else V
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((n, 2, 4, 3))
    im = rng.standard_normal((n, 2, 4, 3))
    return re + 1j * im


def gaussian_vectors(shape, seed: int) -> np.ndarray:
    """Complex Gaussian array of any shape (Re, Im iid N(0,1))."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def random_su3(n: int, seed: int) -> np.ndarray:
    """n Haar-ish random SU(3) matrices (QR of a complex Gaussian, phases fixed)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[:, None, None]
    return q


def unit_gauge(dims) -> np.ndarray:
    V = volume(dims)
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1
    return U
