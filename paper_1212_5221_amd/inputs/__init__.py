"""Seeded synthetic gauge configurations (input generator).

The C source ``gen.c`` next to this file produces links in the natural
layout (t, x, y, z, mu, i, j, re/im; z fastest; FP64, 18 reals per link).  It
holds no gauge-fixing arithmetic; the CPU oracle and the GPU library both take
its output as their input.

Recipes (all keyed by a 64-bit seed, independent of thread count):

* ``smooth(dims, eps, seed)``: U_mu(x) = h(x) exp(i eps sum_a lambda_a xi_a) h(x+mu)^dag
* ``pure_gauge(dims, seed)``: U_mu(x) = h(x) h(x+mu)^dag
* ``hot(dims, seed)``: Haar-random links
* ``gauge_copy(U, dims, seed)``: a random gauge transform of U (Gribov copies)

and, for the gauge group SU(2) (numpy, links (V, 4, 2, 2, 2)), ``su2_hot``,
``su2_smooth``, ``su2_pure_gauge``, ``su2_gauge_field`` and ``su2_gauge_copy``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libgfgen.so")
_lib = None

_I32_4 = ctypes.c_int32 * 4


def build(force: bool = False) -> str:
    """Compile gen.c into libgfgen.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
             "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        u64 = ctypes.c_uint64
        lib.gen_smooth.argtypes = [_I32_4, ctypes.c_double, u64, ctypes.c_int32, ctypes.c_int32, dp]
        lib.gen_pure_gauge.argtypes = [_I32_4, u64, ctypes.c_int32, ctypes.c_int32, dp]
        lib.gen_hot.argtypes = [_I32_4, u64, ctypes.c_int32, ctypes.c_int32, dp]
        lib.gen_gauge_copy.argtypes = [_I32_4, u64, dp]
        lib.gen_haar_field.argtypes = [_I32_4, u64, ctypes.c_int64, ctypes.c_int64, dp]
        lib.gen_link_exponential.argtypes = [dp, ctypes.c_double, dp]
        lib.gen_link_xi.argtypes = [u64, ctypes.c_int64, ctypes.c_int32, dp]
        lib.gen_philox4x64_10.argtypes = [ctypes.POINTER(ctypes.c_uint64)] * 3
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _dims(dims) -> "ctypes.Array":
    d = [int(x) for x in dims]
    if len(d) != 4 or any(x < 1 for x in d):
        raise ValueError("dims must be four positive extents (Nt, Nx, Ny, Nz)")
    return _I32_4(*d)


def _slab(dims, t0, nt):
    if nt is None:
        nt = int(dims[0]) - t0
    if t0 < 0 or nt < 0 or t0 + nt > int(dims[0]):
        raise ValueError("time slab out of range")
    vs = int(dims[1]) * int(dims[2]) * int(dims[3])
    return t0, nt, vs


def smooth(dims, eps: float, seed: int, t0: int = 0, nt: int | None = None, out=None) -> np.ndarray:
    """Smooth configuration (links of time-slices [t0, t0+nt)), shape (sites, 4, 3, 3, 2)."""
    t0, nt, vs = _slab(dims, t0, nt)
    if out is None:
        out = np.empty((nt * vs, 4, 3, 3, 2), dtype=np.float64)
    _load().gen_smooth(_dims(dims), float(eps), int(seed), t0, nt, _dp(out))
    return out


def pure_gauge(dims, seed: int, t0: int = 0, nt: int | None = None, out=None) -> np.ndarray:
    t0, nt, vs = _slab(dims, t0, nt)
    if out is None:
        out = np.empty((nt * vs, 4, 3, 3, 2), dtype=np.float64)
    _load().gen_pure_gauge(_dims(dims), int(seed), t0, nt, _dp(out))
    return out


def hot(dims, seed: int, t0: int = 0, nt: int | None = None, out=None) -> np.ndarray:
    t0, nt, vs = _slab(dims, t0, nt)
    if out is None:
        out = np.empty((nt * vs, 4, 3, 3, 2), dtype=np.float64)
    _load().gen_hot(_dims(dims), int(seed), t0, nt, _dp(out))
    return out


def gauge_copy(U: np.ndarray, dims, seed: int) -> np.ndarray:
    """In-place random gauge transform of a whole lattice; returns U."""
    assert U.dtype == np.float64 and U.flags.c_contiguous
    V = int(np.prod(dims))
    assert U.size == V * 72
    _load().gen_gauge_copy(_dims(dims), int(seed), _dp(U))
    return U


def haar_field(dims, seed: int) -> np.ndarray:
    """The Haar h(x) field the smooth/pure-gauge recipes use, shape (V, 3, 3, 2)."""
    V = int(np.prod(dims))
    out = np.empty((V, 3, 3, 2), dtype=np.float64)
    _load().gen_haar_field(_dims(dims), int(seed), 0, V, _dp(out))
    return out


def link_exponential(xi, eps: float) -> np.ndarray:
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    out = np.empty(18, dtype=np.float64)
    _load().gen_link_exponential(_dp(xi), float(eps), _dp(out))
    return out.reshape(3, 3, 2)


def link_xi(seed: int, site: int, mu: int) -> np.ndarray:
    out = np.empty(8, dtype=np.float64)
    _load().gen_link_xi(int(seed), int(site), int(mu), _dp(out))
    return out


def philox4x64_10(ctr, key) -> np.ndarray:
    c = (ctypes.c_uint64 * 4)(*[int(x) for x in ctr])
    k = (ctypes.c_uint64 * 2)(*[int(x) for x in key])
    o = (ctypes.c_uint64 * 4)()
    _load().gen_philox4x64_10(c, k, o)
    return np.array(list(o), dtype=np.uint64)


def to_complex(U: np.ndarray) -> np.ndarray:
    """View (..., 3, 3, 2) float64 as (..., 3, 3) complex128."""
    return U[..., 0] + 1j * U[..., 1]


# ---------------------------------------------------------------- SU(2)
# SU(2) gauge fields for the SU(2) gauge group: links (V, 4, 2, 2, 2)
# float64 in the natural order, each the Cayley-Klein matrix
# [[u0 + i u3, u2 + i u1], [-u2 + i u1, u0 - i u3]] with |u| = 1.  numpy's
# generator keyed by the seed; the recipes mirror the SU(3) ones:
#   su2_hot: Haar-random links (normalised Gaussian 4-vectors);
#   su2_smooth: h(x) exp(i eps xi.sigma) h(x+mu)^dag with xi ~ N(0, 1)^3;
#   su2_pure_gauge: h(x) h(x+mu)^dag.
def _su2_matrices(q: np.ndarray) -> np.ndarray:
    """(..., 4) unit 4-vectors -> (..., 2, 2) complex Cayley-Klein matrices."""
    m = np.empty(q.shape[:-1] + (2, 2), dtype=np.complex128)
    m[..., 0, 0] = q[..., 0] + 1j * q[..., 3]
    m[..., 0, 1] = q[..., 2] + 1j * q[..., 1]
    m[..., 1, 0] = -q[..., 2] + 1j * q[..., 1]
    m[..., 1, 1] = q[..., 0] - 1j * q[..., 3]
    return m


def _su2_real(m: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.stack([m.real, m.imag], axis=-1))


def _su2_haar(rng, shape) -> np.ndarray:
    q = rng.standard_normal(shape + (4,))
    q /= np.linalg.norm(q, axis=-1, keepdims=True)
    return _su2_matrices(q)


def su2_gauge_field(dims, seed: int) -> np.ndarray:
    """A Haar-random gauge transformation h(x), shape (V, 2, 2, 2)."""
    rng = np.random.default_rng([int(seed), 2, 1])
    return _su2_real(_su2_haar(rng, (int(np.prod(dims)),)))


def su2_hot(dims, seed: int) -> np.ndarray:
    rng = np.random.default_rng([int(seed), 2, 0])
    return _su2_real(_su2_haar(rng, (int(np.prod(dims)), 4)))


def su2_smooth(dims, eps: float, seed: int) -> np.ndarray:
    d = tuple(int(x) for x in dims)
    h = to_complex(su2_gauge_field(d, seed)).reshape(d + (2, 2))
    rng = np.random.default_rng([int(seed), 2, 2])
    xi = rng.standard_normal(d + (4, 3))
    n = np.linalg.norm(xi, axis=-1, keepdims=True)
    a = float(eps) * n
    q = np.concatenate([np.cos(a), np.sin(a) * xi / np.where(n > 0, n, 1.0)], axis=-1)
    w = _su2_matrices(q)
    out = np.empty(d + (4, 2, 2), dtype=np.complex128)
    for mu in range(4):
        hf = np.roll(h, -1, axis=mu)
        out[..., mu, :, :] = h @ w[..., mu, :, :] @ np.conj(np.swapaxes(hf, -1, -2))
    return _su2_real(out.reshape((-1, 4, 2, 2)))


def su2_pure_gauge(dims, seed: int) -> np.ndarray:
    return su2_smooth(dims, 0.0, seed)


def su2_gauge_copy(U: np.ndarray, dims, seed: int) -> np.ndarray:
    """A random gauge transform of an SU(2) field (a new array)."""
    d = tuple(int(x) for x in dims)
    h = to_complex(su2_gauge_field(d, seed + 7919)).reshape(d + (2, 2))
    u = to_complex(U).reshape(d + (4, 2, 2))
    out = np.empty_like(u)
    for mu in range(4):
        hf = np.roll(h, -1, axis=mu)
        out[..., mu, :, :] = h @ u[..., mu, :, :] @ np.conj(np.swapaxes(hf, -1, -2))
    return _su2_real(out.reshape((-1, 4, 2, 2)))
