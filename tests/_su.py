"""Small numpy helpers for the tests: matrices written out from the paper's
definitions, independent of both the oracle and the GPU library."""
import numpy as np


def ck(g):
    """Cayley-Klein 2x2 matrix of a quaternion (g0, g1, g2, g3) (Sec. 2.2.2)."""
    g0, g1, g2, g3 = g
    return np.array([[g0 + 1j * g3, g2 + 1j * g1], [-g2 + 1j * g1, g0 - 1j * g3]])


def embed(g, i, j):
    """SU(2) element acting on rows/columns (i, j) of an SU(3) matrix."""
    m = np.eye(3, dtype=complex)
    c = ck(g)
    m[i, i], m[i, j], m[j, i], m[j, j] = c[0, 0], c[0, 1], c[1, 0], c[1, 1]
    return m


def to_c(M):
    M = np.asarray(M)
    return M[..., 0] + 1j * M[..., 1]


def to_r(C):
    C = np.asarray(C)
    return np.ascontiguousarray(np.stack([C.real, C.imag], axis=-1))


def random_su2(rng, n=None):
    v = rng.normal(size=(4,) if n is None else (n, 4))
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def random_su3(rng):
    z = (rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    q = q @ np.diag(np.diag(r) / np.abs(np.diag(r)))
    q = q / np.linalg.det(q) ** (1.0 / 3.0)
    return q


GELL_MANN = np.zeros((8, 3, 3), dtype=complex)
GELL_MANN[0][0, 1] = GELL_MANN[0][1, 0] = 1
GELL_MANN[1][0, 1], GELL_MANN[1][1, 0] = -1j, 1j
GELL_MANN[2][0, 0], GELL_MANN[2][1, 1] = 1, -1
GELL_MANN[3][0, 2] = GELL_MANN[3][2, 0] = 1
GELL_MANN[4][0, 2], GELL_MANN[4][2, 0] = -1j, 1j
GELL_MANN[5][1, 2] = GELL_MANN[5][2, 1] = 1
GELL_MANN[6][1, 2], GELL_MANN[6][2, 1] = -1j, 1j
GELL_MANN[7] = np.diag([1, 1, -2]) / np.sqrt(3)


def site_index(dims, t, x, y, z):
    return ((t * dims[1] + x) * dims[2] + y) * dims[3] + z


def coords(dims, s):
    z = s % dims[3]
    s //= dims[3]
    y = s % dims[2]
    s //= dims[2]
    x = s % dims[1]
    t = s // dims[1]
    return t, x, y, z


def unit_links(dims):
    V = int(np.prod(dims))
    U = np.zeros((V, 4, 3, 3, 2))
    for i in range(3):
        U[:, :, i, i, 0] = 1.0
    return U
