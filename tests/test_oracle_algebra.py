"""Pins of the oracle's site-level algebra against the paper's definitions.

Each check uses an independent route: numpy matrix products of the
Cayley-Klein embedding, brute-force maximisation over SU(2), closed forms of
the local optimum, or the paper's SU(2) formulas.
"""
import numpy as np
import pytest

import oracle as O
from tests._su import ck, embed, random_su2, random_su3, to_c, to_r

SUBS = [(0, 1), (0, 2), (1, 2)]


def _rand_links(rng, n):
    return np.stack([to_r(random_su3(rng)) for _ in range(n)])


@pytest.mark.parametrize("i,j", SUBS)
def test_subgroup_quaternion_projects_embedding(i, j):
    # App. A, Fig. getSubgroupQuaternion: an embedded SU(2) element g gives 2g.
    rng = np.random.default_rng(1)
    for _ in range(20):
        g = random_su2(rng)
        q = O.subgroup_quaternion(to_r(embed(g, i, j)), i, j)
        np.testing.assert_allclose(q, 2 * g, atol=1e-15)


@pytest.mark.parametrize("i,j", SUBS)
def test_retrace_is_conjugate_inner_product(i, j):
    # Re tr[g M] = <g, conj(q(M))> + Re M_kk for the subgroup element g.
    rng = np.random.default_rng(2)
    k = 3 - i - j
    for _ in range(20):
        M = rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3))
        g = random_su2(rng)
        q = O.subgroup_quaternion(to_r(M), i, j)
        lhs = np.trace(embed(g, i, j) @ M).real
        rhs = g[0] * q[0] - g[1] * q[1] - g[2] * q[2] - g[3] * q[3] + M[k, k].real
        assert abs(lhs - rhs) < 1e-13


@pytest.mark.parametrize("i,j", SUBS)
def test_left_and_right_subgroup_mult(i, j):
    # App. A, Fig. subgroupmult; and the backward-link product U g^dag
    rng = np.random.default_rng(3)
    for _ in range(10):
        M = random_su3(rng)
        g = random_su2(rng)
        left = to_c(O.left_subgroup_mult(to_r(M), i, j, g))
        np.testing.assert_allclose(left, embed(g, i, j) @ M, atol=1e-15)
        right = to_c(O.right_subgroup_mult_dag(to_r(M), i, j, g))
        np.testing.assert_allclose(right, M @ embed(g, i, j).conj().T, atol=1e-15)


def test_quaternion_product_is_matrix_product():
    rng = np.random.default_rng(4)
    for _ in range(20):
        a, b = random_su2(rng), random_su2(rng)
        c = O.quat_mul(a, b)
        np.testing.assert_allclose(ck(c), ck(a) @ ck(b), atol=1e-15)


def _angle_axis(q):
    v = np.asarray(q[1:])
    return np.arctan2(np.linalg.norm(v), q[0]), v / np.linalg.norm(v)


def test_or_map_properties():
    # Sec. 2.2.3 / Fig. calculateUpdate: g -> g^omega to first order.
    rng = np.random.default_rng(5)
    for omega in (1.0, 1.35, 1.7, 1.95):
        for _ in range(10):
            a = random_su2(rng)
            g = O.or_map(a, omega)
            assert abs(np.linalg.norm(g) - 1) < 1e-15          # stays in SU(2)
            np.testing.assert_allclose(O.or_map(3.7 * a, omega), g, atol=1e-15)  # scale invariant
            if omega == 1.0:
                np.testing.assert_allclose(g, a, atol=1e-15)    # omega = 1 is relaxation
            phi, ax = _angle_axis(a)
            phi2, ax2 = _angle_axis(g)
            np.testing.assert_allclose(ax2, ax, atol=1e-12)      # same rotation axis
    # first order: the angle is multiplied by omega up to O(phi^3)
    ax = np.array([0.3, -0.5, 0.81])
    ax /= np.linalg.norm(ax)
    for omega in (1.35, 1.7):
        for phi in (1e-1, 1e-2, 1e-3):
            a = np.concatenate([[np.cos(phi)], np.sin(phi) * ax])
            phi2, _ = _angle_axis(O.or_map(a, omega))
            # exact third-order coefficient: omega/3 - (omega - 1) - omega^3/3
            c3 = omega / 3 - (omega - 1) - omega ** 3 / 3
            assert abs(phi2 - omega * phi - c3 * phi ** 3) < 5 * phi ** 5 + 1e-15


def _landau_f(links_f, links_b, g, i, j):
    """Re tr of all adjacent links after applying g at x (links as complex)."""
    G = embed(g, i, j)
    return sum(np.trace(G @ u).real for u in links_f) + sum(np.trace(u @ G.conj().T).real for u in links_b)


def _mag_f(links_f, links_b, g, i, j):
    G = embed(g, i, j)
    return (sum(np.sum(np.abs(np.diag(G @ u)) ** 2) for u in links_f) +
            sum(np.sum(np.abs(np.diag(u @ G.conj().T)) ** 2) for u in links_b))


@pytest.mark.parametrize("i,j", SUBS)
def test_landau_relaxation_is_local_maximum(i, j):
    # Sec. 2.2.1: g maximises Re tr[g K]; maximum = |q| + Re K_kk (closed form)
    rng = np.random.default_rng(6)
    for trial in range(3):
        fwd, bwd = _rand_links(rng, 4), _rand_links(rng, 4)
        Fc, Bc = to_c(fwd), to_c(bwd)
        g = O.local_g(fwd, bwd, "landau", "or", i, j, omega=1.0)
        f_best = _landau_f(Fc, Bc, g, i, j)
        K = sum(Fc) + sum(u.conj().T for u in Bc)
        q = O.subgroup_quaternion(to_r(K), i, j)
        k = 3 - i - j
        assert abs(f_best - (np.linalg.norm(q) + K[k, k].real)) < 1e-12
        samples = random_su2(rng, 20000)
        # f is linear in g: f(g) = <g, conj q> + const
        const = _landau_f(Fc, Bc, np.array([1.0, 0, 0, 0]), i, j) - q[0]
        vals = samples @ (q * np.array([1, -1, -1, -1])) + const
        assert vals.max() <= f_best + 1e-12
        for s in samples[:50]:
            assert _landau_f(Fc, Bc, s, i, j) <= f_best + 1e-12


def test_landau_su2_closed_form():
    # eq. localsolution: for SU(2), g = K^dag / sqrt(det K^dag)
    rng = np.random.default_rng(7)
    for _ in range(10):
        fwd = np.stack([to_r(embed(random_su2(rng), 0, 1)) for _ in range(4)])
        bwd = np.stack([to_r(embed(random_su2(rng), 0, 1)) for _ in range(4)])
        K = (sum(to_c(fwd)) + sum(u.conj().T for u in to_c(bwd)))[:2, :2]
        expect = K.conj().T / np.sqrt(np.linalg.det(K.conj().T))
        g = O.local_g(fwd, bwd, "landau", "or", 0, 1, omega=1.0)
        np.testing.assert_allclose(ck(g), expect, atol=1e-13)


@pytest.mark.parametrize("i,j", SUBS)
def test_mag_relaxation_is_local_maximum(i, j):
    # Sec. 2.2.2: the top eigenvector maximises the local MAG functional,
    # and the maximal gain over g = 1 is lambda - D.
    rng = np.random.default_rng(8)
    for trial in range(3):
        fwd, bwd = _rand_links(rng, 4), _rand_links(rng, 4)
        Fc, Bc = to_c(fwd), to_c(bwd)
        g = O.local_g(fwd, bwd, "mag", "or", i, j, omega=1.0)
        assert abs(g[3]) < 1e-15
        f_best = _mag_f(Fc, Bc, g, i, j)
        D, E, F = O.mag_coefficients(fwd, bwd, i, j)
        lam = np.sqrt(D * D + E * E + F * F)
        f_one = _mag_f(Fc, Bc, np.array([1.0, 0, 0, 0]), i, j)
        assert abs((f_best - f_one) - (lam - D)) < 1e-12
        for s in random_su2(rng, 3000):
            assert _mag_f(Fc, Bc, s, i, j) <= f_best + 1e-12


def test_mag_su2_matches_paper_formulas():
    # Sec. 2.2.2 with SU(2) links: E and F as printed, D twice the printed value
    # (the value that makes eq. upMatrix agree with eq. up).
    rng = np.random.default_rng(9)
    for _ in range(10):
        uf = random_su2(rng, 4)
        ub = random_su2(rng, 4)
        fwd = np.stack([to_r(embed(u, 0, 1)) for u in uf])
        bwd = np.stack([to_r(embed(u, 0, 1)) for u in ub])
        D, E, F = O.mag_coefficients(fwd, bwd, 0, 1)
        # backward link enters through U^dag: Cayley-Klein of U^dag is (u0,-u1,-u2,-u3)
        allu = np.concatenate([uf, ub * np.array([1, -1, -1, -1])])
        Dp = np.sum(allu[:, 0] ** 2 + allu[:, 3] ** 2 - 0.5)
        Ep = 2 * np.sum(-allu[:, 0] * allu[:, 1] - allu[:, 2] * allu[:, 3])
        Fp = 2 * np.sum(-allu[:, 0] * allu[:, 2] + allu[:, 1] * allu[:, 3])
        np.testing.assert_allclose([D, E, F], [2 * Dp, Ep, Fp], atol=1e-13)
        # eq. upMatrix eigenvector with the corrected D
        M = np.array([[D, E, F], [E, -D, 0], [F, 0, -D]])
        w, v = np.linalg.eigh(M)
        top = v[:, -1] * np.sign(v[0, -1])
        g = O.local_g(fwd, bwd, "mag", "or", 0, 1, omega=1.0)
        np.testing.assert_allclose(g[:3] * np.sign(g[0]), top, atol=1e-12)


@pytest.mark.parametrize("gauge", ["landau", "mag"])
@pytest.mark.parametrize("i,j", SUBS)
def test_microcanonical_keeps_local_functional(gauge, i, j):
    # Sec. 2.2.4: the microcanonical step leaves the local functional invariant
    rng = np.random.default_rng(10)
    f = _landau_f if gauge == "landau" else _mag_f
    for _ in range(10):
        fwd, bwd = _rand_links(rng, 4), _rand_links(rng, 4)
        Fc, Bc = to_c(fwd), to_c(bwd)
        g = O.local_g(fwd, bwd, gauge, "micro", i, j)
        h = O.local_g(fwd, bwd, gauge, "or", i, j, omega=1.0)
        np.testing.assert_allclose(g, O.quat_mul(h, h), atol=1e-15)
        before = f(Fc, Bc, np.array([1.0, 0, 0, 0]), i, j)
        assert abs(f(Fc, Bc, g, i, j) - before) < 1e-12


def test_or_interpolates_between_relaxation_and_micro():
    # Sec. 2.2.3/2.2.4: omega = 1 is relaxation; the local functional after an
    # OR step lies between the relaxed maximum and the microcanonical value.
    rng = np.random.default_rng(11)
    for _ in range(10):
        fwd, bwd = _rand_links(rng, 4), _rand_links(rng, 4)
        Fc, Bc = to_c(fwd), to_c(bwd)
        f1 = _landau_f(Fc, Bc, np.array([1.0, 0, 0, 0]), 0, 1)
        fr = _landau_f(Fc, Bc, O.local_g(fwd, bwd, "landau", "or", 0, 1, omega=1.0), 0, 1)
        fo = _landau_f(Fc, Bc, O.local_g(fwd, bwd, "landau", "or", 0, 1, omega=1.7), 0, 1)
        assert f1 - 1e-12 <= fo <= fr + 1e-12
