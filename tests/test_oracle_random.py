"""Pins of the oracle's random streams and heatbath samplers (Sec. 2.3).

Philox4x64-10 against numpy's implementation of the same published
generator; the samplers against their target distributions (numerically
integrated CDFs) by Kolmogorov-Smirnov tests.
"""
import numpy as np
import pytest
from scipy import integrate, stats

import oracle as O
from tests._su import random_su3, to_r


def _numpy_philox(ctr, key):
    # numpy advances the 256-bit counter by one before producing a block
    c = list(ctr)
    carry = 1
    for k in range(4):
        if carry == 0:
            break
        c[k] = (c[k] - 1) % 2 ** 64
        carry = 1 if c[k] == 2 ** 64 - 1 else 0
    g = np.random.Philox(counter=np.array(c, dtype=np.uint64), key=np.array(list(key), dtype=np.uint64))
    return g.random_raw(4)


@pytest.mark.parametrize("ctr,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (0, 0)),
    ((2 ** 64 - 1, 5, 7, 2 ** 63), (123456789, 987654321)),
    ((0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0, 0x082EFA98EC4E6C89),
     (0x452821E638D01377, 0xBE5466CF34E90C6C)),
])
def test_philox_matches_numpy(ctr, key):
    np.testing.assert_array_equal(O.philox4x64_10(ctr, key), _numpy_philox(ctr, key))


def test_philox_random_counters():
    rng = np.random.default_rng(0)
    for _ in range(50):
        ctr = [int(x) for x in rng.integers(0, 2 ** 63, size=4)]
        key = [int(x) for x in rng.integers(0, 2 ** 63, size=2)]
        np.testing.assert_array_equal(O.philox4x64_10(ctr, key), _numpy_philox(ctr, key))


@pytest.mark.parametrize("kappa", [0.0, 1e-9, 0.3, 2.0, 40.0, 800.0])
def test_exp_inverse_cdf(kappa):
    # CDF of exp(kappa w) on [-1, 1] evaluated at the sample equals u
    for u in (1e-12, 0.01, 0.3, 0.5, 0.77, 0.999999):
        w = O.exp_inverse_cdf(kappa, u)
        assert -1 <= w <= 1
        if kappa == 0:
            assert abs(w - (2 * u - 1)) < 1e-15
            continue
        if kappa < 1:
            cdf = np.expm1(kappa * (w + 1)) / np.expm1(2 * kappa)
        else:
            cdf = (np.exp(kappa * (w - 1)) - np.exp(-2 * kappa)) / -np.expm1(-2 * kappa)
        assert abs(cdf - u) < 1e-9


def _r0_cdf(a):
    xs = np.linspace(-1, 1, 4001)
    f = np.sqrt(1 - xs ** 2) * np.exp(a * (xs - 1))
    c = integrate.cumulative_trapezoid(f, xs, initial=0)
    c /= c[-1]
    return lambda x: np.interp(x, xs, c)


@pytest.mark.parametrize("a", [0.05, 1.0, 1.99, 2.0, 6.0, 30.0])
def test_r0_sampler_distribution(a):
    n = 4000
    r0 = np.array([O.sample_r0(a, (77, 3), 5, s, 1)[0] for s in range(n)])
    res = stats.kstest(r0, _r0_cdf(a))
    assert res.pvalue > 1e-3


def test_landau_heatbath_distribution():
    # g = r h: r0 = <g, h> follows sqrt(1-r0^2) exp(|q| r0 / T); the vector part
    # of r is isotropic.
    rng = np.random.default_rng(3)
    fwd = np.stack([to_r(random_su3(rng)) for _ in range(4)])
    bwd = np.stack([to_r(random_su3(rng)) for _ in range(4)])
    h = O.local_g(fwd, bwd, "landau", "or", 0, 1, omega=1.0)
    q = O.subgroup_quaternion(to_r(sum(fwd[..., 0] + 1j * fwd[..., 1]) +
                                    sum((b[..., 0] + 1j * b[..., 1]).conj().T for b in bwd)), 0, 1)
    T = 1.3
    a = np.linalg.norm(q) / T
    r0s, cz = [], []
    hinv = h * np.array([1, -1, -1, -1])
    for s in range(3000):
        g = O.local_g(fwd, bwd, "landau", "heatbath", 0, 1, T=T, seed=11, site=s)
        r = O.quat_mul(g, hinv)
        r0s.append(r[0])
        cz.append(r[3] / np.linalg.norm(r[1:]))
    assert stats.kstest(r0s, _r0_cdf(a)).pvalue > 1e-3
    assert stats.kstest(cz, stats.uniform(loc=-1, scale=2).cdf).pvalue > 1e-3


@pytest.mark.parametrize("T", [0.2, 1.5, 8.0])
def test_mag_heatbath_distribution(T):
    # n(g) follows von Mises-Fisher exp(kappa n.yhat) on S^2 with kappa = lambda/T
    rng = np.random.default_rng(4)
    fwd = np.stack([to_r(random_su3(rng)) for _ in range(4)])
    bwd = np.stack([to_r(random_su3(rng)) for _ in range(4)])
    D, E, F = O.mag_coefficients(fwd, bwd, 0, 2)
    y = np.array([F, -E, D])
    lam = np.linalg.norm(y)
    yh = y / lam
    kappa = lam / T
    ws, phis = [], []
    for s in range(3000):
        g = O.local_g(fwd, bwd, "mag", "heatbath", 0, 2, T=T, seed=12, site=s, subgroup=1)
        assert abs(g[3]) < 1e-15 and abs(np.linalg.norm(g) - 1) < 1e-14
        g0, g1, g2 = g[:3]
        n = np.array([2 * g0 * g2, -2 * g0 * g1, g0 ** 2 - g1 ** 2 - g2 ** 2])
        ws.append(n @ yh)
    cdf = lambda w: (np.exp(kappa * (np.asarray(w) - 1)) - np.exp(-2 * kappa)) / -np.expm1(-2 * kappa)
    assert stats.kstest(ws, cdf).pvalue > 1e-3
