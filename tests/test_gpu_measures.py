"""GPU parity of the measurements and the reprojection (Sec. 2.1.1, 2.1.2,
Sec. 4.5) against the oracle, value by value.

* F and theta of the MAG and Coulomb gauges (theta_t per time-slice) after
  every sweep of an FP64 run, to the bound of the C1 trajectory:
  |F_gpu - F_oracle| <= 1e-10 F and |theta_gpu - theta_oracle| <=
  1e-10 theta + 1e-13 sqrt(theta).  The second term of the theta bound is the
  rounding floor: theta sums squares of Delta, a difference of O(8) numbers
  that each carry an absolute error of about 1e-15, so theta cannot agree
  relatively below theta ~ 1e-6.
* gf_reunitarise on links pushed off SU(3) against the oracle's
  reprojection.  Row 0 is the input row times 1/|row|, row 1 the projected
  and normalised second row: each entry has a relative error of a few ulp on
  either side (different operation order, fused multiply-adds on the GPU),
  so |error| <= 8 ulp(1) = 9e-16 for rows 0 and 1.  Row 2 is (u x v)^*, two
  products of such entries per component: twice their error, 2e-15.
* gf_unitarity (mean and max of |1 - det U|) against the oracle's on the
  same links: relative 1e-12 (the determinant differs by rounding, ~1e-16,
  against defects of ~1e-4).
* Whole runs with reprojection every 7 sweeps against the oracle's run with
  the same interval (reading 14: stopped Coulomb time-slices are left
  alone): identical sweep counts, links within 1e-9, and the spatial links
  of a time-slice that stops at the first check bit-identical to the input.
"""
import numpy as np
import pytest

import oracle as O
from paper_1212_5221_amd import inputs as I
from tests.test_gpu_parity import fixer, say

pytestmark = pytest.mark.gpu


def _theta_bound(th):
    return 1e-10 * th + 1e-13 * np.sqrt(th) + 1e-18


def _perturbed(dims, seed, amp):
    U = I.smooth(dims, 0.5, seed)
    rng = np.random.default_rng(seed)
    return U + amp * rng.standard_normal(U.shape)


@pytest.mark.parametrize("storage", ["f64r18", "f64r12"])
@pytest.mark.parametrize("gauge", ["landau", "coulomb"])
def test_reunitarise_matches_oracle(gauge, storage):
    dims = (4, 6, 4, 6)
    say("reunitarise", gauge, storage)
    # 12-real storage keeps rows 0 and 1, from which both sides reproject
    U = _perturbed(dims, 8101, 1e-3)
    fx = fixer([dims], gauge, storage)
    fx.upload(0, U)
    fx.reunitarise()
    out = fx.download(0)
    fx.close()
    ref = U.copy()
    O.reunitarise(ref)
    e01 = float(np.max(np.abs(out[..., 0:2, :, :] - ref[..., 0:2, :, :])))
    e2 = float(np.max(np.abs(out[..., 2, :, :] - ref[..., 2, :, :])))
    say("max |gpu - oracle| rows 0-1", e01, "row 2", e2)
    assert e01 <= 9e-16 and e2 <= 2e-15
    assert O.unitarity(out)[1] < 1e-14


@pytest.mark.parametrize("storage", ["f64r18", "f64r12", "mixed"])
def test_unitarity_matches_oracle(storage):
    dims = (4, 4, 6, 4)
    say("unitarity", storage)
    U = _perturbed(dims, 8102, 1e-4)
    fx = fixer([dims], "landau", storage)
    fx.upload(0, U)
    mean, mx = fx.unitarity(0)
    # what the storage holds: 12-real storages rebuild row 2 from rows 0, 1
    held = fx.download(0)
    fx.close()
    mo, xo = O.unitarity(held)
    say("gpu", mean, mx, "oracle", mo, xo)
    assert abs(mean - mo) <= 1e-12 * mo and abs(mx - xo) <= 1e-12 * xo
    if storage == "f64r18":
        mi, xi = O.unitarity(U)
        assert abs(mean - mi) <= 1e-12 * mi and abs(mx - xi) <= 1e-12 * xi


@pytest.mark.parametrize("storage", ["f64r18", "f64r12"])
def test_mag_trajectory(storage):
    # 8^4, eps 0.3, seed 1001: F_MAG and theta_MAG after every sweep
    dims = (8, 8, 8, 8)
    nsw = 150
    say("MAG trajectory", storage)
    U = I.smooth(dims, 0.3, 1001)
    r = O.run(U.copy(), dims, "mag", "or", omega=1.7, max_sweeps=nsw, tol=0.0, check_every=1)
    assert len(r.F) == nsw + 1
    fx = fixer([dims], "mag", storage)
    fx.upload(0, U)
    fx.set_overrelax(1.7)
    F, th = [], []
    for k in range(nsw + 1):
        f, t = fx.measure(0)
        F.append(f)
        th.append(t)
        if k < nsw:
            fx.sweep("or", max_sweeps=1, tol=0.0, check_every=1)
    fx.close()
    F, th = np.array(F), np.array(th)
    relF = np.max(np.abs(F - r.F) / np.abs(r.F))
    ratio = np.max(np.abs(th - r.theta) / _theta_bound(r.theta))
    say("theta from", r.theta[0], "to", r.theta[-1], "max rel dF", relF, "max dtheta/bound", ratio)
    assert relF < 1e-10 and ratio <= 1.0


@pytest.mark.parametrize("storage", ["f64r18", "f64r12"])
def test_coulomb_per_slice_trajectory(storage):
    # 8^4, eps 0.3, seed 1001: F_t and theta_t of every time-slice after every
    # sweep, until every slice is below 1e-13
    dims = (8, 8, 8, 8)
    say("Coulomb trajectory", storage)
    U = I.smooth(dims, 0.3, 1001)
    ref = U.copy()
    V = int(np.prod(dims))
    G = O.identity_field(V)
    fx = fixer([dims], "coulomb", storage)
    fx.upload(0, U)
    fx.set_overrelax(1.7)
    worst_F, worst_th, k = 0.0, 0.0, 0
    while True:
        Ft, tht = fx.measure_timeslices(0)
        Fo, tho = O.measure_slices(ref, dims)
        worst_F = max(worst_F, float(np.max(np.abs(Ft - Fo) / np.abs(Fo))))
        worst_th = max(worst_th, float(np.max(np.abs(tht - tho) / _theta_bound(tho))))
        if np.all(tho < 1e-13) or k >= 600:
            break
        fx.sweep("or", max_sweeps=1, tol=0.0, check_every=1)
        O.sweep(ref, dims, "coulomb", "or", omega=1.7, G=G)
        k += 1
    fx.close()
    say("sweeps", k, "max rel dF_t", worst_F, "max dtheta_t/bound", worst_th)
    assert k < 600
    assert worst_F < 1e-10 and worst_th <= 1.0


@pytest.mark.parametrize("storage", ["f64r18", "f64r12"])
@pytest.mark.parametrize("gauge", ["landau", "coulomb", "mag"])
def test_run_with_reprojection_matches_oracle(gauge, storage):
    dims = (4, 6, 4, 6)
    vs = 6 * 4 * 6
    say("run with reprojection every 7 sweeps", gauge, storage)
    U = I.smooth(dims, 0.5, 8103)
    if gauge == "coulomb":
        # time-slice 1 of constant spatial links: fixed already (theta_t = 0),
        # it stops at the first check and must keep its links exactly
        C = I.hot((2, 2, 2, 2), 17)[0]
        U[vs:2 * vs, 1:4] = C[1:4]
    ref = U.copy()
    r = O.run(ref, dims, gauge, "or", omega=1.7, max_sweeps=4000, tol=1e-12, check_every=5, reunit_every=7)
    fx = fixer([dims], gauge, storage, reunit_every=7)
    fx.upload(0, U)
    fx.set_overrelax(1.7)
    st, done = fx.sweep("or", max_sweeps=4000, tol=1e-12, check_every=5)
    out = fx.download(0)
    fx.close()
    say("oracle sweeps", r.sweeps_done.tolist(), "gpu", done.tolist())
    assert st == 0 and r.status == 0
    np.testing.assert_array_equal(done, r.sweeps_done.astype(np.int32))
    assert np.max(np.abs(out - ref)) < 1e-9
    if gauge == "coulomb":
        assert done[1] == 0
        rows = 3 if storage == "f64r18" else 2  # 12-real storage rebuilds row 2
        np.testing.assert_array_equal(out[vs:2 * vs, 1:4, :rows], U[vs:2 * vs, 1:4, :rows])
