"""Coulomb gauge at full size: 64^3 x 256 (256 independent time-slices of 64^3,
about 13 GB of FP32 12-real links) fixed in one batched launch with
per-time-slice stopping, mixed storage, omega = 1.7, theta < 1e-12.

Checked on sampled time-slices {0, 85, 170, 255}: one half-sweep recomputed
site by site by the oracle from the same FP32-rounded input slice (the
update of a time-slice depends on that slice only), and after the full fix
the oracle's per-slice F_t and theta_t of the downloaded slice, after a
bounded chunk of 2000 sweeps of all slices.  The complete fix (every
time-slice below 1e-12, about 150k sweeps and 9 minutes) runs only with
GF_LONG_TESTS=1.
"""
import os

import numpy as np
import pytest

import oracle as O
from paper_1212_5221_amd import inputs as I
from tests.test_gpu_parity import f32_round, fixer, say

pytestmark = pytest.mark.gpu

DIMS = (256, 64, 64, 64)
SLICES = (0, 85, 170, 255)
SLAB = 16


def _device_input():
    """the natural-order FP64 input (38.7 GB) generated slab by slab into HBM"""
    import torch
    Vs = DIMS[1] * DIMS[2] * DIMS[3]
    buf = torch.empty(DIMS[0] * Vs * 72, dtype=torch.float64, device="cuda:0")
    for t0 in range(0, DIMS[0], SLAB):
        slab = I.smooth(DIMS, 0.5, 3001, t0=t0, nt=SLAB).reshape(-1)
        buf[t0 * Vs * 72:(t0 + SLAB) * Vs * 72].copy_(torch.from_numpy(slab))
        say("  generated time-slices", t0, "to", t0 + SLAB - 1)
    return buf


def _upload(fx, buf):
    fx.upload(0, buf)  # device-resident input: conversion only


@pytest.fixture(scope="module")
def c3():
    say("C3: generating and uploading 64^3 x 256 in slabs of", SLAB)
    fx = fixer([DIMS], "coulomb", "mixed", reunit_every=100, tail_theta=1e-9)
    buf = _device_input()
    _upload(fx, buf)
    fx.set_overrelax(1.7)
    fx.autotune(reps=1)
    yield fx, buf
    fx.close()


def test_c3_halfsweep_sampled_sites(c3):
    fx, buf = c3
    _upload(fx, buf)  # autotuning ran real sweeps: start again from the input
    say("C3: one half-sweep, sampled sites")
    fx.halfsweep("or", 0)
    d1 = (1,) + DIMS[1:]
    Vs = DIMS[1] * DIMS[2] * DIMS[3]
    rng = np.random.default_rng(7)
    from tests._su import coords, site_index
    for t in SLICES:
        got = fx.download(0, t0=t, nt=1)
        ref = f32_round(I.smooth(DIMS, 0.5, 3001, t0=t, nt=1))
        sites = []
        while len(sites) < 64:
            s = int(rng.integers(0, Vs))
            if sum(coords(d1, s)[1:]) % 2 == 0:
                sites.append(s)
        O.update_sites(ref, d1, "coulomb", "or", sites, omega=1.7, G=O.identity_field(Vs))
        err = 0.0
        for s in sites:
            _, x, y, z = coords(d1, s)
            for mu, c in ((1, (0, x, y, z)), (2, (0, x, y, z)), (3, (0, x, y, z))):
                err = max(err, float(np.max(np.abs(got[s, mu] - ref[s, mu]))))
                b = list(c)
                b[mu] = (b[mu] - 1) % d1[mu]
                q = site_index(d1, *b)
                err = max(err, float(np.max(np.abs(got[q, mu] - ref[q, mu]))))
        say("slice", t, "max |gpu - oracle|", err)
        assert err < 3e-5


def test_c3_chunk_measures_match_oracle(c3):
    # One bounded chunk of the full workload: 2000 sweeps of all 256
    # time-slices in one batched launch with per-slice stopping (checks every
    # 10 sweeps), then F_t and theta_t of the sampled slices measured by the
    # GPU against the oracle's measurement of the downloaded slices
    # (theta_t to the bound of the C1 trajectory), and every slice that
    # stopped below the tolerance.
    fx, buf = c3
    _upload(fx, buf)
    _, th_in = fx.measure_timeslices(0)
    say("C3: a chunk of 2000 sweeps; input theta_t max", float(th_in.max()))
    st, done = fx.sweep("or", max_sweeps=2000, tol=1e-12, check_every=10)
    Ft, tht = fx.measure_timeslices(0)
    stopped = done < 2000
    say("status", st, "slices stopped", int(stopped.sum()), "theta_t min/median/max", float(tht.min()),
        float(np.median(tht)), float(tht.max()))
    assert np.all(tht[stopped] < 1e-12)
    assert np.all(tht < 1e-2 * th_in)  # every slice well on its way
    d1 = (1,) + DIMS[1:]
    for t in SLICES:
        got = fx.download(0, t0=t, nt=1)
        Fo, tho = O.measure_slices(got, d1)
        bound = 1e-10 * tho[0] + 1e-13 * np.sqrt(tho[0]) + 1e-18
        say("slice", t, "sweeps", int(done[t]), "F gpu", Ft[t], "oracle", Fo[0], "theta gpu", tht[t], "oracle",
            tho[0])
        assert abs(Fo[0] - Ft[t]) <= 1e-12 * Fo[0]
        assert abs(tho[0] - tht[t]) <= bound


@pytest.mark.skipif(os.environ.get("GF_LONG_TESTS") != "1",
                    reason="the complete 64^3 x 256 fix runs about 150k sweeps (about 9 minutes); "
                           "set GF_LONG_TESTS=1")
def test_c3_full_fix(c3):
    # The time-slices converge at very different rates (the slowest gauge
    # modes of a 64^3 slice decay by about 1 - c omega lambda_min per sweep,
    # and lambda_min varies between slices): most stop between 30k and 100k
    # sweeps, the last few need up to about 150k (one run: 31,080 to 150,020
    # sweeps, quartiles 45.8k / 56.2k / 68.8k).  Once most slices have
    # stopped a sweep costs well under a millisecond, so the test runs until
    # every slice has stopped, within 300k sweeps, in calls of 10k sweeps
    # (checks every 20; a converged time-slice stops at the first check of
    # the next call, and each call ends with the U_0 fix-up, so the calls
    # continue one run).
    fx, buf = c3
    say("C3: full fix")
    _upload(fx, buf)
    done = np.zeros(DIMS[0], dtype=np.int64)
    st = 1
    for chunk in range(30):
        st, d = fx.sweep("or", max_sweeps=10000, tol=1e-12, check_every=20)
        done += d
        running = d == 10000
        _, th = fx.measure_timeslices(0)
        say("  after", int(done.max()), "sweeps: status", st, "slices still running", int(np.sum(running)),
            "their theta max", float(th[running].max()) if running.any() else 0.0)
        if st == 0:
            break
    Ft, tht = fx.measure_timeslices(0)
    say("status", st, "sweeps min/max", done.min(), done.max(), "quartiles", np.percentile(done, [25, 50, 75]),
        "theta_t max", tht.max())
    assert st == 0  # every time-slice stopped
    assert np.all(tht < 1e-12)
    assert len(set(done.tolist())) > 1  # time-slices stop on their own
    d1 = (1,) + DIMS[1:]
    for t in SLICES:
        got = fx.download(0, t0=t, nt=1)
        Fo, tho = O.measure_slices(got, d1)
        say("slice", t, "sweeps", done[t], "F gpu", Ft[t], "oracle", Fo[0], "theta", tho[0])
        assert abs(Fo[0] - Ft[t]) < 1e-9 and abs(tho[0] - tht[t]) < 1e-9 * max(tht[t], 1e-3)
