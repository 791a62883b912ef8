"""Simulated annealing (Sec. 2.3) on the GPU against the oracle.

FP64 storage: the GPU and the oracle draw the same Philox4x64-10 numbers
(keyed by seed and instance, counter by sweep index, site, subgroup, draw).
The annealing dynamics amplify any difference by about 1e3 per annealing
step (one heatbath and three microcanonical sweeps; the oracle against a
1e-15-perturbed copy of itself shows the same growth, see
tests/test_oracle_iteration.py), so GPU and oracle chains are compared over
one annealing step, where rounding differences stay below 1e-8, and longer
chains by invariants and convergence.
Mixed storage cannot follow the FP64 chain (FP32 rounding changes the
samples), so its heatbath and stochastic-relaxation half-sweeps are each
recomputed by the oracle from the state the GPU stored before them, and at
full size (32^4 MAG, the annealing workload) the chain is checked by
properties and by one overrelaxation half-sweep recomputed by the oracle on
sampled sites of the annealed state.
"""
import numpy as np
import pytest

import oracle as O
from paper_1212_5221_amd import inputs as I
from tests.test_gpu_parity import f_orbit_tol, fixer, launch_shapes, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("gauge", ["mag", "landau", "coulomb"])
@pytest.mark.parametrize("storage", ["f64r18", "f64r12"])
def test_anneal_matches_oracle(gauge, storage):
    dims = (4, 4, 6, 4)
    say("anneal", gauge, storage)
    U = I.smooth(dims, 0.7, 4001)
    ref = U.copy()
    V = int(np.prod(dims))
    G = O.identity_field(V) if gauge == "coulomb" else None
    ctr = O.anneal(ref, dims, gauge, 1.5, 1.5, 1, nmicro=3, seed=4002, instance=0, sweep_counter=0, G=G)
    if gauge == "coulomb":
        O.coulomb_fix_u0(ref, dims, G)
    fx = fixer([dims], gauge, storage)
    fx.upload(0, U)
    fx.set_anneal(1.5, 1.5, 1, nmicro=3, seed=4002)
    st, done = fx.sweep("anneal")
    assert fx.get_sweep_index(0) == ctr == 4
    out = fx.download(0)
    err = np.max(np.abs(out - ref))
    say("max |gpu - oracle| after one annealing step", err)
    assert err < 1e-8
    # then overrelaxation to theta < 1e-12 on both sides
    r = O.run(ref, dims, gauge, "or", omega=1.7, max_sweeps=3000, tol=1e-12, check_every=5, sweep_counter=ctr)
    fx.set_overrelax(1.7)
    st, done = fx.sweep("or", max_sweeps=3000, tol=1e-12, check_every=5)
    out = fx.download(0)
    fx.close()
    assert st == 0 and r.status == 0
    np.testing.assert_array_equal(done, r.sweeps_done.astype(np.int32))
    assert np.max(np.abs(out - ref)) < 1e-7


@pytest.mark.parametrize("storage", ["f64r18", "f64r12", "mixed"])
@pytest.mark.parametrize("gauge", ["mag", "landau"])
def test_long_anneal_keeps_invariants_and_converges(gauge, storage):
    # 800 annealing sweeps with no periodic reprojection: the links must stay
    # on SU(3) (12-real storage rebuilds the third row, which would let a norm
    # defect grow exponentially under these large updates) and keep their
    # gauge invariants; then overrelaxation converges
    dims = (4, 4, 6, 4)
    say("long anneal", gauge, storage)
    U = I.smooth(dims, 0.7, 4004)
    before = [O.wilson_loop(U, dims, r, t) for r, t in ((1, 1), (1, 2))]
    fx = fixer([dims], gauge, storage, reunit_every=0)
    fx.upload(0, U)
    fx.set_anneal(1.5, 0.01, 200, nmicro=3, seed=4005)
    fx.sweep("anneal")
    assert fx.get_sweep_index(0) == 800
    umean, umax = fx.unitarity()
    say("unitarity after annealing: mean", umean, "max", umax)
    f64 = storage != "mixed"
    # FP64: rounding drift of at most 1e-15 per sweep (as for the oracle)
    assert umax < (1e-15 * 800 if f64 else 2e-6)
    fx.set_overrelax(1.7)
    st, done = fx.sweep("or", max_sweeps=5000, tol=1e-12, check_every=5)
    F, th = fx.measure(0)
    out = fx.download(0)
    fx.close()
    assert st == 0
    tol_inv = 1e-13 if f64 else 2e-6
    np.testing.assert_allclose([O.wilson_loop(out, dims, r, t) for r, t in ((1, 1), (1, 2))], before, atol=tol_inv)
    Fo, tho = O.measure(out, dims, gauge)
    if f64:
        assert abs(Fo - F) < 1e-12 and tho < 1e-12
    else:
        # the download rebuilds row 2 in FP64 from the FP32 rows, as the kernels do
        assert abs(Fo - F) < 1e-9 and tho < 1e-11


@pytest.mark.parametrize("gauge", ["mag", "landau"])
def test_cooling_pipeline_matches_oracle(gauge):
    # annealing (one step, see above), then stochastic relaxation (p = 0.5,
    # same Philox streams; unlike annealing its dynamics contract, so the two
    # chains stay within rounding), then overrelaxation to theta < 1e-12
    dims = (4, 4, 6, 4)
    say("cooling pipeline", gauge)
    U = I.smooth(dims, 0.7, 4001)
    ref = U.copy()
    ctr = O.anneal(ref, dims, gauge, 1.5, 1.5, 1, nmicro=3, seed=4002)
    r1 = O.run(ref, dims, gauge, "sr", max_sweeps=300, tol=0.0, check_every=300, p_sr=0.5, seed=4003,
               sweep_counter=ctr)
    r2 = O.run(ref, dims, gauge, "or", omega=1.7, max_sweeps=3000, tol=1e-12, check_every=5,
               sweep_counter=r1.sweep_counter)
    fx = fixer([dims], gauge, "f64r18")
    fx.upload(0, U)
    fx.set_anneal(1.5, 1.5, 1, nmicro=3, seed=4002)
    fx.sweep("anneal")
    fx.set_seed(4003)
    fx.set_stochastic(0.5)
    fx.sweep("sr", max_sweeps=300, tol=0.0, check_every=300)
    assert fx.get_sweep_index(0) == r1.sweep_counter
    mid = fx.download(0)
    fx.set_overrelax(1.7)
    st, done = fx.sweep("or", max_sweeps=3000, tol=1e-12, check_every=5)
    out = fx.download(0)
    fx.close()
    say("SR stage: theta", O.measure(mid, dims, gauge)[1], "OR sweeps gpu", done.tolist(),
        "oracle", r2.sweeps_done.tolist(), "max |gpu - oracle|", np.max(np.abs(out - ref)))
    assert st == 0 and r2.status == 0
    np.testing.assert_array_equal(done, r2.sweeps_done.astype(np.int32))
    assert np.max(np.abs(out - ref)) < 1e-8


def test_batched_gribov_annealing_matches_oracle():
    # the annealing search over Gribov copies (Landau gauge, FP64): random
    # gauge copies of two uneven lattices in one batch, two annealing steps
    # (T 4 then 1e-4, 3 microcanonical sweeps each; each copy has its own
    # Philox key (seed, instance)), then overrelaxation to theta < 1e-10 per
    # copy.  The oracle runs each copy alone with the same key: links after
    # the annealing to 1e-7 (two steps amplify rounding by about 1e6), then
    # identical overrelaxation sweep counts and F to 1e-12; and the ranking
    # of the copies by F, which is what the search reports, is the same.
    shapes = [(4, 4, 6, 4), (6, 4, 4, 2)]
    ncopy = 3
    dl = [d for d in shapes for _ in range(ncopy)]
    say("batched gribov annealing", dl)
    Us = []
    for li, d in enumerate(shapes):
        base = I.smooth(d, 0.5, 7101 + li)
        for c in range(ncopy):
            Us.append(I.gauge_copy(base.copy(), d, 7200 + 8 * li + c))
    fx = fixer(dl, "landau", "f64r18")
    for k, U in enumerate(Us):
        fx.upload(k, U)
    fx.set_anneal(4.0, 1e-4, 2, nmicro=3, seed=7001)
    fx.sweep("anneal")
    mids = [fx.download(k) for k in range(len(dl))]
    fx.set_overrelax(1.7)
    st, done = fx.sweep("or", max_sweeps=5000, tol=1e-10, check_every=5)
    Fg = [fx.measure(k)[0] for k in range(len(dl))]
    fx.close()
    assert st == 0
    Fo = []
    for k, (U, d) in enumerate(zip(Us, dl)):
        ref = U.copy()
        ctr = O.anneal(ref, d, "landau", 4.0, 1e-4, 2, nmicro=3, seed=7001, instance=k, sweep_counter=0)
        assert ctr == 8
        err = np.max(np.abs(mids[k] - ref))
        r = O.run(ref, d, "landau", "or", omega=1.7, max_sweeps=5000, tol=1e-10, check_every=5, sweep_counter=ctr)
        Fo.append(O.measure(ref, d, "landau")[0])
        say("copy", k, "annealed |gpu - oracle|", err, "OR sweeps", int(done[k]), int(r.sweeps_done[0]),
            "F", Fg[k], Fo[k])
        assert err < 1e-7
        assert r.status == 0 and int(done[k]) == int(r.sweeps_done[0])
        assert abs(Fg[k] - Fo[k]) < 1e-12
    for li in range(len(shapes)):
        sl = slice(li * ncopy, (li + 1) * ncopy)
        assert int(np.argmax(Fg[sl])) == int(np.argmax(Fo[sl]))


def test_anneal_resume_is_bit_identical():
    # checkpoint/resume: the random streams depend only on (seed, instance,
    # sweep index, site), so two halves with the sweep index carried over
    # give the same chain as one run
    dims = (4, 4, 4, 4)
    say("anneal resume")
    U = I.smooth(dims, 0.7, 4003)
    a = fixer([dims], "mag", "f64r18")
    a.upload(0, U)
    a.set_seed(9)
    a.set_temperature(0.8)
    for k in range(6):
        a.sweep("heatbath", max_sweeps=1, tol=0.0)
    full = a.download(0)
    a.close()
    b = fixer([dims], "mag", "f64r18")
    b.upload(0, U)
    b.set_seed(9)
    b.set_temperature(0.8)
    for k in range(3):
        b.sweep("heatbath", max_sweeps=1, tol=0.0)
    idx = b.get_sweep_index(0)
    mid = b.download(0)
    b.close()
    c = fixer([dims], "mag", "f64r18")
    c.upload(0, mid)
    c.set_seed(9)
    c.set_temperature(0.8)
    c.set_sweep_index(0, idx)
    for k in range(3):
        c.sweep("heatbath", max_sweeps=1, tol=0.0)
    np.testing.assert_array_equal(c.download(0), full)
    c.close()


def test_c4_mag_anneal_full_size():
    # 32^4, eps = 0.7: T 1.5 -> 0.01 over 3000 heatbath sweeps (+3 micro),
    # then overrelaxation omega = 1.7 to theta < 1e-12, mixed storage
    dims = (32, 32, 32, 32)
    say("C4 full size")
    U = I.smooth(dims, 0.7, 4001)
    plaq = O.plaquette(U, dims)
    fx = fixer([dims], "mag", "mixed", reunit_every=100, tail_theta=1e-9)
    fx.upload(0, U)
    fx.set_anneal(1.5, 0.01, 3000, nmicro=3, seed=4002)
    st, done = fx.sweep("anneal")
    assert fx.get_sweep_index(0) == 12000
    F_sa, th_sa = fx.measure(0)
    annealed = fx.download(0)
    # one OR half-sweep on the annealed state vs the oracle on sampled sites
    from tests.test_gpu_fullsize import _site_links
    from tests._su import coords
    fx.set_overrelax(1.7)
    fx.halfsweep("or", 0)
    one = fx.download(0)
    ref = annealed.copy()  # the download is the FP32 state (row 2 rebuilt in FP64)
    rng = np.random.default_rng(6)
    sites = []
    while len(sites) < 128:
        s = int(rng.integers(0, U.shape[0]))
        if sum(coords(dims, s)) % 2 == 0:
            sites.append(s)
    O.update_sites(ref, dims, "mag", "or", sites, omega=1.7)
    err = max(float(np.max(np.abs(one[q, m] - ref[q, m]))) for s in sites for (q, m) in _site_links(U, dims, s))
    say("annealed: F", F_sa, "theta", th_sa, "OR half-sweep max err", err)
    assert err < 3e-5
    # the sweeps end on links reprojected in FP64 (reprojection in use on
    # FP32 storage), checked again after that reprojection
    st, done = fx.sweep("or", max_sweeps=100000, tol=1e-12, check_every=10)
    F, th = fx.measure(0)
    out = fx.download(0)
    fx.close()
    say("after OR: status", st, "sweeps", done, "F", F, "theta of the delivered links", th)
    assert st == 0 and th < 1e-12
    assert F > F_sa
    assert abs(O.plaquette(out, dims) - plaq) < 1e-6
    Fo, tho = O.measure(out, dims, "mag")
    assert abs(Fo - F) < 1e-9 and tho < 1e-12
    # the overrelaxation stage against the oracle's, from the same annealed
    # (FP32-rounded) state: same even half-sweep first, then sweeps to
    # theta < 1e-12 in FP64.  F agrees within the storage-rounding bound (MAG's
    # F averages |U_ii|^2, twice the relative rounding of Re tr U) unless the
    # runs end in different copies.  MAG leaves a local U(1) x U(1) freedom
    # (diagonal phases), which changes Re tr U but not the per-link
    # sum_i |U_ii|^2: within one copy the two fixes differ in it by the
    # residual of the stopping tolerance (~1e-3 for MAG's slow modes),
    # distinct copies by O(0.1).
    ref = annealed.copy()
    O.halfsweep(ref, dims, "mag", "or", 0, omega=1.7)
    r = O.run(ref, dims, "mag", "or", omega=1.7, max_sweeps=100000, tol=1e-12, check_every=10)
    Fr = O.measure(ref, dims, "mag")[0]
    dia = lambda W: sum(W[..., i, i, 0] ** 2 + W[..., i, i, 1] ** 2 for i in range(3))
    ddia = float(np.max(np.abs(dia(out) - dia(ref))))
    say("OR stage: oracle sweeps", r.sweeps_done.tolist(), "F", Fr, "gpu F", F, "rel", abs(F - Fr) / Fr,
        "max |d sum |U_ii|^2|", ddia)
    assert r.status == 0
    if ddia >= 2e-2:
        pytest.skip("the GPU (FP32 storage) and oracle (FP64) overrelaxation stages ended in different MAG "
                    "copies: max |d sum_i |U_ii|^2| = %.3g, F %.12f vs %.12f" % (ddia, F, Fr))
    assert abs(F - Fr) < 2 * f_orbit_tol(done[0], np.prod(dims)) * Fr


@pytest.mark.parametrize("storage", ["f64r18", "mixed"])
def test_checkpoint_files_resume_bit_identically(storage, tmp_path):
    # annealing in two halves with a checkpoint on disk in between equals the
    # uninterrupted run (mixed storage: the FP32 links round-trip exactly).
    # Schedule T 1 -> 0.5 over 5 steps (T_k = 1 - k/8, exact in binary),
    # split into the steps k = 0..2 and k = 3..4.
    from paper_1212_5221_amd import checkpoint
    dims = (4, 4, 4, 4)
    say("checkpoint files", storage)
    U = I.smooth(dims, 0.7, 4006)
    a = fixer([dims, dims], "mag", storage)
    a.upload(0, U)
    a.upload(1, U[::-1].copy())
    a.set_anneal(1.0, 0.5, 5, nmicro=3, seed=11)
    a.sweep("anneal")
    full = [a.download(0), a.download(1)]
    a.close()
    b = fixer([dims, dims], "mag", storage)
    b.upload(0, U)
    b.upload(1, U[::-1].copy())
    b.set_anneal(1.0, 0.75, 3, nmicro=3, seed=11)
    b.sweep("anneal")
    checkpoint.save(b, str(tmp_path), extra={"step": 3})
    b.close()
    c = fixer([dims, dims], "mag", storage)
    assert checkpoint.load(c, str(tmp_path)) == {"step": 3}
    c.set_anneal(0.625, 0.5, 2, nmicro=3, seed=11)
    c.sweep("anneal")
    np.testing.assert_array_equal(c.download(0), full[0])
    np.testing.assert_array_equal(c.download(1), full[1])
    c.close()


@pytest.mark.parametrize("gauge,waves", launch_shapes(["landau", "coulomb", "mag"]))
@pytest.mark.parametrize("update", ["heatbath", "sr"])
def test_mixed_random_halfsweeps_match_oracle_from_the_stored_state(gauge, waves, update):
    # Mixed storage cannot follow the FP64 chain, so each half-sweep of the
    # heatbath and stochastic-relaxation kernels on FP32-12 storage is
    # recomputed by the oracle from the state the GPU stored before it (same
    # seed, temperature and sweep index).  Stochastic relaxation computes the
    # update in FP64: the result differs only by the FP32 rounding of the
    # stored rows and the first-order renormalisation of the forward links
    # before it, each a few ulp(1) = 6e-8: bound 1e-6.  The heatbath computes
    # its local algebra (K, the MAG coefficients, the subgroup products) in
    # FP32 like overrelaxation and draws the sample in FP64 from it: the
    # sample is a smooth function of the FP32 direction and strength, with
    # the errors of a few ulp(8) that bound the FP32 overrelaxation step:
    # 3e-5.  (A rejection decision within ~1e-7 of its boundary could flip;
    # at these temperatures the Kennedy-Pendleton branch, where that
    # probability is ~1e-9 per decision, draws almost all samples.)
    dims = (4, 4, 6, 4)
    say("mixed", update, "half-sweeps from the stored state", gauge, "waves", waves)
    fx = fixer([dims], gauge, "mixed", waves=waves)
    fx.upload(0, I.smooth(dims, 0.7, 4101))
    fx.set_seed(41)
    fx.set_temperature(0.8)
    fx.set_stochastic(0.5)
    for k in range(3):
        fx.set_sweep_index(0, k)
        for parity in (0, 1):
            S = fx.download(0)
            fx.halfsweep(update, parity)
            out = fx.download(0)
            O.halfsweep(S, dims, gauge, update, parity, omega=1.0, T=0.8, p_sr=0.5, seed=41, instance=0, sweep=k)
            err = np.max(np.abs(out - S))
            assert err < (3e-5 if update == "heatbath" else 1e-6), (k, parity, err)
    fx.close()
