"""Every launch shape of every half-sweep kernel table against the oracle,
and the autotuner's contract.

A shape is W wavefronts per group of 64 sites (1, 2, 4; Coulomb 1, 2), B
threads per block (64 ... 512, B >= 64 W), cached or non-temporal link
traffic, and the XCD-contiguous or linear tile order.  The shapes of a table
are found by asking the library for each combination (gf_set_shape refuses
the ones that are not built), so a shape the autotuner can pick is never
left out.  Each shape runs one even and one odd half-sweep of the ragged
6x4x6x4 lattice (288 sites per parity: 4.5 blocks of 64 sites, half a block
of 512), compared with the oracle to the bounds of test_gpu_parity, and --
since block size, cache policy and tile order do not touch the arithmetic of
a site -- bit for bit with the other shapes of the same W.  Random updates
on FP32 storage are compared half-sweep by half-sweep with the oracle run
from the state the GPU stored (1e-6; the heatbath on mixed storage, whose
local algebra is FP32, 3e-5; as in test_gpu_anneal).

The autotuner: the bound state (links, sweep indices, stop flags) is the
same before and after tuning, and a tuning cache hands a second handle of
the same configuration the stored shapes without timing.
"""
import itertools
import os

import numpy as np
import pytest

import oracle as O
from paper_1212_5221_amd import gf
from paper_1212_5221_amd import inputs as I
from tests.test_gpu_parity import FP32_MODES, TOL_LINK, f32_round, fixer, say

pytestmark = pytest.mark.gpu

DIMS = (6, 4, 6, 4)
FLAGS = (0, gf.SHAPE_NONTEMPORAL, gf.SHAPE_LINEAR_TILES, gf.SHAPE_NONTEMPORAL | gf.SHAPE_LINEAR_TILES)


def _table(storage, update):
    if update == "heatbath":
        return "heatbath"
    if update == "sr" or storage in ("f64r18", "f64r12", "mixed64"):
        return "fp64"
    return "fp32"


def _shapes(fx, table, update):
    out = []
    for w, b, f in itertools.product((1, 2, 4), (64, 128, 256, 512), FLAGS):
        # the random updates have cached variants only
        if update in ("heatbath", "sr") and (f & gf.SHAPE_NONTEMPORAL):
            continue
        try:
            fx.set_shape(table, w, b, f)
        except gf.GFError as e:
            assert e.code == gf.E_INVALID
            continue
        assert fx.get_shape(table) == (w, b, f)
        out.append((w, b, f))
    return out


def _oracle(U, gauge, update, storage):
    ref = f32_round(U) if storage in FP32_MODES else U.copy()
    G = O.identity_field(int(np.prod(DIMS))) if gauge == "coulomb" else None
    for parity in (0, 1):
        O.halfsweep(ref, DIMS, gauge, update, parity, omega=1.7, T=0.7, p_sr=0.5, seed=77, instance=0, sweep=0, G=G)
    return ref


@pytest.mark.parametrize("storage", ["f64r18", "f64r12", "mixed", "mixed64", "single"])
@pytest.mark.parametrize("gauge", ["landau", "coulomb", "mag"])
def test_every_shape_matches_oracle(gauge, storage):
    U = I.smooth(DIMS, 0.6, 11)
    updates = ["or", "micro"] + (["heatbath", "sr"] if storage != "single" else [])
    fx = fixer([DIMS], gauge, storage)
    fx.set_overrelax(1.7)
    fx.set_seed(77)
    fx.set_temperature(0.7)
    fx.set_stochastic(0.5)
    n = 0
    for update in updates:
        table = _table(storage, update)
        ref = _oracle(U, gauge, update, storage)  # the whole sweep from the input
        by_w = {}
        shapes = _shapes(fx, table, update)
        assert shapes, (gauge, storage, update)
        # random updates on FP32 storage: each half-sweep against the oracle
        # from the state the GPU stored before it (FP64 arithmetic on FP32
        # links; a poorly determined direction amplifies the storage
        # rounding of the first half-sweep in the second's sample)
        stepwise = storage in FP32_MODES and update in ("heatbath", "sr")
        for w, b, f in shapes:
            fx.set_shape(table, w, b, f)
            fx.upload(0, U)
            for parity in (0, 1):
                S = fx.download(0) if stepwise else None
                fx.halfsweep(update, parity)
                if stepwise:
                    out = fx.download(0)
                    O.halfsweep(S, DIMS, gauge, update, parity, omega=1.7, T=0.7, p_sr=0.5, seed=77, instance=0,
                                sweep=0, G=O.identity_field(int(np.prod(DIMS))) if gauge == "coulomb" else None)
                    err = float(np.max(np.abs(out - S)))
                    # the heatbath on mixed storage: FP32 local algebra (test_gpu_anneal)
                    tol = 3e-5 if (update == "heatbath" and storage == "mixed") else 1e-6
                    assert err < tol, (gauge, storage, update, w, b, f, parity, err)
            out = fx.download(0)
            if not stepwise:
                err = float(np.max(np.abs(out - ref)))
                assert err < TOL_LINK[storage], (gauge, storage, update, w, b, f, err)
            if w in by_w:
                np.testing.assert_array_equal(out, by_w[w], err_msg=str((gauge, storage, update, w, b, f)))
            else:
                by_w[w] = out
            n += 1
        say(gauge, storage, update, table, "shapes", len(shapes))
    fx.close()
    say("checked", n, "shape runs")


def _state(fx, ninst):
    return ([fx.download(k) for k in range(ninst)], [fx.get_sweep_index(k) for k in range(ninst)],
            [fx.measure(k) for k in range(ninst)])


def _fresh(dl, gauge, storage):
    fx = fixer(dl, gauge, storage, reunit_every=7)
    for k, d in enumerate(dl):
        fx.upload(k, I.smooth(d, 0.5, 61 + k))
    fx.set_overrelax(1.7)
    fx.set_temperature(0.5)
    # a partly fixed state with some units stopped
    fx.sweep("or", max_sweeps=30, tol=1e-3, check_every=5)
    return fx


@pytest.mark.parametrize("gauge,storage", [("landau", "mixed"), ("coulomb", "mixed"), ("mag", "f64r12")])
def test_autotune_leaves_the_state_unchanged(gauge, storage, tmp_path):
    dl = [(4, 6, 4, 6), (8, 4, 4, 4)]
    fx = _fresh(dl, gauge, storage)
    before = _state(fx, len(dl))
    cache = str(tmp_path / "tune.txt")
    fx.set_tune_cache(cache)
    fx.autotune(reps=2)
    fx.autotune_heatbath(reps=1)
    after = _state(fx, len(dl))
    for x, y in zip(before[0], after[0]):
        np.testing.assert_array_equal(x, y)
    assert before[1] == after[1] and before[2] == after[2]
    shapes = {t: fx.get_shape(t) for t in ("fp32", "fp64", "heatbath")}
    say("tuned", gauge, storage, shapes)
    # the run goes on exactly as a run that never tuned but switches to the
    # same shapes at the same point
    st1, d1 = fx.sweep("or", max_sweeps=200, tol=1e-11, check_every=5)
    out1 = [fx.download(k) for k in range(len(dl))]
    fx.close()
    ref = _fresh(dl, gauge, storage)
    used = ["fp32"] if storage == "mixed" else ["fp64"]
    for t in used + ["heatbath"]:
        ref.set_shape(t, *shapes[t])
    st2, d2 = ref.sweep("or", max_sweeps=200, tol=1e-11, check_every=5)
    out2 = [ref.download(k) for k in range(len(dl))]
    ref.close()
    assert st1 == st2
    np.testing.assert_array_equal(d1, d2)
    for x, y in zip(out1, out2):
        np.testing.assert_array_equal(x, y)
    # the cache holds one line per tuned table; a second handle of the same
    # configuration takes the stored shapes without timing (here: shapes
    # written into the file by hand)
    lines = [l.split() for l in open(cache).read().split("\n") if l.strip()]
    assert len(lines) >= 2 and all(len(l) == 5 for l in lines)
    with open(cache, "w") as f:
        for l in lines:
            heat = "/kernels2/" in l[0]
            f.write("%s 2 128 %d 0\n" % (l[0], 0 if heat else 1))
    fx2 = fixer(dl, gauge, storage, reunit_every=7)
    fx2.set_tune_cache(cache)
    w2, b2 = fx2.autotune(reps=1)
    fx2.autotune_heatbath(reps=1)
    assert (w2, b2) == (2, 128)
    for t in used:
        assert fx2.get_shape(t) == (2, 128, gf.SHAPE_NONTEMPORAL | gf.SHAPE_LINEAR_TILES)
    assert fx2.get_shape("heatbath") == (2, 128, gf.SHAPE_LINEAR_TILES)
    fx2.close()


def test_tune_cache_errors(tmp_path):
    fx = fixer([(4, 4, 4, 4)], "landau", "mixed")
    d = tmp_path / "nodir" / "tune.txt"
    fx.set_tune_cache(str(d))  # a missing file is an empty cache
    with pytest.raises(gf.GFError) as e:
        fx.autotune(reps=1)  # but the choice cannot be written there
    assert e.value.code == gf.E_INVALID
    # malformed lines are ignored
    p = tmp_path / "bad.txt"
    p.write_text("garbage\nkey 3 64 0 1\n")
    fx.set_tune_cache(str(p))
    fx.autotune(reps=1)
    assert os.path.exists(p)
    with pytest.raises(gf.GFError):
        fx.set_shape("fp32", 3, 64, 0)
    with pytest.raises(gf.GFError):
        fx.set_shape("fp32", 4, 128, 0)  # B < 64 W
    with pytest.raises(gf.GFError):
        fx.set_shape("heatbath", 1, 256, gf.SHAPE_NONTEMPORAL)
    with pytest.raises(gf.GFError):
        fx.set_shape(7, 1, 256, 0)
    fx.close()
