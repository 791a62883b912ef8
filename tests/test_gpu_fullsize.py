"""GPU parity at the benchmark's full size (32^4 Landau, mixed FP32-12 storage)
in the launch configuration bench.py times (autotuned waves per site group).

* One even half-sweep: sampled sites are recomputed by the oracle one by one
  from the same FP32-rounded input (sites of one parity are independent, so
  updating only the sampled sites reproduces their links exactly).
* A complete fix to theta < 1e-12: properties that hold at any size (theta
  measured by the oracle on the downloaded links, gauge invariants unchanged,
  unitarity after the final FP64 reprojection) and F against the oracle's
  converged F stored in tests/golden (written by a script calling only the
  oracle), relative 1e-9 unless the two runs ended in different Gribov
  copies.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle as O
from paper_1212_5221_amd import inputs as I
from tests.test_gpu_parity import f32_round, say

pytestmark = pytest.mark.gpu

DIMS = (32, 32, 32, 32)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_landau_oracle.json")


def bench_fixer(U, storage="mixed"):
    """the benchmark's fixer, autotuned on U as bench.py does; U uploaded"""
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    from paper_1212_5221_amd import gf
    fx = bench.make_fixer(gf, storage)
    fx.upload(0, U)
    fx.autotune(reps=10)
    fx.upload(0, U)
    return fx


def _site_links(U, dims, s):
    """the 8 links adjacent to site s (4 forward, 4 backward) as (site, mu) pairs"""
    from tests._su import coords, site_index
    t, x, y, z = coords(dims, s)
    out = [(s, mu) for mu in range(4)]
    c = [t, x, y, z]
    for mu in range(4):
        b = list(c)
        b[mu] = (b[mu] - 1) % dims[mu]
        out.append((site_index(dims, *b), mu))
    return out


def test_c2_one_halfsweep_sampled_sites():
    say("C2 full-size half-sweep, sampled sites")
    U = I.smooth(DIMS, 0.5, 2001)
    fx = bench_fixer(U)
    fx.halfsweep("or", 0)
    out = fx.download(0)
    fx.close()
    ref = f32_round(U)
    rng = np.random.default_rng(5)
    from tests._su import coords
    sites = []
    while len(sites) < 256:
        s = int(rng.integers(0, U.shape[0]))
        if sum(coords(DIMS, s)) % 2 == 0:
            sites.append(s)
    # include the first and last sites of the half-volume (tile edges)
    sites += [0, U.shape[0] - 2 + (sum(coords(DIMS, U.shape[0] - 2)) % 2)]
    O.update_sites(ref, DIMS, "landau", "or", sites, omega=1.7)
    err = 0.0
    for s in sites:
        for (q, mu) in _site_links(U, DIMS, s):
            err = max(err, float(np.max(np.abs(out[q, mu] - ref[q, mu]))))
    say("max |gpu - oracle| over sampled links", err)
    assert err < 3e-5  # FP32 update arithmetic, see test_gpu_parity


def test_c2_full_fix_properties():
    say("C2 full fix, seed 2001")
    U = I.smooth(DIMS, 0.5, 2001)
    before = [O.wilson_loop(U, DIMS, r, t) for r, t in ((1, 1), (1, 2))]
    fx = bench_fixer(U)
    # FP32 storage with reprojection in use: the sweeps end on links
    # reprojected in FP64 (rounded to FP32) and checked again after it
    st, done = fx.sweep("or", max_sweeps=50000, tol=1e-12, check_every=10)
    F, th = fx.measure(0)
    out = fx.download(0)
    fx.close()
    say("status", st, "sweeps", done, "F", F, "theta of the delivered links", th)
    assert st == 0 and th < 1e-12
    Fo, tho = O.measure(out, DIMS, "landau")
    assert tho < 1e-12
    assert abs(Fo - F) < 1e-9 * F
    after = [O.wilson_loop(out, DIMS, r, t) for r, t in ((1, 1), (1, 2))]
    # FP32 storage: gauge invariants agree to FP32 rounding averaged over the lattice
    np.testing.assert_allclose(after, before, atol=1e-6)
    # FP32 rows: unitary to their rounding
    assert O.unitarity(out)[1] < 1e-6
    if os.path.exists(GOLDEN):
        g = json.load(open(GOLDEN)).get("2001")
        if g:
            rel = abs(F - g["F"]) / g["F"]
            say("F vs oracle F", F, g["F"], "rel", rel)
            # Re tr U per link (invariant under the global transformations the
            # Landau condition leaves free): within one Gribov copy the two
            # fixes differ by the residual of the stopping tolerance (up to
            # ~1e-4 here), distinct copies by O(0.1)
            dtr = max(abs((out[s, m, 0, 0, 0] + out[s, m, 1, 1, 0] + out[s, m, 2, 2, 0]) - v)
                      for s, m, v in g["retrace_samples"])
            say("max |d Re tr U| over the sampled links", dtr)
            same_copy = dtr < 1e-2
            if same_copy:
                # the 1e-9 target for this workload; the rounding-walk bound
                # f_orbit_tol (9e-9 here) would allow more
                assert rel < 1e-9
            else:
                pytest.skip("mixed and FP64 runs ended in different Gribov copies (F differs by %.2e)" % rel)
