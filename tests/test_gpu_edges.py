"""Edge cases of the HIP path against the oracle: the smallest lattices (an
extent of 2 makes the forward and backward neighbour the same site), input
that already satisfies the stopping rule, zero sweeps, and the size limit."""
import numpy as np
import pytest

import oracle as O
from paper_1212_5221_amd import inputs as I
from tests.test_gpu_parity import fixer, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 4, 2, 6)])
@pytest.mark.parametrize("gauge", ["landau", "coulomb", "mag"])
def test_smallest_lattices_match_oracle(gauge, dims):
    say("smallest lattice", gauge, dims)
    U = I.smooth(dims, 0.5, 61)
    ref = U.copy()
    r = O.run(ref, dims, gauge, "or", omega=1.7, max_sweeps=2000, tol=1e-12, check_every=1)
    fx = fixer([dims], gauge, "f64r18")
    fx.upload(0, U)
    fx.set_overrelax(1.7)
    st, done = fx.sweep("or", max_sweeps=2000, tol=1e-12, check_every=1)
    out = fx.download(0)
    fx.close()
    assert st == r.status
    np.testing.assert_array_equal(done, r.sweeps_done.astype(np.int32))
    assert np.max(np.abs(out - ref)) < 1e-10


@pytest.mark.parametrize("storage", ["f64r18", "f64r12", "mixed"])
def test_fixed_input_stops_before_any_sweep(storage):
    # unit links: theta = 0 at the input check, so no sweep runs
    dims = (4, 4, 4, 4)
    say("unit links", storage)
    U = np.zeros((256, 4, 3, 3, 2))
    for i in range(3):
        U[:, :, i, i, 0] = 1.0
    fx = fixer([dims], "landau", storage)
    fx.upload(0, U)
    st, done = fx.sweep("or", max_sweeps=100, tol=1e-12, check_every=5)
    F, th = fx.measure(0)
    out = fx.download(0)
    fx.close()
    assert st == 0 and done[0] == 0
    assert F == 1.0 and th == 0.0
    np.testing.assert_array_equal(out, U)


def test_zero_sweeps():
    dims = (4, 4, 4, 4)
    say("zero sweeps")
    U = I.smooth(dims, 0.5, 62)
    fx = fixer([dims], "landau", "f64r18")
    fx.upload(0, U)
    st, done = fx.sweep("or", max_sweeps=0, tol=1e-12, check_every=5)
    out = fx.download(0)
    fx.close()
    from paper_1212_5221_amd import gf
    assert st == gf.NOT_CONVERGED and done[0] == 0
    np.testing.assert_array_equal(out, U)


def test_size_limit_and_bad_arguments():
    from paper_1212_5221_amd import gf
    say("size limit")
    with pytest.raises(gf.GFError) as e:
        gf.GaugeFixer([(512, 512, 512, 16)])  # 2^31 sites
    assert e.value.code == gf.E_DIMS
    with pytest.raises(gf.GFError) as e:
        gf.GaugeFixer([(4, 4, 0, 4)])
    assert e.value.code == gf.E_DIMS
    fx = fixer([(4, 4, 4, 4)], "landau", "f64r18")
    with pytest.raises(gf.GFError) as e:
        fx.sweep("or", max_sweeps=-1)
    assert e.value.code == gf.E_INVALID
    with pytest.raises(gf.GFError) as e:
        fx.download(0, t0=3, nt=2)
    assert e.value.code == gf.E_INVALID
    with pytest.raises(gf.GFError) as e:
        fx.set_timing(True, every=-1)
    assert e.value.code == gf.E_INVALID
    fx.close()


def test_two_handles_interleaved():
    # two handles (own workspaces, own graphs) on the same stream, their
    # sweeps interleaved chunk by chunk, end where each ends alone
    say("two handles")
    dims = (4, 4, 6, 4)
    UA = I.smooth(dims, 0.5, 63)
    UB = I.smooth(dims, 0.5, 64)

    def alone(U):
        fx = fixer([dims], "landau", "mixed", reunit_every=5)
        fx.upload(0, U)
        fx.set_overrelax(1.7)
        st, done = fx.sweep("or", max_sweeps=3000, tol=1e-12, check_every=10)
        out = fx.download(0)
        fx.close()
        return st, done, out

    ra, rb = alone(UA), alone(UB)
    fa = fixer([dims], "landau", "mixed", reunit_every=5)
    fb = fixer([dims], "landau", "mixed", reunit_every=5)
    fa.upload(0, UA)
    fb.upload(0, UB)
    for f in (fa, fb):
        f.set_overrelax(1.7)
    da = db = 0
    for _ in range(300):
        if da >= 0:
            st, d = fa.sweep("or", max_sweeps=10, tol=1e-12, check_every=10)
            da = -1 if st == 0 else da
        if db >= 0:
            st, d = fb.sweep("or", max_sweeps=10, tol=1e-12, check_every=10)
            db = -1 if st == 0 else db
        if da < 0 and db < 0:
            break
    assert da < 0 and db < 0
    np.testing.assert_array_equal(fa.download(0), ra[2])
    np.testing.assert_array_equal(fb.download(0), rb[2])
    fa.close()
    fb.close()
