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
