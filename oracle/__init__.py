"""Plain FP64 CPU oracle for SU(3) and SU(2) gauge fixing (arXiv:1212.5221).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
leg of the benchmark use it to check the GPU library.  It shares no code with
the GPU path (see ``gf_oracle.c`` for the readings of the paper it takes).

Links are numpy float64 arrays in the natural layout
(sites, 4, 3, 3, 2) = t, x, y, z, mu, i, j, re/im with z fastest; the su2_*
functions take SU(2) links (sites, 4, 2, 2, 2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gf_oracle.c")
_LIB = os.path.join(_HERE, "libgforacle.so")
_lib = None

LANDAU, COULOMB, MAG = 0, 1, 2
OR, MICRO, HEATBATH, SR = 0, 1, 2, 3

_GAUGES = {"landau": LANDAU, "coulomb": COULOMB, "mag": MAG}
_UPDATES = {"or": OR, "micro": MICRO, "heatbath": HEATBATH, "sr": SR}

_I32_4 = ctypes.c_int32 * 4
_dp = ctypes.POINTER(ctypes.c_double)
_u64 = ctypes.c_uint64
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_d = ctypes.c_double


def build(force: bool = False) -> str:
    """Compile gf_oracle.c (gcc -O2, OpenMP, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
             "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    L = ctypes.CDLL(_LIB)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i64p = ctypes.POINTER(ctypes.c_int64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    L.gfo_halfsweep.argtypes = [_dp, _I32_4, _i32, _i32, _i32, _d, _d, _d, _u64, _u64, _u64, _dp, u8p]
    L.gfo_sweep.argtypes = [_dp, _I32_4, _i32, _i32, _d, _d, _d, _u64, _u64, _u64, _dp, u8p]
    L.gfo_update_sites.argtypes = [_dp, _I32_4, _i32, _i32, _d, _d, _d, _u64, _u64, _u64, _dp, i64p, _i64]
    L.gfo_local_g.argtypes = [_dp, _dp, _i32, _i32, _i32, _i32, _i32, _d, _d, _d, _u64, _u64, _u64, _u64,
                              _i32, _dp]
    L.gfo_mag_coefficients.argtypes = [_dp, _dp, _i32, _i32, _i32, _dp]
    L.gfo_subgroup_quaternion.argtypes = [_dp, _i32, _i32, _dp]
    L.gfo_left_subgroup_mult.argtypes = [_dp, _i32, _i32, _dp]
    L.gfo_right_subgroup_mult_dag.argtypes = [_dp, _i32, _i32, _dp]
    L.gfo_or_map.argtypes = [_dp, _d, _dp]
    L.gfo_quat_mul.argtypes = [_dp, _dp, _dp]
    L.gfo_measure.argtypes = [_dp, _I32_4, _i32, _dp, _dp]
    L.gfo_measure_slices.argtypes = [_dp, _I32_4, _dp, _dp]
    L.gfo_theta_via_K.argtypes = [_dp, _I32_4, _i32]
    L.gfo_theta_via_K.restype = _d
    L.gfo_theta_mag_via_subgroups.argtypes = [_dp, _I32_4]
    L.gfo_theta_mag_via_subgroups.restype = _d
    L.gfo_theta_mag_literal.argtypes = [_dp, _I32_4]
    L.gfo_theta_mag_literal.restype = _d
    L.gfo_unitarity.argtypes = [_dp, _i64, _dp, _dp]
    L.gfo_unitarity_defect.argtypes = [_dp, _i64]
    L.gfo_unitarity_defect.restype = _d
    L.gfo_reunitarise.argtypes = [_dp, _i64]
    L.gfo_wilson_loop.argtypes = [_dp, _I32_4, _i32, _i32]
    L.gfo_wilson_loop.restype = _d
    L.gfo_plaquette.argtypes = [_dp, _I32_4]
    L.gfo_plaquette.restype = _d
    L.gfo_apply_gauge.argtypes = [_dp, _I32_4, _dp]
    L.gfo_coulomb_fix_u0.argtypes = [_dp, _I32_4, _dp]
    L.gfo_run.argtypes = [_dp, _I32_4, _i32, _i32, _d, _d, _i32, _d, _i32, _i32, _u64, _u64, u64p, i64p,
                          _dp, _dp, i32p, _i32, i32p]
    L.gfo_run.restype = ctypes.c_int
    L.gfo_anneal.argtypes = [_dp, _I32_4, _i32, _d, _d, _i32, _i32, _u64, _u64, u64p, _dp]
    L.gfo_philox4x64_10.argtypes = [u64p, u64p, u64p]
    L.gfo_exp_inverse_cdf.argtypes = [_d, _d]
    L.gfo_exp_inverse_cdf.restype = _d
    L.gfo_sample_r0.argtypes = [_d, u64p, _u64, _u64, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.gfo_sample_r0.restype = _d
    L.gfo2_halfsweep.argtypes = [_dp, _I32_4, _i32, _i32, _i32, _d, _d, _d, _u64, _u64, _u64, _dp, u8p]
    L.gfo2_update_sites.argtypes = [_dp, _I32_4, _i32, _i32, _d, _d, _d, _u64, _u64, _u64, _dp, i64p, _i64]
    L.gfo2_local_g.argtypes = [_dp, _dp, _i32, _i32, _i32, _d, _d, _d, _u64, _u64, _u64, _u64, _dp]
    L.gfo2_measure.argtypes = [_dp, _I32_4, _i32, _dp, _dp]
    L.gfo2_measure_slices.argtypes = [_dp, _I32_4, _dp, _dp]
    L.gfo2_unitarity.argtypes = [_dp, _i64, _dp, _dp]
    L.gfo2_reunitarise.argtypes = [_dp, _i64]
    L.gfo2_plaquette.argtypes = [_dp, _I32_4]
    L.gfo2_plaquette.restype = _d
    L.gfo2_apply_gauge.argtypes = [_dp, _I32_4, _dp]
    L.gfo2_coulomb_fix_u0.argtypes = [_dp, _I32_4, _dp]
    _lib = L
    return L


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _dims(dims):
    d = [int(x) for x in dims]
    return _I32_4(*d)


def _gauge(g):
    return _GAUGES[g] if isinstance(g, str) else int(g)


def _update(u):
    return _UPDATES[u] if isinstance(u, str) else int(u)


def _nsites(dims):
    return int(np.prod([int(x) for x in dims]))


def _check_links(U, dims):
    assert U.dtype == np.float64 and U.flags.c_contiguous, "links must be contiguous float64"
    assert U.size == _nsites(dims) * 72, "links must hold V*4*18 reals"


def identity_field(V: int) -> np.ndarray:
    g = np.zeros((V, 3, 3, 2))
    for i in range(3):
        g[:, i, i, 0] = 1.0
    return g


# ---------------------------------------------------------------- sweeps
def halfsweep(U, dims, gauge, update, parity, omega=1.0, T=0.0, p_sr=0.5, seed=0, instance=0, sweep=0,
              G=None, slice_active=None):
    _check_links(U, dims)
    sa = None
    if slice_active is not None:
        slice_active = np.ascontiguousarray(slice_active, dtype=np.uint8)
        sa = slice_active.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    _load().gfo_halfsweep(_ptr(U), _dims(dims), _gauge(gauge), _update(update), int(parity), float(omega),
                          float(T), float(p_sr), int(seed), int(instance), int(sweep),
                          _ptr(G) if G is not None else None, sa)


def sweep(U, dims, gauge, update, omega=1.0, T=0.0, p_sr=0.5, seed=0, instance=0, sweep=0, G=None,
          slice_active=None):
    for p in (0, 1):
        halfsweep(U, dims, gauge, update, p, omega, T, p_sr, seed, instance, sweep, G, slice_active)


def update_sites(U, dims, gauge, update, sites, omega=1.0, T=0.0, p_sr=0.5, seed=0, instance=0, sweep=0,
                 G=None):
    _check_links(U, dims)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    _load().gfo_update_sites(_ptr(U), _dims(dims), _gauge(gauge), _update(update), float(omega), float(T),
                             float(p_sr), int(seed), int(instance), int(sweep),
                             _ptr(G) if G is not None else None,
                             sites.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(sites))


def local_g(fwd, bwd, gauge, update, i, j, omega=1.0, T=0.0, p_sr=0.5, seed=0, instance=0, sweep=0, site=0,
            subgroup=0):
    fwd = np.ascontiguousarray(fwd, dtype=np.float64)
    bwd = np.ascontiguousarray(bwd, dtype=np.float64)
    nd = fwd.size // 18
    out = np.empty(4)
    _load().gfo_local_g(_ptr(fwd), _ptr(bwd), nd, _gauge(gauge), _update(update), i, j, float(omega), float(T),
                        float(p_sr), int(seed), int(instance), int(sweep), int(site), int(subgroup), _ptr(out))
    return out


def mag_coefficients(fwd, bwd, i, j):
    fwd = np.ascontiguousarray(fwd, dtype=np.float64)
    bwd = np.ascontiguousarray(bwd, dtype=np.float64)
    out = np.empty(3)
    _load().gfo_mag_coefficients(_ptr(fwd), _ptr(bwd), fwd.size // 18, i, j, _ptr(out))
    return out


def subgroup_quaternion(M, i, j):
    M = np.ascontiguousarray(M, dtype=np.float64)
    out = np.empty(4)
    _load().gfo_subgroup_quaternion(_ptr(M), i, j, _ptr(out))
    return out


def left_subgroup_mult(M, i, j, g):
    M = np.array(M, dtype=np.float64, copy=True, order="C")
    g = np.ascontiguousarray(g, dtype=np.float64)
    _load().gfo_left_subgroup_mult(_ptr(M), i, j, _ptr(g))
    return M


def right_subgroup_mult_dag(M, i, j, g):
    M = np.array(M, dtype=np.float64, copy=True, order="C")
    g = np.ascontiguousarray(g, dtype=np.float64)
    _load().gfo_right_subgroup_mult_dag(_ptr(M), i, j, _ptr(g))
    return M


def or_map(a, omega):
    a = np.ascontiguousarray(a, dtype=np.float64)
    out = np.empty(4)
    _load().gfo_or_map(_ptr(a), float(omega), _ptr(out))
    return out


def quat_mul(a, b):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    out = np.empty(4)
    _load().gfo_quat_mul(_ptr(a), _ptr(b), _ptr(out))
    return out


# ---------------------------------------------------------------- measures
def measure(U, dims, gauge):
    """(F, theta) of the whole lattice (Coulomb: averages over time-slices)."""
    _check_links(U, dims)
    F = ctypes.c_double()
    th = ctypes.c_double()
    _load().gfo_measure(_ptr(U), _dims(dims), _gauge(gauge), ctypes.byref(F), ctypes.byref(th))
    return F.value, th.value


def measure_slices(U, dims):
    _check_links(U, dims)
    Nt = int(dims[0])
    F = np.empty(Nt)
    th = np.empty(Nt)
    _load().gfo_measure_slices(_ptr(U), _dims(dims), _ptr(F), _ptr(th))
    return F, th


def theta_via_K(U, dims, gauge):
    return _load().gfo_theta_via_K(_ptr(U), _dims(dims), _gauge(gauge))


def theta_mag_via_subgroups(U, dims):
    return _load().gfo_theta_mag_via_subgroups(_ptr(U), _dims(dims))


def theta_mag_literal(U, dims):
    return _load().gfo_theta_mag_literal(_ptr(U), _dims(dims))


def unitarity(U):
    U = np.ascontiguousarray(U)
    m = ctypes.c_double()
    x = ctypes.c_double()
    _load().gfo_unitarity(_ptr(U), U.size // 18, ctypes.byref(m), ctypes.byref(x))
    return m.value, x.value


def unitarity_defect(U):
    U = np.ascontiguousarray(U)
    return _load().gfo_unitarity_defect(_ptr(U), U.size // 18)


def reunitarise(U):
    _load().gfo_reunitarise(_ptr(U), U.size // 18)
    return U


def wilson_loop(U, dims, R, T):
    _check_links(U, dims)
    return _load().gfo_wilson_loop(_ptr(U), _dims(dims), int(R), int(T))


def plaquette(U, dims):
    _check_links(U, dims)
    return _load().gfo_plaquette(_ptr(U), _dims(dims))


def apply_gauge(U, dims, g):
    _check_links(U, dims)
    g = np.ascontiguousarray(g, dtype=np.float64)
    _load().gfo_apply_gauge(_ptr(U), _dims(dims), _ptr(g))
    return U


def coulomb_fix_u0(U, dims, G):
    _check_links(U, dims)
    _load().gfo_coulomb_fix_u0(_ptr(U), _dims(dims), _ptr(np.ascontiguousarray(G)))
    return U


# ---------------------------------------------------------------- drivers
class RunResult:
    def __init__(self, status, sweeps_done, F, theta, check_sweeps, sweep_counter):
        self.status = status
        self.sweeps_done = sweeps_done
        self.F = F
        self.theta = theta
        self.check_sweeps = check_sweeps
        self.sweep_counter = sweep_counter

    def __repr__(self):
        return ("RunResult(status=%d, sweeps=%s, F=%r, theta=%r)" %
                (self.status, self.sweeps_done.tolist()[:4], self.F[-1] if len(self.F) else None,
                 self.theta[-1] if len(self.theta) else None))


def run(U, dims, gauge, update="or", omega=1.7, max_sweeps=1000, tol=1e-12, check_every=1, reunit_every=0,
        p_sr=0.5, seed=0, instance=0, sweep_counter=0, traj_cap=None):
    """Alg. 1 with the stop rule: modifies U in place, returns a RunResult."""
    _check_links(U, dims)
    g = _gauge(gauge)
    nslots = int(dims[0]) if g == COULOMB else 1
    if traj_cap is None:
        traj_cap = max_sweeps // max(1, check_every) + 2
    done = np.zeros(nslots, dtype=np.int64)
    F = np.zeros(traj_cap)
    th = np.zeros(traj_cap)
    ks = np.zeros(traj_cap, dtype=np.int32)
    n = ctypes.c_int32()
    ctr = ctypes.c_uint64(int(sweep_counter))
    st = _load().gfo_run(_ptr(U), _dims(dims), g, _update(update), float(omega), float(p_sr), int(max_sweeps),
                         float(tol), int(check_every), int(reunit_every), int(seed), int(instance),
                         ctypes.byref(ctr), done.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                         _ptr(F), _ptr(th), ks.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), traj_cap,
                         ctypes.byref(n))
    k = n.value
    return RunResult(st, done, F[:k].copy(), th[:k].copy(), ks[:k].copy(), ctr.value)


def anneal(U, dims, gauge, T0, T1, nsteps, nmicro=3, seed=0, instance=0, sweep_counter=0, G=None):
    """Simulated annealing schedule; returns the advanced sweep counter."""
    _check_links(U, dims)
    ctr = ctypes.c_uint64(int(sweep_counter))
    _load().gfo_anneal(_ptr(U), _dims(dims), _gauge(gauge), float(T0), float(T1), int(nsteps), int(nmicro),
                       int(seed), int(instance), ctypes.byref(ctr), _ptr(G) if G is not None else None)
    return ctr.value


# ---------------------------------------------------------------- randoms
def philox4x64_10(ctr, key):
    c = (ctypes.c_uint64 * 4)(*[int(x) for x in ctr])
    k = (ctypes.c_uint64 * 2)(*[int(x) for x in key])
    o = (ctypes.c_uint64 * 4)()
    _load().gfo_philox4x64_10(c, k, o)
    return np.array(list(o), dtype=np.uint64)


def exp_inverse_cdf(kappa, u):
    return _load().gfo_exp_inverse_cdf(float(kappa), float(u))


def sample_r0(a, key, sweep, site, subgroup):
    k = (ctypes.c_uint64 * 2)(*[int(x) for x in key])
    tries = ctypes.c_int()
    r0 = _load().gfo_sample_r0(float(a), k, int(sweep), int(site), int(subgroup), ctypes.byref(tries))
    return r0, tries.value


# ---------------------------------------------------------------- SU(2)
# Links of the SU(2) gauge group: (sites, 4, 2, 2, 2) float64, 8 reals per
# link; gauge fields (Coulomb G): (sites, 2, 2, 2).
def _check_links2(U, dims):
    assert U.dtype == np.float64 and U.flags.c_contiguous, "links must be contiguous float64"
    assert U.size == _nsites(dims) * 32, "SU(2) links must hold V*4*8 reals"


def su2_identity_field(V: int) -> np.ndarray:
    g = np.zeros((V, 2, 2, 2))
    g[:, 0, 0, 0] = g[:, 1, 1, 0] = 1.0
    return g


def su2_halfsweep(U, dims, gauge, update, parity, omega=1.0, T=0.0, p_sr=0.5, seed=0, instance=0, sweep=0,
                  G=None, slice_active=None):
    _check_links2(U, dims)
    sa = None
    if slice_active is not None:
        slice_active = np.ascontiguousarray(slice_active, dtype=np.uint8)
        sa = slice_active.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    _load().gfo2_halfsweep(_ptr(U), _dims(dims), _gauge(gauge), _update(update), int(parity), float(omega),
                           float(T), float(p_sr), int(seed), int(instance), int(sweep),
                           _ptr(G) if G is not None else None, sa)


def su2_sweep(U, dims, gauge, update, omega=1.0, T=0.0, p_sr=0.5, seed=0, instance=0, sweep=0, G=None,
              slice_active=None):
    for p in (0, 1):
        su2_halfsweep(U, dims, gauge, update, p, omega, T, p_sr, seed, instance, sweep, G, slice_active)


def su2_update_sites(U, dims, gauge, update, sites, omega=1.0, T=0.0, p_sr=0.5, seed=0, instance=0, sweep=0,
                     G=None):
    _check_links2(U, dims)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    _load().gfo2_update_sites(_ptr(U), _dims(dims), _gauge(gauge), _update(update), float(omega), float(T),
                              float(p_sr), int(seed), int(instance), int(sweep),
                              _ptr(G) if G is not None else None,
                              sites.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(sites))


def su2_local_g(fwd, bwd, gauge, update, omega=1.0, T=0.0, p_sr=0.5, seed=0, instance=0, sweep=0, site=0):
    """g(x) (2x2 complex as 8 reals) from ndir forward and backward links."""
    fwd = np.ascontiguousarray(fwd, dtype=np.float64)
    bwd = np.ascontiguousarray(bwd, dtype=np.float64)
    out = np.empty(8)
    _load().gfo2_local_g(_ptr(fwd), _ptr(bwd), fwd.size // 8, _gauge(gauge), _update(update), float(omega),
                         float(T), float(p_sr), int(seed), int(instance), int(sweep), int(site), _ptr(out))
    return out.reshape(2, 2, 2)


def su2_measure(U, dims, gauge):
    _check_links2(U, dims)
    F = ctypes.c_double()
    th = ctypes.c_double()
    _load().gfo2_measure(_ptr(U), _dims(dims), _gauge(gauge), ctypes.byref(F), ctypes.byref(th))
    return F.value, th.value


def su2_measure_slices(U, dims):
    _check_links2(U, dims)
    Nt = int(dims[0])
    F = np.empty(Nt)
    th = np.empty(Nt)
    _load().gfo2_measure_slices(_ptr(U), _dims(dims), _ptr(F), _ptr(th))
    return F, th


def su2_unitarity(U):
    U = np.ascontiguousarray(U)
    m = ctypes.c_double()
    x = ctypes.c_double()
    _load().gfo2_unitarity(_ptr(U), U.size // 8, ctypes.byref(m), ctypes.byref(x))
    return m.value, x.value


def su2_reunitarise(U):
    assert U.dtype == np.float64 and U.flags.c_contiguous
    _load().gfo2_reunitarise(_ptr(U), U.size // 8)


def su2_plaquette(U, dims):
    _check_links2(U, dims)
    return _load().gfo2_plaquette(_ptr(U), _dims(dims))


def su2_apply_gauge(U, dims, g):
    _check_links2(U, dims)
    _load().gfo2_apply_gauge(_ptr(U), _dims(dims), _ptr(np.ascontiguousarray(g, dtype=np.float64)))


def su2_coulomb_fix_u0(U, dims, G):
    _check_links2(U, dims)
    _load().gfo2_coulomb_fix_u0(_ptr(U), _dims(dims), _ptr(np.ascontiguousarray(G)))


def su2_run(U, dims, gauge, update="or", omega=1.7, max_sweeps=1000, tol=1e-12, check_every=1):
    """Sweeps until theta < tol at a check (Landau, MAG; Coulomb: every
    time-slice stops on its own and U_0 is fixed up at the end).  Returns
    (status, sweeps per unit)."""
    _check_links2(U, dims)
    if _gauge(gauge) != COULOMB:
        k = 0
        while True:
            if k % check_every == 0 and su2_measure(U, dims, gauge)[1] < tol:
                return 0, [k]
            if k >= max_sweeps:
                return 1, [k]
            su2_sweep(U, dims, gauge, update, omega=omega, sweep=k)
            k += 1
    Nt = int(dims[0])
    G = np.ascontiguousarray(np.broadcast_to(su2_identity_field(1), (_nsites(dims), 2, 2, 2)))
    active = np.ones(Nt, np.uint8)
    done = np.zeros(Nt, np.int64)
    k = 0
    while True:
        if k % check_every == 0:
            th = su2_measure_slices(U, dims)[1]
            active &= (th >= tol).astype(np.uint8)
        if not active.any() or k >= max_sweeps:
            break
        su2_sweep(U, dims, COULOMB, update, omega=omega, sweep=k, G=G, slice_active=active)
        done += active
        k += 1
    su2_coulomb_fix_u0(U, dims, G)
    return (0 if not active.any() else 1), list(done)


def su2_anneal(U, dims, gauge, T0, T1, nsteps, nmicro=3, seed=0, instance=0, sweep_counter=0, G=None):
    """The annealing schedule of ``anneal`` for SU(2) (reading R11: T linear
    from T0 to T1 over nsteps steps, one heatbath sweep then nmicro
    microcanonical sweeps per step, one random-counter step per sweep);
    returns the advanced sweep counter."""
    _check_links2(U, dims)
    ctr = int(sweep_counter)
    for k in range(int(nsteps)):
        T = T0 + (T1 - T0) * k / (nsteps - 1) if nsteps > 1 else T0
        su2_sweep(U, dims, gauge, HEATBATH, T=T, seed=seed, instance=instance, sweep=ctr, G=G)
        ctr += 1
        for _ in range(int(nmicro)):
            su2_sweep(U, dims, gauge, MICRO, seed=seed, instance=instance, sweep=ctr, G=G)
            ctr += 1
    return ctr
