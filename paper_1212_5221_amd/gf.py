"""Python binding of libgf (include/gf.h): argument marshalling only.

Every step of the gauge-fixing path runs in the HIP kernels of libgf.so;
PyTorch supplies the device workspace and the stream.  There is no CPU
fallback: importing this module without a built libgf.so raises.

    from paper_1212_5221_amd import gf
    fx = gf.GaugeFixer([(32, 32, 32, 32)], gauge="landau", storage="mixed")
    fx.upload(0, links)                       # natural layout, float64
    fx.set_overrelax(1.7)
    status, sweeps = fx.sweep("or", max_sweeps=20000, tol=1e-12, check_every=10)
    F, theta = fx.measure(0)
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgf.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "gf.h")

OK, NOT_CONVERGED = 0, 1
E_INVALID, E_DIMS, E_STATE, E_HIP, E_NOMEM, E_NONFINITE = -1, -2, -3, -4, -5, -6
LANDAU, COULOMB, MAG = 0, 1, 2
OR, MICRO, ANNEAL, SR, HEATBATH = 0, 1, 2, 3, 4
F64_R18, F64_R12, MIXED_F32_R12, F32_R12 = 0, 1, 2, 3
DL_REUNITARISE = 1
KERNELS_FP32, KERNELS_FP64, KERNELS_HEATBATH = 0, 1, 2
SHAPE_NONTEMPORAL, SHAPE_LINEAR_TILES = 1, 2
KERNEL_TABLES = {"fp32": KERNELS_FP32, "fp64": KERNELS_FP64, "heatbath": KERNELS_HEATBATH}

GAUGES = {"landau": LANDAU, "coulomb": COULOMB, "mag": MAG}
UPDATES = {"or": OR, "micro": MICRO, "anneal": ANNEAL, "sr": SR, "heatbath": HEATBATH}
STORAGES = {"f64r18": F64_R18, "f64r12": F64_R12, "mixed": MIXED_F32_R12, "f32r12": MIXED_F32_R12,
            "single": F32_R12}

_lib = None


class GFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("gf error %d: %s" % (code, msg))
        self.code = code


def load():
    """Load libgf.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libgf.so not built: run paper_1212_5221_amd.build.build() (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i32 = ctypes.c_int32
    i32p = ctypes.POINTER(ctypes.c_int32)
    dp = ctypes.POINTER(ctypes.c_double)
    u64 = ctypes.c_uint64
    ci = ctypes.c_int
    L.gf_create.argtypes = [ctypes.POINTER(vp), ci, vp]
    L.gf_destroy.argtypes = [vp]
    L.gf_destroy.restype = None
    L.gf_last_error.argtypes = [vp]
    L.gf_last_error.restype = ctypes.c_char_p
    L.gf_add_instance.argtypes = [vp, i32p, i32p]
    L.gf_set_gauge.argtypes = [vp, ci]
    L.gf_set_group.argtypes = [vp, ci]
    L.gf_set_precision.argtypes = [vp, ci, i32, ctypes.c_double]
    L.gf_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.gf_bind_workspace.argtypes = [vp, vp, ctypes.c_size_t]
    L.gf_upload.argtypes = [vp, i32, vp, i32, i32, ci]
    L.gf_download.argtypes = [vp, i32, vp, i32, i32, ci, ci]
    L.gf_set_overrelax.argtypes = [vp, ctypes.c_double]
    L.gf_set_stochastic.argtypes = [vp, ctypes.c_double]
    L.gf_set_seed.argtypes = [vp, u64]
    L.gf_set_temperature.argtypes = [vp, ctypes.c_double]
    L.gf_set_anneal.argtypes = [vp, ctypes.c_double, ctypes.c_double, i32, i32, u64]
    L.gf_sweep.argtypes = [vp, ci, i32, ctypes.c_double, i32, i32p]
    L.gf_halfsweep.argtypes = [vp, ci, ci]
    L.gf_measure.argtypes = [vp, i32, dp, dp]
    L.gf_measure_timeslices.argtypes = [vp, i32, dp, dp]
    L.gf_unitarity.argtypes = [vp, i32, dp, dp]
    L.gf_reunitarise.argtypes = [vp]
    L.gf_get_sweep_index.argtypes = [vp, i32, ctypes.POINTER(u64)]
    L.gf_set_sweep_index.argtypes = [vp, i32, u64]
    L.gf_set_launch.argtypes = [vp, ci, ci]
    L.gf_autotune.argtypes = [vp, ci, ctypes.POINTER(ci), ctypes.POINTER(ci)]
    L.gf_autotune_heatbath.argtypes = [vp, ci, ctypes.POINTER(ci), ctypes.POINTER(ci)]
    L.gf_set_shape.argtypes = [vp, ci, ci, ci, ci]
    L.gf_get_shape.argtypes = [vp, ci, ctypes.POINTER(ci), ctypes.POINTER(ci), ctypes.POINTER(ci)]
    L.gf_set_tune_cache.argtypes = [vp, ctypes.c_char_p]
    L.gf_set_timing.argtypes = [vp, ci]
    L.gf_kernel_time.argtypes = [vp, ci, ctypes.POINTER(ctypes.c_int64), dp]
    L.gf_set_graph.argtypes = [vp, ci]
    L.gf_set_cache_budget.argtypes = [vp, ctypes.c_int64]
    L.gf_measure_noalloc.argtypes = [ci, vp, ci, i32p, vp, vp]
    L.gf_stream.argtypes = [vp, ci, vp, vp, ctypes.c_size_t]
    L.gf_stream_blocks.argtypes = [ctypes.c_size_t, ctypes.POINTER(ctypes.c_int64)]
    L.gf_cache_groups.argtypes = [vp, i32p]
    _lib = L
    return L


def header_functions(path: str = HEADER):
    """Names of the functions include/gf.h declares."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gf_[a-z0-9_]+)\s*\(", txt)))


def _key(table, v):
    return table[v.lower()] if isinstance(v, str) else int(v)


def measure_noalloc(links, dims, gauge, out, device=0, stream=None):
    """gf_measure_noalloc: F and theta of an SU(3) field held on the device
    (float64 CUDA tensor, natural layout) into the CUDA tensor out[0:2],
    enqueued on `stream` (default: torch's current stream); allocates nothing
    on the device and does not wait."""
    import torch
    L = load()
    d = [int(x) for x in dims]
    assert links.is_cuda and links.dtype == torch.float64 and links.is_contiguous()
    assert links.numel() == int(np.prod(d)) * 4 * 18
    assert out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.numel() >= 2
    if stream is None:
        stream = torch.cuda.current_stream(int(device))
    rc = L.gf_measure_noalloc(int(device), ctypes.c_void_p(stream.cuda_stream), _key(GAUGES, gauge),
                              (ctypes.c_int32 * 4)(*d), ctypes.c_void_p(links.data_ptr()),
                              ctypes.c_void_p(out.data_ptr()))
    if rc != OK:
        msg = L.gf_last_error(None)
        raise GFError(rc, msg.decode() if msg else "")
    return out


STREAM_KINDS = {"copy": 0, "copy_nt_load": 1, "copy_nt_store": 2, "copy_nt": 3, "read": 4}


def stream(kind, dst, src, nbytes, stream=None):
    """gf_stream: one streaming pass (copy, or read) over nbytes of CUDA
    tensors, enqueued on `stream` (default: torch's current stream); a copy
    with dst the same tensor as src is an in-place pass."""
    import torch
    L = load()
    if stream is None:
        stream = torch.cuda.current_stream()
    rc = L.gf_stream(ctypes.c_void_p(stream.cuda_stream), STREAM_KINDS[kind], ctypes.c_void_p(dst.data_ptr()),
                     ctypes.c_void_p(src.data_ptr()), int(nbytes))
    if rc != OK:
        raise GFError(rc, "gf_stream failed")


def stream_blocks(nbytes):
    n = ctypes.c_int64()
    if load().gf_stream_blocks(int(nbytes), ctypes.byref(n)) != OK:
        raise GFError(E_INVALID, "gf_stream_blocks: bytes must be a multiple of 16")
    return n.value


class GaugeFixer:
    """One libgf handle with its instances and the torch-owned workspace."""

    def __init__(self, dims_list, gauge="landau", storage="f64r18", reunit_every=0, tail_theta=0.0, device=0,
                 stream=None, group=3):
        """group: 3 for SU(3) (links (sites, 4, 3, 3, 2)) or 2 for SU(2)
        (links (sites, 4, 2, 2, 2))."""
        import torch

        self._torch = torch
        self.lib = load()
        self.device = int(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self._h = ctypes.c_void_p()
        self._check(self.lib.gf_create(ctypes.byref(self._h), self.device, ctypes.c_void_p(stream.cuda_stream)),
                    create=True)
        self.dims = []
        try:
            for d in dims_list:
                d = [int(x) for x in d]
                arr = (ctypes.c_int32 * 4)(*d)
                inst = ctypes.c_int32()
                self._check(self.lib.gf_add_instance(self._h, arr, ctypes.byref(inst)))
                self.dims.append(tuple(d))
            self.gauge = _key(GAUGES, gauge)
            self.storage = _key(STORAGES, storage)
            self.nc = int(group)
            self._check(self.lib.gf_set_group(self._h, self.nc))
            self._check(self.lib.gf_set_gauge(self._h, self.gauge))
            self._check(self.lib.gf_set_precision(self._h, self.storage, int(reunit_every), float(tail_theta)))
            nbytes = ctypes.c_size_t()
            self._check(self.lib.gf_workspace_size(self._h, ctypes.byref(nbytes)))
            self.workspace_bytes = nbytes.value
            self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda:%d" % self.device)
            ptr = self.workspace.data_ptr()
            ptr = (ptr + 255) & ~255
            self._check(self.lib.gf_bind_workspace(self._h, ctypes.c_void_p(ptr), nbytes.value))
        except Exception:
            self.close()
            raise

    # ------------------------------------------------------------ plumbing
    def _check(self, rc, create=False, allow=(OK,)):
        if rc in allow:
            return rc
        if rc > 0:
            return rc
        msg = self.lib.gf_last_error(None if create else self._h)
        raise GFError(rc, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self.lib.gf_destroy(self._h)
            self._h = ctypes.c_void_p()
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def nunits(self):
        return sum(d[0] for d in self.dims) if self.gauge == COULOMB else len(self.dims)

    def _vs(self, inst):
        d = self.dims[inst]
        return d[1] * d[2] * d[3]

    @property
    def link_shape(self):
        """Shape of one link in the natural layout: (nc, nc, 2)."""
        return (self.nc, self.nc, 2)

    @property
    def _site_reals(self):
        return 8 * self.nc * self.nc

    # ------------------------------------------------------------ data
    def upload(self, inst, links, t0=0, nt=None):
        """Links of time-slices [t0, t0+nt): numpy float64 (host) or a CUDA tensor."""
        d = self.dims[inst]
        nt = d[0] - t0 if nt is None else nt
        n = nt * self._vs(inst) * self._site_reals
        torch = self._torch
        if isinstance(links, torch.Tensor):
            assert links.dtype == torch.float64 and links.is_contiguous() and links.numel() == n
            on_dev = 1 if links.is_cuda else 0
            ptr = links.data_ptr()
            keep = links
        else:
            keep = np.ascontiguousarray(links, dtype=np.float64)
            assert keep.size == n, "expected %d reals" % n
            on_dev = 0
            ptr = keep.ctypes.data
        self._check(self.lib.gf_upload(self._h, inst, ctypes.c_void_p(ptr), t0, nt, on_dev))
        del keep

    def download(self, inst, t0=0, nt=None, reunitarise=False, out=None):
        """Links of time-slices [t0, t0+nt) as numpy float64 (sites, 4, nc, nc, 2)."""
        d = self.dims[inst]
        nt = d[0] - t0 if nt is None else nt
        ns = nt * self._vs(inst)
        flags = DL_REUNITARISE if reunitarise else 0
        torch = self._torch
        if out is not None and isinstance(out, torch.Tensor) and out.is_cuda:
            assert out.dtype == torch.float64 and out.is_contiguous() and out.numel() == ns * self._site_reals
            self._check(self.lib.gf_download(self._h, inst, ctypes.c_void_p(out.data_ptr()), t0, nt, 1, flags))
            return out
        if out is None:
            out = np.empty((ns, 4) + self.link_shape, dtype=np.float64)
        assert out.dtype == np.float64 and out.flags.c_contiguous and out.size == ns * self._site_reals
        self._check(self.lib.gf_download(self._h, inst, ctypes.c_void_p(out.ctypes.data), t0, nt, 0, flags))
        return out

    # ------------------------------------------------------------ parameters
    def set_overrelax(self, omega):
        self._check(self.lib.gf_set_overrelax(self._h, float(omega)))

    def set_stochastic(self, p):
        self._check(self.lib.gf_set_stochastic(self._h, float(p)))

    def set_seed(self, seed):
        self._check(self.lib.gf_set_seed(self._h, int(seed)))

    def set_temperature(self, T):
        self._check(self.lib.gf_set_temperature(self._h, float(T)))

    def set_anneal(self, T0, T1, nsteps, nmicro=3, seed=0):
        self._check(self.lib.gf_set_anneal(self._h, float(T0), float(T1), int(nsteps), int(nmicro), int(seed)))

    def get_sweep_index(self, inst):
        v = ctypes.c_uint64()
        self._check(self.lib.gf_get_sweep_index(self._h, inst, ctypes.byref(v)))
        return v.value

    def set_sweep_index(self, inst, index):
        self._check(self.lib.gf_set_sweep_index(self._h, inst, int(index)))

    def set_launch(self, waves_per_site=0, block=0):
        self._check(self.lib.gf_set_launch(self._h, int(waves_per_site), int(block)))

    def set_shape(self, kernels, waves_per_site, block, flags=0):
        """launch shape of one kernel table ("fp32", "fp64", "heatbath")"""
        self._check(self.lib.gf_set_shape(self._h, _key(KERNEL_TABLES, kernels), int(waves_per_site), int(block),
                                          int(flags)))

    def get_shape(self, kernels):
        """(waves_per_site, block, flags) of one kernel table"""
        w, b, f = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.gf_get_shape(self._h, _key(KERNEL_TABLES, kernels), ctypes.byref(w), ctypes.byref(b),
                                          ctypes.byref(f)))
        return w.value, b.value, f.value

    def autotune(self, reps=3):
        """tune the OR kernel tables in use; returns (waves_per_site, block)"""
        w = ctypes.c_int()
        b = ctypes.c_int()
        self._check(self.lib.gf_autotune(self._h, int(reps), ctypes.byref(w), ctypes.byref(b)))
        return w.value, b.value

    def autotune_heatbath(self, reps=3):
        """tune the heatbath kernel table; returns (waves_per_site, block)"""
        w = ctypes.c_int()
        b = ctypes.c_int()
        self._check(self.lib.gf_autotune_heatbath(self._h, int(reps), ctypes.byref(w), ctypes.byref(b)))
        return w.value, b.value

    def set_tune_cache(self, path):
        """file of persisted autotuning choices (None: off)"""
        self._check(self.lib.gf_set_tune_cache(self._h, None if path is None else str(path).encode()))

    def set_timing(self, enable=True, every=1):
        """time every `every`-th half-sweep launch with HIP events (enable=False: off)"""
        self._check(self.lib.gf_set_timing(self._h, int(every) if enable else 0))

    def kernel_time(self, which="all"):
        """(launches, mean ms) of the timed half-sweeps: which = all | fp32 | fp64 update"""
        w = {"all": 0, "fp32": 1, "fp64": 2}[which]
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        self._check(self.lib.gf_kernel_time(self._h, w, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def set_cache_budget(self, nbytes):
        """Infinity-Cache grouping of independent units inside sweep(); 0 turns it off"""
        self._check(self.lib.gf_set_cache_budget(self._h, ctypes.c_int64(int(nbytes))))

    def cache_groups(self):
        g = ctypes.c_int32()
        self._check(self.lib.gf_cache_groups(self._h, ctypes.byref(g)))
        return g.value

    def set_graph(self, enable=True):
        self._check(self.lib.gf_set_graph(self._h, 1 if enable else 0))

    # ------------------------------------------------------------ work
    def sweep(self, update="or", max_sweeps=1000, tol=1e-12, check_every=1):
        """Run Alg. 1; returns (status, sweeps per unit)."""
        done = np.zeros(self.nunits, dtype=np.int32)
        rc = self.lib.gf_sweep(self._h, _key(UPDATES, update), int(max_sweeps), float(tol), int(check_every),
                               done.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        self._check(rc, allow=(OK, NOT_CONVERGED))
        return rc, done

    def halfsweep(self, update="or", parity=0):
        self._check(self.lib.gf_halfsweep(self._h, _key(UPDATES, update), int(parity)))

    def measure(self, inst=0):
        F = ctypes.c_double()
        th = ctypes.c_double()
        self._check(self.lib.gf_measure(self._h, inst, ctypes.byref(F), ctypes.byref(th)))
        return F.value, th.value

    def measure_timeslices(self, inst=0):
        nt = self.dims[inst][0]
        F = np.zeros(nt)
        th = np.zeros(nt)
        dp = ctypes.POINTER(ctypes.c_double)
        self._check(self.lib.gf_measure_timeslices(self._h, inst, F.ctypes.data_as(dp), th.ctypes.data_as(dp)))
        return F, th

    def unitarity(self, inst=0):
        m = ctypes.c_double()
        x = ctypes.c_double()
        self._check(self.lib.gf_unitarity(self._h, inst, ctypes.byref(m), ctypes.byref(x)))
        return m.value, x.value

    def reunitarise(self):
        self._check(self.lib.gf_reunitarise(self._h))

    def synchronize(self):
        self._torch.cuda.synchronize(self.device)
