"""Thin Python binding of libmts (include/mts.h): argument marshalling only.

Every step of the lattice update and of the diagnostics runs in the HIP
kernels of libmts.so; PyTorch only allocates the device state buffer and
supplies the stream.  The library must have been built
(``python -m paper_2208_01525_amd.build`` or ``__graft_entry__.build()``);
loading fails loudly otherwise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MTS_LIBRARY names another build of the same library (the sanitizer test
# loads a host-sanitized build this way)
LIB_PATH = os.environ.get("MTS_LIBRARY") or os.path.join(_HERE, "libmts.so")

MTS_OK, MTS_EINVAL, MTS_EUNSTABLE, MTS_ENOMEM, MTS_EHIP, MTS_ENONFINITE = 0, -1, -2, -3, -4, -5
MTS_FP32, MTS_FP64 = 1, 2
NOALLOC_MAX_SITES = 8192        # MTS_NOALLOC_MAX_SITES of include/mts.h

EXPORTS = ("mts_state_bytes", "mts_create", "mts_destroy", "mts_init_fields", "mts_step", "mts_cool", "mts_diagnostics",
           "mts_get_fields", "mts_set_fields", "mts_get_windings", "mts_get_cells", "mts_get_sites", "mts_get_sites_noalloc", "mts_segments", "mts_set_tile", "mts_get_tile", "mts_set_streaming_stores", "mts_bandwidth_probe", "mts_get_streaming_stores", "mts_autotune", "mts_autotune_cached", "mts_timing_enable",
           "mts_timing_read", "mts_set_time_blocking", "mts_get_time_blocking", "mts_set_prefetch", "mts_get_prefetch", "mts_set_fused_diagnostics", "mts_get_fused_diagnostics", "mts_set_momentum_pingpong", "mts_get_momentum_pingpong", "mts_set_tile_order", "mts_get_tile_order", "mts_last_error", "mts_strerror",
           "mts_batch_state_bytes", "mts_batch_create", "mts_batch_destroy", "mts_batch_size",
           "mts_batch_init_fields", "mts_batch_step", "mts_batch_diagnostics", "mts_batch_get_fields",
           "mts_batch_set_fields", "mts_batch_set_tile", "mts_batch_set_streaming_stores", "mts_batch_get_streaming_stores", "mts_batch_set_momentum_pingpong",
           "mts_batch_get_momentum_pingpong", "mts_batch_set_fused_diagnostics", "mts_batch_get_fused_diagnostics", "mts_batch_set_tile_order", "mts_batch_get_tile_order", "mts_batch_timing_read", "mts_batch_autotune",
           "mts_batch_set_persistent", "mts_batch_get_persistent", "mts_batch_autotune_times", "mts_batch_last_error")


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dt", ctypes.c_double),
        ("lambda_p", ctypes.c_double), ("lambda_q", ctypes.c_double),
        ("e_p", ctypes.c_double), ("e_q", ctypes.c_double),
        ("sigma_p", ctypes.c_double), ("sigma_q", ctypes.c_double),
        ("kappa", ctypes.c_double), ("eta_ref", ctypes.c_double),
        ("diag_every", ctypes.c_int32), ("overlap_radius", ctypes.c_int32),
    ]


class Diag(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("eta", ctypes.c_double), ("a", ctypes.c_double), ("s", ctypes.c_double),
        ("sum_energy", ctypes.c_double), ("sum_lagrangian", ctypes.c_double),
        ("sum_KL", ctypes.c_double), ("sum_GL", ctypes.c_double),
        ("sum_KV", ctypes.c_double), ("sum_GV", ctypes.c_double),
        ("gauss_abs", ctypes.c_double * 2), ("gauss_scale", ctypes.c_double * 2),
        ("wind_abs", ctypes.c_int64 * 2), ("pq_count2", ctypes.c_int64),
        ("L_p", ctypes.c_double), ("L_q", ctypes.c_double), ("L_pq", ctypes.c_double),
        ("xi_p", ctypes.c_double), ("xi_q", ctypes.c_double), ("xi_pq", ctypes.c_double), ("xi_W", ctypes.c_double),
        ("xi_lag", ctypes.c_double), ("f_total", ctypes.c_double), ("f_p", ctypes.c_double),
        ("v2_lag", ctypes.c_double), ("v2_pq", ctypes.c_double), ("gauss_rel", ctypes.c_double * 2),
        ("flags", ctypes.c_int32), ("pad", ctypes.c_int32),
    ]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            if name == "pad":
                continue
            v = getattr(self, name)
            out[name] = tuple(v) if isinstance(v, ctypes.Array) else v
        return out


class Segments(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("marked_cells", ctypes.c_int64), ("regions", ctypes.c_int64),
                ("n_pq", ctypes.c_int64), ("largest", ctypes.c_int64), ("L_pq", ctypes.c_double),
                ("l_pq", ctypes.c_double), ("xi_pq", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class MtsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_strerror(code)}: {msg}")
        self.code = code


_LIB = None


def load():
    """Load libmts.so (no fallback: the HIP library is the implementation)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2208_01525_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, pp = ctypes.c_void_p, ctypes.POINTER(Params)
    L.mts_state_bytes.argtypes = [pp]
    L.mts_state_bytes.restype = ctypes.c_size_t
    L.mts_create.argtypes = [pp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.mts_destroy.argtypes = [vp]
    L.mts_init_fields.argtypes = [vp, ctypes.c_uint64]
    L.mts_step.argtypes = [vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    L.mts_cool.argtypes = [vp, ctypes.c_int32, ctypes.c_double]
    L.mts_diagnostics.argtypes = [vp, ctypes.POINTER(Diag), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.mts_get_fields.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.mts_set_fields.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.mts_get_windings.argtypes = [vp, ctypes.POINTER(ctypes.c_int8)]
    L.mts_get_cells.argtypes = [vp, ctypes.POINTER(ctypes.c_uint8)]
    L.mts_segments.argtypes = [vp, ctypes.c_double, ctypes.POINTER(Segments), ctypes.POINTER(ctypes.c_int64),
                               ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    L.mts_get_sites.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
    L.mts_get_sites_noalloc.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_double)]
    L.mts_set_tile.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    L.mts_set_streaming_stores.argtypes = [vp, ctypes.c_int32]
    L.mts_bandwidth_probe.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]
    L.mts_batch_set_streaming_stores.argtypes = [vp, ctypes.c_int32]
    L.mts_get_streaming_stores.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.mts_batch_get_streaming_stores.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.mts_batch_set_momentum_pingpong.argtypes = [vp, ctypes.c_int32]
    L.mts_batch_get_momentum_pingpong.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.mts_batch_set_fused_diagnostics.argtypes = [vp, ctypes.c_int32]
    L.mts_batch_get_fused_diagnostics.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.mts_batch_set_tile_order.argtypes = [vp, ctypes.c_int32]
    L.mts_batch_get_tile_order.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.mts_batch_set_persistent.argtypes = [vp, ctypes.c_int32, ctypes.c_double]
    L.mts_batch_get_persistent.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.mts_batch_autotune_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.mts_get_tile.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    i32p = ctypes.POINTER(ctypes.c_int32)
    L.mts_autotune.argtypes = [vp, ctypes.c_int32, i32p, i32p, ctypes.POINTER(ctypes.c_double)]
    L.mts_autotune_cached.argtypes = [vp, ctypes.c_int32, ctypes.c_char_p, i32p, i32p, i32p,
                                      ctypes.POINTER(ctypes.c_double)]
    L.mts_batch_autotune.argtypes = [vp, ctypes.c_int32, i32p, i32p, ctypes.POINTER(ctypes.c_double)]
    L.mts_timing_enable.argtypes = [vp, ctypes.c_int32]
    i64p, dp = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)
    L.mts_timing_read.argtypes = [vp, i64p, dp, i64p, dp, dp, i64p, dp]
    L.mts_set_time_blocking.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.mts_get_time_blocking.argtypes = [vp, i32p, i32p, i32p]
    L.mts_set_prefetch.argtypes = [vp, ctypes.c_int32]
    L.mts_set_fused_diagnostics.argtypes = [vp, ctypes.c_int32]
    L.mts_get_fused_diagnostics.argtypes = [vp, i32p]
    L.mts_set_momentum_pingpong.argtypes = [vp, ctypes.c_int32]
    L.mts_get_momentum_pingpong.argtypes = [vp, i32p]
    L.mts_set_tile_order.argtypes = [vp, ctypes.c_int32]
    L.mts_get_tile_order.argtypes = [vp, i32p]
    L.mts_get_prefetch.argtypes = [vp, i32p]
    L.mts_last_error.argtypes = [vp]
    L.mts_last_error.restype = ctypes.c_char_p
    L.mts_strerror.argtypes = [ctypes.c_int]
    L.mts_strerror.restype = ctypes.c_char_p
    dpp = ctypes.POINTER(ctypes.c_double)
    L.mts_batch_state_bytes.argtypes = [pp, ctypes.c_int32]
    L.mts_batch_state_bytes.restype = ctypes.c_size_t
    L.mts_batch_create.argtypes = [pp, ctypes.c_int32, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.mts_batch_destroy.argtypes = [vp]
    L.mts_batch_size.argtypes = [vp]
    L.mts_batch_size.restype = ctypes.c_int32
    L.mts_batch_init_fields.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
    L.mts_batch_step.argtypes = [vp, ctypes.c_int32, dpp, dpp, dpp, dpp, dpp]
    L.mts_batch_diagnostics.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(Diag), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32)]
    L.mts_batch_get_fields.argtypes = [vp, ctypes.c_int32, dpp]
    L.mts_batch_set_fields.argtypes = [vp, ctypes.c_int32, dpp]
    L.mts_batch_set_tile.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.mts_batch_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), dpp]
    L.mts_batch_last_error.argtypes = [vp]
    L.mts_batch_last_error.restype = ctypes.c_char_p
    _LIB = L
    return L


def _strerror(code):
    try:
        return load().mts_strerror(code).decode()
    except Exception:
        return str(code)


def make_params(nx, ny=None, nz=None, *, precision="fp32", dx=0.5, dt=0.1, lam=(2.0, 2.0), e=(1.0, 1.0),
                sig=(1.0, 1.0), kappa=0.9, eta_ref=1.0, diag_every=0, overlap_radius=1):
    p = Params()
    p.nx = nx
    p.ny = nx if ny is None else ny
    p.nz = nx if nz is None else nz
    p.precision = {"fp32": MTS_FP32, "fp64": MTS_FP64}[precision]
    p.dx, p.dt = dx, dt
    p.lambda_p, p.lambda_q = lam
    p.e_p, p.e_q = e
    p.sigma_p, p.sigma_q = sig
    p.kappa, p.eta_ref = kappa, eta_ref
    p.diag_every, p.overlap_radius = diag_every, overlap_radius
    return p


def state_bytes(params):
    return load().mts_state_bytes(ctypes.byref(params))


class Lattice:
    """One periodic box on one GPU.  The device state buffer is a torch uint8
    tensor of mts_state_bytes() bytes; all work goes to `stream` (default: the
    current torch stream of `device`)."""

    def __init__(self, params, device="cuda:0", stream=None):
        import torch

        self.L = load()
        self.params = params
        self.device = torch.device(device)
        self.shape = (params.nz, params.ny, params.nx)
        self.sites = params.nx * params.ny * params.nz
        nbytes = state_bytes(params)
        if nbytes == 0:
            raise MtsError(MTS_EINVAL, "invalid parameters")
        self.state = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        rc = self.L.mts_create(ctypes.byref(params), ctypes.c_void_p(self.state.data_ptr()), nbytes,
                               ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        if rc != MTS_OK:
            raise MtsError(rc, "mts_create failed")
        self.ctx = ctx

    def _check(self, rc):
        if rc != MTS_OK:
            raise MtsError(rc, self.L.mts_last_error(self.ctx).decode())

    def close(self):
        if getattr(self, "ctx", None):
            self.L.mts_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the C ABI, name for name --
    def init_fields(self, seed):
        self._check(self.L.mts_init_fields(self.ctx, ctypes.c_uint64(seed)))

    def step(self, n, eta, era_m, s):
        self._check(self.L.mts_step(self.ctx, int(n), float(eta), float(era_m), float(s)))

    def cool(self, n, dt_cool=1.0 / 30.0):
        self._check(self.L.mts_cool(self.ctx, int(n), float(dt_cool)))

    def diagnostics(self, max_records=8192, allow_nonfinite=False):
        buf = (Diag * max_records)()
        cnt = ctypes.c_int32()
        rc = self.L.mts_diagnostics(self.ctx, buf, max_records, ctypes.byref(cnt))
        if rc == MTS_ENONFINITE and allow_nonfinite:
            rc = MTS_OK
        self._check(rc)
        return [buf[i].as_dict() for i in range(cnt.value)]

    def get_fields(self):
        out = np.empty((20,) + self.shape, dtype=np.float64)
        self._check(self.L.mts_get_fields(self.ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def set_fields(self, host):
        host = np.ascontiguousarray(host, dtype=np.float64)
        assert host.shape == (20,) + self.shape
        self._check(self.L.mts_set_fields(self.ctx, host.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def get_sites(self, sites):
        sites = np.ascontiguousarray(sites, dtype=np.uint64)
        out = np.empty((len(sites), 20), dtype=np.float64)
        self._check(self.L.mts_get_sites(self.ctx, sites.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), len(sites),
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def get_sites_noalloc(self, sites):
        """get_sites staged through the library's static device scratch (no device
        allocation; at most NOALLOC_MAX_SITES sites)."""
        sites = np.ascontiguousarray(sites, dtype=np.uint64)
        out = np.empty((len(sites), 20), dtype=np.float64)
        self._check(self.L.mts_get_sites_noalloc(self.ctx, sites.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                                 len(sites), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def segments(self, min_length=0.0, max_sizes=1 << 20):
        """Robust-method segments of the last diagnostic step: (summary dict, sizes)."""
        out = Segments()
        sizes = np.zeros(max_sizes, dtype=np.int64)
        n = ctypes.c_int64()
        self._check(self.L.mts_segments(self.ctx, float(min_length), ctypes.byref(out),
                                        sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), max_sizes,
                                        ctypes.byref(n)))
        return out.as_dict(), sizes[:min(n.value, max_sizes)]

    def get_windings(self):
        out = np.empty((6,) + self.shape, dtype=np.int8)
        self._check(self.L.mts_get_windings(self.ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))))
        return out

    def get_cells(self):
        out = np.empty((2,) + self.shape, dtype=np.uint8)
        self._check(self.L.mts_get_cells(self.ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
        return out

    def set_tile(self, ty, tz):
        self._check(self.L.mts_set_tile(self.ctx, int(ty), int(tz)))

    def set_streaming_stores(self, on):
        self._check(self.L.mts_set_streaming_stores(self.ctx, 1 if on else 0))

    def bandwidth_probe(self, reps=5):
        """GB/s of a plain copy and of the update's access pattern on this machine (overwrites
        the lattice)."""
        cp, pt = ctypes.c_double(), ctypes.c_double()
        self._check(self.L.mts_bandwidth_probe(self.ctx, int(reps), ctypes.byref(cp), ctypes.byref(pt)))
        return {"copy_GBps": cp.value, "pattern_GBps": pt.value}

    def get_streaming_stores(self):
        v = ctypes.c_int32()
        self._check(self.L.mts_get_streaming_stores(self.ctx, ctypes.byref(v)))
        return bool(v.value)

    def get_tile(self):
        ty, tz = ctypes.c_int32(), ctypes.c_int32()
        self._check(self.L.mts_get_tile(self.ctx, ctypes.byref(ty), ctypes.byref(tz)))
        return ty.value, tz.value

    def autotune(self, steps=5, cache=None):
        """(ty, tz, ms per step); with `cache` (a file path) through mts_autotune_cached, whose
        hit flag is then in `self.autotune_hit`."""
        ty, tz, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        if cache is None:
            self._check(self.L.mts_autotune(self.ctx, int(steps), ctypes.byref(ty), ctypes.byref(tz), ctypes.byref(ms)))
        else:
            hit = ctypes.c_int32()
            self._check(self.L.mts_autotune_cached(self.ctx, int(steps), str(cache).encode(), ctypes.byref(hit),
                                                   ctypes.byref(ty), ctypes.byref(tz), ctypes.byref(ms)))
            self.autotune_hit = hit.value
        return ty.value, tz.value, ms.value

    def timing_enable(self, on=True):
        self._check(self.L.mts_timing_enable(self.ctx, 1 if on else 0))

    def timing_read(self):
        n0, n1, n2 = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        t0, t1, t2, t3 = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(self.L.mts_timing_read(self.ctx, ctypes.byref(n0), ctypes.byref(t0), ctypes.byref(n1),
                                           ctypes.byref(t1), ctypes.byref(t2), ctypes.byref(n2), ctypes.byref(t3)))
        return {"n_plain": n0.value, "ms_plain": t0.value, "n_diag": n1.value, "ms_diag": t1.value,
                "ms_post": t2.value, "n_pair": n2.value, "ms_pair": t3.value}

    def set_time_blocking(self, steps, ty=7, tz=32):
        self._check(self.L.mts_set_time_blocking(self.ctx, int(steps), int(ty), int(tz)))

    def set_momentum_pingpong(self, on):
        self._check(self.L.mts_set_momentum_pingpong(self.ctx, 1 if on else 0))

    def get_momentum_pingpong(self):
        v = ctypes.c_int32()
        self._check(self.L.mts_get_momentum_pingpong(self.ctx, ctypes.byref(v)))
        return bool(v.value)

    def set_tile_order(self, xcd_runs):
        self._check(self.L.mts_set_tile_order(self.ctx, 1 if xcd_runs else 0))

    def get_tile_order(self):
        v = ctypes.c_int32()
        self._check(self.L.mts_get_tile_order(self.ctx, ctypes.byref(v)))
        return bool(v.value)

    def set_prefetch(self, on):
        self._check(self.L.mts_set_prefetch(self.ctx, 1 if on else 0))

    def get_prefetch(self):
        v = ctypes.c_int32()
        self._check(self.L.mts_get_prefetch(self.ctx, ctypes.byref(v)))
        return bool(v.value)

    def set_fused_diagnostics(self, rows):
        """Rows of the fused diagnostic tile (4, 5 or 8), or 0 for the post-step kernels."""
        self._check(self.L.mts_set_fused_diagnostics(self.ctx, int(rows)))

    def get_fused_diagnostics(self):
        v = ctypes.c_int32()
        self._check(self.L.mts_get_fused_diagnostics(self.ctx, ctypes.byref(v)))
        return v.value

    def get_time_blocking(self):
        n, ty, tz = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self.L.mts_get_time_blocking(self.ctx, ctypes.byref(n), ctypes.byref(ty), ctypes.byref(tz)))
        return n.value, ty.value, tz.value


def _darr(values, n):
    if values is None:
        return None
    v = [float(x) for x in (values if hasattr(values, "__len__") else [values] * n)]
    assert len(v) == n
    return (ctypes.c_double * n)(*v)


class Batch:
    """An ensemble of independent boxes advanced together (one update launch per
    step over all boxes, each n-step call captured into one HIP graph)."""

    def __init__(self, params_list, device="cuda:0", stream=None):
        import torch

        self.L = load()
        self.n = len(params_list)
        arr = (Params * self.n)(*params_list)
        self.params = list(params_list)
        nbytes = self.L.mts_batch_state_bytes(arr, self.n)
        if nbytes == 0:
            raise MtsError(MTS_EINVAL, "invalid box parameters")
        self.device = torch.device(device)
        self.pool = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        b = ctypes.c_void_p()
        rc = self.L.mts_batch_create(arr, self.n, ctypes.c_void_p(self.pool.data_ptr()), nbytes,
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(b))
        if rc != MTS_OK:
            raise MtsError(rc, "mts_batch_create failed")
        self.b = b

    def _check(self, rc):
        if rc != MTS_OK:
            raise MtsError(rc, self.L.mts_batch_last_error(self.b).decode())

    def close(self):
        if getattr(self, "b", None):
            self.L.mts_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_fields(self, seeds):
        arr = (ctypes.c_uint64 * self.n)(*[int(s) for s in seeds])
        self._check(self.L.mts_batch_init_fields(self.b, arr))

    def step(self, n, eta0, era_m, s_before, s_after=None, eta_switch=None):
        self._check(self.L.mts_batch_step(self.b, int(n), _darr(eta0, self.n), _darr(era_m, self.n),
                                          _darr(s_before, self.n), _darr(s_after, self.n),
                                          _darr(eta_switch, self.n)))

    def diagnostics(self, box, max_records=8192):
        buf = (Diag * max_records)()
        cnt = ctypes.c_int32()
        self._check(self.L.mts_batch_diagnostics(self.b, int(box), buf, max_records, ctypes.byref(cnt)))
        return [buf[i].as_dict() for i in range(cnt.value)]

    def get_fields(self, box):
        p = self.params[box]
        out = np.empty((20, p.nz, p.ny, p.nx), dtype=np.float64)
        self._check(self.L.mts_batch_get_fields(self.b, int(box), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def set_fields(self, box, host):
        host = np.ascontiguousarray(host, dtype=np.float64)
        self._check(self.L.mts_batch_set_fields(self.b, int(box), host.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def set_tile(self, ty, tz):
        tzs = tz if hasattr(tz, "__len__") else [tz] * self.n
        self._check(self.L.mts_batch_set_tile(self.b, int(ty), (ctypes.c_int32 * self.n)(*[int(v) for v in tzs])))

    def autotune(self, steps=3):
        ty, tz, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        self._check(self.L.mts_batch_autotune(self.b, int(steps), ctypes.byref(ty), ctypes.byref(tz),
                                              ctypes.byref(ms)))
        return ty.value, tz.value, ms.value

    def set_streaming_stores(self, on):
        self._check(self.L.mts_batch_set_streaming_stores(self.b, 1 if on else 0))

    def get_streaming_stores(self):
        v = ctypes.c_int32()
        self._check(self.L.mts_batch_get_streaming_stores(self.b, ctypes.byref(v)))
        return bool(v.value)

    def set_momentum_pingpong(self, on):
        self._check(self.L.mts_batch_set_momentum_pingpong(self.b, 1 if on else 0))

    def set_fused_diagnostics(self, rows):
        """8: fused diagnostic steps with batched post-step launches; 0: box by box."""
        self._check(self.L.mts_batch_set_fused_diagnostics(self.b, int(rows)))

    def get_fused_diagnostics(self):
        v = ctypes.c_int32()
        self._check(self.L.mts_batch_get_fused_diagnostics(self.b, ctypes.byref(v)))
        return v.value

    def set_tile_order(self, xcd_runs):
        self._check(self.L.mts_batch_set_tile_order(self.b, 1 if xcd_runs else 0))

    def get_tile_order(self):
        v = ctypes.c_int32()
        self._check(self.L.mts_batch_get_tile_order(self.b, ctypes.byref(v)))
        return bool(v.value)

    def get_momentum_pingpong(self):
        v = ctypes.c_int32()
        self._check(self.L.mts_batch_get_momentum_pingpong(self.b, ctypes.byref(v)))
        return bool(v.value)

    def set_persistent(self, on, wait_limit_s=0.0):
        """Runs of plain steps as one persistent launch (a grid barrier per step); wait_limit_s
        bounds each barrier wait (0: 10 s)."""
        self._check(self.L.mts_batch_set_persistent(self.b, 1 if on else 0, float(wait_limit_s)))

    def get_persistent(self):
        v = ctypes.c_int32()
        self._check(self.L.mts_batch_get_persistent(self.b, ctypes.byref(v)))
        return bool(v.value)

    def autotune_times(self):
        """Per-step ms of the per-step graph and of the persistent launch, as the last autotune timed them."""
        g, p = ctypes.c_double(), ctypes.c_double()
        self._check(self.L.mts_batch_autotune_times(self.b, ctypes.byref(g), ctypes.byref(p)))
        return {"graph_ms": g.value, "persistent_ms": p.value}

    def timing_read(self):
        st, ms = ctypes.c_int64(), ctypes.c_double()
        self._check(self.L.mts_batch_timing_read(self.b, ctypes.byref(st), ctypes.byref(ms)))
        return {"steps": st.value, "ms": ms.value}
