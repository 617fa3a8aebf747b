"""Python binding of the ripk C ABI (``include/ripk.h``) -- argument marshalling only.

Every step of the computation runs in ``libripk.so`` (HIP kernels for gfx950).
This module converts arguments and results: numpy arrays are passed as host
buffers, torch CUDA tensors as device pointers ordered on the caller's current
torch stream (torch serves only as the device allocator and stream source).
Function names follow the C ABI.  There is no fallback: if the library is not
built, every call raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# RIPK_LIB names another build of the same library (the host-sanitizer build
# of the CPU tests)
LIB_PATH = os.environ.get("RIPK_LIB") or os.path.join(HERE, "libripk.so")

RIPK_OK = 0
RIPK_PENDING = 1
RIPK_EINVAL = -1
RIPK_ERANGE = -2
RIPK_ENOMEM = -3
RIPK_EDEVICE = -4
RIPK_E2BIG = -5
RIPK_EAGAIN = -6
RIPK_EOVERFLOW = -7
RIPK_ECANCELED = -8
RIPK_ENOTFOUND = -9

RIPK_EDGE_SPATIAL_ISO = 1
RIPK_EDGE_TEMPORAL = 2
RIPK_EDGE_ISO = 3
RIPK_NORM_NN1 = 0
RIPK_NORM_N2 = 1
RIPK_SIM_CSR = 0
RIPK_SIM_PERMUTE = 1
RIPK_SIM_BOOTSTRAP = 2
RIPK_PLAN_ORDERED = 1
RIPK_PLAN_TIMING = 2
RIPK_PLAN_WIDE_COUNTS = 4
RIPK_PLAN_AUTOTUNE = 8
RIPK_PLAN_GRAPH = 16
RIPK_PLAN_CROSS = 32
RIPK_PLAN_INHOM = 64
RIPK_PLAN_SPLIT_RUNS = 128
RIPK_PLAN_COST_ORDER = 256
RIPK_REQ_KEEP_SIMS = 1

_i64, _i32, _u32, _u64, _f64 = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                                ctypes.c_uint64, ctypes.c_double)
_P = ctypes.POINTER


class PlanDesc(ctypes.Structure):
    _fields_ = [("x0", _i64), ("y0", _i64), ("x1", _i64), ("y1", _i64),
                ("t0", _i64), ("t1", _i64), ("s_max", _i64), ("t_max", _i64),
                ("n_s", _i32), ("n_t", _i32), ("edge", _u32), ("norm", _u32),
                ("sim_method", _u32), ("n_max", _i64), ("m_max", _i32), ("flags", _u32),
                ("device", _i32), ("cell_div", _i32), ("tcell_div", _i32),
                ("poly", ctypes.POINTER(_i32)), ("poly_n", _i32), ("reserved", _i32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("S2", _i64 * 64), ("T", _i64 * 64), ("cell_s", _i64), ("cell_t", _i64),
                ("nx", _i32), ("ny", _i32), ("nt", _i32), ("reach_s", _i32),
                ("reach_t", _i32), ("n_cells", _i64), ("dist_mode", _i32), ("n_bins", _i32),
                ("device_bytes", _i64), ("near_edges_max", _i32), ("near_cells", _i32)]


class Points(ctypes.Structure):
    _fields_ = [("x", _P(_i32)), ("y", _P(_i32)), ("t", _P(_i32)), ("n", _i64),
                ("n_centres", _i64), ("on_device", _i32), ("lambda", _P(_f64))]


class KOut(ctypes.Structure):
    _fields_ = [("C", _P(_u64)), ("W", _P(_f64)), ("K", _P(_f64)), ("L", _P(_f64))]


class EnvOut(ctypes.Structure):
    _fields_ = [("K_lo", _P(_f64)), ("K_hi", _P(_f64)), ("L_lo", _P(_f64)),
                ("L_hi", _P(_f64)), ("dL_hi", _P(_f64)), ("C_sims", _P(_u64)),
                ("W_sims", _P(_f64)), ("K_sims", _P(_f64))]


class DeviceProps(ctypes.Structure):
    _fields_ = [("compute_units", _i32), ("clock_khz", _i32), ("lds_per_cu_bytes", _i64),
                ("hbm_bytes", _i64), ("wavefront", _i32), ("arch", ctypes.c_char * 68)]


class Stats(ctypes.Structure):
    _fields_ = [("n_sets", _i64), ("n_points", _i64), ("n_in", _i64), ("n_eval", _i64),
                ("n_items", _i64), ("pair_grid", _i32), ("symmetric", _i32), ("split", _i32),
                ("bin_layout", _i32),
                ("us_total", _f64), ("us_gen", _f64), ("us_grid", _f64), ("us_pair", _f64),
                ("us_finalize", _f64), ("us_wg_end_median", _f64), ("us_wg_end_p90", _f64),
                ("us_wg_end_max", _f64), ("cost_ordered", _i32), ("reserved", _i32)]


class ServerDesc(ctypes.Structure):
    _fields_ = [("device", _i32), ("slots", _i32), ("queue_cap", _i32), ("admission", _u32),
                ("hbm_budget_bytes", _i64), ("large_work", _f64), ("age_ms", _f64),
                ("max_large", _i32), ("device_share", ctypes.c_float),
                ("slice_ms", ctypes.c_float), ("reserved", _i32)]


class Request(ctypes.Structure):
    _fields_ = [("plan", PlanDesc), ("pts", Points), ("m", _i32), ("flags", _u32),
                ("seed", _u64)]


class Result(ctypes.Structure):
    _fields_ = [("k", KOut), ("env", EnvOut), ("status", _i32), ("slot", _i32),
                ("t_submit", _f64), ("t_admit", _f64), ("t_done", _f64), ("n_in", _i64)]


class ServerState(ctypes.Structure):
    _fields_ = [("queued", _i64), ("unpolled", _i64), ("device_bytes", _i64),
                ("busy_slots", _i32), ("reserved", _i32)]


class RipkError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = f"{where}: {ripk_status_str(status)} ({status})"
        detail = ripk_last_error()
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


_lib = None

# every function the header declares, with (restype, argtypes)
_SIGS = {
    "ripk_plan_check": (_i32, [_P(PlanDesc), _P(PlanInfo)]),
    "ripk_plan": (_i32, [_P(PlanDesc), _P(ctypes.c_void_p)]),
    "ripk_plan_destroy": (None, [ctypes.c_void_p]),
    "ripk_compute_K": (_i32, [ctypes.c_void_p, _P(Points), ctypes.c_void_p, _P(KOut)]),
    "ripk_simulate_envelope": (_i32, [ctypes.c_void_p, _i64, _i32, _u64, _P(_f64),
                                      ctypes.c_void_p, _P(EnvOut)]),
    "ripk_compute_K_envelope": (_i32, [ctypes.c_void_p, _P(Points), _i32, _u64, ctypes.c_void_p,
                                       _P(KOut), _P(EnvOut)]),
    "ripk_compute_K_noalloc": (_i32, [_P(PlanDesc), _P(Points), ctypes.c_void_p, _P(KOut)]),
    "ripk_plan_stats": (_i32, [ctypes.c_void_p, _P(Stats)]),
    "ripk_plan_get_info": (_i32, [ctypes.c_void_p, _P(PlanInfo)]),
    "ripk_plan_set_flush_bound": (_i32, [ctypes.c_void_p, ctypes.c_int64]),
    "ripk_device_query": (_i32, [_i32, _P(DeviceProps)]),
    "ripk_server_create": (_i32, [_P(ServerDesc), _P(ctypes.c_void_p)]),
    "ripk_server_destroy": (None, [ctypes.c_void_p]),
    "ripk_submit": (_i32, [ctypes.c_void_p, _P(Request), _P(_u64)]),
    "ripk_poll": (_i32, [ctypes.c_void_p, _u64, _P(Result), _i32]),
    "ripk_server_status": (_i32, [ctypes.c_void_p, _P(ServerState)]),
    "ripk_status_str": (ctypes.c_char_p, [_i32]),
    "ripk_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load ``libripk.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        # One HIP runtime per process: torch ships its own libamdhip64 with the
        # same soname, so load torch first and let the library bind to it.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def ripk_status_str(s):
    return lib().ripk_status_str(int(s)).decode()


def ripk_last_error():
    r = lib().ripk_last_error()
    return r.decode() if r else ""


def _check(status, where):
    if status != RIPK_OK:
        raise RipkError(status, where)


def make_desc(window, s_max, t_max, n_s, n_t, edge=RIPK_EDGE_ISO, norm=RIPK_NORM_NN1,
              n_max=2, m_max=0, flags=0, device=0, cell_div=0, tcell_div=0,
              sim_method=RIPK_SIM_CSR, poly=None):
    """Descriptor for a window ``(x0, y0, x1, y1, t0, t1)`` and an (s, t) grid;
    ``poly``: optional (k, 2) integer vertices of a polygon study area."""
    x0, y0, x1, y1, t0, t1 = (int(v) for v in window)
    d = PlanDesc(x0, y0, x1, y1, t0, t1, int(s_max), int(t_max), int(n_s), int(n_t),
                 int(edge), int(norm), int(sim_method), int(n_max), int(m_max), int(flags),
                 int(device), int(cell_div), int(tcell_div))
    if poly is not None:
        v = np.ascontiguousarray(np.asarray(poly, np.int32).reshape(-1, 2))
        d.poly = v.ctypes.data_as(ctypes.POINTER(_i32))
        d.poly_n = len(v)
        d.keep = v  # the vertex array lives as long as the descriptor
    return d


def _info_dict(info, desc):
    ns, nt = desc.n_s, desc.n_t
    return {"S2": np.array(info.S2[:ns], np.int64), "T": np.array(info.T[:nt], np.int64),
            "cell_s": info.cell_s, "cell_t": info.cell_t, "nx": info.nx, "ny": info.ny,
            "nt": info.nt, "reach_s": info.reach_s, "reach_t": info.reach_t,
            "n_cells": info.n_cells, "dist_mode": info.dist_mode, "n_bins": info.n_bins,
            "device_bytes": info.device_bytes, "near_edges_max": info.near_edges_max,
            "near_cells": info.near_cells}


def ripk_plan_check(desc):
    """Validate a descriptor and return its derived geometry (no device use)."""
    info = PlanInfo()
    _check(lib().ripk_plan_check(ctypes.byref(desc), ctypes.byref(info)), "ripk_plan_check")
    return _info_dict(info, desc)


def ripk_plan_get_info(plan):
    """Geometry of the plan's last compute call (tuned cells with RIPK_PLAN_AUTOTUNE)."""
    info = PlanInfo()
    _check(lib().ripk_plan_get_info(plan.handle, ctypes.byref(info)), "ripk_plan_get_info")
    return _info_dict(info, plan.desc)


class Plan:
    """Owns a ``ripk_plan_t``; destroyed explicitly or when garbage collected."""

    def __init__(self, handle, desc):
        self.handle = handle
        self.desc = desc

    @property
    def shape(self):
        return (self.desc.n_s, self.desc.n_t)

    def destroy(self):
        if self.handle:
            lib().ripk_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def ripk_plan(desc):
    h = ctypes.c_void_p()
    _check(lib().ripk_plan(ctypes.byref(desc), ctypes.byref(h)), "ripk_plan")
    return Plan(h, desc)


def ripk_plan_destroy(plan):
    plan.destroy()


def _is_torch(a):
    return type(a).__module__.split(".")[0] == "torch"


def _stream_for(arrays, stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    if any(_is_torch(a) and a.is_cuda for a in arrays):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(0)


def _coord_ptr(a, n):
    if _is_torch(a):
        import torch
        if a.dtype != torch.int32 or not a.is_contiguous() or a.numel() != n:
            raise ValueError("coordinate tensors must be contiguous int32 of equal length")
        return ctypes.cast(ctypes.c_void_p(a.data_ptr()), _P(_i32)), bool(a.is_cuda), a
    arr = np.ascontiguousarray(a, dtype=np.int32)
    if arr.shape != (n,):
        raise ValueError("coordinate arrays must be 1-D of equal length")
    return arr.ctypes.data_as(_P(_i32)), False, arr


def _lambda_ptr(a, n):
    """Intensities: contiguous float64, host or device (None: no array)."""
    if a is None:
        return _P(_f64)(), None, None
    if _is_torch(a):
        import torch
        if a.dtype != torch.float64 or not a.is_contiguous() or a.numel() != n:
            raise ValueError("lambda must be a contiguous float64 tensor of length n")
        return ctypes.cast(ctypes.c_void_p(a.data_ptr()), _P(_f64)), bool(a.is_cuda), a
    arr = np.ascontiguousarray(a, dtype=np.float64)
    if arr.shape != (n,):
        raise ValueError("lambda must be 1-D of length n")
    return arr.ctypes.data_as(_P(_f64)), False, arr


def _out(shape, dtype):
    return np.zeros(shape, dtype)


def ripk_compute_K(plan, x, y, t, n_centres=0, stream=None, lam=None):
    """K, L of one point set (Eq. 2-4).  Returns numpy arrays C, W, K, L of shape (n_s, n_t).
    ``lam``: intensity per point (float64), for plans made with RIPK_PLAN_INHOM."""
    n = len(x)
    px, dx, kx = _coord_ptr(x, n)
    py, dy, ky = _coord_ptr(y, n)
    pt, dt, kt = _coord_ptr(t, n)
    pl, dl, kl = _lambda_ptr(lam, n)
    if not (dx == dy == dt) or (lam is not None and dl != dx):
        raise ValueError("coordinates (and lambda) must all be on the host or all on the device")
    pts = Points(px, py, pt, n, int(n_centres), 1 if dx else 0, pl)
    shp = plan.shape
    C = _out(shp, np.uint64)
    W = _out(shp, np.float64)
    K = _out(shp, np.float64)
    L = _out(shp, np.float64)
    out = KOut(C.ctypes.data_as(_P(_u64)), W.ctypes.data_as(_P(_f64)),
               K.ctypes.data_as(_P(_f64)), L.ctypes.data_as(_P(_f64)))
    st = _stream_for([x, y, t], stream)
    _check(lib().ripk_compute_K(plan.handle, ctypes.byref(pts), st, ctypes.byref(out)),
           "ripk_compute_K")
    del kx, ky, kt, kl
    return {"C": C, "W": W, "K": K, "L": L}


def ripk_simulate_envelope(plan, n, m, seed, L_obs=None, stream=None, per_sim=False):
    """Envelopes over m on-device CSR simulations of n points (Sec. 3)."""
    shp = plan.shape
    res = {k: _out(shp, np.float64) for k in ("K_lo", "K_hi", "L_lo", "L_hi")}
    ptr = lambda a, ct: a.ctypes.data_as(_P(ct))
    lobs = None
    null_d = _P(_f64)()
    null_u = _P(_u64)()
    if L_obs is not None:
        lobs = np.ascontiguousarray(L_obs, np.float64).reshape(shp)
        res["dL_hi"] = _out(shp, np.float64)
    if per_sim:
        res["C_sims"] = _out((m,) + shp, np.uint64)
        res["W_sims"] = _out((m,) + shp, np.float64)
        res["K_sims"] = _out((m,) + shp, np.float64)
    out = EnvOut(ptr(res["K_lo"], _f64), ptr(res["K_hi"], _f64), ptr(res["L_lo"], _f64),
                 ptr(res["L_hi"], _f64),
                 ptr(res["dL_hi"], _f64) if lobs is not None else null_d,
                 ptr(res["C_sims"], _u64) if per_sim else null_u,
                 ptr(res["W_sims"], _f64) if per_sim else null_d,
                 ptr(res["K_sims"], _f64) if per_sim else null_d)
    st = ctypes.c_void_p(int(stream)) if stream is not None else ctypes.c_void_p(0)
    _check(lib().ripk_simulate_envelope(plan.handle, int(n), int(m), int(seed) & (2**64 - 1),
                                        ptr(lobs, _f64) if lobs is not None else null_d, st,
                                        ctypes.byref(out)), "ripk_simulate_envelope")
    return res


def ripk_compute_K_envelope(plan, x, y, t, m, seed, n_centres=0, stream=None, per_sim=False):
    """K, L of the observed set and the envelopes of m simulations in one call
    (the observed set evaluated beside CSR simulations).  Returns the keys of
    ``ripk_compute_K`` and of ``ripk_simulate_envelope`` (with dL_hi)."""
    n = len(x)
    px, dx, kx = _coord_ptr(x, n)
    py, dy, ky = _coord_ptr(y, n)
    pt, dt, kt = _coord_ptr(t, n)
    if not (dx == dy == dt):
        raise ValueError("coordinates must all be on the host or all on the device")
    pts = Points(px, py, pt, n, int(n_centres), 1 if dx else 0, _P(_f64)())
    shp = plan.shape
    res = {"C": _out(shp, np.uint64)}
    for k in ("W", "K", "L", "K_lo", "K_hi", "L_lo", "L_hi", "dL_hi"):
        res[k] = _out(shp, np.float64)
    if per_sim:
        res["C_sims"] = _out((m,) + shp, np.uint64)
        res["W_sims"] = _out((m,) + shp, np.float64)
        res["K_sims"] = _out((m,) + shp, np.float64)
    ptr = lambda a, ct: a.ctypes.data_as(_P(ct))
    kout = KOut(ptr(res["C"], _u64), ptr(res["W"], _f64), ptr(res["K"], _f64), ptr(res["L"], _f64))
    eout = EnvOut(ptr(res["K_lo"], _f64), ptr(res["K_hi"], _f64), ptr(res["L_lo"], _f64),
                  ptr(res["L_hi"], _f64), ptr(res["dL_hi"], _f64),
                  ptr(res["C_sims"], _u64) if per_sim else _P(_u64)(),
                  ptr(res["W_sims"], _f64) if per_sim else _P(_f64)(),
                  ptr(res["K_sims"], _f64) if per_sim else _P(_f64)())
    st = _stream_for([x, y, t], stream)
    _check(lib().ripk_compute_K_envelope(plan.handle, ctypes.byref(pts), int(m),
                                         int(seed) & (2**64 - 1), st, ctypes.byref(kout),
                                         ctypes.byref(eout)), "ripk_compute_K_envelope")
    del kx, ky, kt
    return res


RIPK_NOALLOC_SCRATCH_BYTES = 64 << 20


def ripk_compute_K_noalloc(desc, x, y, t, out, n_centres=0, stream=None):
    """The allocation-free K, L of one observed set: ``out`` is a dict of torch
    CUDA tensors "C" (uint64 or int64), "W", "K", "L" (float64), each of
    n_s*n_t elements (any may be missing), written on success."""
    n = len(x)
    px, dx, kx = _coord_ptr(x, n)
    py, dy, ky = _coord_ptr(y, n)
    pt, dt, kt = _coord_ptr(t, n)
    if not (dx == dy == dt):
        raise ValueError("coordinates must all be on the host or all on the device")
    nb = desc.n_s * desc.n_t

    def dptr(key, ct):
        a = out.get(key)
        if a is None:
            return _P(ct)()
        if not (_is_torch(a) and a.is_cuda and a.is_contiguous() and a.numel() == nb
                and a.element_size() == 8):
            raise ValueError(f"out[{key!r}] must be a contiguous 8-byte CUDA tensor of n_s*n_t")
        return ctypes.cast(ctypes.c_void_p(a.data_ptr()), _P(ct))

    pts = Points(px, py, pt, n, int(n_centres), 1 if dx else 0, _P(_f64)())
    kout = KOut(dptr("C", _u64), dptr("W", _f64), dptr("K", _f64), dptr("L", _f64))
    st = _stream_for([x, y, t] + [v for v in out.values() if v is not None], stream)
    _check(lib().ripk_compute_K_noalloc(ctypes.byref(desc), ctypes.byref(pts), st,
                                        ctypes.byref(kout)), "ripk_compute_K_noalloc")
    del kx, ky, kt


def ripk_device_query(device=0):
    p = DeviceProps()
    _check(lib().ripk_device_query(int(device), ctypes.byref(p)), "ripk_device_query")
    d = {k: getattr(p, k) for k, _ in DeviceProps._fields_}
    d["arch"] = p.arch.decode(errors="replace")
    return d


def ripk_plan_set_flush_bound(plan, candidates):
    _check(lib().ripk_plan_set_flush_bound(plan.handle, int(candidates)),
           "ripk_plan_set_flush_bound")


def ripk_plan_stats(plan):
    s = Stats()
    _check(lib().ripk_plan_stats(plan.handle, ctypes.byref(s)), "ripk_plan_stats")
    return {k: getattr(s, k) for k, _ in Stats._fields_}


class Server:
    """Owns a ``ripk_server_t`` and remembers each ticket's output shapes."""

    def __init__(self, handle):
        self.handle = handle
        self.pending = {}  # ticket -> (n_s, n_t, m, keep_sims)

    def destroy(self):
        if self.handle:
            lib().ripk_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


RIPK_ADMIT_FIFO, RIPK_ADMIT_SIZE = 0, 1


def ripk_server_create(device=0, slots=4, queue_cap=4096, hbm_budget_bytes=64 << 30,
                       admission=RIPK_ADMIT_FIFO, large_work=0.0, age_ms=0.0, max_large=0,
                       device_share=0.0, slice_ms=0.0):
    d = ServerDesc(int(device), int(slots), int(queue_cap), int(admission),
                   int(hbm_budget_bytes), float(large_work), float(age_ms), int(max_large),
                   float(device_share), float(slice_ms), 0)
    h = ctypes.c_void_p()
    _check(lib().ripk_server_create(ctypes.byref(d), ctypes.byref(h)), "ripk_server_create")
    return Server(h)


def ripk_server_destroy(server):
    server.destroy()


def ripk_submit(server, desc, x, y, t, m=0, seed=0, n_centres=0, keep_sims=False, lam=None):
    """Queue a request (host points, copied before return); returns its ticket."""
    n = len(x)
    px, _, kx = _coord_ptr(np.asarray(x), n)
    py, _, ky = _coord_ptr(np.asarray(y), n)
    pt, _, kt = _coord_ptr(np.asarray(t), n)
    pl, _, kl = _lambda_ptr(None if lam is None else np.asarray(lam), n)
    req = Request(desc, Points(px, py, pt, n, int(n_centres), 0, pl), int(m),
                  RIPK_REQ_KEEP_SIMS if keep_sims else 0, int(seed) & (2**64 - 1))
    ticket = _u64()
    _check(lib().ripk_submit(server.handle, ctypes.byref(req), ctypes.byref(ticket)), "ripk_submit")
    del kx, ky, kt, kl
    server.pending[ticket.value] = (desc.n_s, desc.n_t, int(m), bool(keep_sims))
    return ticket.value


def ripk_poll(server, ticket, timeout_ms=-1):
    """None while the request runs; else a dict of its outputs and timings.
    Raises RipkError if the request failed."""
    ns, nt, m, keep = server.pending[ticket]
    shp = (ns, nt)
    ptr = lambda a, ct: a.ctypes.data_as(_P(ct))
    res = {"C": _out(shp, np.uint64), "W": _out(shp, np.float64), "K": _out(shp, np.float64),
           "L": _out(shp, np.float64)}
    r = Result()
    r.k = KOut(ptr(res["C"], _u64), ptr(res["W"], _f64), ptr(res["K"], _f64), ptr(res["L"], _f64))
    if m > 0:
        for key in ("K_lo", "K_hi", "L_lo", "L_hi", "dL_hi"):
            res[key] = _out(shp, np.float64)
        env = EnvOut(ptr(res["K_lo"], _f64), ptr(res["K_hi"], _f64), ptr(res["L_lo"], _f64),
                     ptr(res["L_hi"], _f64), ptr(res["dL_hi"], _f64), _P(_u64)(), _P(_f64)(),
                     _P(_f64)())
        if keep:
            res["C_sims"] = _out((m,) + shp, np.uint64)
            res["W_sims"] = _out((m,) + shp, np.float64)
            res["K_sims"] = _out((m,) + shp, np.float64)
            env.C_sims = ptr(res["C_sims"], _u64)
            env.W_sims = ptr(res["W_sims"], _f64)
            env.K_sims = ptr(res["K_sims"], _f64)
        r.env = env
    st = lib().ripk_poll(server.handle, _u64(ticket), ctypes.byref(r), int(timeout_ms))
    if st == RIPK_PENDING:
        return None
    server.pending.pop(ticket, None)
    _check(st, "ripk_poll")
    res.update(slot=r.slot, t_submit=r.t_submit, t_admit=r.t_admit, t_done=r.t_done, n_in=r.n_in)
    return res


def ripk_server_status(server):
    s = ServerState()
    _check(lib().ripk_server_status(server.handle, ctypes.byref(s)), "ripk_server_status")
    return {k: getattr(s, k) for k, _ in ServerState._fields_ if k != "reserved"}
