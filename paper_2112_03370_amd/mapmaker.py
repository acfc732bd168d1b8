"""Python binding of the HIP map-making library (libmm.so) -- argument marshalling only.

Every computation runs in the library's kernels; torch is used for device memory and streams.
Names follow the C ABI in include/mm.h.  Loading fails loudly when the library is missing.
"""

from __future__ import annotations

import ctypes
import os
import typing
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmm.so")

MM_OK = 0
MM_PENDING = 1
STATUS = {
    0: "MM_OK", 1: "MM_PENDING", -1: "MM_ERR_INVALID", -2: "MM_ERR_NOT_SPD",
    -3: "MM_ERR_NO_CONV", -4: "MM_ERR_OOM", -5: "MM_ERR_HIP", -6: "MM_ERR_BUDGET",
    -7: "MM_ERR_UNSUPPORTED", -8: "MM_ERR_NOT_FOUND",
}
TOEPLITZ_AUTO, TOEPLITZ_DIRECT, TOEPLITZ_FFT = 0, 1, 2
FLAG_UNFUSED = 1
FLAG_LDS_FFT = 2
PRECISION_MIXED, PRECISION_FP64 = 0, 1
KIND_UNPOINT, KIND_TOEPLITZ, KIND_POINT, KIND_CG = 0, 1, 2, 3

_c_i32, _c_i64, _c_dbl, _vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class MMError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{STATUS.get(status, status)}: {detail}")
        self.status = status
        self.detail = detail


class Geometry(ctypes.Structure):
    _fields_ = [
        ("n_samples", _c_i64), ("pix", _vp), ("w_q", _vp), ("w_u", _vp),
        ("n_pix_global", _c_i64), ("n_blocks", _c_i32), ("blk_start", _vp), ("blk_len", _vp),
        ("blk_band", _vp), ("n_bands", _c_i32), ("band_ncoef", _vp), ("band_offset", _vp),
        ("band_coef", _vp), ("n_dets", _c_i32), ("det_offset", _vp), ("cond_max", _c_dbl),
        ("toeplitz_algo", _c_i32), ("fft_size", _c_i32), ("flags", _c_i32),
        ("precision", _c_i32), ("n_poly", _c_i32), ("pad0", _c_i32), ("n_baselines", _c_i64),
        ("base_start", _vp), ("base_len", _vp),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("n_samples", _c_i64), ("n_pix_global", _c_i64), ("n_obs", _c_i64), ("n_kept", _c_i64),
        ("n_excised", _c_i64), ("n_gap_samples", _c_i64), ("device_bytes", _c_i64),
        ("lambda_max", _c_i32), ("toeplitz_algo", _c_i32), ("fft_size", _c_i32),
        ("n_blocks", _c_i32), ("n_chunks", _c_i32), ("fused", _c_i32),
        ("precision", _c_i32), ("n_poly", _c_i32), ("n_baselines", _c_i64),
    ]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", _c_dbl), ("max_iter", _c_i32), ("use_x0", _c_i32),
                ("check_every", _c_i32), ("use_graph", _c_i32), ("block", _c_i32),
                ("precond", _c_i32), ("refine", _c_i32), ("check_fp64", _c_i32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", _c_i32), ("converged", _c_i32), ("relres", _c_dbl),
                ("true_relres", _c_dbl), ("bnorm", _c_dbl), ("ms", _c_dbl), ("block", _c_i32),
                ("refine_steps", _c_i32), ("true_relres64", _c_dbl),
                ("inner_iterations", _c_i32), ("pad0", _c_i32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad0"}


class DeflationInfo(ctypes.Structure):
    _fields_ = [("m", _c_i32), ("rank", _c_i32), ("e_min", _c_dbl), ("e_max", _c_dbl),
                ("build_ms", _c_dbl), ("device_bytes", _c_i64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", _c_i64), ("n_slots", _c_i32), ("max_bypass", _c_i32),
                ("large_work", _c_i64), ("large_slots", _c_i32), ("pad0", _c_i32)]


class RequestTimes(ctypes.Structure):
    _fields_ = [("queued_ms", _c_dbl), ("run_ms", _c_dbl), ("total_ms", _c_dbl),
                ("slot", _c_i32), ("pad", _c_i32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class ServerStats(ctypes.Structure):
    _fields_ = [("hbm_budget", _c_i64), ("bytes_in_use", _c_i64), ("peak_bytes", _c_i64),
                ("submitted", _c_i64), ("completed", _c_i64), ("plan_hits", _c_i64),
                ("plan_misses", _c_i64), ("evictions", _c_i64), ("queued", _c_i32),
                ("running", _c_i32), ("peak_running", _c_i32), ("n_plans", _c_i32),
                ("peak_large", _c_i32), ("pad0", _c_i32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad0"}


_lib = None


def load(path: Optional[str] = None):
    """Load libmm.so (raises FileNotFoundError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise FileNotFoundError(f"{p} not found: build it with `python -m paper_2112_03370_amd.build`")
    lib = ctypes.CDLL(p)
    P = ctypes.POINTER
    sigs = {
        "mm_plan": [P(Geometry), _vp, P(_vp)],
        "mm_plan_destroy": [_vp],
        "mm_plan_info": [_vp, P(PlanInfo)],
        "mm_plan_pixels": [_vp, _vp, _vp],
        "mm_unpoint": [_vp, _vp, _vp, _vp],
        "mm_noise_weight": [_vp, _vp, _vp, _vp],
        "mm_point": [_vp, _vp, _vp, _vp],
        "mm_rhs": [_vp, _vp, _c_i32, _c_i64, _vp, _vp],
        "mm_apply_A": [_vp, _vp, _vp, _c_i32, _vp],
        "mm_precond_bj": [_vp, _vp, _vp, _c_i32, _vp],
        "mm_pcg_solve": [_vp, _vp, _c_i32, _c_i64, _vp, P(SolveOpts), P(SolveInfo), _vp],
        "mm_pcg_solve_noalloc": [_vp, _vp, _c_i32, _c_i64, _vp, P(SolveOpts), P(SolveInfo),
                                 _vp],
        "mm_set_timing": [_vp, _c_i32],
        "mm_kernel_time": [_vp, _c_i32, P(_c_dbl), P(_c_i64)],
        "mm_deflation_build": [_vp, _vp, _c_i32, _vp],
        "mm_deflation_info": [_vp, P(DeflationInfo)],
        "mm_deflation_clear": [_vp],
        "mm_deflation_vectors": [_vp, _vp, _vp],
        "mm_precond_2lvl": [_vp, _vp, _vp, _c_i32, _vp],
        "mm_server_create": [P(ServerOpts), P(_vp)],
        "mm_server_destroy": [_vp],
        "mm_server_plan": [_vp, P(Geometry), ctypes.c_uint64, P(PlanInfo)],
        "mm_submit": [_vp, ctypes.c_uint64, _vp, _c_i32, _c_i64, _vp, P(SolveOpts),
                      P(ctypes.c_uint64)],
        "mm_poll": [_vp, ctypes.c_uint64, P(SolveInfo), P(RequestTimes)],
        "mm_wait": [_vp, ctypes.c_uint64, P(SolveInfo), P(RequestTimes)],
        "mm_server_stats": [_vp, P(ServerStats)],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = _c_i32
    lib.mm_status_string.argtypes = [_c_i32]
    lib.mm_status_string.restype = ctypes.c_char_p
    lib.mm_last_error.argtypes = []
    lib.mm_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(status: int, ok=(MM_OK,)):
    if status not in ok:
        raise MMError(status, (_lib.mm_last_error() or b"").decode())
    return status


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _data_ld(d, n=None) -> int:
    """Leading dimension of data rows: a [k, n] view whose rows are contiguous may be strided
    (rows of a larger buffer, ld = row stride); a 1-D vector is one row."""
    if d.dim() == 1:
        if d.stride(0) != 1:
            raise ValueError("data vector must be contiguous")
        return int(n if n is not None else d.shape[0])
    if d.stride(-1) != 1 or d.stride(0) < d.shape[-1]:
        raise ValueError("data rows must be contiguous, with a row stride >= their length")
    return int(d.stride(0))


def _host(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


class BandTable(typing.NamedTuple):
    """Band coefficients in the ABI's layout: band b is coef[offset[b] : offset[b] + ncoef[b]]
    (c_0 .. c_lambda).  Accepted wherever a list of per-band arrays is, without the per-plan
    concatenation."""
    ncoef: np.ndarray   # int32 [n_bands]
    offset: np.ndarray  # int64 [n_bands]
    coef: np.ndarray    # float32


def band_arrays(bands):
    """(ncoef int32, offset int64, coef float32, n_bands) for the geometry's band table, from a
    BandTable (checked: ncoef and offset of one length, every band inside coef) or from a list
    of per-band coefficient arrays (concatenated)."""
    if isinstance(bands, BandTable):
        ncoef = np.ascontiguousarray(bands.ncoef, np.int32)
        off = np.ascontiguousarray(bands.offset, np.int64)
        coef = np.ascontiguousarray(bands.coef, np.float32)
        if ncoef.ndim != 1 or off.shape != ncoef.shape or coef.ndim != 1:
            raise ValueError("band table: ncoef and offset of one length, coef one-dimensional")
        if ncoef.size and (int(off.min()) < 0 or int((off + ncoef).max()) > coef.size):
            raise ValueError("band table: a band outside coef")
        if coef.size == 0:
            coef = np.zeros(1, np.float32)
        return ncoef, off, coef, int(ncoef.size)
    ncoef = np.array([len(b) for b in bands], np.int32)
    off = np.zeros(len(bands), np.int64)
    if len(bands) > 1:
        off[1:] = np.cumsum(ncoef[:-1])
    coef = (np.concatenate([np.asarray(b, np.float32) for b in bands]) if len(bands)
            else np.zeros(1, np.float32))
    return ncoef, off, np.ascontiguousarray(coef, np.float32), len(bands)


def make_geometry(pix, wq, wu, n_pix_global, blk_start, blk_len, blk_band, bands,
                  det_offset=None, cond_max=0.0, toeplitz_algo=TOEPLITZ_AUTO, fft_size=0, flags=0,
                  precision=PRECISION_MIXED, n_poly=0, base_start=None, base_len=None):
    """mm_geometry for device pointing tensors and host tables; returns (Geometry, keep-alive
    list of the host arrays it points into)."""
    import torch
    for name, t, dt in (("pix", pix, torch.int32), ("wq", wq, torch.float32),
                        ("wu", wu, torch.float32)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous CUDA {dt} tensor")
    n = int(pix.numel())
    if wq.numel() != n or wu.numel() != n:
        raise ValueError("pix, wq, wu sizes differ")
    bs = _host(blk_start, np.int64)
    bl = _host(blk_len, np.int64)
    bb = _host(blk_band, np.int32)
    ncoef, off, coef, n_bands = band_arrays(bands)
    det = None if det_offset is None else _host(det_offset, np.int64)
    g = Geometry()
    g.n_samples = n
    g.pix, g.w_q, g.w_u = _ptr(pix), _ptr(wq), _ptr(wu)
    g.n_pix_global = int(n_pix_global)
    g.n_blocks = len(bs)
    g.blk_start = bs.ctypes.data
    g.blk_len = bl.ctypes.data
    g.blk_band = bb.ctypes.data
    g.n_bands = n_bands
    g.band_ncoef = ncoef.ctypes.data
    g.band_offset = off.ctypes.data
    g.band_coef = coef.ctypes.data
    g.n_dets = 0 if det is None else len(det) - 1
    g.det_offset = None if det is None else det.ctypes.data
    g.cond_max = float(cond_max)
    g.toeplitz_algo = int(toeplitz_algo)
    g.fft_size = int(fft_size)
    g.flags = int(flags)
    g.precision = int(precision)
    g.n_poly = int(n_poly)
    bst = _host(base_start if base_start is not None else [], np.int64)
    bln = _host(base_len if base_len is not None else [], np.int64)
    if bst.size != bln.size:
        raise ValueError("base_start and base_len sizes differ")
    g.n_baselines = int(bst.size)
    g.base_start = bst.ctypes.data if bst.size else None
    g.base_len = bln.ctypes.data if bln.size else None
    return g, [bs, bl, bb, ncoef, off, coef, det, pix, wq, wu, bst, bln]


class Plan:
    """Device plan of one geometry.  Time-ordered inputs are torch CUDA tensors."""

    def __init__(self, pix, wq, wu, n_pix_global, blk_start, blk_len, blk_band, bands,
                 det_offset=None, cond_max=0.0, toeplitz_algo=TOEPLITZ_AUTO, fft_size=0,
                 flags=0, precision=PRECISION_MIXED, n_poly=0, base_start=None, base_len=None,
                 stream=None):
        lib = load()
        self._lib = lib
        self.device = pix.device
        n = int(pix.numel())
        g, self._keep = make_geometry(pix, wq, wu, n_pix_global, blk_start, blk_len, blk_band,
                                      bands, det_offset, cond_max, toeplitz_algo, fft_size, flags,
                                      precision, n_poly, base_start, base_len)
        h = _vp()
        self._h = None
        check(lib.mm_plan(ctypes.byref(g), _stream(stream), ctypes.byref(h)))
        self._h = h.value
        self.info = self.plan_info()
        self.n_kept = int(self.info["n_kept"])
        self.n_samples = n

    @classmethod
    def from_problem(cls, prob, device="cuda", **kw):
        import torch
        pix = torch.from_numpy(np.ascontiguousarray(prob.pix)).to(device)
        wq = torch.from_numpy(np.ascontiguousarray(prob.wq)).to(device)
        wu = torch.from_numpy(np.ascontiguousarray(prob.wu)).to(device)
        return cls(pix, wq, wu, prob.n_pix_global, prob.blk_start, prob.blk_len, prob.blk_band,
                   prob.bands, det_offset=prob.det_offset, **kw)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- queries -------------------------------------------------------------------------
    def plan_info(self) -> dict:
        inf = PlanInfo()
        check(self._lib.mm_plan_info(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in inf._fields_}

    def pixels(self):
        ids = np.zeros(max(1, self.n_kept), np.int64)
        hits = np.zeros(max(1, self.n_kept), np.int32)
        check(self._lib.mm_plan_pixels(self._h, ids.ctypes.data, hits.ctypes.data))
        return ids[:self.n_kept], hits[:self.n_kept]

    # ---- operators -------------------------------------------------------------------------
    def _map(self, k=1):
        import torch
        return torch.empty((k, self.n_kept, 3) if k > 1 else (self.n_kept, 3), dtype=torch.float64,
                           device=self.device)

    def unpoint(self, x, t=None, stream=None):
        import torch
        t = t if t is not None else torch.empty(self.n_samples, dtype=torch.float32, device=self.device)
        check(self._lib.mm_unpoint(self._h, _ptr(x), _ptr(t), _stream(stream)))
        return t

    def noise_weight(self, t, u=None, stream=None):
        import torch
        u = u if u is not None else torch.empty_like(t)
        check(self._lib.mm_noise_weight(self._h, _ptr(t), _ptr(u), _stream(stream)))
        return u

    def point(self, u, y=None, stream=None):
        y = y if y is not None else self._map()
        check(self._lib.mm_point(self._h, _ptr(u), _ptr(y), _stream(stream)))
        return y

    def rhs(self, d, b=None, stream=None):
        k = 1 if d.dim() == 1 else int(d.shape[0])
        ld = _data_ld(d, self.n_samples)
        b = b if b is not None else self._map(k)
        check(self._lib.mm_rhs(self._h, _ptr(d), k, ld, _ptr(b), _stream(stream)))
        return b

    def apply_A(self, x, y=None, stream=None):
        k = 1 if x.dim() == 2 else int(x.shape[0])
        y = y if y is not None else self._map(k)
        check(self._lib.mm_apply_A(self._h, _ptr(x), _ptr(y), k, _stream(stream)))
        return y

    def precond_bj(self, r, z=None, stream=None):
        k = 1 if r.dim() == 2 else int(r.shape[0])
        z = z if z is not None else self._map(k)
        check(self._lib.mm_precond_bj(self._h, _ptr(r), _ptr(z), k, _stream(stream)))
        return z

    def pcg_solve(self, d, x=None, tol=1e-8, max_iter=10000, use_x0=False, check_every=0,
                  use_graph=True, block=0, precond=0, refine=0, check_fp64=False, stream=None,
                  raise_on_error=True):
        """block 0/1: PCG per column; >= 2: columns solved together in groups of `block` by the
        enlarged-CG recurrences; < 0: group size tuned among 8, 16, 32.  refine > 0: up to that
        many FP64 refinement steps; check_fp64: report the FP64 true residual."""
        k = 1 if d.dim() == 1 else int(d.shape[0])
        ld = _data_ld(d, self.n_samples)
        x = x if x is not None else self._map(k)
        o = SolveOpts(tol=tol, max_iter=max_iter, use_x0=int(use_x0), check_every=check_every,
                      use_graph=int(use_graph), block=int(block), precond=int(precond),
                      refine=int(refine), check_fp64=int(bool(check_fp64)))
        infos = (SolveInfo * max(1, k))()
        st = self._lib.mm_pcg_solve(self._h, _ptr(d), k, ld, _ptr(x), ctypes.byref(o), infos,
                                    _stream(stream))
        if raise_on_error:
            check(st)
        res = [infos[j].as_dict() for j in range(k)]
        for r in res:
            r["status"] = STATUS.get(st, st)
        return x, (res[0] if k == 1 else res)

    def pcg_solve_noalloc(self, d, x, tol=1e-8, max_iter=10000, use_x0=False, check_every=0,
                          stream=None, raise_on_error=True):
        """mm_pcg_solve_noalloc: PCG per column with the library's static scratch (x must be
        allocated by the caller)."""
        k = 1 if d.dim() == 1 else int(d.shape[0])
        ld = _data_ld(d, self.n_samples)
        o = SolveOpts(tol=tol, max_iter=max_iter, use_x0=int(use_x0), check_every=check_every)
        infos = (SolveInfo * max(1, k))()
        st = self._lib.mm_pcg_solve_noalloc(self._h, _ptr(d), k, ld, _ptr(x), ctypes.byref(o),
                                            infos, _stream(stream))
        if raise_on_error:
            check(st)
        res = [infos[j].as_dict() for j in range(k)]
        for r in res:
            r["status"] = STATUS.get(st, st)
        return x, (res[0] if k == 1 else res)

    # ---- two-level preconditioner ------------------------------------------------------------
    def deflation_build(self, d, m, stream=None):
        """Lanczos (Alg. 3) from b = P^T N^-1 d, m steps; later solves may pass precond=1."""
        check(self._lib.mm_deflation_build(self._h, _ptr(d), int(m), _stream(stream)))
        return self.deflation_info()

    def deflation_info(self) -> dict:
        out = DeflationInfo()
        check(self._lib.mm_deflation_info(self._h, ctypes.byref(out)))
        return out.as_dict()

    def deflation_clear(self):
        check(self._lib.mm_deflation_clear(self._h))

    def deflation_vectors(self, stream=None):
        import torch
        m = self.deflation_info()["m"]
        z = torch.empty((m, self.n_kept, 3), dtype=torch.float64, device=self.device)
        check(self._lib.mm_deflation_vectors(self._h, _ptr(z), _stream(stream)))
        return z

    def precond_2lvl(self, r, z=None, stream=None):
        k = 1 if r.dim() == 2 else int(r.shape[0])
        z = z if z is not None else self._map(k)
        check(self._lib.mm_precond_2lvl(self._h, _ptr(r), _ptr(z), k, _stream(stream)))
        return z

    # ---- timing ------------------------------------------------------------------------------
    def set_timing(self, enable: bool):
        check(self._lib.mm_set_timing(self._h, int(enable)))

    def kernel_time(self, kind: int):
        ms = _c_dbl()
        n = _c_i64()
        check(self._lib.mm_kernel_time(self._h, int(kind), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


def exported_symbols(header: Optional[str] = None) -> Sequence[str]:
    """Function names declared in include/*.h (used by the ABI export test)."""
    import glob
    import re
    inc = header or os.path.join(os.path.dirname(_HERE), "include")
    names = []
    for h in sorted(glob.glob(os.path.join(inc, "*.h"))):
        src = open(h).read()
        names += re.findall(r"^\s*(?:mm_status|const char\*)\s+(mm_\w+)\s*\(", src, re.M)
    return names


class Server:
    """Serving loop: device-cached plans and continuously batched solves (mm_server_*)."""

    def __init__(self, hbm_budget=0, n_slots=4, max_bypass=-1, large_work=0, large_slots=1):
        """large_work > 0: requests of n_samples x k >= large_work run at most large_slots at
        a time (size classes)."""
        self._lib = load()
        o = ServerOpts(hbm_budget=int(hbm_budget), n_slots=int(n_slots),
                       max_bypass=int(max_bypass), large_work=int(large_work),
                       large_slots=int(large_slots))
        h = _vp()
        self._h = None
        check(self._lib.mm_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h.value
        self._inflight = {}   # ticket -> (d, x, k) kept alive until polled

    def plan(self, key, pix=None, wq=None, wu=None, n_pix_global=0, blk_start=(), blk_len=(),
             blk_band=(), bands=(), det_offset=None, geometry=None, **kw) -> dict:
        """Make the plan of a geometry available under `key` (no geometry needed on a hit;
        `geometry` may be a prepared Geometry from make_geometry)."""
        info = PlanInfo()
        if geometry is not None:
            check(self._lib.mm_server_plan(self._h, ctypes.byref(geometry), ctypes.c_uint64(key),
                                           ctypes.byref(info)))
        elif pix is None:
            check(self._lib.mm_server_plan(self._h, None, ctypes.c_uint64(key), ctypes.byref(info)))
        else:
            g, keep = make_geometry(pix, wq, wu, n_pix_global, blk_start, blk_len, blk_band,
                                    bands, det_offset, **kw)
            check(self._lib.mm_server_plan(self._h, ctypes.byref(g), ctypes.c_uint64(key),
                                           ctypes.byref(info)))
            del keep
        return {k: getattr(info, k) for k, _ in info._fields_}

    def plan_from_problem(self, key, prob, device="cuda", **kw):
        import torch
        pix = torch.from_numpy(np.ascontiguousarray(prob.pix)).to(device)
        wq = torch.from_numpy(np.ascontiguousarray(prob.wq)).to(device)
        wu = torch.from_numpy(np.ascontiguousarray(prob.wu)).to(device)
        return self.plan(key, pix, wq, wu, prob.n_pix_global, prob.blk_start, prob.blk_len,
                         prob.blk_band, prob.bands, det_offset=prob.det_offset, **kw)

    def submit(self, key, d, x, tol=1e-8, max_iter=10000, block=0, use_graph=True,
               check_every=0) -> int:
        """Queue a solve of the rows of d (CUDA float32, [k, n] or [n]) into x (CUDA float64,
        [k, n_kept, 3] or [n_kept, 3]); returns the ticket."""
        k = 1 if d.dim() == 1 else int(d.shape[0])
        ld = _data_ld(d)
        o = SolveOpts(tol=tol, max_iter=max_iter, use_x0=0, check_every=check_every,
                      use_graph=int(use_graph), block=int(block))
        t = ctypes.c_uint64()
        check(self._lib.mm_submit(self._h, ctypes.c_uint64(key), _ptr(d), k, ld, _ptr(x),
                                  ctypes.byref(o), ctypes.byref(t)))
        self._inflight[t.value] = (d, x, k)
        return t.value

    def _finish(self, fn, ticket, raise_on_error):
        d, x, k = self._inflight.get(ticket, (None, None, 1))
        infos = (SolveInfo * max(1, k))()
        times = RequestTimes()
        st = fn(self._h, ctypes.c_uint64(ticket), infos, ctypes.byref(times))
        if st == MM_PENDING:
            return None
        self._inflight.pop(ticket, None)
        if raise_on_error:
            check(st)
        res = [infos[j].as_dict() for j in range(k)]
        return {"status": STATUS.get(st, st), "info": res, "times": times.as_dict(), "x": x}

    def poll(self, ticket, raise_on_error=True):
        """None while pending, else a dict with status, per-column info, times and x."""
        return self._finish(self._lib.mm_poll, ticket, raise_on_error)

    def wait(self, ticket, raise_on_error=True):
        return self._finish(self._lib.mm_wait, ticket, raise_on_error)

    def stats(self) -> dict:
        s = ServerStats()
        check(self._lib.mm_server_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mm_server_destroy(self._h)
            self._h = None
            self._inflight.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
