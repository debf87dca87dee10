"""Python binding of libtpcf.so (angular two-point pair counting on MI355X).

Argument marshalling only: every pair is counted by the HIP kernels behind the
C ABI declared in ``include/tpcf.h``.  The functions keep the C names and
semantics; see that header for the counting rule, layouts and error codes.

If the library is not built, importing this package still works (so the
build step can run), but every call raises ``RuntimeError``: there is no
fallback.
"""

from __future__ import annotations

import collections
import ctypes
import os

import numpy as np

__all__ = [
    "DD", "DR", "RR", "FP32_CHORD", "FP64", "TpcfError", "Context", "lib", "lib_path",
    "landy_szalay", "jackknife", "compile_edges_3d", "MAX_REGIONS", "compile_edges", "compile_cells", "compile_wrap32", "compile_dot", "version", "EXPORTED_SYMBOLS", "JobDesc",
    "BATCH_GRAPH", "Tuning", "Counters", "Stats",
]

DD, DR, RR = 0, 1, 2
FP32_CHORD, FP64 = 0, 1
MAX_REGIONS = 1024

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libtpcf.so")
_lib = None

# every symbol declared in include/tpcf.h
EXPORTED_SYMBOLS = (
    "tpcf_open", "tpcf_close", "tpcf_upload_catalog", "tpcf_upload_catalog_xyz",
    "tpcf_attach_catalog", "tpcf_catalog_order", "tpcf_catalog_size", "tpcf_release_catalog",
    "tpcf_upload_catalog_regions", "tpcf_catalog_regions", "tpcf_count_regions", "tpcf_jackknife", "tpcf_count",
    "tpcf_count_async", "tpcf_count_noalloc", "tpcf_count_batch", "tpcf_submit", "tpcf_poll", "tpcf_wait",
    "tpcf_cancel", "tpcf_set_tuning", "tpcf_get_tuning", "tpcf_set_hbm_budget",
    "tpcf_hbm_usage", "tpcf_synchronize", "tpcf_set_timing", "tpcf_kernel_time",
    "tpcf_stats", "tpcf_landy_szalay", "tpcf_compile_cells", "tpcf_compile_wrap32",
    "tpcf_compile_edges", "tpcf_compile_screen", "tpcf_compile_dot", "tpcf_upload_catalog_3d", "tpcf_upload_catalog_3d_regions", "tpcf_compile_edges_3d",
    "tpcf_last_error", "tpcf_version",
)

_ERRORS = {
    -1: "TPCF_E_INVALID", -2: "TPCF_E_NOMEM", -3: "TPCF_E_HIP", -4: "TPCF_E_BADID",
    -5: "TPCF_E_BUDGET", -6: "TPCF_E_CANCELLED", -7: "TPCF_E_INTERNAL",
}


class JobDesc(ctypes.Structure):
    """struct tpcf_job_desc"""
    _fields_ = [("kind", ctypes.c_int), ("cat_a", ctypes.c_int32), ("cat_b", ctypes.c_int32),
                ("bin_edges_deg", ctypes.c_void_p), ("nbins", ctypes.c_int32),
                ("precision", ctypes.c_int), ("row_begin", ctypes.c_int64),
                ("row_end", ctypes.c_int64)]


BATCH_GRAPH = 1


class Counters(ctypes.Structure):
    """struct tpcf_counters"""
    _fields_ = [(n, ctypes.c_uint64) for n in ("pairs", "flagged", "exact", "rare_steps",
                                               "beyond_steps", "one_slot_steps", "pruned_pairs",
                                               "two_slot_steps", "chord_steps")]


Stats = collections.namedtuple("Stats", [n for n, _ in Counters._fields_])


class Tuning(ctypes.Structure):
    """struct tpcf_tuning"""
    _fields_ = [("rows_per_lane", ctypes.c_int32), ("hist_copies", ctypes.c_int32),
                ("max_cols", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("lut_bytes", ctypes.c_int32), ("lut_direct", ctypes.c_int32),
                ("prune", ctypes.c_int32)]


class TpcfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


def lib_path() -> str:
    return _LIB_PATH


def _share_torch_hip_runtime():
    """Make libtpcf.so resolve to the HIP runtime torch uses, if torch is
    installed.  torch ships its own libamdhip64 (needed by file name); the
    library needs it by SONAME.  Loading torch first puts that runtime in the
    process under the SONAME, so both share one runtime, and torch streams and
    device pointers are valid handles for the library.  Loading the library
    first would pull in a second runtime that torch cannot initialise beside."""
    try:
        import torch  # noqa: F401
    except Exception:  # pragma: no cover - torch is optional for the binding
        pass


def lib():
    """Load libtpcf.so (raises RuntimeError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    _share_torch_hip_runtime()
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(
            f"{_LIB_PATH} is missing: build it with `python -m paper_1204_6630_amd.build`")
    L = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    cint = ctypes.c_int
    sig = {
        "tpcf_open": ([cint, P, P], cint),
        "tpcf_close": ([P], cint),
        "tpcf_upload_catalog": ([P, P, P, i64, P], cint),
        "tpcf_upload_catalog_xyz": ([P, P, P, P, i64, P], cint),
        "tpcf_upload_catalog_3d": ([P, P, P, P, i64, P], cint),
        "tpcf_upload_catalog_3d_regions": ([P, P, P, P, i64, P, i32, P], cint),
        "tpcf_compile_edges_3d": ([P, i32, ctypes.c_double, P, P, P], cint),
        "tpcf_attach_catalog": ([P, P, P, i64, P], cint),
        "tpcf_catalog_order": ([P, i32, P], cint),
        "tpcf_catalog_size": ([P, i32, P], cint),
        "tpcf_release_catalog": ([P, i32], cint),
        "tpcf_upload_catalog_regions": ([P, P, P, i64, P, i32, P], cint),
        "tpcf_catalog_regions": ([P, i32, P, P], cint),
        "tpcf_count_regions": ([P, cint, i32, i32, P, i32, cint, P, P], cint),
        "tpcf_jackknife": ([P, P, P, P, P, P, i32, i32, i64, P, i64, P, cint, P, P, P], cint),
        "tpcf_count": ([P, cint, i32, i32, P, i32, cint, i64, i64, P], cint),
        "tpcf_count_async": ([P, cint, i32, i32, P, i32, cint, i64, i64, P], cint),
        "tpcf_count_noalloc": ([P, cint, i32, i32, P, i32, cint, i64, i64, P], cint),
        "tpcf_count_batch": ([P, P, i32, cint, P], cint),
        "tpcf_submit": ([P, P, P], cint),
        "tpcf_poll": ([P, i64, P, P], cint),
        "tpcf_wait": ([P, i64, P], cint),
        "tpcf_cancel": ([P, i64], cint),
        "tpcf_set_tuning": ([P, P], cint),
        "tpcf_get_tuning": ([P, P], cint),
        "tpcf_set_hbm_budget": ([P, i64], cint),
        "tpcf_hbm_usage": ([P, P, P], cint),
        "tpcf_synchronize": ([P], cint),
        "tpcf_set_timing": ([P, cint], cint),
        "tpcf_kernel_time": ([P, P, P, cint], cint),
        "tpcf_stats": ([P, P, cint], cint),
        "tpcf_landy_szalay": ([P, P, P, i32, i64, i64, cint, P], cint),
        "tpcf_compile_cells": ([P, i32, cint, ctypes.c_double, i32, i32, P, P, P, P, P], cint),
        "tpcf_compile_wrap32": ([P, i32, ctypes.c_double, i32, i32, P, P, P, P, P, P, P, P, P], cint),
        "tpcf_compile_edges": ([P, i32, ctypes.c_double, P, P, P], cint),
        "tpcf_compile_screen": ([P, i32, ctypes.c_double, P], cint),
        "tpcf_compile_dot": ([P, i32, ctypes.c_double, i32, P, P, P, P, P, P, P, P], cint),
        "tpcf_last_error": ([P], ctypes.c_char_p),
        "tpcf_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        msg = lib().tpcf_last_error(None).decode(errors="replace")
        raise TpcfError(rc, msg)


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def version() -> str:
    return lib().tpcf_version().decode()


class Context:
    """One device context (``tpcf_open``); ``stream`` is an optional
    ``hipStream_t`` handle (e.g. ``torch.cuda.Stream().cuda_stream``) to
    launch on.  None or 0 gives the context a stream of its own (torch's
    default stream has handle 0 and is not borrowed): then call
    ``synchronize()`` before torch reads what ``count_async`` wrote."""

    def __init__(self, device: int = 0, stream: int | None = None):
        self._h = ctypes.c_void_p()
        _check(lib().tpcf_open(device, ctypes.c_void_p(stream) if stream else None,
                               ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            _check(lib().tpcf_close(self._h))
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- catalogs ---------------------------------------------------------
    def upload_catalog(self, ra_deg, dec_deg) -> int:
        ra, dec = _f64(ra_deg), _f64(dec_deg)
        if ra.shape != dec.shape or ra.ndim != 1:
            raise ValueError("ra and dec must be 1-D arrays of the same length")
        cid = ctypes.c_int32()
        _check(lib().tpcf_upload_catalog(self._h, _p(ra), _p(dec), ra.size, ctypes.byref(cid)))
        return cid.value

    def upload_catalog_regions(self, ra_deg, dec_deg, region, nreg: int) -> int:
        """Upload with a jackknife region label in [0, nreg) per object."""
        ra, dec = _f64(ra_deg), _f64(dec_deg)
        reg = np.ascontiguousarray(region, dtype=np.int32)
        if ra.shape != dec.shape or ra.ndim != 1 or reg.shape != ra.shape:
            raise ValueError("ra, dec and region must be 1-D arrays of the same length")
        cid = ctypes.c_int32()
        _check(lib().tpcf_upload_catalog_regions(self._h, _p(ra), _p(dec), ra.size, _p(reg), nreg,
                                                 ctypes.byref(cid)))
        return cid.value

    def catalog_regions(self, cat: int) -> np.ndarray:
        """Objects per region (empty for an unlabelled catalog)."""
        nreg = ctypes.c_int32()
        _check(lib().tpcf_catalog_regions(self._h, cat, ctypes.byref(nreg), None))
        out = np.zeros(nreg.value, dtype=np.int64)
        _check(lib().tpcf_catalog_regions(self._h, cat, ctypes.byref(nreg), _p(out)))
        return out

    def upload_catalog_3d(self, x, y, z) -> int:
        """3-D catalog of Cartesian points; counts of it bin pairs by
        Euclidean distance, with edges in the coordinates' unit."""
        x, y, z = _f64(x), _f64(y), _f64(z)
        if not (x.shape == y.shape == z.shape) or x.ndim != 1:
            raise ValueError("x, y, z must be 1-D arrays of the same length")
        cid = ctypes.c_int32()
        _check(lib().tpcf_upload_catalog_3d(self._h, _p(x), _p(y), _p(z), x.size, ctypes.byref(cid)))
        return cid.value

    def upload_catalog_3d_regions(self, x, y, z, region, nreg: int) -> int:
        """3-D catalog with a jackknife region label in [0, nreg) per point."""
        x, y, z = _f64(x), _f64(y), _f64(z)
        reg = np.ascontiguousarray(region, dtype=np.int32)
        if not (x.shape == y.shape == z.shape == reg.shape) or x.ndim != 1:
            raise ValueError("x, y, z and region must be 1-D arrays of the same length")
        cid = ctypes.c_int32()
        _check(lib().tpcf_upload_catalog_3d_regions(self._h, _p(x), _p(y), _p(z), x.size, _p(reg), nreg,
                                                    ctypes.byref(cid)))
        return cid.value

    def upload_catalog_xyz(self, x, y, z) -> int:
        x, y, z = _f64(x), _f64(y), _f64(z)
        if not (x.shape == y.shape == z.shape) or x.ndim != 1:
            raise ValueError("x, y, z must be 1-D arrays of the same length")
        cid = ctypes.c_int32()
        _check(lib().tpcf_upload_catalog_xyz(self._h, _p(x), _p(y), _p(z), x.size,
                                             ctypes.byref(cid)))
        return cid.value

    def attach_catalog(self, xyz64_device, xyz32_device=None) -> int:
        """Attach a contiguous float64 device tensor of shape (3, n) (rows x, y,
        z) and, optionally, a float32 tensor of the same shape holding its
        round-to-nearest copies (else the library makes its own); both must
        stay alive and unchanged while the id is in use."""
        def ok(t, dtype):
            return getattr(t, "dtype", None) is not None and str(t.dtype) == dtype and t.dim() == 2 \
                and t.shape[0] == 3 and t.is_contiguous() and t.is_cuda
        t = xyz64_device
        if not ok(t, "torch.float64"):
            raise ValueError("need a contiguous float64 CUDA tensor of shape (3, n)")
        f = xyz32_device
        if f is not None and (not ok(f, "torch.float32") or f.shape != t.shape or f.device != t.device):
            raise ValueError("the FP32 copies must be a contiguous float32 CUDA tensor shaped like the FP64 one")
        # the tensors may still be being written on torch's stream; the
        # library reads them on its own
        import torch
        torch.cuda.current_stream(t.device).synchronize()
        cid = ctypes.c_int32()
        _check(lib().tpcf_attach_catalog(self._h, ctypes.c_void_p(t.data_ptr()),
                                         ctypes.c_void_p(f.data_ptr()) if f is not None else None, t.shape[1],
                                         ctypes.byref(cid)))
        return cid.value

    def catalog_order(self, cat: int) -> np.ndarray:
        """Upload index of every stored row (row ranges use stored order)."""
        out = np.empty(self.catalog_size(cat), dtype=np.int64)
        _check(lib().tpcf_catalog_order(self._h, cat, _p(out)))
        return out

    def catalog_size(self, cat: int) -> int:
        n = ctypes.c_int64()
        _check(lib().tpcf_catalog_size(self._h, cat, ctypes.byref(n)))
        return n.value

    def release_catalog(self, cat: int):
        _check(lib().tpcf_release_catalog(self._h, cat))

    # -- counting -----------------------------------------------------------
    def count(self, kind: int, cat_a: int, edges_deg, cat_b: int = -1,
              precision: int = FP32_CHORD, row_begin: int = -1, row_end: int = -1) -> np.ndarray:
        e = _f64(edges_deg)
        out = np.zeros(e.size + 1, dtype=np.uint64)
        _check(lib().tpcf_count(self._h, kind, cat_a, cat_b, _p(e), e.size - 1, precision,
                                row_begin, row_end, _p(out)))
        return out

    def count_regions(self, kind: int, cat_a: int, edges_deg, cat_b: int = -1,
                      precision: int = FP32_CHORD):
        """(total, touch): total as ``count``; touch[r] the pairs with a member
        in region r (tpcf_count_regions)."""
        e = _f64(edges_deg)
        nreg = len(self.catalog_regions(cat_a))
        total = np.zeros(e.size + 1, dtype=np.uint64)
        touch = np.zeros((max(nreg, 1), e.size + 1), dtype=np.uint64)
        _check(lib().tpcf_count_regions(self._h, kind, cat_a, cat_b, _p(e), e.size - 1, precision,
                                        _p(total), _p(touch)))
        return total, touch[:nreg]

    def count_async(self, kind: int, cat_a: int, edges_deg, out_device_ptr: int, cat_b: int = -1,
                    precision: int = FP32_CHORD, row_begin: int = -1, row_end: int = -1):
        e = _f64(edges_deg)
        _check(lib().tpcf_count_async(self._h, kind, cat_a, cat_b, _p(e), e.size - 1, precision,
                                      row_begin, row_end, ctypes.c_void_p(out_device_ptr)))

    def synchronize(self):
        _check(lib().tpcf_synchronize(self._h))

    # -- batches and jobs -----------------------------------------------------
    @staticmethod
    def _desc(kind, cat_a, edges, cat_b=-1, precision=FP32_CHORD, row_begin=-1, row_end=-1):
        return JobDesc(kind, cat_a, cat_b, edges.ctypes.data, edges.size - 1, precision,
                       row_begin, row_end)

    def count_batch(self, jobs, edges_deg, precision: int = FP32_CHORD,
                    graph: bool = False) -> np.ndarray:
        """jobs: list of (kind, cat_a, cat_b) or (kind, cat_a, cat_b, row_begin,
        row_end); returns an array (njobs, nbins+2)."""
        e = _f64(edges_deg)
        arr = (JobDesc * len(jobs))()
        for k, jb in enumerate(jobs):
            kind, ca, cb = jb[:3]
            rb, re = (jb[3], jb[4]) if len(jb) > 3 else (-1, -1)
            arr[k] = self._desc(kind, ca, e, cb, precision, rb, re)
        out = np.zeros((len(jobs), e.size + 1), dtype=np.uint64)
        _check(lib().tpcf_count_batch(self._h, arr, len(jobs), BATCH_GRAPH if graph else 0,
                                      _p(out)))
        return out

    def submit(self, kind: int, cat_a: int, edges_deg, cat_b: int = -1,
               precision: int = FP32_CHORD, row_begin: int = -1, row_end: int = -1) -> int:
        e = _f64(edges_deg)
        d = self._desc(kind, cat_a, e, cat_b, precision, row_begin, row_end)
        jid = ctypes.c_int64()
        _check(lib().tpcf_submit(self._h, ctypes.byref(d), ctypes.byref(jid)))
        return jid.value

    def poll(self, job: int, nslots: int):
        """None while running; the nslots histogram once done (the id retires)."""
        out = np.zeros(nslots, dtype=np.uint64)
        done = ctypes.c_int()
        _check(lib().tpcf_poll(self._h, job, _p(out), ctypes.byref(done)))
        return out if done.value else None

    def wait(self, job: int, nslots: int) -> np.ndarray:
        out = np.zeros(nslots, dtype=np.uint64)
        _check(lib().tpcf_wait(self._h, job, _p(out)))
        return out

    def cancel(self, job: int):
        _check(lib().tpcf_cancel(self._h, job))

    def set_tuning(self, rows_per_lane: int = 0, hist_copies: int = 0, max_cols: int = 0,
                   blocks_per_cu: int = 0, lut_bytes: int = 0, lut_direct: int = 0, prune: int = 0):
        t = Tuning(rows_per_lane, hist_copies, max_cols, blocks_per_cu, lut_bytes, lut_direct, prune)
        _check(lib().tpcf_set_tuning(self._h, ctypes.byref(t)))

    def get_tuning(self) -> dict:
        """The launch shape as set (0: default)."""
        t = Tuning()
        _check(lib().tpcf_get_tuning(self._h, ctypes.byref(t)))
        return {name: getattr(t, name) for name, _ in Tuning._fields_}

    def set_hbm_budget(self, nbytes: int):
        _check(lib().tpcf_set_hbm_budget(self._h, int(nbytes)))

    def hbm_usage(self):
        """(bytes in use, budget)"""
        u, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().tpcf_hbm_usage(self._h, ctypes.byref(u), ctypes.byref(b)))
        return u.value, b.value

    def set_timing(self, on: bool = True):
        _check(lib().tpcf_set_timing(self._h, 1 if on else 0))

    def kernel_time(self, reset: bool = False):
        """(summed pair-kernel milliseconds, launches) since the last reset."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().tpcf_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0))
        return ms.value, n.value

    def stats(self, reset: bool = False) -> "Stats":
        """Work statistics since the last reset (``tpcf_counters``)."""
        c = Counters()
        _check(lib().tpcf_stats(self._h, ctypes.byref(c), 1 if reset else 0))
        return Stats(*(getattr(c, n) for n, _ in Counters._fields_))


def landy_szalay(dd, dr, rr, n_d: int, n_r: int, form: int = 0) -> np.ndarray:
    """w(theta) per in-range bin from nbins+2-slot histograms (tpcf_landy_szalay)."""
    dd = np.ascontiguousarray(dd, dtype=np.uint64)
    dr = np.ascontiguousarray(dr, dtype=np.uint64)
    rr = np.ascontiguousarray(rr, dtype=np.uint64)
    if not (dd.shape == dr.shape == rr.shape) or dd.ndim != 1 or dd.size < 3:
        raise ValueError("need three slot arrays of the same length nbins+2")
    nbins = dd.size - 2
    w = np.empty(nbins, dtype=np.float64)
    _check(lib().tpcf_landy_szalay(_p(dd), _p(dr), _p(rr), nbins, n_d, n_r, form, _p(w)))
    return w


def jackknife(dd, dd_touch, dr, dr_touch, rr, rr_touch, n_d: int, nd_reg, n_r: int, nr_reg,
              form: int = 0):
    """Delete-one jackknife of w (tpcf_jackknife): (samples [nreg, nbins],
    mean [nbins], cov [nbins, nbins])."""
    arrs = [np.ascontiguousarray(a, dtype=np.uint64) for a in (dd, dd_touch, dr, dr_touch, rr, rr_touch)]
    ndr = np.ascontiguousarray(nd_reg, dtype=np.int64)
    nrr = np.ascontiguousarray(nr_reg, dtype=np.int64)
    nslots = arrs[0].size
    nreg = ndr.size
    if arrs[0].ndim != 1 or nslots < 3 or nrr.size != nreg:
        raise ValueError("need nbins+2-slot totals and one size per region")
    for t, touch in zip(arrs[0::2], arrs[1::2]):
        if t.shape != (nslots,) or touch.shape != (nreg, nslots):
            raise ValueError("totals must have nbins+2 slots and touch arrays shape (nreg, nbins+2)")
    nbins = nslots - 2
    samples = np.empty((nreg, nbins), dtype=np.float64)
    mean = np.empty(nbins, dtype=np.float64)
    cov = np.empty((nbins, nbins), dtype=np.float64)
    _check(lib().tpcf_jackknife(*(_p(a) for a in arrs), nbins, nreg, n_d, _p(ndr), n_r, _p(nrr), form,
                                _p(samples), _p(mean), _p(cov)))
    return samples, mean, cov


def compile_edges(edges_deg, delta_max: float = 0.0):
    """(D, qlo, qhi) of tpcf_compile_edges."""
    e = _f64(edges_deg)
    D = np.empty(e.size, np.float64)
    qlo = np.empty(e.size, np.float32)
    qhi = np.empty(e.size, np.float32)
    _check(lib().tpcf_compile_edges(_p(e), e.size - 1, delta_max, _p(D), _p(qlo), _p(qhi)))
    return D, qlo, qhi


def compile_screen(edges_deg, delta_max: float = 0.0) -> float:
    """The FP32 dot-product screen of the last edge (tpcf_compile_screen)."""
    e = _f64(edges_deg)
    out = np.zeros(1, dtype=np.float32)
    _check(lib().tpcf_compile_screen(_p(e), e.size - 1, float(delta_max), _p(out)))
    return float(out[0])


def compile_dot(edges_deg, delta_max: float = 0.0, max_cells: int = 1024):
    """Tables of the dot-product path (tpcf_compile_dot): a dict with the key
    band klo, khi, the band in p plo, phi, and the cell table shift, lo, hi,
    cells of the key q' = fl32(2 - 2p)."""
    e = _f64(edges_deg)
    out = {n: np.empty(e.size, np.float32) for n in ("klo", "khi", "plo", "phi")}
    cells = np.zeros(max_cells, np.uint16)
    sh, lo, hi = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().tpcf_compile_dot(_p(e), e.size - 1, float(delta_max), int(max_cells), _p(out["klo"]),
                                  _p(out["khi"]), _p(out["plo"]), _p(out["phi"]), ctypes.byref(sh),
                                  ctypes.byref(lo), ctypes.byref(hi), _p(cells)))
    out.update(shift=sh.value, lo=lo.value, hi=hi.value, cells=cells[:hi.value - lo.value + 1].copy())
    return out


def compile_edges_3d(edges, rmax: float):
    """(S, qlo, qhi) of tpcf_compile_edges_3d."""
    e = _f64(edges)
    S = np.empty(e.size, dtype=np.float64)
    qlo = np.empty(e.size, dtype=np.float32)
    qhi = np.empty(e.size, dtype=np.float32)
    _check(lib().tpcf_compile_edges_3d(_p(e), e.size - 1, rmax, _p(S), _p(qlo), _p(qhi)))
    return S, qlo, qhi


def compile_wrap32(edges_deg, delta_max: float = 0.0, max_bytes: int = 32768, aux_bytes: int = 0):
    """Wrapped FP32 byte table of tpcf_compile_wrap32: a dict with shift,
    wrap_bits, lo, hi, aux_off, q0 (the floor), qlo, qhi (the band with the
    floor) and image (2^wrap_bits bytes)."""
    e = _f64(edges_deg)
    sh, wb, lo, hi, ao = (ctypes.c_int32() for _ in range(5))
    q0 = ctypes.c_float()
    qlo = np.empty(e.size, np.float32)
    qhi = np.empty(e.size, np.float32)
    _check(lib().tpcf_compile_wrap32(_p(e), e.size - 1, delta_max, max_bytes, aux_bytes, ctypes.byref(sh),
                                     ctypes.byref(wb), ctypes.byref(lo), ctypes.byref(hi), ctypes.byref(ao),
                                     ctypes.byref(q0), _p(qlo), _p(qhi), None))
    image = np.zeros(1 << wb.value, np.uint8)
    _check(lib().tpcf_compile_wrap32(_p(e), e.size - 1, delta_max, max_bytes, aux_bytes, ctypes.byref(sh),
                                     ctypes.byref(wb), ctypes.byref(lo), ctypes.byref(hi), ctypes.byref(ao),
                                     ctypes.byref(q0), None, None, _p(image)))
    return {"shift": sh.value, "wrap_bits": wb.value, "lo": lo.value, "hi": hi.value, "aux_off": ao.value,
            "q0": np.float32(q0.value), "qlo": qlo, "qhi": qhi, "image": image}


def compile_cells(edges_deg, precision: int, delta_max: float = 0.0, max_cells: int | None = None,
                  direct: bool = False):
    """(shift, lo, hi, cells, E) of tpcf_compile_cells; by default the table
    size the kernels use for this many bins and layout."""
    e = _f64(edges_deg)
    byte_table = e.size + 1 <= 127
    if max_cells is None:
        max_cells = 32768 if direct else 24576 if byte_table else 12288
    cells = np.zeros(max_cells, np.uint16)
    E = np.empty(e.size, np.float64)
    sh, lo, hi = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().tpcf_compile_cells(_p(e), e.size - 1, precision, delta_max, max_cells, int(direct),
                                    ctypes.byref(sh), ctypes.byref(lo), ctypes.byref(hi),
                                    _p(cells), _p(E)))
    return sh.value, lo.value, hi.value, cells[:hi.value - lo.value + 1].copy(), E
