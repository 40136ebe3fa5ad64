"""Python binding of the MI355X lattice-sum library (``include/lsum.h``).

Argument marshalling only: every step of the computation runs in the HIP library
``lib/liblsum.so``.  Importing this package loads that library and raises if it is missing;
there is no fallback implementation.  Functions keep the C names (``lsum_*``); device
pointers may be passed as integers or as objects with ``data_ptr()`` (e.g. torch tensors).
"""
from __future__ import annotations

import ctypes as C
import json
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "liblsum.so")

LSUM_OK = 0
ERRORS = {-1: "INVALID", -2: "OUT_OF_BOX", -3: "DUP_DEFECT", -4: "NOMEM", -5: "BUSY", -6: "CANCELLED",
          -7: "DEVICE", -8: "TIMEOUT", -9: "STATE", -10: "NOCONV"}
NEWTON, YUKAWA, SLATER = 0, 1, 2
FP64, FP32, BF16X3 = 0, 1, 2
SUM_CANONICAL, SUM_TUCKER_REF = 0, 1

# every symbol declared in include/lsum.h
SYMBOLS = ["lsum_nodes", "lsum_block_offsets", "lsum_shear_blocks", "lsum_column_blocks", "lsum_sinc_error", "lsum_choose_M", "lsum_create", "lsum_destroy", "lsum_last_error",
           "lsum_collocate", "lsum_shift_sum", "lsum_shift_sum_noalloc", "lsum_sample_canonical", "lsum_jacobi_svd",
           "lsum_contract",
           "lsum_submit", "lsum_submit_many", "lsum_wait", "lsum_cancel", "lsum_get_info", "lsum_get_canonical",
           "lsum_get_tucker", "lsum_tucker_to_canonical", "lsum_galerkin", "lsum_get_sigma", "lsum_sample", "lsum_get_tile", "lsum_get_stats",
           "lsum_release", "lsum_finish_many", "lsum_set_option", "lsum_get_profile", "lsum_reset_profile",
           "lsum_tune_file", "lsum_get_tuning"]
OPT_MAX_BATCH, OPT_REF_CACHE_BYTES, OPT_RANGE_MIN, OPT_JACOBI_STOP, OPT_JACOBI_MAX_SWEEPS, OPT_GRAPHS = 1, 2, 3, 4, 5, 6
OPT_JACOBI_PERSISTENT, OPT_JACOBI_WAIT_US, OPT_AUTOTUNE, OPT_GEMM_LIBRARY = 7, 8, 9, 11
OPT_JACOBI_BLOCK = 12
OPT_JACOBI_SKIP = 13


class LsumError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lsum error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


class lsum_kernel(C.Structure):
    _fields_ = [("kind", C.c_int), ("param", C.c_double), ("M", C.c_int), ("h_u", C.c_double),
                ("s", C.c_double)]


class lsum_block(C.Structure):
    _fields_ = [("L", C.c_int * 3), ("b", C.c_double * 3), ("center", C.c_double * 3),
                ("charge", C.c_double), ("x", C.c_void_p * 3)]


class lsum_defect(C.Structure):
    _fields_ = [("block", C.c_int), ("site", C.c_int * 3), ("dZ", C.c_double)]


class lsum_problem(C.Structure):
    _fields_ = [("kernel", lsum_kernel), ("N", C.c_int * 3), ("h", C.c_double),
                ("n_blocks", C.c_int), ("blocks", C.POINTER(lsum_block)),
                ("n_defects", C.c_int), ("defects", C.POINTER(lsum_defect)),
                ("eps", C.c_double), ("precision", C.c_int), ("tile_lo", C.c_int * 3),
                ("tile_T", C.c_int * 3), ("n_points", C.c_int), ("points", C.c_void_p),
                ("values", C.c_void_p), ("points_on_device", C.c_int), ("exact_sites", C.c_int),
                ("method", C.c_int), ("als_sweeps", C.c_int)]


class lsum_info(C.Structure):
    _fields_ = [("status", C.c_int), ("R", C.c_int), ("n_terms", C.c_int), ("is_tucker", C.c_int),
                ("r", C.c_int * 3), ("D", C.c_int * 3), ("norm_A", C.c_double),
                ("norm_xi", C.c_double), ("bound", C.c_double), ("rel_bound", C.c_double),
                ("t_queue_ms", C.c_double), ("t_run_ms", C.c_double), ("probe_err", C.c_double),
                ("n_probe", C.c_int)]


def _load():
    # One HIP runtime per process: torch ships its own libamdhip64 with the same SONAME as the
    # system one this library links against, so whichever is loaded first serves both.  Load
    # torch's first (when installed) so torch tensors and this library share the runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1411_1994_amd/build.py` "
                          "(there is no non-HIP implementation)")
    lib = C.CDLL(LIB_PATH)
    P, I, D, VP = C.POINTER, C.c_int, C.c_double, C.c_void_p
    sig = {
        "lsum_nodes": (I, [P(lsum_kernel), P(I), D, P(D), P(D), I, P(I)]),
        "lsum_block_offsets": (I, [P(lsum_block), P(I), D, P(C.c_int32)]),
        "lsum_sinc_error": (I, [P(lsum_kernel), P(I), D, P(D)]),
        "lsum_shear_blocks": (I, [P(lsum_block), I, I, D, I, P(lsum_block), P(I)]),
        "lsum_column_blocks": (I, [P(lsum_block), I, I, P(D), I, P(lsum_block)]),
        "lsum_choose_M": (I, [P(lsum_kernel), P(I), D, D, I, P(I), P(D)]),
        "lsum_create": (I, [P(VP), I, C.c_size_t, I]),
        "lsum_destroy": (I, [VP]),
        "lsum_last_error": (C.c_char_p, []),
        "lsum_collocate": (I, [VP, VP, I, P(D), P(D), I, D, VP, I]),
        "lsum_shift_sum": (I, [VP, VP, I, VP, I, I, I, I, P(C.c_int32), VP, I]),
        "lsum_shift_sum_noalloc": (I, [VP, VP, I, VP, I, I, I, I, P(C.c_int32), VP, I]),
        "lsum_sample_canonical": (I, [VP, VP, I, I, VP, I, P(D), P(I), D, I, VP, VP]),
        "lsum_jacobi_svd": (I, [VP, VP, I, I, VP, I, D, D, I, P(D), P(I)]),
        "lsum_galerkin": (I, [VP, I, VP, VP, VP, VP, I]),
        "lsum_tucker_to_canonical": (I, [VP, D, I, P(I), P(D), P(D), P(D), P(D), P(D), I]),
        "lsum_contract": (I, [VP, VP, I, I, I, I, VP, C.c_long, C.c_long, VP, C.c_long, C.c_long, VP,
                              C.c_long, C.c_long, D, D]),
        "lsum_submit": (I, [VP, P(lsum_problem), I, P(VP)]),
        "lsum_submit_many": (I, [VP, I, P(lsum_problem), I, P(VP)]),
        "lsum_wait": (I, [VP, I]),
        "lsum_cancel": (I, [VP]),
        "lsum_get_info": (I, [VP, P(lsum_info)]),
        "lsum_get_canonical": (I, [VP, I, VP, VP, VP, P(D), I]),
        "lsum_get_tucker": (I, [VP, VP, VP, VP, VP, I]),
        "lsum_get_sigma": (I, [VP, P(D), P(D), P(D)]),
        "lsum_sample": (I, [VP, I, VP, VP, I]),
        "lsum_get_tile": (I, [VP, VP, I, I]),
        "lsum_get_stats": (I, [VP, C.c_char_p, C.c_size_t]),
        "lsum_release": (I, [VP]),
        "lsum_finish_many": (I, [I, P(VP), P(I), P(lsum_info)]),
        "lsum_set_option": (I, [VP, I, D]),
        "lsum_get_profile": (I, [VP, C.c_char_p, C.c_size_t]),
        "lsum_tune_file": (I, [VP, C.c_char_p]),
        "lsum_get_tuning": (I, [VP, C.c_char_p, C.c_size_t]),
        "lsum_reset_profile": (I, [VP]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def _check(rc: int) -> int:
    if rc < 0:
        msg = _lib.lsum_last_error()
        raise LsumError(rc, msg.decode() if msg else "")
    return rc


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take a pointer of {type(x)}")


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _stream(s) -> Optional[int]:
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return int(s.cuda_stream)      # torch.cuda.Stream


# ------------------------------------------------------------------------------------------
# host-side steps
# ------------------------------------------------------------------------------------------

def lsum_nodes(kind: int, param: float, M: int, N: Sequence[int], h: float, h_u: float = 0.0,
               s: float = 0.0):
    k = lsum_kernel(kind, param, M, h_u, s)
    t = np.zeros(M + 1)
    w = np.zeros(M + 1)
    R = C.c_int(0)
    _check(_lib.lsum_nodes(C.byref(k), (C.c_int * 3)(*N), h, _dptr(t), _dptr(w), M + 1, C.byref(R)))
    return t[:R.value].copy(), w[:R.value].copy()


def lsum_sinc_error(kind: int, param: float, M: int, N: Sequence[int], h: float, h_u: float = 0.0,
                    s: float = 0.0) -> float:
    """Max-norm relative error of the sinc rule against the exact Galerkin tensor of one charge."""
    k = lsum_kernel(kind, param, M, h_u, s)
    err = C.c_double(0.0)
    _check(_lib.lsum_sinc_error(C.byref(k), (C.c_int * 3)(*N), h, C.byref(err)))
    return err.value


def lsum_choose_M(kind: int, param: float, N: Sequence[int], h: float, eps: float, M_max: int = 256,
                  h_u: float = 0.0, s: float = 0.0):
    """(M, err): the smallest M whose rule meets eps in the max norm; LsumError NOCONV if none."""
    k = lsum_kernel(kind, param, 0, h_u, s)
    M = C.c_int(0)
    err = C.c_double(0.0)
    _check(_lib.lsum_choose_M(C.byref(k), (C.c_int * 3)(*N), h, eps, M_max, C.byref(M), C.byref(err)))
    return M.value, err.value


def _block(b, keep=None) -> lsum_block:
    """The C block of a workloads.Block; explicit per-axis coordinates (``coords``) are passed by
    pointer, and their arrays appended to ``keep`` so they outlive the call."""
    st = lsum_block((C.c_int * 3)(*b.L), (C.c_double * 3)(*b.b), (C.c_double * 3)(*b.center),
                    float(getattr(b, "charge", 1.0)))
    coords = getattr(b, "coords", None)
    if coords is not None:
        for l in range(3):
            if coords[l] is None:
                continue
            arr = np.ascontiguousarray(coords[l], dtype=np.float64)
            if arr.shape != (b.L[l],):
                raise ValueError("coords[l] must hold L[l] coordinates")
            st.x[l] = arr.ctypes.data
            if keep is None:
                raise ValueError("explicit coordinates need a keep-alive list")
            keep.append(arr)
    return st


def lsum_shear_blocks(base, shear_axis: int, along_axis: int, shear: float) -> list:
    """A parallelogram-type lattice as rectangular blocks (``lsum_shear_blocks``): objects with the
    fields of workloads.Block (L, b, center, charge, coords)."""
    import types
    keep = []
    bst = _block(base, keep)
    n = C.c_int(0)
    _check(_lib.lsum_shear_blocks(C.byref(bst), shear_axis, along_axis, shear, 0, None, C.byref(n)))
    out = (lsum_block * n.value)()
    _check(_lib.lsum_shear_blocks(C.byref(bst), shear_axis, along_axis, shear, n.value, out, C.byref(n)))
    base_coords = getattr(base, "coords", None) or (None, None, None)
    res = []
    for b in out:
        coords = tuple(None if l == along_axis else base_coords[l] for l in range(3))
        res.append(types.SimpleNamespace(L=tuple(b.L), b=tuple(b.b), center=tuple(b.center), charge=b.charge,
                                         coords=coords if any(c is not None for c in coords) else None))
    return res


def lsum_column_blocks(base, axis: int, pts) -> list:
    """A lattice with tensor structure along one axis only (``lsum_column_blocks``): one block per
    point of the other two axes' plane; objects with the fields of workloads.Block."""
    import types
    keep = []
    bst = _block(base, keep)
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 2)
    n = pts.shape[0]
    out = (lsum_block * max(n, 1))()
    _check(_lib.lsum_column_blocks(C.byref(bst), axis, n, _dptr(pts), n, out))
    coords = getattr(base, "coords", None)
    res = []
    for b in out[:n]:
        c = tuple(coords[l] if (coords is not None and l == axis) else None for l in range(3))
        res.append(types.SimpleNamespace(L=tuple(b.L), b=tuple(b.b), center=tuple(b.center), charge=b.charge,
                                         coords=c if any(x is not None for x in c) else None))
    return res


def lsum_block_offsets(block, N: Sequence[int], h: float):
    keep = []
    blk = _block(block, keep)
    out = np.zeros(sum(block.L), dtype=np.int32)
    _check(_lib.lsum_block_offsets(C.byref(blk), (C.c_int * 3)(*N), h,
                                   out.ctypes.data_as(C.POINTER(C.c_int32))))
    L = block.L
    return [out[:L[0]].copy(), out[L[0]:L[0] + L[1]].copy(), out[L[0] + L[1]:].copy()]


# ------------------------------------------------------------------------------------------
# context and device steps
# ------------------------------------------------------------------------------------------

class Context:
    """A library context on one device: request slots, buffer pool, reference cache."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, n_slots: int = 0):
        h = C.c_void_p()
        _check(_lib.lsum_create(C.byref(h), device, hbm_budget_bytes, n_slots))
        self.handle = h

    def close(self):
        if self.handle:
            _lib.lsum_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- device steps --------------------------------------------------------------------
    def collocate(self, t: np.ndarray, w: np.ndarray, N_ref: int, h: float, G_dev, ldg: int, stream=None):
        t = np.ascontiguousarray(t, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        _check(_lib.lsum_collocate(self.handle, _stream(stream), len(t), _dptr(t), _dptr(w), N_ref, h,
                                   _ptr(G_dev), ldg))

    def shift_sum(self, R: int, G_dev, ldg: int, N_ref: int, N_axis: int, sites: np.ndarray, U_dev,
                  ldu: int, stream=None):
        sites = np.ascontiguousarray(sites, dtype=np.int32)
        _check(_lib.lsum_shift_sum(self.handle, _stream(stream), R, _ptr(G_dev), ldg, N_ref, N_axis,
                                   len(sites), sites.ctypes.data_as(C.POINTER(C.c_int32)),
                                   _ptr(U_dev), ldu))

    def shift_sum_noalloc(self, R: int, G_dev, ldg: int, N_ref: int, N_axis: int, sites: np.ndarray, U_dev,
                          ldu: int, stream=None):
        """lsum_shift_sum without allocation (the device's static scratch array)."""
        sites = np.ascontiguousarray(sites, dtype=np.int32)
        _check(_lib.lsum_shift_sum_noalloc(self.handle, _stream(stream), R, _ptr(G_dev), ldg, N_ref, N_axis,
                                           len(sites), sites.ctypes.data_as(C.POINTER(C.c_int32)),
                                           _ptr(U_dev), ldu))

    def sample_canonical(self, n_fac: int, R: int, U_dev, ldu: int, lam: np.ndarray, N, h: float,
                         n_pts: int, xyz_dev, out_dev, stream=None):
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        _check(_lib.lsum_sample_canonical(self.handle, _stream(stream), n_fac, R, _ptr(U_dev), ldu,
                                          _dptr(lam), (C.c_int * 3)(*N), h, n_pts, _ptr(xyz_dev),
                                          _ptr(out_dev)))

    def jacobi_svd(self, D: int, N: int, A_dev, lda: int, tol: float = 1e-12, irrelevant: float = 0.0,
                   max_sweeps: int = 40, stream=None):
        sig = np.zeros(D)
        sweeps = C.c_int(0)
        rc = _lib.lsum_jacobi_svd(self.handle, _stream(stream), D, N, _ptr(A_dev), lda, tol, irrelevant,
                                  max_sweeps, _dptr(sig), C.byref(sweeps))
        _check(rc)
        return sig, sweeps.value

    def contract(self, prec: int, m: int, n: int, k: int, A_dev, sam: int, sak: int, B_dev, sbk: int,
                 sbn: int, C_dev, scm: int, scn: int, alpha: float = 1.0, beta: float = 0.0, stream=None):
        _check(_lib.lsum_contract(self.handle, _stream(stream), prec, m, n, k, _ptr(A_dev), sam, sak,
                                  _ptr(B_dev), sbk, sbn, _ptr(C_dev), scm, scn, alpha, beta))

    # -- options and profile --------------------------------------------------------------
    def set_option(self, key: int, value: float):
        _check(_lib.lsum_set_option(self.handle, key, float(value)))

    def tune_file(self, path: str):
        """Read and append the autotuner's decisions in a text file (lsum_tune_file)."""
        _check(_lib.lsum_tune_file(self.handle, path.encode()))

    def tuning(self) -> dict:
        n = _lib.lsum_get_tuning(self.handle, None, 0)
        buf = C.create_string_buffer(n + 16)
        _lib.lsum_get_tuning(self.handle, buf, n + 16)
        return json.loads(buf.value.decode())

    def profile(self) -> dict:
        n = _lib.lsum_get_profile(self.handle, None, 0)
        buf = C.create_string_buffer(n + 16)
        _lib.lsum_get_profile(self.handle, buf, n + 16)
        return json.loads(buf.value.decode())

    def reset_profile(self):
        _check(_lib.lsum_reset_profile(self.handle))

    # -- requests -------------------------------------------------------------------------
    def submit(self, problem, nonblocking: bool = False, points=None, values=None) -> "Request":
        """Submit a problem; optional sample points (n x 3) and an output array (n) -- numpy arrays
        (host) or device tensors -- are evaluated as part of the request."""
        return Request(self, problem, nonblocking, points, values)

    def submit_set(self, prepared, n, points=None, values=None, nonblocking: bool = False) -> "RequestSet":
        """n requests of one problem as a RequestSet (one library call to submit, one to finish)."""
        return RequestSet(self, prepared, n, points, values, nonblocking)

    def submit_many(self, problems, nonblocking: bool = False, points=None, values=None) -> list:
        """Submit several problems at once; they enter the queue together, so a slot fuses
        consecutive canonical ones into one batch.  points / values: optional per-problem lists
        (as for submit; None entries allowed)."""
        n = len(problems)
        arr = (lsum_problem * n)()
        size = C.sizeof(lsum_problem)
        out = []
        for i, p in enumerate(problems):
            if isinstance(p, Prepared):
                C.memmove(C.addressof(arr[i]), C.addressof(p.struct), size)
                keep = [p]
                prob = p.problem
            else:
                st, kp = make_problem(p)
                C.memmove(C.addressof(arr[i]), C.addressof(st), size)
                keep = [kp]
                prob = p
            pts = points[i] if points is not None else None
            vals = values[i] if values is not None else None
            if pts is not None:
                if isinstance(pts, np.ndarray):
                    pts = np.ascontiguousarray(pts, dtype=np.float64)
                    if vals is None:
                        vals = np.zeros(pts.shape[0])
                e = arr[i]
                e.n_points = int(pts.shape[0])
                e.points = _ptr(pts)
                e.values = _ptr(vals)
                e.points_on_device = 0 if isinstance(pts, np.ndarray) else 1
                keep += [pts, vals]
            r = Request.__new__(Request)
            r.ctx = self
            r.problem = prob
            r._keep = keep
            r.values = vals
            out.append(r)
        handles = (C.c_void_p * n)()
        _check(_lib.lsum_submit_many(self.handle, n, arr, 1 if nonblocking else 0, handles))
        for i, r in enumerate(out):
            r.handle = C.c_void_p(handles[i])
        return out


def finish_many(requests):
    """Wait for, describe and release several requests with one library call
    (``lsum_finish_many``); returns [(status, lsum_info)] in order.  The requests are released."""
    n = len(requests)
    handles = (C.c_void_p * n)(*[r.handle for r in requests])
    status = (C.c_int * n)()
    infos = (lsum_info * n)()
    _check(_lib.lsum_finish_many(n, handles, status, infos))
    for r in requests:
        r.handle = None
    return [(status[i], infos[i]) for i in range(n)]


def problem_array(prepared, n, points=None, values=None):
    """n copies of a prepared problem's C struct in one array (one copy), with request k's point
    and value pointers written in by vectorised stores (pure marshalling, no library call)."""
    size = C.sizeof(lsum_problem)
    arr = (lsum_problem * n).from_buffer_copy(bytes(prepared.struct) * n)
    if points is not None:
        pts = points if isinstance(points, (list, tuple)) else [points] * n
        if values is None or len(values) != n or len(pts) != n:
            raise ValueError("points need n output arrays")
        rows = np.frombuffer(arr, dtype=np.uint8).reshape(n, size)

        def put(field, vals, dtype):
            off = getattr(lsum_problem, field).offset
            width = np.dtype(dtype).itemsize
            rows[:, off:off + width] = np.asarray(vals, dtype=dtype).view(np.uint8).reshape(n, width)

        put("n_points", [int(x.shape[0]) for x in pts], np.int32)
        put("points", [_ptr(x) for x in pts], np.uint64)
        put("values", [_ptr(v) for v in values], np.uint64)
        put("points_on_device", [0 if isinstance(x, np.ndarray) else 1 for x in pts], np.int32)
    return arr


class RequestSet:
    """n requests of one prepared problem, submitted with one ``lsum_submit_many`` call and finished
    with one ``lsum_finish_many`` call; for clients that submit and collect in batches.  points: one
    array/tensor shared by all requests or a list of n; values: a list of n outputs (device tensors
    or numpy arrays, caller-owned until the set is finished)."""

    def __init__(self, ctx, prepared, n, points=None, values=None, nonblocking=False):
        if not isinstance(prepared, Prepared):
            prepared = Prepared(prepared)
        self.ctx, self.n, self.problem = ctx, n, prepared.problem
        self._arr = problem_array(prepared, n, points, values)
        self._keep = [prepared, points, values]
        self._handles = None
        handles = (C.c_void_p * n)()
        _check(_lib.lsum_submit_many(ctx.handle, n, self._arr, 1 if nonblocking else 0, handles))
        self._handles = handles
        self.values = values

    def finish(self):
        """Wait for, report and release every request: (status array, lsum_info array)."""
        status = (C.c_int * self.n)()
        infos = (lsum_info * self.n)()
        _check(_lib.lsum_finish_many(self.n, self._handles, status, infos))
        self._handles = None
        return status, infos

    def __del__(self):
        try:
            if self._handles is not None:
                self.finish()
        except Exception:
            pass


class Prepared:
    """A problem marshalled once into its C struct, for submitting many times (the library
    deep-copies the struct at every submit, so one Prepared may back any number of requests)."""

    def __init__(self, problem):
        self.problem = problem
        self.struct, self._keep = make_problem(problem)


def prepare(problem) -> Prepared:
    return Prepared(problem)


def make_problem(p, points=None, values=None) -> tuple:
    """A C ``lsum_problem`` from any object with the fields of ``workloads.Problem``; returns
    (struct, keep-alive list)."""
    coord_keep = []
    blocks = (lsum_block * len(p.blocks))(*[_block(b, coord_keep) for b in p.blocks])
    nd = len(p.defects)
    defects = (lsum_defect * max(nd, 1))(*[lsum_defect(d.block, (C.c_int * 3)(*d.site), float(d.dZ))
                                          for d in p.defects])
    prob = lsum_problem(lsum_kernel(p.kind, float(p.param), p.M, float(getattr(p, "h_u", 0.0)),
                                    float(getattr(p, "s", 0.0))),
                        (C.c_int * 3)(*p.N), float(p.h), len(p.blocks),
                        C.cast(blocks, C.POINTER(lsum_block)), nd,
                        C.cast(defects, C.POINTER(lsum_defect)) if nd else None,
                        float(p.eps), int(p.precision), (C.c_int * 3)(*p.tile_lo),
                        (C.c_int * 3)(*p.tile_T))
    prob.exact_sites = 1 if getattr(p, "exact_sites", False) else 0
    prob.method = int(getattr(p, "method", SUM_CANONICAL))
    prob.als_sweeps = int(getattr(p, "als_sweeps", 0))
    keep = [blocks, defects, coord_keep]
    if points is not None:
        on_dev = not isinstance(points, np.ndarray)
        prob.n_points = int(points.shape[0])
        prob.points = _ptr(points)
        prob.values = _ptr(values)
        prob.points_on_device = 1 if on_dev else 0
        keep += [points, values]
    return prob, keep


class Request:
    """One submitted problem (``lsum_submit`` ... ``lsum_release``)."""

    def __init__(self, ctx: Context, problem, nonblocking: bool = False, points=None, values=None):
        self.ctx = ctx
        if points is not None and isinstance(points, np.ndarray):
            points = np.ascontiguousarray(points, dtype=np.float64)
            if values is None:
                values = np.zeros(points.shape[0])
        if isinstance(problem, Prepared):
            self.problem = problem.problem
            prob = lsum_problem.from_buffer_copy(problem.struct)
            keep = [problem]
            if points is not None:
                prob.n_points = int(points.shape[0])
                prob.points = _ptr(points)
                prob.values = _ptr(values)
                prob.points_on_device = 0 if isinstance(points, np.ndarray) else 1
                keep += [points, values]
        else:
            self.problem = problem
            prob, keep = make_problem(problem, points, values)
        self._keep = keep            # caller memory must outlive the request
        self.values = values
        h = C.c_void_p()
        _check(_lib.lsum_submit(ctx.handle, C.byref(prob), 1 if nonblocking else 0, C.byref(h)))
        self.handle = h

    def wait(self, timeout_ms: int = -1) -> int:
        """The request's final status (0, or a negative LSUM_E_* code such as -6 for a cancelled
        request), or -8 (TIMEOUT) if it is still running after timeout_ms."""
        return int(_lib.lsum_wait(self.handle, timeout_ms))

    def cancel(self):
        _check(_lib.lsum_cancel(self.handle))

    def info(self) -> lsum_info:
        inf = lsum_info()
        _check(_lib.lsum_get_info(self.handle, C.byref(inf)))
        return inf

    def canonical(self, block: int = 0, with_weight: bool = False):
        """Factors [U0, U1, U2] (R x N_l) of a block's canonical sum, and with with_weight the
        block's weight (its charge) as a second result."""
        p = self.problem
        inf = self.info()
        U = [np.zeros((inf.R, n)) for n in p.N]
        w = C.c_double(0.0)
        _check(_lib.lsum_get_canonical(self.handle, block, *[u.ctypes.data for u in U], C.byref(w), 0))
        return (U, w.value) if with_weight else U

    def tucker(self):
        p = self.problem
        inf = self.info()
        r = list(inf.r)
        Z = [np.zeros((r[l], p.N[l])) for l in range(3)]
        core = np.zeros(tuple(r))
        _check(_lib.lsum_get_tucker(self.handle, *[z.ctypes.data for z in Z], core.ctypes.data, 0))
        return Z, core

    def galerkin(self, G):
        """V (nb x nb): the Galerkin matrix of the Tucker result in the separable basis whose
        per-axis values at the cell centres are G[l] (nb x N_l)."""
        G = [np.ascontiguousarray(g, dtype=np.float64) for g in G]
        nb = G[0].shape[0]
        V = np.zeros((nb, nb))
        _check(_lib.lsum_galerkin(self.handle, nb, G[0].ctypes.data, G[1].ctypes.data, G[2].ctypes.data,
                                  V.ctypes.data, 0))
        return V

    def tucker_to_canonical(self, eps: float):
        """(xi, [U0, U1, U2], err): canonical form of the Tucker result (U_l vector-major, R x N_l)."""
        R = C.c_int(0)
        err = C.c_double(0.0)
        _check(_lib.lsum_tucker_to_canonical(self.handle, eps, 0, C.byref(R), None, None, None, None,
                                             C.byref(err), 0))
        n = R.value
        p = self.problem
        xi = np.zeros(n)
        U = [np.zeros((n, p.N[l])) for l in range(3)]
        _check(_lib.lsum_tucker_to_canonical(self.handle, eps, n, C.byref(R), _dptr(xi), *[_dptr(u) for u in U],
                                             C.byref(err), 0))
        return xi, U, err.value

    def sigma(self):
        inf = self.info()
        s = [np.zeros(inf.D[l]) for l in range(3)]
        _check(_lib.lsum_get_sigma(self.handle, *[_dptr(x) for x in s]))
        return s

    def sample(self, xyz, out=None, on_device: bool = False):
        if on_device:
            n = int(xyz.shape[0])
            _check(_lib.lsum_sample(self.handle, n, _ptr(xyz), _ptr(out), 1))
            return out
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        res = np.zeros(xyz.shape[0])
        _check(_lib.lsum_sample(self.handle, xyz.shape[0], xyz.ctypes.data, res.ctypes.data, 0))
        return res

    def tile(self):
        p = self.problem
        dt = np.float64 if p.precision == FP64 else np.float32
        out = np.zeros(tuple(p.tile_T), dtype=dt)
        _check(_lib.lsum_get_tile(self.handle, out.ctypes.data, out.itemsize, 0))
        return out

    def stats(self) -> dict:
        n = _lib.lsum_get_stats(self.handle, None, 0)
        buf = C.create_string_buffer(n + 16)
        _lib.lsum_get_stats(self.handle, buf, n + 16)
        return json.loads(buf.value.decode())

    def release(self):
        if self.handle:
            _lib.lsum_release(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass
