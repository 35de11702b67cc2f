"""Python binding of libasdg (ctypes). Argument marshalling only: assembly,
factorisation and every step of the solve run inside the native library.
PyTorch provides the caller-owned device buffers and the stream.

The native library is required; importing this module without a built
libasdg.so raises immediately (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Callable, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libasdg.so")

OK, EINVAL, ENOMEM, ENOTSPD, ENOCONV, EBREAKDOWN, EHIP, ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
FP64, FP32_LOCAL = 0, 1
APPLY_OPERATOR, APPLY_LOCAL, APPLY_COARSE, APPLY_PRECOND = 0, 1, 2, 3
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "ENOTSPD", -4: "ENOCONV", -5: "EBREAKDOWN",
                -6: "EHIP", -7: "ESTATE"}


class AsdgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Mesh_(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("xy", C.POINTER(C.c_double)), ("n_cells", C.c_int32),
                ("cell_ptr", C.POINTER(C.c_int32)), ("cell_vertices", C.POINTER(C.c_int32))]


class PcgOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int32), ("check_every", C.c_int32),
                ("use_graph", C.c_int32), ("time_kernels", C.c_int32)]


class PcgStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("rel_res", C.c_double),
                ("lambda_min", C.c_double), ("lambda_max", C.c_double), ("t_solve_ms", C.c_double),
                ("t_local_ms", C.c_double), ("n_local", C.c_int32), ("failed_subdomain", C.c_int32),
                ("true_rel_res", C.c_double), ("t_assemble_ms", C.c_double), ("t_factor_ms", C.c_double),
                ("t_coarse_ms", C.c_double)]


class TuneReport(C.Structure):
    _fields_ = [("chol_wg_per_cu", C.c_int32), ("inv_wg_per_cu", C.c_int32), ("trsv_wg_per_cu", C.c_int32),
                ("symv_waves", C.c_int32), ("task_chunk", C.c_int32), ("factor_ms", C.c_double),
                ("local_ms", C.c_double),
                ("candidates", C.c_int32), ("from_cache", C.c_int32), ("factor_schedule", C.c_int32),
                ("inverse_schedule", C.c_int32), ("tile", C.c_int32)]


class TetMesh_(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("xyz", C.POINTER(C.c_double)), ("n_cells", C.c_int32),
                ("tets", C.POINTER(C.c_int32))]


FIELD_FN = C.CFUNCTYPE(None, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p)


class SineSeries_(C.Structure):
    _fields_ = [("kx", C.c_int32), ("ky", C.c_int32), ("coef", C.POINTER(C.c_double))]

_lib = None

# exported symbols and their signatures (restype, argtypes)
_SIGS = {
    "asdg_field_sine_series": (None, [C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p]),
    "asdg_create": (C.c_int, [C.POINTER(C.c_void_p)]),
    "asdg_destroy": (None, [C.c_void_p]),
    "asdg_last_error": (C.c_char_p, [C.c_void_p]),
    "asdg_assemble": (C.c_int, [C.c_void_p, C.POINTER(Mesh_), C.c_int32, C.c_double, C.POINTER(C.c_double),
                                C.POINTER(C.c_int32), FIELD_FN, C.c_void_p]),
    "asdg_assemble_tet": (C.c_int, [C.c_void_p, C.POINTER(TetMesh_), C.c_int32, C.c_double, C.POINTER(C.c_double),
                                    C.POINTER(C.c_int32), FIELD_FN, C.c_void_p]),
    "asdg_plan": (C.c_int, [C.c_void_p, C.c_int, C.c_int32, C.POINTER(C.c_int32), C.POINTER(Mesh_),
                            C.POINTER(C.c_size_t)]),
    "asdg_bind": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_size_t), C.c_void_p]),
    "asdg_factor": (C.c_int, [C.c_void_p, C.c_void_p]),
    "asdg_setup_coarse": (C.c_int, [C.c_void_p, C.c_void_p]),
    "asdg_pcg_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(PcgOpts), C.POINTER(PcgStats),
                                 C.c_void_p]),
    "asdg_apply": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "asdg_apply_operator_static": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "asdg_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "asdg_export_rhs": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "asdg_export_operator": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                       C.POINTER(C.c_double)]),
    "asdg_export_coarse": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "asdg_failed_subdomain": (C.c_int32, [C.c_void_p]),
    "asdg_local_mode": (C.c_int32, [C.c_void_p]),
    "asdg_export_factor_tiles": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t]),
    "asdg_set_tuning": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "asdg_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(TuneReport)]),
    "asdg_tune_cache_save": (C.c_int, [C.c_char_p]),
    "asdg_tune_cache_load": (C.c_int, [C.c_char_p, C.POINTER(C.c_int32)]),
    "asdg_export_trace": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_int64),
                                    C.POINTER(C.c_double)]),
    "asdg_pcg_begin": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(PcgOpts), C.c_void_p]),
    "asdg_pcg_step": (C.c_int, [C.c_void_p, C.c_void_p]),
    "asdg_pcg_poll": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "asdg_pcg_finish": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(PcgStats), C.c_void_p]),
}
TUNE_CHOL_WG_PER_CU, TUNE_TRSV_WG_PER_CU, TUNE_CHOL_GRID, TUNE_TRACE, TUNE_LOCAL_INVERSE, TUNE_SMALL_OFF, \
    TUNE_NO_PRECOND, TUNE_INV_WG_PER_CU, TUNE_SYMV_WAVES, TUNE_TASK_CHUNK, TUNE_HOST_THREADS, TUNE_COARSE_PACKED, \
    TUNE_FACTOR_SCHEDULE, TUNE_INVERSE_SCHEDULE, TUNE_TILE = 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14
AUTOTUNE_FACTOR, AUTOTUNE_LOCAL, AUTOTUNE_REUSE = 1, 2, 4
LOCAL_SWEEPS, LOCAL_INVERSE, LOCAL_SMALL = 0, 1, 2


def lib():
    """Loads libasdg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libasdg.so not built ({LIB_PATH}); run __graft_entry__.build()")
        # torch first: the library must resolve to the HIP runtime torch has
        # loaded, because the device buffers and streams it is given are torch's
        # (loaded the other way round, the process ends up with two runtimes)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _mesh_struct(mesh):
    xy = np.ascontiguousarray(mesh.xy, dtype=np.float64)
    ptr = np.ascontiguousarray(mesh.cell_ptr, dtype=np.int32)
    cv = np.ascontiguousarray(mesh.cell_vertices, dtype=np.int32)
    m = Mesh_(xy.shape[0], _dptr(xy, C.c_double), ptr.shape[0] - 1, _dptr(ptr, C.c_int32), _dptr(cv, C.c_int32))
    return m, (xy, ptr, cv)


class Problem:
    """One SIPG problem + its two-level Schwarz preconditioner on one GPU."""

    def __init__(self):
        self._L = lib()
        h = C.c_void_p()
        self._check(self._L.asdg_create(C.byref(h)), handle=False)
        self.h = h
        self.buffers = None
        self.bytes = None
        self.n_cells = self.n_p = self.n = 0

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self._L.asdg_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def _check(self, st, handle=True):
        if st != OK:
            msg = self._L.asdg_last_error(self.h).decode() if handle else "asdg_create failed"
            raise AsdgError(st, msg)

    # ---------------------------------------------------------------- setup
    def assemble(self, mesh, p: int, c_sigma: float, rho, subdomain, f: Optional[Callable] = None):
        dim = getattr(mesh, "dim", 2)
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        sub = np.ascontiguousarray(subdomain, dtype=np.int32)

        def cb(n, xy_p, out_p, user):
            xy = np.ctypeslib.as_array(xy_p, shape=(n, dim))
            out = np.ctypeslib.as_array(out_p, shape=(n,))
            out[:] = f(xy) if f is not None else 0.0

        # a load that is a double sine series (it exposes `sine_series_coef`)
        # goes to the library's native callback, asdg_field_sine_series
        coef = getattr(f, "sine_series_coef", None) if dim == 2 else None
        user = None
        if coef is not None:
            coef = np.ascontiguousarray(coef, dtype=np.float64)
            self._cb = FIELD_FN(C.cast(self._L.asdg_field_sine_series, C.c_void_p).value)
            series = SineSeries_(coef.shape[0], coef.shape[1], _dptr(coef, C.c_double))
            user = C.cast(C.byref(series), C.c_void_p)
        else:
            self._cb = FIELD_FN(cb)
        if dim == 3:
            xyz = np.ascontiguousarray(mesh.xyz, dtype=np.float64)
            tets = np.ascontiguousarray(mesh.tets, dtype=np.int32)
            m = TetMesh_(xyz.shape[0], _dptr(xyz, C.c_double), tets.shape[0], _dptr(tets, C.c_int32))
            keep = (xyz, tets)
            self._check(self._L.asdg_assemble_tet(self.h, C.byref(m), p, c_sigma, _dptr(rho, C.c_double),
                                                  _dptr(sub, C.c_int32), self._cb, None))
            npb = (p + 1) * (p + 2) * (p + 3) // 6
        else:
            m, keep = _mesh_struct(mesh)
            self._check(self._L.asdg_assemble(self.h, C.byref(m), p, c_sigma, _dptr(rho, C.c_double),
                                              _dptr(sub, C.c_int32), self._cb, user))
            npb = (p + 1) * (p + 2) // 2
        self._subsizes = np.bincount(sub) * npb
        del keep
        info = self.info()
        self.n_cells, self.n_p, self.n = int(info[0]), int(info[1]), int(info[2])
        return self

    def plan(self, precision: int = FP64, q: int = 1, coarse_of_cell=None, coarse_mesh=None):
        b = (C.c_size_t * 4)()
        coc = None
        cm = None
        keep = None
        if coarse_of_cell is not None:
            coc_a = np.ascontiguousarray(coarse_of_cell, dtype=np.int32)
            coc = _dptr(coc_a, C.c_int32)
        if coarse_mesh is not None:
            m, keep = _mesh_struct(coarse_mesh)
            cm = C.byref(m)
        self._check(self._L.asdg_plan(self.h, precision, q, coc, cm, b))
        del keep
        self.precision = precision
        self.bytes = [int(v) for v in b]
        return self.bytes

    def bind(self, device="cuda", stream=None):
        import torch

        self.device = torch.device(device)
        self.buffers = [torch.empty(max(int(n), 256), dtype=torch.uint8, device=self.device) for n in self.bytes]
        ptrs = (C.c_void_p * 4)(*[t.data_ptr() for t in self.buffers])
        sizes = (C.c_size_t * 4)(*[t.numel() for t in self.buffers])
        self._check(self._L.asdg_bind(self.h, ptrs, sizes, self._stream(stream)))
        return self

    def _stream(self, stream):
        import torch

        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return C.c_void_p(s.cuda_stream)

    def factor(self, stream=None):
        self._check(self._L.asdg_factor(self.h, self._stream(stream)))

    def set_tuning(self, what: int, value: int):
        self._check(self._L.asdg_set_tuning(self.h, what, value))

    def autotune(self, what: int = AUTOTUNE_FACTOR | AUTOTUNE_LOCAL, stream=None) -> dict:
        """Times the launch-shape candidates of the factorisation and/or the
        batched local solves on this problem and keeps the fastest
        (asdg_autotune); returns the chosen shapes and best times."""
        r = TuneReport()
        self._check(self._L.asdg_autotune(self.h, what, self._stream(stream), C.byref(r)))
        return {k: getattr(r, k) for k, _ in TuneReport._fields_}

    def small_inverse(self, sub: int) -> np.ndarray:
        """A_i^{-1} of subdomain ``sub`` in small-subdomain mode (every
        subdomain <= 64 DoFs), as formed on the device."""
        n = int(self._sub_sizes()[sub])
        dt = np.float32 if self.precision == FP32_LOCAL else np.float64
        buf = np.empty(n * n, dtype=dt)
        self._check(self._L.asdg_export_factor_tiles(self.h, sub, buf.ctypes.data_as(C.c_void_p), buf.nbytes))
        return buf.reshape(n, n).astype(np.float64)

    def is_small(self) -> bool:
        """True when the plan uses whole small inverses (every subdomain at
        most 64 DoFs and ASDG_TUNE_SMALL_OFF not set)."""
        return int(self._L.asdg_local_mode(self.h)) == LOCAL_SMALL

    def _sub_sizes(self):
        return self._subsizes

    def export_trace(self):
        """(tasks [n,4] int32, times [n,3] uint64, clock MHz) of the last
        traced batched local solve."""
        n = C.c_int64()
        mhz = C.c_double()
        self._check(self._L.asdg_export_trace(self.h, None, None, 0, C.byref(n), C.byref(mhz)))
        tasks = np.empty((n.value, 4), dtype=np.int32)
        times = np.empty((n.value, 3), dtype=np.uint64)
        self._check(self._L.asdg_export_trace(self.h, tasks.ctypes.data_as(C.c_void_p),
                                              times.ctypes.data_as(C.c_void_p), n.value, C.byref(n),
                                              C.byref(mhz)))
        return tasks, times, mhz.value

    def failed_subdomain(self) -> int:
        return int(self._L.asdg_failed_subdomain(self.h))

    def setup_coarse(self, stream=None):
        self._check(self._L.asdg_setup_coarse(self.h, self._stream(stream)))

    # ---------------------------------------------------------------- solve
    def solve(self, b=None, rtol=1e-8, max_iter=20000, check_every=16, use_graph=True, time_kernels=False,
              x=None, stream=None, raise_on_noconv=True):
        import torch

        if x is None:
            x = torch.empty(self.n, dtype=torch.float64, device=self.device)
        bp = C.c_void_p(b.data_ptr()) if b is not None else None
        o = PcgOpts(rtol, max_iter, check_every, int(use_graph), int(time_kernels))
        s = PcgStats()
        st = self._L.asdg_pcg_solve(self.h, bp, C.c_void_p(x.data_ptr()), C.byref(o), C.byref(s),
                                    self._stream(stream))
        stats = {k: getattr(s, k) for k, _ in PcgStats._fields_}
        stats["status"] = STATUS_NAMES.get(st, st)
        if st != OK and not (st == ENOCONV and not raise_on_noconv):
            self._check(st)
        return x, stats

    # ------------------------------------------------------- non-blocking
    def begin(self, b=None, rtol=1e-8, max_iter=20000, check_every=16, stream=None):
        bp = C.c_void_p(b.data_ptr()) if b is not None else None
        o = PcgOpts(rtol, max_iter, check_every, 1, 0)
        self._check(self._L.asdg_pcg_begin(self.h, bp, C.byref(o), self._stream(stream)))

    def step(self, stream=None):
        self._check(self._L.asdg_pcg_step(self.h, self._stream(stream)))

    def poll(self):
        """(chunk_done, solve_done, iterations); never blocks."""
        c, d, it = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(self._L.asdg_pcg_poll(self.h, C.byref(c), C.byref(d), C.byref(it)))
        return bool(c.value), bool(d.value), int(it.value)

    def finish(self, x=None, stream=None, raise_on_noconv=True):
        import torch

        if x is None:
            x = torch.empty(self.n, dtype=torch.float64, device=self.device)
        s = PcgStats()
        st = self._L.asdg_pcg_finish(self.h, C.c_void_p(x.data_ptr()), C.byref(s), self._stream(stream))
        stats = {k: getattr(s, k) for k, _ in PcgStats._fields_}
        stats["status"] = STATUS_NAMES.get(st, st)
        if st != OK and not (st == ENOCONV and not raise_on_noconv):
            self._check(st)
        return x, stats

    def apply(self, what: int, v, out=None, stream=None):
        import torch

        if out is None:
            out = torch.empty_like(v)
        self._check(self._L.asdg_apply(self.h, what, C.c_void_p(v.data_ptr()), C.c_void_p(out.data_ptr()),
                                       self._stream(stream)))
        return out

    def apply_operator_static(self, v, out=None, stream=None):
        """out = A v through asdg_apply_operator_static (no allocation, no
        synchronisation inside the library; staging in its static device
        array)."""
        import torch

        if out is None:
            out = torch.empty_like(v)
        self._check(self._L.asdg_apply_operator_static(self.h, C.c_void_p(v.data_ptr()), C.c_void_p(out.data_ptr()),
                                                       self._stream(stream)))
        return out

    # ---------------------------------------------------------------- export
    def info(self):
        a = (C.c_int64 * 8)()
        self._check(self._L.asdg_info(self.h, a))
        return [int(v) for v in a]

    def export_rhs(self) -> np.ndarray:
        b = np.empty(self.n)
        self._check(self._L.asdg_export_rhs(self.h, _dptr(b, C.c_double)))
        return b

    def export_operator(self):
        import scipy.sparse as sp

        nnzb = self.info()[5]
        m = nnzb * self.n_p * self.n_p
        r = np.empty(m, dtype=np.int64)
        c = np.empty(m, dtype=np.int64)
        v = np.empty(m)
        self._check(self._L.asdg_export_operator(self.h, _dptr(r, C.c_int64), _dptr(c, C.c_int64),
                                                 _dptr(v, C.c_double)))
        return sp.coo_matrix((v, (r, c)), shape=(self.n, self.n)).tocsr()

    def export_coarse(self) -> np.ndarray:
        n0 = self.info()[4]
        a = np.empty(n0 * n0)
        self._check(self._L.asdg_export_coarse(self.h, _dptr(a, C.c_double)))
        return a.reshape(n0, n0)


def tune_cache_save(path: str) -> None:
    """Writes the process's autotuning cache (asdg_tune_cache_save)."""
    st = lib().asdg_tune_cache_save(os.fsencode(path))
    if st != OK:
        raise AsdgError(st, f"cannot write the tuning cache to {path}")


def tune_cache_load(path: str) -> int:
    """Adds the entries of a saved tuning cache (asdg_tune_cache_load);
    returns how many."""
    n = C.c_int32(0)
    st = lib().asdg_tune_cache_load(os.fsencode(path), C.byref(n))
    if st != OK:
        raise AsdgError(st, f"cannot read a tuning cache from {path}")
    return int(n.value)


def setup_problem(P, precision=FP64, device="cuda", factor=True, local_inverse=False, small=True, tile=0):
    """Assemble + plan (+ bind/factor/coarse if a device is given) for an
    ``inputs.Problem``. small=False keeps subdomains of <= 64 DoFs on the
    tile path; tile: edge of the local factor tiles with the sweeps (0
    automatic, 32 or 64)."""
    pr = Problem()
    pr.assemble(P.mesh, P.p, P.c_sigma, P.rho, P.subdomain, P.f)
    if local_inverse:
        pr.set_tuning(TUNE_LOCAL_INVERSE, 1)
    if not small:
        pr.set_tuning(TUNE_SMALL_OFF, 1)
    if tile:
        pr.set_tuning(TUNE_TILE, tile)
    pr.plan(precision, P.q, coarse_of_cell=P.coarse_of_cell if P.coarse_mesh is None else None,
            coarse_mesh=P.coarse_mesh)
    if device is not None:
        pr.bind(device)
        if factor:
            pr.factor()
            pr.setup_coarse()
    return pr
