"""Python binding of liblamg (include/lamg.h): argument marshalling only.

Every function here has the name of the C entry point it calls. Device memory and
streams come from PyTorch (ROCm); every step of setup and solve runs inside the HIP
library. If liblamg.so has not been built, importing this module raises ImportError:
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library then shares with PyTorch)

_LIB_PATH = Path(__file__).resolve().parent / "liblamg.so"
if not _LIB_PATH.exists():
    raise ImportError(f"{_LIB_PATH} is not built (run __graft_entry__.build())")
_lib = C.CDLL(str(_LIB_PATH))

MAX_LEVELS = 64
SETUP_PHASES = 9
SETUP_PHASE_NAMES = ("input", "color", "level", "aggregate", "interp", "eliminate", "galerkin",
                     "coarsest", "layout")

(OK, INVALID_ARG, NOT_SYMMETRIC, SELF_LOOP, BAD_WEIGHT, DISCONNECTED, OOM, COARSENING_STALLED,
 NOT_CONVERGED, HIP_ERROR, UNAVAILABLE, SCRATCH_TOO_SMALL) = range(12)
NOALLOC_SCRATCH_BYTES = 64 << 20
MEM_HOST, MEM_DEVICE = 0, 1
FP64, FP32_IR = 0, 1


class lamg_graph(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("weight", C.c_void_p), ("mem", C.c_int32)]


class lamg_options(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("n_direct", C.c_int32), ("enable_veto", C.c_int32),
                ("enable_caliber2", C.c_int32), ("kappa", C.c_int32), ("build_fp32", C.c_int32),
                ("keep_setup_data", C.c_int32), ("tail_rows", C.c_int32),
                ("elimination", C.c_int32), ("smoother", C.c_int32), ("graphs", C.c_int32),
                ("tail_finest", C.c_int32), ("reorder", C.c_int32)]


class lamg_hier_info(C.Structure):
    _fields_ = [("levels", C.c_int32), ("n", C.c_int64 * MAX_LEVELS),
                ("nnz", C.c_int64 * MAX_LEVELS), ("ncolors", C.c_int32 * MAX_LEVELS),
                ("n_caliber2", C.c_int64 * MAX_LEVELS), ("gamma", C.c_double * MAX_LEVELS),
                ("tau", C.c_double * MAX_LEVELS), ("bytes_device", C.c_int64),
                ("op_complexity", C.c_double), ("setup_seconds", C.c_double),
                ("bytes_peak", C.c_int64), ("elim", C.c_int32 * MAX_LEVELS),
                ("tail_level", C.c_int32), ("timed_level", C.c_int32),
                ("cheb", C.c_int32 * MAX_LEVELS), ("cheb_lmax", C.c_double * MAX_LEVELS),
                ("setup_phase_seconds", C.c_double * SETUP_PHASES),
                ("bjgs", C.c_int32 * MAX_LEVELS), ("reordered", C.c_int32)]


class lamg_solve_info(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("relres_max", C.c_double), ("acf_max", C.c_double),
                ("seconds", C.c_double), ("relres", C.c_void_p), ("col_cycles", C.c_void_p),
                ("history", C.c_void_p), ("history_len", C.c_int32), ("graph_cycles", C.c_int32),
                ("bytes", C.c_double)]


class lamg_level_export(C.Structure):
    _fields_ = [(name, C.c_void_p) for name in (
        "row_ptr", "col_idx", "val", "color", "strong", "x", "affinity", "moments", "seed",
        "aggregate", "p0", "p1", "w0", "w1")]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)

_lib.lamg_set_allocator.argtypes = [ALLOC_FN, FREE_FN, C.c_void_p]
_lib.lamg_set_allocator.restype = None
_lib.lamg_status_string.argtypes = [C.c_int]
_lib.lamg_status_string.restype = C.c_char_p
_lib.lamg_version.argtypes = []
_lib.lamg_version.restype = C.c_char_p
_lib.lamg_default_options.argtypes = [C.POINTER(lamg_options)]
_lib.lamg_default_options.restype = None
_lib.lamg_setup.argtypes = [C.POINTER(lamg_graph), C.POINTER(lamg_options), C.c_void_p,
                            C.POINTER(C.c_void_p)]
_lib.lamg_setup.restype = C.c_int
_lib.lamg_solve.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_int32, C.c_int,
                            C.c_void_p, C.POINTER(lamg_solve_info), C.c_void_p]
_lib.lamg_solve.restype = C.c_int
_lib.lamg_solve_noalloc.argtypes = _lib.lamg_solve.argtypes
_lib.lamg_solve_noalloc.restype = C.c_int
_lib.lamg_solve_group.argtypes = [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                  C.POINTER(C.c_int32), C.c_double, C.c_int32, C.c_int,
                                  C.POINTER(C.c_void_p), C.c_void_p, C.POINTER(C.c_int),
                                  C.c_void_p]
_lib.lamg_solve_group.restype = C.c_int
_lib.lamg_destroy.argtypes = [C.c_void_p]
_lib.lamg_destroy.restype = None
_lib.lamg_hierarchy_info.argtypes = [C.c_void_p, C.POINTER(lamg_hier_info)]
_lib.lamg_hierarchy_info.restype = C.c_int
_lib.lamg_export_level.argtypes = [C.c_void_p, C.c_int32, C.POINTER(lamg_level_export)]
_lib.lamg_export_level.restype = C.c_int
_lib.lamg_profile_kernel.argtypes = [C.c_void_p, C.c_int32, C.c_int, C.c_int, C.c_int32, C.c_int32,
                                     C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p]
_lib.lamg_profile_kernel.restype = C.c_int

(KERNEL_GS_COLOR, KERNEL_RESIDUAL, KERNEL_RESTRICT, KERNEL_PROLONG, KERNEL_TAIL, KERNEL_REDUCE,
 KERNEL_VECTOR, KERNEL_CHEB, KERNEL_BJGS) = range(9)
KERNEL_NAMES = ("gs_color", "residual", "restrict", "prolong", "tail", "reduce", "vector", "cheb",
                "bjgs")


class lamg_kernel_time(C.Structure):
    _fields_ = [("launches", C.c_int64), ("seconds", C.c_double), ("bytes", C.c_double)]


_lib.lamg_timing_start.argtypes = [C.c_void_p, C.c_int32]
_lib.lamg_timing_start.restype = C.c_int
_lib.lamg_timing_start_all.argtypes = [C.c_void_p, C.c_int32]
_lib.lamg_timing_start_all.restype = C.c_int
_lib.lamg_timing_stop.argtypes = [C.c_void_p]
_lib.lamg_timing_stop.restype = C.c_int
_lib.lamg_timing_get.argtypes = [C.c_void_p, C.c_int, C.c_int, C.POINTER(lamg_kernel_time)]
_lib.lamg_timing_get.restype = C.c_int


class LamgError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {lamg_status_string(status)} ({status})")
        self.status = status


def library_path() -> str:
    return str(_LIB_PATH)


def lamg_status_string(status: int) -> str:
    return _lib.lamg_status_string(int(status)).decode()


def lamg_version() -> str:
    return _lib.lamg_version().decode()


def lamg_default_options(**overrides) -> lamg_options:
    o = lamg_options()
    _lib.lamg_default_options(C.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, int(v))
    return o


_alloc_keepalive = []


def lamg_set_allocator(alloc=None, free=None, ctx=None) -> None:
    """Routes the library's device allocations through alloc(bytes, stream, ctx) /
    free(ptr, stream, ctx) (ctypes-callable), or back to hipMalloc with no arguments."""
    if alloc is None:
        _lib.lamg_set_allocator(ALLOC_FN(0), FREE_FN(0), None)
        return
    a, f = ALLOC_FN(alloc), FREE_FN(free)
    # handles keep the hook they were built with, so every hook ever installed stays alive
    _alloc_keepalive.extend([a, f])
    _lib.lamg_set_allocator(a, f, ctx)


def _stream_ptr(stream) -> int | None:
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Handle:
    """Owns a lamg_handle*; lamg_destroy runs when it is closed or collected."""

    def __init__(self, ptr: C.c_void_p, n: int):
        self._ptr = ptr
        self.n = n

    @property
    def ptr(self):
        if not self._ptr:
            raise ValueError("handle is closed")
        return self._ptr

    def close(self):
        if self._ptr:
            _lib.lamg_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _graph_struct(graph, device: bool, keep: list) -> lamg_graph:
    g = lamg_graph()
    g.n = int(graph.n)
    g.nnz = int(graph.row_ptr[-1])
    if device:
        import torch

        rp = torch.as_tensor(np.ascontiguousarray(graph.row_ptr, np.int32), device="cuda")
        ci = torch.as_tensor(np.ascontiguousarray(graph.col_idx, np.int32), device="cuda")
        w = torch.as_tensor(np.ascontiguousarray(graph.weight, np.float64), device="cuda")
        keep += [rp, ci, w]
        g.row_ptr, g.col_idx, g.weight = rp.data_ptr(), ci.data_ptr(), w.data_ptr()
        g.mem = MEM_DEVICE
    else:
        rp = np.ascontiguousarray(graph.row_ptr, np.int32)
        ci = np.ascontiguousarray(graph.col_idx, np.int32)
        w = np.ascontiguousarray(graph.weight, np.float64)
        keep += [rp, ci, w]
        g.row_ptr, g.col_idx, g.weight = rp.ctypes.data, ci.ctypes.data, w.ctypes.data
        g.mem = MEM_HOST
    return g


def lamg_setup(graph, options: lamg_options | None = None, stream=None, device_input=False,
               raw_stream: int | None = None) -> Handle:
    """Builds the hierarchy of `graph` (an inputs.Graph or any object with n, row_ptr,
    col_idx, weight). Raises LamgError on a non-OK status."""
    keep: list = []
    g = _graph_struct(graph, device_input, keep)
    out = C.c_void_p()
    s = raw_stream if raw_stream is not None else _stream_ptr(stream)
    st = _lib.lamg_setup(C.byref(g), C.byref(options) if options is not None else None, s,
                         C.byref(out))
    if st != OK:
        raise LamgError(st, "lamg_setup")
    return Handle(out, int(graph.n))


def lamg_setup_status(graph, options: lamg_options | None = None) -> int:
    """Status of lamg_setup on a host-memory graph, without raising (input checks)."""
    keep: list = []
    g = _graph_struct(graph, False, keep)
    out = C.c_void_p()
    st = _lib.lamg_setup(C.byref(g), C.byref(options) if options is not None else None, None,
                         C.byref(out))
    if st == OK:
        _lib.lamg_destroy(out)
    return st


def lamg_solve(h: Handle, b, phi, tol: float = 1e-8, max_cycles: int = 300,
               precision: int = FP64, stream=None, history: bool = False, check: bool = True):
    """Solves for the columns of b: torch float64 device tensors of shape (k, n) (row j is
    right-hand side j) or (n,). phi receives the solutions. Returns a dict of statistics."""
    return _solve(_lib.lamg_solve, "lamg_solve", h, b, phi, tol, max_cycles, precision, stream,
                  history, check)


def lamg_solve_noalloc(h: Handle, b, phi, tol: float = 1e-8, max_cycles: int = 300,
                       precision: int = FP64, stream=None, history: bool = False,
                       check: bool = True):
    """lamg_solve through the allocation-free entry point (workspace in the library's fixed
    device scratch array; status SCRATCH_TOO_SMALL when it does not fit)."""
    return _solve(_lib.lamg_solve_noalloc, "lamg_solve_noalloc", h, b, phi, tol, max_cycles,
                  precision, stream, history, check)


def _solve(fn, where, h, b, phi, tol, max_cycles, precision, stream, history, check):
    import torch

    if b.dtype != torch.float64 or phi.dtype != torch.float64 or not b.is_cuda or not phi.is_cuda:
        raise TypeError("b and phi must be float64 CUDA tensors")
    if not b.is_contiguous() or not phi.is_contiguous() or b.shape != phi.shape:
        raise ValueError("b and phi must be contiguous and of equal shape")
    k = 1 if b.dim() == 1 else int(b.shape[0])
    n = int(b.shape[-1])
    if n != h.n:
        raise ValueError(f"right-hand side length {n} != graph size {h.n}")
    rel = np.zeros(k)
    cyc = np.zeros(k, np.int32)
    hist = np.zeros(max(max_cycles, 300) + 1) if history else None
    info = lamg_solve_info()
    info.relres = rel.ctypes.data
    info.col_cycles = cyc.ctypes.data
    info.history = hist.ctypes.data if hist is not None else None
    st = fn(h.ptr, b.data_ptr(), k, float(tol), int(max_cycles), int(precision), phi.data_ptr(),
            C.byref(info), _stream_ptr(stream))
    if check and st not in (OK, NOT_CONVERGED):
        raise LamgError(st, where)
    out = dict(status=st, converged=(st == OK), cycles=int(info.cycles),
               relres_max=float(info.relres_max), acf_max=float(info.acf_max),
               seconds=float(info.seconds), relres=rel, col_cycles=cyc,
               graph_cycles=int(info.graph_cycles), bytes=float(info.bytes))
    if hist is not None:
        out["history"] = hist[: info.history_len].copy()
    return out


def lamg_solve_group(handles, bs, phis, tol: float = 1e-8, max_cycles: int = 300,
                     precision: int = FP32_IR, stream=None, check: bool = True):
    """Solves several requests together (lamg_solve_group): handles[r] with right-hand
    sides bs[r] into phis[r] (float64 CUDA tensors of shape (k_r, n_r) or (n_r,)). Returns
    one statistics dict per request, with its status."""
    import torch

    R = len(handles)
    if not (len(bs) == len(phis) == R):
        raise ValueError("one b and one phi per handle")
    hp = (C.c_void_p * R)()
    bp = (C.c_void_p * R)()
    pp = (C.c_void_p * R)()
    kk = (C.c_int32 * R)()
    rels, cycs = [], []
    infos = (lamg_solve_info * R)()
    for r, (h, b, phi) in enumerate(zip(handles, bs, phis)):
        if b.dtype != torch.float64 or phi.dtype != torch.float64 or not b.is_cuda \
                or not phi.is_cuda or not b.is_contiguous() or not phi.is_contiguous() \
                or b.shape != phi.shape:
            raise TypeError("b and phi must be contiguous float64 CUDA tensors of equal shape")
        k = 1 if b.dim() == 1 else int(b.shape[0])
        if int(b.shape[-1]) != h.n:
            raise ValueError(f"request {r}: right-hand side length {b.shape[-1]} != {h.n}")
        hp[r], bp[r], pp[r], kk[r] = h.ptr, b.data_ptr(), phi.data_ptr(), k
        rels.append(np.zeros(k))
        cycs.append(np.zeros(k, np.int32))
        infos[r].relres = rels[r].ctypes.data
        infos[r].col_cycles = cycs[r].ctypes.data
    sts = (C.c_int * R)()
    st = _lib.lamg_solve_group(R, hp, bp, kk, float(tol), int(max_cycles), int(precision), pp,
                               infos, sts, _stream_ptr(stream))
    if st == INVALID_ARG and all(s == 0 for s in sts):
        raise LamgError(st, "lamg_solve_group")
    out = []
    for r in range(R):
        if check and sts[r] not in (OK, NOT_CONVERGED):
            raise LamgError(sts[r], f"lamg_solve_group request {r}")
        i = infos[r]
        out.append(dict(status=int(sts[r]), converged=(sts[r] == OK), cycles=int(i.cycles),
                        relres_max=float(i.relres_max), acf_max=float(i.acf_max),
                        seconds=float(i.seconds), relres=rels[r], col_cycles=cycs[r],
                        bytes=float(i.bytes)))
    return out


def lamg_destroy(h: Handle) -> None:
    h.close()


def lamg_hierarchy_info(h: Handle) -> dict:
    info = lamg_hier_info()
    st = _lib.lamg_hierarchy_info(h.ptr, C.byref(info))
    if st != OK:
        raise LamgError(st, "lamg_hierarchy_info")
    L = info.levels
    return dict(levels=L, n=list(info.n[:L]), nnz=list(info.nnz[:L]),
                ncolors=list(info.ncolors[:L]), n_caliber2=list(info.n_caliber2[:L]),
                gamma=list(info.gamma[:L]), tau=list(info.tau[:L]),
                bytes_device=int(info.bytes_device), op_complexity=float(info.op_complexity),
                setup_seconds=float(info.setup_seconds), bytes_peak=int(info.bytes_peak),
                elim=[bool(e) for e in info.elim[:L]], tail_level=int(info.tail_level),
                timed_level=int(info.timed_level), cheb=[bool(c) for c in info.cheb[:L]],
                cheb_lmax=list(info.cheb_lmax[:L]), bjgs=[bool(c) for c in info.bjgs[:L]],
                reordered=bool(info.reordered),
                setup_phases=dict(zip(SETUP_PHASE_NAMES, info.setup_phase_seconds)))


def lamg_export_level(h: Handle, level: int) -> dict:
    """Copies one level (canonical operator and every setup artefact) to numpy arrays.
    Needs keep_setup_data=1 at setup."""
    hi = lamg_hierarchy_info(h)
    if not 0 <= level < hi["levels"]:
        raise IndexError(level)
    n, nnz = hi["n"][level], hi["nnz"][level]
    last = level == hi["levels"] - 1
    arrs = dict(row_ptr=np.empty(n + 1, np.int32), col_idx=np.empty(nnz, np.int32),
                val=np.empty(nnz))
    if hi["elim"][level]:
        arrs["aggregate"] = np.empty(n, np.int32)
    elif not last:
        arrs.update(color=np.empty(n, np.int32), strong=np.empty(nnz, np.uint8),
                    x=np.empty((n, 4)), affinity=np.empty(nnz), moments=np.empty((n, 9)),
                    seed=np.empty(n, np.int32), aggregate=np.empty(n, np.int32),
                    p0=np.empty(n, np.int32), p1=np.empty(n, np.int32), w0=np.empty(n),
                    w1=np.empty(n))
    ex = lamg_level_export()
    for name, a in arrs.items():
        setattr(ex, name, a.ctypes.data)
    st = _lib.lamg_export_level(h.ptr, int(level), C.byref(ex))
    if st != OK:
        raise LamgError(st, "lamg_export_level")
    return arrs


def lamg_profile_kernel(h: Handle, level: int, kernel: int, precision: int = FP64, nrhs: int = 1,
                        reps: int = 50, stream=None) -> tuple[float, float]:
    """(mean seconds per launch, algorithmic bytes per launch) of one cycle kernel."""
    sec = C.c_double()
    byt = C.c_double()
    st = _lib.lamg_profile_kernel(h.ptr, int(level), int(kernel), int(precision), int(nrhs),
                                  int(reps), C.byref(sec), C.byref(byt), _stream_ptr(stream))
    if st != OK:
        raise LamgError(st, "lamg_profile_kernel")
    return float(sec.value), float(byt.value)


def lamg_timing_start(h: Handle, max_launches: int = 16384) -> None:
    """Starts in-situ event timing of the cycle kernels of the timed level (timed_level in
    lamg_hierarchy_info) and of the coarse tail."""
    st = _lib.lamg_timing_start(h.ptr, int(max_launches))
    if st != OK:
        raise LamgError(st, "lamg_timing_start")


def lamg_timing_start_all(h: Handle, max_launches: int = 65536) -> None:
    """Starts in-situ event timing of every kernel launch of later solves, on every level,
    grouped by kernel kind."""
    st = _lib.lamg_timing_start_all(h.ptr, int(max_launches))
    if st != OK:
        raise LamgError(st, "lamg_timing_start_all")


def lamg_timing_stop(h: Handle) -> dict:
    """Stops timing; returns {(kernel, precision): dict(launches, seconds, bytes)} for every
    kernel and precision with at least one timed launch."""
    st = _lib.lamg_timing_stop(h.ptr)
    if st != OK:
        raise LamgError(st, "lamg_timing_stop")
    out = {}
    for kern in range(len(KERNEL_NAMES)):
        for prec in (FP64, FP32_IR):
            t = lamg_kernel_time()
            st = _lib.lamg_timing_get(h.ptr, kern, prec, C.byref(t))
            if st != OK:
                raise LamgError(st, "lamg_timing_get")
            if t.launches:
                out[(kern, prec)] = dict(launches=int(t.launches), seconds=float(t.seconds),
                                         bytes=float(t.bytes))
    return out
