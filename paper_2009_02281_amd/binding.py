"""Thin ctypes binding of ``libaimx.so`` (the C ABI in include/aim.h).

Argument marshalling only: every step of the operator and of the solver runs
in the library's HIP kernels.  PyTorch supplies device memory and streams.
There is no fallback: if the library is not built, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libaimx.so")

AIM_OK = 0
STATUS = {0: "AIM_OK", 1: "AIM_ERR_INVALID_ARG", 2: "AIM_ERR_GEOMETRY", 3: "AIM_ERR_GRID",
          4: "AIM_ERR_OOM", 5: "AIM_ERR_DEVICE", 6: "AIM_ERR_NOT_CONVERGED",
          7: "AIM_ERR_BREAKDOWN", 8: "AIM_ERR_STATE"}
PREC = {"c128": 0, "c64": 1}
PC = {"none": 0, "diag": 1, "nearblock": 2, "unet": 3, "nearblock_static": 4}
LOSS = {"error": 0, "residual": 1}
FFT_SHAPES = 12         # AIM_FFT_SHAPES
FFT_LAYOUTS = 4         # AIM_FFT_LAYOUTS
SCHEDULE_LEN = 7        # AIM_SCHEDULE_LEN: five pass shapes, the layout, the stage modes
STAGE = {"project": 0, "convolve": 1, "interpolate": 2, "near": 3, "learned_pc": 4,
         "nearblock_pc": 5}
RHS = {"plane_wave": 0, "gaussian_patch": 1}

EXPORTED = ["aim_setup", "aim_setup_host", "aim_destroy", "aim_plan_query", "aim_matvec",
            "aim_matvec_static", "aim_conventional_fill", "aim_matvec_conventional",
            "aim_conventional_export", "aim_matvec_dlp", "aim_dlp_export",
            "aim_efie_setup", "aim_matvec_efie", "aim_efie_export", "aim_matvec_mfie",
            "aim_mfie_export", "aim_matvec_cfie", "aim_rwg_excitation",
            "aim_solve_rwg",
            "aim_export_clusters", "aim_set_lin_term",
            "aim_export_lin_diag", "aim_apply_stage",
            "aim_excitation", "aim_solve", "aim_export_tables", "aim_profile_matvec",
            "aim_autotune", "aim_set_schedule", "aim_matvec_capture", "aim_graph_launch",
            "aim_graph_destroy", "aim_unet_create", "aim_unet_destroy", "aim_unet_num_params",
            "aim_unet_get_params", "aim_unet_set_params", "aim_unet_forward",
            "aim_unet_train_grid", "aim_unet_save", "aim_unet_load",
            "aim_plan_set_unet", "aim_log_pairs", "aim_pc_targets", "aim_pc_train_step",
            "aim_plan_save", "aim_plan_load", "aim_plan_load_host", "aim_setup_batch",
            "aim_batch_sizes",
            "aim_last_error", "aim_version"]
KERNELS = ["project", "fft_x_fwd", "fft_y_fwd", "fft_z_conv", "fft_y_inv", "fft_x_inv",
           "interp_near"]


class AimError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class SetupDesc(C.Structure):
    _fields_ = [
        ("n_vertices", C.c_int64), ("n_triangles", C.c_int64),
        ("vertices", C.c_void_p), ("triangles", C.c_void_p),
        ("stencil_order", C.c_int32), ("grid_dims", C.c_int32 * 3),
        ("h", C.c_double), ("near_threshold", C.c_double),
        ("n_freq", C.c_int32), ("k", C.c_void_p),
        ("precisions", C.c_uint32), ("max_rhs", C.c_int32), ("n_threads", C.c_int32),
        ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", C.c_void_p),
    ]


class PlanInfo(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("n_grid", C.c_int64), ("nnz", C.c_int64),
        ("dims", C.c_int32 * 3), ("order", C.c_int32), ("n_freq", C.c_int32),
        ("max_rhs", C.c_int32), ("precisions", C.c_uint32), ("h", C.c_double),
        ("origin", C.c_double * 3), ("setup_seconds", C.c_double),
        ("spectra_seconds", C.c_double), ("device_bytes", C.c_int64),
        ("n_clusters", C.c_int32), ("max_cluster", C.c_int32),
        ("near_seconds", C.c_double), ("near_on_device", C.c_int32), ("reserved", C.c_int32),
    ]


class SolveOpts(C.Structure):
    _fields_ = [
        ("rtol", C.c_double), ("restart", C.c_int32), ("max_iter", C.c_int32),
        ("max_refine", C.c_int32), ("inner", C.c_int32), ("pc", C.c_int32),
        ("inner_rtol", C.c_double), ("fallback_pc", C.c_int32), ("gate", C.c_double),
    ]


class SolveInfo(C.Structure):
    _fields_ = [
        ("iters", C.c_int32), ("refinements", C.c_int32), ("matvecs", C.c_int32),
        ("fallback_used", C.c_int32), ("converged", C.c_int32),
        ("rel_resid", C.c_double), ("seconds", C.c_double),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads the library (once) and declares the signatures.  Raises
    FileNotFoundError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is missing: build it with `python -m paper_2009_02281_amd.build`")
    lib = C.CDLL(path)
    vp, i32, ip32 = C.c_void_p, C.c_int32, C.POINTER(C.c_int32)
    lib.aim_setup.argtypes = [C.POINTER(SetupDesc), vp, C.POINTER(vp)]
    lib.aim_setup_host.argtypes = [C.POINTER(SetupDesc), C.POINTER(vp)]
    lib.aim_destroy.argtypes = [vp]
    lib.aim_plan_query.argtypes = [vp, C.POINTER(PlanInfo)]
    lib.aim_matvec.argtypes = [vp, i32, vp, vp, i32, ip32, vp]
    lib.aim_conventional_fill.argtypes = [vp, i32, vp]
    lib.aim_export_clusters.argtypes = [vp, ip32, ip32]
    lib.aim_set_lin_term.argtypes = [vp, i32]
    lib.aim_export_lin_diag.argtypes = [vp, C.POINTER(C.c_double)]
    lib.aim_matvec_conventional.argtypes = [vp, i32, vp, vp, i32, vp]
    lib.aim_conventional_export.argtypes = [vp, C.POINTER(C.c_double), vp]
    lib.aim_matvec_dlp.argtypes = [vp, vp, vp, i32, C.POINTER(C.c_int32), vp]
    lib.aim_dlp_export.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double), vp]
    lib.aim_efie_setup.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_double), vp]
    lib.aim_matvec_efie.argtypes = [vp, i32, vp, vp, i32, C.POINTER(C.c_int32), vp]
    lib.aim_matvec_mfie.argtypes = [vp, i32, vp, vp, i32, C.POINTER(C.c_int32), C.c_double, vp]
    lib.aim_matvec_cfie.argtypes = [vp, i32, vp, vp, i32, C.POINTER(C.c_int32), C.c_double, vp]
    lib.aim_rwg_excitation.argtypes = [vp, i32, C.POINTER(C.c_double), i32,
                                       C.POINTER(C.c_int32), vp, vp]
    lib.aim_solve_rwg.argtypes = [vp, i32, C.c_double, vp, vp, i32, C.POINTER(C.c_int32),
                                  C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]
    lib.aim_mfie_export.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.POINTER(C.c_double), vp]
    lib.aim_efie_export.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                    C.POINTER(C.c_double), vp]
    lib.aim_matvec_static.argtypes = [vp, i32, vp, vp, i32, ip32, vp]
    lib.aim_apply_stage.argtypes = [vp, i32, i32, vp, vp, i32, ip32, vp]
    lib.aim_excitation.argtypes = [vp, i32, C.POINTER(C.c_double), i32, i32, ip32, vp, vp]
    lib.aim_solve.argtypes = [vp, vp, vp, i32, ip32, C.POINTER(SolveOpts),
                              C.POINTER(SolveInfo), vp]
    lib.aim_export_tables.argtypes = [vp, ip32, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                      ip32, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.aim_profile_matvec.argtypes = [vp, i32, vp, vp, i32, ip32, i32,
                                       C.POINTER(C.c_double), vp]
    lib.aim_matvec_capture.argtypes = [vp, i32, vp, vp, i32, ip32, vp, C.POINTER(vp)]
    lib.aim_graph_launch.argtypes = [vp, vp]
    lib.aim_graph_destroy.argtypes = [vp]
    fp = C.POINTER(C.c_float)
    lib.aim_unet_create.argtypes = [i32, C.c_uint64, C.POINTER(vp)]
    lib.aim_unet_destroy.argtypes = [vp]
    lib.aim_unet_num_params.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.aim_unet_get_params.argtypes = [vp, fp, fp]
    lib.aim_unet_set_params.argtypes = [vp, fp]
    lib.aim_unet_forward.argtypes = [vp, vp, vp, i32, ip32, vp]
    lib.aim_unet_train_grid.argtypes = [vp, vp, vp, i32, ip32, C.c_double, i32,
                                        C.POINTER(C.c_double), vp]
    lib.aim_unet_save.argtypes = [vp, C.c_char_p]
    lib.aim_unet_load.argtypes = [C.c_char_p, C.POINTER(vp)]
    lib.aim_autotune.argtypes = [vp, i32, i32, i32, ip32, C.POINTER(C.c_double), vp]
    lib.aim_set_schedule.argtypes = [vp, i32, ip32]
    dp = C.POINTER(C.c_double)
    lib.aim_plan_set_unet.argtypes = [vp, vp, i32, C.c_double]
    lib.aim_log_pairs.argtypes = [vp, vp, i32, ip32, C.c_double, i32, i32, vp, vp, ip32, i32,
                                  ip32, vp]
    lib.aim_pc_targets.argtypes = [vp, i32, i32, vp, vp, i32, vp, vp, dp, vp]
    lib.aim_pc_train_step.argtypes = [vp, vp, i32, vp, vp, i32, ip32, i32, C.c_double,
                                      C.c_double, C.c_double, i32, dp, vp]
    lib.aim_setup_batch.argtypes = [C.POINTER(SetupDesc), i32, vp, C.POINTER(vp)]
    lib.aim_batch_sizes.argtypes = [vp, ip32, C.POINTER(C.c_int64)]
    lib.aim_plan_save.argtypes = [vp, C.c_char_p]
    lib.aim_plan_load.argtypes = [C.c_char_p, ALLOC_FN, FREE_FN, vp, vp, C.POINTER(vp)]
    lib.aim_plan_load_host.argtypes = [C.c_char_p, C.POINTER(vp)]
    lib.aim_last_error.restype = C.c_char_p
    lib.aim_version.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("aim_last_error", "aim_version"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != AIM_OK:
        raise AimError(status, load_library().aim_last_error().decode())


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _freq_arg(freq_idx, nrhs):
    if freq_idx is None:
        return None, None
    arr = np.ascontiguousarray(np.broadcast_to(np.asarray(freq_idx, dtype=np.int32), (nrhs,)))
    return arr, arr.ctypes.data_as(C.POINTER(C.c_int32))


@dataclass
class SolveResult:
    iters: np.ndarray
    refinements: np.ndarray
    matvecs: np.ndarray
    converged: np.ndarray
    rel_resid: np.ndarray
    seconds: float
    status: int
    fallback_used: np.ndarray = None


class UNet:
    """The learned grid preconditioner network (see aim_unet_* in aim.h)."""

    def __init__(self, seed: int = 0, base_channels: int = 16, handle=None):
        self._lib = load_library()
        self._h = C.c_void_p()
        if handle is not None:
            self._h = handle
        else:
            _check(self._lib.aim_unet_create(base_channels, seed, C.byref(self._h)))
        n = C.c_int64()
        _check(self._lib.aim_unet_num_params(self._h, C.byref(n)))
        self.nparam = int(n.value)

    @classmethod
    def load(cls, path: str):
        lib = load_library()
        h = C.c_void_p()
        _check(lib.aim_unet_load(path.encode(), C.byref(h)))
        return cls(handle=h)

    def save(self, path: str):
        _check(self._lib.aim_unet_save(self._h, path.encode()))

    def params(self) -> np.ndarray:
        out = np.empty(self.nparam, dtype=np.float32)
        _check(self._lib.aim_unet_get_params(self._h, out.ctypes.data_as(C.POINTER(C.c_float)),
                                             None))
        return out

    def grads(self) -> np.ndarray:
        out = np.empty(self.nparam, dtype=np.float32)
        _check(self._lib.aim_unet_get_params(self._h, None,
                                             out.ctypes.data_as(C.POINTER(C.c_float))))
        return out

    def set_params(self, p):
        arr = np.ascontiguousarray(p, dtype=np.float32)
        assert arr.size == self.nparam
        _check(self._lib.aim_unet_set_params(self._h, arr.ctypes.data_as(C.POINTER(C.c_float))))

    @staticmethod
    def _dims(t):
        nz, ny, nx = t.shape[-3:]
        return (C.c_int32 * 3)(nx, ny, nz)

    def forward(self, grid, stream=None):
        """grid: complex64 CUDA tensor [nbatch, Nz, Ny, Nx] (or 3-D)."""
        import torch
        g = grid.reshape((-1,) + tuple(grid.shape[-3:]))
        assert g.dtype == torch.complex64 and g.is_cuda and g.is_contiguous()
        out = torch.empty_like(g)
        _check(self._lib.aim_unet_forward(self._h, C.c_void_p(g.data_ptr()),
                                          C.c_void_p(out.data_ptr()), g.shape[0], self._dims(g),
                                          _stream_ptr(stream)))
        return out.reshape(grid.shape)

    def train_grid(self, grid, target, lr: float = 1e-3, apply: bool = True, stream=None) -> float:
        g = grid.reshape((-1,) + tuple(grid.shape[-3:]))
        t = target.reshape(g.shape)
        loss = C.c_double()
        _check(self._lib.aim_unet_train_grid(self._h, C.c_void_p(g.data_ptr()),
                                             C.c_void_p(t.data_ptr()), g.shape[0], self._dims(g),
                                             float(lr), 1 if apply else 0, C.byref(loss),
                                             _stream_ptr(stream)))
        return float(loss.value)

    def close(self):
        if self._h and self._h.value:
            _check(self._lib.aim_unet_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def unet_params_to_layers(flat, C0: int = 16):
    """Splits the flat parameter vector into [(W[co, t, ci], b[co]), ...]."""
    c0, c1, c2 = C0, 2 * C0, 4 * C0
    spec = [(c0, 2, 27), (c0, c0, 27), (c1, c0, 27), (c1, c1, 27), (c2, c1, 27), (c2, c2, 27),
            (c1, c2 + c1, 27), (c1, c1, 27), (c0, c1 + c0, 27), (c0, c0, 27), (2, c0, 1)]
    out, off = [], 0
    for co, ci, t in spec:
        W = np.asarray(flat[off:off + co * t * ci], dtype=np.float64).reshape(co, t, ci)
        off += co * t * ci
        b = np.asarray(flat[off:off + co], dtype=np.float64)
        off += co
        out.append((W, b))
    assert off == len(flat)
    return out


class MatvecGraph:
    """A captured matvec (see aim_matvec_capture); keeps its tensors alive."""

    def __init__(self, lib, handle, keep):
        self._lib, self._g, self._keep = lib, handle, keep

    def launch(self, stream=None):
        _check(self._lib.aim_graph_launch(self._g, _stream_ptr(stream)))

    def close(self):
        if self._g and self._g.value:
            _check(self._lib.aim_graph_destroy(self._g))
            self._g = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _make_desc(vertices, triangles, order, dims, h, near_threshold, k, precisions, max_rhs,
               n_threads=0):
    """aim_setup_desc and the arrays it points into (keep them alive)."""
    V = np.ascontiguousarray(vertices, dtype=np.float64)
    T = np.ascontiguousarray(triangles, dtype=np.int32)
    kk = np.ascontiguousarray(np.atleast_1d(np.asarray(k, dtype=np.float64)))
    d = SetupDesc()
    d.n_vertices = V.shape[0]
    d.n_triangles = T.shape[0]
    d.vertices = V.ctypes.data
    d.triangles = T.ctypes.data
    d.stencil_order = int(order)
    for a in range(3):
        d.grid_dims[a] = int(dims[a])
    d.h = float(h)
    d.near_threshold = float(near_threshold)
    d.n_freq = kk.size
    d.k = kk.ctypes.data
    d.precisions = sum(1 << PREC[p] for p in precisions)
    d.max_rhs = int(max_rhs)
    d.n_threads = int(n_threads)
    return d, (V, T, kk)


class TorchAllocator:
    """Device memory for a plan from PyTorch's caching allocator, passed to
    aim_setup as its allocator callbacks (aim_alloc_fn / aim_free_fn).  Counts
    the live blocks so a caller can see that everything came back."""

    def __init__(self):
        import torch
        self._torch = torch
        self.live = {}
        self.calls = 0
        self._alloc = ALLOC_FN(self._do_alloc)
        self._free = FREE_FN(self._do_free)

    def _do_alloc(self, nbytes, stream, ctx):
        try:
            ptr = int(self._torch.cuda.caching_allocator_alloc(max(int(nbytes), 1)))
        except Exception:  # noqa: BLE001 - the library reports AIM_ERR_OOM for NULL
            return None
        self.live[ptr] = int(nbytes)
        self.calls += 1
        return ptr

    def _do_free(self, ptr, stream, ctx):
        if ptr:
            self.live.pop(int(ptr), None)
            self._torch.cuda.caching_allocator_delete(int(ptr))


class Plan:
    """An AIMx operator for one mesh, grid and frequency set (see aim_setup)."""

    def __init__(self, vertices, triangles, order: int, dims, h: float, near_threshold: float,
                 k, precisions=("c128", "c64"), max_rhs: int = 1, n_threads: int = 0,
                 stream=None, host_only: bool = False, allocator=None):
        """``allocator``: None (the library's own hipMalloc) or a
        TorchAllocator, which the plan keeps until it is closed."""
        lib = load_library()
        self._lib = lib
        d, keep = _make_desc(vertices, triangles, order, dims, h, near_threshold, k, precisions,
                             max_rhs, n_threads)
        self._allocator = allocator
        if allocator is not None:
            d.alloc = allocator._alloc
            d.free = allocator._free
        kk = keep[2]
        self._plan = C.c_void_p()
        self.precisions = tuple(precisions)
        self.host_only = host_only
        if host_only:
            _check(lib.aim_setup_host(C.byref(d), C.byref(self._plan)))
        else:
            import torch
            torch.cuda.init()
            _check(lib.aim_setup(C.byref(d), _stream_ptr(stream), C.byref(self._plan)))
        self.k = kk
        self._finish()

    def _finish(self):
        info = self.info()
        self.n = int(info["n"])
        self.dims = tuple(info["dims"])
        self.n_grid = int(info["n_grid"])
        self.max_rhs = int(info["max_rhs"])

    @classmethod
    def setup_batch(cls, workloads, precisions=("c128", "c64"), stream=None):
        """One plan over several geometries of uneven size (aim_setup_batch).
        ``workloads`` are objects with vertices, triangles, order, dims, h,
        near_threshold and k.  Vectors are [n][N_max] with zero padding; use
        pack/unpack."""
        import torch
        lib = load_library()
        n = len(workloads)
        descs = (SetupDesc * n)()
        keep = []
        for i, w in enumerate(workloads):
            d, kp = _make_desc(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold,
                               w.k, precisions, 1)
            descs[i] = d
            keep.append(kp)
        self = cls.__new__(cls)
        self._lib = lib
        self._plan = C.c_void_p()
        self.host_only = False
        self.precisions = tuple(precisions)
        torch.cuda.init()
        _check(lib.aim_setup_batch(descs, n, _stream_ptr(stream), C.byref(self._plan)))
        self.k = None
        self._finish()
        cnt = C.c_int32(0)
        sizes = (C.c_int64 * n)()
        _check(lib.aim_batch_sizes(self._plan, C.byref(cnt), sizes))
        self.batch_sizes = [int(v) for v in sizes]
        return self

    def pack(self, vectors, dtype=None):
        """[n][N_max] device tensor from n vectors of the instances' sizes."""
        import torch
        dt = dtype or torch.complex128
        out = torch.zeros((len(self.batch_sizes), self.n), dtype=dt, device="cuda")
        for i, v in enumerate(vectors):
            t = torch.as_tensor(v).to(dt).to("cuda")
            out[i, :self.batch_sizes[i]] = t.reshape(-1)
        return out

    def unpack(self, t):
        """List of the instances' vectors from a [n][N_max] tensor."""
        return [t[i, :m] for i, m in enumerate(self.batch_sizes)]

    def save(self, path: str):
        """Checkpoint of the plan's host tables and schedules (aim_plan_save)."""
        _check(self._lib.aim_plan_save(self._plan, str(path).encode()))

    @classmethod
    def load(cls, path: str, host_only: bool = False, stream=None):
        """Plan from a checkpoint, without the host set-up (aim_plan_load)."""
        lib = load_library()
        self = cls.__new__(cls)
        self._lib = lib
        self._plan = C.c_void_p()
        self.host_only = host_only
        if host_only:
            _check(lib.aim_plan_load_host(str(path).encode(), C.byref(self._plan)))
        else:
            import torch
            torch.cuda.init()
            _check(lib.aim_plan_load(str(path).encode(), ALLOC_FN(), FREE_FN(), None,
                                     _stream_ptr(stream), C.byref(self._plan)))
        info = self.info()
        self.precisions = tuple(name for name, bit in PREC.items() if info["precisions"] >> bit & 1)
        self.k = None
        self._finish()
        return self

    # -- lifetime -------------------------------------------------------------
    def close(self):
        if getattr(self, "_plan", None) and self._plan.value:
            _check(self._lib.aim_destroy(self._plan))
            self._plan = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- queries ------------------------------------------------------------
    def info(self) -> dict:
        pi = PlanInfo()
        _check(self._lib.aim_plan_query(self._plan, C.byref(pi)))
        return {
            "n": pi.n, "n_grid": pi.n_grid, "nnz": pi.nnz, "dims": list(pi.dims),
            "order": pi.order, "n_freq": pi.n_freq, "max_rhs": pi.max_rhs,
            "precisions": pi.precisions, "h": pi.h, "origin": list(pi.origin),
            "setup_seconds": pi.setup_seconds, "spectra_seconds": pi.spectra_seconds,
            "device_bytes": pi.device_bytes, "n_clusters": pi.n_clusters,
            "max_cluster": pi.max_cluster, "near_seconds": pi.near_seconds,
            "near_on_device": bool(pi.near_on_device),
        }

    def export_tables(self) -> dict:
        info = self.info()
        n, nnz = int(info["n"]), int(info["nnz"])
        ss = np.empty((3 * n, 3), dtype=np.int32)
        sl = np.empty((3 * n, 3), dtype=np.float64)
        rp = np.empty(n + 1, dtype=np.int64)
        col = np.empty(nnz, dtype=np.int32)
        val = np.empty(nnz, dtype=np.float64)
        ns = np.empty(nnz, dtype=np.float64)
        P = lambda a, t: a.ctypes.data_as(C.POINTER(t))
        _check(self._lib.aim_export_tables(self._plan, P(ss, C.c_int32), P(sl, C.c_double),
                                           P(rp, C.c_int64), P(col, C.c_int32),
                                           P(val, C.c_double), P(ns, C.c_double)))
        return {"stencil_start": ss, "stencil_local": sl, "rowptr": rp, "col": col,
                "val": val, "near_static": ns}

    # -- device work ------------------------------------------------------------
    @staticmethod
    def _dtype(prec):
        import torch
        return torch.complex128 if prec == "c128" else torch.complex64

    def _check_vec(self, t, prec, length, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA tensor")
        if t.dtype != self._dtype(prec):
            raise TypeError(f"{name} must be {self._dtype(prec)}")
        if not t.is_contiguous() or t.shape[-1] != length:
            raise ValueError(f"{name} must be contiguous with last dimension {length}")

    def matvec(self, x, freq_idx=None, prec: str = "c128", out=None, stream=None):
        """y = A(k_f) x for x of shape [N] or [nrhs, N]."""
        import torch
        self._check_vec(x, prec, self.n, "x")
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        y = torch.empty_like(x) if out is None else out
        self._check_vec(y, prec, self.n, "out")
        _, fp = _freq_arg(freq_idx, nrhs)
        _check(self._lib.aim_matvec(self._plan, PREC[prec], C.c_void_p(x.data_ptr()),
                                    C.c_void_p(y.data_ptr()), nrhs, fp, _stream_ptr(stream)))
        return y

    def matvec_static(self, x, freq_idx=None, prec: str = "c128", out=None, stream=None):
        """y = A(k_f) x through aim_matvec_static (no allocation in the call:
        scratch in the library's fixed device array)."""
        import torch
        self._check_vec(x, prec, self.n, "x")
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        y = torch.empty_like(x) if out is None else out
        self._check_vec(y, prec, self.n, "out")
        _, fp = _freq_arg(freq_idx, nrhs)
        _check(self._lib.aim_matvec_static(self._plan, PREC[prec], C.c_void_p(x.data_ptr()),
                                           C.c_void_p(y.data_ptr()), nrhs, fp,
                                           _stream_ptr(stream)))
        return y

    def set_lin_term(self, on: bool = True):
        """Adds (or removes) the linear-term modification k^2 D x to every
        matvec and solve of the plan (aim_set_lin_term)."""
        _check(self._lib.aim_set_lin_term(self._plan, 1 if on else 0))

    def lin_diagonal(self) -> np.ndarray:
        """The linear-term diagonal D, float64 [N]."""
        out = np.empty(int(self.info()["n"]), dtype=np.float64)
        _check(self._lib.aim_export_lin_diag(self._plan, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def export_clusters(self):
        """The near-block preconditioner's clusters: a list of index arrays."""
        info = self.info()
        ptr = np.empty(int(info["n_clusters"]) + 1, dtype=np.int32)
        perm = np.empty(int(info["n"]), dtype=np.int32)
        _check(self._lib.aim_export_clusters(self._plan,
                                             ptr.ctypes.data_as(C.POINTER(C.c_int32)),
                                             perm.ctypes.data_as(C.POINTER(C.c_int32))))
        return [perm[ptr[c]:ptr[c + 1]].copy() for c in range(len(ptr) - 1)]

    def conventional_fill(self, freq_idx: int = 0, stream=None):
        """Conventional AIM: builds the complex near correction of wavenumber
        ``freq_idx`` on the device (aim_conventional_fill)."""
        _check(self._lib.aim_conventional_fill(self._plan, int(freq_idx), _stream_ptr(stream)))

    def matvec_conventional(self, x, prec: str = "c128", out=None, stream=None):
        """y = W H(k) P x + C(k) x with the last filled conventional
        correction."""
        import torch
        self._check_vec(x, prec, self.n, "x")
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        y = torch.empty_like(x) if out is None else out
        self._check_vec(y, prec, self.n, "out")
        _check(self._lib.aim_matvec_conventional(self._plan, PREC[prec], C.c_void_p(x.data_ptr()),
                                                 C.c_void_p(y.data_ptr()), nrhs,
                                                 _stream_ptr(stream)))
        return y

    def conventional_values(self, stream=None) -> np.ndarray:
        """The filled conventional correction, complex128 [nnz] in near-list
        order."""
        nnz = int(self.info()["nnz"])
        out = np.empty(2 * nnz, dtype=np.float64)
        _check(self._lib.aim_conventional_export(
            self._plan, out.ctypes.data_as(C.POINTER(C.c_double)), _stream_ptr(stream)))
        return out.view(np.complex128)

    def matvec_dlp(self, x, freq_idx=None, out=None, stream=None):
        """y = K x, the double-layer operator under AIMx (complex128)."""
        import torch
        self._check_vec(x, "c128", self.n, "x")
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        y = torch.empty_like(x) if out is None else out
        self._check_vec(y, "c128", self.n, "out")
        _, fp = _freq_arg(freq_idx, nrhs)
        _check(self._lib.aim_matvec_dlp(self._plan, C.c_void_p(x.data_ptr()),
                                        C.c_void_p(y.data_ptr()), nrhs, fp,
                                        _stream_ptr(stream)))
        return y

    def dlp_values(self, stream=None):
        """(K_s,NR, C_K) of the double-layer operator on the near list."""
        nnz = int(self.info()["nnz"])
        near = np.empty(max(nnz, 1), dtype=np.float64)
        corr = np.empty(max(nnz, 1), dtype=np.float64)
        _check(self._lib.aim_dlp_export(self._plan, near.ctypes.data_as(C.POINTER(C.c_double)),
                                        corr.ctypes.data_as(C.POINTER(C.c_double)),
                                        _stream_ptr(stream)))
        return near[:nnz], corr[:nnz]

    def efie_setup(self, stream=None) -> dict:
        """Builds the RWG EFIE tables; returns the number of functions, the
        near-list length and the build time."""
        n, nnz, sec = C.c_int64(), C.c_int64(), C.c_double()
        _check(self._lib.aim_efie_setup(self._plan, C.byref(n), C.byref(nnz), C.byref(sec),
                                        _stream_ptr(stream)))
        return {"n_rwg": int(n.value), "nnz": int(nnz.value), "seconds": float(sec.value)}

    def matvec_efie(self, x, freq_idx=None, out=None, stream=None, prec: str = "c128"):
        """y = Z x, the RWG EFIE operator under AIMx (x of [n_rwg] or
        [nrhs, n_rwg], complex128 or, with prec="c64", complex64)."""
        import torch
        n = self.efie_setup(stream)["n_rwg"]
        self._check_vec(x, prec, n, "x")
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        y = torch.empty_like(x) if out is None else out
        self._check_vec(y, prec, n, "out")
        _, fp = _freq_arg(freq_idx, nrhs)
        _check(self._lib.aim_matvec_efie(self._plan, PREC[prec], C.c_void_p(x.data_ptr()),
                                         C.c_void_p(y.data_ptr()), nrhs, fp,
                                         _stream_ptr(stream)))
        return y

    def matvec_mfie(self, x, freq_idx=None, gram_coef: float = 0.0, out=None, stream=None,
                    prec: str = "c128"):
        """y = (K + gram_coef G) x, the RWG double layer under AIMx (x of
        [n_rwg] or [nrhs, n_rwg], complex128 or complex64)."""
        import torch
        n = self.efie_setup(stream)["n_rwg"]
        self._check_vec(x, prec, n, "x")
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        y = torch.empty_like(x) if out is None else out
        self._check_vec(y, prec, n, "out")
        _, fp = _freq_arg(freq_idx, nrhs)
        _check(self._lib.aim_matvec_mfie(self._plan, PREC[prec], C.c_void_p(x.data_ptr()),
                                         C.c_void_p(y.data_ptr()), nrhs, fp,
                                         float(gram_coef), _stream_ptr(stream)))
        return y

    def matvec_cfie(self, x, freq_idx=None, gram_coef: float = 0.0, out=None, stream=None,
                    prec: str = "c128"):
        """y = Z x + (j/k)(K + gram_coef G) x, the combined-field operator
        (x of [n_rwg] or [nrhs, n_rwg], complex128 or complex64)."""
        import torch
        n = self.efie_setup(stream)["n_rwg"]
        self._check_vec(x, prec, n, "x")
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        y = torch.empty_like(x) if out is None else out
        self._check_vec(y, prec, n, "out")
        _, fp = _freq_arg(freq_idx, nrhs)
        _check(self._lib.aim_matvec_cfie(self._plan, PREC[prec], C.c_void_p(x.data_ptr()),
                                         C.c_void_p(y.data_ptr()), nrhs, fp,
                                         float(gram_coef), _stream_ptr(stream)))
        return y

    def rwg_excitation(self, direction, pol, field: str = "E", nrhs=None, freq_idx=None,
                       stream=None):
        """Plane waves tested with the RWG functions: field "E" <f, pol e^{-jk d.r}>,
        "H" <f, n x (d x pol) e^{-jk d.r}>; direction and pol of shape [3] or
        [nrhs, 3].  Returns [nrhs, n_rwg] complex128."""
        import torch
        n = self.efie_setup(stream)["n_rwg"]
        d = np.atleast_2d(np.asarray(direction, dtype=np.float64))
        p = np.atleast_2d(np.asarray(pol, dtype=np.float64))
        nr = max(d.shape[0], p.shape[0]) if nrhs is None else int(nrhs)
        prm = np.ascontiguousarray(np.concatenate([np.broadcast_to(d, (nr, 3)),
                                                   np.broadcast_to(p, (nr, 3))], axis=1))
        b = torch.empty((nr, n), dtype=torch.complex128, device="cuda")
        _, fp = _freq_arg(freq_idx, nr)
        _check(self._lib.aim_rwg_excitation(self._plan, 0 if field == "E" else 1,
                                            prm.ctypes.data_as(C.POINTER(C.c_double)), nr, fp,
                                            C.c_void_p(b.data_ptr()), _stream_ptr(stream)))
        return b

    def solve_rwg(self, op: str, b, x0=None, freq_idx=None, gram_coef: float = -0.5,
                  rtol: float = 1e-6, restart: int = 30, max_iter: int = 1000, stream=None,
                  raise_on_fail=True):
        """Batched GMRES on an RWG operator (op "efie", "mfie" for K + gram G,
        "cfie" for Z + (j/k)(K + gram G)); b of shape [nrhs, n_rwg].  Returns
        (x, SolveResult)."""
        import torch
        n = self.efie_setup(stream)["n_rwg"]
        b2 = b.reshape(-1, n)
        self._check_vec(b2, "c128", n, "b")
        nrhs = b2.shape[0]
        x = torch.zeros_like(b2) if x0 is None else x0.reshape(-1, n).clone()
        opts = SolveOpts(rtol, restart, max_iter, 0, PREC["c128"], PC["none"], 0.0, PC["none"],
                         0.0)
        infos = (SolveInfo * nrhs)()
        _, fp = _freq_arg(freq_idx, nrhs)
        code = {"efie": 1, "mfie": 2, "cfie": 3}[op]
        st = self._lib.aim_solve_rwg(self._plan, code, float(gram_coef),
                                     C.c_void_p(b2.data_ptr()), C.c_void_p(x.data_ptr()), nrhs,
                                     fp, C.byref(opts), infos, _stream_ptr(stream))
        if st not in (AIM_OK, 6) or (st == 6 and raise_on_fail):
            _check(st)
        res = SolveResult(
            iters=np.array([i.iters for i in infos]),
            refinements=np.array([i.refinements for i in infos]),
            matvecs=np.array([i.matvecs for i in infos]),
            converged=np.array([bool(i.converged) for i in infos]),
            rel_resid=np.array([i.rel_resid for i in infos]),
            seconds=float(infos[0].seconds) if nrhs else 0.0, status=st,
            fallback_used=np.array([bool(i.fallback_used) for i in infos]))
        return x.reshape(b.shape), res

    def mfie_values(self, stream=None) -> dict:
        """C_K and the Gram entries on the RWG near list, and the build time."""
        nnz = self.efie_setup(stream)["nnz"]
        ck = np.empty(max(nnz, 1), dtype=np.float64)
        gr = np.empty(max(nnz, 1), dtype=np.float64)
        sec = C.c_double()
        F64 = C.POINTER(C.c_double)
        _check(self._lib.aim_mfie_export(self._plan, ck.ctypes.data_as(F64),
                                         gr.ctypes.data_as(F64), C.byref(sec),
                                         _stream_ptr(stream)))
        return {"ck": ck[:nnz], "gram": gr[:nnz], "seconds": float(sec.value)}

    def efie_tables(self, stream=None) -> dict:
        """The RWG numbering (tri_rwg [N, 3]), the RWG near list and C_A,
        C_phi on it."""
        info = self.efie_setup(stream)
        n, nnz = info["n_rwg"], info["nnz"]
        tri = np.empty((self.n, 3), dtype=np.int32)
        rowptr = np.empty(n + 1, dtype=np.int32)
        col = np.empty(max(nnz, 1), dtype=np.int32)
        ca = np.empty(max(nnz, 1), dtype=np.float64)
        cphi = np.empty(max(nnz, 1), dtype=np.float64)
        I32, F64 = C.POINTER(C.c_int32), C.POINTER(C.c_double)
        _check(self._lib.aim_efie_export(self._plan, tri.ctypes.data_as(I32),
                                         rowptr.ctypes.data_as(I32), col.ctypes.data_as(I32),
                                         ca.ctypes.data_as(F64), cphi.ctypes.data_as(F64),
                                         _stream_ptr(stream)))
        return {"tri_rwg": tri, "rowptr": rowptr, "col": col[:nnz], "ca": ca[:nnz],
                "cphi": cphi[:nnz]}

    def profile_matvec(self, x, reps: int = 10, freq_idx=None, prec: str = "c128", out=None,
                       stream=None) -> dict:
        """Average duration (ms) of each matvec kernel over ``reps`` runs,
        timed with HIP events on the stream."""
        import torch
        self._check_vec(x, prec, self.n, "x")
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        y = torch.empty_like(x) if out is None else out
        ms = (C.c_double * len(KERNELS))()
        _, fp = _freq_arg(freq_idx, nrhs)
        _check(self._lib.aim_profile_matvec(self._plan, PREC[prec], C.c_void_p(x.data_ptr()),
                                            C.c_void_p(y.data_ptr()), nrhs, fp, int(reps), ms,
                                            _stream_ptr(stream)))
        return {k: float(ms[i]) for i, k in enumerate(KERNELS)}

    def capture_matvec(self, x, y, freq_idx=None, prec: str = "c128", stream=None):
        """Captures y = A x on these tensors into a replayable graph."""
        self._check_vec(x, prec, self.n, "x")
        self._check_vec(y, prec, self.n, "y")
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        _, fp = _freq_arg(freq_idx, nrhs)
        g = C.c_void_p()
        _check(self._lib.aim_matvec_capture(self._plan, PREC[prec], C.c_void_p(x.data_ptr()),
                                            C.c_void_p(y.data_ptr()), nrhs, fp,
                                            _stream_ptr(stream), C.byref(g)))
        return MatvecGraph(self._lib, g, (x, y))

    def autotune(self, prec: str = "c128", nrhs: int = 1, reps: int = 5, cache_path=None,
                 stream=None) -> dict:
        """Picks the FFT launch shapes and workspace layout for this plan.
        With ``cache_path`` a JSON file keyed by (grid, precision, nrhs,
        gfx950) is read first and updated after tuning."""
        import json
        key = f"gfx950|{'x'.join(map(str, self.dims))}|{prec}|nrhs={nrhs}|s{SCHEDULE_LEN}m4"
        cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        if key in cache:
            sched = (C.c_int32 * SCHEDULE_LEN)(*cache[key]["schedule"])
            _check(self._lib.aim_set_schedule(self._plan, PREC[prec], sched))
            return dict(cache[key], cached=True)
        sched = (C.c_int32 * SCHEDULE_LEN)()
        ms = (C.c_double * 5)()
        _check(self._lib.aim_autotune(self._plan, PREC[prec], int(nrhs), int(reps), sched, ms,
                                      _stream_ptr(stream)))
        ent = {"schedule": list(sched), "pass_ms": list(ms)}
        if cache_path:
            cache[key] = ent
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        return dict(ent, cached=False)

    def set_schedule(self, sched, prec: str = "c128"):
        """Five pass shapes, the layout and the interpolation mode (missing
        trailing entries are 0)."""
        sched = list(sched) + [0] * (SCHEDULE_LEN - len(sched))
        if len(sched) != SCHEDULE_LEN:
            raise ValueError(f"a schedule has {SCHEDULE_LEN} entries")
        arr = (C.c_int32 * SCHEDULE_LEN)(*sched)
        _check(self._lib.aim_set_schedule(self._plan, PREC[prec], arr))

    def apply_stage(self, stage: str, inp, freq_idx=None, prec: str = "c128", stream=None):
        """One stage of the matvec: 'project' x -> grid, 'convolve' grid ->
        grid, 'interpolate' grid -> y, 'near' x -> C x; or 'learned_pc'
        x -> M(x) of the attached network.  Grids have shape [nrhs, Nz, Ny, Nx]."""
        import torch
        Nx, Ny, Nz = self.dims
        nrhs = inp.shape[0] if inp.dim() in (2, 4) else 1
        if stage in ("project", "near", "learned_pc", "nearblock_pc"):
            self._check_vec(inp, prec, self.n, "input")
        else:
            self._check_vec(inp.reshape(nrhs, -1), prec, self.n_grid, "input grid")
        if stage in ("project", "convolve"):
            out = torch.empty((nrhs, Nz, Ny, Nx), dtype=self._dtype(prec), device=inp.device)
        else:
            out = torch.empty((nrhs, self.n), dtype=self._dtype(prec), device=inp.device)
        _, fp = _freq_arg(freq_idx, nrhs)
        _check(self._lib.aim_apply_stage(self._plan, PREC[prec], STAGE[stage],
                                         C.c_void_p(inp.data_ptr()), C.c_void_p(out.data_ptr()),
                                         nrhs, fp, _stream_ptr(stream)))
        return out

    def excitation(self, kind: str, params, freq_idx=None, stream=None):
        """Galerkin-tested incident fields, complex128 [nrhs, N]."""
        import torch
        pr = np.ascontiguousarray(np.atleast_2d(np.asarray(params, dtype=np.float64)))
        nrhs, npar = pr.shape
        b = torch.empty((nrhs, self.n), dtype=torch.complex128, device="cuda")
        _, fp = _freq_arg(freq_idx, nrhs)
        _check(self._lib.aim_excitation(self._plan, RHS[kind],
                                        pr.ctypes.data_as(C.POINTER(C.c_double)), npar, nrhs, fp,
                                        C.c_void_p(b.data_ptr()), _stream_ptr(stream)))
        return b

    def solve(self, b, x0=None, freq_idx=None, rtol: float = 1e-6, restart: int = 30,
              max_iter: int = 1000, inner: str = "c128", pc: str = "none",
              max_refine: int = 20, inner_rtol: float = 0.0, fallback_pc: str = "none",
              gate: float = 0.0, stream=None, raise_on_fail=True):
        """Batched GMRES on b of shape [nrhs, N] (complex128).  Returns
        (x, SolveResult).  pc="unet" needs a network attached with set_unet;
        fallback_pc and gate govern its fallback."""
        import torch
        b2 = b.reshape(-1, self.n)
        self._check_vec(b2, "c128", self.n, "b")
        nrhs = b2.shape[0]
        x = torch.zeros_like(b2) if x0 is None else x0.reshape(-1, self.n).clone()
        opts = SolveOpts(rtol, restart, max_iter, max_refine, PREC[inner], PC[pc], inner_rtol,
                         PC[fallback_pc], gate)
        infos = (SolveInfo * nrhs)()
        _, fp = _freq_arg(freq_idx, nrhs)
        st = self._lib.aim_solve(self._plan, C.c_void_p(b2.data_ptr()), C.c_void_p(x.data_ptr()),
                                 nrhs, fp, C.byref(opts), infos, _stream_ptr(stream))
        if st not in (AIM_OK, 6) or (st == 6 and raise_on_fail):
            _check(st)
        res = SolveResult(
            iters=np.array([i.iters for i in infos]),
            refinements=np.array([i.refinements for i in infos]),
            matvecs=np.array([i.matvecs for i in infos]),
            converged=np.array([bool(i.converged) for i in infos]),
            rel_resid=np.array([i.rel_resid for i in infos]),
            seconds=float(infos[0].seconds) if nrhs else 0.0, status=st,
            fallback_used=np.array([bool(i.fallback_used) for i in infos]))
        return x.reshape(b.shape), res

    # ---- learned preconditioner -------------------------------------------
    def set_unet(self, net, base_pc: str = "diag", tau: float = 1.0):
        """Attach a UNet (or detach with None) as the pc="unet" preconditioner."""
        self._unet_ref = net
        _check(self._lib.aim_plan_set_unet(self._plan, net._h if net is not None else None,
                                           PC[base_pc], tau))

    def log_pairs(self, b, rtol: float = 1e-8, restart: int = 10, max_iter: int = 2000,
                  max_pairs: int = 256, freq_idx=None, stream=None):
        """Plain GMRES on b [nrhs, N]; returns (r, e, rhs) of the logged pairs:
        r_t, e_t = x* - x_t at each restart (complex128 device tensors)."""
        import torch
        b2 = b.reshape(-1, self.n)
        self._check_vec(b2, "c128", self.n, "b")
        nrhs = b2.shape[0]
        r = torch.empty((max_pairs, self.n), dtype=torch.complex128, device=b2.device)
        e = torch.empty_like(r)
        owner = np.zeros(max(max_pairs, 1), dtype=np.int32)
        cnt = C.c_int32(0)
        _, fp = _freq_arg(freq_idx, nrhs)
        _check(self._lib.aim_log_pairs(self._plan, C.c_void_p(b2.data_ptr()), nrhs, fp, rtol,
                                       restart, max_iter, C.c_void_p(r.data_ptr()),
                                       C.c_void_p(e.data_ptr()),
                                       owner.ctypes.data_as(C.POINTER(C.c_int32)), max_pairs,
                                       C.byref(cnt), _stream_ptr(stream)))
        k = cnt.value
        return r[:k], e[:k], owner[:k].copy()

    def pc_targets(self, r, e, base_pc: str = "diag", loss: str = "error", stream=None):
        """Network inputs [npairs, Nz, Ny, Nx] complex64, targets [npairs, N]
        complex128 of logged pairs for the given loss kind, and the sums
        (sum |error target|^2, sum |residual target|^2)."""
        import torch
        self._check_vec(r, "c128", self.n, "r")
        self._check_vec(e, "c128", self.n, "e")
        if r.shape != e.shape:
            raise ValueError("r and e must have the same shape")
        npairs = r.shape[0]
        Nx, Ny, Nz = self.dims
        grids = torch.empty((npairs, Nz, Ny, Nx), dtype=torch.complex64, device=r.device)
        tg = torch.empty_like(r)
        sums = (C.c_double * 2)()
        _check(self._lib.aim_pc_targets(self._plan, PC[base_pc], LOSS[loss],
                                        C.c_void_p(r.data_ptr()), C.c_void_p(e.data_ptr()),
                                        npairs, C.c_void_p(grids.data_ptr()),
                                        C.c_void_p(tg.data_ptr()), sums, _stream_ptr(stream)))
        return grids, tg, (sums[0], sums[1])

    def pc_train_step(self, net, grids, targets, idx, tau: float, weight: float = 1.0,
                      loss: str = "error", lr: float = 1e-3, apply: bool = True,
                      stream=None) -> float:
        """One Adam step on the samples idx of (grids, targets); returns the
        loss before the step."""
        Nx, Ny, Nz = self.dims
        if grids.shape[1:] != (Nz, Ny, Nx) or grids.dtype != self._dtype("c64"):
            raise ValueError("grids must be [npairs, Nz, Ny, Nx] complex64")
        self._check_vec(targets, "c128", self.n, "targets")
        if targets.shape[0] != grids.shape[0]:
            raise ValueError("grids and targets hold different numbers of pairs")
        ia = np.ascontiguousarray(np.asarray(idx, dtype=np.int32).ravel())
        out = C.c_double(0.0)
        _check(self._lib.aim_pc_train_step(self._plan, net._h, LOSS[loss],
                                           C.c_void_p(grids.data_ptr()),
                                           C.c_void_p(targets.data_ptr()), grids.shape[0],
                                           ia.ctypes.data_as(C.POINTER(C.c_int32)), ia.size,
                                           tau, weight, lr, int(apply), C.byref(out),
                                           _stream_ptr(stream)))
        return out.value
