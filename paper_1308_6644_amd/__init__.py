"""Python binding of libnuasm: non-uniform sampled ASM / Fresnel diffraction
on one MI355X (Shimobaba et al., arXiv 1308.6644, Eqs. 4-9).

Argument marshalling only: every step of the operators runs in the library's
HIP kernels.  PyTorch supplies device memory and streams.  The library must be
built first (``python -m paper_1308_6644_amd.build``); importing this module
raises if it is missing, and there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loads the HIP runtime the library binds to

__all__ = [
    "Plan", "Batch", "make_params", "NUASM1", "NUASM2", "NUASM3", "nuasm1", "nuasm2", "nuasm3", "debug_fft",
    "rs_direct",
    "lib_path", "load", "NuasmError", "TYPE_1", "TYPE_2", "TYPE_3", "TF_ASM", "TF_FRESNEL",
]

TYPE_1, TYPE_2, TYPE_3 = 1, 2, 3
STAGES = ("bin_hist", "bin_colscan", "bin_scan", "bin_scatter", "spread", "spread_reduce",
          "t1_rows", "t1_cols", "t1_rows_inv", "t2_rows", "t2_cols", "t2_rows_inv", "interp", "t3_cols")
TF_ASM, TF_FRESNEL = 0, 1
BAND = {"full": 0, "limited": 1, "explicit": 2}
TF = {"asm": TF_ASM, "fresnel": TF_FRESNEL}
OUT_CROP_N = 0x1
DEFER_RANGE_CHECK = 0x2
FULL_FINE_GRID = 0x4
DETERMINISTIC = 0x8
FORWARD_ONLY = 0x10

_HERE = os.path.dirname(os.path.abspath(__file__))


def lib_path() -> str:
    return os.path.join(_HERE, "libnuasm.so")


class NuasmError(RuntimeError):
    def __init__(self, status: int, name: str, detail: str):
        super().__init__(f"{name}: {detail}")
        self.status = status
        self.name = name


class Params(ctypes.Structure):
    _fields_ = [
        ("type", ctypes.c_int32), ("tf", ctypes.c_int32), ("band", ctypes.c_int32),
        ("phase_fp64", ctypes.c_int32), ("N", ctypes.c_int64),
        ("lam", ctypes.c_double), ("z", ctypes.c_double),
        ("ox", ctypes.c_double), ("oy", ctypes.c_double),
        ("d1", ctypes.c_double), ("d2", ctypes.c_double),
        ("band_c", ctypes.c_double * 2), ("band_w", ctypes.c_double * 2),
        ("tol", ctypes.c_double), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
    ]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64), ("Np", ctypes.c_int64), ("nf", ctypes.c_int64), ("L", ctypes.c_int64),
        ("w", ctypes.c_int32), ("beta", ctypes.c_float), ("tile", ctypes.c_int32),
        ("tiles", ctypes.c_int32), ("kx_lo", ctypes.c_int32), ("kx_hi", ctypes.c_int32),
        ("ky_lo", ctypes.c_int32), ("ky_hi", ctypes.c_int32), ("in_elems", ctypes.c_int64),
        ("out_elems", ctypes.c_int64), ("M", ctypes.c_int64), ("device_bytes", ctypes.c_size_t),
        ("M_dest", ctypes.c_int64), ("spread_chunk", ctypes.c_int32), ("interp_chunk", ctypes.c_int32),
        ("bin_range_points", ctypes.c_int32), ("Npf", ctypes.c_int32),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [("spread_chunk", ctypes.c_int32), ("interp_chunk", ctypes.c_int32),
                ("bin_range_points", ctypes.c_int32), ("spread_method", ctypes.c_int32),
                ("bin_tile", ctypes.c_int32)]


_SIGS = {
    "nuasm_version": (ctypes.c_int32, []),
    "nuasm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "nuasm_last_error": (ctypes.c_char_p, []),
    "nuasm_params_default": (ctypes.c_int, [ctypes.POINTER(Params)]),
    "nuasm_plan_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "nuasm_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "nuasm_plan_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "nuasm_plan_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(PlanInfo)]),
    "nuasm_set_points": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "nuasm_set_dest_points": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "nuasm_set_grid_points": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "nuasm_check_points": (ctypes.c_int, [ctypes.c_void_p]),
    "nuasm_plan_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Tuning)]),
    "nuasm_batch_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Tuning)]),
    "nuasm_batch_set_branches": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "nuasm_batch_set_grouped": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "nuasm_execute": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "nuasm_execute_adjoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "nuasm_execute_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "nuasm_debug_transfer": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "nuasm_plan_set_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "nuasm_plan_read_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_int64)]),
    "nuasm_debug_records": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "nuasm_debug_spread": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "nuasm_debug_interp": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "nuasm_debug_fail_alloc": (ctypes.c_int, [ctypes.c_int64]),
    "nuasm_debug_live_bytes": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "nuasm_debug_fft": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "nuasm_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(Params), ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "nuasm_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "nuasm_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p)]),
    "nuasm_set_points_many": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p)]),
    "nuasm_execute_many": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "nuasm_plan_many_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(Params), ctypes.c_void_p,
                                              ctypes.POINTER(ctypes.c_void_p)]),
    "nuasm_plan_workspace_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]),
    "nuasm_plan_set_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "nuasm_batch_check_points": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "nuasm_batch_plane_times": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)]),
    "nuasm_batch_set_plane_times": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "nuasm_debug_batch_graphs": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                                ctypes.POINTER(ctypes.c_int64)]),
    "nuasm_rs_direct": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                       ctypes.c_void_p]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libnuasm.so (built in-tree).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    p = lib_path()
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with `python -m paper_1308_6644_amd.build`")
    lib = ctypes.CDLL(p)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        lib = load()
        name = lib.nuasm_status_string(status).decode()
        detail = lib.nuasm_last_error().decode()
        raise NuasmError(status, name, detail)


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev_ptr(t: torch.Tensor, dtype, what: str) -> int:
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return t.data_ptr()


def make_params(N: int, type: int, lam: float, z: float, g: float, *, tf: str = "asm",
                ox: float = 0.0, oy: float = 0.0, band: str = "full", band_c=(0.0, 0.0),
                band_w=(0.0, 0.0), tol: float = 1e-6, phase_fp64: bool = True, crop: bool = False,
                defer_range_check: bool = False, full_fine_grid: bool = False,
                deterministic: bool = False, forward_only: bool = False) -> Params:
    lib = load()
    p = Params()
    _check(lib.nuasm_params_default(ctypes.byref(p)))
    p.type = int(type)
    p.tf = TF[tf]
    p.band = BAND[band]
    p.phase_fp64 = 1 if phase_fp64 else 0
    p.N = int(N)
    p.lam = float(lam)
    p.z = float(z)
    p.ox, p.oy = float(ox), float(oy)
    p.d1 = p.d2 = float(g)
    p.band_c[0], p.band_c[1] = float(band_c[0]), float(band_c[1])
    p.band_w[0], p.band_w[1] = float(band_w[0]), float(band_w[1])
    p.tol = float(tol)
    p.flags = ((OUT_CROP_N if crop else 0) | (DEFER_RANGE_CHECK if defer_range_check else 0)
               | (FULL_FINE_GRID if full_fine_grid else 0) | (DETERMINISTIC if deterministic else 0)
               | (FORWARD_ONLY if forward_only else 0))
    return p


class Plan:
    """One operator instance: NU-ASM_1/NU-FRE_1 (type 1, Eq. 6),
    NU-ASM_2/NU-FRE_2 (type 2, Eq. 9) or NU-ASM_3/NU-FRE_3 (type 3, their
    combination) on an N x N window of pitch g.

    Type 1: ``execute(c[M]) -> u2[N'][N']`` (``[N][N]`` with ``crop=True``).
    Type 2: ``execute(u1[N][N]) -> u2[M]``.
    Type 3: ``set_points`` binds the sources, ``set_dest_points`` the
    destinations; ``execute(c[M]) -> u2[M_dest]``.  Points are FP64 metres.
    """

    def __init__(self, N: int, type: int, lam: float, z: float, g: float, *, tf: str = "asm",
                 ox: float = 0.0, oy: float = 0.0, band: str = "full", band_c=(0.0, 0.0),
                 band_w=(0.0, 0.0), tol: float = 1e-6, phase_fp64: bool = True, crop: bool = False,
                 defer_range_check: bool = False, full_fine_grid: bool = False,
                 deterministic: bool = False, forward_only: bool = False, device=None):
        lib = load()
        p = make_params(N, type, lam, z, g, tf=tf, ox=ox, oy=oy, band=band, band_c=band_c, band_w=band_w,
                        tol=tol, phase_fp64=phase_fp64, crop=crop, defer_range_check=defer_range_check,
                        full_fine_grid=full_fine_grid, deterministic=deterministic, forward_only=forward_only)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.params = p
        self.N, self.Np, self.type, self.crop = int(N), 2 * int(N), int(type), bool(crop)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.nuasm_plan_create(ctypes.byref(p), ctypes.c_void_p(_stream_ptr()), ctypes.byref(h)))
        self._h = h
        self.M = 0
        self.M_dest = 0

    # ------------------------------------------------------------ lifecycle
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().nuasm_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        _check(load().nuasm_plan_set_stream(self._h, ctypes.c_void_p(_stream_ptr())))

    @property
    def info(self) -> dict:
        i = PlanInfo()
        _check(load().nuasm_plan_get_info(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in PlanInfo._fields_}

    # ------------------------------------------------------------- calls
    def _bind(self, fn, x: torch.Tensor, y: torch.Tensor) -> int:
        if x.shape != y.shape or x.dim() != 1:
            raise ValueError("x and y must be 1-D tensors of equal length")
        self._sync_stream()
        M = x.numel()
        xp = _dev_ptr(x, torch.float64, "x") if M else None
        yp = _dev_ptr(y, torch.float64, "y") if M else None
        _check(fn(self._h, M, ctypes.c_void_p(xp), ctypes.c_void_p(yp)))
        return M

    def set_points(self, x: torch.Tensor, y: torch.Tensor):
        """Bind the non-uniform points (type 3: the source points)."""
        self.M = self._bind(load().nuasm_set_points, x, y)
        self._points = (x, y)  # keep alive until the stream has read them
        return self

    def set_dest_points(self, x: torch.Tensor, y: torch.Tensor):
        """Type 3: bind the destination points."""
        self.M_dest = self._bind(load().nuasm_set_dest_points, x, y)
        self._dest_points = (x, y)
        return self

    def set_grid_points(self, nx: int, ny: int, pitch: float, cx: float = 0.0, cy: float = 0.0,
                        dest: bool = False):
        """Bind a uniform nx x ny grid of the given pitch centred at (cx, cy)
        (scaled diffraction): the point-side arrays become [ny * nx] in
        row-major grid order.  dest=True binds a type-3 plan's destination."""
        self._sync_stream()
        _check(load().nuasm_set_grid_points(self._h, 1 if dest else 0, int(nx), int(ny), float(pitch),
                                            float(cx), float(cy)))
        if dest:
            self.M_dest = int(nx) * int(ny)
        else:
            self.M = int(nx) * int(ny)
        return self

    def check_points(self):
        _check(load().nuasm_check_points(self._h))

    def debug_spread(self, vals: torch.Tensor, dest: bool = False) -> torch.Tensor:
        """Spreading alone: the point values spread onto the fine-grid
        support, complex64 [L][L]."""
        L = self.info["L"]
        grid = torch.empty((L, L), dtype=torch.complex64, device=self.device)
        n = self.M_dest if dest else self.M
        vp = _dev_ptr(vals, torch.complex64, "vals") if n else None
        if n and vals.numel() != n:
            raise ValueError(f"vals must hold {n} values")
        self._sync_stream()
        _check(load().nuasm_debug_spread(self._h, 1 if dest else 0, ctypes.c_void_p(vp),
                                         ctypes.c_void_p(grid.data_ptr())))
        return grid

    def debug_interp(self, grid: torch.Tensor, dest: bool = False) -> torch.Tensor:
        """Interpolation alone: the support grid (complex64 [L][L]) at the
        bound points, complex64 [M]."""
        L = self.info["L"]
        if tuple(grid.shape) != (L, L):
            raise ValueError(f"grid must be [{L}][{L}]")
        n = self.M_dest if dest else self.M
        out = torch.empty((n,), dtype=torch.complex64, device=self.device)
        gp = _dev_ptr(grid, torch.complex64, "grid")
        self._sync_stream()
        _check(load().nuasm_debug_interp(self._h, 1 if dest else 0, ctypes.c_void_p(gp),
                                         ctypes.c_void_p(out.data_ptr() if n else None)))
        return out

    def debug_records(self, dest: bool = False):
        """The bound point set's bin records in the order the point kernels
        read them, as int32 [R][4] (packed, dx and dy as float32 bits, point
        index), and the records per bin, int32 [tiles]."""
        cap = 4 * max(1, self.M_dest if dest else self.M)
        recs = torch.empty((cap, 4), dtype=torch.int32, device=self.device)
        counts = torch.empty((self.info["tiles"],), dtype=torch.int32, device=self.device)
        n = ctypes.c_int64()
        self._sync_stream()
        _check(load().nuasm_debug_records(self._h, 1 if dest else 0, ctypes.c_void_p(recs.data_ptr()), cap,
                                          ctypes.c_void_p(counts.data_ptr()), ctypes.byref(n)))
        return recs[:n.value], counts

    def workspace_bytes(self, M_max: int) -> int:
        """Bytes of a caller-owned workspace holding M_max points per point set."""
        b = ctypes.c_size_t()
        _check(load().nuasm_plan_workspace_bytes(self._h, int(M_max), ctypes.byref(b)))
        return b.value

    def set_workspace(self, ws: torch.Tensor | None):
        """Carve the plan's grids and point buffers from a caller-owned device
        tensor (uint8, 256-byte aligned; kept alive by the plan), or go back to
        plan-owned memory with None.  Binned points must be set again."""
        self._sync_stream()
        if ws is None:
            _check(load().nuasm_plan_set_workspace(self._h, None, 0))
        else:
            p = _dev_ptr(ws, torch.uint8, "workspace")
            _check(load().nuasm_plan_set_workspace(self._h, ctypes.c_void_p(p), ws.numel()))
        self._ws = ws
        return self

    def set_tuning(self, spread_chunk: int = 0, interp_chunk: int = 0, bin_range_points: int = 0,
                   spread_method: int = 0, bin_tile: int = 0):
        """Launch-shape tuning (0 = default); binned points must be set again.
        spread_method: 0 automatic, 1 register gather, 2 matrix cores;
        bin_tile: 0 (32) or the bin side, 32 or 64."""
        t = Tuning(int(spread_chunk), int(interp_chunk), int(bin_range_points), int(spread_method), int(bin_tile))
        _check(load().nuasm_plan_set_tuning(self._h, ctypes.byref(t)))
        return self

    def _in_shape(self, adjoint: bool):
        if self.type == TYPE_3:
            return (self.M_dest,) if adjoint else (self.M,)
        fwd = (self.M,) if self.type == TYPE_1 else (self.N, self.N)
        if not adjoint:
            return fwd
        return (self.Np, self.Np) if self.type == TYPE_1 else (self.M,)

    def _out_shape(self, adjoint: bool):
        if self.type == TYPE_3:
            return (self.M,) if adjoint else (self.M_dest,)
        if self.type == TYPE_1:
            if adjoint:
                return (self.M,)
            return (self.N, self.N) if self.crop else (self.Np, self.Np)
        return (self.N, self.N) if adjoint else (self.M,)

    def _run(self, fn, inp: torch.Tensor, out, adjoint: bool):
        want = self._in_shape(adjoint)
        if tuple(inp.shape) != want:
            raise ValueError(f"input shape {tuple(inp.shape)} != {want}")
        oshape = self._out_shape(adjoint)
        if out is None:
            out = torch.empty(oshape, dtype=torch.complex64, device=inp.device)
        elif tuple(out.shape) != oshape:
            raise ValueError(f"output shape {tuple(out.shape)} != {oshape}")
        self._sync_stream()
        ip = _dev_ptr(inp, torch.complex64, "input")
        op = _dev_ptr(out, torch.complex64, "output")
        _check(fn(self._h, ctypes.c_void_p(ip), ctypes.c_void_p(op)))
        return out

    def execute(self, inp: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        return self._run(load().nuasm_execute, inp, out, adjoint=False)

    def adjoint(self, inp: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        return self._run(load().nuasm_execute_adjoint, inp, out, adjoint=True)

    def set_timing(self, enable: bool = True):
        _check(load().nuasm_plan_set_timing(self._h, 1 if enable else 0))

    def read_timing(self) -> dict:
        """{stage: (milliseconds, launches)} accumulated since the last read."""
        ms = (ctypes.c_double * len(STAGES))()
        n = (ctypes.c_int64 * len(STAGES))()
        _check(load().nuasm_plan_read_timing(self._h, ms, n))
        return {st: (ms[i], n[i]) for i, st in enumerate(STAGES)}

    def transfer(self) -> torch.Tensor:
        """H(k) Rect(k) as the fused spectral kernel applies it, [N'][N']."""
        out = torch.empty((self.Np, self.Np), dtype=torch.complex64, device=self.device)
        self._sync_stream()
        _check(load().nuasm_debug_transfer(self._h, ctypes.c_void_p(out.data_ptr())))
        return out


class Batch:
    """Many independent planes run as one recorded HIP graph (binning and the
    operator of every plane on parallel branches).  ``specs`` is a list of
    keyword dicts for make_params (N, type, lam, z, g, tf, band, ox, oy, tol)."""

    def __init__(self, specs):
        lib = load()
        self.specs = [dict(s) for s in specs]
        arr = (Params * len(specs))(*[make_params(**s) for s in specs])
        h = ctypes.c_void_p()
        _check(lib.nuasm_batch_create(len(specs), arr, ctypes.c_void_p(_stream_ptr()), ctypes.byref(h)))
        self._h = h
        self.P = len(specs)
        self._keep = None

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().nuasm_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, xs, ys, ins, outs):
        """One-shot run of every plane: bin xs[p], ys[p] and apply the operator
        to ins[p] -> outs[p] (device tensors, shapes as for Plan.execute)."""
        P = self.P
        if not (len(xs) == len(ys) == len(ins) == len(outs) == P):
            raise ValueError("need one x, y, in and out per plane")
        M = (ctypes.c_int64 * P)(*[int(x.numel()) for x in xs])
        vp = ctypes.c_void_p * P

        def ptrs(ts, dtype, what):
            return vp(*[(_dev_ptr(t, dtype, what) if t.numel() else None) for t in ts])
        px, py = ptrs(xs, torch.float64, "x"), ptrs(ys, torch.float64, "y")
        pi, po = ptrs(ins, torch.complex64, "in"), ptrs(outs, torch.complex64, "out")
        _check(load().nuasm_batch_run(self._h, M, px, py, pi, po))
        self._keep = (xs, ys, ins, outs)
        return outs

    def set_points(self, xs, ys):
        """Bin every plane's points (one recorded graph; see nuasm_set_points_many)."""
        if not (len(xs) == len(ys) == self.P):
            raise ValueError("need one x and y per plane")
        M = (ctypes.c_int64 * self.P)(*[int(x.numel()) for x in xs])
        vp = ctypes.c_void_p * self.P
        px = vp(*[(_dev_ptr(t, torch.float64, "x") if t.numel() else None) for t in xs])
        py = vp(*[(_dev_ptr(t, torch.float64, "y") if t.numel() else None) for t in ys])
        _check(load().nuasm_set_points_many(self._h, M, px, py))
        self._keep_pts = (xs, ys)
        return self

    def execute(self, ins, outs):
        """Apply every plane's operator to ins[p] -> outs[p] on the points bound
        by set_points (one recorded graph; see nuasm_execute_many)."""
        if not (len(ins) == len(outs) == self.P):
            raise ValueError("need one in and out per plane")
        vp = ctypes.c_void_p * self.P
        pi = vp(*[(_dev_ptr(t, torch.complex64, "in") if t.numel() else None) for t in ins])
        po = vp(*[(_dev_ptr(t, torch.complex64, "out") if t.numel() else None) for t in outs])
        _check(load().nuasm_execute_many(self._h, pi, po))
        self._keep_io = (ins, outs)
        return outs

    def set_tuning(self, plane: int, spread_chunk: int = 0, interp_chunk: int = 0, bin_range_points: int = 0,
                   spread_method: int = 0, bin_tile: int = 0):
        t = Tuning(int(spread_chunk), int(interp_chunk), int(bin_range_points), int(spread_method), int(bin_tile))
        _check(load().nuasm_batch_set_tuning(self._h, int(plane), ctypes.byref(t)))

    def set_branches(self, branches: int):
        _check(load().nuasm_batch_set_branches(self._h, int(branches)))

    def set_grouped(self, grouped: bool):
        """Grouped stage launches (default) or every plane's own launches on
        parallel branches."""
        _check(load().nuasm_batch_set_grouped(self._h, 1 if grouped else 0))

    def check_points(self) -> int:
        bad = ctypes.c_int32(-1)
        _check(load().nuasm_batch_check_points(self._h, ctypes.byref(bad)))
        return bad.value

    def debug_graphs(self):
        """(graphs recorded, grouped tables rewritten in place) so far."""
        r, f = ctypes.c_int64(), ctypes.c_int64()
        _check(load().nuasm_debug_batch_graphs(self._h, ctypes.byref(r), ctypes.byref(f)))
        return r.value, f.value

    def set_plane_times(self, enabled: bool):
        """Record completion stamps for plane_times (default) or none."""
        _check(load().nuasm_batch_set_plane_times(self._h, 1 if enabled else 0))

    def plane_times(self):
        """Milliseconds from the start of the last run to each plane's completion."""
        ms = (ctypes.c_float * self.P)()
        _check(load().nuasm_batch_plane_times(self._h, ms))
        return [ms[i] for i in range(self.P)]


def debug_fft(x: torch.Tensor, sign: int = -1) -> torch.Tensor:
    """Batched 1-D FFT along the last axis with the library's Stockham kernels."""
    n = x.shape[-1]
    xin = x.contiguous()
    out = torch.empty_like(xin)
    _dev_ptr(xin, torch.complex64, "x")
    _check(load().nuasm_debug_fft(n, xin.numel() // n, int(sign), ctypes.c_void_p(xin.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(_stream_ptr())))
    return out


def rs_direct(x1: torch.Tensor, y1: torch.Tensor, c: torch.Tensor, x2: torch.Tensor, y2: torch.Tensor,
              lam: float, z: float, ox: float = 0.0, oy: float = 0.0,
              out: torch.Tensor | None = None) -> torch.Tensor:
    """Rayleigh-Sommerfeld direct summation (Eq. 10) from weighted source
    points (x1, y1, c: c carries each sample's area element) to destination
    points (x2, y2) offset by (ox, oy); complex64 [M2]."""
    M1, M2 = x1.numel(), x2.numel()
    if x1.shape != y1.shape or c.shape != x1.shape or x2.shape != y2.shape or x1.dim() != 1 or x2.dim() != 1:
        raise ValueError("x1, y1, c and x2, y2 must be 1-D with matching lengths")
    if out is None:
        out = torch.empty((M2,), dtype=torch.complex64, device=x2.device if M2 else c.device)
    elif tuple(out.shape) != (M2,):
        raise ValueError(f"output shape {tuple(out.shape)} != {(M2,)}")
    p = [(_dev_ptr(t, dt, w) if t.numel() else None) for t, dt, w in
         ((x1, torch.float64, "x1"), (y1, torch.float64, "y1"), (c, torch.complex64, "c"),
          (x2, torch.float64, "x2"), (y2, torch.float64, "y2"), (out, torch.complex64, "out"))]
    _check(load().nuasm_rs_direct(M1, p[0], p[1], p[2], M2, p[3], p[4], float(lam), float(z), float(ox),
                                  float(oy), p[5], ctypes.c_void_p(_stream_ptr())))
    return out


# ------------------------------------------------------------- autograd
class NUASM1(torch.autograd.Function):
    """u2 = NU-ASM_1(c) with backward = the hand-written adjoint."""

    @staticmethod
    def forward(ctx, c, plan: Plan):
        ctx.plan = plan
        return plan.execute(c.contiguous())

    @staticmethod
    def backward(ctx, grad):
        return ctx.plan.adjoint(grad.contiguous()), None


class NUASM2(torch.autograd.Function):
    """u2 = NU-ASM_2(u1) with backward = the hand-written adjoint."""

    @staticmethod
    def forward(ctx, u1, plan: Plan):
        ctx.plan = plan
        return plan.execute(u1.contiguous())

    @staticmethod
    def backward(ctx, grad):
        return ctx.plan.adjoint(grad.contiguous()), None


class NUASM3(torch.autograd.Function):
    """u2 = NU-ASM_3(c) with backward = the hand-written adjoint."""

    @staticmethod
    def forward(ctx, c, plan: Plan):
        ctx.plan = plan
        return plan.execute(c.contiguous())

    @staticmethod
    def backward(ctx, grad):
        return ctx.plan.adjoint(grad.contiguous()), None


def nuasm1(c: torch.Tensor, plan: Plan) -> torch.Tensor:
    return NUASM1.apply(c, plan)


def nuasm2(u1: torch.Tensor, plan: Plan) -> torch.Tensor:
    return NUASM2.apply(u1, plan)


def nuasm3(c: torch.Tensor, plan: Plan) -> torch.Tensor:
    return NUASM3.apply(c, plan)
