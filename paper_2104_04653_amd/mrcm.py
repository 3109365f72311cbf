"""ctypes binding of ``libmrcm.so`` (the C ABI declared in include/mrcm.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Host arrays are numpy float64 arrays; device arrays are torch CUDA
(ROCm) tensors, passed as raw pointers together with torch's current stream.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmrcm.so")

OK, E_INVAL, E_NOMEM, E_HIP, E_NOT_SPD, E_NO_CONV, E_STATE, E_UNSUPPORTED = range(8)
ERROR_NAMES = {0: "MRCM_OK", 1: "MRCM_E_INVAL", 2: "MRCM_E_NOMEM", 3: "MRCM_E_HIP",
               4: "MRCM_E_NOT_SPD", 5: "MRCM_E_NO_CONV", 6: "MRCM_E_STATE",
               7: "MRCM_E_UNSUPPORTED"}
SPACES = {"linear": 0, "edge": 1, "full": 2}
PRECISIONS = {"fp64": 0, "fp32_ir": 1}

EXPORTED = [
    "mrcm_setup", "mrcm_update_mobility", "mrcm_solve", "mrcm_fine_flux", "mrcm_get_stats",
    "mrcm_get_sizes", "mrcm_get_interface_solution", "mrcm_get_local_blocks",
    "mrcm_get_basis", "mrcm_last_error", "mrcm_destroy",
]


class MRCMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERROR_NAMES.get(code, code), msg))
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double)]


class BC(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32 * 4), ("value", ctypes.POINTER(ctypes.c_double) * 4)]


class Fluid(ctypes.Structure):
    _fields_ = [("mu_w", ctypes.c_double), ("mu_o", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("ms_local", ctypes.c_double), ("ms_interface", ctypes.c_double),
                ("ms_flux", ctypes.c_double), ("n_sub", ctypes.c_int32),
                ("n_dof", ctypes.c_int32), ("ir_iters_max", ctypes.c_int32),
                ("fallbacks", ctypes.c_int32), ("interface_residual", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libmrcm.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libmrcm.so is not built (%s); run "
                          "`python -m paper_2104_04653_amd.build`" % path)
    # One HIP runtime per process: torch ships its own libamdhip64 with the
    # same soname as the system one; loading torch first makes the library's
    # dependency resolve to that already-loaded copy instead of a second one.
    try:
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover - C users without torch
        pass
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    lib.mrcm_setup.argtypes = [ctypes.POINTER(P), ctypes.POINTER(Grid), dp, ctypes.c_int32,
                               ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                               dp, ctypes.c_double, ctypes.POINTER(BC), dp,
                               ctypes.POINTER(Fluid), ctypes.c_int32, P]
    lib.mrcm_update_mobility.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32]
    lib.mrcm_solve.argtypes = [P]
    lib.mrcm_fine_flux.argtypes = [P, P, P, P, ctypes.c_int32, dp]
    lib.mrcm_get_stats.argtypes = [P, ctypes.POINTER(Stats)]
    lib.mrcm_get_sizes.argtypes = [P, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.mrcm_get_interface_solution.argtypes = [P, dp]
    lib.mrcm_get_local_blocks.argtypes = [P, dp]
    lib.mrcm_get_basis.argtypes = [P, dp]
    lib.mrcm_last_error.argtypes = [P]
    lib.mrcm_last_error.restype = ctypes.c_char_p
    lib.mrcm_destroy.argtypes = [P]
    lib.mrcm_destroy.restype = None
    for name in EXPORTED[:-2]:
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _host(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a


def _is_device(x):
    return hasattr(x, "is_cuda") and bool(x.is_cuda)


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:  # pragma: no cover - torch without a GPU
        pass
    return ctypes.c_void_p(None)


class MRCMSolver:
    """One MRCM Darcy solver on the GPU for a fixed grid, permeability and
    decomposition (mrcm_setup); per step: update_mobility, solve, fine_flux."""

    def __init__(self, prob, precision: str = "fp64", stream=None):
        self.lib = load_library()
        self.prob = prob
        nx, ny = int(prob.nx), int(prob.ny)
        self.nx, self.ny = nx, ny
        self._keep = []
        grid = Grid(nx, ny, float(prob.lx), float(prob.ly))
        perm = _host(prob.perm, nx * ny)
        bc = BC()
        for s in range(4):
            bc.kind[s] = int(prob.bc_kind[s])
            v = prob.bc_value[s]
            if v is None:
                bc.value[s] = ctypes.POINTER(ctypes.c_double)()
            else:
                arr = _host(v, ny if s < 2 else nx)
                self._keep.append(arr)
                bc.value[s] = _dptr(arr)
        src = None if prob.source is None else _host(prob.source, nx * ny)
        alpha_arr = None
        if getattr(prob, "alpha_per_interface", None) is not None:
            alpha_arr = _host(prob.alpha_per_interface)
        fluid = Fluid(float(prob.mu_w), float(prob.mu_o))
        ctx = ctypes.c_void_p()
        st = _current_stream() if stream is None else ctypes.c_void_p(stream)
        rc = self.lib.mrcm_setup(ctypes.byref(ctx), ctypes.byref(grid), _dptr(perm),
                                 int(prob.sub_nx), int(prob.sub_ny), SPACES[prob.space],
                                 int(prob.p_dofs), int(prob.u_dofs),
                                 _dptr(alpha_arr) if alpha_arr is not None else
                                 ctypes.POINTER(ctypes.c_double)(),
                                 float(prob.alpha), ctypes.byref(bc),
                                 _dptr(src) if src is not None else ctypes.POINTER(ctypes.c_double)(),
                                 ctypes.byref(fluid), PRECISIONS[precision], st)
        if rc != OK:
            raise MRCMError(rc, "mrcm_setup failed")
        self.ctx = ctx
        n_dof, n_sub, n_cols = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self.lib.mrcm_get_sizes(self.ctx, ctypes.byref(n_dof), ctypes.byref(n_sub), ctypes.byref(n_cols))
        self.n_dof, self.n_sub, self.n_cols = n_dof.value, n_sub.value, n_cols.value

    # -- helpers ----------------------------------------------------------
    def _check(self, rc, what):
        if rc != OK:
            msg = self.lib.mrcm_last_error(self.ctx).decode(errors="replace")
            raise MRCMError(rc, "%s: %s" % (what, msg))

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.mrcm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):  # pragma: no cover - best effort
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- per-step calls ----------------------------------------------------
    def update_mobility(self, values, is_lambda: bool = False):
        """Set lambda(s) (saturation input) or lambda directly; host numpy
        arrays or torch device tensors of nx*ny float64."""
        n = self.nx * self.ny
        if _is_device(values):
            if values.numel() != n or str(values.dtype) != "torch.float64" or not values.is_contiguous():
                raise ValueError("device mobility must be a contiguous float64 tensor of nx*ny")
            self._dev_in = values   # keep alive until the next solve
            import torch
            torch.cuda.current_stream().synchronize()   # producer work is complete
            rc = self.lib.mrcm_update_mobility(self.ctx, ctypes.c_void_p(values.data_ptr()),
                                               int(is_lambda), 1)
        else:
            arr = _host(values, n)
            rc = self.lib.mrcm_update_mobility(self.ctx, arr.ctypes.data_as(ctypes.c_void_p),
                                               int(is_lambda), 0)
        self._check(rc, "mrcm_update_mobility")

    def solve(self):
        self._check(self.lib.mrcm_solve(self.ctx), "mrcm_solve")

    def fine_flux(self, device: bool = False):
        """Return (p, ux, uy, max_cell_imbalance); numpy, or torch tensors on
        the GPU with device=True."""
        nx, ny = self.nx, self.ny
        imb = ctypes.c_double()
        if device:
            import torch
            p = torch.empty(nx * ny, dtype=torch.float64, device="cuda")
            ux = torch.empty((nx + 1) * ny, dtype=torch.float64, device="cuda")
            uy = torch.empty(nx * (ny + 1), dtype=torch.float64, device="cuda")
            ptrs = [ctypes.c_void_p(t.data_ptr()) for t in (p, ux, uy)]
            rc = self.lib.mrcm_fine_flux(self.ctx, *ptrs, 1, ctypes.byref(imb))
        else:
            p = np.empty(nx * ny)
            ux = np.empty((nx + 1) * ny)
            uy = np.empty(nx * (ny + 1))
            ptrs = [a.ctypes.data_as(ctypes.c_void_p) for a in (p, ux, uy)]
            rc = self.lib.mrcm_fine_flux(self.ctx, *ptrs, 0, ctypes.byref(imb))
        self._check(rc, "mrcm_fine_flux")
        return p, ux, uy, imb.value

    # -- inspection --------------------------------------------------------
    def stats(self) -> dict:
        s = Stats()
        self._check(self.lib.mrcm_get_stats(self.ctx, ctypes.byref(s)), "mrcm_get_stats")
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def interface_solution(self) -> np.ndarray:
        out = np.empty(self.n_dof)
        self._check(self.lib.mrcm_get_interface_solution(self.ctx, _dptr(out)),
                    "mrcm_get_interface_solution")
        return out

    def local_blocks(self) -> np.ndarray:
        R = self.n_cols
        out = np.empty(self.n_sub * (R - 1) * R)
        self._check(self.lib.mrcm_get_local_blocks(self.ctx, _dptr(out)), "mrcm_get_local_blocks")
        return out.reshape(self.n_sub, R - 1, R)

    def basis(self) -> np.ndarray:
        m = int(self.prob.sub_nx)
        out = np.empty(self.n_sub * m * m * self.n_cols)
        self._check(self.lib.mrcm_get_basis(self.ctx, _dptr(out)), "mrcm_get_basis")
        # stored column-major per subdomain; returned as [sub][cell][col]
        return out.reshape(self.n_sub, self.n_cols, m * m).transpose(0, 2, 1).copy()
