"""ctypes binding of the FOFSE C ABI (include/fofse.h).

Argument marshalling only: every step of the extrapolation runs in the HIP
kernels of libfofse.so.  PyTorch supplies device memory and the current stream.
There is no fallback: if the library is not built or cannot be loaded, every
call raises.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfofse.so")

FOFSE_OK = 0
FOFSE_ERR_ARG = 1
FOFSE_ERR_UNSUPPORTED = 2
FOFSE_ERR_NOMEM = 3
FOFSE_ERR_DEVICE = 4
FOFSE_ERR_LIMIT = 5

FOFSE_BLOCK_NO_SUPPORT = 1
FOFSE_BLOCK_NONFINITE = 2
FOFSE_BLOCK_BAD_PARAM = 4

FOFSE_PATH_AUTO = 0
FOFSE_PATH_SPLIT = 1
FOFSE_PATH_GROUPED = 2

FOFSE_BASIS_DFT = 0
FOFSE_BASIS_DCT = 1

FOFSE_COMP_CONSTANT = 0
FOFSE_COMP_FULL = 1

EXPORTED = ("fofse_create", "fofse_target_count", "fofse_set_path", "fofse_set_waves", "fofse_set_occupancy",
            "fofse_set_basis", "fofse_set_compensation",
            "fofse_extrapolate_batch", "fofse_extrapolate_batch_noalloc",
            "fofse_backward", "fofse_set_timing", "fofse_kernel_times", "fofse_destroy",
            "fofse_create_multi", "fofse_multi_geometry_plan", "fofse_extrapolate_multi", "fofse_destroy_multi",
            "fofse_status_str")

BACKWARD_MAX_K = 2048
NOALLOC_MAX_BLOCKS = 65536


class FofseError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {fofse_status_str(status)} ({status})")
        self.status = status


class fofse_geometry(ctypes.Structure):
    _fields_ = [("area_h", ctypes.c_int32), ("area_w", ctypes.c_int32),
                ("fft_size", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("target_mask", ctypes.POINTER(ctypes.c_uint8))]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfofse.so (once) and declare the signatures of include/fofse.h."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() "
                           "or python -m paper_2207_01205_amd.build")
    L = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    L.fofse_create.argtypes = [ctypes.POINTER(fofse_geometry), ctypes.c_int32, ctypes.POINTER(vp)]
    L.fofse_create.restype = ctypes.c_int
    L.fofse_target_count.argtypes = [vp]
    L.fofse_target_count.restype = ctypes.c_int32
    L.fofse_set_path.argtypes = [vp, ctypes.c_int32]
    L.fofse_set_path.restype = ctypes.c_int
    L.fofse_set_waves.argtypes = [vp, ctypes.c_int32]
    L.fofse_set_waves.restype = ctypes.c_int
    L.fofse_set_occupancy.argtypes = [vp, ctypes.c_int32]
    L.fofse_set_occupancy.restype = ctypes.c_int
    L.fofse_set_basis.argtypes = [vp, ctypes.c_int32]
    L.fofse_set_basis.restype = ctypes.c_int
    L.fofse_set_compensation.argtypes = [vp, ctypes.c_int32]
    L.fofse_set_compensation.restype = ctypes.c_int
    L.fofse_extrapolate_batch.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, vp]
    L.fofse_extrapolate_batch.restype = ctypes.c_int
    L.fofse_extrapolate_batch_noalloc.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, vp]
    L.fofse_extrapolate_batch_noalloc.restype = ctypes.c_int
    L.fofse_backward.argtypes = [vp, ctypes.c_int32] + [vp] * 10
    L.fofse_backward.restype = ctypes.c_int
    L.fofse_set_timing.argtypes = [vp, ctypes.c_int32]
    L.fofse_set_timing.restype = ctypes.c_int
    L.fofse_kernel_times.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int32]
    L.fofse_kernel_times.restype = ctypes.c_int32
    L.fofse_destroy.argtypes = [vp]
    L.fofse_destroy.restype = None
    L.fofse_create_multi.argtypes = [ctypes.POINTER(fofse_geometry), ctypes.c_int32, ctypes.c_int32,
                                     ctypes.POINTER(vp)]
    L.fofse_create_multi.restype = ctypes.c_int
    L.fofse_multi_geometry_plan.argtypes = [vp, ctypes.c_int32]
    L.fofse_multi_geometry_plan.restype = vp
    L.fofse_extrapolate_multi.argtypes = [vp, ctypes.c_int32] + [vp] * 8
    L.fofse_extrapolate_multi.restype = ctypes.c_int
    L.fofse_destroy_multi.argtypes = [vp]
    L.fofse_destroy_multi.restype = None
    L.fofse_status_str.argtypes = [ctypes.c_int]
    L.fofse_status_str.restype = ctypes.c_char_p
    _lib = L
    return L


# --- one Python function per C entry point (same names) --------------------

def fofse_status_str(status: int) -> str:
    return load_library().fofse_status_str(int(status)).decode()


def fofse_create(area_h: int, area_w: int, fft_size: int, iterations: int,
                 target_mask, device: int = 0) -> int:
    """Returns the opaque plan handle (an int); raises FofseError."""
    L = load_library()
    tm = np.ascontiguousarray(np.asarray(target_mask, dtype=np.uint8).reshape(-1))
    if tm.size != area_h * area_w:
        raise ValueError("target_mask must hold area_h * area_w bytes")
    g = fofse_geometry(area_h, area_w, fft_size, iterations,
                       tm.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    out = ctypes.c_void_p()
    st = L.fofse_create(ctypes.byref(g), int(device), ctypes.byref(out))
    if st != FOFSE_OK:
        raise FofseError(st, "fofse_create")
    return out.value


def fofse_target_count(plan: int) -> int:
    return int(load_library().fofse_target_count(plan))


def fofse_set_path(plan: int, path: int) -> None:
    st = load_library().fofse_set_path(plan, int(path))
    if st != FOFSE_OK:
        raise FofseError(st, "fofse_set_path")


def fofse_set_waves(plan: int, waves: int) -> None:
    st = load_library().fofse_set_waves(plan, int(waves))
    if st != FOFSE_OK:
        raise FofseError(st, "fofse_set_waves")


def fofse_set_occupancy(plan: int, wg_per_cu: int) -> None:
    st = load_library().fofse_set_occupancy(plan, int(wg_per_cu))
    if st != FOFSE_OK:
        raise FofseError(st, "fofse_set_occupancy")


def fofse_set_basis(plan: int, basis: int) -> None:
    st = load_library().fofse_set_basis(plan, int(basis))
    if st != FOFSE_OK:
        raise FofseError(st, "fofse_set_basis")


def fofse_set_compensation(plan: int, mode: int) -> None:
    st = load_library().fofse_set_compensation(plan, int(mode))
    if st != FOFSE_OK:
        raise FofseError(st, "fofse_set_compensation")


def fofse_extrapolate_batch(plan: int, n_blocks: int, d_areas: int, d_known: int,
                            d_rho_gamma: int, d_out: int, d_sel: int, d_coef: int,
                            d_status: int, stream: int) -> None:
    """Raw call with device addresses (ints, 0 for NULL); raises FofseError."""
    st = load_library().fofse_extrapolate_batch(plan, int(n_blocks), d_areas or None,
                                                d_known or None, d_rho_gamma or None,
                                                d_out or None, d_sel or None, d_coef or None,
                                                d_status or None, stream or None)
    if st != FOFSE_OK:
        raise FofseError(st, "fofse_extrapolate_batch")


def fofse_extrapolate_batch_noalloc(plan: int, n_blocks: int, d_areas: int, d_known: int,
                                    d_rho_gamma: int, d_out: int, d_sel: int, d_coef: int,
                                    d_status: int, stream: int) -> None:
    """Raw call with device addresses (ints, 0 for NULL); raises FofseError."""
    st = load_library().fofse_extrapolate_batch_noalloc(plan, int(n_blocks), d_areas or None,
                                                        d_known or None, d_rho_gamma or None,
                                                        d_out or None, d_sel or None, d_coef or None,
                                                        d_status or None, stream or None)
    if st != FOFSE_OK:
        raise FofseError(st, "fofse_extrapolate_batch_noalloc")


def fofse_backward(plan: int, n_blocks: int, d_areas: int, d_known: int, d_rho_gamma: int,
                   d_sel: int, d_coef: int, d_grad_out: int, d_grad_areas: int,
                   d_grad_rho_gamma: int, d_grad_block: int, stream: int) -> None:
    """Raw call with device addresses (ints, 0 for NULL); raises FofseError."""
    st = load_library().fofse_backward(plan, int(n_blocks), d_areas or None, d_known or None,
                                       d_rho_gamma or None, d_sel or None, d_coef or None,
                                       d_grad_out or None, d_grad_areas or None,
                                       d_grad_rho_gamma or None, d_grad_block or None,
                                       stream or None)
    if st != FOFSE_OK:
        raise FofseError(st, "fofse_backward")


def fofse_set_timing(plan: int, enable: bool) -> None:
    st = load_library().fofse_set_timing(plan, 1 if enable else 0)
    if st != FOFSE_OK:
        raise FofseError(st, "fofse_set_timing")


def fofse_kernel_times(plan: int, max_count: int = 256):
    """Main-kernel durations (ms) of the most recent calls, oldest first."""
    buf = (ctypes.c_float * max_count)()
    n = load_library().fofse_kernel_times(plan, buf, max_count)
    return [float(buf[i]) for i in range(n)]


def fofse_destroy(plan: int) -> None:
    load_library().fofse_destroy(plan)


MULTI_MAX_GEOMS = 16


def fofse_create_multi(geometries, device: int = 0) -> int:
    """geometries: sequence of (area_h, area_w, fft_size, iterations,
    target_mask).  Returns the opaque multi-plan handle; raises FofseError."""
    L = load_library()
    masks = [np.ascontiguousarray(np.asarray(g[4], dtype=np.uint8).reshape(-1)) for g in geometries]
    arr = (fofse_geometry * len(geometries))()
    for i, (g, tm) in enumerate(zip(geometries, masks)):
        if tm.size != g[0] * g[1]:
            raise ValueError("target_mask must hold area_h * area_w bytes")
        arr[i] = fofse_geometry(g[0], g[1], g[2], g[3], tm.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    out = ctypes.c_void_p()
    st = L.fofse_create_multi(arr, len(geometries), int(device), ctypes.byref(out))
    if st != FOFSE_OK:
        raise FofseError(st, "fofse_create_multi")
    return out.value


def fofse_multi_geometry_plan(mplan: int, geom: int) -> int:
    return load_library().fofse_multi_geometry_plan(mplan, int(geom)) or 0


def fofse_extrapolate_multi(mplan: int, n_blocks: int, d_geom_id: int, d_areas: int, d_area_off: int,
                            d_known: int, d_rho_gamma: int, d_out: int, d_status: int, stream: int) -> None:
    """Raw call with device addresses (ints, 0 for NULL); raises FofseError."""
    st = load_library().fofse_extrapolate_multi(mplan, int(n_blocks), d_geom_id or None, d_areas or None,
                                                d_area_off or None, d_known or None, d_rho_gamma or None,
                                                d_out or None, d_status or None, stream or None)
    if st != FOFSE_OK:
        raise FofseError(st, "fofse_extrapolate_multi")


def fofse_destroy_multi(mplan: int) -> None:
    load_library().fofse_destroy_multi(mplan)


# --- torch convenience wrapper ---------------------------------------------

class Plan:
    """A geometry (area M x N, FFT size T, K iterations, missing area B) bound
    to one device.  Tensors are passed by address to the C ABI."""

    def __init__(self, area_h: int, area_w: int, fft_size: int, iterations: int,
                 target_mask, device: int = 0):
        self.M, self.N, self.T, self.K = int(area_h), int(area_w), int(fft_size), int(iterations)
        self.device = int(device)
        self.target_mask = np.asarray(target_mask, dtype=np.uint8).reshape(self.M, self.N)
        self.handle = fofse_create(self.M, self.N, self.T, self.K, self.target_mask, self.device)
        self.nB = fofse_target_count(self.handle)

    def set_path(self, path: int):
        fofse_set_path(self.handle, path)

    def set_waves(self, waves: int):
        fofse_set_waves(self.handle, waves)

    def set_occupancy(self, wg_per_cu: int):
        fofse_set_occupancy(self.handle, wg_per_cu)

    def set_basis(self, basis: int):
        """FOFSE_BASIS_DFT (default) or FOFSE_BASIS_DCT; with the DCT the
        record holds keys k*T + l in [0, T*T) and real coefficients (c, 0)."""
        fofse_set_basis(self.handle, basis)

    def set_compensation(self, mode: int):
        """FOFSE_COMP_CONSTANT (eq. 14, default) or FOFSE_COMP_FULL (eqs. 10-13)."""
        fofse_set_compensation(self.handle, mode)

    def close(self):
        if getattr(self, "handle", None):
            fofse_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def extrapolate(self, areas, rho_gamma, known=None, out=None, record: bool = False,
                    status: bool = True, stream=None):
        """areas: cuda float32 [n, M, N]; rho_gamma: cuda float64 [2];
        known: cuda uint8 [n, M, N] or None.  Returns (out [n, nB] float32,
        sel [n, K] int32 or None, coef [n, K, 2] float64 or None,
        status [n] int32 or None); all on the device, enqueued on ``stream``
        (default: torch's current stream)."""
        import torch
        dev = torch.device("cuda", self.device)
        n = int(areas.shape[0])
        _check(areas, torch.float32, (n, self.M, self.N), dev, "areas")
        _check(rho_gamma, torch.float64, (2,), dev, "rho_gamma")
        if known is not None:
            _check(known, torch.uint8, (n, self.M, self.N), dev, "known")
        if out is None:
            out = torch.empty((n, self.nB), dtype=torch.float32, device=dev)
        else:
            _check(out, torch.float32, (n, self.nB), dev, "out")
        sel = coef = st = None
        if record:
            sel = torch.empty((n, self.K), dtype=torch.int32, device=dev)
            coef = torch.empty((n, self.K, 2), dtype=torch.float64, device=dev)
        if status:
            st = torch.empty((n,), dtype=torch.int32, device=dev)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        fofse_extrapolate_batch(self.handle, n, areas.data_ptr(),
                                known.data_ptr() if known is not None else 0,
                                rho_gamma.data_ptr(), out.data_ptr(),
                                sel.data_ptr() if sel is not None else 0,
                                coef.data_ptr() if coef is not None else 0,
                                st.data_ptr() if st is not None else 0,
                                stream.cuda_stream)
        return out, sel, coef, st


    def backward(self, areas, rho_gamma, sel, coef, grad_out, known=None,
                 grad_areas: bool = True, per_block: bool = False, stream=None):
        """Adjoint of :meth:`extrapolate` for its record (sel, coef).

        grad_out: cuda float32 [n, nB] = dL/dg on B.  Returns (grad_areas
        float32 [n, M, N] or None, grad_rho_gamma float64 [2] summed over the
        blocks, grad_block float64 [n, 2] or None), enqueued on ``stream``."""
        import torch
        dev = torch.device("cuda", self.device)
        n = int(areas.shape[0])
        _check(areas, torch.float32, (n, self.M, self.N), dev, "areas")
        _check(rho_gamma, torch.float64, (2,), dev, "rho_gamma")
        _check(sel, torch.int32, (n, self.K), dev, "sel")
        _check(coef, torch.float64, (n, self.K, 2), dev, "coef")
        _check(grad_out, torch.float32, (n, self.nB), dev, "grad_out")
        if known is not None:
            _check(known, torch.uint8, (n, self.M, self.N), dev, "known")
        ga = torch.empty((n, self.M, self.N), dtype=torch.float32, device=dev) if grad_areas else None
        grg = torch.zeros((2,), dtype=torch.float64, device=dev)
        gb = torch.empty((n, 2), dtype=torch.float64, device=dev) if per_block else None
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        fofse_backward(self.handle, n, areas.data_ptr(),
                       known.data_ptr() if known is not None else 0,
                       rho_gamma.data_ptr(), sel.data_ptr(), coef.data_ptr(), grad_out.data_ptr(),
                       ga.data_ptr() if ga is not None else 0, grg.data_ptr(),
                       gb.data_ptr() if gb is not None else 0, stream.cuda_stream)
        return ga, grg, gb


def _check(t, dtype, shape, dev, name):
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or t.device != dev or not t.is_contiguous():
        raise ValueError(f"{name}: expected contiguous {dtype} {tuple(shape)} on {dev}, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")
