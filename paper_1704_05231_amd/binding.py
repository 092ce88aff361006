"""ctypes binding of libgabor (include/libgabor.h).

Argument marshalling only: every step of the filter runs in the HIP kernels
of libgabor.so.  PyTorch supplies device memory (``data_ptr()``) and the
current HIP stream.  There is no fallback: if libgabor.so is missing or no
GPU is visible, calls raise.

The functions keep the C names: ``gabor_bank_plan``, ``gabor_bank_apply``,
``gabor_bank_destroy``, ``lsdft_apply``, ``lsdft_work``, ``sdft_box_apply``,
``gabor_bank_plan_info``, ``gabor_status_string``.  ``GaborBank`` wraps a
plan for torch tensors, ``lsdft`` wraps ``lsdft_apply`` and ``sdft_box``
wraps ``sdft_box_apply``.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgabor.so")

GABOR_OK = 0
STATUS = {0: "GABOR_OK", 1: "GABOR_ERR_INVALID_ARG", 2: "GABOR_ERR_OUT_OF_MEMORY",
          3: "GABOR_ERR_DEVICE", 4: "GABOR_ERR_UNSUPPORTED"}
BOUNDARY = {"zero": 0, "mirror": 1}
PRECISION = {"fp32": 0, "bf16_split": 1, "fp16_split": 2, "bf16": 3, "fp16": 4}

# Every symbol include/libgabor.h declares; the CPU tests check the exports.
EXPORTS = ["gabor_status_string", "gabor_bank_plan", "gabor_bank_plan_iir", "gabor_bank_apply", "gabor_bank_apply_adjoint",
           "gabor_bank_apply_adjoint_noalloc", "gabor_bank_apply_batched", "gabor_bank_apply_adjoint_batched",
           "gabor_bank_destroy", "gabor_batch_create", "gabor_batch_apply", "gabor_batch_info",
           "gabor_batch_destroy", "gabor_bank_autotune", "gabor_bank_get_tuning", "gabor_bank_set_tuning",
           "gabor_bank_get_grouping", "gabor_bank_set_grouping", "lsdft_apply", "lsdft_work", "sdft_box_apply", "gabor_bank_plan_info", "gabor_profile_enable",
           "gabor_profile_read"]


class GaborError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS.get(status, status)}")
        self.status = status


class PlanInfo(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("n_freq", ctypes.c_int32), ("n_orient", ctypes.c_int32),
                ("max_radius", ctypes.c_int32), ("n_row_passes", ctypes.c_int32),
                ("n_col_passes", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_int64), ("real_macs", ctypes.c_int64),
                ("row_real_macs", ctypes.c_int64), ("col_real_macs", ctypes.c_int64)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("real_macs", ctypes.c_int64),
                ("bytes", ctypes.c_int64)]


_lib = None


def load():
    """Load libgabor.so (built in-tree by paper_1704_05231_amd.build;
    LIBGABOR_LIBRARY may name another build of the same ABI)."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("LIBGABOR_LIBRARY", LIB_PATH)
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run python -m paper_1704_05231_amd.build")
    lib = ctypes.CDLL(path)
    P, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.gabor_status_string.argtypes = [ctypes.c_int]
    lib.gabor_status_string.restype = ctypes.c_char_p
    lib.gabor_bank_plan.argtypes = [ctypes.POINTER(P), i32, i32, i32, P, P, i32, P, f64,
                                    ctypes.c_int, ctypes.c_int, P]
    lib.gabor_bank_plan.restype = ctypes.c_int
    lib.gabor_bank_plan_iir.argtypes = [ctypes.POINTER(P), i32, i32, i32, P, P, i32, P, ctypes.c_int, P]
    lib.gabor_bank_plan_iir.restype = ctypes.c_int
    lib.gabor_bank_apply.argtypes = [P, P, i64, P, P]
    lib.gabor_bank_apply.restype = ctypes.c_int
    lib.gabor_bank_apply_adjoint.argtypes = [P, P, P, i64, P]
    lib.gabor_bank_apply_adjoint.restype = ctypes.c_int
    lib.gabor_bank_apply_adjoint_noalloc.argtypes = [P, P, P, i64, P]
    lib.gabor_bank_apply_adjoint_noalloc.restype = ctypes.c_int
    lib.gabor_bank_apply_batched.argtypes = [P, P, i32, i64, i64, P, P]
    lib.gabor_bank_apply_batched.restype = ctypes.c_int
    lib.gabor_bank_apply_adjoint_batched.argtypes = [P, P, i32, P, i64, i64, P]
    lib.gabor_bank_apply_adjoint_batched.restype = ctypes.c_int
    lib.gabor_bank_destroy.argtypes = [P]
    lib.gabor_bank_destroy.restype = ctypes.c_int
    lib.gabor_bank_plan_info.argtypes = [P, ctypes.POINTER(PlanInfo)]
    lib.gabor_bank_plan_info.restype = ctypes.c_int
    lib.gabor_batch_create.argtypes = [ctypes.POINTER(P), P, i32, P, P, P, P, P, P]
    lib.gabor_batch_create.restype = ctypes.c_int
    lib.gabor_batch_apply.argtypes = [P, P]
    lib.gabor_batch_apply.restype = ctypes.c_int
    lib.gabor_batch_info.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i64)]
    lib.gabor_batch_info.restype = ctypes.c_int
    lib.gabor_batch_destroy.argtypes = [P]
    lib.gabor_batch_destroy.restype = ctypes.c_int
    lib.gabor_bank_autotune.argtypes = [P, P, i64, P, i32, P]
    lib.gabor_bank_autotune.restype = ctypes.c_int
    lib.gabor_bank_get_tuning.argtypes = [P, P, i32, ctypes.POINTER(i32)]
    lib.gabor_bank_get_tuning.restype = ctypes.c_int
    lib.gabor_bank_set_tuning.argtypes = [P, P, i32]
    lib.gabor_bank_set_tuning.restype = ctypes.c_int
    lib.gabor_bank_get_grouping.argtypes = [P, ctypes.POINTER(i32)]
    lib.gabor_bank_get_grouping.restype = ctypes.c_int
    lib.gabor_bank_set_grouping.argtypes = [P, i32]
    lib.gabor_bank_set_grouping.restype = ctypes.c_int
    lib.lsdft_apply.argtypes = [P, i32, i32, i64, i32, i32, f64, ctypes.c_int, ctypes.c_int, P, P]
    lib.lsdft_apply.restype = ctypes.c_int
    lib.lsdft_work.argtypes = [i32, i32, i32, i32, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.lsdft_work.restype = ctypes.c_int
    lib.sdft_box_apply.argtypes = [P, i32, i32, i64, i32, i32, ctypes.c_int, P, P]
    lib.sdft_box_apply.restype = ctypes.c_int
    lib.gabor_profile_enable.argtypes = [P, i32]
    lib.gabor_profile_enable.restype = ctypes.c_int
    lib.gabor_profile_read.argtypes = [P, ctypes.POINTER(KernelStat), i32, ctypes.POINTER(i32)]
    lib.gabor_profile_read.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != GABOR_OK:
        raise GaborError(status, what)


def _f64(a):
    if a is None:
        return None
    return np.ascontiguousarray(np.atleast_1d(np.asarray(a, dtype=np.float64)))


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def gabor_status_string(status: int) -> str:
    return load().gabor_status_string(int(status)).decode()


def gabor_bank_plan(height, width, omega, sigma, n_orient, theta=None, radius_sigmas=3.0,
                    boundary="zero", precision="fp32", stream=None) -> ctypes.c_void_p:
    om, sg, th = _f64(omega), _f64(sigma), _f64(theta)
    if om.shape != sg.shape:
        raise ValueError("omega and sigma must have the same length")
    if th is not None and th.size != n_orient:
        raise ValueError("theta must have n_orient entries")
    plan = ctypes.c_void_p()
    st = load().gabor_bank_plan(ctypes.byref(plan), int(height), int(width), om.size, _p(om),
                                _p(sg), int(n_orient), _p(th), float(radius_sigmas),
                                BOUNDARY[boundary], PRECISION[precision], _stream(stream))
    _check(st, "gabor_bank_plan")
    return plan


def gabor_bank_plan_iir(height, width, omega, sigma, n_orient, theta=None, boundary="zero",
                        stream=None) -> ctypes.c_void_p:
    om, sg, th = _f64(omega), _f64(sigma), _f64(theta)
    if om.shape != sg.shape:
        raise ValueError("omega and sigma must have the same length")
    if th is not None and th.size != n_orient:
        raise ValueError("theta must have n_orient entries")
    plan = ctypes.c_void_p()
    st = load().gabor_bank_plan_iir(ctypes.byref(plan), int(height), int(width), om.size, _p(om), _p(sg),
                                    int(n_orient), _p(th), BOUNDARY[boundary], _stream(stream))
    _check(st, "gabor_bank_plan_iir")
    return plan


def gabor_bank_apply(plan, d_image: int, row_stride_elems: int, d_out: int, stream=None):
    st = load().gabor_bank_apply(plan, ctypes.c_void_p(d_image), int(row_stride_elems),
                                 ctypes.c_void_p(d_out), _stream(stream))
    _check(st, "gabor_bank_apply")


def gabor_bank_apply_adjoint(plan, d_grad_out: int, d_grad_image: int, grad_row_stride_elems: int,
                             stream=None):
    st = load().gabor_bank_apply_adjoint(plan, ctypes.c_void_p(d_grad_out), ctypes.c_void_p(d_grad_image),
                                         int(grad_row_stride_elems), _stream(stream))
    _check(st, "gabor_bank_apply_adjoint")


def gabor_bank_apply_adjoint_noalloc(plan, d_grad_out: int, d_grad_image: int, grad_row_stride_elems: int,
                                     stream=None):
    st = load().gabor_bank_apply_adjoint_noalloc(plan, ctypes.c_void_p(d_grad_out), ctypes.c_void_p(d_grad_image),
                                                 int(grad_row_stride_elems), _stream(stream))
    _check(st, "gabor_bank_apply_adjoint_noalloc")


def gabor_bank_apply_batched(plan, d_images: int, n_images: int, image_stride_elems: int, row_stride_elems: int,
                             d_out: int, stream=None):
    st = load().gabor_bank_apply_batched(plan, ctypes.c_void_p(d_images), int(n_images), int(image_stride_elems),
                                         int(row_stride_elems), ctypes.c_void_p(d_out), _stream(stream))
    _check(st, "gabor_bank_apply_batched")


def gabor_bank_apply_adjoint_batched(plan, d_grad_out: int, n_images: int, d_grad_images: int,
                                     grad_image_stride_elems: int, grad_row_stride_elems: int, stream=None):
    st = load().gabor_bank_apply_adjoint_batched(plan, ctypes.c_void_p(d_grad_out), int(n_images),
                                                 ctypes.c_void_p(d_grad_images), int(grad_image_stride_elems),
                                                 int(grad_row_stride_elems), _stream(stream))
    _check(st, "gabor_bank_apply_adjoint_batched")


def gabor_bank_destroy(plan):
    _check(load().gabor_bank_destroy(plan), "gabor_bank_destroy")


def gabor_bank_autotune(plan, d_image: int, row_stride_elems: int, d_out: int, reps: int = 5, stream=None):
    _check(load().gabor_bank_autotune(plan, ctypes.c_void_p(d_image), int(row_stride_elems),
                                      ctypes.c_void_p(d_out), int(reps), _stream(stream)), "gabor_bank_autotune")


def gabor_bank_get_tuning(plan) -> list[int]:
    n = ctypes.c_int32()
    _check(load().gabor_bank_get_tuning(plan, None, 0, ctypes.byref(n)), "gabor_bank_get_tuning")
    arr = np.zeros(n.value, dtype=np.int32)
    _check(load().gabor_bank_get_tuning(plan, _p(arr), arr.size, ctypes.byref(n)), "gabor_bank_get_tuning")
    return [int(v) for v in arr]


def gabor_bank_set_tuning(plan, seg_rows):
    arr = np.ascontiguousarray(seg_rows, dtype=np.int32)
    _check(load().gabor_bank_set_tuning(plan, _p(arr), arr.size), "gabor_bank_set_tuning")


def gabor_bank_get_grouping(plan) -> int:
    g = ctypes.c_int32()
    _check(load().gabor_bank_get_grouping(plan, ctypes.byref(g)), "gabor_bank_get_grouping")
    return int(g.value)


def gabor_bank_set_grouping(plan, group_small: int):
    _check(load().gabor_bank_set_grouping(plan, int(group_small)), "gabor_bank_set_grouping")


def gabor_batch_create(plan, d_images, heights, widths, row_strides, d_outs, stream=None):
    n = len(d_images)
    if not (len(heights) == len(widths) == len(row_strides) == len(d_outs) == n):
        raise ValueError("batch arrays must have one entry per image")
    imgs = (ctypes.c_void_p * n)(*[int(x) for x in d_images])
    outs = (ctypes.c_void_p * n)(*[int(x) for x in d_outs])
    hs = np.ascontiguousarray(heights, dtype=np.int32)
    ws = np.ascontiguousarray(widths, dtype=np.int32)
    ss = np.ascontiguousarray(row_strides, dtype=np.int64)
    batch = ctypes.c_void_p()
    st = load().gabor_batch_create(ctypes.byref(batch), plan, n, ctypes.cast(imgs, ctypes.c_void_p), _p(hs),
                                   _p(ws), _p(ss), ctypes.cast(outs, ctypes.c_void_p), _stream(stream))
    _check(st, "gabor_batch_create")
    return batch


def gabor_batch_apply(batch, stream=None):
    _check(load().gabor_batch_apply(batch, _stream(stream)), "gabor_batch_apply")


def gabor_batch_info(batch) -> tuple[int, int]:
    nl, nt = ctypes.c_int32(), ctypes.c_int64()
    _check(load().gabor_batch_info(batch, ctypes.byref(nl), ctypes.byref(nt)), "gabor_batch_info")
    return nl.value, nt.value


def gabor_batch_destroy(batch):
    _check(load().gabor_batch_destroy(batch), "gabor_batch_destroy")


def lsdft_apply(d_image: int, height, width, row_stride_elems, m_y, m_x, sigma, boundary="zero",
                precision="fp32", d_out: int = 0, stream=None):
    st = load().lsdft_apply(ctypes.c_void_p(d_image), int(height), int(width), int(row_stride_elems),
                            int(m_y), int(m_x), float(sigma), BOUNDARY[boundary], PRECISION[precision],
                            ctypes.c_void_p(d_out), _stream(stream))
    _check(st, "lsdft_apply")


def lsdft_work(height, width, m_y, m_x) -> tuple[int, int]:
    """(real multiply-adds, bytes) of one lsdft_apply."""
    macs, nbytes = ctypes.c_int64(), ctypes.c_int64()
    _check(load().lsdft_work(int(height), int(width), int(m_y), int(m_x), ctypes.byref(macs),
                             ctypes.byref(nbytes)), "lsdft_work")
    return macs.value, nbytes.value


def lsdft(img, m_y, m_x, sigma, boundary="zero", precision="fp32", out=None, stream=None):
    """Localized SDFT of a (H, W) float32 GPU tensor (row stride may exceed
    W): complex64 [m_y, m_x, H, W], bin (v, u) at out[v, u]."""
    import torch
    if img.dtype != torch.float32 or img.dim() != 2 or not img.is_cuda or img.stride(1) != 1:
        raise ValueError("image must be a row-major 2-D float32 GPU tensor")
    H, W = img.shape
    if out is None:
        out = torch.empty((m_y, m_x, H, W), dtype=torch.complex64, device=img.device)
    elif out.dtype != torch.complex64 or not out.is_contiguous() or tuple(out.shape) != (m_y, m_x, H, W):
        raise ValueError("out must be a contiguous complex64 [m_y, m_x, H, W] tensor")
    lsdft_apply(img.data_ptr(), H, W, img.stride(0), m_y, m_x, sigma, boundary, precision,
                out.data_ptr(), stream)
    return out


def sdft_box_apply(d_image: int, height, width, row_stride_elems, m_y, m_x, boundary="zero",
                   d_out: int = 0, stream=None):
    st = load().sdft_box_apply(ctypes.c_void_p(d_image), int(height), int(width), int(row_stride_elems),
                               int(m_y), int(m_x), BOUNDARY[boundary], ctypes.c_void_p(d_out),
                               _stream(stream))
    _check(st, "sdft_box_apply")


def sdft_box(img, m_y, m_x, boundary="zero", out=None, stream=None):
    """Box-window sliding DFT of a (H, W) float32 GPU tensor (row stride may
    exceed W): complex64 [m_y, m_x, H, W], bin (v, u) at out[v, u]."""
    import torch
    if img.dtype != torch.float32 or img.dim() != 2 or not img.is_cuda or img.stride(1) != 1:
        raise ValueError("image must be a row-major 2-D float32 GPU tensor")
    H, W = img.shape
    if out is None:
        out = torch.empty((m_y, m_x, H, W), dtype=torch.complex64, device=img.device)
    elif out.dtype != torch.complex64 or not out.is_contiguous() or tuple(out.shape) != (m_y, m_x, H, W):
        raise ValueError("out must be a contiguous complex64 [m_y, m_x, H, W] tensor")
    sdft_box_apply(img.data_ptr(), H, W, img.stride(0), m_y, m_x, boundary, out.data_ptr(), stream)
    return out


def gabor_bank_plan_info(plan) -> PlanInfo:
    info = PlanInfo()
    _check(load().gabor_bank_plan_info(plan, ctypes.byref(info)), "gabor_bank_plan_info")
    return info


def gabor_profile_enable(plan, enable: bool):
    _check(load().gabor_profile_enable(plan, int(bool(enable))), "gabor_profile_enable")


def gabor_profile_read(plan) -> dict:
    """{kernel name: {launches, total_ms, real_macs, bytes}} of the launches
    timed so far (real_macs and bytes are algorithmic, per launch)."""
    cap = 64
    arr = (KernelStat * cap)()
    n = ctypes.c_int32()
    _check(load().gabor_profile_read(plan, arr, cap, ctypes.byref(n)), "gabor_profile_read")
    return {arr[i].name.decode(): {"launches": int(arr[i].launches), "total_ms": float(arr[i].total_ms),
                                   "real_macs": int(arr[i].real_macs), "bytes": int(arr[i].bytes)}
            for i in range(min(n.value, cap))}


class GaborBank:
    """A plan bound to one image size, for torch tensors on the GPU.

    ``bank(img)`` takes a (H, W) float32 CUDA tensor (row stride may exceed W)
    and returns a complex64 tensor [O, N, H, W] on the same device.  The
    float16 forms (``fp16``, ``fp16_split``) scale the image by 2^8, so its
    pixels must satisfy |f| < 128; larger values overflow to Inf/NaN outputs
    without an error.
    """

    def __init__(self, height, width, omegas, sigmas, n_orient=None, thetas=None,
                 radius_sigmas=3.0, boundary="zero", precision="fp32", smoother="fir"):
        if thetas is not None:
            thetas = _f64(thetas)
            n_orient = thetas.size if n_orient is None else n_orient
        self.height, self.width = int(height), int(width)
        self.n_freq = _f64(omegas).size
        self.n_orient = int(n_orient)
        self.precision = precision
        self.params = {"height": self.height, "width": self.width,
                       "omegas": [float(v) for v in _f64(omegas)], "sigmas": [float(v) for v in _f64(sigmas)],
                       "n_orient": self.n_orient,
                       "thetas": None if thetas is None else [float(v) for v in thetas],
                       "radius_sigmas": float(radius_sigmas), "boundary": boundary, "precision": precision}
        self.params["smoother"] = smoother
        if smoother == "iir":
            self._plan = gabor_bank_plan_iir(height, width, omegas, sigmas, self.n_orient, thetas, boundary)
        elif smoother == "fir":
            self._plan = gabor_bank_plan(height, width, omegas, sigmas, self.n_orient, thetas,
                                         radius_sigmas, boundary, precision)
        else:
            raise ValueError("smoother must be 'fir' or 'iir'")

    @property
    def info(self) -> PlanInfo:
        return gabor_bank_plan_info(self._plan)

    def __call__(self, img, out=None, stream=None):
        import torch
        if img.dtype != torch.float32 or img.dim() != 2 or not img.is_cuda:
            raise ValueError("image must be a 2-D float32 GPU tensor")
        if tuple(img.shape) != (self.height, self.width) or img.stride(1) != 1:
            raise ValueError("image shape does not match the plan or is not row-major")
        if out is None:
            out = torch.empty((self.n_freq, self.n_orient, self.height, self.width),
                              dtype=torch.complex64, device=img.device)
        elif (out.dtype != torch.complex64 or not out.is_contiguous()
              or tuple(out.shape) != (self.n_freq, self.n_orient, self.height, self.width)):
            raise ValueError("out must be a contiguous complex64 [O, N, H, W] tensor")
        gabor_bank_apply(self._plan, img.data_ptr(), img.stride(0), out.data_ptr(), stream)
        return out

    def adjoint(self, grad_out, grad_img=None, stream=None):
        """dL/df (float32 [H, W]) from dL/dF (complex64 [O, N, H, W])."""
        import torch
        if (grad_out.dtype != torch.complex64 or not grad_out.is_contiguous() or not grad_out.is_cuda
                or tuple(grad_out.shape) != (self.n_freq, self.n_orient, self.height, self.width)):
            raise ValueError("grad_out must be a contiguous complex64 [O, N, H, W] GPU tensor")
        if grad_img is None:
            grad_img = torch.empty((self.height, self.width), dtype=torch.float32, device=grad_out.device)
        elif (grad_img.dtype != torch.float32 or grad_img.dim() != 2 or grad_img.stride(1) != 1
              or tuple(grad_img.shape) != (self.height, self.width)):
            raise ValueError("grad_img must be a row-major float32 [H, W] tensor")
        gabor_bank_apply_adjoint(self._plan, grad_out.data_ptr(), grad_img.data_ptr(), grad_img.stride(0),
                                 stream)
        return grad_img

    def apply_batched(self, imgs, out=None, stream=None):
        """Every image of a float32 [B, H, W] GPU tensor (rows contiguous)
        into complex64 [B, O, N, H, W]: one launch per frequency."""
        import torch
        if imgs.dtype != torch.float32 or imgs.dim() != 3 or not imgs.is_cuda:
            raise ValueError("images must be a 3-D float32 GPU tensor")
        if tuple(imgs.shape[1:]) != (self.height, self.width) or imgs.stride(2) != 1:
            raise ValueError("image shape does not match the plan or rows are not contiguous")
        B = imgs.shape[0]
        shape = (B, self.n_freq, self.n_orient, self.height, self.width)
        if out is None:
            out = torch.empty(shape, dtype=torch.complex64, device=imgs.device)
        elif out.dtype != torch.complex64 or not out.is_contiguous() or tuple(out.shape) != shape:
            raise ValueError("out must be a contiguous complex64 [B, O, N, H, W] tensor")
        gabor_bank_apply_batched(self._plan, imgs.data_ptr(), B, imgs.stride(0), imgs.stride(1), out.data_ptr(),
                                 stream)
        return out

    def adjoint_batched(self, grad_out, grad_imgs=None, stream=None):
        """dL/df (float32 [B, H, W]) from dL/dF (complex64 [B, O, N, H, W])."""
        import torch
        B = grad_out.shape[0] if grad_out.dim() == 5 else -1
        if (grad_out.dtype != torch.complex64 or not grad_out.is_contiguous() or not grad_out.is_cuda
                or tuple(grad_out.shape) != (B, self.n_freq, self.n_orient, self.height, self.width)):
            raise ValueError("grad_out must be a contiguous complex64 [B, O, N, H, W] GPU tensor")
        if grad_imgs is None:
            grad_imgs = torch.empty((B, self.height, self.width), dtype=torch.float32, device=grad_out.device)
        elif (grad_imgs.dtype != torch.float32 or grad_imgs.dim() != 3 or grad_imgs.stride(2) != 1
              or tuple(grad_imgs.shape) != (B, self.height, self.width)):
            raise ValueError("grad_imgs must be a float32 [B, H, W] tensor with contiguous rows")
        gabor_bank_apply_adjoint_batched(self._plan, grad_out.data_ptr(), B, grad_imgs.data_ptr(),
                                         grad_imgs.stride(0), grad_imgs.stride(1), stream)
        return grad_imgs

    def autotune(self, img, out=None, reps: int = 5, stream=None) -> list[int]:
        """Time the candidate schedules on img (and out, overwritten); keep the fastest."""
        import torch
        if out is None:
            out = torch.empty((self.n_freq, self.n_orient, self.height, self.width),
                              dtype=torch.complex64, device=img.device)
        gabor_bank_autotune(self._plan, img.data_ptr(), img.stride(0), out.data_ptr(), reps, stream)
        return self.tuning

    @property
    def tuning(self) -> list[int]:
        return gabor_bank_get_tuning(self._plan)

    @tuning.setter
    def tuning(self, seg_rows):
        gabor_bank_set_tuning(self._plan, seg_rows)

    @property
    def grouping(self) -> int:
        """1: the small operand sizes run in one launch (see gabor_bank_set_grouping)."""
        return gabor_bank_get_grouping(self._plan)

    @grouping.setter
    def grouping(self, group_small: int):
        gabor_bank_set_grouping(self._plan, group_small)

    def profile(self, enable: bool = True):
        gabor_profile_enable(self._plan, enable)

    def profile_read(self) -> dict:
        return gabor_profile_read(self._plan)

    def close(self):
        if self._plan:
            gabor_bank_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GaborBatch:
    """Images of uneven sizes bound to one bank: ``batch()`` fills the bound
    complex64 outputs [O, N, h_i, w_i] (``batch.outputs``).  The images and
    outputs must stay alive and in place while the batch exists."""

    def __init__(self, bank: "GaborBank", images, outputs=None, stream=None):
        import torch
        for im in images:
            if im.dtype != torch.float32 or im.dim() != 2 or not im.is_cuda or im.stride(1) != 1:
                raise ValueError("images must be row-major 2-D float32 GPU tensors")
        if outputs is None:
            outputs = [torch.empty((bank.n_freq, bank.n_orient, im.shape[0], im.shape[1]),
                                   dtype=torch.complex64, device=im.device) for im in images]
        for im, o in zip(images, outputs):
            if (o.dtype != torch.complex64 or not o.is_contiguous()
                    or tuple(o.shape) != (bank.n_freq, bank.n_orient, im.shape[0], im.shape[1])):
                raise ValueError("outputs must be contiguous complex64 [O, N, h, w] tensors")
        self.bank, self.images, self.outputs = bank, list(images), list(outputs)
        self._batch = gabor_batch_create(bank._plan, [im.data_ptr() for im in images],
                                         [im.shape[0] for im in images], [im.shape[1] for im in images],
                                         [im.stride(0) for im in images], [o.data_ptr() for o in outputs],
                                         stream)

    def __call__(self, stream=None):
        gabor_batch_apply(self._batch, stream)
        return self.outputs

    @property
    def info(self) -> tuple[int, int]:
        return gabor_batch_info(self._batch)

    def close(self):
        if self._batch:
            gabor_batch_destroy(self._batch)
            self._batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_thetas(n: int) -> np.ndarray:
    return np.array([math.pi * k / n for k in range(n)])
