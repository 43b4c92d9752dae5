"""Python binding of the C ABI: the same entry points, taking torch tensors.

PyTorch supplies device memory and the current stream; every computation runs
in the HIP kernels of libttcconv.so.  Functions raise when the library is not
built or a tensor is not on the GPU.
"""
from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L

_DT = {torch.uint8: L.TC_U8, torch.float16: L.TC_F16, torch.float32: L.TC_F32, torch.int32: L.TC_I32,
       torch.float64: L.TC_F64}


def _lib():
    return L.load()


def _stream(stream=None) -> C.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _desc(t: torch.Tensor) -> L.TcTensor:
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if t.dtype not in _DT:
        raise ValueError(f"unsupported dtype {t.dtype}")
    d = L.TcTensor()
    d.data = t.data_ptr() if t.numel() > 0 else None
    d.dtype = _DT[t.dtype]
    d.ndim = t.dim()
    for i, (n, s) in enumerate(zip(t.shape, t.stride())):
        d.shape[i] = n
        d.stride[i] = s
    return d


def _shape_desc(shape, dtype_code: int) -> L.TcTensor:
    d = L.TcTensor()
    d.data = None
    d.dtype = dtype_code
    d.ndim = len(shape)
    for i, n in enumerate(shape):
        d.shape[i] = int(n)
        d.stride[i] = 1
    return d


def version() -> int:
    return _lib().tc_version()


def device_check(device: int = 0) -> int:
    """Number of compute units of a gfx950 device (raises on any other device)."""
    n = C.c_int(0)
    L.check("tc_device_check", _lib().tc_device_check(device, C.byref(n)))
    return n.value


# ----------------------------------------------------------------------------- convolution
def conv_out_shape(xshape, kshape, mode: str = "full", xdtype=torch.float32, kdtype=torch.float32):
    lib = _lib()
    out = (C.c_int64 * L.TC_MAX_DIMS)()
    L.check("tc_conv_out_shape", lib.tc_conv_out_shape(C.byref(_shape_desc(xshape, _DT[xdtype])),
                                                       C.byref(_shape_desc(kshape, _DT[kdtype])),
                                                       L.MODES[mode], out))
    return tuple(out[i] for i in range(len(xshape)))


def conv_nd(x: torch.Tensor, k: torch.Tensor, mode: str = "full", out: Optional[torch.Tensor] = None, stream=None,
            k_abs_sum: Optional[int] = None):
    """y = x (*) k, true n-D convolution by the direct kernels (f32*f32->f32,
    f16*f32->f32, u8*i32->i32).  An int32 kernel needs its sum |k|, a host
    value: pass `k_abs_sum`, or it is read from k here (one device-to-host
    read, so such a call cannot be recorded into a graph)."""
    if k.dtype == torch.int32:
        if k_abs_sum is None:
            k_abs_sum = int(k.detach().to(torch.int64).abs().sum().item())
        return conv_nd_ex(x, k, mode, method="direct", k_abs_sum=k_abs_sum, out=out, stream=stream)
    lib = _lib()
    shape = conv_out_shape(tuple(x.shape), tuple(k.shape), mode, x.dtype, k.dtype)
    ydt = torch.int32 if x.dtype == torch.uint8 else torch.float32
    if out is None:
        out = torch.empty(shape, dtype=ydt, device=x.device)
    L.check("tc_conv_nd", lib.tc_conv_nd(C.byref(_desc(x)), C.byref(_desc(k)), L.MODES[mode], C.byref(_desc(out)),
                                         _stream(stream)))
    return out


def conv_workspace_size(x: torch.Tensor, k: torch.Tensor, mode: str = "full", method: str = "auto") -> int:
    n = C.c_size_t(0)
    L.check("tc_conv_workspace_size",
            _lib().tc_conv_workspace_size(C.byref(_desc(x)), C.byref(_desc(k)), L.MODES[mode], L.METHODS[method],
                                          C.byref(n)))
    return n.value


def conv_nd_ex(x: torch.Tensor, k: torch.Tensor, mode: str = "full", method: str = "auto",
               k_abs_sum: Optional[int] = None, k_host: Optional[np.ndarray] = None, fft_threshold: int = 0,
               ws: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None, stream=None,
               band_rows: int = 0):
    """tc_conv_nd_ex: the convolution with the library's method choice.
    `k_host` (a contiguous numpy copy of k) lets the library take sum |k| of an
    int32 kernel and test a square FP32 kernel for separability; `ws` is the
    FFT branch's device workspace (allocated here when None and the method
    may take the FFT branch); `band_rows` forces the output rows per wave of
    the row-streaming direct kernels (2, 4, 8; 0 = the library's table)."""
    lib = _lib()
    shape = conv_out_shape(tuple(x.shape), tuple(k.shape), mode, x.dtype, k.dtype)
    ydt = torch.int32 if x.dtype == torch.uint8 else torch.float32
    if out is None:
        out = torch.empty(shape, dtype=ydt, device=x.device)
    if ws is None and method != "direct":
        nbytes = conv_workspace_size(x, k, mode, method)
        if nbytes > 0:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    o = L.TcConvOpts()
    o.method = L.METHODS[method]
    o.fft_threshold = int(fft_threshold)
    o.band_rows = int(band_rows)
    o.k_abs_sum = -1 if k_abs_sum is None else int(k_abs_sum)
    kh = None
    if k_host is not None:
        kh = np.ascontiguousarray(k_host, dtype=np.int32 if k.dtype == torch.int32 else np.float32)
        if kh.shape != tuple(k.shape):
            raise ValueError("k_host must have the shape of k")
        o.k_host = kh.ctypes.data
    o.workspace = ws.data_ptr() if ws is not None and ws.numel() > 0 else None
    o.workspace_bytes = ws.numel() if ws is not None else 0
    L.check("tc_conv_nd_ex", lib.tc_conv_nd_ex(C.byref(_desc(x)), C.byref(_desc(k)), L.MODES[mode],
                                               C.byref(_desc(out)), C.byref(o), _stream(stream)))
    return out


def conv_kernel_rank1(k, tol: float = 2.0 ** -20):
    """Host test of a 2-D kernel for separability: (True, u, v) with
    k ~= outer(u, v) as FP32 numpy vectors, or (False, None, None)."""
    kh = np.ascontiguousarray(k.detach().cpu().numpy() if isinstance(k, torch.Tensor) else k, dtype=np.float32)
    if kh.ndim != 2:
        raise ValueError("kernel must be 2-D")
    u = np.empty(kh.shape[0], np.float32)
    v = np.empty(kh.shape[1], np.float32)
    fp = C.POINTER(C.c_float)
    r = L.check("tc_conv_kernel_rank1",
                _lib().tc_conv_kernel_rank1(kh.ctypes.data_as(fp), kh.shape[0], kh.shape[1], float(tol),
                                            u.ctypes.data_as(fp), v.ctypes.data_as(fp)))
    return (True, u, v) if r == 1 else (False, None, None)


def conv_nd_separable(x: torch.Tensor, u: torch.Tensor, v: torch.Tensor, mode: str = "full",
                      out: Optional[torch.Tensor] = None, stream=None):
    """y = x (*) outer(u, v) for a 2-D FP32 image, both passes in one kernel."""
    K = int(u.numel())
    shape = conv_out_shape(tuple(x.shape), (K, K), mode, x.dtype, torch.float32)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=x.device)
    L.check("tc_conv_nd_separable",
            _lib().tc_conv_nd_separable(C.byref(_desc(x)), C.byref(_desc(u)), C.byref(_desc(v)), L.MODES[mode],
                                        C.byref(_desc(out)), _stream(stream)))
    return out


def conv_nd_auto(x: torch.Tensor, k: torch.Tensor, mode: str = "full", out: Optional[torch.Tensor] = None,
                 stream=None, tol: float = 2.0 ** -20):
    """conv_nd with separable-kernel detection: a 2-D FP32 kernel that is an
    outer product (within tol * max|k|) and of a supported size runs as the
    fused two-pass convolution, anything else as the direct one.  The kernel is
    read back to the host once per call for the test."""
    if (x.dim() == 2 and k.dim() == 2 and x.dtype == torch.float32 and k.dtype == torch.float32
            and k.shape[0] == k.shape[1] and int(k.shape[0]) in SEPARABLE_SIZES and x.stride(1) == 1
            and (out is None or out.stride(1) == 1)):
        ok, u, v = conv_kernel_rank1(k, tol)
        if ok:
            uu = torch.from_numpy(u).to(x.device)
            vv = torch.from_numpy(v).to(x.device)
            return conv_nd_separable(x, uu, vv, mode, out, stream)
    return conv_nd(x, k, mode, out, stream)


SEPARABLE_SIZES = (3, 5, 7, 9, 11, 15)

# Kernel side length from which the FFT branch beats the direct kernels on
# MI355X (FP32, full mode, cubic kernels; bench.py's crossover sweeps): 2048 x
# 2048 images, and 64 x 256 x 256 volumes.  The library's dispatcher
# (tc_conv_nd_ex) uses the same values.  The FFT branch's error is norm-wise,
# ||y - y64||_2 <= TAU ||x||_2 ||k||_1 with TAU = 3 u sum over the transform's
# radix-R stages of (8 log2 R + 2 (R - 1)) + 4 u (u = 2^-24; about 4.3e-5 for a
# 2048^2 image), not the element-wise (|x| (*) |k|) bound of the direct path.
FFT_THRESHOLD = 19
FFT_THRESHOLD_3D = 9
FFT_MAX_N = 4096


def conv_fft_workspace_size(x: torch.Tensor, k: torch.Tensor, mode: str = "full") -> int:
    n = C.c_size_t(0)
    L.check("tc_conv_fft_workspace_size",
            _lib().tc_conv_fft_workspace_size(C.byref(_desc(x)), C.byref(_desc(k)), L.MODES[mode], C.byref(n)))
    return n.value


def conv_fft(x: torch.Tensor, k: torch.Tensor, mode: str = "full", out: Optional[torch.Tensor] = None,
             ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """2-D or 3-D FP32 convolution through the FFT branch (same result and modes as conv_nd)."""
    if out is None:
        out = torch.empty(conv_out_shape(tuple(x.shape), tuple(k.shape), mode), dtype=torch.float32, device=x.device)
    nbytes = conv_fft_workspace_size(x, k, mode)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=x.device)
    L.check("tc_conv_fft", _lib().tc_conv_fft(C.byref(_desc(x)), C.byref(_desc(k)), L.MODES[mode],
                                              C.byref(_desc(out)), C.c_void_p(ws.data_ptr()), ws.numel(),
                                              _stream(stream)))
    return out


def conv2d_fft_workspace_size(x: torch.Tensor, k: torch.Tensor, mode: str = "full") -> int:
    n = C.c_size_t(0)
    L.check("tc_conv2d_fft_workspace_size",
            _lib().tc_conv2d_fft_workspace_size(C.byref(_desc(x)), C.byref(_desc(k)), L.MODES[mode], C.byref(n)))
    return n.value


def conv2d_fft(x: torch.Tensor, k: torch.Tensor, mode: str = "full", out: Optional[torch.Tensor] = None,
               ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """2-D FP32 convolution through the FFT branch (same result and modes as conv_nd)."""
    if out is None:
        out = torch.empty(conv_out_shape(tuple(x.shape), tuple(k.shape), mode), dtype=torch.float32, device=x.device)
    nbytes = conv2d_fft_workspace_size(x, k, mode)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=x.device)
    L.check("tc_conv2d_fft", _lib().tc_conv2d_fft(C.byref(_desc(x)), C.byref(_desc(k)), L.MODES[mode],
                                                  C.byref(_desc(out)), C.c_void_p(ws.data_ptr()), ws.numel(),
                                                  _stream(stream)))
    return out


def conv_hybrid(x: torch.Tensor, k: torch.Tensor, mode: str = "full", threshold: Optional[int] = None,
                out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """The paper's hybrid: direct convolution for kernels smaller than
    `threshold` on their longest side (default: the measured crossover of the
    rank), the FFT branch from there on (2-D and 3-D FP32, when the padded
    transform fits, else direct)."""
    if x.dim() in (2, 3) and x.dim() == k.dim() and x.dtype == torch.float32:
        thr = threshold if threshold is not None else (FFT_THRESHOLD if x.dim() == 2 else FFT_THRESHOLD_3D)
        fits = all(a + b - 1 <= FFT_MAX_N for a, b in zip(x.shape, k.shape))
        if max(k.shape) >= thr and fits:
            return conv_fft(x, k, mode, out=out, stream=stream)
    return conv_nd(x, k, mode, out=out, stream=stream)


def conv2d_hybrid(x: torch.Tensor, k: torch.Tensor, mode: str = "full", threshold: int = FFT_THRESHOLD,
                  out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """conv_hybrid for 2-D images."""
    return conv_hybrid(x, k, mode, threshold, out=out, stream=stream)


# ----------------------------------------------------------------------------- pyramid / derivatives
def image_pyramid(frame: torch.Tensor, levels: int, stream=None) -> List[torch.Tensor]:
    """[level 1, ..., level levels-1] as float32 tensors (level 0 is the frame itself)."""
    lib = _lib()
    H, W = frame.shape
    outs = [torch.empty((H >> l, W >> l), dtype=torch.float32, device=frame.device) for l in range(1, levels)]
    arr = (L.TcTensor * max(1, len(outs)))(*[_desc(o) for o in outs]) if outs else None
    L.check("tc_image_pyramid", lib.tc_image_pyramid(C.byref(_desc(frame)), levels, arr, _stream(stream)))
    return outs


def horn_derivs(prev: torch.Tensor, nxt: torch.Tensor, exact_int: bool = False, stream=None):
    """(E_x, E_y, E_t) of the first-difference cube; exact_int returns the int32 numerators 4E (u8 only)."""
    lib = _lib()
    H, W = prev.shape
    dt = torch.int32 if exact_int else torch.float32
    outs = [torch.empty((H - 1, W - 1), dtype=dt, device=prev.device) for _ in range(3)]
    L.check("tc_horn_derivs", lib.tc_horn_derivs(C.byref(_desc(prev)), C.byref(_desc(nxt)), C.byref(_desc(outs[0])),
                                                 C.byref(_desc(outs[1])), C.byref(_desc(outs[2])), _stream(stream)))
    return tuple(outs)


STENCILS = {"fd2": L.TC_STENCIL_FD2, "roberts": L.TC_STENCIL_ROBERTS, "prewitt3": L.TC_STENCIL_PREWITT3,
            "sobel3": L.TC_STENCIL_SOBEL3}


def gradient(image: torch.Tensor, stencil: str = "fd2", want=("ex", "ey", "mag", "dir"), out=None, stream=None):
    """Gradient (E_x, E_y), magnitude and direction of a 2-D image under one of
    the masks of ``STENCILS``: a dict of the FP32 outputs asked for in ``want``
    (or the tensors given in ``out``, a dict by the same names), each
    (H-k+1) x (W-k+1) for a k x k mask."""
    lib = _lib()
    st = STENCILS[stencil]
    k = 3 if st >= L.TC_STENCIL_PREWITT3 else 2
    H, W = image.shape
    shape = (max(H - k + 1, 0), max(W - k + 1, 0))
    outs = dict(out) if out is not None else \
        {n: torch.empty(shape, dtype=torch.float32, device=image.device) for n in want}
    ds = [C.byref(_desc(outs[n])) if n in outs else None for n in ("ex", "ey", "mag", "dir")]
    L.check("tc_gradient", lib.tc_gradient(C.byref(_desc(image)), st, *ds, _stream(stream)))
    return outs


# ----------------------------------------------------------------------------- time to contact
SELECT_RULES = {"decreasing_ttc": L.TC_SELECT_DECREASING_TTC, "min_residual": L.TC_SELECT_MIN_RESIDUAL}


def ttc_reselect(levels_buf: torch.Tensor, n_pairs: int, levels: int, rule: str = "min_residual",
                 out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """The multi-scale choice re-applied to device level records (n_pairs x
    levels records, pair-major) by ``rule``: a device buffer of n_pairs picks."""
    if levels_buf.numel() < n_pairs * levels * L.LEVEL_DTYPE.itemsize:
        raise ValueError("level buffer smaller than n_pairs x levels records")
    if out is None:
        out = torch.empty(max(n_pairs, 1) * L.PICK_DTYPE.itemsize, dtype=torch.uint8, device=levels_buf.device)
    elif out.numel() < n_pairs * L.PICK_DTYPE.itemsize:
        raise ValueError("pick buffer smaller than n_pairs picks")
    L.check("tc_ttc_reselect", _lib().tc_ttc_reselect(C.c_void_p(levels_buf.data_ptr()), n_pairs, levels,
                                                       SELECT_RULES[rule], C.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def decode_levels(buf: torch.Tensor) -> np.ndarray:
    """tc_ttc_level records (device bytes) -> numpy structured array."""
    return buf.cpu().numpy().view(L.LEVEL_DTYPE)


def decode_picks(buf: torch.Tensor) -> np.ndarray:
    return buf.cpu().numpy().view(L.PICK_DTYPE)


def ttc_workspace_size(H: int, W: int, levels: int) -> int:
    n = C.c_size_t(0)
    L.check("tc_ttc_workspace_size", _lib().tc_ttc_workspace_size(H, W, levels, C.byref(n)))
    return n.value


def ttc_solve(prev: torch.Tensor, nxt: torch.Tensor, levels: int = 1, ws: Optional[torch.Tensor] = None,
              out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None, stream=None):
    """One frame pair -> (levels buffer [levels*152 B], pick buffer [56 B]) on the device."""
    lib = _lib()
    H, W = prev.shape
    nbytes = ttc_workspace_size(H, W, levels)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=prev.device)
    if out is None:
        out = (torch.empty(levels * L.LEVEL_DTYPE.itemsize, dtype=torch.uint8, device=prev.device),
               torch.empty(L.PICK_DTYPE.itemsize, dtype=torch.uint8, device=prev.device))
    L.check("tc_ttc_solve", lib.tc_ttc_solve(C.byref(_desc(prev)), C.byref(_desc(nxt)), levels, C.c_void_p(ws.data_ptr()),
                                             ws.numel(), C.c_void_p(out[0].data_ptr()), C.c_void_p(out[1].data_ptr()),
                                             _stream(stream)))
    return out


VARIANT_STENCILS = {"cube": L.TC_STENCIL_FD2, "prewitt3": L.TC_STENCIL_PREWITT3, "sobel3": L.TC_STENCIL_SOBEL3}
LOWPASS = {"none": L.TC_LOWPASS_NONE, "binomial3": L.TC_LOWPASS_BINOMIAL3}


def ttc_variant_workspace_size(H: int, W: int, levels: int, stencil: str = "cube", lowpass: str = "none") -> int:
    n = C.c_size_t(0)
    L.check("tc_ttc_variant_workspace_size",
            _lib().tc_ttc_variant_workspace_size(H, W, levels, VARIANT_STENCILS[stencil], LOWPASS[lowpass],
                                                 C.byref(n)))
    return n.value


def ttc_solve_variant(prev: torch.Tensor, nxt: torch.Tensor, levels: int = 1, stencil: str = "cube",
                      lowpass: str = "none", ws: Optional[torch.Tensor] = None,
                      out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None, stream=None):
    """One frame pair with the given derivative stencil and pyramid low-pass ->
    (levels buffer [levels*152 B], pick buffer [56 B]) on the device."""
    H, W = prev.shape
    nbytes = ttc_variant_workspace_size(H, W, levels, stencil, lowpass)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=prev.device)
    if out is None:
        out = (torch.empty(levels * L.LEVEL_DTYPE.itemsize, dtype=torch.uint8, device=prev.device),
               torch.empty(L.PICK_DTYPE.itemsize, dtype=torch.uint8, device=prev.device))
    L.check("tc_ttc_solve_variant",
            _lib().tc_ttc_solve_variant(C.byref(_desc(prev)), C.byref(_desc(nxt)), levels, VARIANT_STENCILS[stencil],
                                        LOWPASS[lowpass], C.c_void_p(ws.data_ptr()), ws.numel(),
                                        C.c_void_p(out[0].data_ptr()), C.c_void_p(out[1].data_ptr()),
                                        _stream(stream)))
    return out


def seq_from_frames(frames: torch.Tensor, levels: int) -> L.TcSeq:
    """A [F, H, W] u8/f16 video tensor (row-contiguous) as a tc_seq descriptor."""
    if frames.dim() != 3 or frames.stride(2) != 1:
        raise ValueError("frames must be [F, H, W] with contiguous rows")
    q = L.TcSeq()
    q.frame0 = frames.data_ptr()
    q.frame_stride = frames.stride(0)
    q.row_stride = frames.stride(1)
    q.H, q.W = int(frames.shape[1]), int(frames.shape[2])
    q.n_frames = int(frames.shape[0])
    q.levels = levels
    return q


def seq_from_pair(prev: torch.Tensor, nxt: torch.Tensor, levels: int) -> L.TcSeq:
    """Two unrelated frames as a 2-frame stream (frame_stride = next - prev)."""
    es = prev.element_size()
    diff = nxt.data_ptr() - prev.data_ptr()
    if diff % es:
        raise ValueError("frames are not element-aligned relative to each other")
    q = L.TcSeq()
    q.frame0 = prev.data_ptr()
    q.frame_stride = diff // es
    q.row_stride = prev.stride(0)
    q.H, q.W = int(prev.shape[0]), int(prev.shape[1])
    q.n_frames = 2
    q.levels = levels
    return q


class TTCPlan:
    """A batch of streams planned once and run many times (graph-capturable run)."""

    def __init__(self, seqs: Sequence[L.TcSeq], dtype: torch.dtype, device=None, keep: Sequence = (),
                 tuning: Optional[Tuple[int, int]] = None):
        self._lib = _lib()
        self._keep = list(keep)  # tensors the descriptors point into
        arr = (L.TcSeq * len(seqs))(*seqs)
        h = C.c_void_p()
        tn = None
        if tuning is not None:
            tn = L.TcTuning()
            tn.band_rows, tn.groups_per_cu = int(tuning[0]), int(tuning[1])
        L.check("tc_ttc_plan_create_ex",
                self._lib.tc_ttc_plan_create_ex(arr, len(seqs), _DT[dtype], C.byref(tn) if tn is not None else None,
                                                C.byref(h)))
        self._h = h
        self._dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.ws = self.levels_buf = self.picks_buf = None
        self._size_buffers()

    def _size_buffers(self):
        ws = C.c_size_t(0)
        npairs = C.c_int64(0)
        nrec = C.c_int64(0)
        L.check("tc_ttc_plan_info", self._lib.tc_ttc_plan_info(self._h, C.byref(ws), C.byref(npairs), C.byref(nrec)))
        self.ws_bytes = ws.value
        self.n_pairs = npairs.value
        self.n_records = nrec.value
        need = (max(1, self.ws_bytes), max(1, self.n_records) * L.LEVEL_DTYPE.itemsize,
                max(1, self.n_pairs) * L.PICK_DTYPE.itemsize)
        if self.ws is None or self.ws.numel() < need[0]:
            self.ws = torch.empty(need[0], dtype=torch.uint8, device=self._dev)
        if self.levels_buf is None or self.levels_buf.numel() < need[1]:
            self.levels_buf = torch.empty(need[1], dtype=torch.uint8, device=self._dev)
        if self.picks_buf is None or self.picks_buf.numel() < need[2]:
            self.picks_buf = torch.empty(need[2], dtype=torch.uint8, device=self._dev)
        self.uploaded = False

    def reset(self, seqs: Sequence[L.TcSeq], keep: Sequence = ()):
        """Re-plan for a new batch with the same dtype and levels.  The previous
        upload must have completed; buffers grow when the new batch needs more."""
        arr = (L.TcSeq * len(seqs))(*seqs)
        L.check("tc_ttc_plan_reset", self._lib.tc_ttc_plan_reset(self._h, arr, len(seqs)))
        self._keep = list(keep)
        self._size_buffers()

    def upload(self, stream=None):
        L.check("tc_ttc_plan_upload", self._lib.tc_ttc_plan_upload(self._h, C.c_void_p(self.ws.data_ptr()),
                                                                   self.ws.numel(), _stream(stream)))
        self.uploaded = True

    def run(self, stream=None):
        if not self.uploaded:
            self.upload(stream)
        L.check("tc_ttc_plan_run", self._lib.tc_ttc_plan_run(self._h, C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                                             C.c_void_p(self.levels_buf.data_ptr()),
                                                             C.c_void_p(self.picks_buf.data_ptr()), _stream(stream)))

    def run_phase(self, phase: int, stream=None):
        """Phase 1: fused pass only; phase 2: finishing pass only; 3: both."""
        if not self.uploaded:
            self.upload(stream)
        L.check("tc_ttc_plan_run_phase",
                self._lib.tc_ttc_plan_run_phase(self._h, C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                                C.c_void_p(self.levels_buf.data_ptr()),
                                                C.c_void_p(self.picks_buf.data_ptr()), phase, _stream(stream)))

    def results(self):
        return decode_levels(self.levels_buf[: self.n_records * L.LEVEL_DTYPE.itemsize]), \
            decode_picks(self.picks_buf[: self.n_pairs * L.PICK_DTYPE.itemsize])

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.tc_ttc_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tuning_default(dtype: torch.dtype, levels: int) -> Tuple[int, int]:
    """The library's built-in (band_rows, groups_per_cu) for a dtype and level count."""
    t = L.TcTuning()
    L.check("tc_ttc_tuning_default", _lib().tc_ttc_tuning_default(_DT[dtype], levels, C.byref(t)))
    return t.band_rows, t.groups_per_cu


def ttc_solve_batched(videos: Sequence[torch.Tensor], levels: int, stream=None, tuning=None):
    """Every consecutive pair of every [F, H, W] video -> (levels records, picks) as numpy arrays."""
    dtype = videos[0].dtype
    plan = TTCPlan([seq_from_frames(v, levels) for v in videos], dtype, videos[0].device, keep=videos, tuning=tuning)
    plan.run(stream)
    torch.cuda.synchronize()
    out = plan.results()
    plan.close()
    return out
