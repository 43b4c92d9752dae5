"""Seeded synthetic inputs shared by the GPU path, the oracle and the benchmark.

This module only *generates data*: textured approaching-plane videos, random
images and kernels for the convolution sweep, and the analytic ground truth of
the videos' motion.  It holds none of the method's arithmetic (no convolution,
no pyramid, no derivative, no least-squares sum); both sides of every parity
check consume the arrays produced here.

Video model (Time to Contact section, perspective projection and the FOE/TTC
definitions): a frontal textured plane translating with constant direction is
imaged as frame 0 magnified about the fixed focus of expansion f by
m(t) = Z0 / Z(t).  A scene point therefore moves as p(t) = f + m(t) (p0 - f),
so the image flow is u = (m'/m)(x - f_x), v = (m'/m)(y - f_y): C = m'/m,
A = -C f_x, B = -C f_y and TTC = 1/C.  For a frame pair (t, t+1) the ground
truth is TTC = 1 / ln(m(t+1)/m(t)) frames, FOE = f.

The paper builds its videos by repeatedly zooming into random points with cubic
interpolation; it does not give the interpolation kernel, so the videos here are
rendered analytically (no interpolation) at every pixel centre instead.

Coordinates: x grows to the right (column j), y grows downward (row i); the
origin is the base-image centre ((W-1)/2, (H-1)/2); units are base pixels.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

SEED_ROOT = 1612

#: The frame sizes (W, H) the batched and serving workloads draw from.
STREAM_SIZES: Tuple[Tuple[int, int], ...] = ((320, 240), (640, 480), (1280, 720), (1920, 1080))


def rng_for(config: int, case: int = 0) -> np.random.Generator:
    """Seeded generator for workload ``config`` (1..5) and sub-case ``case``."""
    return np.random.default_rng([SEED_ROOT, int(config), int(case)])


# --------------------------------------------------------------------------
# Texture and renderer
# --------------------------------------------------------------------------
@dataclass
class Texture:
    """Sum of sinusoids T(X,Y) = 128 + (112/n) sum_i s(2 pi (X cos th_i + Y sin th_i)/P_i + ph_i).

    ``s`` is sin, or cos when ``symmetric`` (then every phase is 0 and the
    texture is point-symmetric about the origin).  Values lie in [16, 240].
    """

    theta: np.ndarray
    period: np.ndarray
    phase: np.ndarray
    symmetric: bool = False

    @staticmethod
    def random(rng: np.random.Generator, n: int = 6, pmin: float = 8.0, pmax: float = 64.0,
               symmetric: bool = False) -> "Texture":
        theta = rng.uniform(0.0, math.pi, n)
        period = np.exp(rng.uniform(math.log(pmin), math.log(pmax), n))
        phase = np.zeros(n) if symmetric else rng.uniform(0.0, 2.0 * math.pi, n)
        return Texture(theta, period, phase, symmetric)

    def eval_numpy(self, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
        acc = np.zeros(np.broadcast(X, Y).shape, dtype=np.float64)
        for th, p, ph in zip(self.theta, self.period, self.phase):
            z = (2.0 * math.pi / p) * (X * math.cos(th) + Y * math.sin(th))
            if self.symmetric:
                acc += np.cos(np.abs(z))  # evaluated on |z| so that mirrored pixels match bit for bit
            else:
                acc += np.sin(z + ph)
        return 128.0 + (112.0 / len(self.theta)) * acc

    def eval_torch(self, X, Y):
        import torch

        acc = torch.zeros(torch.broadcast_shapes(X.shape, Y.shape), dtype=torch.float64, device=X.device)
        for th, p, ph in zip(self.theta, self.period, self.phase):
            z = (2.0 * math.pi / float(p)) * (X * math.cos(float(th)) + Y * math.sin(float(th)))
            if self.symmetric:
                acc += torch.cos(torch.abs(z))
            else:
                acc += torch.sin(z + float(ph))
        return 128.0 + (112.0 / len(self.theta)) * acc


def quantize_numpy(v: np.ndarray, dtype: str) -> np.ndarray:
    """u8: clip(rint(v), 0, 255) (round half to even); f16: IEEE round to nearest even; f32 likewise."""
    if dtype == "u8":
        return np.clip(np.rint(v), 0, 255).astype(np.uint8)
    if dtype == "f16":
        return v.astype(np.float16)
    if dtype == "f32":
        return v.astype(np.float32)
    raise ValueError(f"unknown dtype {dtype!r}")


def _quantize_torch(v, dtype: str):
    import torch

    if dtype == "u8":
        return torch.clamp(torch.round(v), 0, 255).to(torch.uint8)
    if dtype == "f16":
        return v.to(torch.float16)
    if dtype == "f32":
        return v.to(torch.float32)
    raise ValueError(f"unknown dtype {dtype!r}")


def centered_coords(H: int, W: int):
    """Pixel-centre coordinates (x, y) of an H x W image, origin at the image centre."""
    x = np.arange(W, dtype=np.float64) - (W - 1) / 2.0
    y = np.arange(H, dtype=np.float64) - (H - 1) / 2.0
    return x, y


def render_frame(tex: Texture, H: int, W: int, foe: Tuple[float, float], m: float, dtype: str = "u8",
                 device=None):
    """Frame I(p) = T(f + (p - f)/m) rendered at every pixel centre, then quantised.

    Returns a numpy array when ``device`` is None, else a torch tensor on ``device``
    (rendered there in float64; only used to build large benchmark inputs quickly).
    """
    fx, fy = float(foe[0]), float(foe[1])
    if device is None:
        x, y = centered_coords(H, W)
        X = fx + (x[None, :] - fx) / m
        Y = fy + (y[:, None] - fy) / m
        return quantize_numpy(tex.eval_numpy(X, Y), dtype)
    import torch

    x = torch.arange(W, dtype=torch.float64, device=device) - (W - 1) / 2.0
    y = torch.arange(H, dtype=torch.float64, device=device) - (H - 1) / 2.0
    X = fx + (x[None, :] - fx) / m
    Y = fy + (y[:, None] - fy) / m
    return _quantize_torch(tex.eval_torch(X, Y), dtype)


# --------------------------------------------------------------------------
# Motion laws and ground truth
# --------------------------------------------------------------------------
@dataclass
class Motion:
    """Magnification law m(t) and its per-pair ground truth."""

    m: Callable[[float], float]
    log_ratio: Callable[[int], float]  # ln(m(t+1)/m(t)) evaluated without cancellation

    def ttc_gt(self, t: int) -> float:
        return 1.0 / self.log_ratio(t)


def constant_ttc(ttc: float) -> Motion:
    """m(t) = exp(t/ttc): every pair has TTC = ttc frames."""
    return Motion(m=lambda t: math.exp(t / ttc), log_ratio=lambda t: 1.0 / ttc)


def linear_ttc(a: float, b: float) -> Motion:
    """TTC(t) = a - b t  =>  m(t) = (a / (a - b t))^(1/b)."""
    return Motion(
        m=lambda t: (a / (a - b * t)) ** (1.0 / b),
        log_ratio=lambda t: math.log((a - b * t) / (a - b * (t + 1))) / b,
    )


@dataclass
class Video:
    frames: object  # numpy [F, H, W] or torch tensor
    foe: Tuple[float, float]
    motion: Motion
    texture: Texture
    dtype: str

    @property
    def n_frames(self) -> int:
        return int(self.frames.shape[0])

    def ttc_gt(self) -> np.ndarray:
        return np.array([self.motion.ttc_gt(t) for t in range(self.n_frames - 1)])

    def abc_gt(self) -> np.ndarray:
        """Ground-truth (A, B, C) per pair in base-pixel units."""
        out = []
        for t in range(self.n_frames - 1):
            C = self.motion.log_ratio(t)
            out.append((-C * self.foe[0], -C * self.foe[1], C))
        return np.array(out)


def render_video(tex: Texture, H: int, W: int, F: int, foe, motion: Motion, dtype: str = "u8",
                 device=None) -> Video:
    if device is None:
        frames = np.stack([render_frame(tex, H, W, foe, motion.m(t), dtype) for t in range(F)])
    else:
        import torch

        frames = torch.stack([render_frame(tex, H, W, foe, motion.m(t), dtype, device) for t in range(F)])
    return Video(frames, (float(foe[0]), float(foe[1])), motion, tex, dtype)


# --------------------------------------------------------------------------
# The workloads
# --------------------------------------------------------------------------
def plain_ttc_video(case: int = 0, H: int = 128, W: int = 128, F: int = 8, ttc: float = 40.0,
                    dtype: str = "u8", symmetric: bool = False) -> Video:
    """Single stream approaching head-on (FOE at the centre) with constant TTC."""
    rng = rng_for(1, case)
    tex = Texture.random(rng, symmetric=symmetric)
    return render_video(tex, H, W, F, (0.0, 0.0), constant_ttc(ttc), dtype)


def multiscale_video(case: int = 0, H: int = 480, W: int = 640, F: int = 300, dtype: str = "u8",
                     foe=(60.0, -40.0), ttc_start: float = 300.0, ttc_end: float = 30.0,
                     device=None) -> Video:
    """Plane approaching with FOE offset and TTC falling linearly from ttc_start to ttc_end."""
    rng = rng_for(3, case)
    tex = Texture.random(rng)
    b = (ttc_start - ttc_end) / (F - 1)
    return render_video(tex, H, W, F, foe, linear_ttc(ttc_start, b), dtype, device)


@dataclass
class StreamSpec:
    H: int
    W: int
    foe: Tuple[float, float]
    ttc: float
    texture: Texture
    n_frames: int
    dtype: str
    frames: object = None

    @property
    def motion(self) -> Motion:
        return constant_ttc(self.ttc)

    def render(self, device=None):
        v = render_video(self.texture, self.H, self.W, self.n_frames, self.foe, self.motion, self.dtype, device)
        self.frames = v.frames
        return self.frames


def stream_specs(config: int, n_streams: int, n_frames: int, dtype: str,
                 sizes: Sequence[Tuple[int, int]] = STREAM_SIZES, case: int = 0) -> List[StreamSpec]:
    """Streams of uneven sizes: size uniform over ``sizes``, FOE uniform in
    [-W/8, W/8] x [-H/8, H/8], constant TTC uniform in [30, 300] frames."""
    rng = rng_for(config, case)
    specs = []
    for _ in range(n_streams):
        W, H = sizes[int(rng.integers(len(sizes)))]
        foe = (float(rng.uniform(-W / 8, W / 8)), float(rng.uniform(-H / 8, H / 8)))
        ttc = float(rng.uniform(30.0, 300.0))
        tex = Texture.random(rng)
        specs.append(StreamSpec(H, W, foe, ttc, tex, n_frames, dtype))
    return specs


def batched_specs(case: int = 0, n_streams: int = 64, n_frames: int = 16, dtype: str = "f16",
                  sizes: Sequence[Tuple[int, int]] = STREAM_SIZES) -> List[StreamSpec]:
    """The batched workload: 64 streams of uneven sizes, 16 FP16 frames each."""
    return stream_specs(4, n_streams, n_frames, dtype, sizes, case)


def serving_specs(case: int = 0, n_streams: int = 256, n_frames: int = 16, dtype: str = "u8",
                  sizes: Sequence[Tuple[int, int]] = STREAM_SIZES) -> List[StreamSpec]:
    """The serving workload: 256 camera streams of mixed sizes, u8 frames."""
    return stream_specs(5, n_streams, n_frames, dtype, sizes, case)


def poisson_arrivals(rate_hz: float, duration_s: float, n_streams: int, case: int = 0):
    """Open-loop Poisson arrivals: (times [s], stream ids) with aggregate rate ``rate_hz``."""
    rng = rng_for(5, 1000 + case)
    n = int(rng.poisson(rate_hz * duration_s))
    gaps = rng.exponential(1.0 / rate_hz, n)
    times = np.cumsum(gaps)
    times = times[times < duration_s]
    ids = rng.integers(0, n_streams, times.shape[0])
    return times, ids


# --------------------------------------------------------------------------
# Convolution sweep inputs
# --------------------------------------------------------------------------
def conv_image(shape, case: int = 0, dtype: str = "f32") -> np.ndarray:
    """f32: U[0,1) drawn in FP64 then cast; u8: U{0..255}; f16: U[0,1) cast to f16."""
    rng = rng_for(2, case)
    if dtype == "u8":
        return rng.integers(0, 256, size=shape, dtype=np.int64).astype(np.uint8)
    v = rng.random(shape)
    return v.astype(np.float16 if dtype == "f16" else np.float32)


def conv_kernel(shape, case: int = 0, dtype: str = "f32", int_range: int = 8) -> np.ndarray:
    """f32: N(0,1) drawn in FP64 then cast; i32: U{-int_range..int_range}."""
    rng = rng_for(2, 10_000 + case)
    if dtype == "i32":
        return rng.integers(-int_range, int_range + 1, size=shape, dtype=np.int64).astype(np.int32)
    return rng.standard_normal(shape).astype(np.float32)
