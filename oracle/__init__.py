"""CPU oracle for the convolution / derivative / time-to-contact hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything under ``oracle/``; only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.

Every function here is a plain, slow, FP64 (or exact-integer) restatement of
what the paper defines, written so that it can be checked against the paper by
eye: no blocking, no fusion, no reordering beyond the definition.  It shares no
code with the HIP path; the two meet only through the seeded inputs produced by
``paper_1612_08825_amd.synth``.

Modules:
  conv     -- n-D direct convolution and its output modes (Discrete Derivatives
              section, spatial convolution equation; Accelerating Convolutions)
  pyramid  -- 2x2 block-average down-sampling (Time to Contact, Results)
  horn     -- 2x2x2 first-difference derivative cube (Discrete Derivatives,
              the 2x2 derivative kernel, extended over two frames)
  ttc      -- radial gradient, least-squares normal equations, 3x3 solve,
              FOE / TTC, multi-scale level selection (Time to Contact)
  gradient -- image gradient with the 2x2 / 3x3 masks, its magnitude and
              direction (Discrete Derivatives; Convolutions)
  variant  -- time to contact with the centred 3x3 Prewitt / Sobel stencils
              and the pyramid low-pass filter (Convolutions; Time to Contact,
              Results)
"""
from .conv import conv, conv_full, conv_at, conv_bruteforce, conv_out_shape  # noqa: F401
from .pyramid import pyramid, reduce2  # noqa: F401
from .horn import horn, horn_numerators  # noqa: F401
from .ttc import (  # noqa: F401
    SUM_NAMES,
    STATUS_OK,
    STATUS_SINGULAR,
    STATUS_NEED_PREV,
    STATUS_NONFINITE,
    cube_coords,
    level_terms,
    level_sums,
    level_sums_exact,
    solve3,
    solve_level,
    ttc_pair,
    select_level,
    select_level_residual,
    ttc_sequence,
)
from .gradient import STENCILS, apply_mask, gradient, masks  # noqa: F401
from . import variant  # noqa: F401,E402
