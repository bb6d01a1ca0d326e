"""Seeded generators for the workloads the library is measured and checked on.

Two families:

* ``make_exact_rank`` / ``make_tiny``: an order-N tensor with a known multilinear
  rank (a random core times random orthonormal factors) plus optional Gaussian
  noise.  Used to pin the oracle against closed forms.
* ``make_stereo_stack``: a stand-in for the paper's multi-exposure stereo LDR
  stacks (Sec. IV uses 2208x1242 ZED stereo pairs at several exposures; that
  dataset is not available).  A log-normal-like radiance field with a 1e4:1
  dynamic range is rendered into two views with a smooth horizontal disparity,
  exposed at several EV steps through a 1/2.2 gamma, quantised to 8 bits, and
  converted to one of the two colour spaces of Sec. III-A (Y'CbCr or IPT).
  The stack is stored (H, W, 3, 2E) with image index i = view*E + exposure,
  which is the order-4 tensor that Sec. III-B decomposes.

All randomness comes from numpy's PCG64 (``np.random.default_rng(seed)``) with a
fixed draw order, so a seed names a tensor exactly.
"""

from __future__ import annotations

import math

import numpy as np

# Named stack workloads: (H, W, exposures, colour space, ranks, sweeps, seed).
STACK_CONFIGS = {
    # 1080p stereo stack, 7 exposures (EV -3..+3), Y'CbCr.
    "stack1080": dict(H=1080, W=1920, E=7, colorspace="ycbcr", ranks=(256, 384, 3, 8), sweeps=20, seed=1),
    # 4K stereo stack, 5 exposures (EV -2..+2), IPT.
    "stack2160": dict(H=2160, W=3840, E=5, colorspace="ipt", ranks=(512, 768, 3, 6), sweeps=15, seed=2),
    # Reduced stacks from the same generator: small enough for the FP64 oracle
    # to finish in seconds, large enough to span several GPU tiles.
    "stack_mini": dict(H=180, W=320, E=7, colorspace="ycbcr", ranks=(48, 64, 3, 8), sweeps=10, seed=11),
    "stack_mini_ipt": dict(H=144, W=256, E=5, colorspace="ipt", ranks=(40, 56, 3, 6), sweeps=10, seed=12),
}


# --------------------------------------------------------------------------
# Exact multilinear-rank tensors
# --------------------------------------------------------------------------

def haar_orthonormal(rng: np.random.Generator, s: int, r: int) -> np.ndarray:
    """An s x r matrix with orthonormal columns, Haar-distributed.

    QR of a standard Gaussian matrix with the sign of R's diagonal folded into Q
    (Mezzadri's correction), so the distribution is exactly Haar.
    """
    a = rng.standard_normal((s, r))
    q, rr = np.linalg.qr(a)
    d = np.sign(np.diag(rr))
    d[d == 0] = 1.0
    return q * d[None, :]


def _expand(core: np.ndarray, factors) -> np.ndarray:
    """core x_1 F1 x_2 F2 ... (each F_n is s_n x r_n); used only to build inputs."""
    out = core
    for n, f in enumerate(factors):
        # contract axis n of `out` with axis 1 of f, then move the new axis back to n
        out = np.moveaxis(np.tensordot(f, out, axes=([1], [n])), 0, n)
    return out


def make_exact_rank(dims, ranks, seed: int, noise_rel: float = 0.0):
    """X = G x_1 U1 ... x_N UN + noise.

    G ~ N(0,1) of shape ``ranks``; U_n Haar s_n x R_n; noise ~ N(0, (noise_rel*RMS(X0))^2)
    where RMS(X0) is the root-mean-square of the noiseless tensor.
    Returns (X, G, [U_n]) in float64.
    """
    dims = tuple(int(d) for d in dims)
    ranks = tuple(int(r) for r in ranks)
    if len(dims) != len(ranks):
        raise ValueError("dims and ranks differ in length")
    rng = np.random.default_rng(seed)
    core = rng.standard_normal(ranks)
    factors = [haar_orthonormal(rng, s, r) for s, r in zip(dims, ranks)]
    x0 = _expand(core, factors)
    if noise_rel > 0.0:
        rms = math.sqrt(float(np.mean(x0 * x0)))
        x = x0 + rng.standard_normal(dims) * (noise_rel * rms)
    else:
        x = x0
    return x, core, factors


def make_tiny(seed: int = 0, noise_rel: float = 1e-3):
    """The tiny order-4 case: 64x48x3x6 built from a 16x12x3x4 core, ranks (16,12,3,4)."""
    return make_exact_rank((64, 48, 3, 6), (16, 12, 3, 4), seed, noise_rel)


# --------------------------------------------------------------------------
# Multi-exposure stereo stacks
# --------------------------------------------------------------------------

# ITU-R BT.601 luma weights and the full-range colour-difference scalings.
_BT601_KR, _BT601_KG, _BT601_KB = 0.299, 0.587, 0.114
# ITU-R BT.709 / sRGB primaries, D65 white: linear RGB -> CIE XYZ.
_RGB709_TO_XYZ = np.array([[0.4124, 0.3576, 0.1805],
                           [0.2126, 0.7152, 0.0722],
                           [0.0193, 0.1192, 0.9505]])
# Ebner & Fairchild (1998), "Development and testing of a color space (IPT) with
# improved hue uniformity": XYZ (D65) -> LMS, the 0.43 power, and LMS' -> IPT.
_XYZ_TO_LMS = np.array([[0.4002, 0.7075, -0.0807],
                        [-0.2280, 1.1500, 0.0612],
                        [0.0000, 0.0000, 0.9184]])
_IPT_EXPONENT = 0.43
_LMS_TO_IPT = np.array([[0.4000, 0.4000, 0.2000],
                        [4.4550, -4.8510, 0.3960],
                        [0.8056, 0.3572, -1.1628]])


def _gaussian_blobs(rng, n, H, W, scale_lo, scale_hi, channels):
    """Sum of n random anisotropic Gaussians on the unit square, one image per channel.

    Returns an array (channels, H, W).  Draw order per blob: centre (2), log-scales (2),
    angle (1), amplitude (1), tint (channels).
    """
    v = (np.arange(H, dtype=np.float64) + 0.5) / H
    u = (np.arange(W, dtype=np.float64) + 0.5) / W
    out = np.zeros((channels, H, W))
    for _ in range(n):
        cu, cv = rng.uniform(0.0, 1.0, size=2)
        su, sv = np.exp(rng.uniform(math.log(scale_lo), math.log(scale_hi), size=2))
        th = rng.uniform(0.0, math.pi)
        amp = rng.standard_normal()
        tint = rng.uniform(0.7, 1.3, size=channels) if channels > 1 else np.ones(1)
        ct, st = math.cos(th), math.sin(th)
        du = u[None, :] - cu
        dv = v[:, None] - cv
        a = (ct * du + st * dv) / su
        b = (-st * du + ct * dv) / sv
        g = np.exp(-0.5 * (a * a + b * b))
        out += (amp * tint)[:, None, None] * g[None, :, :]
    return out


def _gradient(rng, H, W):
    gu, gv = rng.normal(0.0, 0.5, size=2)
    v = (np.arange(H, dtype=np.float64) + 0.5) / H
    u = (np.arange(W, dtype=np.float64) + 0.5) / W
    return gu * u[None, :] + gv * v[:, None]


def _minmax(a):
    lo, hi = float(a.min()), float(a.max())
    return (a - lo) / (hi - lo) if hi > lo else np.zeros_like(a)


def _shift_rows(img, disp):
    """img (C,H,W); returns img sampled at x + disp(y, x), linear interpolation, edge clamp."""
    C, H, W = img.shape
    xs = np.arange(W, dtype=np.float64)[None, :] + disp
    x0 = np.floor(xs)
    fr = xs - x0
    x0 = x0.astype(np.int64)
    i0 = np.clip(x0, 0, W - 1)
    i1 = np.clip(x0 + 1, 0, W - 1)
    rows = np.arange(H)[:, None]
    return img[:, rows, i0] * (1.0 - fr)[None] + img[:, rows, i1] * fr[None]


def _to_ycbcr(rgbp):
    """Gamma-encoded R'G'B' (3,H,W) -> Y'CbCr, BT.601 weights, full range, Cb/Cr centred on 0."""
    r, g, b = rgbp
    y = _BT601_KR * r + _BT601_KG * g + _BT601_KB * b
    cb = (b - y) / (2.0 * (1.0 - _BT601_KB))
    cr = (r - y) / (2.0 * (1.0 - _BT601_KR))
    return np.stack([y, cb, cr])


def _to_ipt(rgbp):
    """Gamma-encoded R'G'B' (3,H,W) -> IPT (Ebner & Fairchild), via linear BT.709 RGB and XYZ."""
    lin = np.power(rgbp, 2.2)
    xyz = np.tensordot(_RGB709_TO_XYZ, lin, axes=([1], [0]))
    lms = np.tensordot(_XYZ_TO_LMS, xyz, axes=([1], [0]))
    lmsp = np.sign(lms) * np.power(np.abs(lms), _IPT_EXPONENT)
    return np.tensordot(_LMS_TO_IPT, lmsp, axes=([1], [0]))


def make_stereo_stack(H: int, W: int, E: int, colorspace: str = "ycbcr", seed: int = 1,
                      dtype=np.float32) -> np.ndarray:
    """A multi-exposure stereo stack of shape (H, W, 3, 2E), image index i = view*E + exposure.

    1. log-radiance L: 64 anisotropic Gaussian blobs (centres U[0,1)^2, axis scales
       log-uniform in [0.02, 0.25], angle U[0,pi), amplitude N(0,1), per-channel tint
       U(0.7,1.3)) plus a linear gradient N(0, 0.5^2) per axis; min-max normalised over
       all channels; radiance = 10^(4 L), a 1e4:1 range.
    2. depth: min-max normalised sum of 8 broad blobs plus a gradient; disparity 32*depth px;
       right view E_R(y,x) = E_L(y, x + d) (linear interpolation, edge clamp).
    3. exposures EV = -(E-1)/2 ... +(E-1)/2; k = 0.18 / geomean(E_L);
       I = clip((k 2^EV E)^(1/2.2), 0, 1), quantised to round_half_even(255 I)/255.
    4. colour: Y'CbCr (BT.601 full range) or IPT.
    """
    if colorspace not in ("ycbcr", "ipt"):
        raise ValueError("colorspace must be 'ycbcr' or 'ipt'")
    if H < 2 or W < 2 or E < 1:
        raise ValueError("need H, W >= 2 and E >= 1")
    rng = np.random.default_rng(seed)
    logr = _gaussian_blobs(rng, 64, H, W, 0.02, 0.25, 3) + _gradient(rng, H, W)[None]
    logr = _minmax(logr)
    rad_l = np.power(10.0, 4.0 * logr)
    depth = _gaussian_blobs(rng, 8, H, W, 0.15, 0.6, 1)[0] + _gradient(rng, H, W)
    disp = 32.0 * _minmax(depth)
    rad_r = _shift_rows(rad_l, disp)
    k = 0.18 / math.exp(float(np.mean(np.log(rad_l))))
    evs = [e - (E - 1) / 2.0 for e in range(E)]
    out = np.empty((H, W, 3, 2 * E), dtype=dtype)
    convert = _to_ycbcr if colorspace == "ycbcr" else _to_ipt
    for v, rad in enumerate((rad_l, rad_r)):
        for e, ev in enumerate(evs):
            lin = np.clip(k * (2.0 ** ev) * rad, 0.0, None)
            img = np.clip(np.power(lin, 1.0 / 2.2), 0.0, 1.0)
            img = np.round(255.0 * img) / 255.0
            col = convert(img)
            out[:, :, :, v * E + e] = np.moveaxis(col, 0, -1).astype(dtype)
    return out


# --------------------------------------------------------------------------
# Serving workload: a stream of stacks of mixed size
# --------------------------------------------------------------------------

_SERVE_RES = ((640, 480), (1280, 720), (1920, 1080), (2560, 1440))  # (W, H)
_SERVE_EXPOSURES = (3, 5, 7)


def serving_requests(n: int = 512, mean_interarrival_s: float = 0.025, seed: int = 3):
    """Poisson arrivals of stereo-stack requests of mixed resolution and exposure count.

    Returns a list of dicts {t_arrive, H, W, E, ranks, seed}; the tensor of request j is
    ``make_stereo_stack(H, W, E, 'ycbcr', seed=1000 + j)`` and its ranks are (H/4, W/4, 3, 2E-1).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(mean_interarrival_s, size=n)
    res = rng.integers(0, len(_SERVE_RES), size=n)
    exps = rng.integers(0, len(_SERVE_EXPOSURES), size=n)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for j in range(n):
        Wd, Hd = _SERVE_RES[int(res[j])]
        E = _SERVE_EXPOSURES[int(exps[j])]
        reqs.append(dict(t_arrive=float(t[j]), H=Hd, W=Wd, E=E,
                         ranks=(Hd // 4, Wd // 4, 3, 2 * E - 1), seed=1000 + j))
    return reqs
