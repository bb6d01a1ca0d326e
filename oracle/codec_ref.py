"""Ordered core and core quantisation (the codec hand-off) -- TEST INFRASTRUCTURE, NOT PRODUCT CODE.

Only the tests may import this module.  It shares no code with the HIP library.

The paper adjusts the bit rate of the Tucker representation by the rank of the core and by its
quantisation (Abstract; Sec. I).  Two steps prepare a decomposition for that:

* order_core: rotate each factor inside its column space so that the core becomes all-orthogonal
  with its mode-n slices sorted by energy: with C_n = G_(n) G_(n)^T = V_n diag(sigma_n^2) V_n^T
  (descending), U_n <- U_n V_n and G <- G x_n V_n^T for every n.  Xhat is unchanged (eq. (1) holds for
  any orthonormal basis of the same subspaces), slices of G along mode n are mutually orthogonal
  with norms sigma_n (the mode-n singular values of the core), and the leading k_n slices are the
  best rank-(k_1, ..., k_N) truncation in the sense that the discarded energy is known per mode.
* truncate + quantize_core: keep the leading k_n slices of the ordered core (and columns of the
  factors), then quantise the kept core uniformly: step = max|G| / (2^(b-1) - 1), codes =
  round-half-even(G / step) in [-(2^(b-1) - 1), 2^(b-1) - 1], dequantised core = codes * step.  The
  quantiser works in binary32 (the core's own precision), one correctly rounded operation at a time,
  so that an implementation on the same binary32 core reaches the same integer codes.

Pins: tests/test_codec_pins.py.
"""

from __future__ import annotations

import numpy as np

from .hooi_ref import ttm, unfold


def order_core(core: np.ndarray, factors):
    """All-orthogonal, energy-ordered core (FP64).  Returns (core, factors, sigma) with sigma[n] the
    mode-n singular values of the core, descending."""
    g = np.asarray(core, dtype=np.float64)
    vs, sig = [], []
    for n in range(g.ndim):
        c = unfold(g, n) @ unfold(g, n).T
        lam, v = np.linalg.eigh(c)
        order = np.argsort(lam)[::-1]
        vs.append(v[:, order])
        sig.append(np.sqrt(np.maximum(lam[order], 0.0)))
    out = g
    for n, v in enumerate(vs):
        out = ttm(out, v.T, n)
    facs = [np.asarray(u, dtype=np.float64) @ v for u, v in zip(factors, vs)]
    return out, facs, sig


def truncate(core: np.ndarray, factors, keep):
    """The leading keep[n] slices of the core along every mode and the matching factor columns."""
    idx = tuple(slice(0, int(k)) for k in keep)
    return np.array(core[idx]), [np.array(u[:, : int(k)]) for u, k in zip(factors, keep)]


def quantize_core(core: np.ndarray, bits: int):
    """Uniform mid-tread quantiser in binary32.  Returns (codes int32, dequantised float32, step float32)."""
    if not 2 <= int(bits) <= 24:
        raise ValueError("bits must be in [2, 24]")
    g = np.asarray(core, dtype=np.float32)
    levels = np.float32(2 ** (int(bits) - 1) - 1)
    amax = np.float32(np.max(np.abs(g))) if g.size else np.float32(0.0)
    if amax == 0.0:
        return np.zeros(g.shape, dtype=np.int32), np.zeros(g.shape, dtype=np.float32), np.float32(0.0)
    step = np.float32(amax / levels)
    q = np.rint(g / step).astype(np.float32)              # binary32 quotient, ties to even
    q = np.clip(q, -levels, levels)
    deq = (q * step).astype(np.float32)
    return q.astype(np.int32), deq, step
