"""Rotation-invariant comparison of two Tucker decompositions -- TEST INFRASTRUCTURE.

Factors are only defined up to a rotation inside their column space (eq. (1) holds for
any orthonormal basis of the same subspaces, with the core rotated to match), so two
results are compared through quantities that do not depend on that choice:

* the fit and the relative residual rho = 1 - fit;
* the core norm ||G||;
* the reconstruction difference ||Xhat_a - Xhat_b|| / ||Xhat_b||, evaluated in core space:
  ||Xhat_a - Xhat_b||^2 = ||G_a||^2 + ||G_b||^2 - 2 <G_a, G_b x_n (U_a,n^T U_b,n)>;
* the largest principal-angle sine per mode, sin theta_max = ||U_a - U_b (U_b^T U_a)||_2.

All arithmetic is float64.  The norm expansion resolves reconstruction differences down to about
2e-8 relative (cancellation in ||G_a||^2 + ||G_b||^2 - 2<.,.>), far below the tolerances it checks.

Pins: tests/test_compare_pins.py checks every function here against reconstructions written out
with einsum, subspaces with principal angles fixed by construction, singular values of U_a^T U_b
and closed forms, and plants mistakes in source copies of this file to show that they are caught.
"""

from __future__ import annotations

import math

import numpy as np


def _ttm(x, m, n):
    return np.moveaxis(np.tensordot(m, x, axes=([1], [n])), 0, n)


def recon_diff(core_a, factors_a, core_b, factors_b) -> float:
    """||Xhat_a - Xhat_b|| / ||Xhat_b|| without forming either reconstruction."""
    ga = np.asarray(core_a, dtype=np.float64)
    gb = np.asarray(core_b, dtype=np.float64)
    # <Xhat_a, Xhat_b> = <G_a, G_b x_1 (U_a1^T U_b1) ... x_N (U_aN^T U_bN)>
    t = gb
    for n, (ua, ub) in enumerate(zip(factors_a, factors_b)):
        m = np.asarray(ua, dtype=np.float64).T @ np.asarray(ub, dtype=np.float64)
        t = _ttm(t, m, n)
    # Xhat norms equal core norms only for orthonormal factors: use Gram-corrected norms.
    def _norm2(g, fs):
        y = g
        for n, u in enumerate(fs):
            u = np.asarray(u, dtype=np.float64)
            y = _ttm(y, u.T @ u, n)
        return float(np.sum(g * y))
    na2 = _norm2(ga, factors_a)
    nb2 = _norm2(gb, factors_b)
    cross = float(np.sum(ga * t))
    d2 = max(na2 + nb2 - 2.0 * cross, 0.0)
    return math.sqrt(d2) / math.sqrt(nb2) if nb2 > 0 else math.sqrt(d2)


def sin_theta_max(ua, ub) -> float:
    """Largest principal-angle sine between span(ua) and span(ub) (both orthonormal)."""
    ua = np.asarray(ua, dtype=np.float64)
    ub = np.asarray(ub, dtype=np.float64)
    d = ua - ub @ (ub.T @ ua)
    if d.size == 0:
        return 0.0
    return float(np.linalg.norm(d, 2))


def orthonormality_error(u) -> float:
    u = np.asarray(u, dtype=np.float64)
    return float(np.linalg.norm(u.T @ u - np.eye(u.shape[1]), 2))


def compare(result_a, result_b) -> dict:
    """Metrics of decomposition a (e.g. the GPU) against b (the oracle).

    Each argument is a mapping with keys core, factors, fit.
    """
    ga = np.asarray(result_a["core"], dtype=np.float64)
    gb = np.asarray(result_b["core"], dtype=np.float64)
    nga, ngb = float(np.linalg.norm(ga)), float(np.linalg.norm(gb))
    out = {
        "fit": abs(float(result_a["fit"]) - float(result_b["fit"])),
        "rho": abs((1.0 - float(result_a["fit"])) - (1.0 - float(result_b["fit"]))),
        "core_norm": abs(nga - ngb) / ngb if ngb > 0 else abs(nga - ngb),
        "recon": recon_diff(ga, result_a["factors"], gb, result_b["factors"]),
        "sin_theta": [sin_theta_max(ua, ub) for ua, ub in zip(result_a["factors"], result_b["factors"])],
        "orth": [orthonormality_error(u) for u in result_a["factors"]],
    }
    return out
