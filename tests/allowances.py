"""Tolerance allowances for comparing the GPU HOOI with the FP64 oracle on image stacks.

The GPU finds the leading R_n-dimensional eigenspace of each large mode's Gram by orthogonal
(subspace) iteration: a cold start from a seeded random basis, then warm steps, one per sweep by
default.  The oracle takes exact eigenvectors (LAPACK).  Subspace iteration converges direction by
direction: after q steps the component of the i-th leading eigenvector outside the iterated
subspace is bounded by tan theta_i <= (lam_{R+1} / lam_i)^q tan theta_0 (Golub & Van Loan,
Matrix Computations, Thm. 8.2.2, applied to the leading i-dimensional eigenspace), with
tan theta_0 <= sqrt(s R) for a random start of s x R uniform entries.  On the image stacks the
ratio lam_{R+1} / lam_R sits between 0.90 and 0.9985 (the Gram spectra decay smoothly), so the
directions next to the rank boundary cannot converge in the step counts used, while the leading
ones do.  A direction i that is off by theta_i moves the reconstruction by at most
theta_i sqrt(2 lam_i) (the energy it carries into the complement), so per mode

    a_n = sqrt(2 sum_{i <= R} lam_i min(1, (lam_{R+1} / lam_i)^q sqrt(s R))^2 / sum(lam)),

relative to ||Xhat|| ~ sqrt(sum(lam)).  The reconstruction difference is then bounded by
1e-5 + sum_n a_n, while the fit, the residual and the core norm, second-order in the angles,
stay binding at 1e-5.  Modes with R_n = s_n, or small enough to be diagonalised exactly (Jacobi),
contribute nothing.
"""

from __future__ import annotations

import math

import numpy as np

SMALL_MODE = 64        # modes up to this size use the exact Jacobi eigensolver on the GPU


def _direction_bounds(lam, s, r, steps=None, resid=None):
    """Per-direction bounds on sin theta_i, i = 1..R: the subspace-iteration term after `steps`
    steps, or, for an iteration stopped on a relative residual ||S U - U U^T S U||_F <= resid ||S||_F,
    the residual form of the Davis-Kahan sin-theta theorem, resid ||S||_F / (lam_i - lam_{R+1})."""
    if steps is not None:
        return np.minimum(1.0, (lam[r] / lam[:r]) ** steps * math.sqrt(s * r))
    gap = np.maximum(lam[:r] - lam[r], 1e-300)
    return np.minimum(1.0, resid * math.sqrt(float(np.sum(lam * lam))) / gap)


def si_allowance(spectra, dims, ranks, steps=None, resid=None) -> float:
    """sum_n a_n over the modes updated by orthogonal iteration; steps: iteration count per mode
    (or resid: the relative residual the iteration was stopped on)."""
    total = 0.0
    for n, (s, r) in enumerate(zip(dims, ranks)):
        if r >= s or s <= SMALL_MODE:
            continue
        lam = np.asarray(spectra[n], dtype=np.float64)
        lam = np.maximum(lam, 0.0)
        if lam[r] <= 0.0:
            continue
        t = _direction_bounds(lam, s, r, steps, resid)
        total += math.sqrt(2.0 * float(np.sum(lam[:r] * t * t)) / float(np.sum(lam)))
    return total


def _ritz_bounds(lam, s, r, steps, oversample):
    """Per-direction bounds on sin theta_i, i = 1..R, for orthogonal iteration on Rc = min(s, R + p)
    columns followed by Rayleigh-Ritz (the R leading Ritz vectors of U^T S U).

    The iteration leaves the i-th eigenvector at angle <= (lam_{Rc+1} / lam_i)^q sqrt(s Rc) from the
    Rc-dimensional iterate (the subspace-iteration term above with Rc columns; 0 when Rc = s).  The
    Ritz vectors taken from that subspace are off the eigenvectors by at most that angle times
    sqrt(1 + gamma^2 / delta^2) (Saad, Numerical Methods for Large Eigenvalue Problems, Thm. 4.6),
    with gamma = ||P S (I - P)|| <= lam_1 and delta >= lam_R - lam_{R+1} (Cauchy interlacing puts
    every discarded Ritz value at or below lam_{R+1}), so the amplification is at most
    sqrt(1 + g^2) with g = lam_1 / (lam_R - lam_{R+1}), the boundary gap factor."""
    rc = min(s, r + oversample)
    if rc >= s:
        return np.zeros(r)
    gap = lam[r - 1] - lam[r]
    amp = math.sqrt(1.0 + (lam[0] / gap) ** 2) if gap > 0 else math.inf
    cont = (lam[rc] / lam[:r]) ** steps * math.sqrt(s * rc)
    return np.minimum(1.0, cont * amp)


def rr_allowance(spectra, dims, ranks, steps, oversample) -> float:
    """sum_n a_n as in si_allowance, for the oversampled start closed by Rayleigh-Ritz."""
    total = 0.0
    for n, (s, r) in enumerate(zip(dims, ranks)):
        if r >= s or s <= SMALL_MODE:
            continue
        lam = np.maximum(np.asarray(spectra[n], dtype=np.float64), 0.0)
        t = _ritz_bounds(lam, s, r, steps, oversample)
        total += math.sqrt(2.0 * float(np.sum(lam[:r] * t * t)) / float(np.sum(lam)))
    return total


def rr_sine_bound(spectrum, s, r, steps, oversample) -> float:
    """Bound on the largest principal-angle sine between the R-dimensional result of the oversampled
    start and the leading eigenspace (the boundary direction's term of _ritz_bounds)."""
    lam = np.maximum(np.asarray(spectrum, dtype=np.float64), 0.0)
    return float(_ritz_bounds(lam, s, r, steps, oversample)[-1])


def pair_allowance(spectra, ranks, gap_limit=1e8) -> float:
    """One boundary direction pair, sqrt(2 lam_R / sum(lam)), for every mode whose boundary gap
    factor lam_1 / (lam_R - lam_{R+1}) exceeds gap_limit (a degenerate boundary)."""
    extra = 0.0
    for n, r in enumerate(ranks):
        lam = np.asarray(spectra[n], dtype=np.float64)
        if r >= len(lam):
            continue
        gap = lam[r - 1] - lam[r]
        g = lam[0] / gap if gap > 0 else math.inf
        if g > gap_limit:
            extra += math.sqrt(2.0 * max(lam[r - 1], 0.0) / float(np.sum(lam)))
    return extra


def leading_containment(u_oracle, u_gpu, spectrum, steps=None, resid=None, gram_err=1e-6, limit=1e-4):
    """How well span(u_gpu) contains the oracle's k leading eigenvectors (columns of u_oracle,
    descending), for the largest k whose a-priori bound stays within `limit`.

    Bound for the leading-k eigenspace against the GPU's R-dimensional subspace: the subspace
    iteration term (lam_{R+1} / lam_k)^q sqrt(s R) plus the Davis-Kahan term of a Gram perturbation
    ||dS|| <= gram_err lam_1 over the gap lam_k - lam_{R+1} (the sin-theta theorem for a k-dimensional
    eigenspace against an R-dimensional invariant subspace of the perturbed matrix).
    With resid instead of steps, the first term is the residual bound of _direction_bounds.
    Returns (k, measured sine, bound); k = 0 when no direction qualifies."""
    u_o = np.asarray(u_oracle, dtype=np.float64)
    u_g = np.asarray(u_gpu, dtype=np.float64)
    s, r = u_o.shape
    lam = np.maximum(np.asarray(spectrum, dtype=np.float64), 0.0)
    k, bound = 0, 0.0
    it = _direction_bounds(lam, s, r, steps, resid)
    for i in range(1, r + 1):
        gap = lam[i - 1] - lam[r]
        if gap <= 0.0:
            break
        b = float(it[i - 1]) + gram_err * lam[0] / gap
        if b > limit:
            break
        k, bound = i, b
    if k == 0:
        return 0, 0.0, 0.0
    v = u_o[:, :k]
    sine = float(np.linalg.norm(v - u_g @ (u_g.T @ v), 2))
    return k, sine, bound
