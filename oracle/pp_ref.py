"""Pairwise-perturbation HOOI in FP64 -- TEST INFRASTRUCTURE, NOT PRODUCT CODE.

Only the tests may import this module.  It shares no code with the HIP library.

The paper accelerates the ALS sweeps by pairwise perturbation (Sec. III-B, eq. (9)-(13)): when the
factors change little between sweeps, each factor S(i) is written as S_p(i) + dS(i) around factors
S_p computed p sweeps earlier, and the tensor of an update,
    Y(n) = X x_{i != n} (S_p(i) + dS(i))^T                                   (eq. (9)),
is replaced by its expansion to first order in the dS(i):
    Y~(n) = Y_p(n) + sum_{i != n} Y_p(i,n) x_i dS(i)^T                        (eq. (11)),
    Y_p(n) = X x_{l != n} S_p(l)^T                                            (eq. (12)),
    Y_p(i,n) = X x_{j not in {i,n}} S_p(j)^T                                  (eq. (13)).
The operators Y_p(n) and Y_p(i,n) are formed once per reference point; the sweeps that follow read
only them (never X) until the factors move too far from the reference.

Readings where the paper is silent (each listed with the others in the design notes):
* Factor representative.  dS(i) compares two orthonormal bases, which the eigenvectors of a Gram fix
  only up to a rotation (and sign).  In a perturbation sweep every new factor is therefore represented
  by the orthonormal basis of its column space closest to the reference in the Frobenius norm
  (orthogonal Procrustes: S <- S W V^T with S^T S_p = W Sigma V^T); this changes no subspace.  The
  paper's remark that the Gram route keeps "singular vector signatures consistent" across sweeps is
  read as this alignment.  Ordinary sweeps are plain HOOI.
* Switching rule, on the representative-free distance of two subspaces,
  d(S, S') = ||S S^T - S' S'^T||_F / sqrt(2 R) (the root-mean-square sine of their principal angles):
  ordinary sweeps run until max_i d(S(i), S_prev(i)) between consecutive sweeps falls below pp_tol;
  the current factors then become the reference, the operators are formed, and perturbation sweeps
  run while max_i d(S(i), S_p(i)) stays below pp_tol; a larger distance sends the next sweep back to an
  ordinary one.
* Fit.  A perturbation sweep's fit comes from its first-order core G~ = Y~(N) x_N S(N)^T; the returned
  core and fit are always recomputed exactly from X.

Pins: tests/test_pp_pins.py.
"""

from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

from .hooi_ref import (fit_from_norms, gram, leading_eigvecs, project_all, project_all_but, thosvd_factors,
                       ttm, validate)


def procrustes_align(u: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """The orthonormal basis of span(u) closest to ref: u Q with Q the polar factor of u^T ref."""
    w, _, vt = np.linalg.svd(u.T @ ref)
    return u @ (w @ vt)


def pp_operators(x: np.ndarray, ref):
    """Y_p(n) (eq. (12)) for every n and Y_p(i,n) (eq. (13)) for every pair i < n (symmetric in i, n)."""
    n_modes = x.ndim
    single = [project_all_but(x, ref, n) for n in range(n_modes)]
    pair = {}
    for i in range(n_modes):
        for n in range(i + 1, n_modes):
            y = x
            for j, u in enumerate(ref):
                if j not in (i, n):
                    y = ttm(y, u.T, j)
            pair[(i, n)] = y
    return single, pair


def pp_tensor(single, pair, factors, ref, n):
    """Y~(n) = Y_p(n) + sum_{i != n} Y_p(i,n) x_i (S(i) - S_p(i))^T (eq. (11))."""
    y = single[n].copy()
    for i in range(len(factors)):
        if i == n:
            continue
        ds = factors[i] - ref[i]
        y = y + ttm(pair[(min(i, n), max(i, n))], ds.T, i)
    return y


def subspace_distance(u: np.ndarray, v: np.ndarray) -> float:
    """||u u^T - v v^T||_F / sqrt(2 R) for orthonormal u, v (s x R)."""
    r = u.shape[1]
    return float(np.linalg.norm(u @ u.T - v @ v.T)) / math.sqrt(2.0 * r)


def rel_change(a, b) -> float:
    return max(subspace_distance(u, v) for u, v in zip(a, b))


@dataclass
class PPResult:
    core: np.ndarray
    factors: list
    fits: list                     # fits[0] start; fits[k] after sweep k (first-order core in PP sweeps)
    kinds: list                    # "als" or "pp" per sweep
    changes: list                  # subspace distance after each sweep (the switching quantity)
    fit: float                     # exact fit of the returned decomposition
    norm_x2: float
    spectra: list = field(default_factory=list)


def hooi_pp(x: np.ndarray, ranks, max_iters: int = 10, pp_tol: float = 0.1) -> PPResult:
    """HOOI from the T-HOSVD start with pairwise-perturbation sweeps (switching rule above)."""
    x = np.asarray(x, dtype=np.float64)
    ranks = [int(r) for r in ranks]
    validate(x.shape, ranks, max_iters, 0.0)
    nx2 = float(np.sum(x * x))
    factors, spectra = thosvd_factors(x, ranks)
    core = project_all(x, factors)
    fits = [fit_from_norms(nx2, float(np.sum(core * core)))]
    kinds, changes = [], []
    mode, ref, ops = "als", None, None
    for _ in range(max_iters):
        prev = [u.copy() for u in factors]
        y = None
        for n, r in enumerate(ranks):
            if mode == "pp":
                y = pp_tensor(ops[0], ops[1], factors, ref, n)
            else:
                y = project_all_but(x, factors, n)
            if r < x.shape[n]:
                u, lam = leading_eigvecs(gram(y, n), r)
                factors[n] = procrustes_align(u, ref[n]) if mode == "pp" else u
                spectra[n] = lam
        core = ttm(y, factors[-1].T, x.ndim - 1)
        fits.append(fit_from_norms(nx2, float(np.sum(core * core))))
        kinds.append(mode)
        if mode == "pp":
            ch = rel_change(factors, ref)
            changes.append(ch)
            if ch > pp_tol:
                mode = "als"
        else:
            ch = rel_change(factors, prev)
            changes.append(ch)
            if ch < pp_tol:
                mode, ref = "pp", [u.copy() for u in factors]
                ops = pp_operators(x, ref)
    core = project_all(x, factors)
    fit = fit_from_norms(nx2, float(np.sum(core * core)))
    return PPResult(core, factors, fits, kinds, changes, fit, nx2, spectra)
