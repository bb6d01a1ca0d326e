"""Pins of the oracle's sequentially truncated ("interlaced") HOSVD start -- CPU only.

The paper offers the interlaced HOSVD as a cheaper way to the start (Sec. III-B.1, after
eq. (7)); oracle/hooi_ref.py reads it as the sequentially truncated HOSVD.  Its result is fixed
without reusing the oracle by:

* brute force: each factor equals the leading left singular vectors (np.linalg.svd) of the mode-n
  unfolding, built entry by entry, of the tensor projected on the earlier factors (einsum);
* the exact error identity of the sequentially truncated HOSVD (Vannieuwenhoven, Vandebril and
  Meerbergen, SIAM J. Sci. Comput. 34 (2012), Thm. 5.1): ||X - Xhat||^2 equals the sum over modes of
  the squared singular values discarded at that mode's step;
* the T-HOSVD truncation bounds max_n tau_n^2 <= ||X - Xhat||^2 <= sum_n tau_n^2, with tau_n^2 the
  discarded energy of the unprojected unfoldings (Thm. 6.5 of the same paper);
* exact multilinear rank: the start equals the T-HOSVD and reconstructs X;
* order 2: the truncated SVD (Eckart-Young);
* HOOI from this start never decreases the fit;
and planted mistakes in source copies of the function fail these checks.
"""

import inspect
import math
import types

import numpy as np
import pytest

import oracle
from oracle import hooi_ref
from synth import make_exact_rank
from test_oracle_pins import einsum_project, einsum_reconstruct, loop_unfold, sin_theta, svd_left


def _project_first(x, factors, upto):
    """X x_1 U_1^T ... x_upto U_upto^T (einsum), the other modes untouched."""
    fs = [factors[m] if m < upto else np.eye(x.shape[m]) for m in range(x.ndim)]
    return einsum_project(x, fs)


def _generic(dims, ranks, seed, noise=0.05):
    x, _, _ = make_exact_rank(dims, ranks, seed, noise)
    return x


def _st_checks(fn, x, ranks, tol=1e-10):
    """Brute-force and identity checks of a sequentially truncated HOSVD implementation fn."""
    factors, spectra, core = fn(x, ranks)
    discarded = 0.0
    for n, r in enumerate(ranks):
        y = _project_first(x, factors, n)
        u, sv = svd_left(loop_unfold(y, n), r)
        if r < x.shape[n] and sin_theta(factors[n], u) > tol:
            return False
        if np.linalg.norm(factors[n].T @ factors[n] - np.eye(r), 2) > tol:
            return False
        discarded += float(np.sum(sv[r:] ** 2))
    if np.max(np.abs(core - einsum_project(x, factors))) > tol * np.max(np.abs(x)):
        return False
    err2 = float(np.sum((x - einsum_reconstruct(core, factors)) ** 2))
    return abs(err2 - discarded) <= tol * float(np.sum(x * x))


@pytest.mark.parametrize("dims,ranks,seed", [((6, 5, 4, 3), (3, 2, 2, 2), 1), ((7, 6, 5), (3, 4, 2), 2),
                                             ((5, 4, 3, 3, 2), (2, 2, 2, 1, 2), 3)])
def test_factors_match_brute_force_svd_and_error_identity(dims, ranks, seed):
    x = _generic(dims, ranks, seed)
    assert _st_checks(hooi_ref.st_hosvd_factors, x, ranks)


@pytest.mark.parametrize("seed", [4, 5])
def test_truncation_bounds_of_thosvd_hold(seed):
    dims, ranks = (9, 8, 3, 6), (4, 3, 2, 3)
    x = _generic(dims, ranks, seed, noise=0.3)
    factors, _, core = hooi_ref.st_hosvd_factors(x, ranks)
    err2 = float(np.sum((x - einsum_reconstruct(core, factors)) ** 2))
    tau2 = [float(np.sum(np.linalg.svd(loop_unfold(x, n), compute_uv=False)[r:] ** 2)) for n, r in enumerate(ranks)]
    assert max(tau2) * (1 - 1e-12) <= err2 <= sum(tau2) * (1 + 1e-12)


def test_exact_rank_equals_thosvd_and_reconstructs():
    x, _, facs_true = make_exact_rank((10, 9, 3, 5), (4, 3, 2, 2), 6, 0.0)
    ranks = (4, 3, 2, 2)
    st, _, core = hooi_ref.st_hosvd_factors(x, ranks)
    th, _ = hooi_ref.thosvd_factors(x, ranks)
    for a, b, t in zip(st, th, facs_true):
        assert sin_theta(a, b) <= 1e-10
        assert sin_theta(a, t) <= 1e-10
    assert np.linalg.norm(x - einsum_reconstruct(core, st)) <= 1e-12 * np.linalg.norm(x)


def test_order2_is_the_truncated_svd():
    rng = np.random.default_rng(8)
    x = rng.standard_normal((12, 9))
    r = 4
    factors, _, core = hooi_ref.st_hosvd_factors(x, (r, r))
    u, s, vt = np.linalg.svd(x)
    assert sin_theta(factors[0], u[:, :r]) <= 1e-12
    assert sin_theta(factors[1], vt[:r].T) <= 1e-12
    err = np.linalg.norm(x - factors[0] @ core @ factors[1].T)
    assert abs(err - math.sqrt(float(np.sum(s[r:] ** 2)))) <= 1e-12 * np.linalg.norm(x)


def test_hooi_from_sthosvd_start_is_monotone_and_starts_there():
    x = _generic((12, 10, 3, 6), (5, 4, 2, 3), 9, noise=0.2)
    ranks = (5, 4, 2, 3)
    res = oracle.hooi(x, ranks, 6, start="sthosvd")
    factors, _, core = hooi_ref.st_hosvd_factors(x, ranks)
    nx2 = float(np.sum(x * x))
    assert abs(res.fits[0] - (1 - math.sqrt(max(nx2 - float(np.sum(core ** 2)), 0)) / math.sqrt(nx2))) <= 1e-13
    assert all(b >= a - 1e-13 for a, b in zip(res.fits, res.fits[1:]))
    th = oracle.hooi(x, ranks, 0)
    assert res.fits[0] >= th.fits[0] - 0.05       # both are quasi-optimal starts of similar quality
    with pytest.raises(ValueError):
        oracle.hooi(x, ranks, 1, start="hosvd")


# ---------------------------------------------------------------- planted mistakes

def _mutant(old, new):
    src = inspect.getsource(hooi_ref.st_hosvd_factors)
    assert src.count(old) == 1, old
    ns = dict(hooi_ref.__dict__)
    exec(compile(src.replace(old, new), "st_mutant", "exec"), ns)
    return ns["st_hosvd_factors"]


@pytest.mark.parametrize("old,new", [
    # no projection between steps: every factor from the unprojected X (the T-HOSVD)
    ("y = ttm(y, u.T, n)", "y = ttm(x, u.T, n) if n == len(ranks) - 1 else y"),
    # Gram of the original tensor instead of the projected one
    ("s_n = gram(y, n)", "s_n = gram(x, n)"),
    # the trailing block of the spectrum
    ("u, lam = leading_eigvecs(s_n, r)", "lam, v = np.linalg.eigh(s_n); u = v[:, :r]; lam = lam[::-1]"),
    # the projected tensor contracted in the wrong mode
    ("y = ttm(y, u.T, n)", "y = ttm(y, u.T, n) if u.shape[0] == u.shape[1] else "
                           "ttm(y, np.eye(y.shape[(n + 1) % y.ndim])[:1], (n + 1) % y.ndim)"),
])
def test_planted_mistakes_are_caught(old, new):
    x = _generic((6, 5, 4, 3), (3, 2, 2, 2), 1)
    assert _st_checks(hooi_ref.st_hosvd_factors, x, (3, 2, 2, 2))
    try:
        ok = _st_checks(_mutant(old, new), x, (3, 2, 2, 2))
    except Exception:
        ok = False
    assert not ok
