"""Pins of the oracle's comparison functions and of its reconstruction.

Every GPU parity verdict goes through oracle.compare: the reconstruction difference computed in
core space (the norm expansion of eq. (1)), the largest principal-angle sine between factor
subspaces, orthonormality, fit and core norm.  These tests check each of them against a route
that does not reuse the oracle:

* reconstructions written out with one einsum (the definition of eq. (1));
* subspaces with principal angles fixed by construction, and the singular values of U_a^T U_b;
* closed forms (a scaled copy, rotated-equivalent decompositions, scaled columns).

The last test plants mistakes in source copies of oracle/compare.py and shows that the pins fail
on each of them.
"""

import importlib
import math
import os
import types

import numpy as np
import pytest

import oracle
from oracle import hooi_ref

cmp_mod = importlib.import_module("oracle.compare")    # the package re-exports a function of that name

HERE = os.path.dirname(os.path.abspath(__file__))
COMPARE_SRC = os.path.join(os.path.dirname(HERE), "oracle", "compare.py")


def einsum_reconstruct(core, factors):
    """Xhat[i, j, ...] = sum_r G[r...] prod_n U_n[i_n, r_n] (eq. (1)), one einsum."""
    lr = "abcdefgh"[: core.ndim]
    li = "ijklmnop"[: core.ndim]
    spec = lr + "," + ",".join(i + r for i, r in zip(li, lr)) + "->" + li
    return np.einsum(spec, core, *factors, optimize=True)


def explicit_recon_diff(ga, fa, gb, fb):
    xa = einsum_reconstruct(ga, fa)
    xb = einsum_reconstruct(gb, fb)
    return float(np.linalg.norm(xa - xb) / np.linalg.norm(xb))


def haar(rng, s, r):
    q, rr = np.linalg.qr(rng.standard_normal((s, r)))
    return q * np.sign(np.diag(rr))[None, :]


def known_angle_pair(rng, s, thetas):
    """(U_a, U_b) with principal angles exactly `thetas`, in random bases of both subspaces."""
    r = len(thetas)
    assert 2 * r <= s
    basis = haar(rng, s, 2 * r)                     # orthonormal e_1 .. e_2r in R^s
    ub = basis[:, :r]
    ua = basis[:, :r] * np.cos(thetas)[None, :] + basis[:, r:] * np.sin(thetas)[None, :]
    # any orthonormal basis of the same subspaces: rotate each by an independent orthogonal matrix
    return ua @ haar(rng, r, r), ub @ haar(rng, r, r)


def random_decomp(rng, dims, ranks, orthonormal=True):
    core = rng.standard_normal(ranks)
    facs = [haar(rng, s, r) if orthonormal else rng.standard_normal((s, r)) for s, r in zip(dims, ranks)]
    return core, facs


# ---------------------------------------------------------------- reconstruct

@pytest.mark.parametrize("dims,ranks", [
    ((7, 5), (3, 2)),
    ((6, 5, 4), (3, 3, 2)),
    ((5, 6, 3, 4), (2, 3, 3, 2)),
    ((4, 3, 5, 2, 3), (2, 2, 3, 1, 2)),
])
def test_reconstruct_matches_einsum(dims, ranks):
    rng = np.random.default_rng(len(dims))
    core, facs = random_decomp(rng, dims, ranks, orthonormal=False)
    got = hooi_ref.reconstruct(core, facs)
    ref = einsum_reconstruct(core, facs)
    assert got.shape == tuple(dims)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_reconstruct_rank_one_outer_product():
    rng = np.random.default_rng(3)
    vs = [rng.standard_normal(s) for s in (4, 3, 5, 2)]
    core = np.full((1, 1, 1, 1), 2.5)
    got = hooi_ref.reconstruct(core, [v[:, None] for v in vs])
    ref = 2.5 * np.multiply.outer(np.multiply.outer(np.multiply.outer(vs[0], vs[1]), vs[2]), vs[3])
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))


# ---------------------------------------------------------------- recon_diff

@pytest.mark.parametrize("orthonormal", [True, False])
@pytest.mark.parametrize("ranks_b", [(3, 2, 2, 2), (2, 3, 1, 2)])
def test_recon_diff_matches_explicit(orthonormal, ranks_b):
    rng = np.random.default_rng(11 if orthonormal else 12)
    dims, ranks_a = (8, 7, 3, 5), (3, 2, 2, 2)
    ga, fa = random_decomp(rng, dims, ranks_a, orthonormal)
    gb, fb = random_decomp(rng, dims, ranks_b, orthonormal)
    got = oracle.recon_diff(ga, fa, gb, fb)
    ref = explicit_recon_diff(ga, fa, gb, fb)
    assert abs(got - ref) <= 1e-12 * max(ref, 1.0), (got, ref)


def test_recon_diff_nearby_decompositions():
    """Small differences (the size parity tests resolve) are computed accurately."""
    rng = np.random.default_rng(5)
    dims, ranks = (9, 8, 3, 4), (4, 3, 2, 2)
    ga, fa = random_decomp(rng, dims, ranks)
    for eps in (1e-3, 1e-5):
        gb = ga + eps * rng.standard_normal(ranks)
        fb = [np.linalg.qr(u + eps * rng.standard_normal(u.shape))[0] for u in fa]
        got = oracle.recon_diff(ga, fa, gb, fb)
        ref = explicit_recon_diff(ga, fa, gb, fb)
        # the norm expansion loses about sqrt(machine epsilon) relative to ||Xhat|| to cancellation
        assert abs(got - ref) <= 1e-3 * ref + 5e-8, (eps, got, ref)


def test_recon_diff_rotated_equivalent_is_zero():
    """(G x_n Q_n^T, U_n Q_n) reconstructs the same tensor for orthogonal Q_n."""
    rng = np.random.default_rng(6)
    dims, ranks = (9, 8, 3, 5), (4, 3, 3, 2)
    ga, fa = random_decomp(rng, dims, ranks)
    qs = [haar(rng, r, r) for r in ranks]
    gb = ga
    for n, q in enumerate(qs):
        gb = np.moveaxis(np.tensordot(q.T, gb, axes=([1], [n])), 0, n)
    fb = [u @ q for u, q in zip(fa, qs)]
    assert explicit_recon_diff(ga, fa, gb, fb) <= 1e-13
    assert oracle.recon_diff(ga, fa, gb, fb) <= 1e-7


def test_recon_diff_scaled_copy_closed_form():
    """Xhat_b = 2 Xhat_a gives ||Xhat_a - Xhat_b|| / ||Xhat_b|| = 1/2, for any factor scaling."""
    rng = np.random.default_rng(7)
    dims, ranks = (6, 7, 3, 4), (3, 3, 2, 2)
    ga, fa = random_decomp(rng, dims, ranks, orthonormal=False)
    fb = [u * 2.0 ** (1.0 / 4.0) for u in fa]         # (2^(1/4))^4 = 2 over the four modes
    assert abs(oracle.recon_diff(ga, fa, ga, fb) - 0.5) <= 1e-12
    assert abs(oracle.recon_diff(ga, fa, 2.0 * ga, fa) - 0.5) <= 1e-12


# ---------------------------------------------------------------- principal angles

@pytest.mark.parametrize("thetas", [
    [0.3, 0.1, 0.0],
    [1e-6, 2e-7, 5e-7, 0.0],
    [math.pi / 2, 0.2],
    [0.05, 0.9, 0.4, 0.7, 0.01],
])
def test_sin_theta_known_angles(thetas):
    rng = np.random.default_rng(len(thetas))
    ua, ub = known_angle_pair(rng, 13, np.array(thetas))
    want = math.sin(max(thetas))
    assert abs(oracle.sin_theta_max(ua, ub) - want) <= 1e-14 + 1e-12 * want
    assert abs(oracle.sin_theta_max(ub, ua) - want) <= 1e-14 + 1e-12 * want


def test_sin_theta_matches_singular_values():
    """sin theta_max = sqrt(1 - sigma_min(U_a^T U_b)^2) for equal-dimension subspaces."""
    rng = np.random.default_rng(9)
    # (s = r would make the reference itself cancel: sqrt(1 - sigma^2) with sigma = 1 - O(eps))
    for s, r in ((10, 3), (40, 12), (9, 4)):
        ua, ub = haar(rng, s, r), haar(rng, s, r)
        smin = np.linalg.svd(ua.T @ ub, compute_uv=False).min()
        want = math.sqrt(max(0.0, 1.0 - smin ** 2))
        assert abs(oracle.sin_theta_max(ua, ub) - want) <= 1e-12


def test_sin_theta_same_subspace_is_zero():
    rng = np.random.default_rng(10)
    u = haar(rng, 20, 6)
    assert oracle.sin_theta_max(u, u @ haar(rng, 6, 6)) <= 1e-14
    assert oracle.sin_theta_max(haar(rng, 7, 7), haar(rng, 7, 7)) <= 1e-14     # both span R^7


def test_orthonormality_error_closed_form():
    rng = np.random.default_rng(13)
    u = haar(rng, 12, 4)
    eps = 1e-3
    v = u.copy()
    v[:, 2] *= 1.0 + eps                             # U^T U - I = diag(0, 0, 2 eps + eps^2, 0)
    assert abs(oracle.orthonormality_error(v) - (2 * eps + eps * eps)) <= 1e-15
    assert oracle.orthonormality_error(u) <= 1e-14


def test_compare_assembles_the_metrics():
    rng = np.random.default_rng(14)
    dims, ranks = (8, 6, 3, 4), (3, 3, 2, 2)
    ga, fa = random_decomp(rng, dims, ranks)
    gb = 1.5 * ga
    m = oracle.compare(dict(core=ga, factors=fa, fit=0.9), dict(core=gb, factors=fa, fit=0.95))
    assert abs(m["fit"] - 0.05) <= 1e-15
    assert abs(m["rho"] - 0.05) <= 1e-15
    assert abs(m["core_norm"] - 1.0 / 3.0) <= 1e-14          # | ||G|| - 1.5 ||G|| | / (1.5 ||G||)
    assert abs(m["recon"] - 1.0 / 3.0) <= 1e-12
    assert max(m["sin_theta"]) <= 1e-14
    assert len(m["orth"]) == 4 and max(m["orth"]) <= 1e-14


# ---------------------------------------------------------------- planted mistakes

def _pins_pass(mod):
    """A reduced set of the pins above run against a (possibly broken) copy of compare.py."""
    try:
        rng = np.random.default_rng(21)
        dims = (8, 7, 3, 5)
        ga, fa = random_decomp(rng, dims, (3, 2, 2, 2), orthonormal=False)
        gb, fb = random_decomp(rng, dims, (2, 3, 1, 2), orthonormal=False)
        ref = explicit_recon_diff(ga, fa, gb, fb)
        if abs(mod.recon_diff(ga, fa, gb, fb) - ref) > 1e-12 * max(ref, 1.0):
            return False
        ga, fa = random_decomp(rng, dims, (3, 2, 2, 2))
        gb, fb = random_decomp(rng, dims, (3, 2, 2, 2))
        ref = explicit_recon_diff(ga, fa, gb, fb)
        if abs(mod.recon_diff(ga, fa, gb, fb) - ref) > 1e-12 * max(ref, 1.0):
            return False
        thetas = np.array([0.05, 0.9, 0.4, 0.7, 0.01])
        ua, ub = known_angle_pair(rng, 13, thetas)
        if abs(mod.sin_theta_max(ua, ub) - math.sin(0.9)) > 1e-12:
            return False
        m = mod.compare(dict(core=ga, factors=fa, fit=0.9), dict(core=1.5 * ga, factors=fa, fit=0.95))
        if abs(m["core_norm"] - 1.0 / 3.0) > 1e-14 or abs(m["recon"] - 1.0 / 3.0) > 1e-12:
            return False
        return True
    except Exception:
        return False


def _mutant(old, new):
    src = open(COMPARE_SRC).read()
    assert src.count(old) == 1, old
    mod = types.ModuleType("compare_mutant")
    exec(compile(src.replace(old, new), "compare_mutant", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("old,new", [
    # the norm of a reconstruction without the factor Gram correction (exact only for orthonormal U)
    ("y = _ttm(y, u.T @ u, n)", "y = y"),
    # cross term built from U_b^T U_a instead of U_a^T U_b
    ("m = np.asarray(ua, dtype=np.float64).T @ np.asarray(ub, dtype=np.float64)",
     "m = np.asarray(ub, dtype=np.float64).T @ np.asarray(ua, dtype=np.float64)"),
    # normalised by the wrong reconstruction
    ("return math.sqrt(d2) / math.sqrt(nb2) if nb2 > 0", "return math.sqrt(d2) / math.sqrt(na2) if nb2 > 0"),
    # a factor 2 dropped from the cross term
    ("d2 = max(na2 + nb2 - 2.0 * cross, 0.0)", "d2 = max(na2 + nb2 - cross, 0.0)"),
    # Frobenius norm of the residual instead of the spectral norm (sums the angles)
    ("return float(np.linalg.norm(d, 2))", "return float(np.linalg.norm(d))"),
    # residual against the wrong projector
    ("d = ua - ub @ (ub.T @ ua)", "d = ua - ua @ (ub.T @ ub)"),
    # core norm compared as squares
    ("\"core_norm\": abs(nga - ngb) / ngb", "\"core_norm\": abs(nga ** 2 - ngb ** 2) / ngb ** 2"),
])
def test_planted_mistakes_in_compare_are_caught(old, new):
    assert _pins_pass(cmp_mod)
    assert not _pins_pass(_mutant(old, new))
