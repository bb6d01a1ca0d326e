"""Pins of the oracle's ordered core and core quantisation (oracle/codec_ref.py) -- CPU only.

* order_core leaves the reconstruction unchanged (eq. (1): any orthonormal basis of the same
  subspaces), makes the core all-orthogonal (slices along every mode mutually orthogonal, checked
  slice by slice with explicit loops) with slice norms equal to the returned sigma, descending, and
  sum_i sigma_n,i^2 = ||G||^2 for every n;
* on a full-rank decomposition (R_n = s_n) the ordered core is the HOSVD core of X itself: sigma_n are
  the singular values of the unfolding X_(n) (np.linalg.svd);
* a closed form: a super-diagonal core hidden behind permuted, sign-flipped factors comes back as the
  sorted super-diagonal;
* truncation of the ordered core: ||Xhat - Xhat_k||^2 = ||G||^2 - ||G_k||^2 exactly;
* quantisation: |G - deq| <= step / 2, codes in range, ties to even, the extreme entry maps to the
  extreme code, and ||Xhat(G) - Xhat(deq)|| = ||G - deq|| for orthonormal factors;
and planted mistakes in source copies of the module fail these checks.
"""

import inspect
import math
import types

import numpy as np
import pytest

from oracle import codec_ref
from oracle.hooi_ref import ttm
from test_oracle_pins import einsum_reconstruct, loop_unfold


def _random_decomp(rng, dims, ranks):
    core = rng.standard_normal(ranks) * np.exp(rng.uniform(-2, 2, ranks))
    facs = [np.linalg.qr(rng.standard_normal((s, r)))[0] for s, r in zip(dims, ranks)]
    return core, facs


def _slice_gram(g, n):
    """<G[.., a, ..], G[.., b, ..]> for all a, b along mode n, by explicit slicing."""
    r = g.shape[n]
    out = np.zeros((r, r))
    for a in range(r):
        sa = np.take(g, a, axis=n)
        for b in range(r):
            out[a, b] = float(np.sum(sa * np.take(g, b, axis=n)))
    return out


def _order_ok(fn, core, facs, tol=1e-10):
    g, f, sig = fn(core, facs)
    x0 = einsum_reconstruct(core, facs)
    if np.linalg.norm(einsum_reconstruct(g, f) - x0) > tol * np.linalg.norm(x0):
        return False
    total = float(np.sum(core ** 2))
    for n in range(core.ndim):
        sg = _slice_gram(g, n)
        if np.max(np.abs(sg - np.diag(np.diag(sg)))) > tol * total:
            return False
        if np.max(np.abs(np.sqrt(np.maximum(np.diag(sg), 0)) - sig[n])) > tol * math.sqrt(total):
            return False
        if np.any(np.diff(sig[n]) > tol * math.sqrt(total)):
            return False
        if abs(float(np.sum(sig[n] ** 2)) - total) > tol * total:
            return False
        if np.linalg.norm(f[n].T @ f[n] - np.eye(f[n].shape[1]), 2) > tol:
            return False
    return True


@pytest.mark.parametrize("dims,ranks,seed", [((9, 8, 3, 6), (4, 5, 2, 3), 1), ((12, 10, 7), (6, 3, 5), 2),
                                             ((5, 6, 4, 3, 2), (3, 2, 4, 3, 2), 3)])
def test_order_core_all_orthogonal_and_reconstruction_unchanged(dims, ranks, seed):
    core, facs = _random_decomp(np.random.default_rng(seed), dims, ranks)
    assert _order_ok(codec_ref.order_core, core, facs)


def test_full_rank_ordered_core_is_the_hosvd_of_x():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((6, 5, 4))
    q = [np.linalg.qr(rng.standard_normal((s, s)))[0] for s in x.shape]
    core = x
    for n, u in enumerate(q):
        core = ttm(core, u.T, n)                  # X = core x_n Q_n
    g, f, sig = codec_ref.order_core(core, q)
    for n in range(3):
        sv = np.linalg.svd(loop_unfold(x, n), compute_uv=False)
        assert np.max(np.abs(sig[n] - sv)) <= 1e-12 * sv[0]


def test_superdiagonal_closed_form():
    rng = np.random.default_rng(5)
    d = np.array([0.5, 3.0, 1.5, 2.0])
    core = np.zeros((4, 4, 4))
    for i, v in enumerate(d):
        core[i, i, i] = v
    perm = np.array([2, 0, 3, 1])
    facs = []
    pcore = core[np.ix_(perm, perm, perm)]
    for s in (7, 6, 5):
        u = np.linalg.qr(rng.standard_normal((s, 4)))[0] * np.array([1, -1, 1, -1])
        facs.append(u)
    g, f, sig = codec_ref.order_core(pcore, facs)
    want = np.sort(d)[::-1]
    for n in range(3):
        assert np.max(np.abs(sig[n] - want)) <= 1e-13
    assert np.max(np.abs(np.abs(g) - np.einsum("i,ij,ik->ijk", want, np.eye(4), np.eye(4)))) <= 1e-13


def test_truncation_error_identity():
    core, facs = _random_decomp(np.random.default_rng(6), (10, 9, 8), (6, 5, 4))
    g, f, _ = codec_ref.order_core(core, facs)
    keep = (4, 3, 2)
    gk, fk = codec_ref.truncate(g, f, keep)
    x = einsum_reconstruct(g, f)
    xk = einsum_reconstruct(gk, fk)
    assert abs(float(np.sum((x - xk) ** 2)) - (float(np.sum(g ** 2)) - float(np.sum(gk ** 2)))) <= 1e-12 * float(
        np.sum(g ** 2))
    assert gk.shape == keep and all(u.shape[1] == k for u, k in zip(fk, keep))


def _quant_ok(fn, g, bits):
    codes, deq, step = fn(g, bits)
    g32 = np.asarray(g, dtype=np.float32)
    levels = 2 ** (bits - 1) - 1
    if codes.dtype != np.int32 or deq.dtype != np.float32:
        return False
    if np.any(np.abs(codes) > levels):
        return False
    if np.any(np.abs(g32.astype(np.float64) - deq.astype(np.float64)) > 0.5 * float(step) * (1 + 1e-6)):
        return False
    i = np.argmax(np.abs(g32))
    if abs(int(codes.flat[i])) != levels:
        return False
    if not np.array_equal(deq, (codes.astype(np.float32) * np.float32(step)).astype(np.float32)):
        return False
    return True


@pytest.mark.parametrize("bits", [2, 4, 8, 12])
def test_quantize_core_bounds(bits):
    g = (np.random.default_rng(bits).standard_normal((8, 7, 3, 5)) * 3.0).astype(np.float32)
    assert _quant_ok(codec_ref.quantize_core, g, bits)


def test_quantize_ties_to_even_and_distortion_identity():
    codes, deq, step = codec_ref.quantize_core(np.array([7.0, 0.5, 1.5, -2.5], dtype=np.float32), 4)
    assert step == np.float32(1.0)
    assert codes.tolist() == [7, 0, 2, -2]
    rng = np.random.default_rng(9)
    core, facs = _random_decomp(rng, (8, 7, 6), (4, 3, 3))
    codes, deq, step = codec_ref.quantize_core(core, 6)
    d1 = np.linalg.norm(einsum_reconstruct(core, facs) - einsum_reconstruct(deq.astype(np.float64), facs))
    d2 = np.linalg.norm(core - deq.astype(np.float64))
    assert abs(d1 - d2) <= 1e-12 * np.linalg.norm(core)
    z, dz, sz = codec_ref.quantize_core(np.zeros((3, 2)), 8)
    assert not np.any(z) and sz == 0.0


# ---------------------------------------------------------------- planted mistakes

def _mutant(old, new):
    src = inspect.getsource(codec_ref)
    assert src.count(old) == 1, old
    mod = types.ModuleType("codec_mutant")
    mod.__dict__["__name__"] = "oracle.codec_mutant"
    mod.__dict__["__package__"] = "oracle"
    exec(compile(src.replace(old, new), "codec_mutant", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("old,new,which", [
    ("order = np.argsort(lam)[::-1]", "order = np.argsort(lam)", "order"),          # ascending energies
    ("out = ttm(out, v.T, n)", "out = ttm(out, v, n)", "order"),                   # core rotated the wrong way
    ("facs = [np.asarray(u, dtype=np.float64) @ v", "facs = [np.asarray(u, dtype=np.float64) @ v.T", "order"),
    ("c = unfold(g, n) @ unfold(g, n).T", "c = unfold(g, (n + 1) % g.ndim) @ unfold(g, (n + 1) % g.ndim).T",
     "order"),
    ("q = np.rint(g / step).astype(np.float32)", "q = np.floor(g / step).astype(np.float32)", "quant"),
    ("levels = np.float32(2 ** (int(bits) - 1) - 1)", "levels = np.float32(2 ** int(bits) - 1)", "quant"),
])
def test_planted_mistakes_are_caught(old, new, which):
    rng = np.random.default_rng(21)
    core, facs = _random_decomp(rng, (7, 6, 5), (4, 3, 3))
    g = (rng.standard_normal((6, 5, 4)) * 2).astype(np.float32)
    assert _order_ok(codec_ref.order_core, core, facs) and _quant_ok(codec_ref.quantize_core, g, 5)
    mod = _mutant(old, new)
    try:
        ok = _order_ok(mod.order_core, core, facs) if which == "order" else _quant_ok(mod.quantize_core, g, 5)
    except Exception:
        ok = False
    assert not ok
