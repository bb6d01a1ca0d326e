"""Step-level parity of the HIP kernels against FP64 definitions (needs an MI355X).

Each building block of a sweep is called through the C ABI and compared with its plain
definition evaluated in numpy float64 on the same (float32) inputs.  FP32 tolerances are the
standard a-priori bound of a length-K dot product accumulated in binary32,
|err| <= K u sum_k |a_k b_k| with u = 2^-24 (Higham, Thm 3.1), so they hold for any
accumulation order.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_2104_04726_amd as tk
    c = tk.Context(0)
    yield c
    c.close()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _ttm_ref(x, u, mode):
    y = np.tensordot(u.T.astype(np.float64), x.astype(np.float64), axes=([1], [mode]))
    return np.moveaxis(y, 0, mode)


def _ttm_abs(x, u, mode):
    y = np.tensordot(np.abs(u.T).astype(np.float64), np.abs(x).astype(np.float64), axes=([1], [mode]))
    return np.moveaxis(y, 0, mode)


def test_sumsq(ctx):
    rng = np.random.default_rng(0)
    for n in (1, 7, 1_000_003):
        x = rng.standard_normal(n).astype(np.float32)
        _say(f"sumsq n={n}")
        got = ctx.sumsq(_dev(x))
        ref = float(np.sum(x.astype(np.float64) ** 2))
        assert abs(got - ref) <= 1e-12 * ref


@pytest.mark.parametrize("shape,mode,r", [
    ((200, 300, 3, 14), 0, 72),       # mode-1 product, MFMA, ragged tiles
    ((200, 300, 3, 14), 1, 96),       # middle mode with folded columns (B = 42)
    ((37, 260, 24), 1, 130),          # B = 24, R > 128
    ((50, 130), 1, 70),               # last mode (B = 1): swapped operand form
    ((20, 30, 7), 1, 5),              # small-mode kernel
    ((9, 8, 7, 6), 3, 4),             # small, last mode
])
def test_ttm_matches_definition(ctx, shape, mode, r):
    rng = np.random.default_rng(hash((shape, mode)) % 2**32)
    x = rng.standard_normal(shape).astype(np.float32)
    u = rng.standard_normal((shape[mode], r)).astype(np.float32)
    _say(f"ttm shape={shape} mode={mode} r={r}")
    got = ctx.ttm(_dev(x), mode, _dev(u)).cpu().numpy().astype(np.float64)
    ref = _ttm_ref(x, u, mode)
    bound = shape[mode] * U32 * _ttm_abs(x, u, mode)
    assert got.shape == ref.shape
    assert np.all(np.abs(got - ref) <= bound + 1e-30)
    assert np.linalg.norm(got - ref) <= 1e-6 * np.linalg.norm(ref)


@pytest.mark.parametrize("shape,mode", [
    ((3, 200, 50), 1),                # MFMA Gram, folded k (B = 50)
    ((300, 70), 0),                   # s = 300, B = 70
    ((500, 130), 1),                  # B = 1 (last mode)
    ((2, 257, 3, 14), 1),             # ragged s, folded k of 42
    ((40, 20, 30), 1),                # small-mode Gram
    ((64, 48, 3, 6), 0),              # small, s = 64
    ((5, 300, 24), 1),                # k runs of 24: 16-byte vector loads
    ((200, 96), 0),                   # contiguous rows, vector loads, ragged tiles
    ((130, 7, 4), 0),                 # k = 28 not a multiple of the tile depth (vector tail)
    ((4, 150, 18), 1),                # k runs of 18: 8-byte vector loads
    ((3, 90, 42), 1),                 # k runs of 42 (pixel fibres): 8-byte vector loads
])
def test_gram_matches_definition(ctx, shape, mode):
    rng = np.random.default_rng(1 + mode)
    x = (rng.standard_normal(shape) + 0.5).astype(np.float32)   # non-zero mean like image data
    _say(f"gram shape={shape} mode={mode}")
    got = ctx.gram(_dev(x), mode).cpu().numpy().astype(np.float64)
    xn = np.moveaxis(x.astype(np.float64), mode, 0).reshape(shape[mode], -1)
    ref = xn @ xn.T
    K = xn.shape[1]
    bound = K * U32 * (np.abs(xn) @ np.abs(xn).T) + 2 * U32 * np.abs(ref)
    assert np.all(np.abs(got - ref) <= bound)
    # FP64 accumulation across k-tiles keeps the error near the output rounding
    assert np.linalg.norm(got - ref) <= 1e-6 * np.linalg.norm(ref)
    assert np.array_equal(got, got.T)


@pytest.mark.parametrize("rows,cols", [(1000, 96), (130, 17), (2000, 384)])
def test_gram_tn64(ctx, rows, cols):
    rng = np.random.default_rng(rows)
    z = rng.standard_normal((rows, cols)).astype(np.float32)
    _say(f"gram_tn64 {rows}x{cols}")
    w = ctx.gram_tn64(_dev(z)).cpu().numpy()
    z64 = z.astype(np.float64)
    ref = z64.T @ z64
    # products of binary32 values are exact in binary64; only FP64 accumulation error remains
    assert np.all(np.abs(w - ref) <= rows * 2.0 ** -53 * (np.abs(z64).T @ np.abs(z64)))


@pytest.mark.parametrize("n,cond", [(3, 10.0), (32, 1e3), (96, 1e6), (200, 1e4), (384, 1e8)])
def test_chol_inv(ctx, n, cond):
    import torch
    rng = np.random.default_rng(n)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    w = (q * np.geomspace(1.0, 1.0 / cond, n)) @ q.T
    w = (w + w.T) / 2
    _say(f"chol_inv n={n} cond={cond}")
    t = ctx.chol_inv(torch.from_numpy(w).cuda()).cpu().numpy()
    assert np.all(np.triu(t, 1) == 0.0)
    # T W T^T = I up to the conditioning of the scaled matrix
    d = 1.0 / np.sqrt(np.diag(w))
    ws = w * d[:, None] * d[None, :]
    kappa = np.linalg.cond(ws)
    e = t @ w @ t.T - np.eye(n)
    assert np.linalg.norm(e, 2) <= 50 * n * 2.0 ** -53 * kappa
    ref = np.linalg.inv(np.linalg.cholesky(ws)) * d[None, :]
    assert np.linalg.norm(t - ref) <= 50 * n * 2.0 ** -53 * kappa * np.linalg.norm(ref)


@pytest.mark.parametrize("rows,cols,cond", [
    (1000, 96, 1e4),
    (1080, 256, 1e6),
    (1920, 384, 1e6),
    (300, 100, 10.0),                 # ragged tile count
    (40, 40, 1e3),                    # square
])
def test_orthonormalize(ctx, rows, cols, cond):
    rng = np.random.default_rng(cols)
    q0, _ = np.linalg.qr(rng.standard_normal((rows, cols)))
    v0, _ = np.linalg.qr(rng.standard_normal((cols, cols)))
    sv = np.geomspace(1.0, 1.0 / cond, cols)
    z = ((q0 * sv) @ v0.T).astype(np.float32)
    _say(f"orthonormalize {rows}x{cols} cond={cond}")
    q = ctx.orthonormalize(_dev(z)).cpu().numpy().astype(np.float64)
    assert np.linalg.norm(q.T @ q - np.eye(cols), 2) <= 10 * np.sqrt(rows) * U32 * 2
    z64 = z.astype(np.float64)
    # same column space: the part of Z outside span(Q) is at rounding level
    resid = z64 - q @ (q.T @ z64)
    assert np.linalg.norm(resid) <= 1e-5 * np.linalg.norm(z64)


@pytest.mark.parametrize("n,r", [(3, 2), (14, 8), (33, 7), (64, 16)])
def test_sym_eig(ctx, n, r):
    rng = np.random.default_rng(n)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.linspace(10.0, 0.5, n)
    s = ((q * lam) @ q.T).astype(np.float32)
    s = (s + s.T) / 2
    _say(f"sym_eig n={n} r={r}")
    u, lam_gpu = ctx.sym_eig(_dev(s), r)
    u = u.cpu().numpy().astype(np.float64)
    lam_gpu = lam_gpu.cpu().numpy()
    ref = np.linalg.eigvalsh(s.astype(np.float64))[::-1]
    assert np.max(np.abs(lam_gpu - ref)) <= 1e-12 * np.max(np.abs(ref))
    w, v = np.linalg.eigh(s.astype(np.float64))
    vt = v[:, ::-1][:, :r]
    d = u - vt @ (vt.T @ u)
    assert np.linalg.norm(d, 2) <= 1e-6      # FP32 output rounding of an exact FP64 subspace
    assert np.linalg.norm(u.T @ u - np.eye(r), 2) <= 1e-6
