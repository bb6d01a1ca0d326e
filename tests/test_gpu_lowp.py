"""Parity of the reduced-precision sweep variants (BF16 / FP16 / FP8-e4m3) (needs an MI355X).

* Storage: the GPU encode/decode round trip equals the reference encodings of
  oracle/quant_ref.py bit for bit (including the FP8 slice scales).
* Contractions: products and Grams on the 16-/8-bit matrix cores, compared with their FP64
  definition evaluated on the quantized operands.  Products of two 16-bit (or 8-bit) values are
  exact in binary32, so the FP32 accumulation error obeys |err| <= K u sum_k |a_k b_k|
  (u = 2^-24, Higham Thm 3.1); the FP8 instruction's block accumulation is coarser than binary32
  and gets 2^-14 sum_k |a_k b_k| on top.
* End to end: the reduced-precision sweeps followed by one FP32 refinement sweep reproduce the
  FP64 oracle's fit and core norm to 1e-3 and its reconstruction to 1e-3 (relative, rotation
  invariant), plus one boundary direction pair for each mode whose rank boundary is degenerate.
"""

import numpy as np
import pytest

import oracle
from oracle import quant_ref
from synth import make_stereo_stack, STACK_CONFIGS

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
PRECS = ["bf16", "fp16", "fp8"]


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


def _wide(rng, shape):
    """Values over many binades, with exact zeros and tiny entries."""
    x = rng.standard_normal(shape) * np.exp(rng.uniform(-6, 3, shape))
    x.flat[::97] = 0.0
    x.flat[5::131] = 1e-30
    return x.astype(np.float32)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("rows,L", [(1000, 42), (37, 30), (1, 7)])
def test_quantize_bit_exact(ctx, prec, rows, L):
    rng = np.random.default_rng(rows * 7 + L)
    x = _wide(rng, (rows, L))
    _say(f"quantize {prec} {rows}x{L}")
    got, sc = ctx.quantize(_dev(x), prec)
    ref, rsc = quant_ref.quantize(x, prec)
    got = got.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    if prec == "fp8":
        assert np.array_equal(sc.cpu().numpy().view(np.uint32), rsc.view(np.uint32))


def _qt(x, prec):
    """Quantized tensor as the product sees it (FP8: per index of the last mode)."""
    last = x.shape[-1]
    q, _ = quant_ref.quantize(x.reshape(-1, last), prec)
    return q.reshape(x.shape)


def _qu(u, prec):
    q, _ = quant_ref.quantize(u, prec)    # FP8: per column of U
    return q


def _ttm64(x, u, mode):
    y = np.tensordot(u.T.astype(np.float64), x.astype(np.float64), axes=([1], [mode]))
    return np.moveaxis(y, 0, mode)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape,mode,r", [
    ((200, 300, 3, 14), 0, 72),       # first mode, many columns
    ((200, 300, 3, 14), 1, 96),       # middle mode, folded columns of 42
    ((37, 260, 24), 1, 130),          # R > 128, ragged tiles
    ((64, 96, 3, 8), 1, 40),          # column folding of 24 (vector loads)
    ((50, 130), 1, 70),               # last mode (not for FP8)
])
def test_ttm_lowp(ctx, prec, shape, mode, r):
    if prec == "fp8" and mode == len(shape) - 1:
        pytest.skip("FP8 scales the last mode; the product over it is not provided")
    rng = np.random.default_rng(hash((shape, mode, prec)) % 2**32)
    x = (rng.standard_normal(shape) + 0.3).astype(np.float32)
    u = rng.standard_normal((shape[mode], r)).astype(np.float32)
    _say(f"ttm_lowp {prec} shape={shape} mode={mode} r={r}")
    got = ctx.ttm_lowp(_dev(x), mode, _dev(u), prec).cpu().numpy().astype(np.float64)
    xq, uq = _qt(x, prec), _qu(u, prec)
    ref = _ttm64(xq, uq, mode)
    absr = _ttm64(np.abs(xq), np.abs(uq), mode)
    # FP8: the matrix instruction sums each 32-product block with less than binary32 precision
    # (measured up to 2e-5 sum|ab| at K = 96..200, the 16-bit types stay within K u); the bound
    # adds 2^-14 sum|ab|, far below the 2^-4 quantization step of the format itself
    extra = 2.0 ** -14 * absr if prec == "fp8" else 0.0
    assert np.all(np.abs(got - ref) <= shape[mode] * U32 * absr + extra + 1e-30)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("shape,mode", [
    ((3, 200, 56), 1),                # folded k (B = 56)
    ((300, 72), 0),                   # k contiguous rows
    ((500, 130), 1),                  # last mode (B = 1)
    ((2, 257, 3, 14), 1),             # ragged s, folded k of 42
    ((1100, 24), 0),                  # s > 1024: many lower-triangle tiles
])
def test_gram_lowp(ctx, prec, shape, mode):
    rng = np.random.default_rng(11 + mode)
    x = (rng.standard_normal(shape) + 0.5).astype(np.float32)
    _say(f"gram_lowp {prec} shape={shape} mode={mode}")
    got = ctx.gram_lowp(_dev(x), mode, prec).cpu().numpy().astype(np.float64)
    xq = quant_ref.quantize(x.reshape(-1, 1), prec)[0].reshape(shape).astype(np.float64)
    xn = np.moveaxis(xq, mode, 0).reshape(shape[mode], -1)
    ref = xn @ xn.T
    K = xn.shape[1]
    bound = K * U32 * (np.abs(xn) @ np.abs(xn).T) + 2 * U32 * np.abs(ref)
    assert np.all(np.abs(got - ref) <= bound)
    assert np.array_equal(got, got.T)


def _degenerate_allowance(o, ranks):
    """Modes whose rank boundary is degenerate (gap factor g = lam_1 / (lam_R - lam_{R+1}) above
    1e8) do not determine the boundary directions: stationary points of equal fit may hold a
    different direction there.  Each such mode may move Xhat by one boundary direction pair,
    sqrt(2 lam_R / sum(lam)) relative; the second-order quantities (fit, core norm) stay binding."""
    extra = 0.0
    for n, r in enumerate(ranks):
        lam = o.spectra[n]
        if r < len(lam) and o.gap_factor(n, r) > 1e8:
            extra += float(np.sqrt(2.0 * max(lam[r - 1], 0.0) / np.sum(lam)))
    return extra


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", ["stack_mini", "stack_mini_ipt"])
def test_lowp_sweeps_then_refine_match_oracle(prec, name):
    import paper_2104_04726_amd as tk
    c = STACK_CONFIGS[name]
    x32 = make_stereo_stack(c["H"], c["W"], c["E"], c["colorspace"], c["seed"])
    ranks, iters = c["ranks"], c["sweeps"]
    _say(f"lowp {prec} {name}: {iters} sweeps + 1 FP32 refinement")
    ctx = tk.Context(0, precision=prec, refine_sweeps=1)
    try:
        res = ctx.decompose(_dev(x32), ranks, iters)
    finally:
        ctx.close()
    g = dict(core=res.core.cpu().numpy().astype(np.float64),
             factors=[u.cpu().numpy().astype(np.float64) for u in res.factors], fit=res.fit)
    assert res.sweeps == iters and res.stats["refine_sweeps"] == 1
    o = oracle.hooi(x32.astype(np.float64), ranks, iters + 1)
    m = oracle.compare(g, dict(core=o.core, factors=o.factors, fit=o.fits[-1]))
    tol = 1e-3 + _degenerate_allowance(o, ranks)
    _say(f"  metrics {m}  recon tol {tol:.3g}")
    assert m["recon"] <= tol, m
    assert m["fit"] <= 1e-3 and m["core_norm"] <= 1e-3, m
    assert max(m["orth"]) <= 1e-5, m
    # the per-sweep fit of the refinement sweep (||X||^2 - ||G||^2, FP32 core) tracks the oracle's;
    # during the reduced-precision sweeps that estimate carries the storage error amplified by the
    # cancellation in ||X||^2 - ||G||^2 (about 2^-8 / (2 (1 - fit))) and is only checked for range
    assert abs(res.stats["fit_gram"] - o.fits[-1]) <= 1e-4
    assert all(0.0 <= f <= 1.0 for f in res.fit_history)


def test_lowp_unsupported_shape():
    import paper_2104_04726_amd as tk
    ctx = tk.Context(0, precision="bf16")
    try:
        x = _dev(np.random.default_rng(0).standard_normal((40, 30, 20)))
        with pytest.raises(tk.TuckerError) as e:
            ctx.decompose(x, (5, 5, 5), 2)
        assert e.value.code == 5
    finally:
        ctx.close()


@pytest.mark.parametrize("prec", PRECS)
def test_lowp_tile_variants_bit_identical(ctx, prec):
    """The LDS stagings the autotuner chooses between (operation 3) leave every output element's sum
    and its order unchanged: each candidate's products and Grams equal the first's bit for bit, on
    shapes with interior tiles (unchecked loads) and ragged edge tiles."""
    import paper_2104_04726_amd as tk
    rng = np.random.default_rng(23)
    cases = [((520, 96, 3, 14), 0, 300), ((40, 530, 42), 1, 270), ((200, 300, 3, 14), 1, 130)]
    grams = [((300, 200), 0), ((2, 390, 42), 1)] if prec != "fp8" else []
    data = [(_dev((rng.standard_normal(s) + 0.2).astype(np.float32)), m,
             _dev(rng.standard_normal((s[m], r)).astype(np.float32))) for s, m, r in cases]
    gdata = [(_dev((rng.standard_normal(s) + 0.5).astype(np.float32)), m) for s, m in grams]
    outs = []
    try:
        for c in range(2):
            tk.autotune_force(3, c)
            _say(f"{prec}: tile variant {c}")
            outs.append([ctx.ttm_lowp(x, m, u, prec).cpu().numpy() for x, m, u in data] +
                        [ctx.gram_lowp(x, m, prec).cpu().numpy() for x, m in gdata])
    finally:
        tk.autotune_force(3, -1)
    for c in range(1, 2):
        for a, b in zip(outs[0], outs[c]):
            assert a.shape == b.shape and np.array_equal(a, b), (prec, c)


def test_lowp_decomposition_same_for_every_tile_variant():
    import paper_2104_04726_amd as tk
    c = STACK_CONFIGS["stack_mini"]
    x = _dev(make_stereo_stack(c["H"], c["W"], c["E"], c["colorspace"], c["seed"]))
    res = []
    try:
        for v in (0, 1):
            tk.autotune_force(3, v)
            with tk.Context(0, precision="bf16", refine_sweeps=1) as cx:
                r = cx.decompose(x, c["ranks"], 3)
            res.append((r.fit, r.core.cpu().numpy(), [u.cpu().numpy() for u in r.factors]))
    finally:
        tk.autotune_force(3, -1)
    assert res[0][0] == res[1][0]
    assert np.array_equal(res[0][1], res[1][1])
    for a, b in zip(res[0][2], res[1][2]):
        assert np.array_equal(a, b)
