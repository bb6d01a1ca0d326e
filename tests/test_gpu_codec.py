"""The codec hand-off on the GPU (needs an MI355X): the FP64 block-Jacobi eigensolver, the ordered
(all-orthogonal) core, and the uniform core quantiser, against oracle/codec_ref.py and numpy.

* Eigensolver (n up to 1024): eigenvalues within 50 n u of LAPACK's relative to the largest, leading
  eigenvectors spanning LAPACK's subspace (FP32 output rounding) on gapped spectra.
* Ordered core: on the same FP32 core and factors, the mode singular values equal the oracle's to
  1e-6 (relative to sigma_1), the GPU core is all-orthogonal to FP32 rounding, and the reconstruction is
  unchanged (rotation-invariant core-space difference <= 1e-6).
* Quantiser: codes, dequantised values and the step are bit-for-bit the oracle's (both take every
  rounding decision in binary32 on the same core values).
"""

import numpy as np
import pytest

import oracle
from oracle import codec_ref
from synth import make_stereo_stack, STACK_CONFIGS

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("n,r", [(100, 10), (384, 384), (700, 64), (1024, 200)])
def test_sym_eig_blocked_matches_lapack(ctx, n, r):
    rng = np.random.default_rng(n)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.geomspace(1.0, 1e-6, n) * (1 + 0.1 * rng.random(n))
    s = ((q * lam) @ q.T).astype(np.float32)
    s = (s + s.T) / 2
    _say(f"sym_eig n={n} r={r}")
    u, lg = ctx.sym_eig(_dev(s), r)
    u = u.cpu().numpy().astype(np.float64)
    lg = lg.cpu().numpy()
    w, v = np.linalg.eigh(s.astype(np.float64))
    ref = w[::-1]
    # backward-stable orthogonal transformations: |lam~ - lam| <= c n u ||A||_2 (Weyl), with c = 50
    # covering the sweeps of accumulated rotations (measured 1.1e-12 .. 3.4e-12 at n = 384 .. 1024)
    assert np.max(np.abs(lg - ref)) <= 50 * n * 2.0 ** -53 * ref[0]
    vt = v[:, ::-1][:, :r]
    assert np.linalg.norm(u.T @ u - np.eye(r), 2) <= 1e-5
    if r < n:
        gap = (ref[r - 1] - ref[r]) / ref[0]
        assert np.linalg.norm(u - vt @ (vt.T @ u), 2) <= 1e-6 + 1e-12 / gap


@pytest.mark.parametrize("n", [96, 448])
def test_sym_eig_blocked_repeated_and_graded_eigenvalues(ctx, n):
    """Exactly repeated eigenvalues (clusters of 8), a zero block and a graded tail: the
    eigenvalues to the backward-stable bound, the eigenvectors orthonormal, and the residual
    ||S U - U diag(lam)|| small against ||S||.  Within a cluster any orthonormal basis is correct, so
    the subspaces, not the vectors, are compared through the residual."""
    rng = np.random.default_rng(7 + n)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.repeat(np.geomspace(1.0, 1e-5, n // 8), 8)[:n]
    lam[-8:] = 0.0
    s = ((q * lam) @ q.T).astype(np.float32)
    s = (s + s.T) / 2
    _say(f"sym_eig repeated n={n}")
    u, lg = ctx.sym_eig(_dev(s), n)
    u = u.cpu().numpy().astype(np.float64)
    lg = lg.cpu().numpy()
    s64 = s.astype(np.float64)
    ref = np.linalg.eigvalsh(s64)[::-1]
    assert np.max(np.abs(lg - ref)) <= 50 * n * 2.0 ** -53 * ref[0]
    assert np.linalg.norm(u.T @ u - np.eye(n), 2) <= 1e-5                  # FP32 vectors
    assert np.linalg.norm(s64 @ u - u * lg, 2) <= 1e-5 * ref[0]


def _slice_offdiag(g, n):
    gn = np.moveaxis(g, n, 0).reshape(g.shape[n], -1)
    c = gn @ gn.T
    return float(np.max(np.abs(c - np.diag(np.diag(c))))), np.sqrt(np.maximum(np.diag(c), 0))


@pytest.mark.parametrize("name,iters", [("stack_mini", 5), ("stack1080", 3)])
def test_order_core_matches_oracle(ctx, name, iters):
    import torch
    c = STACK_CONFIGS[name]
    x32 = make_stereo_stack(c["H"], c["W"], c["E"], c["colorspace"], c["seed"])
    ranks = c["ranks"]
    _say(f"decompose {name}, {iters} sweeps, then order the core")
    res = ctx.decompose(_dev(x32), ranks, iters)
    g_out, f_out, sig = ctx.order_core(res.core, res.factors)
    torch.cuda.synchronize()
    core = res.core.cpu().numpy().astype(np.float64)
    facs = [u.cpu().numpy().astype(np.float64) for u in res.factors]
    g2 = g_out.cpu().numpy().astype(np.float64)
    f2 = [u.cpu().numpy().astype(np.float64) for u in f_out]
    og, of, osig = codec_ref.order_core(core, facs)
    total = float(np.sum(core ** 2))
    for n in range(len(ranks)):
        s_gpu = sig[n].cpu().numpy()
        assert np.max(np.abs(s_gpu - osig[n])) <= 1e-6 * osig[n][0], n
        off, norms = _slice_offdiag(g2, n)
        assert off <= 1e-5 * total, (n, off / total)
        assert np.max(np.abs(norms - osig[n])) <= 1e-5 * osig[n][0]
        assert np.linalg.norm(f2[n].T @ f2[n] - np.eye(ranks[n]), 2) <= 1e-5
    d = oracle.recon_diff(g2, f2, core, facs)
    d_or = oracle.recon_diff(g2, f2, og, of)
    _say(f"  reconstruction moved by {d:.2e}; against the oracle's ordered decomposition {d_or:.2e}")
    assert d <= 1e-6 and d_or <= 1e-6


@pytest.mark.parametrize("bits,keep", [(8, (20, 30, 3, 5)), (4, (48, 64, 3, 8)), (12, (7, 9, 2, 8))])
def test_quantize_core_bit_exact(ctx, bits, keep):
    rng = np.random.default_rng(bits)
    core = (rng.standard_normal((48, 64, 3, 8)) * np.exp(rng.uniform(-3, 3, (48, 64, 3, 8)))).astype(np.float32)
    core[0, 0, 0, 0] = 0.0
    _say(f"quantize_core bits={bits} keep={keep}")
    codes, deq, step = ctx.quantize_core(_dev(core), keep, bits)
    kept, _ = codec_ref.truncate(core, [np.zeros((1, r)) for r in core.shape], keep)
    rc, rd, rs = codec_ref.quantize_core(kept, bits)
    assert np.float32(step).view(np.uint32) == np.float32(rs).view(np.uint32)
    assert np.array_equal(codes.cpu().numpy(), rc)
    assert np.array_equal(deq.cpu().numpy().view(np.uint32), rd.view(np.uint32))


def test_quantize_core_zero_and_invalid(ctx):
    import paper_2104_04726_amd as tk
    z = np.zeros((4, 3, 2), dtype=np.float32)
    codes, deq, step = ctx.quantize_core(_dev(z), (4, 3, 2), 8)
    assert step == 0.0 and not codes.cpu().numpy().any() and not deq.cpu().numpy().any()
    with pytest.raises(tk.TuckerError) as e:
        ctx.quantize_core(_dev(z), (5, 3, 2), 8)
    assert e.value.code == 1
    with pytest.raises(tk.TuckerError) as e:
        ctx.quantize_core(_dev(z), (4, 3, 2), 1)
    assert e.value.code == 1
