"""Failure handling of the library on the GPU, forced from the host (needs an MI355X).

* A wait of the Cholesky task graph that gives up (its bound set to one sleep step through
  tucker_options.wait_spin_limit) is reported as TUCKER_ERR_DEVICE with a message, by the
  step-level entry points and by a whole decomposition; every kernel still finishes normally,
  and a context with the default bound then computes the same problem correctly.
* A rank-deficient input to CholeskyQR (exactly repeated columns) drives pivots below the
  breakdown threshold: they are shifted and counted, and the shifted CholeskyQR3 still returns
  an orthonormal basis whose span contains the input (the orthogonalisation of orthogonal
  iteration, the text after eq. (8)).
"""

import numpy as np
import pytest

from synth import make_exact_rank

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _say(msg):
    print(msg, flush=True)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    w = (q * np.geomspace(1.0, 1e-4, n)) @ q.T
    return (w + w.T) / 2


def test_chol_wait_timeout_is_a_device_error():
    import torch
    import paper_2104_04726_amd as tk
    w = _spd(384, 3)
    _say("chol_inv n=384 with a one-step wait bound")
    with tk.Context(0, wait_spin_limit=1) as ctx:
        with pytest.raises(tk.TuckerError) as ei:
            ctx.chol_inv(torch.from_numpy(w).cuda())
        assert ei.value.code == 3
        assert "wait gave up" in str(ei.value)
        assert ctx.stats()["wait_timeouts"] == 1
    _say("chol_inv n=384 with the default bound")
    with tk.Context(0) as ctx:
        t = ctx.chol_inv(torch.from_numpy(w).cuda()).cpu().numpy()
        assert ctx.stats()["wait_timeouts"] == 0
    d = 1.0 / np.sqrt(np.diag(w))
    ref = np.linalg.inv(np.linalg.cholesky(w * d[:, None] * d[None, :])) * d[None, :]
    assert np.linalg.norm(t - ref) <= 1e-9 * np.linalg.norm(ref)


def test_orthonormalize_wait_timeout_is_a_device_error():
    import paper_2104_04726_amd as tk
    z = np.random.default_rng(4).standard_normal((1000, 200)).astype(np.float32)
    _say("orthonormalize 1000x200 with a one-step wait bound")
    with tk.Context(0, wait_spin_limit=1) as ctx:
        with pytest.raises(tk.TuckerError) as ei:
            ctx.orthonormalize(_dev(z))
        assert ei.value.code == 3


def test_decompose_wait_timeout_is_a_device_error():
    import paper_2104_04726_amd as tk
    x, _, _ = make_exact_rank((300, 200, 3, 6), (80, 70, 3, 4), seed=9, noise_rel=1e-3)
    x32 = x.astype(np.float32)
    _say("decompose 300x200x3x6 (ranks 80/70: two Cholesky tile columns) with a one-step wait bound")
    with tk.Context(0, wait_spin_limit=1) as ctx:
        with pytest.raises(tk.TuckerError) as ei:
            ctx.decompose(_dev(x32), (80, 70, 3, 4), 2)
        assert ei.value.code == 3
        assert "wait gave up" in str(ei.value)
        assert ctx.stats()["wait_timeouts"] >= 1
    _say("the same decomposition with the default bound")
    with tk.Context(0) as ctx:
        res = ctx.decompose(_dev(x32), (80, 70, 3, 4), 2)
        assert ctx.stats()["wait_timeouts"] == 0
    assert 0.99 < res.fit <= 1.0


def test_orthonormalize_rank_deficient_shifts_and_stays_orthonormal():
    import paper_2104_04726_amd as tk
    rng = np.random.default_rng(12)
    rows, cols = 1080, 256
    z = rng.standard_normal((rows, cols)).astype(np.float32)
    z[:, 200:] = z[:, :56]                      # exact rank 200
    _say("orthonormalize 1080x256 of rank 200")
    with tk.Context(0) as ctx:
        q = ctx.orthonormalize(_dev(z)).cpu().numpy().astype(np.float64)
        shifts = ctx.stats()["chol_shifts"]
    _say(f"  pivot shifts {shifts}")
    assert shifts > 0
    assert np.all(np.isfinite(q))
    assert np.linalg.norm(q.T @ q - np.eye(cols), 2) <= 10 * np.sqrt(rows) * U32 * 2
    z64 = z.astype(np.float64)
    assert np.linalg.norm(z64 - q @ (q.T @ z64)) <= 1e-5 * np.linalg.norm(z64)
