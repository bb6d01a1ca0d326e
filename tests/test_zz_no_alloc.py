"""The allocation-free variant tucker_chol_inv_noalloc against tucker_chol_inv (needs an MI355X).

Both run the same task-graph Cholesky kernels; the variant keeps its scratch in a fixed per-GPU
device array instead of the context's workspace.  Two calls in a row (the second smaller, so that
the scratch holds the first call's leftovers) must each equal the allocating entry point bit for
bit and satisfy T W T^T = I; sizes above the scratch limit are rejected.
"""

import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _spd(n, cond, seed):
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    w = (q * np.geomspace(1.0, 1.0 / cond, n)) @ q.T
    return (w + w.T) / 2


def test_noalloc_chol_inv_equals_allocating_entry_point():
    import torch
    import paper_2104_04726_amd as tk
    from paper_2104_04726_amd import _lib
    lib = _lib.lib()
    with tk.Context(0) as ctx:
        for n, cond in ((448, 1e6), (200, 1e3)):
            print(f"chol_inv_noalloc n={n}", flush=True)
            w = torch.from_numpy(_spd(n, cond, n)).cuda()
            t_ref = torch.empty_like(w)
            t_new = torch.full_like(w, float("nan"))
            assert lib.tucker_chol_inv(ctx._h, C.c_void_p(w.data_ptr()), n, C.c_void_p(t_ref.data_ptr())) == 0
            assert lib.tucker_chol_inv_noalloc(ctx._h, C.c_void_p(w.data_ptr()), n,
                                               C.c_void_p(t_new.data_ptr())) == 0
            torch.cuda.synchronize()
            a, b = t_ref.cpu().numpy(), t_new.cpu().numpy()
            assert np.array_equal(a, b)
            wn = w.cpu().numpy()
            d = 1.0 / np.sqrt(np.diag(wn))
            kappa = np.linalg.cond(wn * d[:, None] * d[None, :])
            assert np.linalg.norm(b @ wn @ b.T - np.eye(n), 2) <= 50 * n * 2.0 ** -53 * kappa
        big = torch.eye(513, dtype=torch.float64, device="cuda")
        out = torch.empty_like(big)
        code = lib.tucker_chol_inv_noalloc(ctx._h, C.c_void_p(big.data_ptr()), 513, C.c_void_p(out.data_ptr()))
        assert code == _lib.ERR_INVALID_ARG
        assert b"scratch limit" in lib.tucker_last_error(ctx._h)
