"""Pairwise-perturbation HOOI on the GPU against the oracle's (needs an MI355X).

Sec. III-B, eq. (9)-(13): after the ordinary sweeps settle, perturbation sweeps take each update's
tensor to first order around reference factors.  The GPU run is compared with oracle/pp_ref.py on the
same input: perturbation sweeps taken, fit, residual and core norm within 1e-5, the reconstruction within
1e-5 plus the subspace-iteration allowance, and the fit within 1e-5 of plain HOOI's.
"""

import numpy as np
import pytest

import oracle
from oracle import pp_ref
from allowances import si_allowance
from synth import make_exact_rank, make_stereo_stack, STACK_CONFIGS

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _host(res):
    return dict(core=res.core.cpu().numpy().astype(np.float64),
                factors=[u.cpu().numpy().astype(np.float64) for u in res.factors], fit=res.fit)


@pytest.mark.parametrize("name,pp_tol", [("stack_mini", 0.05), ("stack_mini_ipt", 0.05)])
def test_pp_matches_oracle(name, pp_tol):
    import paper_2104_04726_amd as tk
    c = STACK_CONFIGS[name]
    x32 = make_stereo_stack(c["H"], c["W"], c["E"], c["colorspace"], c["seed"])
    ranks, iters = c["ranks"], c["sweeps"]
    _say(f"{name}: {iters} sweeps, pp_tol {pp_tol}")
    with tk.Context(0, pp_tol=pp_tol) as ctx:
        res = ctx.decompose(_dev(x32), ranks, iters)
    o = pp_ref.hooi_pp(x32.astype(np.float64), ranks, iters, pp_tol)
    st = res.stats
    _say(f"  GPU: {st['pp_sweeps']} perturbation sweeps, {st['pp_refs']} reference point(s); oracle kinds {o.kinds}, "
         f"distances {['%.1e' % v for v in o.changes]}")
    # the switching decisions need not coincide: the GPU's one-step orthogonal iteration keeps turning
    # the directions next to the rank boundary for many sweeps (they are not determined by the data to
    # that precision), so its factors may leave the reference sooner than the oracle's exact ones
    assert st["pp_sweeps"] > 0 and st["pp_refs"] >= 1
    m = oracle.compare(_host(res), dict(core=o.core, factors=o.factors, fit=o.fit))
    tol = 1e-5 + si_allowance(o.spectra, x32.shape, ranks, 20 + iters)
    _say(f"  fit {m['fit']:.2e} rho {m['rho']:.2e} core {m['core_norm']:.2e} recon {m['recon']:.2e} (bound {tol:.2e})")
    assert m["fit"] <= 1e-5 and m["rho"] <= 1e-5 and m["core_norm"] <= 1e-5, m
    assert m["recon"] <= tol
    assert max(m["orth"]) <= 1e-5
    plain = oracle.hooi(x32.astype(np.float64), ranks, iters)
    assert abs(res.fit - plain.fits[-1]) <= 1e-5
    # the returned fit is the exact one of the returned factors
    nx2 = float(np.sum(x32.astype(np.float64) ** 2))
    g = _host(res)["core"]
    assert abs(res.fit - (1.0 - np.sqrt(max(nx2 - float(np.sum(g * g)), 0.0)) / np.sqrt(nx2))) <= 1e-5


def test_pp_unsupported_cases():
    import paper_2104_04726_amd as tk
    x, _, _ = make_exact_rank((40, 36, 30), (6, 5, 4), 3, 1e-3)
    with tk.Context(0, pp_tol=0.1) as ctx:
        with pytest.raises(tk.TuckerError) as e:
            ctx.decompose(_dev(x), (6, 5, 4), 3)
        assert e.value.code == 5
        c = STACK_CONFIGS["stack_mini"]
        x32 = make_stereo_stack(c["H"], c["W"], c["E"], c["colorspace"], c["seed"])
        with pytest.raises(tk.TuckerError) as e:
            ctx.decompose(_dev(x32), c["ranks"], 3, tol=1e-9)
        assert e.value.code == 5
