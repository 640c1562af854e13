"""fsi_residual_noalloc (scratch in the library's static device array) against
fsi_debug_residual (scratch in the problem's workspace): the same kernels on
the same inputs, so the residuals must agree bit for bit.  Two calls in a row
on one problem, the second with fewer slices, in 2d and 3d; and the size limit
of the static scratch.
"""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fsi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1907_01252_amd import fsi as f
    f.load()
    return f


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _pair(fsi, prob, B, U, Uo, t, k):
    nc = prob.n_dofs // prob.n_nodes
    Ra = torch.full((B, prob.n_nodes, nc), np.nan, dtype=torch.float64, device="cuda")
    Rb = torch.full_like(Ra, np.nan)
    prob.debug_residual(B, _dev(U[:B]), _dev(Uo[:B]), t[:B], k, Ra)
    code = prob.residual_noalloc(B, _dev(U[:B]), _dev(Uo[:B]), t[:B], k, Rb)
    torch.cuda.synchronize()
    return code, Ra.cpu().numpy(), Rb.cpu().numpy()


@pytest.mark.parametrize("name,level,Bs", [("c1", 1, (3, 2)), ("c5", 1, (2, 1)), ("c1q2", 0, (3, 2))])
def test_noalloc_residual_equals_workspace_residual(fsi, name, level, Bs):
    p = synth.workload(name, seed=5, level=level)
    _say("case: residual_noalloc vs debug_residual", name, "level", level, "B", Bs)
    prob = fsi.Problem(fsi.make_params(p, max_batch=max(Bs), batch_split=0))
    Bmax = max(Bs)
    U = np.stack([synth.random_state(p, 700 + b) for b in range(Bmax)])
    Uo = np.stack([synth.random_state(p, 800 + b) for b in range(Bmax)])
    t = [0.013, 0.31, 0.0731][:Bmax]
    k = p["k_fine"]
    prev = None
    for B in Bs:   # two calls in a row, the second with a smaller batch
        code, Ra, Rb = _pair(fsi, prob, B, U, Uo, t, k)
        assert code == fsi.FSI_OK
        assert np.all(np.isfinite(Rb))
        assert np.array_equal(Ra, Rb), np.abs(Ra - Rb).max()
        if prev is not None:
            # the smaller call recomputes its slices from scratch (no stale values kept)
            assert np.array_equal(prev[:B], Rb)
        prev = Rb
    prob.close()


def test_noalloc_residual_size_limit(fsi):
    """128x32 cells: 20 x 4096 doubles of element residuals per slice, so 51 slices fit in
    the 32 MiB scratch and 52 do not (FSI_ERR_ARG; the output is not written)."""
    p = synth.workload("c2", seed=0)
    _say("case: residual_noalloc size limit c2 mesh B=51/52")
    prob = fsi.Problem(fsi.make_params(p, max_batch=52, batch_split=0))
    nd = prob.n_dofs // prob.n_nodes
    U1 = synth.random_state(p, 11)
    U = np.broadcast_to(U1, (52,) + U1.shape)
    t = [0.05] * 52
    k = p["k_fine"]
    R = torch.full((52, prob.n_nodes, nd), -7.0, dtype=torch.float64, device="cuda")
    code = prob.residual_noalloc(52, _dev(U), _dev(U), t, k, R, raise_on_error=False)
    assert code == fsi.FSI_ERR_ARG
    assert bool((R == -7.0).all())
    code, Ra, Rb = _pair(fsi, prob, 51, U, U, t, k)
    assert code == fsi.FSI_OK
    assert np.array_equal(Ra, Rb)
    prob.close()
