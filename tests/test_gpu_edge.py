"""Edge cases of the propagators through the C ABI on the GPU.

- Sizes out of range (B = 0, B above max_batch, no steps, a slice length that
  is zero, negative or NaN) are refused with FSI_ERR_ARG, and U_out is left as
  it was.
- A non-finite input state is refused with FSI_ERR_NONFINITE before any work:
  U_out is left as it was and the slice status names the bad slice.
- U_in and U_out may alias (include/fsi.h): the in-place call gives the
  out-of-place result bit for bit.
- The degenerate case of the method: with no inflow, the fluid at rest and
  the structure undeformed, every step's residual vanishes (no velocity,
  pressure, displacement or boundary data), so the zero state is a fixed point
  of the scheme. Both precisions must return exactly zero after one Newton
  iteration per step; a zero right-hand side in FGMRES must not divide by its
  zero norm.
- A batch that is not full (B = 2 of max_batch 4, with different start times)
  gives the results of the full batch's first two slices.
- Concurrent slice groups (batch_split 2 and 3, B = 5 of max_batch 5, so the
  groups are uneven) give the single batch's states bit for bit and the same
  per-slice Newton and Krylov counts; an infinite value in the last group's input stops
  the call before any group writes U_out.
"""
import sys

import numpy as np
import pytest

import synth
from oracle.residual import Discretization

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


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_size_errors_leave_output_alone(fsi):
    p = synth.workload("c1", seed=2)
    _say("case: argument errors on a live c1 problem, max_batch 2")
    prob = fsi.Problem(fsi.make_params(p, precision="fp64", max_batch=2))
    U_in = torch.zeros(3, prob.n_nodes, 5, dtype=torch.float64, device="cuda")
    U_out = torch.full_like(U_in, 7.0)
    dl = p["slice_len"]
    for B, m, sl in ((0, 2, dl), (3, 2, dl), (1, 0, dl), (1, -1, dl), (1, 2, 0.0), (1, 2, -dl), (1, 2, float("nan"))):
        for fn in (prob.fine_propagate, prob.coarse_propagate):
            code, _ = fn(B, [0.0] * B, sl, m, U_in, U_out, raise_on_error=False)
            assert code == fsi.FSI_ERR_ARG, (fn.__name__, B, m, sl, code)
    assert bool((_host(U_out) == 7.0).all())
    prob.close()


def test_nonfinite_input_is_refused_before_any_work(fsi):
    p = synth.workload("c1", seed=2)
    _say("case: NaN in slice 1 of a c1 batch of 2")
    D = Discretization(p)
    prob = fsi.Problem(fsi.make_params(p, precision="fp64", max_batch=2))
    U = np.stack([D.apply_dirichlet(synth.smooth_state(p, 40 + l), 0.0) for l in range(2)])
    U[1, 17, 3] = np.nan
    U_out = torch.full((2, prob.n_nodes, 5), 7.0, dtype=torch.float64, device="cuda")
    code, st = prob.fine_propagate(2, [0.0, 0.0], p["slice_len"], 2, _dev(U), U_out, raise_on_error=False)
    assert code == fsi.FSI_ERR_NONFINITE
    assert list(st.slice_status[:2]) == [fsi.FSI_OK, fsi.FSI_ERR_NONFINITE]
    assert bool((_host(U_out) == 7.0).all())
    prob.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_in_place_equals_out_of_place(fsi, precision):
    p = synth.workload("c1", seed=3)
    _say("case: aliased U_in/U_out, c1 B=2,", precision)
    D = Discretization(p)
    dl = p["slice_len"]
    t0 = [0.0, dl]
    U = np.stack([D.apply_dirichlet(synth.smooth_state(p, 60 + l), t0[l]) for l in range(2)])
    prob = fsi.Problem(fsi.make_params(p, precision=precision, max_batch=2))
    out = torch.zeros(2, prob.n_nodes, 5, dtype=torch.float64, device="cuda")
    prob.fine_propagate(2, t0, dl, 3, _dev(U), out)
    inplace = _dev(U)
    prob.fine_propagate(2, t0, dl, 3, inplace, inplace)
    a, b = _host(out), _host(inplace)
    assert np.array_equal(a, b), np.abs(a - b).max()
    prob.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_rest_state_is_a_fixed_point(fsi, precision):
    p = synth.workload("c1", seed=0, inflow_peak=0.0)
    m = 3
    _say("case: zero inflow, zero state, c1 B=2,", precision)
    prob = fsi.Problem(fsi.make_params(p, precision=precision, max_batch=2))
    U = torch.zeros(2, prob.n_nodes, 5, dtype=torch.float64, device="cuda")
    prob.initial_state(U[0])
    prob.initial_state(U[1])
    assert not bool(U.any())
    out = torch.full_like(U, 7.0)
    code, st = prob.fine_propagate(2, [0.0, p["slice_len"]], p["slice_len"], m, U, out)
    assert code == fsi.FSI_OK
    assert not bool(out.any()), _host(out).max()
    assert list(st.newton_its[:2]) == [m, m] and list(st.krylov_its[:2]) == [0, 0], (list(st.newton_its[:2]),
                                                                                     list(st.krylov_its[:2]))
    code, st = prob.coarse_propagate(2, [0.0, p["slice_len"]], p["slice_len"], 1, U, out)
    assert code == fsi.FSI_OK and not bool(out.any())
    prob.close()


def test_partial_batch_equals_full_batch(fsi):
    p = synth.workload("c1", seed=4)
    _say("case: c1 B=2 of max_batch 4 vs the full batch")
    D = Discretization(p)
    dl = p["slice_len"]
    t0 = [l * dl for l in range(4)]
    U = np.stack([D.apply_dirichlet(synth.smooth_state(p, 80 + l), t0[l]) for l in range(4)])
    prob = fsi.Problem(fsi.make_params(p, precision="fp64", max_batch=4))
    full = torch.zeros(4, prob.n_nodes, 5, dtype=torch.float64, device="cuda")
    prob.fine_propagate(4, t0, dl, 2, _dev(U), full)
    part = torch.zeros(2, prob.n_nodes, 5, dtype=torch.float64, device="cuda")
    prob.fine_propagate(2, t0[:2], dl, 2, _dev(U[:2]), part)
    a, b = _host(part), _host(full)[:2]
    err = np.abs(a - b).max() / np.abs(b).max()
    assert err <= 1e-12, err
    prob.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_concurrent_groups_equal_one_batch(fsi, precision):
    p = synth.workload("c1", seed=5)
    _say("case: c1 B=5, batch_split 0 vs 2 vs 3,", precision)
    D = Discretization(p)
    dl = p["slice_len"]
    t0 = [l * dl for l in range(5)]
    U = np.stack([D.apply_dirichlet(synth.smooth_state(p, 100 + l), t0[l]) for l in range(5)])
    res = {}
    for split in (0, 2, 3):
        prob = fsi.Problem(fsi.make_params(p, precision=precision, max_batch=5, batch_split=split))
        out = torch.zeros(5, prob.n_nodes, 5, dtype=torch.float64, device="cuda")
        code, st = prob.fine_propagate(5, t0, dl, 3, _dev(U), out)
        res[split] = (_host(out), list(st.newton_its[:5]), list(st.krylov_its[:5]), st.newton_total, st.krylov_total)
        if split == 3:
            bad = U.copy()
            bad[4, 3, 0] = np.inf
            sentinel = torch.full_like(out, 7.0)
            code, st = prob.fine_propagate(5, t0, dl, 3, _dev(bad), sentinel, raise_on_error=False)
            assert code == fsi.FSI_ERR_NONFINITE and list(st.slice_status[:5]) == [0, 0, 0, 0, fsi.FSI_ERR_NONFINITE]
            assert bool((_host(sentinel) == 7.0).all())
        prob.close()
    for split in (2, 3):
        assert np.array_equal(res[split][0], res[0][0]), (split, np.abs(res[split][0] - res[0][0]).max())
        assert res[split][1:] == res[0][1:], (split, res[split][1:], res[0][1:])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_linear_failure_is_reported_per_slice(fsi, precision):
    """With one FGMRES iteration per linear solve no solve reaches its tolerance: Newton must
    not accept any update from such a solve, so every slice ends with FSI_ERR_LINEAR (the
    call returns it) instead of a state that only looks converged."""
    p = synth.workload("c1", seed=3)
    _say("case: linear failure c1 B=2 gmres_maxit=1", precision)
    prob = fsi.Problem(fsi.make_params(p, precision=precision, max_batch=2, gmres_maxit=1, newton_maxit=4,
                                       batch_split=0))
    U0 = torch.zeros(2, prob.n_nodes, 5, dtype=torch.float64, device="cuda")
    prob.initial_state(U0[0])
    prob.initial_state(U0[1])
    k = p["k_fine"]
    out = torch.zeros_like(U0)
    code, st = prob.fine_propagate(2, [0.05, 0.2], 2 * k, 2, U0, out, raise_on_error=False)
    assert code == fsi.FSI_ERR_LINEAR, code
    assert [st.slice_status[b] for b in range(2)] == [fsi.FSI_ERR_LINEAR] * 2
    assert all(st.newton_its[b] == 4 for b in range(2)), [st.newton_its[b] for b in range(2)]
    prob.close()


def test_stage_times_are_reported(fsi):
    """stats.stage_ms[0..3] (residual, Jacobian and multigrid setup, linear solve, update and
    tests) are the HIP-event times of the Newton stages: positive, and together not more
    than the call's wall time; the linear solve dominates."""
    p = synth.workload("c1", seed=1)
    _say("case: stage times c1 B=2 m=3")
    prob = fsi.Problem(fsi.make_params(p, precision="fp64", max_batch=2, batch_split=0))
    U0 = torch.zeros(2, prob.n_nodes, 5, dtype=torch.float64, device="cuda")
    prob.initial_state(U0[0])
    prob.initial_state(U0[1])
    k = p["k_fine"]
    out = torch.zeros_like(U0)
    prob.fine_propagate(2, [0.0, 0.03], 3 * k, 3, U0, out)   # warm-up (graph capture)
    code, st = prob.fine_propagate(2, [0.0, 0.03], 3 * k, 3, U0, out)
    ms = [st.stage_ms[i] for i in range(5)]
    _say("stage ms", ms)
    assert code == fsi.FSI_OK
    assert all(m > 0.0 for m in ms[:4]), ms
    assert sum(ms[:4]) <= 1.05 * ms[4], ms
    assert ms[2] == max(ms[:4]), ms
    prob.close()
