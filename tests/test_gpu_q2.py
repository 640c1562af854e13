"""GPU parity of the biquadratic (Q2) cells of Section 2.2 through the C ABI (FP64 and
mixed precision).

The Q2 problem on level l has the nodes of the Q1 level l + 1 and nine per
cell; the library solves each Newton step with FGMRES on the exact Q2 Jacobian,
preconditioned by the Q1 multigrid V-cycle on the same nodes.  Compared with the
FP64 oracle's Q2 discretisation (oracle.residual with degree 2): the residual
and Jacobian products to 1e-12, fine propagation to 1e-10 (c1q2: 16x4 cells,
the 297 nodes of c1), batched against single-slice calls, and one step of a
sampled slice of the 32-slice c2q2 batch (64x16 cells, the 21,285 unknowns of
c2) in the launch configuration of a full sweep.  Mixed precision (FP32 Q2 product
and V-cycle inside the FP64 Newton loop): c1q2 against the oracle to 1e-6, and the
64-slice c3q2 batch (128x32 cells, the 83,525 unknowns of c3) against the FP64 Q2
path to 1e-6.
"""
import sys

import numpy as np
import pytest

import synth
from oracle.residual import Discretization
from oracle import propagate as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FIELDS = {"v": slice(0, 2), "u": slice(2, 4), "p": slice(4, 5)}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def field_rel(a, b, norm="max"):
    out = {}
    for k, sl in FIELDS.items():
        x, y = a[..., sl], b[..., sl]
        if norm == "max":
            out[k] = np.abs(x - y).max() / max(np.abs(y).max(), 1e-300)
        else:
            out[k] = np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300)
    return out


@pytest.fixture(scope="module")
def fsi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1907_01252_amd import fsi as f
    f.load()
    return f


@pytest.fixture(scope="module")
def c1q2(fsi):
    p = synth.workload("c1q2", seed=1)
    prob = fsi.Problem(fsi.make_params(p, precision="fp64", max_batch=4, batch_split=0))
    return p, prob, Discretization(p)


def test_sizes_q2(fsi, c1q2):
    p, prob, D = c1q2
    assert prob.n_nodes == D.mesh.n_nodes == 33 * 9


def test_residual_parity_q2(fsi, c1q2):
    p, prob, D = c1q2
    _say("case: Q2 residual parity c1q2 B=3")
    B = 3
    U = np.stack([synth.random_state(p, 100 + b) for b in range(B)])
    Uo = np.stack([synth.random_state(p, 200 + b) for b in range(B)])
    t = [0.05, 0.3, 0.0731]
    k = p["k_fine"]
    R = torch.zeros(B, prob.n_nodes, 5, dtype=torch.float64, device="cuda")
    prob.debug_residual(B, _dev(U), _dev(Uo), t, k, R)
    Rg = _host(R)
    for b in range(B):
        err = field_rel(Rg[b], D.residual(U[b], Uo[b], t[b], k))
        assert max(err.values()) <= 1e-12, (b, err)


def test_jacobian_parity_q2(fsi, c1q2):
    p, prob, D = c1q2
    _say("case: Q2 jacobian parity c1q2 B=2")
    B = 2
    U = np.stack([synth.random_state(p, 300 + b) for b in range(B)])
    Uo = np.stack([synth.random_state(p, 400 + b) for b in range(B)])
    X = np.stack([synth.random_state(p, 500 + b) for b in range(B)])
    t = [0.02, 0.5]
    k = p["k_fine"]
    Y = torch.zeros(B, prob.n_nodes, 5, dtype=torch.float64, device="cuda")
    prob.debug_jacobian_apply(B, _dev(U), _dev(Uo), t, k, _dev(X), Y)
    Yg = _host(Y)
    for b in range(B):
        Yo = (D.jacobian(U[b], Uo[b], t[b], k) @ X[b].ravel()).reshape(-1, 5)
        err = field_rel(Yg[b], Yo)
        assert max(err.values()) <= 1e-12, (b, err)


def test_fine_propagate_parity_q2(fsi, c1q2):
    p, prob, D = c1q2
    _say("case: Q2 fine_propagate fp64 c1q2 B=2 m=3")
    k = p["k_fine"]
    m = 3
    dl = m * k
    U0 = np.zeros((D.mesh.n_nodes, 5))
    Ua = P.propagate(D, U0, 0.0, 2 * dl, 6)
    inputs, t0 = [U0, Ua], [0.0, 2 * dl]
    ref = [P.propagate(D, inputs[b], t0[b], dl, m) for b in range(2)]
    Uin = _dev(np.stack(inputs))
    Uout = torch.zeros_like(Uin)
    code, st = prob.fine_propagate(2, t0, dl, m, Uin, Uout)
    Ug = _host(Uout)
    for b in range(2):
        err = field_rel(Ug[b], ref[b], norm="l2")
        _say("slice", b, "newton", st.newton_its[b], "krylov", st.krylov_its[b], "err", err)
        assert max(err.values()) <= 1e-10, (b, err)


def test_batched_equals_sequential_q2(fsi, c1q2):
    p, prob, D = c1q2
    _say("case: Q2 batched vs sequential c1q2 B=3")
    k = p["k_fine"]
    dl = 2 * k
    ins = np.stack([synth.random_state(p, 600 + q, grad_u_max=0.02) * [0.3, 0.3, 1, 1, 0] for q in range(3)])
    t0 = [0.1 + q * dl for q in range(3)]
    for q in range(3):
        ins[q] = D.apply_dirichlet(ins[q], t0[q])
    Uin = _dev(ins)
    Ub = torch.zeros_like(Uin)
    prob.fine_propagate(3, t0, dl, 2, Uin, Ub)
    Us = torch.zeros_like(Uin)
    for q in range(3):
        out = torch.zeros_like(Uin[q:q + 1])
        prob.fine_propagate(1, [t0[q]], dl, 2, Uin[q:q + 1].contiguous(), out)
        Us[q] = out[0]
    err = field_rel(_host(Ub), _host(Us), norm="l2")
    assert max(err.values()) <= 1e-10, err


def test_c2q2_fullsize_sampled_slice(fsi):
    """32 slices of c2q2 (64x16 Q2 cells, 21,285 unknowns) in one call, one fine step; slice 13
    against the oracle (about half a minute on the host)."""
    p = synth.workload("c2q2", seed=0)
    _say("case: c2q2 full size, 32 slices in one call, one step; slice 13 vs oracle")
    D = Discretization(p)
    N, dl = p["N"], p["slice_len"]
    t0s = [l * dl for l in range(N)]
    U_in = np.stack([D.apply_dirichlet(synth.smooth_state(p, 200 + l), t0s[l]) for l in range(N)])
    prob = fsi.Problem(fsi.make_params(p, precision="fp64", max_batch=N))
    Uin = _dev(U_in)
    Uout = torch.zeros_like(Uin)
    code, st = prob.fine_propagate(N, t0s, p["k_fine"], 1, Uin, Uout)
    Ug = _host(Uout)
    prob.close()
    assert code == fsi.FSI_OK
    l = 13
    ref = P.propagate(D, U_in[l], t0s[l], p["k_fine"], 1)
    err = field_rel(Ug[l], ref, norm="l2")
    _say("slice", l, "newton", st.newton_its[l], "krylov", st.krylov_its[l], err)
    assert max(err.values()) <= 1e-10, err


# ---- edge cases of the Q2 path (as for Q1 in test_gpu_edge.py)

def test_q2_rest_state_is_a_fixed_point(fsi):
    """Zero inflow from rest: every step's residual is zero at the guess, so no linear solve runs
    and the state stays exactly zero (fine and coarse propagator)."""
    p = synth.workload("c1q2", seed=0, inflow_peak=0.0)
    m = 3
    _say("case: Q2 zero inflow, zero state, c1q2 B=2")
    prob = fsi.Problem(fsi.make_params(p, precision="fp64", max_batch=2))
    U = torch.zeros(2, prob.n_nodes, 5, dtype=torch.float64, device="cuda")
    out = torch.full_like(U, 7.0)
    code, st = prob.fine_propagate(2, [0.0, p["slice_len"]], p["slice_len"], m, U, out)
    assert code == fsi.FSI_OK
    assert not bool(out.any()), _host(out).max()
    assert list(st.krylov_its[:2]) == [0, 0], list(st.krylov_its[:2])
    code, st = prob.coarse_propagate(2, [0.0, p["slice_len"]], p["slice_len"], 1, U, out)
    assert code == fsi.FSI_OK and not bool(out.any())
    prob.close()


def test_q2_nonfinite_input_is_refused(fsi):
    p = synth.workload("c1q2", seed=2)
    _say("case: Q2 NaN in slice 1 of a c1q2 batch of 2")
    D = Discretization(p)
    prob = fsi.Problem(fsi.make_params(p, precision="fp64", max_batch=2))
    U = np.stack([D.apply_dirichlet(synth.smooth_state(p, 40 + l), 0.0) for l in range(2)])
    U[1, 17, 4] = np.nan
    out = torch.full((2, prob.n_nodes, 5), 7.0, dtype=torch.float64, device="cuda")
    code, st = prob.fine_propagate(2, [0.0, 0.0], p["slice_len"], 2, _dev(U), out, raise_on_error=False)
    assert code == fsi.FSI_ERR_NONFINITE
    assert list(st.slice_status[:2]) == [fsi.FSI_OK, fsi.FSI_ERR_NONFINITE]
    assert bool((_host(out) == 7.0).all())
    prob.close()


def test_q2_groups_and_aliasing_equal_one_batch(fsi):
    """Concurrent slice groups (batch_split 2 and 3) and an aliased U_in/U_out give the single
    batch's outputs and iteration counts bit for bit (c1q2, B = 5)."""
    p = synth.workload("c1q2", seed=5)
    _say("case: Q2 c1q2 B=5, batch_split 0 vs 2 vs 3, and in place")
    D = Discretization(p)
    dl = p["slice_len"]
    t0 = [l * dl for l in range(5)]
    U = np.stack([D.apply_dirichlet(synth.smooth_state(p, 100 + l), t0[l]) for l in range(5)])
    res = {}
    for split in (0, 2, 3):
        prob = fsi.Problem(fsi.make_params(p, precision="fp64", max_batch=5, batch_split=split))
        out = torch.zeros(5, prob.n_nodes, 5, dtype=torch.float64, device="cuda")
        code, st = prob.fine_propagate(5, t0, dl, 2, _dev(U), out)
        assert code == fsi.FSI_OK
        res[split] = (_host(out), list(st.newton_its[:5]), list(st.krylov_its[:5]))
        if split == 0:
            inplace = _dev(U)
            prob.fine_propagate(5, t0, dl, 2, inplace, inplace)
            assert np.array_equal(_host(inplace), res[0][0])
        prob.close()
    for split in (2, 3):
        assert np.array_equal(res[split][0], res[0][0]), (split, np.abs(res[split][0] - res[0][0]).max())
        assert res[split][1:] == res[0][1:], (split, res[split][1:], res[0][1:])


# ---- Q2 cells in the mixed-precision path (FP32 Krylov/multigrid, FP64 Newton)

def test_fine_propagate_parity_q2_mixed(fsi, c1q2):
    """c1q2, two slices of three steps, with the FP32 inner solve: the FP64 Newton refinement
    brings the steps to the FP64 oracle within 1e-6."""
    p, _, D = c1q2
    _say("case: Q2 fine_propagate mixed c1q2 B=2 m=3")
    k = p["k_fine"]
    m = 3
    dl = m * k
    U0 = np.zeros((D.mesh.n_nodes, 5))
    Ua = P.propagate(D, U0, 0.0, 2 * dl, 6)
    inputs, t0 = [U0, Ua], [0.0, 2 * dl]
    ref = [P.propagate(D, inputs[b], t0[b], dl, m) for b in range(2)]
    prob = fsi.Problem(fsi.make_params(p, precision="mixed", max_batch=2, batch_split=0))
    Uin = _dev(np.stack(inputs))
    Uout = torch.zeros_like(Uin)
    code, st = prob.fine_propagate(2, t0, dl, m, Uin, Uout)
    Ug = _host(Uout)
    prob.close()
    assert code == fsi.FSI_OK
    for b in range(2):
        err = field_rel(Ug[b], ref[b], norm="l2")
        _say("slice", b, "newton", st.newton_its[b], "krylov", st.krylov_its[b], "err", err)
        assert max(err.values()) <= 1e-6, (b, err)


def test_c3q2_fullsize_mixed_equals_fp64(fsi):
    """64 slices of c3q2 (128x32 Q2 cells on the 16,705 nodes of c3) in one call, one step, in
    mixed precision and in FP64: the refined steps agree within 1e-6 per field on every slice
    (the FP64 Q2 path is compared with the oracle at the c2q2 size above)."""
    p = synth.workload("c3q2", seed=0)
    _say("case: c3q2 full size, 64 slices in one call, one step, mixed vs FP64")
    D = Discretization(p)
    N, dl = p["N"], p["slice_len"]
    t0s = [l * dl for l in range(N)]
    U_in = np.stack([D.apply_dirichlet(synth.smooth_state(p, 300 + l), t0s[l]) for l in range(N)])
    Uin = _dev(U_in)
    out = {}
    for prec in ("fp64", "mixed"):
        prob = fsi.Problem(fsi.make_params(p, precision=prec, max_batch=N))
        o = torch.zeros_like(Uin)
        code, st = prob.fine_propagate(N, t0s, p["k_fine"], 1, Uin, o)
        assert code == fsi.FSI_OK, prec
        out[prec] = _host(o)
        _say(prec, "newton", st.newton_total, "krylov", st.krylov_total)
        prob.close()
    worst = max(max(field_rel(out["mixed"][l], out["fp64"][l], norm="l2").values()) for l in range(N))
    _say("worst slice difference", worst)
    assert worst <= 1e-6, worst
