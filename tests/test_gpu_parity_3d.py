"""GPU parity in 3d (Q1 hexahedra, 7 unknowns per node) through the C ABI.

The workload is the c5 geometry and physics (duct with an elastic block on the
floor) at refinement level 1, 32x8x8 cells, so that the FP64 oracle runs in
seconds per residual / Jacobian.  Its Newton steps take about a minute per
slice, so the reference states of the propagator tests are stored in
tests/golden/c5_level1_steps.npz, written by tests/golden/make_c5_level1_steps.py
from the oracle alone.

Tolerances as in 2d: residual and Jacobian products 1e-12 relative per field,
FP64 propagation 1e-10, mixed-precision propagation 1e-6.
"""
import os
import sys

import numpy as np
import pytest

import synth
from oracle.residual import Discretization

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_level1_steps.npz")
FIELDS = {"v": slice(0, 3), "u": slice(3, 6), "p": slice(6, 7)}


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
def c5l1(fsi):
    p = synth.workload("c5", seed=0, level=1)
    prob = fsi.Problem(fsi.make_params(p, precision="fp64", max_batch=2))
    return p, prob, Discretization(p)


def test_sizes_3d(fsi, c5l1):
    p, prob, D = c5l1
    assert prob.n_nodes == 33 * 9 * 9 == D.mesh.n_nodes
    assert prob.n_dofs == 7 * prob.n_nodes


def test_residual_parity_3d(fsi, c5l1):
    p, prob, D = c5l1
    _say("case: residual parity 3d c5-level1 B=2")
    B = 2
    U = np.stack([synth.random_state(p, 100 + b) for b in range(B)])
    Uo = np.stack([synth.random_state(p, 200 + b) for b in range(B)])
    t = [0.05, 0.3]
    k = p["k_fine"]
    R = torch.zeros(B, prob.n_nodes, 7, dtype=torch.float64, device="cuda")
    prob.debug_residual(B, _dev(U), _dev(Uo), t, k, R)
    Rg = _host(R)
    for b in range(B):
        Ro = D.residual(U[b], Uo[b], t[b], k)
        err = field_rel(Rg[b], Ro)
        _say("slice", b, err)
        assert max(err.values()) <= 1e-12, (b, err)


def test_jacobian_parity_3d(fsi, c5l1):
    p, prob, D = c5l1
    _say("case: jacobian parity 3d c5-level1 B=1")
    U = synth.random_state(p, 300)[None]
    Uo = synth.random_state(p, 400)[None]
    X = synth.random_state(p, 500)[None]
    t = [0.2]
    k = p["k_fine"]
    Y = torch.zeros(1, prob.n_nodes, 7, dtype=torch.float64, device="cuda")
    prob.debug_jacobian_apply(1, _dev(U), _dev(Uo), t, k, _dev(X), Y)
    Yg = _host(Y)
    A = D.jacobian(U[0], Uo[0], t[0], k)
    Yo = (A @ X[0].ravel()).reshape(-1, 7)
    err = field_rel(Yg[0], Yo)
    _say(err)
    assert max(err.values()) <= 1e-12, err


def test_vcycle_contracts_3d(fsi, c5l1):
    """The 3d V-cycle (Vanka sweeps down to level 0) contracts on the Newton Jacobian."""
    p, prob, D = c5l1
    _say("case: vcycle contraction 3d c5-level1")
    g = np.load(GOLDEN)
    k = float(g["k"])
    t = [float(g["t0"]) + k]
    U1 = g["U_out"][0]
    Ug = D.apply_dirichlet(U1, t[0])
    rng = np.random.default_rng(5)
    e = rng.normal(size=U1.shape) * np.array([0.3, 0.3, 0.3, 1e-3, 1e-3, 1e-3, 100.0])
    e[D.dirichlet] = 0.0
    Ud, Uod = _dev(Ug[None]), _dev(U1[None])
    E = _dev(e[None])
    AE = torch.zeros_like(E)
    ME = torch.zeros_like(E)
    ratios = []
    for _ in range(6):
        prob.debug_jacobian_apply(1, Ud, Uod, t, k, E, AE)
        prob.debug_vcycle(1, Ud, Uod, t, k, AE, ME)
        E2 = E - ME
        ratios.append((torch.linalg.norm(E2) / torch.linalg.norm(E)).item())
        E = E2.contiguous()
    _say("ratios", ratios)
    assert max(ratios[2:]) < 0.9, ratios


def _golden_run(fsi, p, prob):
    g = np.load(GOLDEN)
    U_in, U_ref = g["U_in"], g["U_out"]
    t0, k, steps = float(g["t0"]), float(g["k"]), int(g["steps"])
    B = U_in.shape[0]
    Uin = _dev(U_in)
    Uout = torch.zeros_like(Uin)
    code, st = prob.fine_propagate(B, [t0] * B, steps * k, steps, Uin, Uout)
    return _host(Uout), U_ref, st


def test_fine_propagate_parity_fp64_3d(fsi, c5l1):
    p, prob, D = c5l1
    _say("case: fine_propagate fp64 3d c5-level1 B=2 m=2 (golden)")
    Ug, Uref, st = _golden_run(fsi, p, prob)
    for b in range(Ug.shape[0]):
        err = field_rel(Ug[b], Uref[b], norm="l2")
        _say("slice", b, "newton", st.newton_its[b], "krylov", st.krylov_its[b], "err", err)
        assert max(err.values()) <= 1e-10, (b, err)


def test_fine_propagate_parity_mixed_3d(fsi):
    p = synth.workload("c5", seed=0, level=1)
    _say("case: fine_propagate mixed 3d c5-level1 B=2 m=2 (golden)")
    prob = fsi.Problem(fsi.make_params(p, precision="mixed", max_batch=2))
    Ug, Uref, st = _golden_run(fsi, p, prob)
    for b in range(Ug.shape[0]):
        err = field_rel(Ug[b], Uref[b], norm="l2")
        _say("mixed slice", b, "newton", st.newton_its[b], "krylov", st.krylov_its[b], "err", err)
        assert max(err.values()) <= 1e-6, (b, err)
    prob.close()


def test_batched_equals_sequential_3d(fsi, c5l1):
    p, prob, D = c5l1
    _say("case: batched vs sequential 3d c5-level1 B=2")
    g = np.load(GOLDEN)
    t0, k = float(g["t0"]), float(g["k"])
    Uin = _dev(g["U_in"])
    Ub = torch.zeros_like(Uin)
    prob.fine_propagate(2, [t0, t0], k, 1, Uin, Ub)
    Us = torch.zeros_like(Uin)
    for q in range(2):
        out = torch.zeros_like(Uin[q:q + 1])
        prob.fine_propagate(1, [t0], k, 1, Uin[q:q + 1].contiguous(), out)
        Us[q] = out[0]
    err = field_rel(_host(Ub), _host(Us), norm="l2")
    assert max(err.values()) <= 1e-10, err


def test_adjoint_rejects_3d(fsi, c5l1):
    p, prob, D = c5l1
    U0 = torch.zeros(1, prob.n_nodes, 7, dtype=torch.float64, device="cuda")
    with pytest.raises(fsi.FsiError):
        prob.adjoint_gradient(0.01, 1, 1, U0[0])


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_wide_block_variant_vs_golden_3d(fsi, precision, tol):
    """32 slices in one batch: the finest level's colours then hold (256 cells x 32 slices)
    >= 8192 cells over the batch, so the fused Vanka pass and the factor run with 32 cells per
    block (the variant of the 64x16x16-cell workload) instead of 8.  Every slice (the two golden
    inputs repeated) against the stored oracle steps."""
    p = synth.workload("c5", seed=0, level=1)
    _say("case: 3d wide-block variant c5-level1 B=32", precision)
    prob = fsi.Problem(fsi.make_params(p, precision=precision, max_batch=32, batch_split=0))
    g = np.load(GOLDEN)
    U_in, U_ref = g["U_in"], g["U_out"]
    t0, k, steps = float(g["t0"]), float(g["k"]), int(g["steps"])
    B = 32
    Uin = _dev(np.stack([U_in[b % 2] for b in range(B)]))
    Uout = torch.zeros_like(Uin)
    code, st = prob.fine_propagate(B, [t0] * B, steps * k, steps, Uin, Uout)
    Ug = _host(Uout)
    worst = 0.0
    for b in range(B):
        err = field_rel(Ug[b], U_ref[b % 2], norm="l2")
        worst = max(worst, max(err.values()))
        assert max(err.values()) <= tol, (b, err)
    _say("worst", worst, "newton", st.newton_total, "krylov", st.krylov_total)
    prob.close()


def test_block_width_choice_does_not_change_results_3d(fsi):
    """The autotuner's 3d block-width threshold only changes how the fused Vanka pass is launched
    (8 or 32 cells per block, with the matching inverse storage): the same 32-slice call with
    both widths gives the same states."""
    p = synth.workload("c5", seed=0, level=1)
    _say("case: 3d block width 8 vs 32, c5-level1 B=32 mixed")
    g = np.load(GOLDEN)
    t0, k = float(g["t0"]), float(g["k"])
    Uin = _dev(np.stack([g["U_in"][b % 2] for b in range(32)]))
    outs = []
    for wide in (8192, 1 << 30):
        prob = fsi.Problem(fsi.make_params(p, precision="mixed", max_batch=32, batch_split=0, vanka_wide_cells=wide))
        o = torch.zeros_like(Uin)
        prob.fine_propagate(32, [t0] * 32, k, 1, Uin, o)
        outs.append(_host(o))
        prob.close()
    d = np.abs(outs[0] - outs[1]).max() / np.abs(outs[1]).max()
    _say("max rel diff", d)
    assert d <= 1e-12, d
