"""Oracle pins for the drag functional and its discrete adjoint gradient."""
import numpy as np
import pytest

import synth
from oracle.residual import Discretization
from oracle import adjoint as A


def test_drag_closed_form():
    """Shear flow v = (a y, 0), pressure p = P0 - G x, u = 0 on the bar faces.

    Traction e_x . sigma n_s: left face (n_s = -e_x) gives +p(0.4), right face
    -p(0.5), top face (n_s = +e_y) rho nu a; hence D = w (h G + rho nu a) with
    bar width w = 0.1 and height h = 0.25 (the bottom face is on the wall).
    """
    p = synth.workload("c1")
    D = Discretization(p)
    X = D.mesh.X
    a, P0, G = 0.7, 3.0, 12.0
    U = np.zeros((D.mesh.n_nodes, 5))
    U[:, 0] = a * X[:, 1]
    U[:, 4] = P0 - G * X[:, 0]
    expect = 0.1 * (0.25 * G + p["rho_f"] * p["nu_f"] * a)
    assert abs(A.drag(D, U) - expect) <= 1e-12 * abs(expect)
    # a rigid translation of the mesh (grad u = 0) changes nothing
    U[:, 2] = 0.01
    U[:, 3] = -0.02
    assert abs(A.drag(D, U) - expect) <= 1e-12 * abs(expect)
    # the faces: 4 + 4 vertical, 2 horizontal at level 1
    assert len(A.drag_faces(D)) == 10


@pytest.fixture(scope="module")
def small():
    p = synth.workload("c1", T=0.04, N=2, dt_fine=0.01)
    D = Discretization(p)
    U0 = np.zeros((D.mesh.n_nodes, 5))
    J, g = A.adjoint_gradient(D, p, U0)
    return p, D, U0, J, g


def test_adjoint_equals_tangent_linear(small):
    """Duality: the adjoint gradient equals the forward (tangent-linear) sensitivities."""
    p, D, U0, J, g = small
    gt = A.tangent_gradient(D, p, U0)
    assert np.all(np.abs(g - gt) <= 1e-10 * np.abs(gt)), (g, gt)


def test_adjoint_equals_complex_step_through_forward_solve(small):
    p, D, U0, J, g = small
    gc = A.complex_step_gradient(D, p, U0)
    assert np.all(np.abs(g - gc) <= 1e-10 * np.abs(gc)), (g, gc)


def test_adjoint_matches_central_differences(small):
    """Central differences with relative step 1e-6 on the full forward solve."""
    p, D, U0, J, g = small
    for i, q in enumerate(A.PARAMS):
        h = 1e-6 * abs(p[q])
        vals = []
        for s in (1, -1):
            params = {q: p[q] + s * h}
            states, times, k = A.trajectory(D, p, U0, params=params)
            vals.append(A.functional(D, states, k))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-5 * abs(g[i]), (q, fd, g[i])
    assert J > 0  # flow in +x pushes the bar downstream (sanity only, parity unpinned)
