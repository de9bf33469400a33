"""Pins of the oracle's damage update (Sec. 2.1, 2.2, 2.4)."""
import itertools

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as w
from oracle.damage import DamageQP, assemble_damage, kkt_residuals, node_area, solve_bound_qp, solve_box_qp
from oracle.fem import make_mesh
from tests._helpers import rel

GC, L0 = 3.0, 5e-4


def mesh_of(nx, ny, h, jitter=0.0, seed=0, random_diag=False):
    m = w.plate_mesh(nx, ny, h, jitter, seed, random_diag=random_diag)
    return m, make_mesh(m["xy"], m["tri"])


def quadrature_system(mesh, H, Gc, l0, model):
    """Dense A and b from a degree-2 exact edge-midpoint rule on every element.

    Gc is a scalar or one value per element."""
    n = mesh.n_nodes
    Gce = np.broadcast_to(np.asarray(Gc, dtype=np.float64), (len(mesh.tri),))
    A = np.zeros((n, n))
    b = np.zeros(n)
    X = mesh.xy.numpy()
    # barycentric coordinates of the three edge midpoints, weight 1/3 each
    pts = np.array([[0.5, 0.5, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5]])
    for e, t in enumerate(mesh.tri.numpy()):
        P = np.hstack([np.ones((3, 1)), X[t]])
        C = np.linalg.inv(P)
        grads = C[1:, :].T                       # row k = grad phi_k
        area = abs(np.linalg.det(P)) / 2
        g = Gce[e]
        if model == 2:
            kappa, c, load = g * l0, g / l0 + 2 * H[e], 2 * H[e]
        else:
            kappa, c, load = 0.75 * g * l0, 2 * H[e], 2 * H[e] - 3 * g / (8 * l0)
        Ke = area * grads @ grads.T
        Me = sum(area / 3 * np.outer(p, p) for p in pts)
        fe = sum(area / 3 * p for p in pts)
        A[np.ix_(t, t)] += kappa * Ke + c * Me
        b[t] += load * fe
    return A, b


@pytest.mark.parametrize("model", [1, 2])
def test_assembly_against_quadrature(model):
    """P7: the consistent-mass assembly equals an independent quadrature assembly."""
    m, mesh = mesh_of(7, 5, 2.5e-4, 0.2, 3, random_diag=True)
    H = np.random.default_rng(0).uniform(0, 5000, mesh.n_elems)
    A, b = assemble_damage(mesh, H, GC, L0, model)
    Aq, bq = quadrature_system(mesh, H, GC, L0, model)
    assert rel(A.toarray(), Aq) < 1e-14 * 10
    assert rel(b, bq) < 1e-14 * 10
    p = np.random.default_rng(1).normal(size=mesh.n_nodes)
    assert rel(A @ p, Aq @ p) < 1e-13


def test_unconstrained_equals_dense_solve():
    """P8 (a): with an inactive bound the QP solution is the linear solve."""
    m, mesh = mesh_of(9, 6, 2.5e-4, 0.1, 4)
    H = np.random.default_rng(2).uniform(100, 5000, mesh.n_elems)
    A, b = assemble_damage(mesh, H, GC, L0, 2)
    x, act = solve_bound_qp(A, b, np.full(mesh.n_nodes, -1.0))
    assert not act.any()
    assert rel(x, np.linalg.solve(A.toarray(), b)) < 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_qp_unique_kkt_point_by_enumeration(seed):
    """P8 (b): enumerate all 2^n active sets on a 12-node mesh; exactly one KKT point exists."""
    m, mesh = mesh_of(3, 2, 2.5e-4, 0.2, seed, random_diag=True)
    n = mesh.n_nodes
    r = np.random.default_rng(seed)
    H = r.uniform(0, 3000, mesh.n_elems)
    lb = np.where(r.random(n) < 0.4, r.uniform(0, 0.6, n), 0.0)
    A, b = assemble_damage(mesh, H, GC, L0, 1)
    Ad = A.toarray()
    sols = []
    for mask in itertools.product([False, True], repeat=n):
        act = np.array(mask)
        free = ~act
        x = lb.copy()
        if free.any():
            x[free] = np.linalg.solve(Ad[np.ix_(free, free)], b[free] - Ad[np.ix_(free, act)] @ lb[act])
        mu = Ad @ x - b
        if np.all(x[free] >= lb[free] - 1e-13) and np.all(mu[act] >= -1e-13 * np.abs(Ad).max()):
            sols.append(x)
    assert len(sols) >= 1
    ref = sols[0]
    assert all(np.allclose(s, ref, atol=1e-12, rtol=0) for s in sols)
    x, _ = solve_bound_qp(A, b, lb)
    assert np.max(np.abs(x - ref)) < 1e-12
    viol, rf, ra, ru = kkt_residuals(A, b, lb, x)
    assert viol <= 0 and rf < 1e-12 and ra < 1e-12


@pytest.mark.parametrize("inner", ["lu", "cg"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_box_qp_unique_kkt_point_by_enumeration(seed, inner):
    """P8 (c): with d <= 1 as well, enumerate all 3^9 (free / lower / upper) sets on a 9-node mesh."""
    m, mesh = mesh_of(2, 2, 2.5e-4, 0.2, seed, random_diag=True)
    n = mesh.n_nodes
    r = np.random.default_rng(10 + seed)
    H = r.uniform(0, 40000, mesh.n_elems)
    lb = np.where(r.random(n) < 0.5, r.uniform(0.3, 1.0, n), 0.0)
    ub = np.ones(n)
    A, b = assemble_damage(mesh, H, GC, L0, 2)
    Ad = A.toarray()
    sols = []
    for mask in itertools.product([0, 1, 2], repeat=n):
        st = np.array(mask)
        lo, up = st == 1, st == 2
        free = st == 0
        x = np.where(lo, lb, np.where(up, ub, 0.0))
        if free.any():
            held = ~free
            x[free] = np.linalg.solve(Ad[np.ix_(free, free)], b[free] - Ad[np.ix_(free, held)] @ x[held])
        g = Ad @ x - b
        eps = 1e-13 * np.abs(Ad).max()
        if (np.all(x[free] >= lb[free] - 1e-13) and np.all(x[free] <= 1 + 1e-13)
                and np.all(g[lo] >= -eps) and np.all(g[up] <= eps) and np.all(lb <= ub)):
            sols.append(x)
    assert len(sols) >= 1
    assert all(np.allclose(s, sols[0], atol=1e-12, rtol=0) for s in sols)
    x, lo, up = solve_box_qp(A, b, lb, ub, inner=inner)
    assert np.max(np.abs(x - sols[0])) < 1e-12
    viol, rf, ra, ru = kkt_residuals(A, b, lb, x, ub)
    assert viol <= 0 and rf < 1e-12 and ra < 1e-12 and ru < 1e-12


@pytest.mark.parametrize("model", [1, 2])
def test_cg_free_set_solver_matches_sparse_lu(model):
    """The conjugate-gradient free-set solves reach the sparse-LU minimiser of the same box QP
    (a 96x48 plate with a damaged band and random history), and the dense solve when no bound
    is active."""
    m, mesh = mesh_of(96, 48, 2.5e-4, 0.1, 5, random_diag=True)
    n = mesh.n_nodes
    r = np.random.default_rng(20 + model)
    H = r.uniform(0, 6000, mesh.n_elems) * (r.random(mesh.n_elems) < 0.6)
    lb = np.where(np.abs(m["ij"][:, 1] - 24) <= 2, r.uniform(0.2, 1.0, n), 0.0)
    A, b = assemble_damage(mesh, H, GC, L0, model)
    x_lu, lo_lu, up_lu = solve_box_qp(A, b, lb, np.ones(n), x0=lb, inner="lu")
    x_cg, lo_cg, up_cg = solve_box_qp(A, b, lb, np.ones(n), x0=lb, inner="cg")
    assert lo_lu.any() and np.max(np.abs(x_cg - x_lu)) < 1e-12
    viol, rf, ra, ru = kkt_residuals(A, b, lb, x_cg, np.ones(n))
    assert viol <= 0 and rf < 1e-12 and ra < 1e-12 and ru < 1e-12
    m2, mesh2 = mesh_of(20, 10, 2.5e-4, 0.1, 6)
    A2, b2 = assemble_damage(mesh2, r.uniform(100, 5000, mesh2.n_elems), GC, L0, 2)
    x2, act = solve_bound_qp(A2, b2, np.full(mesh2.n_nodes, -1.0), inner="cg")
    assert not act.any() and rel(x2, np.linalg.solve(A2.toarray(), b2)) < 1e-12


def test_upper_bound_is_a_constraint_of_the_programme():
    """The update over [d_prev, 1] differs from clamping the lower-bounded minimiser."""
    from oracle.step import Sim, initial_state
    p = w.small_plate(32, 16, seed=3)
    sim = Sim(p)
    st = initial_state(p)
    found = False
    for _ in range(120):
        u1, v1, a1, H1, _ = sim.explicit(st)
        A, b = sim.qp.system(H1.numpy(), p.Gc)
        lb = st.d.numpy()
        x1, _ = solve_bound_qp(A, b, lb, x0=lb)
        if x1.max() > 1.0:
            xb, lo, up = solve_box_qp(A, b, lb, np.ones_like(lb), x0=lb)
            assert up.any() and np.all(xb <= 1.0) and np.all(xb >= lb)
            viol, rf, ra, ru = kkt_residuals(A, b, lb, xb, np.ones_like(lb))
            assert viol <= 0 and rf < 1e-12 and ra < 1e-12 and ru < 1e-12
            # clamping the lower-bounded minimiser is not the box minimiser
            assert np.max(np.abs(np.minimum(x1, 1.0) - xb)) > 1e-8
            found = True
            break
        st = sim.step(st)
    assert found


def crack_row_problem(ny_cells, ratio, model, nx=None):
    """Unjittered strip with a full-width crack (d_prev = 1) on the bottom row and H = 0."""
    h = L0 / ratio
    nx = nx or int(50 * ratio)
    m, mesh = mesh_of(nx, ny_cells, h)
    ij = m["ij"]
    lb = np.where(ij[:, 1] == 0, 1.0, 0.0)
    H = np.zeros(mesh.n_elems)
    qp = DamageQP(mesh, L0, model)
    d, act, upper, x, A = qp.solve(H, GC, lb)
    col = ij[:, 0] == nx // 2
    order = np.argsort(ij[col, 1])
    return d[col][order], h


@pytest.mark.parametrize("ratio,tol", [(2, 1e-13), (8, 1e-10)])
def test_at2_discrete_profile_closed_form(ratio, tol):
    """P9: AT2 profile from a crack row against the exact solution of the 3-point recurrence.

    For an x-independent field the scheme reduces to
    (rho^2/6 - 1)(d_{j-1} + d_{j+1}) + (2 + 2 rho^2/3) d_j = 0, rho = h/l0, whose
    solution with d_0 = 1 and a natural boundary at j = N is
    (r^j + r^{2N-j})/(1 + r^{2N}), r + 1/r = q.  It tends to the paper's
    1D profile exp(-|n|/l0) (Sec. 2.1) as h -> 0.
    """
    N = 12 * ratio // 2
    d, h = crack_row_problem(N, ratio, 2)
    rho = h / L0
    q = (2 * rho ** 2 / 3 + 2) / (1 - rho ** 2 / 6)
    rr = (q - np.sqrt(q * q - 4)) / 2
    j = np.arange(N + 1)
    exact = (rr ** j + rr ** (2 * N - j)) / (1 + rr ** (2 * N))
    assert np.max(np.abs(d - exact)) < tol
    cont = np.cosh((N - j) * h / L0) / np.cosh(N * h / L0)
    assert np.max(np.abs(d - cont)) < {2: 4e-3, 8: 3e-4}[ratio]


def test_at1_profile_exact():
    """P10: AT1 profile <1 - |n|/(2 l0)>+^2 (Sec. 2.1) is reproduced at the nodes.

    The profile is quadratic, the load of the AT1 operator with H = 0 is
    constant, and linear elements are nodally exact for that 1D problem; the
    free boundary 2 l0 falls on a node for these spacings, so the discrete
    minimiser equals the closed form to rounding, and d equals the bound
    beyond 2 l0.
    """
    for ratio in (2, 4, 8):
        N = 4 * ratio
        d, h = crack_row_problem(N, ratio, 1)
        y = np.arange(N + 1) * h
        exact = np.maximum(1 - y / (2 * L0), 0) ** 2
        assert np.max(np.abs(d - exact)) < 1e-12
        assert np.all(d[y >= 2 * L0 - 1e-12] == 0.0)


@pytest.mark.parametrize("model", [1, 2])
def test_uniform_history_closed_form(model):
    """P13: uniform H gives a uniform d; AT1 grows only above H_crit = 3Gc/(16 l0)."""
    m, mesh = mesh_of(8, 5, 2.5e-4, 0.15, 1, random_diag=True)
    qp = DamageQP(mesh, L0, model)
    hc = 3 * GC / (16 * L0)
    for Hv in (0.5 * hc, 0.999 * hc, 1.001 * hc, 3.0 * hc, 40.0 * hc):
        d, act, upper, x, A = qp.solve(np.full(mesh.n_elems, Hv), GC, np.zeros(mesh.n_nodes))
        if model == 2:
            expect = 2 * Hv / (GC / L0 + 2 * Hv)
        else:
            expect = max(1 - hc / Hv, 0.0)
        assert np.max(np.abs(d - expect)) < 1e-12
        if model == 1 and Hv < hc:
            assert np.all(d == 0)


def test_postclamp_mode():
    """AT2 alternative: unconstrained solve, then clamp to [d_prev, 1] (Sec. 2.4)."""
    m, mesh = mesh_of(9, 6, 2.5e-4, 0.1, 4)
    r = np.random.default_rng(5)
    H = r.uniform(0, 8000, mesh.n_elems)
    lb = r.uniform(0, 0.5, mesh.n_nodes)
    qp = DamageQP(mesh, L0, 2, bounds="postclamp")
    d, act, upper, x, A = qp.solve(H, GC, lb)
    A2, b2 = assemble_damage(mesh, H, GC, L0, 2)
    ref = np.minimum(np.maximum(np.linalg.solve(A2.toarray(), b2), lb), 1.0)
    assert rel(d, ref) < 1e-12
    # the projected minimiser differs and satisfies the KKT conditions
    qpp = DamageQP(mesh, L0, 2)
    dp, actp, _, xp, _ = qpp.solve(H, GC, lb)
    viol, rf, ra, ru = kkt_residuals(A2, b2, lb, xp, np.ones_like(lb))
    assert viol <= 0 and rf < 1e-11 and ra < 1e-11 and ru < 1e-11


def test_qp_tangent_by_finite_differences():
    """Implicit rule (Sec. 4.2) against central differences of the exact QP solution."""
    m, mesh = mesh_of(6, 4, 2.5e-4, 0.2, 8, random_diag=True)
    r = np.random.default_rng(3)
    for model in (1, 2):
        qp = DamageQP(mesh, L0, model)
        H = r.uniform(0, 4000, mesh.n_elems)
        lb = np.where(r.random(mesh.n_nodes) < 0.3, r.uniform(0, 0.4, mesh.n_nodes), 0.0)
        dH = r.normal(size=mesh.n_elems) * 100
        dlb = np.where(lb > 0, r.normal(size=mesh.n_nodes) * 0.01, 0.0)
        d, act, upper, x, A = qp.solve(H, GC, lb)
        t = qp.tangent(A, x, act, upper, H, GC, dH, 0.3, dlb)
        eps = 1e-6
        dp = qp.solve(H + eps * dH, GC + eps * 0.3, lb + eps * dlb)[0]
        dm = qp.solve(H - eps * dH, GC - eps * 0.3, lb - eps * dlb)[0]
        fd = (dp - dm) / (2 * eps)
        assert np.max(np.abs(fd - t)) < 1e-6 * max(1.0, np.abs(t).max())


def test_at1_degenerate_free_boundary_early_steps():
    """AT1 with sub-threshold history: the support edge is degenerate (d = lb, mu = 0).

    The active-set iteration must still return the KKT point there; this
    plate's second step used to make it flip nodes on rounding noise.
    """
    from oracle.step import Sim, initial_state
    p = w.small_plate(48, 24, jitter=0.1, seed=2, model=1, split="starconvex", gamma_star=1.0, plane="stress")
    sim = Sim(p)
    st = initial_state(p)
    for _ in range(4):
        u1, v1, a1, H1, _ = sim.explicit(st)
        A, b = sim.qp.system(H1.numpy(), p.Gc)
        x, act = solve_bound_qp(A, b, st.d.numpy(), x0=st.d.numpy())
        viol, rf, ra, ru = kkt_residuals(A, b, st.d.numpy(), x)
        assert viol <= 0 and rf < 1e-12 and ra < 1e-12
        st = sim.step(st)
