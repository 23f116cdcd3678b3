"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every check uses an
independent route -- a textbook diagram computed with a KD-tree, a closed
form, an exact invariance, a brute force written another way, a library
optimiser, or a value printed in the paper.
"""
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

import apd_synth as S
import oracle as O
from oracle import ref_numpy as R

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _gap_ok(best, second, rel=1e-9):
    """pixels whose top-two gap is clear of rounding (exact ties excluded)"""
    return (second - best) > rel * (1.0 + np.abs(best))


# ----------------------------------------------------------- brute force --

@pytest.mark.parametrize("dim,n,grid,seed", [
    (2, 1, (5, 7), 0), (2, 9, (31, 17), 1), (2, 40, (64, 48), 2),
    (3, 7, (9, 11, 6), 3), (3, 25, (16, 16, 16), 4)])
def test_c_oracle_matches_numpy_brute_force(oracle_lib, dim, n, grid, seed):
    inst = S.custom(dim, n, grid, seed=seed, sigma=0.3, lo=[0.1] * dim, hi=[1.3] * dim)
    w = np.random.default_rng(seed).normal(0.0, 0.02, n)
    lab, best, second = O.assign(inst, w)
    lab2, C = R.assign(inst, w)
    assert np.array_equal(lab, lab2)
    np.testing.assert_allclose(best, C.min(axis=0), rtol=1e-13, atol=1e-15)
    ev = O.evaluate(inst, w)
    g2, grad2, cnt2 = R.evaluate(inst, w)
    assert np.array_equal(ev.counts, cnt2)
    np.testing.assert_allclose(ev.grad, grad2, rtol=0, atol=1e-15)
    assert abs(ev.g - g2) <= 1e-12 * max(1.0, abs(g2))


@pytest.mark.parametrize("dim,n,grid,lo,hi,seed", [
    (2, 23, (37, 29), (-0.5, 1.0), (1.5, 2.25), 5),
    (3, 17, (11, 9, 13), (0.25, -1.0, 2.0), (1.25, 0.5, 2.75), 6)])
def test_assign_pixels_equals_the_full_assignment(oracle_lib, dim, n, grid, lo, hi, seed):
    """Algorithm 1 at a list of pixels (the spot checker of the large grids)
    against the full assignment and the NumPy cost matrix, at the first and
    last pixel and random ones, on non-unit boxes."""
    inst = S.custom(dim, n, grid, seed=seed, sigma=0.3, lo=list(lo), hi=list(hi))
    w = np.random.default_rng(seed).normal(0.0, 0.05, n)
    J = inst.J
    idx = np.concatenate([[0, J - 1, J // 2], np.random.default_rng(seed + 1).choice(J, 200)])
    lab, best, second = O.assign_pixels(inst, w, idx)
    full_lab, full_best, full_second = O.assign(inst, w)
    np.testing.assert_array_equal(lab, full_lab[idx])
    np.testing.assert_array_equal(best, full_best[idx])
    np.testing.assert_array_equal(second, full_second[idx])
    lab2, C = R.assign(inst, w)
    np.testing.assert_array_equal(lab, lab2[idx])
    part = np.partition(C, 1, axis=0)
    np.testing.assert_allclose(best, part[0, idx], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(second, part[1, idx], rtol=1e-13, atol=1e-15)


def _dyadic_instance(dupes=True):
    """A 2D instance whose every cost is computed exactly in double in any
    order: unit pixels on [0, 12] x [0, 10] (centres k + 1/2), seeds on a
    quarter grid, matrix entries and weights small dyadic numbers.  Seeds 3
    and 4 are copies of seeds 1 and 2 (exact ties everywhere they win)."""
    rng = np.random.default_rng(21)
    n = 9
    x = rng.integers(0, 48, (n, 2)) / 4.0
    x[:, 1] = rng.integers(0, 40, n) / 4.0
    A = np.zeros((n, 2, 2))
    for i in range(n):
        a, c = rng.choice([0.5, 1.0, 2.0], 2)
        b = rng.choice([-0.25, 0.0, 0.25])
        A[i] = [[a, b], [b, c]]
    w = rng.integers(-16, 16, n) / 4.0
    if dupes:
        x[3], A[3], w[3] = x[1], A[1], w[1]
        x[4], A[4], w[4] = x[2], A[2], w[2]
    v = np.full(n, 120.0 / n)
    return S.Instance(2, (12, 10), (0.0, 0.0), (12.0, 10.0), x, A, v), w


def test_runner_up_is_the_second_order_statistic(oracle_lib):
    """C_(2) of the oracle is the second smallest cost over the seeds
    (np.partition of the NumPy cost matrix), exact ties counted twice, on an
    instance whose costs are exact in double; +inf when there is one seed."""
    inst, w = _dyadic_instance()
    lab, best, second = O.assign(inst, w)
    lab2, C = R.assign(inst, w)
    part = np.partition(C, 1, axis=0)
    np.testing.assert_array_equal(lab, lab2)
    np.testing.assert_array_equal(best, part[0])
    np.testing.assert_array_equal(second, part[1])
    # where a duplicated seed wins, the runner-up is its copy: a zero gap,
    # and the lower index is the label
    tie = np.isin(lab, [1, 2])
    assert tie.sum() > 0
    np.testing.assert_array_equal(second[tie], best[tie])
    assert not np.isin(lab, [3, 4]).any()
    # the same through the pixel-list form
    idx = np.arange(inst.J)
    l3, b3, s3 = O.assign_pixels(inst, w, idx)
    np.testing.assert_array_equal(s3, part[1])
    # a single seed: no runner-up
    one = S.Instance(2, (12, 10), (0.0, 0.0), (12.0, 10.0), inst.x[:1], inst.A[:1], inst.v[:1] * 0 + 120.0)
    l1, b1, s1 = O.assign(one, w[:1])
    assert np.all(l1 == 0) and np.all(np.isinf(s1)) and np.all(s1 > 0)
    np.testing.assert_array_equal(b1, R.cost_matrix(one, w[:1])[0])


def test_pixel_volume_and_centres(oracle_lib):
    inst = S.custom(3, 3, (4, 5, 8), seed=0, lo=[-1.0, 0.0, 2.0], hi=[1.0, 0.5, 6.0])
    assert O.pixel_volume(inst) == pytest.approx((2 / 4) * (0.5 / 5) * (4 / 8), rel=1e-15)
    y = O.pixel_centres(inst)
    # pixel 1 is the second along the last axis (row-major, last axis fastest)
    np.testing.assert_allclose(y[0], [-0.75, 0.05, 2.25])
    np.testing.assert_allclose(y[1], [-0.75, 0.05, 2.75])
    np.testing.assert_allclose(y[8], [-0.75, 0.15, 2.25])


# ------------------------------------------------------- special cases --

def _kd_labels(points_seed, points_query, lift_seed=None):
    if lift_seed is not None:
        points_seed = np.concatenate([points_seed, lift_seed[:, None]], axis=1)
        points_query = np.concatenate([points_query, np.zeros((len(points_query), 1))], axis=1)
    d, idx = cKDTree(points_seed).query(points_query, k=2)
    return idx[:, 0], d


@pytest.mark.parametrize("dim,n,M", [(2, 50, 96), (3, 60, 24)])
def test_voronoi_special_case(oracle_lib, dim, n, M):
    """A_i = Id and w = 0 give the Voronoi diagram (Section 2.1, case (i))."""
    inst = S.custom(dim, n, M, seed=10 + dim, iso=True)
    lab, best, second = O.assign(inst, np.zeros(n))
    kd, d = _kd_labels(inst.x, O.pixel_centres(inst))
    ok = (d[:, 1] ** 2 - d[:, 0] ** 2) > 1e-10
    assert ok.mean() > 0.99
    assert np.array_equal(lab[ok], kd[ok])


@pytest.mark.parametrize("dim,n,M", [(2, 50, 96), (3, 60, 24)])
def test_power_diagram_special_case(oracle_lib, dim, n, M):
    """A_i = Id gives the power diagram (case (ii)): nearest neighbour after
    lifting each seed to (x_i, sqrt(max w - w_i))."""
    inst = S.custom(dim, n, M, seed=20 + dim, iso=True)
    w = np.random.default_rng(1).uniform(-0.01, 0.01, n)
    lab, best, second = O.assign(inst, w)
    kd, d = _kd_labels(inst.x, O.pixel_centres(inst), np.sqrt(w.max() - w))
    ok = (d[:, 1] ** 2 - d[:, 0] ** 2) > 1e-10
    assert ok.mean() > 0.99
    assert np.array_equal(lab[ok], kd[ok])


def test_common_matrix_reduces_to_power_diagram(oracle_lib):
    """A_i = A for all i: y -> L^T y with A = L L^T maps it to a power
    diagram (and A = c Id to a scaled one)."""
    inst = S.custom(2, 40, 80, seed=7)
    A = np.array([[2.5, 0.7], [0.7, 0.6]])
    inst.A = np.broadcast_to(A, (inst.n, 2, 2)).copy()
    w = np.random.default_rng(2).uniform(-0.02, 0.02, inst.n)
    lab, _, _ = O.assign(inst, w)
    L = np.linalg.cholesky(A)
    kd, d = _kd_labels(inst.x @ L, O.pixel_centres(inst) @ L, np.sqrt(w.max() - w))
    ok = (d[:, 1] ** 2 - d[:, 0] ** 2) > 1e-10
    assert np.array_equal(lab[ok], kd[ok])


def test_two_seeds_straight_boundary(oracle_lib):
    """Two seeds with the same A: the boundary is the line
    2 y^T A (x2 - x1) = x2^T A x2 - x1^T A x1 + w1 - w2."""
    inst = S.custom(2, 2, (120, 90), seed=3)
    A = np.array([[1.7, -0.4], [-0.4, 0.9]])
    inst.A = np.stack([A, A])
    w = np.array([0.013, -0.021])
    lab, _, _ = O.assign(inst, w)
    y = O.pixel_centres(inst)
    x1, x2 = inst.x
    lhs = 2 * y @ (A @ (x2 - x1))
    rhs = x2 @ A @ x2 - x1 @ A @ x1 + w[0] - w[1]
    side = np.where(lhs > rhs, 1, 0)     # C_2 < C_1  <=>  lhs > rhs
    ok = np.abs(lhs - rhs) > 1e-12
    assert np.array_equal(lab[ok], side[ok])
    assert 0 < lab.sum() < len(lab)


def _mobius_disk(A, x1, x2, c, w):
    """Two seeds, A_1 = A, A_2 = c A, c > 1 (Moebius, case (iv) with
    weights): cell 2 is the A-disk |y - z|_A^2 < r^2."""
    z = (c * x2 - x1) / (c - 1.0)
    dx = x1 - x2
    r2 = c * (dx @ A @ dx) / (c - 1.0) ** 2 + (w[1] - w[0]) / (c - 1.0)
    return z, r2


def test_mobius_disk_closed_form(oracle_lib):
    A = np.array([[1.3, 0.25], [0.25, 0.9]])
    c = 4.0
    inst = S.Instance(2, (256, 256), (0.0, 0.0), (1.0, 1.0),
                      np.array([[0.3, 0.4], [0.55, 0.5]]), np.stack([A, c * A]),
                      np.array([0.8, 0.2]))
    w = np.array([0.0, 0.05])
    lab, _, _ = O.assign(inst, w)
    z, r2 = _mobius_disk(A, inst.x[0], inst.x[1], c, w)
    y = O.pixel_centres(inst)
    q = np.einsum("ja,ab,jb->j", y - z, A, y - z)
    ok = np.abs(q - r2) > 1e-12
    assert np.array_equal(lab[ok], (q < r2)[ok].astype(np.int32))
    area = np.pi * r2 / np.sqrt(np.linalg.det(A))
    assert abs(lab.sum() * O.pixel_volume(inst) - area) < 5e-3 * area


# ---------------------------------------------------------- invariances --

def test_invariances(oracle_lib):
    inst = S.custom(2, 30, 64, seed=11)
    w = np.random.default_rng(3).uniform(-0.01, 0.01, inst.n)
    lab, best, second = O.assign(inst, w)
    ok = _gap_ok(best, second)
    # w -> w + c leaves the diagram unchanged (g depends on w only up to a constant)
    lab_c, _, _ = O.assign(inst, w + 0.37)
    assert np.array_equal(lab[ok], lab_c[ok])
    # (A, w) -> (2A, 2w) scales every cost by an exact power of two
    inst2 = S.Instance(2, inst.grid, inst.lo, inst.hi, inst.x, 2.0 * inst.A, inst.v)
    lab2, _, _ = O.assign(inst2, 2.0 * w)
    assert np.array_equal(lab, lab2)
    # a permutation of the seeds relabels the cells
    perm = np.random.default_rng(4).permutation(inst.n)
    inst3 = S.Instance(2, inst.grid, inst.lo, inst.hi, inst.x[perm], inst.A[perm], inst.v[perm])
    lab3, _, _ = O.assign(inst3, w[perm])
    assert np.array_equal(perm[lab3][ok], lab[ok])
    # rotating seeds and matrices by 90 degrees about the centre of the
    # square permutes the pixels: (k0, k1) -> (M - 1 - k1, k0)
    Rm = np.array([[0.0, -1.0], [1.0, 0.0]])
    xr = (inst.x - 0.5) @ Rm.T + 0.5
    Ar = Rm @ inst.A @ Rm.T
    inst4 = S.Instance(2, inst.grid, inst.lo, inst.hi, xr, Ar, inst.v)
    lab4, _, _ = O.assign(inst4, w)
    M = inst.grid[0]
    k0, k1 = np.divmod(np.arange(M * M), M)
    rot_index = (M - 1 - k1) * M + k0
    ok4 = ok & _gap_ok(*O.assign(inst4, w)[1:])[rot_index]
    assert np.array_equal(lab4[rot_index][ok4], lab[ok4])


def test_conservation(oracle_lib):
    for dim, M in ((2, 50), (3, 14)):
        inst = S.custom(dim, 37, M, seed=5, sigma=0.4)
        w = np.random.default_rng(5).uniform(-0.01, 0.01, inst.n)
        ev = O.evaluate(inst, w)
        assert ev.counts.sum() == inst.J
        assert abs(ev.grad.sum()) < 1e-14


# -------------------------------------------------- objective, gradient --

def test_supergradient_inequality_and_finite_differences(oracle_lib):
    """g~ is concave and piecewise linear (a linear term plus a sum of
    minima of affine functions of w), so v - m|P| is a supergradient:
    g~(w + h d) <= g~(w) + h <grad, d> for every h, d; and a central
    difference equals the gradient up to the pixels that switch cell."""
    inst = S.custom(2, 12, 40, seed=8)
    rng = np.random.default_rng(6)
    w = rng.uniform(-0.01, 0.01, inst.n)
    ev = O.evaluate(inst, w)
    viol = 0
    for _ in range(60):
        d = rng.standard_normal(inst.n)
        for h in (1e-1, 1e-3, 1e-6):
            gp = O.evaluate(inst, w + h * d).g
            viol += gp > ev.g + h * (ev.grad @ d) + 1e-14
    assert viol == 0
    P = O.pixel_volume(inst)
    h = 1e-7
    for k in range(inst.n):
        e = np.zeros(inst.n)
        e[k] = 1.0
        lp, _, _ = O.assign(inst, w + h * e)
        lm, _, _ = O.assign(inst, w - h * e)
        flips = int(np.sum(lp != lm))
        fd = (O.evaluate(inst, w + h * e).g - O.evaluate(inst, w - h * e).g) / (2 * h)
        assert abs(fd - ev.grad[k]) <= flips * P / h + 1e-7


def test_objective_is_eq_2_7_cell_by_cell(oracle_lib):
    """The oracle sums min_i C_ij over pixels; eq. (2.7) sums per cell the
    (v_i - m_i|P|) w_i term and the |P| |y_j - x_i|^2_{A_i} integral term.
    They are the same number."""
    inst = S.custom(2, 20, 70, seed=9, sigma=0.3)
    w = np.random.default_rng(7).uniform(-0.01, 0.01, inst.n)
    lab, C = R.assign(inst, w)
    P = O.pixel_volume(inst)
    y = O.pixel_centres(inst)
    g = 0.0
    for i in range(inst.n):
        sel = lab == i
        d = y[sel] - inst.x[i]
        g += (inst.v[i] - sel.sum() * P) * w[i] + P * np.einsum("ja,ab,jb->", d, inst.A[i], d)
    assert abs(O.evaluate(inst, w).g - g) < 1e-13


# ------------------------------------------------------------ the solver --

def test_lattice_is_optimal_at_zero(oracle_lib):
    """4 seeds at the centres of the quarters, A = Id, v = 1/4: W = 0 is
    optimal, so Algorithm 2 stops at its first evaluation."""
    x = np.array([[0.25, 0.25], [0.75, 0.25], [0.25, 0.75], [0.75, 0.75]])
    inst = S.Instance(2, (64, 64), (0.0, 0.0), (1.0, 1.0), x,
                      np.broadcast_to(np.eye(2), (4, 2, 2)).copy(), np.full(4, 0.25))
    w, rep = O.fit_weights(inst)
    assert rep.converged and rep.iters == 0 and rep.evals == 1
    assert rep.crit == 0.0


def test_two_seed_fit_hits_the_closed_form_interval(oracle_lib):
    """Two seeds on a horizontal line with a common A: the cell boundary is
    the line of test_two_seeds_straight_boundary.  With A diagonal it is a
    vertical line x = b(w1 - w2); the fit must put b within the band of
    columns whose area errors are under eps."""
    A = np.diag([1.0, 1.0])
    x = np.array([[0.2, 0.5], [0.8, 0.5]])
    v = np.array([0.3, 0.7])
    M = 200
    inst = S.Instance(2, (M, M), (0.0, 0.0), (1.0, 1.0), x, np.stack([A, A]), v)
    w, rep = O.fit_weights(inst, eps=0.01)
    assert rep.converged
    # boundary abscissa from 2 y.A(x2 - x1) = x2.A.x2 - x1.A.x1 + w1 - w2
    dx = x[1] - x[0]
    b = (x[1] @ x[1] - x[0] @ x[0] + w[0] - w[1]) / (2 * dx[0])
    # cell 1 = the columns with centre < b: area = ceil(b M - 1/2) / M
    area1 = np.ceil(b * M - 0.5) / M
    assert abs(area1 - v[0]) < 0.01 * v[0]
    assert abs((1 - area1) - v[1]) < 0.01 * v[1]


def test_fit_is_certified_by_a_recount(oracle_lib):
    for inst in (S.make_c1(), S.custom(2, 60, 160, seed=1, sigma=0.3, amax=3.0),
                 S.custom(3, 30, 40, seed=2, sigma=0.2)):
        w, rep = O.fit_weights(inst, eps=0.01)
        assert rep.converged, rep
        lab = R.assign(inst, w)[0]      # recount with the independent brute force
        counts = np.bincount(lab, minlength=inst.n)
        rel = np.abs(inst.v - counts * O.pixel_volume(inst)) / inst.v
        assert rel.max() < 0.01
        assert rel.max() == pytest.approx(rep.crit, abs=1e-15)


def test_lloyd_fixed_point(oracle_lib):
    """The 4-seed lattice is a fixed point of Algorithm 3: every seed is the
    discrete centroid of its cell."""
    x = np.array([[0.25, 0.25], [0.75, 0.25], [0.25, 0.75], [0.75, 0.75]])
    inst = S.Instance(2, (64, 64), (0.0, 0.0), (1.0, 1.0), x,
                      np.broadcast_to(np.eye(2), (4, 2, 2)).copy(), np.full(4, 0.25))
    x1, w1, rep = O.lloyd_step(inst, x, np.zeros(4))
    assert rep.converged
    assert np.array_equal(x1, x)


def test_lloyd_centroids_are_cell_means(oracle_lib):
    inst = S.custom(2, 15, 48, seed=12)
    w = np.zeros(inst.n)
    x1, w1, rep = O.lloyd_step(inst, inst.x, w)
    lab, _ = R.assign(inst, w1)
    y = O.pixel_centres(inst)
    for i in range(inst.n):
        sel = lab == i
        expect = y[sel].mean(axis=0) if sel.any() else inst.x[i]
        np.testing.assert_allclose(x1[i], expect, rtol=0, atol=1e-14)


def test_lbfgs_matches_scipy_on_a_smooth_quadratic(oracle_lib):
    """On a smooth strictly convex quadratic the solver reaches the unique
    minimiser that scipy's L-BFGS-B also finds."""
    from scipy.optimize import minimize
    rng = np.random.default_rng(0)
    n = 30
    B = rng.standard_normal((n, n))
    Q = B @ B.T / n + np.eye(n)
    b = rng.standard_normal(n)
    b -= b.mean()  # keep the minimiser reachable inside the sum-zero gauge
    Q = Q - Q.mean(axis=0, keepdims=True) - Q.mean(axis=1, keepdims=True) + Q.mean() \
        + np.ones((n, n)) / n
    fun = lambda w: (0.5 * w @ Q @ w - b @ w, Q @ w - b)

    def fg(w):
        f, g = fun(w)
        return f, g, np.abs(g).max()

    w, rep = O.lbfgs(fg, np.zeros(n), eps=1e-10, gamma0=0.5, max_evals=5000)
    assert rep.converged
    ref = minimize(fun, np.zeros(n), jac=True, method="L-BFGS-B",
                   options={"gtol": 1e-12, "ftol": 1e-15, "maxiter": 10000})
    exact = np.linalg.solve(Q, b)
    np.testing.assert_allclose(w, exact, atol=1e-8)
    np.testing.assert_allclose(ref.x, exact, atol=1e-6)


def test_two_loop_secant_identity(oracle_lib):
    """The L-BFGS inverse-Hessian satisfies the newest secant equation
    H y_k = s_k whatever the older pairs and the initial scale."""
    rng = np.random.default_rng(1)
    n, m = 12, 5
    B = rng.standard_normal((n, n))
    Q = B @ B.T + n * np.eye(n)
    S_ = rng.standard_normal((m, n))
    Y_ = S_ @ Q
    for gamma in (0.37, 2.0):
        r = O.two_loop(S_, Y_, gamma, Y_[-1])
        np.testing.assert_allclose(r, S_[-1], rtol=1e-11, atol=1e-12)
    # with no pairs the matrix is gamma * Id
    q = rng.standard_normal(n)
    np.testing.assert_allclose(O.two_loop(np.zeros((0, n)), np.zeros((0, n)), 0.5, q), 0.5 * q)


# ------------------------------------------------------- the resolution --

def _table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1_resolution.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(tuple(int(t) for t in line.split()))
    return rows


def test_table1_reproduced_by_eq_2_9(oracle_lib):
    rows = _table1()
    assert len(rows) == 18
    for D, N, M in rows:
        assert round(O.resolution_lower_bound(D, N, 0.01)) == M, (D, N, M)


def test_eq_2_10_is_about_twice_table1_single_phase(oracle_lib):
    """The caption of Table 1: twice the lower bound usually suffices; for
    equal volumes (2.10) reads M > 2 (N/eps)^(1/D).  The smallest-integer
    claim is checked in exact rational arithmetic on the decimal inputs
    (eps = 1/100, v = 1/N), where ties such as N = 10^4 in 2D are exact."""
    from fractions import Fraction
    for D, N, M in _table1():
        Mc = O.choose_resolution(D, 0.01, 1.0 / N, 1.0)
        assert abs(Mc - 2 * M) <= 2, (D, N, Mc, M)
        rhs = Fraction(1, 100) / 2 ** D / N
        assert Fraction(1, Mc ** D) < rhs
        assert Fraction(1, (Mc - 1) ** D) >= rhs
    # the 3D single-phase N = 10^4 case is exactly on a tie at M = 200
    assert O.choose_resolution(3, 0.01, 1e-4, 1.0) == 201
    assert O.choose_resolution(2, 0.01, 1e-4, 1.0) == 2001
    # the box measure enters through |P| = |Omega| / M^D
    assert O.choose_resolution(2, 0.01, 4 * 3.1e-4, 4.0) == O.choose_resolution(2, 0.01, 3.1e-4, 1.0)


# ------------------------------------------------ warm-start network (O3)

def test_mlp_gradient_matches_central_differences():
    """The back-propagated gradient of the FP64 reference network against
    central differences of its loss (an independent pin of the formulas)."""
    from oracle import mlp
    rng = np.random.default_rng(0)
    p = mlp.init_params(1).astype(np.float64)
    p += 0.01 * rng.standard_normal(p.size)        # non-zero biases too
    X = rng.standard_normal((9, mlp.N_FEAT))
    t = rng.standard_normal(9)
    loss, g = mlp.loss_and_grad(p, X, t)
    idx = rng.choice(p.size, 60, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros(p.size)
        e[k] = h
        fd = (mlp.loss_and_grad(p + e, X, t)[0] - mlp.loss_and_grad(p - e, X, t)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])
    assert mlp.n_params() == p.size


def _torch_network(params):
    """The same network built from torch.nn layers in float64: each layer's
    weight is the transpose of the flat vector's W[in][out] block."""
    import torch
    from oracle import mlp
    mods = []
    k = 0
    for li, (i, o) in enumerate(mlp.LAYERS):
        lin = torch.nn.Linear(i, o, dtype=torch.float64)
        W = np.asarray(params[k:k + i * o], np.float64).reshape(i, o)
        k += i * o
        b = np.asarray(params[k:k + o], np.float64)
        k += o
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(W.T.copy()))
            lin.bias.copy_(torch.from_numpy(b))
        mods.append(lin)
        if li < len(mlp.LAYERS) - 1:
            mods.append(torch.nn.ReLU())
    return torch.nn.Sequential(*mods)


def test_mlp_forward_and_gradient_match_torch_nn():
    """The reference network against torch.nn layers built from the same
    flat vector (ReLU after every hidden layer, none after the last), and its
    back-propagated gradient against torch autograd of the same loss."""
    import torch
    from oracle import mlp
    rng = np.random.default_rng(11)
    p = mlp.init_params(4).astype(np.float64) + 0.02 * rng.standard_normal(mlp.n_params())
    X = rng.standard_normal((33, mlp.N_FEAT))
    t = rng.standard_normal(33)
    y, acts = mlp.forward(p, X)
    net = _torch_network(p)
    Xt = torch.from_numpy(X)
    yt = net(Xt)[:, 0]
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)
    # the output layer is linear: negative outputs survive
    assert np.any(y < 0)
    loss, g = mlp.loss_and_grad(p, X, t)
    lt = torch.mean((yt - torch.from_numpy(t)) ** 2)
    lt.backward()
    assert loss == pytest.approx(float(lt.detach()), rel=1e-12)
    flat = []
    for m in net:
        if isinstance(m, torch.nn.Linear):
            flat += [m.weight.grad.numpy().T.ravel(), m.bias.grad.numpy()]
    np.testing.assert_allclose(g, np.concatenate(flat), rtol=1e-10, atol=1e-13)


def test_mlp_adam_matches_torch_over_several_steps():
    """Adam with bias correction against torch.optim.Adam (float64) over
    eight steps with changing gradients: the bias-correction factors
    1 - beta^step differ at every step."""
    import torch
    from oracle import mlp
    rng = np.random.default_rng(12)
    p = rng.standard_normal(64)
    m = np.zeros(64)
    v = np.zeros(64)
    pt = torch.nn.Parameter(torch.from_numpy(p.copy()))
    opt = torch.optim.Adam([pt], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 9):
        g = rng.standard_normal(64) * (1.0 + step)
        p, m, v = mlp.adam_step(p, g, m, v, step, 3e-3)
        opt.zero_grad()
        pt.grad = torch.from_numpy(g.copy())
        opt.step()
        np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_mlp_adam_matches_the_published_update():
    """One Adam step from zero moments moves every parameter by lr*sign(g)
    (bias correction makes mh/sqrt(vh) = sign(g) up to eps)."""
    from oracle import mlp
    rng = np.random.default_rng(2)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = mlp.adam_step(p, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    np.testing.assert_allclose(p1, p - 1e-3 * np.sign(g), rtol=0, atol=1e-3 * 1e-8 / np.abs(g).min() * 2)


def test_knn_features_brute_force():
    """The pooled features against a per-seed loop over sorted distances."""
    from oracle import mlp
    inst = S.custom(2, 40, 8, seed=3, sigma=0.3)
    F = mlp.features(inst.x, inst.A, inst.v)
    n = inst.n
    for i in (0, 7, 39):
        d = [(float(np.sum((inst.x[j] - inst.x[i]) ** 2)), j) for j in range(n) if j != i]
        nb = [j for _, j in sorted(d)[:16]]
        dx = inst.x[nb] - inst.x[i]
        assert F[i, 6] == pytest.approx(np.sqrt(n) * dx[:, 0].mean(), rel=1e-12)
        assert F[i, 11] == pytest.approx((n * inst.v[nb]).mean(), rel=1e-12)
        q = np.mean([dd @ inst.A[i] @ dd for dd in dx]) * n
        assert F[i, 12] == pytest.approx(q, rel=1e-12)
        q2 = np.mean([dd @ inst.A[j] @ dd for dd, j in zip(dx, nb)]) * n
        assert F[i, 13] == pytest.approx(q2, rel=1e-12)
        # the pooled second offset coordinate and the pooled upper triangle
        # of the neighbours' matrices
        assert F[i, 7] == pytest.approx(np.sqrt(n) * dx[:, 1].mean(), rel=1e-12)
        assert F[i, 8] == pytest.approx(np.mean([inst.A[j][0, 0] for j in nb]), rel=1e-12)
        assert F[i, 9] == pytest.approx(np.mean([inst.A[j][0, 1] for j in nb]), rel=1e-12)
        assert F[i, 10] == pytest.approx(np.mean([inst.A[j][1, 1] for j in nb]), rel=1e-12)
        # the seed's own entries
        assert list(F[i, 0:6]) == [inst.x[i][0], inst.x[i][1], inst.A[i][0, 0], inst.A[i][0, 1],
                                   inst.A[i][1, 1], n * inst.v[i]]
    np.testing.assert_allclose(F[:, 14], np.sqrt(n) * np.minimum(inst.x[:, 0], 1 - inst.x[:, 0]))
    np.testing.assert_allclose(F[:, 15], np.sqrt(n) * np.minimum(inst.x[:, 1], 1 - inst.x[:, 1]))
    # on a non-unit box the boundary distance is scaled by sqrt(N / |Omega|)
    lo, hi = (0.5, -1.0), (2.5, 0.0)
    xs = np.column_stack([0.5 + 2.0 * np.random.default_rng(8).random(n),
                          -1.0 + np.random.default_rng(9).random(n)])
    Fb = mlp.features(xs, inst.A, inst.v, lo=lo, hi=hi)
    sc = np.sqrt(n / 2.0)
    for i in (0, 11, 39):
        assert Fb[i, 14] == pytest.approx(sc * min(xs[i, 0] - 0.5, 2.5 - xs[i, 0]), rel=1e-12)
        assert Fb[i, 15] == pytest.approx(sc * min(xs[i, 1] + 1.0, 0.0 - xs[i, 1]), rel=1e-12)


def test_bf16_rounding_and_reference_inference():
    """BF16 rounding keeps 8 significant bits, ties to even; the reference
    BF16 inference equals the FP64 network when every weight, input and
    hidden value is already a BF16 number."""
    from oracle import mlp
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -8 + 2.0 ** -20,
                     -1.5, 3.0e38, 2.0 ** -130])
    want = np.array([1.0, 1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7, -1.5, 2.99684e38, 2.0 ** -130])
    got = mlp.to_bf16(vals)
    np.testing.assert_array_equal(got[[0, 1, 2, 3, 4, 6]], want[[0, 1, 2, 3, 4, 6]])
    assert abs(got[5] - 3.0e38) <= 2.0 ** -8 * 3.0e38
    # a sparse network of quarters on inputs in {-1, 0, 1}: two non-zero
    # weights per unit keep every hidden value a short dyadic fraction, so
    # every value is exact in BF16 and the two inferences agree exactly
    rng = np.random.default_rng(3)
    parts = []
    for i, o in mlp.LAYERS:
        W = np.zeros((i, o))
        for c in range(o):
            W[rng.choice(i, 2, replace=False), c] = rng.choice([-0.25, 0.25], 2)
        parts += [W.ravel(), np.zeros(o)]
    p = np.concatenate(parts)
    X = rng.integers(-1, 2, (7, mlp.N_FEAT)).astype(np.float64)
    y64, _ = mlp.forward(p, X)
    yb, sc = mlp.forward_bf16(p, X)
    np.testing.assert_array_equal(yb, y64)
    assert np.all(sc >= np.abs(yb))
    # otherwise BF16 inference differs from FP64 by about 2^-8 of the scale
    p2 = mlp.init_params(1).astype(np.float64)
    X2 = rng.standard_normal((50, mlp.N_FEAT))
    y64, _ = mlp.forward(p2, X2)
    yb, sc = mlp.forward_bf16(p2, X2)
    assert 0 < np.max(np.abs(yb - y64) / sc) < 2.0 ** -6


def test_pooled_deficit_features_brute_force():
    """The deficit and its repeated neighbour means against explicit loops;
    a constant deficit stays constant under the means."""
    from oracle import mlp
    inst = S.custom(2, 40, 8, seed=4)
    n = inst.n
    rng = np.random.default_rng(5)
    d = rng.standard_normal(n)
    F = mlp.features(inst.x, inst.A, inst.v, d=d)
    nbs = []
    for i in range(n):
        dist = [(float(np.sum((inst.x[j] - inst.x[i]) ** 2)), j) for j in range(n) if j != i]
        nbs.append([j for _, j in sorted(dist)[:16]])
    p = list(d)
    np.testing.assert_array_equal(F[:, 16], d)
    for h in range(3):
        p = [sum(p[j] for j in nbs[i]) / 16.0 for i in range(n)]
        np.testing.assert_allclose(F[:, 17 + h], p, rtol=1e-12, atol=1e-14)
    Fc = mlp.features(inst.x, inst.A, inst.v, d=np.full(n, 2.5))
    np.testing.assert_allclose(Fc[:, 16:20], 2.5, rtol=1e-15)
    # the deficit is N times the gradient of a pass at W = 0; it sums to zero
    g0 = O.evaluate(inst, np.zeros(n)).grad
    assert abs(mlp.deficit(n, g0).sum()) < 1e-9


# ------------------------------------------- pixel weights and refinement

def test_full_weights_equal_the_unweighted_problem(oracle_lib):
    """Every pixel at weight 255 is the unweighted problem: the same
    objective, gradient and centroids, counts scaled by 255."""
    inst = S.custom(2, 25, (50, 37), seed=31, sigma=0.3)
    w = np.random.default_rng(1).uniform(-0.004, 0.004, inst.n)
    a = O.evaluate(inst, w)
    mi = S.masked(inst, np.full(inst.J, 255, np.uint8))
    np.testing.assert_array_equal(mi.v, inst.v)
    b = O.evaluate(mi, w)
    np.testing.assert_array_equal(b.counts, 255 * a.counts)
    assert b.g == pytest.approx(a.g, rel=1e-13)
    np.testing.assert_allclose(b.grad, a.grad, rtol=0, atol=1e-15)
    np.testing.assert_allclose(b.centroids, a.centroids, rtol=0, atol=1e-14)


def test_rectangular_mask_equals_the_sub_box(oracle_lib):
    """Weight 255 on an aligned sub-rectangle, 0 elsewhere, is the problem
    on that sub-box with the same pixels: equal counts, objective and
    centroids (the general-tessellation objective of Section 2.3)."""
    inst = S.custom(2, 18, (40, 50), seed=32)
    s0, s1 = 1.0 / 40, 1.0 / 50
    q = np.zeros((40, 50), np.uint8)
    q[10:30, 5:45] = 255
    sub_lo, sub_hi = (10 * s0, 5 * s1), (30 * s0, 45 * s1)
    x = np.column_stack([sub_lo[0] + (sub_hi[0] - sub_lo[0]) * np.random.default_rng(2).random(18),
                         sub_lo[1] + (sub_hi[1] - sub_lo[1]) * np.random.default_rng(3).random(18)])
    measure = 20 * 40 * s0 * s1
    v = np.full(18, measure / 18)
    v[0] += measure - v.sum()
    full = S.Instance(2, (40, 50), (0.0, 0.0), (1.0, 1.0), x, inst.A, v, mass=q.reshape(-1))
    sub = S.Instance(2, (20, 40), sub_lo, sub_hi, x, inst.A, v)
    w = np.random.default_rng(4).uniform(-1e-3, 1e-3, 18)
    a = O.evaluate(full, w)
    b = O.evaluate(sub, w)
    np.testing.assert_array_equal(a.counts, 255 * b.counts)
    assert a.g == pytest.approx(b.g, rel=1e-12)
    np.testing.assert_allclose(a.grad, b.grad, rtol=0, atol=1e-15)
    np.testing.assert_allclose(a.centroids, b.centroids, rtol=0, atol=1e-13)
    assert O.domain_measure(full) == pytest.approx(measure, rel=1e-14)


def test_weighted_objective_identities(oracle_lib):
    """A disk domain with fractional boundary pixels: the weights sum to
    the counts, the gradient sums to zero when the volumes sum to the
    domain measure, and the objective is concave (supergradient
    inequality) in random directions."""
    inst = S.custom(2, 30, (64, 64), seed=33, sigma=0.3)
    q = S.disk_weights(inst.grid, inst.lo, inst.hi, (0.5, 0.45), 0.41)
    assert 0 < np.sum((q > 0) & (q < 255))
    mi = S.masked(inst, q)
    rng = np.random.default_rng(5)
    w = rng.uniform(-2e-3, 2e-3, inst.n)
    e = O.evaluate(mi, w)
    assert int(e.counts.sum()) == int(q.astype(np.int64).sum())
    assert abs(e.grad.sum()) < 1e-14
    for _ in range(20):
        d = rng.standard_normal(inst.n)
        h = 10 ** rng.uniform(-5, -2)
        assert O.evaluate(mi, w + h * d).g <= e.g + h * float(e.grad @ d) + 1e-15


def test_refinement_reaches_the_tolerance(oracle_lib):
    """The last step of Algorithm 2: on a grid too coarse for 1 % the fit
    fails; with refinement it restarts on a finer grid (at least the (2.10)
    pixel size) and converges, certified by a recount on that grid."""
    inst = S.custom(2, 40, (20, 20), seed=34, sigma=0.3)
    w, rep = O.fit_weights(inst, eps=0.01, max_evals=300)
    assert not rep.converged
    w2, rep2, grid = O.fit_weights_refine(inst, eps=0.01, max_refine=4, max_evals=300)
    assert rep2.converged
    assert grid[0] > 20 and grid[0] == grid[1]
    M = O.choose_resolution(2, 0.01, float(inst.v.min()), 1.0)
    assert grid[0] >= M
    fine = S.Instance(2, grid, inst.lo, inst.hi, inst.x, inst.A, inst.v)
    assert O.evaluate(fine, w2).maxrel < 0.01


# ---------------------------------------------- costs beyond |.|^2_A (p) --

def _with_power(inst, p):
    import dataclasses
    return dataclasses.replace(inst, power=p)


@pytest.mark.parametrize("p", [1, 3, 4])
@pytest.mark.parametrize("dim,n,M", [(2, 50, 96), (3, 60, 24)])
def test_power_costs_at_zero_weights_are_voronoi(oracle_lib, p, dim, n, M):
    """With w = 0 every increasing function of the distance gives the same
    cells: |.|_A^p with A = Id is the Voronoi diagram (KD-tree) for any p."""
    inst = _with_power(S.custom(dim, n, M, seed=10 + dim, iso=True), p)
    lab, best, second = O.assign(inst, np.zeros(n))
    kd, d = _kd_labels(inst.x, O.pixel_centres(inst))
    ok = (d[:, 1] ** 2 - d[:, 0] ** 2) > 1e-10
    assert ok.mean() > 0.99
    assert np.array_equal(lab[ok], kd[ok])


@pytest.mark.parametrize("w1,w2", [(0.06, 0.0), (0.0, 0.11), (-0.02, 0.05)])
def test_norm_cost_two_seeds_hyperbola(oracle_lib, w1, w2):
    """p = 1, A = Id, two seeds: the boundary |y - x1| - |y - x2| = w1 - w2
    is a branch of the hyperbola with foci x1, x2 and semi-axis
    a = (w1 - w2) / 2.  In coordinates u along x2 - x1 and v across it, from
    the midpoint, b^2 = c^2 - a^2 with c = |x2 - x1| / 2, the first cell is
    u < a sqrt(1 + v^2 / b^2) (closed form; pixels within 1e-9 of the branch
    excluded)."""
    x = np.array([[0.31, 0.44], [0.66, 0.58]])
    A = np.broadcast_to(np.eye(2), (2, 2, 2)).copy()
    inst = S.Instance(2, (180, 150), (0.0, 0.0), (1.0, 1.0), x, A, np.full(2, 0.5), power=1)
    w = np.array([w1, w2])
    lab, _, _ = O.assign(inst, w)
    y = O.pixel_centres(inst)
    mid = 0.5 * (x[0] + x[1])
    e = (x[1] - x[0]) / np.linalg.norm(x[1] - x[0])
    f = np.array([-e[1], e[0]])
    u, v = (y - mid) @ e, (y - mid) @ f
    c = 0.5 * np.linalg.norm(x[1] - x[0])
    a = 0.5 * (w1 - w2)
    b2 = c * c - a * a
    assert b2 > 0
    branch = a * np.sqrt(1.0 + v * v / b2)
    cell0 = u < branch
    ok = np.abs(u - branch) > 1e-9
    assert 0.1 < cell0.mean() < 0.9
    assert np.array_equal(lab[ok] == 0, cell0[ok])


@pytest.mark.parametrize("p", [1, 3, 4])
def test_power_cost_scaling_invariance(oracle_lib, p):
    """(A, w) -> (4A, 2^p w) multiplies every cost by 2^p exactly (the norm
    doubles), so the labels are identical bit for bit, and the objective
    scales by 2^p."""
    inst = _with_power(S.custom(2, 30, (70, 60), seed=31), p)
    w = np.random.default_rng(3).uniform(-0.02, 0.02, inst.n)
    lab, b, s = O.assign(inst, w)
    import dataclasses
    big = dataclasses.replace(inst, A=4.0 * inst.A)
    lab2, b2, s2 = O.assign(big, (2.0 ** p) * w)
    assert np.array_equal(lab, lab2)
    assert np.array_equal(b2, (2.0 ** p) * b)
    assert O.evaluate(big, (2.0 ** p) * w).g == (2.0 ** p) * O.evaluate(inst, w).g


@pytest.mark.parametrize("p", [1, 4])
def test_power_cost_supergradient(oracle_lib, p):
    """The objective stays concave for any cost (a linear term plus minima
    of affine functions of w): v - m|P| is a supergradient."""
    inst = _with_power(S.custom(2, 12, 40, seed=8), p)
    rng = np.random.default_rng(6)
    w = rng.uniform(-0.05, 0.05, inst.n)
    ev = O.evaluate(inst, w)
    viol = 0
    for _ in range(40):
        d = rng.standard_normal(inst.n)
        for h in (1e-1, 1e-3, 1e-6):
            gp = O.evaluate(inst, w + h * d).g
            viol += gp > ev.g + h * (ev.grad @ d) + 1e-14
    assert viol == 0


def test_power_cost_fit_is_certified(oracle_lib):
    """Algorithm 2 with the norm cost (p = 1) reaches 1 % by a recount."""
    inst = _with_power(S.custom(2, 20, 128, seed=9, sigma=0.3), 1)
    w, rep = O.fit_weights(inst, eps=0.01)
    assert rep.converged
    assert O.evaluate(inst, w).maxrel < 0.01
