"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these tests retypes the oracle's own formulas: each compares it with a
closed form, a brute-force definition, a library routine, an invariance or a
hand-worked example, chosen so that a dropped term, a wrong sign, a wrong
index or a transposed operand in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
from paper_1812_09869_amd import synth


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


# ---------------------------------------------------------------------------
# Input similarities (section "Similarities in the input space")
# ---------------------------------------------------------------------------

def test_sqdist_matches_library_and_invariances():
    x = _rng(1).standard_normal((37, 7)) * 3.0
    d = oracle.sqdist(x)
    np.testing.assert_allclose(d, cdist(x, x, "sqeuclidean"), rtol=1e-13, atol=1e-12)
    assert np.all(np.diag(d) == 0.0)
    q, _ = np.linalg.qr(_rng(2).standard_normal((7, 7)))
    d2 = oracle.sqdist(x @ q.T + 11.0)
    np.testing.assert_allclose(d2, d, rtol=1e-11, atol=1e-10)


# ---------------------------------------------------------------------------
# Calibration (Eqs. 1-2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,dim,perp", [(17, 3, 5.0), (40, 10, 12.5), (64, 50, 30.0)])
def test_entropy_brute_force(n, dim, perp):
    """Entropy of p_{.|i}, recomputed from its definition, equals ln(perplexity) to 1e-10."""
    x = _rng(n).standard_normal((n, dim)) * 2.0
    st = oracle.calibrate(x, perp)
    assert np.all(st.iters > 0)
    d = cdist(x, x, "sqeuclidean")
    for i in range(n):
        mask = np.arange(n) != i
        logits = -st.beta[i] * d[i, mask]
        p = np.exp(logits - logits.max())
        p /= p.sum()
        h = -np.sum(p * np.log(p))
        assert abs(h - math.log(perp)) <= 1e-10
        # 2^{H in bits} is the perplexity of Eq. 2
        assert abs(2.0 ** (h / math.log(2.0)) - perp) <= 1e-9 * perp


def _binary_entropy_inverse(target):
    """p in (1/2, 1) with -p ln p - (1-p) ln(1-p) = target, by bisection on p."""
    lo, hi = 0.5, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        h = -mid * math.log(mid) - (1 - mid) * math.log1p(-mid)
        if h > target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("perp", [1.2, 1.5, 1.9])
def test_three_points_closed_form(perp):
    """Row with two neighbours at d_a < d_b: p_a = 1/(1+exp(-beta (d_b - d_a)))."""
    x = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, -2.5]])
    d_a, d_b = 1.0, 6.25
    pa = _binary_entropy_inverse(math.log(perp))
    beta_closed = math.log(pa / (1 - pa)) / (d_b - d_a)
    st = oracle.calibrate(x, perp, rows=[0])
    assert st.iters[0] > 0
    assert abs(st.beta[0] - beta_closed) <= 1e-9 * beta_closed
    assert st.m[0] == d_a


def test_equidistant_points_uniform_and_unreachable():
    """All neighbours equidistant: p_{j|i} = 1/(n-1) for any beta, so H = ln(n-1) (the
    maximum perplexity n-1 of Eq. 2); a lower target is unreachable and reported."""
    n = 9
    x = np.eye(n)  # every pair at squared distance 2
    st = oracle.calibrate(x, 4.0, max_iter=60)
    assert np.all(st.iters < 0)
    np.testing.assert_allclose(st.H, math.log(n - 1), rtol=0, atol=1e-14)
    P = oracle.joint_p(x, st)
    off = P[~np.eye(n, dtype=bool)]
    np.testing.assert_allclose(off, 1.0 / (n * (n - 1)), rtol=1e-14)


def test_scale_covariance():
    """X -> cX gives beta -> beta / c^2 and leaves P unchanged."""
    x = _rng(3).standard_normal((30, 5))
    c = 3.0
    s1 = oracle.calibrate(x, 8.0)
    s2 = oracle.calibrate(c * x, 8.0)
    np.testing.assert_allclose(s2.beta, s1.beta / c**2, rtol=1e-9)
    np.testing.assert_allclose(oracle.joint_p(c * x, s2), oracle.joint_p(x, s1), rtol=1e-8,
                               atol=1e-16)


def test_beta_decreases_with_perplexity():
    """Smaller beta means higher entropy (text after Eq. 1): beta is monotone in perplexity."""
    x = _rng(4).standard_normal((50, 6))
    betas = [oracle.calibrate(x, u).beta for u in (3.0, 6.0, 12.0, 24.0, 40.0)]
    for a, b in zip(betas, betas[1:]):
        assert np.all(b < a)


def test_calibrate_rows_matches_all_rows():
    x = _rng(5).standard_normal((80, 4))
    full = oracle.calibrate(x, 10.0)
    rows = np.array([79, 3, 40, 0])
    part = oracle.calibrate(x, 10.0, rows=rows)
    np.testing.assert_array_equal(part.beta, full.beta[rows])
    np.testing.assert_array_equal(part.S, full.S[rows])


# ---------------------------------------------------------------------------
# Joint P (Eq. 3)
# ---------------------------------------------------------------------------

def test_joint_p_properties():
    x, _ = synth.plain_small(300, seed=11)
    st = oracle.calibrate(x, 30.0)
    P = oracle.joint_p(x, st)
    n = P.shape[0]
    assert abs(P.sum() - 1.0) <= 1e-14 * n
    assert np.array_equal(P, P.T)
    assert np.all(np.diag(P) == 0.0)
    assert np.all(P.sum(axis=1) > 1.0 / (2 * n))
    # single entries agree with the full matrix
    ii = np.array([0, 5, 299, 17])
    jj = np.array([1, 5, 3, 250])
    si = oracle.calibrate(x, 30.0, rows=ii)
    sj = oracle.calibrate(x, 30.0, rows=jj)
    np.testing.assert_allclose(oracle.p_entries(x, ii, jj, si, sj), P[ii, jj], rtol=1e-13)


def test_p_rows_equal_rows_of_joint_p():
    """Rows of P formed from every row's statistics are the rows of the full P."""
    x, _ = synth.plain_small(300, seed=11)
    st = oracle.calibrate(x, 30.0)
    P = oracle.joint_p(x, st)
    rows = np.array([0, 17, 150, 299])
    pr = oracle.p_rows(x, rows, st)
    np.testing.assert_array_equal(pr, P[rows])
    assert np.all(pr[np.arange(rows.size), rows] == 0.0)


def test_p_entropy_term_closed_forms():
    """sum_{i != j, p > 0} p ln p: -ln 2 for two points (p = 1/2 each way, Eq. 3
    at n = 2), -ln(n(n - 1)) for the uniform P; zero entries and the diagonal
    add nothing."""
    assert abs(oracle.p_entropy_term(np.array([[0.0, 0.5], [0.5, 0.0]])) + math.log(2.0)) <= 1e-15
    n = 7
    P = np.full((n, n), 1.0 / (n * (n - 1)))
    np.fill_diagonal(P, 0.0)
    assert abs(oracle.p_entropy_term(P) + math.log(n * (n - 1))) <= 1e-14
    # three points with p_12 = p_21 = 1/2 and the rest zero: still -ln 2, and a
    # value on the diagonal is ignored
    P = np.zeros((3, 3))
    P[0, 1] = P[1, 0] = 0.5
    P[2, 2] = 0.3
    assert abs(oracle.p_entropy_term(P) + math.log(2.0)) <= 1e-15


def test_two_points():
    """n = 2: p_12 = p_21 = 1/2 for any X; q = 1/2 too, so g = 0 and KL = 0."""
    x = np.array([[0.3, -1.0, 2.0], [5.0, 1.0, 0.0]])
    st = oracle.calibrate(x, 1.0 + 1e-9, max_iter=5)
    P = oracle.joint_p(x, st)
    np.testing.assert_allclose(P, [[0, 0.5], [0.5, 0]], rtol=1e-15)
    y = np.array([[0.1, 0.2], [-3.0, 4.0]])
    g, _ = oracle.gradient(P, y)
    assert np.all(np.abs(g) < 1e-16)
    kl, _ = oracle.cost(P, y)
    assert abs(kl) < 1e-15


# ---------------------------------------------------------------------------
# Output side (Eqs. 4-6, 9)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small_problem():
    x, lab = synth.plain_small(120, seed=21)
    st = oracle.calibrate(x, 15.0)
    P = oracle.joint_p(x, st)
    y = synth.clustered_state(lab, seed=22, spread=3.0).astype(np.float64)
    return x, P, y


def test_z_matches_library(small_problem):
    _, _, y = small_problem
    w = 1.0 / (1.0 + cdist(y, y, "sqeuclidean"))
    np.fill_diagonal(w, 0.0)
    assert abs(oracle.z(y) - w.sum()) <= 1e-12 * w.sum()


def test_kl_matches_definition(small_problem):
    """KL of Eq. 5 computed from q_ij = w_ij / Z (Eq. 4), entry by entry."""
    _, P, y = small_problem
    w = 1.0 / (1.0 + cdist(y, y, "sqeuclidean"))
    np.fill_diagonal(w, 0.0)
    q = w / w.sum()
    mask = P > 0
    kl_def = np.sum(P[mask] * np.log(P[mask] / q[mask]))
    kl, cn = oracle.cost(P, y)
    assert kl > 0
    assert abs(kl - kl_def) <= 1e-12 * abs(kl_def)
    n = P.shape[0]
    h_pq = -np.sum(P[mask] * np.log(q[mask]))
    assert abs(cn - h_pq / math.log(n * (n - 1))) <= 1e-12
    # the average of q over the n(n-1) ordered pairs (Eq. 7)
    assert abs(q.sum() / (n * (n - 1)) - 1.0 / (n * (n - 1))) < 1e-18


def test_normalized_cost_near_one_at_random_start():
    """A random initial map gives a pseudo-normalised cost very close to 1 (Eq. 9)."""
    x, _ = synth.plain_small(400, seed=31)
    P = oracle.joint_p(x, oracle.calibrate(x, 30.0))
    y0 = synth.embedding_init(400, seed=32)
    _, cn = oracle.cost(P, y0)
    # "very close to 1": a given random map can sit slightly on either side of the
    # uniform reference, so the pin is two-sided
    assert abs(cn - 1.0) <= 1e-3


def test_gradient_finite_differences(small_problem):
    """Eq. 6 equals central differences of the KL cost (alpha = 1) to 1e-6 of max|g|.

    h = 1e-5 keeps both the O(h^2) truncation and the cancellation noise of the
    cost difference (~1e-16 KL / h) near 1e-11, far below the bound."""
    _, P, y = small_problem
    g, _ = oracle.gradient(P, y, 1.0)
    h = 1e-5
    rng = _rng(7)
    for i in rng.choice(y.shape[0], 12, replace=False):
        for c in range(2):
            yp = y.copy()
            ym = y.copy()
            yp[i, c] += h
            ym[i, c] -= h
            fd = (oracle.cost(P, yp)[0] - oracle.cost(P, ym)[0]) / (2 * h)
            assert abs(fd - g[i, c]) <= 1e-6 * np.abs(g).max()


def test_gradient_zero_sum_and_equivariance(small_problem):
    _, P, y = small_problem
    for alpha in (1.0, 12.0):
        g, _ = oracle.gradient(P, y, alpha)
        assert np.all(np.abs(g.sum(axis=0)) <= 1e-12 * np.abs(g).sum())
    th = 0.7
    r = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    g, z0 = oracle.gradient(P, y, 1.0)
    g2, z1 = oracle.gradient(P, y @ r.T + np.array([4.0, -2.0]), 1.0)
    np.testing.assert_allclose(g2, g @ r.T, rtol=1e-9, atol=1e-12 * np.abs(g).max())
    assert abs(z0 - z1) <= 1e-11 * z0


def test_exaggeration_is_linear_in_p(small_problem):
    """alpha multiplies only the attractive term: g(a) - g(0) = a (g(1) - g(0))."""
    _, P, y = small_problem
    g0, _ = oracle.gradient(P, y, 0.0)
    g1, _ = oracle.gradient(P, y, 1.0)
    g12, _ = oracle.gradient(P, y, 12.0)
    np.testing.assert_allclose(g12 - g0, 12.0 * (g1 - g0), rtol=1e-10,
                               atol=1e-13 * np.abs(g12).max())


def test_repulsion_rows(small_problem):
    _, P, y = small_problem
    g0, z0 = oracle.gradient(P, y, 0.0)
    rows = np.array([0, 7, 119])
    np.testing.assert_allclose(oracle.repulsion_rows(y, rows, z0), g0[rows], rtol=1e-12)


def test_gradient_rows_equal_gradient(small_problem):
    """Eq. 6 for listed rows from their rows of P and the global Z is the whole-map gradient."""
    _, P, y = small_problem
    rows = np.array([0, 7, 64, 119])
    for alpha in (1.0, 12.0):
        g, z0 = oracle.gradient(P, y, alpha)
        np.testing.assert_array_equal(oracle.gradient_rows(P[rows], y, rows, alpha, z0), g[rows])


def test_kl_rows_sum_to_kl(small_problem):
    """The per-row shares of Eq. 5 sum to the KL; each share is sum_j p ln(p / q)."""
    _, P, y = small_problem
    n = P.shape[0]
    z0 = oracle.z(y)
    shares = oracle.kl_rows(P, y, np.arange(n), z0)
    kl, _ = oracle.cost(P, y)
    assert abs(shares.sum() - kl) <= 1e-12 * kl
    w = 1.0 / (1.0 + cdist(y, y, "sqeuclidean"))
    q = w / z0
    i = 33
    mask = P[i] > 0
    mask[i] = False
    assert abs(shares[i] - np.sum(P[i, mask] * np.log(P[i, mask] / q[i, mask]))) <= 1e-13


def test_cost_invariances(small_problem):
    _, P, y = small_problem
    kl, cn = oracle.cost(P, y)
    th = 1.1
    r = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    kl2, cn2 = oracle.cost(P, y @ r.T - 3.0)
    assert abs(kl - kl2) <= 1e-11 * kl and abs(cn - cn2) <= 1e-11


# ---------------------------------------------------------------------------
# Update (Eq. 10, gains, momentum)
# ---------------------------------------------------------------------------

def test_step_hand_worked():
    """Two points at (0,0), (1,0) with p_12 = p_21 = 0.3 (a bare input to Eq. 6).

    w = 1/2, Z = 1, g_1 = 4 (0.3 - 0.5) 0.5 (-1, 0) = (0.4, 0), g_2 = (-0.4, 0).
    Gains from G = 1: g1x>0, U1x>0 -> same -> 0.8; g1y=0, U1y=0 -> same -> 0.8;
    g2x<0, U2x>0 -> differ -> 1.2; g2y=0, U2y<0 -> same -> 0.8.
    U <- 0.5 U - 200 G g; Y <- Y + U; then the mean is removed.
    """
    P = np.array([[0.0, 0.3], [0.3, 0.0]])
    y = np.array([[0.0, 0.0], [1.0, 0.0]])
    u = np.array([[0.1, 0.0], [0.1, -0.1]])
    gains = np.ones((2, 2))
    prm = oracle.StepParams(alpha=1.0, mu=0.5, eta=200.0, min_gain=0.01, recentre=True)
    g, zz = oracle.step(P, y, u, gains, prm, want_grad=True)
    assert zz == 1.0
    np.testing.assert_allclose(g, [[0.4, 0.0], [-0.4, 0.0]], rtol=1e-15, atol=1e-17)
    np.testing.assert_allclose(gains, [[0.8, 0.8], [1.2, 0.8]], rtol=1e-15)
    np.testing.assert_allclose(u, [[0.05 - 64.0, 0.0], [0.05 + 96.0, -0.05]], rtol=1e-15)
    y_before_centre = np.array([[-63.95, 0.0], [1.0 + 96.05, -0.05]])
    np.testing.assert_allclose(y, y_before_centre - y_before_centre.mean(axis=0), rtol=1e-14)


def test_gain_floor():
    P = np.array([[0.0, 0.5], [0.5, 0.0]])  # gradient is exactly zero here
    y = np.array([[0.0, 0.0], [1.0, 0.0]])
    u = np.zeros((2, 2))
    gains = np.full((2, 2), 0.011)
    oracle.step(P, y, u, gains, oracle.StepParams(1.0, 0.5, 200.0, min_gain=0.01))
    np.testing.assert_array_equal(gains, np.full((2, 2), 0.01))


def test_adaptive_eta_hand_worked():
    """Eq. 11 on a 3-point map with coordinate ranges 3 (x) and 4 (y).

    eta = ln(n - 1) * max(3, 4) / 2 = 2 ln 2; the embedding size (diagonal of
    the box) is the 3-4-5 hypotenuse. A base-2 or base-10 logarithm, n for
    n - 1, the diagonal or the smaller range in Eq. 11, or a missing halving
    all give other values.
    """
    y = np.array([[0.0, 0.0], [3.0, 1.0], [1.0, -3.0]])
    assert oracle.adaptive_eta(y) == pytest.approx(2.0 * math.log(2.0), rel=1e-15)
    assert oracle.embedding_size(y) == pytest.approx(5.0, rel=1e-15)


def test_adaptive_eta_invariances():
    """eta is translation and order invariant and scales with the map (Eq. 11)."""
    y = _rng(21).standard_normal((50, 2)) * 4.0
    e = oracle.adaptive_eta(y)
    assert oracle.adaptive_eta(y + [7.0, -3.0]) == pytest.approx(e, rel=1e-14)
    assert oracle.adaptive_eta(y[::-1].copy()) == e
    assert oracle.adaptive_eta(2.5 * y) == pytest.approx(2.5 * e, rel=1e-14)
    assert oracle.adaptive_eta(y[:, ::-1].copy()) == e
    s = oracle.embedding_size(y)
    assert oracle.embedding_size(3.0 * y + 1.0) == pytest.approx(3.0 * s, rel=1e-14)


def test_step_range_hand_worked():
    """Three collinear points (-1,0), (0,0), (1,0) with uniform p_ij = 1/6.

    w = 1/2 for the two unit pairs, 1/5 for the outer pair; Z = 2 (1/2 + 1/2 +
    1/5) = 2.4, q = 5/24 and 1/12. Eq. 6 for point 1:
    4 [(1/6 - 5/24)(1/2)(-1) + (1/6 - 1/12)(1/5)(-2)] = 4 (1/48 - 1/30) = -1/20,
    point 2 has zero gradient by symmetry and point 3 the opposite of point 1.
    Ranges 2 (x) and 0 (y): eta = ln 2 * 2 / 2 = ln 2 (Eq. 11). With
    mu = 0.8 and U_1 = (0.1, 0.2): U_1 <- (0.08 + 0.05 ln 2, 0.16),
    U_3 <- (-0.05 ln 2, 0); Y <- Y + U, then the mean is removed.
    """
    P = np.full((3, 3), 1.0 / 6.0)
    np.fill_diagonal(P, 0.0)
    y = np.array([[-1.0, 0.0], [0.0, 0.0], [1.0, 0.0]])
    u = np.array([[0.1, 0.2], [0.0, 0.0], [0.0, 0.0]])
    g, zz, eta = oracle.step_range(P, y, u, mu=0.8, want_grad=True)
    assert zz == pytest.approx(2.4, rel=1e-15)
    assert eta == pytest.approx(math.log(2.0), rel=1e-15)
    np.testing.assert_allclose(g, [[-0.05, 0.0], [0.0, 0.0], [0.05, 0.0]], rtol=1e-13,
                               atol=1e-17)
    l2 = math.log(2.0)
    np.testing.assert_allclose(u, [[0.08 + 0.05 * l2, 0.16], [0.0, 0.0], [-0.05 * l2, 0.0]],
                               rtol=1e-13, atol=1e-17)
    yb = np.array([[-1.0 + 0.08 + 0.05 * l2, 0.16], [0.0, 0.0], [1.0 - 0.05 * l2, 0.0]])
    np.testing.assert_allclose(y, yb - yb.mean(axis=0), rtol=1e-13, atol=1e-16)


def test_step_range_two_points_is_pure_momentum():
    """n = 2: ln(n - 1) = 0, so eta = 0 and only the momentum term moves Y."""
    P = np.array([[0.0, 0.5], [0.5, 0.0]])
    y = np.array([[0.0, 0.0], [2.0, 1.0]])
    u = np.array([[0.3, -0.1], [0.1, 0.4]])
    _, _, eta = oracle.step_range(P, y, u, mu=0.5, recentre=False)
    assert eta == 0.0
    np.testing.assert_allclose(u, [[0.15, -0.05], [0.05, 0.2]], rtol=1e-15)
    np.testing.assert_allclose(y, [[0.15, -0.05], [2.05, 1.2]], rtol=1e-15)


def test_step_range_preserves_mean_without_recentring():
    """The gradient of Eq. 6 sums to zero, so from U = 0 the mean of the map
    stays where it is even when the map is not re-centred."""
    x, _ = synth.plain_small(120, seed=23)
    P = oracle.joint_p(x, oracle.calibrate(x, 15.0))
    y = _rng(24).standard_normal((120, 2)) + [3.0, -1.0]
    m0 = y.mean(axis=0)
    u = np.zeros_like(y)
    for _ in range(5):
        oracle.step_range(P, y, u, mu=0.8, recentre=False)
    np.testing.assert_allclose(y.mean(axis=0), m0, rtol=0, atol=1e-11)


def test_bitwise_resume(small_problem):
    """Running 3 + 4 iterations through a saved state equals 7 straight through."""
    _, P, y = small_problem
    y0 = y * 0.01
    a = oracle.run(P, y0, 7, start=246)
    s = oracle.run(P, y0, 3, start=246)
    saved = tuple(np.array(v) for v in s)
    b = oracle.run(P, None, 4, start=249, state=saved)
    for va, vb in zip(a, b):
        assert np.array_equal(va, vb)


def test_descent_lowers_cost():
    """The descent reading of Eq. 10 lowers KL over the first iterations without exaggeration."""
    x, _ = synth.plain_small(200, seed=41)
    P = oracle.joint_p(x, oracle.calibrate(x, 20.0))
    y0 = synth.embedding_init(200, seed=42).astype(np.float64)
    k0 = oracle.cost(P, y0)[0]
    y, _, _ = oracle.run(P, y0, 30, sched=lambda t: oracle.StepParams(1.0, 0.5, 100.0))
    assert oracle.cost(P, y)[0] < k0


# ---------------------------------------------------------------------------
# Evaluation: kNN overlap
# ---------------------------------------------------------------------------

def test_knn_overlap_brute_force():
    rng = _rng(9)
    x = rng.standard_normal((60, 5))
    y = rng.standard_normal((60, 2))
    rows = np.arange(60)
    k = 4

    def knn(a, i):
        d = cdist(a[i:i + 1], a, "sqeuclidean")[0]
        d[i] = np.inf
        return set(np.argsort(d, kind="stable")[:k])

    ref = np.mean([len(knn(x, i) & knn(y, i)) / k for i in rows])
    assert abs(oracle.knn_overlap(x, y, rows, k) - ref) < 1e-15
    # a map that keeps the first two coordinates of 2-D data keeps every neighbour
    x2 = rng.standard_normal((60, 2))
    assert oracle.knn_overlap(x2, x2, rows, k) == 1.0


# ---------------------------------------------------------------------------
# Given dissimilarities instead of points (section "ptSNE: parallelized t-SNE")
# ---------------------------------------------------------------------------

def test_dissimilarity_input_equals_point_input_for_euclidean_distances():
    """Euclidean distances of X given as dissimilarities reproduce the
    affinities of X itself (the squared dissimilarity enters Eq. 1)."""
    x = _rng(61).standard_normal((45, 6)) * 2.0
    dis = np.sqrt(cdist(x, x, "sqeuclidean"))
    st_x = oracle.calibrate(x, 9.0)
    st_d = oracle.calibrate_dissim(dis, 9.0)
    np.testing.assert_allclose(st_d.beta, st_x.beta, rtol=1e-9)
    P = oracle.joint_p_dissim(dis, st_d)
    np.testing.assert_allclose(P, oracle.joint_p(x, st_x), rtol=1e-9, atol=1e-15)


def test_dissimilarity_path_graph():
    """Shortest-path distances of a 4-node path graph (1-2-3-4): node 1 has
    neighbours at distances 1, 2, 3, so with squared distances 1, 4, 9 its
    entropy at the returned beta is that of the weights e^{-beta}, e^{-4 beta},
    e^{-9 beta} (brute force), and P is symmetric with unit sum (Eq. 3)."""
    dis = np.abs(np.subtract.outer(np.arange(4.0), np.arange(4.0)))
    st = oracle.calibrate_dissim(dis, 2.0)
    b = st.beta[0]
    w = np.exp(-b * np.array([1.0, 4.0, 9.0]))
    p = w / w.sum()
    assert -(p * np.log(p)).sum() == pytest.approx(math.log(2.0), abs=1e-10)
    P = oracle.joint_p_dissim(dis, st)
    np.testing.assert_allclose(P, P.T, rtol=0, atol=1e-17)
    assert P.sum() == pytest.approx(1.0, abs=1e-14)
