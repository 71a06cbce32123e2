"""Pins for the oracle's resist, loss gradient and level-set step (CPU only)."""
import numpy as np
import pytest

from oracle import levelset, litho, resist
from paper_2303_12529_amd.inputs import random_mask


def test_sigmoid_at_threshold_and_slope():
    assert resist.sigmoid_resist(np.array([0.225]), 50.0, 0.225)[0] == 0.5
    I = np.linspace(0.0, 0.6, 13)
    h = 1e-6
    Z = resist.sigmoid_resist(I, 50.0, 0.225)
    fd = (resist.sigmoid_resist(I + h, 50.0, 0.225) - resist.sigmoid_resist(I - h, 50.0, 0.225)) / (2 * h)
    np.testing.assert_allclose(fd, 50.0 * Z * (1 - Z), rtol=1e-8, atol=1e-10)


def test_loss_gradient_finite_difference():
    rng = np.random.default_rng(1)
    N = 16
    I0 = rng.uniform(0.0, 0.5, size=(N, N))
    I1 = rng.uniform(0.0, 0.5, size=(N, N))
    Zt = random_mask(N, 0.3, seed=2)
    corners = [(0, 1.0, 1.0), (0, 1.02, 7.5), (1, 0.98, 7.5)]
    L, G = resist.dso_loss_and_grad([I0, I1], Zt, corners, 50.0, 0.225)
    h = 1e-6
    for s, Is in enumerate([I0, I1]):
        for (y, x) in rng.integers(0, N, size=(10, 2)):
            Ip = [I0.copy(), I1.copy()]; Ip[s][y, x] += h
            Im = [I0.copy(), I1.copy()]; Im[s][y, x] -= h
            fd = (resist.dso_loss_and_grad(Ip, Zt, corners, 50.0, 0.225)[0]
                  - resist.dso_loss_and_grad(Im, Zt, corners, 50.0, 0.225)[0]) / (2 * h)
            assert abs(fd - G[s][y, x]) <= 1e-5 * max(1.0, abs(G[s][y, x]))


def test_print_metrics_by_hand():
    Zt = np.array([[1, 0], [0, 1]], dtype=np.uint8)
    Inom = np.array([[0.3, 0.3], [0.1, 0.225]])
    Idef = np.array([[0.3, 0.1], [0.1, 0.2]])
    corners = [(0, 1.0, 1.0), (0, 1.02, 7.5), (1, 0.98, 7.5)]
    l2, pvb = resist.print_metrics([Inom, Idef], Zt, corners, 0.225)
    # nominal print [[1,1],[0,1]] (tie prints) vs target -> 1 pixel differs
    assert l2 == 1
    # outer = 1.02*Inom >= .225 -> [[1,1],[0,1]]; inner = .98*Idef -> [[1,0],[0,0]]
    assert pvb == 2


def test_full_loss_gradient_through_litho():
    """dL_DSO/dM by the chain G -> adjoint against a central difference."""
    rng = np.random.default_rng(5)
    N, P, K = 20, 5, 3
    H = rng.normal(size=(2, K, P, P)) + 1j * rng.normal(size=(2, K, P, P))
    H *= 0.5 / np.abs(H[:, :, 2, 2]).max()
    w = rng.uniform(0.2, 1.0, size=(2, K))
    Zt = random_mask(N, 0.3, seed=6)
    M = rng.uniform(size=(N, N))
    corners = [(0, 1.0, 1.0), (0, 1.02, 7.5), (1, 0.98, 7.5)]

    def loss(Mx):
        I = [litho.aerial_image(Mx, H[s], w[s]) for s in range(2)]
        return resist.dso_loss_and_grad(I, Zt, corners, 50.0, 0.225)

    L, G = loss(M)
    g = sum(litho.litho_adjoint(M, G[s], H[s], w[s]) for s in range(2))
    h = 1e-5
    scale = np.abs(g).max()
    for (y, x) in rng.integers(0, N, size=(16, 2)):
        Mp = M.copy(); Mp[y, x] += h
        Mm = M.copy(); Mm[y, x] -= h
        fd = (loss(Mp)[0] - loss(Mm)[0]) / (2 * h)
        assert abs(fd - g[y, x]) <= 2e-5 * scale


def test_stencils_exact_on_quadratics():
    N = 12
    yy, xx = np.mgrid[0:N, 0:N].astype(np.float64)
    a, b, c, d, e = 0.3, -0.7, 1.1, 0.25, -2.0
    phi = a * xx ** 2 + b * xx * yy + c * yy ** 2 + d * xx + e * yy
    px, py, pxx, pyy, pxy = levelset.central_differences(phi)
    s = np.s_[1:-1, 1:-1]
    np.testing.assert_allclose(px[s], (2 * a * xx + b * yy + d)[s], atol=1e-12)
    np.testing.assert_allclose(py[s], (b * xx + 2 * c * yy + e)[s], atol=1e-12)
    np.testing.assert_allclose(pxx[s], 2 * a, atol=1e-12)
    np.testing.assert_allclose(pyy[s], 2 * c, atol=1e-12)
    np.testing.assert_allclose(pxy[s], b, atol=1e-12)


def test_curvature_zero_on_planes_and_circle_value():
    N = 64
    yy, xx = np.mgrid[0:N, 0:N].astype(np.float64)
    _, K = levelset.grad_norm_and_curvature(0.3 * xx - 0.8 * yy + 2.0, 1e-12)
    assert np.abs(K[1:-1, 1:-1]).max() < 1e-12
    # SDF of a circle: |grad phi| div(n) = 1/r away from the centre
    r = np.hypot(yy - 31.5, xx - 31.5)
    gn, K = levelset.grad_norm_and_curvature(r - 20.0, 1e-12)
    ring = (r > 10) & (r < 25)
    np.testing.assert_allclose(K[ring], 1.0 / r[ring], rtol=2e-2)
    np.testing.assert_allclose(gn[ring], 1.0, rtol=2e-2)


def test_circle_curvature_flow_area_rate():
    """Curvature-only flow (lambda = 1): area falls at 2 pi lambda per unit
    time (R^2 = R0^2 - 2 lambda t); a straight edge does not move."""
    N, R0, lam, dt, steps = 128, 30.0, 1.0, 0.2, 1000
    yy, xx = np.mgrid[0:N, 0:N].astype(np.float64)
    phi = np.hypot(yy - 63.5, xx - 63.5) - R0
    a0 = np.sum(phi <= 0)
    zero = np.zeros((N, N))
    for _ in range(steps):
        phi, _, _, _ = levelset.levelset_step(phi, zero, None, dt, lam, 1e-12, dt_mode=1)
    a1 = np.sum(phi <= 0)
    rate = (a0 - a1) / (steps * dt)
    assert abs(rate - 2 * np.pi * lam) <= 0.05 * 2 * np.pi * lam
    edge = xx - 63.5
    e2 = edge.copy()
    flips = 0
    for _ in range(50):
        e2, _, _, f = levelset.levelset_step(e2, zero, None, dt, lam, 1e-12, dt_mode=1)
        flips += f
    assert flips == 0 and np.array_equal(e2 <= 0, edge <= 0)


def test_modulated_curvature_flow():
    """The modulation map scales the curvature term pointwise (Sec. III-C):
    m = 1/2 everywhere halves the circle's area rate (pi lambda); m = 0 keeps
    phi unchanged; m = 0 on the left half and 1 on the right leaves the left
    half of the disc where it was while the right half shrinks."""
    N, R0, lam, dt, steps = 128, 30.0, 1.0, 0.2, 1000
    yy, xx = np.mgrid[0:N, 0:N].astype(np.float64)
    phi0 = np.hypot(yy - 63.5, xx - 63.5) - R0
    zero = np.zeros((N, N))
    phi = phi0.copy()
    half = np.full((N, N), 0.5)
    for _ in range(steps):
        phi, _, _, _ = levelset.levelset_step(phi, zero, half, dt, lam, 1e-12, dt_mode=1)
    rate = (np.sum(phi0 <= 0) - np.sum(phi <= 0)) / (steps * dt)
    assert abs(rate - np.pi * lam) <= 0.05 * np.pi * lam
    frozen, _, _, f = levelset.levelset_step(phi0, zero, zero, dt, lam, 1e-12, dt_mode=1)
    assert f == 0 and np.array_equal(frozen, phi0)
    side = (xx >= 63.5).astype(np.float64)
    phi = phi0.copy()
    for _ in range(200):
        phi, _, _, _ = levelset.levelset_step(phi, zero, side, dt, lam, 1e-12, dt_mode=1)
    left = xx < 58.0                    # a few pixels clear of the stencil's reach across the seam
    assert np.array_equal((phi <= 0) & left, (phi0 <= 0) & left)
    right = xx > 69.0
    assert np.sum((phi <= 0) & right) < np.sum((phi0 <= 0) & right)


def test_descent_sign_and_loss_decrease():
    """A motion-only step flips only pixels with g * dM < 0, and a small CFL
    step lowers the DSO loss."""
    from paper_2303_12529_amd.inputs import build_optics
    from oracle import edt
    N = 64
    H, w = build_optics(N, 8.0, 9, 6)
    Zt = np.zeros((N, N), dtype=np.uint8)
    Zt[20:44, 26:38] = 1
    phi, _, _ = edt.tsdf_from_mask(Zt, -12.5, 112.5)
    corners = [(0, 1.0, 1.0)]

    def L_of(phi_):
        M = levelset.mask_from_phi(phi_)
        I = [litho.aerial_image(M, H[0], w[0])]
        return resist.dso_loss_and_grad(I, Zt, corners, 50.0, 0.225), M

    (L0, G), M0 = L_of(phi)
    g = litho.litho_adjoint(M0, G[0], H[0], w[0])
    new, dt, m_v, flips = levelset.levelset_step(phi, g, None, 0.85, 0.0, 1e-12)
    assert m_v == np.abs(g).max() and abs(dt - 0.85 / m_v) < 1e-15
    M1 = levelset.mask_from_phi(new)
    dM = M1.astype(np.float64) - M0
    assert flips == int(np.sum(dM != 0)) and flips > 0
    assert np.all(g[dM != 0] * dM[dM != 0] < 0)
    (L1, _), _ = L_of(new)
    assert L1 < L0


def test_cfl_dt_rules():
    g = np.array([[0.5, -2.0], [1.0, 0.0]])
    assert levelset.cfl_dt(g, 0.85, 0, 0.0) == (0.85 / 2.0, 2.0)
    assert levelset.cfl_dt(g, 0.85, 0, 0.1) == (0.1, 2.0)
    assert levelset.cfl_dt(g, 0.1, 1, 0.0) == (0.1, 2.0)
    assert levelset.cfl_dt(np.zeros((2, 2)), 0.85, 0, 5.0) == (5.0, 0.0)
    assert levelset.cfl_dt(np.zeros((2, 2)), 0.85, 0, 0.0) == (0.0, 0.0)


def test_cg_direction_recurrence_and_restart():
    from oracle import levelset as ls
    st = {}
    d, b = ls.cg_direction(np.array([1.0, 0.0]), st)
    assert b == 0.0 and np.array_equal(d, [1.0, 0.0])
    st["d_prev"] = np.array([2.0, 0.0])
    d, b = ls.cg_direction(np.array([1.0, 1.0]), st)
    # <g, g - g_prev> = <(1,1), (0,1)> = 1, <g_prev, g_prev> = 1
    assert b == 1.0 and np.array_equal(d, [3.0, 1.0])
    # a negative Polak-Ribiere coefficient restarts along the gradient
    # <(0.5, 0.5), (0.5, 0.5) - (1, 1)> = -0.5 < 0
    d, b = ls.cg_direction(np.array([0.5, 0.5]), st)
    assert b == 0.0 and np.array_equal(d, [0.5, 0.5])


def test_cg_direction_solves_a_quadratic_in_n_steps():
    """With exact line searches, PR conjugate gradient minimises a strictly
    convex n-dimensional quadratic in n steps (textbook property)."""
    from oracle import levelset as ls
    rng = np.random.default_rng(3)
    n = 6
    Q = rng.normal(size=(n, n))
    A = Q @ Q.T + n * np.eye(n)
    b = rng.normal(size=n)
    x = np.zeros(n)
    st = {}
    for _ in range(n):
        g = b - A @ x                  # descent velocity: minus the gradient
        d, _ = ls.cg_direction(g, st)
        alpha = float(g @ d) / float(d @ A @ d)
        x = x + alpha * d
    assert np.linalg.norm(A @ x - b) <= 1e-9 * np.linalg.norm(b)
    # plain steepest descent with the same line searches does not get there
    x = np.zeros(n)
    for _ in range(n):
        g = b - A @ x
        x = x + float(g @ g) / float(g @ A @ g) * g
    assert np.linalg.norm(A @ x - b) > 1e-6 * np.linalg.norm(b)
