"""Pins of the learned-preconditioner oracle: exact reduction to the base
preconditioner when the network output is zero, positive homogeneity, the
gradient of the mesh loss (through W = P^T) against finite differences, and
the gate/fallback logic of the flexible GMRES on small dense systems."""
import numpy as np
import pytest

from oracle import aimx, learned_pc, solver, unet
from paper_2009_02281_amd import inputs as I


@pytest.fixture(scope="module")
def tiny():
    w = I.sphere_tiny(level=1, radius=0.5, dims=(8, 8, 8), h=0.2)
    o = aimx.AimOracle(w.vertices, w.triangles, w.order, w.dims, w.h, w.near_threshold)
    return o


def _net(seed, C=4, bias=0.1):
    params = unet.init_params(C, seed=seed)
    rng = np.random.default_rng(seed + 1)
    for W, b in params:
        b += bias * rng.standard_normal(b.shape)
    return params


def test_zero_output_reduces_to_base(tiny):
    params = _net(1)
    W, b = params[10]
    W[:] = 0.0
    b[:] = 0.0
    net = unet.UNet(params)
    d = np.arange(1, tiny.N + 1, dtype=float)
    base = lambda v: v / d
    v = I.complex_gaussian(tiny.N, 5)
    assert np.array_equal(learned_pc.apply(tiny, net, base, 0.7, v), base(v))


def test_positive_homogeneity(tiny):
    net = unet.UNet(_net(2))
    base = lambda v: 0.5 * v
    v = I.complex_gaussian(tiny.N, 6)
    a = learned_pc.apply(tiny, net, base, 1.3, v)
    b = learned_pc.apply(tiny, net, base, 1.3, 3.0 * v)
    assert np.allclose(b, 3.0 * a, rtol=1e-12, atol=0)
    # and the correction is not trivially zero
    assert np.linalg.norm(a - base(v)) > 1e-3 * np.linalg.norm(a)


def test_network_input_is_unit_rms(tiny):
    g = learned_pc.network_input(tiny, I.complex_gaussian(tiny.N, 7))
    assert np.sqrt(np.mean(np.abs(g) ** 2)) == pytest.approx(1.0, rel=1e-14)


def test_mesh_loss_gradient_matches_finite_differences(tiny):
    params = _net(3)
    r = I.complex_gaussian(tiny.N, 8)
    t = I.complex_gaussian(tiny.N, 9)
    grid = learned_pc.network_input(tiny, r)
    tau = 0.8
    loss, g = learned_pc.mesh_loss(tiny, unet.UNet(params), grid, t, tau)
    rng = np.random.default_rng(10)
    eps = 1e-6
    for li in (0, 4, 9, 10):
        W, _ = params[li]
        for _ in range(2):
            idx = tuple(int(rng.integers(0, s)) for s in W.shape)
            Pp = [(w.copy(), bb.copy()) for w, bb in params]
            Pm = [(w.copy(), bb.copy()) for w, bb in params]
            Pp[li][0][idx] += eps
            Pm[li][0][idx] -= eps
            lp, _ = learned_pc.mesh_loss(tiny, unet.UNet(Pp), grid, t, tau)
            lm, _ = learned_pc.mesh_loss(tiny, unet.UNet(Pm), grid, t, tau)
            assert g[li][0][idx] == pytest.approx((lp - lm) / (2 * eps), rel=1e-5, abs=1e-11)


def test_residual_loss_gradient_matches_finite_differences(tiny):
    params = _net(4)
    k = 2.0
    A = lambda x: tiny.matvec(x, k)
    r = I.complex_gaussian(tiny.N, 12)
    d = np.linspace(1.0, 2.0, tiny.N)
    base = lambda v: v / d
    s = learned_pc.residual_target(A, base, r)
    grid = learned_pc.network_input(tiny, r)
    tau, weight = 0.6, 3.0
    loss, g = learned_pc.residual_loss(tiny, unet.UNet(params), A, grid, s, tau, weight)
    rng = np.random.default_rng(13)
    eps = 1e-6
    for li in (0, 5, 10):
        W, _ = params[li]
        for _ in range(2):
            idx = tuple(int(rng.integers(0, n)) for n in W.shape)
            Pp = [(w.copy(), bb.copy()) for w, bb in params]
            Pm = [(w.copy(), bb.copy()) for w, bb in params]
            Pp[li][0][idx] += eps
            Pm[li][0][idx] -= eps
            lp, _ = learned_pc.residual_loss(tiny, unet.UNet(Pp), A, grid, s, tau, weight)
            lm, _ = learned_pc.residual_loss(tiny, unet.UNet(Pm), A, grid, s, tau, weight)
            assert g[li][0][idx] == pytest.approx((lp - lm) / (2 * eps), rel=1e-5, abs=1e-11)


def test_residual_target_of_an_exact_base_is_zero(tiny):
    """If B inverts A, nothing is left for the network: s = 0."""
    k = 2.0
    N = tiny.N
    Ad = np.stack([tiny.matvec(np.eye(N, dtype=complex)[j], k) for j in range(N)], axis=1)
    Ainv = np.linalg.inv(Ad)
    s = learned_pc.residual_target(lambda x: Ad @ x, lambda v: Ainv @ v,
                                   I.complex_gaussian(N, 14))
    assert np.linalg.norm(s) <= 1e-10


def _dense_system(n=60, seed=11):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 4 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return A, b


def test_gate_keeps_a_good_preconditioner():
    A, b = _dense_system()
    Ainv = np.linalg.inv(A)
    x, info = solver.gated_fgmres(lambda v: A @ v, b, lambda v: Ainv @ v, tol=1e-10, restart=5)
    assert info.converged and not info.fallback_used
    assert info.iters <= 2


def test_gate_falls_back_on_non_finite_output():
    A, b = _dense_system()
    bad = lambda v: np.full_like(v, np.nan)
    x, info = solver.gated_fgmres(lambda v: A @ v, b, bad, tol=1e-10, restart=5)
    assert info.fallback_used and info.converged
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b) * 1.01


def test_gate_falls_back_on_stagnation():
    A, b = _dense_system()
    # a preconditioner whose range is one fixed direction: GMRES stalls
    u = np.ones(b.size, dtype=complex)
    stall = lambda v: u * np.vdot(u, v) / b.size
    x, info = solver.gated_fgmres(lambda v: A @ v, b, stall, tol=1e-10, restart=5)
    assert info.fallback_used and info.converged
