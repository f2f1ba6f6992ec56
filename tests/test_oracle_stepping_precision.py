"""Pins of the oracle's time stepping and reduced-precision storage (CPU only)."""
import numpy as np
import pytest
import torch

from oracle import geometry, precision, stepping
from oracle.stepping import advance, jeffery_rhs, normalize, EULER, HEUN, AB2

L = geometry.L


def _dist(a, b):
    return np.abs(a - b)


def shear(X):
    u = np.zeros_like(X)
    u[:, 0] = np.sin(X[:, 1])
    return u


def abc(X):
    return np.stack([np.sin(X[:, 1]) + 0.5 * np.cos(X[:, 2]),
                     np.sin(X[:, 2]) + 0.5 * np.cos(X[:, 0]),
                     np.sin(X[:, 0]) + 0.5 * np.cos(X[:, 1])], axis=1)


def rk4(X, f, dt, n):
    for _ in range(n):
        k1 = f(X)
        k2 = f(X + 0.5 * dt * k1)
        k3 = f(X + 0.5 * dt * k2)
        k4 = f(X + dt * k3)
        X = X + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return X


ALL = [stepping.EULER, stepping.HEUN, stepping.AB2, stepping.AB3, stepping.AB4]


@pytest.mark.parametrize("scheme", ALL)
def test_shear_flow_exact(scheme):
    X0 = np.random.default_rng(0).uniform(0, L, (500, 3))
    dt, n = 1e-2, 37
    X, _, _, _ = stepping.advance(X0, shear, scheme, dt, n)
    ex = X0.copy()
    ex[:, 0] = X0[:, 0] + n * dt * np.sin(X0[:, 1])
    assert np.max(_dist(X, ex)) < 1e-12
    # the state is not wrapped: particles that crossed a face keep going
    assert np.any((X < 0) | (X >= L))


@pytest.mark.parametrize("scheme", ALL)
def test_constant_velocity(scheme):
    X0 = np.random.default_rng(1).uniform(0, L, (100, 3))
    c = np.array([0.7, -1.3, 2.1])
    X, _, _, _ = stepping.advance(X0, lambda X: np.broadcast_to(c, X.shape).copy(), scheme, 1e-3, 50)
    assert np.max(_dist(X, X0 + 50 * 1e-3 * c)) < 1e-13


@pytest.mark.parametrize("scheme,order", [(stepping.EULER, 1), (stepping.HEUN, 2), (stepping.AB2, 2)])
def test_convergence_order_in_dt(scheme, order):
    X0 = np.random.default_rng(2).uniform(0, L, (200, 3))
    T = 0.5
    ref = rk4(X0.copy(), abc, T / 2000, 2000)
    errs = []
    for n in [50, 100, 200]:
        X, _, _, _ = stepping.advance(X0, abc, scheme, T / n, n)
        errs.append(np.max(_dist(X, ref)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - order) < 0.25), rates


def test_ab_weights_consistent():
    """Each Adams-Bashforth rule integrates polynomials of degree < k exactly:
    sum_j b_j (-j)^p = 1/(p+1) for p < k (exact rationals)."""
    from fractions import Fraction as F
    exact = {2: (F(3, 2), F(-1, 2)), 3: (F(23, 12), F(-16, 12), F(5, 12)),
             4: (F(55, 24), F(-59, 24), F(37, 24), F(-9, 24))}
    for k, b in exact.items():
        for p in range(k):
            assert sum(bj * F(-j) ** p for j, bj in enumerate(b)) == F(1, p + 1)
        assert all(abs(float(bj) - w) == 0.0 for bj, w in zip(b, stepping.AB_WEIGHTS[k]))


@pytest.mark.parametrize("scheme,order", [(stepping.AB3, 3), (stepping.AB4, 4)])
def test_ab_high_order_convergence_with_exact_history(scheme, order):
    """With the history taken from the exact trajectory (RK4 with a fine step,
    run backwards), AB3 and AB4 converge at their full order."""
    X0 = np.random.default_rng(2).uniform(0, L, (200, 3))
    T = 0.5
    ref = rk4(X0.copy(), abc, T / 4000, 4000)
    K = stepping.AB_ORDER[scheme]
    errs = []
    for n in [40, 80, 160]:
        dt = T / n
        hist = np.zeros((K, 200, 3))
        for j in range(1, K):
            Xj = rk4(X0.copy(), abc, -dt * j / 200, 200)
            hist[j - 1] = abc(Xj)
        X, _, _, _ = stepping.advance(X0, abc, scheme, dt, n, hist=hist, hist_len=K - 1)
        errs.append(np.max(_dist(X, ref)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - order) < 0.3), rates


@pytest.mark.parametrize("scheme", [stepping.AB3, stepping.AB4])
def test_ab_startup_lowers_order(scheme):
    """From an empty history the first steps use Euler, AB2, ...: the first
    step equals an Euler step and the second an AB2 step."""
    X0 = np.random.default_rng(5).uniform(0, L, (50, 3))
    dt = 1e-2
    X1, h1, l1, _ = stepping.advance(X0, abc, scheme, dt, 1)
    assert np.array_equal(X1, stepping.euler_update(X0, dt, abc(X0))) and l1 == 1
    X2, h2, l2, _ = stepping.advance(X1, abc, scheme, dt, 1, hist=h1, hist_len=l1)
    assert np.array_equal(X2, stepping.ab2_update(X1, dt, abc(X1), abc(X0))) and l2 == 2


def test_ab2_resume_bitwise():
    X0 = np.random.default_rng(3).uniform(0, L, (300, 3))
    Xa, ha, la, _ = stepping.advance(X0, abc, stepping.AB2, 2e-3, 40)
    Xb, hb, lb, _ = stepping.advance(X0, abc, stepping.AB2, 2e-3, 17)
    Xb, hb, lb, _ = stepping.advance(Xb, abc, stepping.AB2, 2e-3, 23, hist=hb, hist_len=lb)
    assert np.array_equal(Xa, Xb) and np.array_equal(ha, hb) and la == lb == 2


def test_ab4_resume_bitwise():
    X0 = np.random.default_rng(3).uniform(0, L, (300, 3))
    Xa, ha, la, _ = stepping.advance(X0, abc, stepping.AB4, 2e-3, 40)
    Xb, hb, lb, _ = stepping.advance(X0, abc, stepping.AB4, 2e-3, 2)
    Xb, hb, lb, _ = stepping.advance(Xb, abc, stepping.AB4, 2e-3, 38, hist=hb, hist_len=lb)
    assert np.array_equal(Xa, Xb) and np.array_equal(ha, hb) and la == lb == 4


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.standard_normal(100000).astype(np.float32),
                        np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 0.0, -0.0,
                                  1e-40, 3.0e38, 65504.0, 2 ** -126], dtype=np.float32)])
    ours = precision.f32_to_bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


def test_f16_rounding_matches_torch():
    x = np.random.default_rng(5).standard_normal(100000).astype(np.float32) * 3
    ref = torch.from_numpy(x).to(torch.float16).to(torch.float64).numpy()
    assert np.array_equal(x.astype(np.float16).astype(np.float64), ref)


@pytest.mark.parametrize("storage,rel", [(precision.BF16, 2.0 ** -8), (precision.F16, 2.0 ** -11)])
def test_store_scale_and_error(storage, rel):
    rng = np.random.default_rng(6)
    u = (rng.standard_normal((8, 8, 8, 3)) * np.array([0.5, 2.0, 7.0])).astype(np.float32)
    vals, s = precision.store(u, storage)
    assert np.allclose(np.sqrt(np.mean(vals.reshape(-1, 3) ** 2, axis=0)), 1.0, rtol=1e-2)
    back = vals * s
    assert np.max(np.abs(back - u) / np.abs(u).clip(1e-3)) <= rel * 1.01


def test_heun_two_fields_exact_for_linear_time_dependence():
    """A shear flow whose amplitude grows linearly in time,
    u = ((a + b t) sin x2, 0, 0): x2 stays fixed, and the trapezoid rule of
    Heun's two stages integrates the linear-in-time velocity exactly, so
    n steps reproduce X1(t) = X1(0) + (a t + b t^2 / 2) sin X2 to rounding.
    Taking both stages from the start time's field instead (the frozen-field
    step) misses the b t^2 / 2 term's half."""
    a, b = 0.8, 3.0
    X0 = np.random.default_rng(7).uniform(0, L, (400, 3))
    dt, n = 1e-2, 25

    def field_at(t):
        def vel(X):
            u = np.zeros_like(X)
            u[:, 0] = (a + b * t) * np.sin(X[:, 1])
            return u
        return vel

    X = X0.copy()
    Xf = X0.copy()
    for k in range(n):
        X, _ = stepping.heun_two_fields(X, field_at(k * dt), field_at((k + 1) * dt), dt)
        Xf, _ = stepping.heun_two_fields(Xf, field_at(k * dt), field_at(k * dt), dt)
    T = n * dt
    ex = X0.copy()
    ex[:, 0] = X0[:, 0] + (a * T + 0.5 * b * T * T) * np.sin(X0[:, 1])
    assert np.max(np.abs(X - ex)) < 1e-12
    assert np.max(np.abs(Xf - ex)) > 1e-3
    # the frozen-field scheme of ``advance`` is the two-field step with one field
    Xa, _, _, _ = stepping.advance(X0, field_at(0.0), stepping.HEUN, dt, 1)
    Xb, _ = stepping.heun_two_fields(X0, field_at(0.0), field_at(0.0), dt)
    assert np.array_equal(Xa, Xb)


# ---- Jeffery's equation (orientation of axisymmetric ellipsoids)

def _const_grad(A):
    def g(X):
        return np.zeros_like(X), np.broadcast_to(A, (X.shape[0], 3, 3)).copy()
    return g


def test_jeffery_pure_rotation_is_a_rigid_rotation():
    """A antisymmetric (a solid-body rotation, A p = w x p): S = 0 and W = A,
    so dp/dt = w x p rotates p rigidly by the angle |w| t about w whatever the
    shape; Heun converges to that rotation at second order."""
    from scipy.spatial.transform import Rotation
    wv = np.array([0.3, -0.7, 1.1])
    # A such that A p = wv x p: A_ab = -eps_abc wv_c
    A = np.array([[0.0, -wv[2], wv[1]], [wv[2], 0.0, -wv[0]], [-wv[1], wv[0], 0.0]])
    rng = np.random.default_rng(3)
    p0 = normalize(rng.standard_normal((50, 3)))
    X0 = np.zeros((50, 3))
    T = 1.0
    ex = Rotation.from_rotvec(wv * T).apply(p0)
    errs = []
    for n in (40, 80, 160):
        out = advance(X0, None, HEUN, T / n, n, gradient=_const_grad(A), orientation=(p0, 0.7))
        errs.append(np.max(np.abs(out[4] - ex)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2) < 0.2), rates
    assert errs[-1] < 3e-5


def test_jeffery_rods_in_steady_strain_follow_the_closed_form():
    """shape = 1 (thin rods) in a constant symmetric gradient S: dp/dt =
    S p - (p.S p) p has the solution p(t) = e^{St} p0 / |e^{St} p0|; Heun, AB2
    and AB4 (started from the exact history) converge to it at their order."""
    from scipy.linalg import expm
    B = np.array([[0.4, 0.2, -0.1], [0.2, -0.3, 0.25], [-0.1, 0.25, -0.1]])
    rng = np.random.default_rng(4)
    p0 = normalize(rng.standard_normal((30, 3)))
    X0 = np.zeros((30, 3))
    T = 1.0
    ex = normalize(p0 @ expm(B * T).T)
    for scheme, order in ((HEUN, 2), (AB2, 2), (EULER, 1)):
        errs = []
        for n in (50, 100, 200):
            out = advance(X0, None, scheme, T / n, n, gradient=_const_grad(B), orientation=(p0, 1.0))
            errs.append(np.max(np.abs(out[4] - ex)))
        rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        assert np.all(np.abs(rates - order) < 0.3), (scheme, rates)
    # the unit length is kept and the rods turn towards the largest strain axis
    out = advance(X0, None, HEUN, 0.01, 2000, gradient=_const_grad(B), orientation=(p0, 1.0))
    w, v = np.linalg.eigh(B)
    assert np.allclose(np.sum(out[4] ** 2, axis=1), 1.0, atol=1e-14)
    assert np.min(np.abs(out[4] @ v[:, -1])) > 0.999


def test_jeffery_rhs_special_cases():
    """Spheres (shape 0) only rotate with the fluid, W p; the rhs is
    orthogonal to p for every shape (the length is conserved); discs (shape
    -1) and rods (1) differ by the sign of the strain term."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((100, 3, 3))
    p = normalize(rng.standard_normal((100, 3)))
    W = 0.5 * (A - np.swapaxes(A, 1, 2))
    assert np.allclose(jeffery_rhs(A, p, 0.0), np.einsum("pab,pb->pa", W, p), atol=1e-15)
    for shape in (-1.0, 0.3, 1.0):
        r = jeffery_rhs(A, p, shape)
        assert np.max(np.abs(np.sum(r * p, axis=1))) < 1e-14
    strain = jeffery_rhs(A, p, 1.0) - jeffery_rhs(A, p, 0.0)
    assert np.allclose(jeffery_rhs(A, p, -1.0), jeffery_rhs(A, p, 0.0) - strain, atol=1e-15)


# ---- inertial particles: dX/dt = V, dV/dt = (u(X) - V)/tau

def _const_field(U0):
    return lambda Y: np.broadcast_to(U0, np.shape(Y)).copy()


@pytest.mark.parametrize("scheme", [EULER, HEUN])
def test_inertial_constant_field_closed_forms(scheme):
    """In a uniform field U0 the schemes' recurrences close: V_n - U0 =
    (V_0 - U0) g^n with g = 1 - h (Euler) or 1 - h + h^2/2 (Heun), h = dt/tau,
    and X_n = X_0 + n dt U0 + c (V_0 - U0) (1 - g^n)/(1 - g) with c = dt
    (Euler) or dt (1 - h/2) (Heun)."""
    rng = np.random.default_rng(40)
    X0, V0 = rng.uniform(-3, 3, (50, 3)), rng.standard_normal((50, 3))
    U0 = np.array([0.7, -1.3, 0.2])
    tau, dt, n = 0.37, 0.05, 23
    h = dt / tau
    X, V, _, _, _ = stepping.advance_inertial(X0, V0, _const_field(U0), tau, scheme, dt, n)
    g = 1 - h if scheme == EULER else 1 - h + h * h / 2
    c = dt if scheme == EULER else dt * (1 - h / 2)
    assert np.allclose(V, U0 + (V0 - U0) * g ** n, rtol=0, atol=1e-13)
    assert np.allclose(X, X0 + n * dt * U0 + c * (V0 - U0) * (1 - g ** n) / (1 - g), rtol=0, atol=1e-12)


def _shear_u(Y):
    Y = np.asarray(Y)
    return np.stack([np.sin(Y[..., 1]), 0.5 * np.cos(Y[..., 2]), 0.3 * np.sin(Y[..., 0] + Y[..., 1])], axis=-1)


def _exact_inertial(X0, V0, tau, T):
    """The continuous solution by scipy's adaptive Runge-Kutta (tight tolerances)."""
    from scipy.integrate import solve_ivp

    def f(t, y):
        Y = y.reshape(-1, 6)
        Xp, Vp = Y[:, :3], Y[:, 3:]
        return np.concatenate([Vp, (_shear_u(Xp) - Vp) / tau], axis=1).ravel()
    y0 = np.concatenate([X0, V0], axis=1).ravel()
    sol = solve_ivp(f, (0.0, T), y0, method="DOP853", rtol=1e-12, atol=1e-13)
    Y = sol.y[:, -1].reshape(-1, 6)
    return Y[:, :3], Y[:, 3:]


@pytest.mark.parametrize("scheme,order", [(EULER, 1), (HEUN, 2), (AB2, 2)])
def test_inertial_convergence_order(scheme, order):
    """Against the continuous solution in a smooth steady field, halving dt
    divides the error at a fixed time by about 2^order."""
    rng = np.random.default_rng(41)
    X0, V0 = rng.uniform(0, 6, (8, 3)), 0.5 * rng.standard_normal((8, 3))
    tau, T = 0.4, 0.8
    Xe, Ve = _exact_inertial(X0, V0, tau, T)
    errs = []
    for n in (40, 80):
        X, V, _, _, _ = stepping.advance_inertial(X0, V0, _shear_u, tau, scheme, T / n, n)
        errs.append(max(np.abs(X - Xe).max(), np.abs(V - Ve).max()))
    ratio = errs[0] / errs[1]
    assert 2 ** order * 0.8 < ratio < 2 ** order * 1.25, (errs, ratio)


@pytest.mark.parametrize("scheme,order", [(stepping.AB3, 3), (stepping.AB4, 4)])
def test_inertial_ab_high_order_with_exact_history(scheme, order):
    """AB3/AB4 started from the exact particle velocities and drag terms at
    the previous times (no lower-order start-up) converge at their order."""
    rng = np.random.default_rng(42)
    X0, V0 = rng.uniform(0, 6, (6, 3)), 0.5 * rng.standard_normal((6, 3))
    tau, T = 0.5, 0.6
    K = order
    errs = []
    for n in (30, 60):
        dt = T / n
        # exact states at times 0, dt, ..., (K-1) dt; start at (K-1) dt
        states = [(X0, V0)] + [_exact_inertial(X0, V0, tau, j * dt) for j in range(1, K)]
        Xs, Vs = states[-1]
        vh = np.stack([states[K - 2 - j][1] for j in range(K - 1)] + [np.zeros_like(V0)])
        rh = np.stack([stepping.drag_rhs(_shear_u(states[K - 2 - j][0]), states[K - 2 - j][1], tau)
                       for j in range(K - 1)] + [np.zeros_like(V0)])
        steps = n - (K - 1)
        X, V, _, _, _ = stepping.advance_inertial(Xs, Vs, _shear_u, tau, scheme, dt, steps, vhist=vh, rhist=rh,
                                                  hist_len=K - 1)
        Xe, Ve = _exact_inertial(X0, V0, tau, T)
        errs.append(max(np.abs(X - Xe).max(), np.abs(V - Ve).max()))
    ratio = errs[0] / errs[1]
    assert 2 ** order * 0.75 < ratio < 2 ** order * 1.3, (errs, ratio)


@pytest.mark.parametrize("scheme", [AB2, stepping.AB4])
def test_inertial_resume_bitwise(scheme):
    rng = np.random.default_rng(43)
    X0, V0 = rng.uniform(0, 6, (10, 3)), rng.standard_normal((10, 3))
    a = stepping.advance_inertial(X0, V0, _shear_u, 0.3, scheme, 0.02, 7)
    b = stepping.advance_inertial(X0, V0, _shear_u, 0.3, scheme, 0.02, 3)
    b = stepping.advance_inertial(b[0], b[1], _shear_u, 0.3, scheme, 0.02, 4, vhist=b[2], rhist=b[3],
                                  hist_len=b[4])
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)
    assert a[4] == b[4]


def test_inertial_two_fields_equal_fields_is_one_heun_step():
    rng = np.random.default_rng(44)
    X0, V0 = rng.uniform(0, 6, (10, 3)), rng.standard_normal((10, 3))
    a = stepping.heun_inertial_two_fields(X0, V0, _shear_u, _shear_u, 0.3, 0.02)
    b = stepping.advance_inertial(X0, V0, _shear_u, 0.3, HEUN, 0.02, 1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_inertial_two_fields_second_order_in_a_field_linear_in_time():
    """A uniform field u(t) = A + B t: dV/dt = (A + B t - V)/tau has the
    closed form V(t) = A + B (t - tau) + (V0 - A + B tau) e^(-t/tau), and
    X(t) = X0 + (A - B tau) t + B t^2/2 + tau (V0 - A + B tau)(1 - e^(-t/tau)).
    Steps that take each stage's field at its own time converge to it at
    second order."""
    A, B = np.array([0.4, -0.2, 0.9]), np.array([1.5, 0.7, -2.0])
    tau, T = 0.3, 0.6
    X0, V0 = np.array([[1.0, 2.0, 3.0]]), np.array([[-0.5, 0.25, 0.1]])
    e = np.exp(-T / tau)
    Ve = A + B * (T - tau) + (V0 - A + B * tau) * e
    Xe = X0 + (A - B * tau) * T + B * T * T / 2 + tau * (V0 - A + B * tau) * (1 - e)
    errs = []
    for n in (30, 60):
        dt = T / n
        X, V = X0, V0
        for k in range(n):
            t0, t1 = k * dt, (k + 1) * dt
            X, V = stepping.heun_inertial_two_fields(X, V, lambda Y, t=t0: np.broadcast_to(A + B * t, np.shape(Y)),
                                                     lambda Y, t=t1: np.broadcast_to(A + B * t, np.shape(Y)),
                                                     tau, dt)
        errs.append(max(np.abs(X - Xe).max(), np.abs(V - Ve).max()))
    ratio = errs[0] / errs[1]
    assert 3.4 < ratio < 4.6, (errs, ratio)
