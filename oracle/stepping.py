"""Tracer time stepping for dX/dt = u(X) (oracle; test infrastructure only),
and the other particle types built on it (ellipsoid axes, inertial
particles).

Follows Sec. 2.2, Eq. "tracers" (tracer ODE with X(x,0) = x) and the
multi-step Adams-Bashforth integration with an rhs history kept per particle
(Sec. 2.2; Sec. 3.3.1, the *state* and *rhs* arrays).

Readings (the paper gives neither the order nor the start-up):

* The field is frozen (no fluid solver runs beside the particles); the
  two-field Heun step (``heun_two_fields``) takes each stage's velocity from
  the field of that stage's time.
* Euler:  X <- X + dt*u(X).
* Heun:   k1 = u(X); Xs = X + dt*k1; k2 = u(Xs); X <- X + (dt/2)*(k1 + k2).
* AB2:    X <- X + dt*(3/2*u_n - 1/2*u_{n-1}) with an Euler first step; the
  history holds [u_n, u_{n-1}] and its length (0, 1 or 2) so a run can resume.
* AB3, AB4 (the paper's "multi-step" read as orders up to 4): the textbook
  Adams-Bashforth weights (from integrating the interpolant of the last k
  velocities over one step) -- AB3: 23/12, -16/12, 5/12; AB4: 55/24, -59/24,
  37/24, -9/24 -- applied as X + dt*sum_j b_j*u_{n-j} in the order j = 0, 1, ...
  While the history is shorter, the step uses the highest order it allows
  (Euler, then AB2, AB3).  The history holds the last k velocities, most
  recent first, and its length (0..k).
* The state X is the particle's position itself, not wrapped: the reduction
  modulo 2*pi is step 1 of the interpolation (Sec. 2.2), applied where the
  field is evaluated, so a trajectory keeps its crossings of the periodic
  faces (the displacement statistics the method is for need them).
* Every operation is a separately rounded binary64 operation in the order
  written (``dt/2`` is formed once as 0.5*dt).
* When a gradient is requested it is evaluated at each step's start position
  (together with the first velocity evaluation); the value returned is the one
  of the last step.
"""
from __future__ import annotations

import numpy as np

EULER, HEUN, AB2, AB3, AB4 = 1, 2, 3, 4, 5

# Adams-Bashforth weights b_j of u_{n-j}, by order
AB_WEIGHTS = {1: (1.0,), 2: (1.5, -0.5), 3: (23.0 / 12.0, -16.0 / 12.0, 5.0 / 12.0),
              4: (55.0 / 24.0, -59.0 / 24.0, 37.0 / 24.0, -9.0 / 24.0)}
AB_ORDER = {AB2: 2, AB3: 3, AB4: 4}


def euler_update(X, dt, u):
    return np.add(X, np.multiply(dt, u))


def heun_predict(X, dt, k1):
    return np.add(X, np.multiply(dt, k1))


def heun_correct(X, dt, k1, k2):
    return np.add(X, np.multiply(0.5 * dt, np.add(k1, k2)))


def ab2_update(X, dt, u_n, u_prev):
    inc = np.subtract(np.multiply(1.5, u_n), np.multiply(0.5, u_prev))
    return np.add(X, np.multiply(dt, inc))


def ab_update(X, dt, us, order: int):
    """X + dt*sum_j b_j*us[j] for us = [u_n, u_{n-1}, ...] (j = 0..order-1)."""
    b = AB_WEIGHTS[order]
    inc = np.multiply(b[0], us[0])
    for j in range(1, order):
        inc = np.add(inc, np.multiply(b[j], us[j]))
    return np.add(X, np.multiply(dt, inc))


def jeffery_rhs(A, p, shape: float):
    """Jeffery's equation for the unit axis p of an axisymmetric ellipsoid in
    a velocity gradient A[..][a][b] = du_a/dx_b (Jeffery 1922; the paper names
    ellipsoids among TurTLE's particle types, Sec. 2.2, without the equation):

        dp/dt = W p + shape (S p - (p . S p) p),

    S = (A + A^T)/2 the strain rate, W = (A - A^T)/2 the rotation rate,
    shape = (r^2 - 1)/(r^2 + 1) for the axis ratio r (0 for spheres, 1 for
    thin rods, -1 for flat discs)."""
    A = np.asarray(A, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    S = 0.5 * (A + np.swapaxes(A, -1, -2))
    W = 0.5 * (A - np.swapaxes(A, -1, -2))
    Sp = np.einsum("...ab,...b->...a", S, p)
    Wp = np.einsum("...ab,...b->...a", W, p)
    pSp = np.sum(p * Sp, axis=-1, keepdims=True)
    return Wp + shape * (Sp - pSp * p)


def normalize(p):
    """p / |p| per row (the unit length Jeffery's equation conserves)."""
    p = np.asarray(p, dtype=np.float64)
    return p / np.sqrt(np.sum(p * p, axis=-1, keepdims=True))


def advance(X, velocity, scheme: int, dt: float, nsteps: int, hist=None, hist_len: int = 0,
            gradient=None, orientation=None):
    """Advance positions X[Np][3] by nsteps.

    ``velocity(X) -> u[Np][3]``; ``gradient(X) -> (u, grad)`` if given.
    ``orientation = (p, shape[, p_hist])``: also advance unit axes p[Np][3]
    by Jeffery's equation with the same scheme (reading: every stage of the
    position scheme evaluates the gradient at its own position and the axis
    rhs with it, the axis history holds the rhs as the position history holds
    the velocity, and p is normalized once at the end of each step); needs
    ``gradient``.  Returns (X, hist, hist_len, grad_last), plus (p, p_hist)
    when an orientation is given.
    """
    X = np.array(X, dtype=np.float64)
    grad_last = None
    if hist is None:
        hist = np.zeros((AB_ORDER.get(scheme, 2),) + X.shape)
    hist = np.array(hist, dtype=np.float64)
    P = None
    if orientation is not None:
        if gradient is None:
            raise ValueError("the orientation needs the gradient")
        P = np.array(orientation[0], dtype=np.float64)
        shape = float(orientation[1])
        ph = np.array(orientation[2], dtype=np.float64) if len(orientation) > 2 and orientation[2] is not None \
            else np.zeros_like(hist)
    for _ in range(nsteps):
        if gradient is not None:
            u0, grad_last = gradient(X)
        else:
            u0 = velocity(X)
        r0 = jeffery_rhs(grad_last, P, shape) if P is not None else None
        if scheme == EULER:
            X = euler_update(X, dt, u0)
            if P is not None:
                P = normalize(euler_update(P, dt, r0))
        elif scheme == HEUN:
            Xs = heun_predict(X, dt, u0)
            if P is not None:
                Ps = heun_predict(P, dt, r0)
                k2, g2 = gradient(Xs)
                r2 = jeffery_rhs(g2, Ps, shape)
                P = normalize(heun_correct(P, dt, r0, r2))
            else:
                k2 = velocity(Xs)
            X = heun_correct(X, dt, u0, k2)
        elif scheme == AB2:
            if hist_len == 0:
                Xn = euler_update(X, dt, u0)
                Pn = euler_update(P, dt, r0) if P is not None else None
            else:
                Xn = ab2_update(X, dt, u0, hist[0])
                Pn = ab2_update(P, dt, r0, ph[0]) if P is not None else None
            hist[1] = hist[0]
            hist[0] = u0
            if P is not None:
                ph[1] = ph[0]
                ph[0] = r0
                P = normalize(Pn)
            hist_len = min(hist_len + 1, 2)
            X = Xn
        elif scheme in (AB3, AB4):
            K = AB_ORDER[scheme]
            q = min(K, hist_len + 1)
            Xn = ab_update(X, dt, [u0] + [hist[j] for j in range(q - 1)], q)
            if P is not None:
                Pn = ab_update(P, dt, [r0] + [ph[j] for j in range(q - 1)], q)
            for j in range(K - 1, 0, -1):
                hist[j] = hist[j - 1]
                if P is not None:
                    ph[j] = ph[j - 1]
            hist[0] = u0
            if P is not None:
                ph[0] = r0
                P = normalize(Pn)
            hist_len = min(hist_len + 1, K)
            X = Xn
        else:
            raise ValueError("unknown scheme")
    if P is not None:
        return X, hist, hist_len, grad_last, P, ph
    return X, hist, hist_len, grad_last


def drag_rhs(u, V, tau: float):
    """Rate of change of an inertial particle's velocity V in the fluid
    velocity u at its position, (u - V)/tau: a small heavy particle under
    linear (Stokes) drag with response time tau.  Reading: the paper names
    inertial particles among TurTLE's particle types (Sec. 2.2) without their
    equation; this is the heavy-particle limit with drag only (no gravity,
    added mass or history force)."""
    return np.divide(np.subtract(u, V), tau)


def advance_inertial(X, V, velocity, tau: float, scheme: int, dt: float, nsteps: int, vhist=None, rhist=None,
                     hist_len: int = 0):
    """Advance inertial particles, dX/dt = V and dV/dt = drag_rhs(u(X), V, tau),
    by nsteps with the tracer schemes applied to the pair (X, V) (reading, as
    for the ellipsoid axes: every stage evaluates u at its own position):

    * Euler:  r = drag(u(X), V); X <- X + dt*V; V <- V + dt*r.
    * Heun:   r1 = drag(u(X), V); Xs = X + dt*V; Vs = V + dt*r1;
              r2 = drag(u(Xs), Vs); X <- X + (dt/2)*(V + Vs);
              V <- V + (dt/2)*(r1 + r2).
    * AB2..AB4: X <- X + dt*sum_j b_j*V_{n-j}, V <- V + dt*sum_j b_j*r_{n-j}
      with the weights, start-up and history rules of ``advance``: vhist holds
      the earlier particle velocities and rhist the earlier drag terms, most
      recent first, with one shared length.

    ``velocity(X) -> u[Np][3]``.  Returns (X, V, vhist, rhist, hist_len)."""
    X = np.array(X, dtype=np.float64)
    V = np.array(V, dtype=np.float64)
    K = AB_ORDER.get(scheme, 2)
    vh = np.zeros((K,) + X.shape) if vhist is None else np.array(vhist, dtype=np.float64)
    rh = np.zeros((K,) + X.shape) if rhist is None else np.array(rhist, dtype=np.float64)
    for _ in range(nsteps):
        r1 = drag_rhs(velocity(X), V, tau)
        if scheme == EULER:
            X, V = euler_update(X, dt, V), euler_update(V, dt, r1)
        elif scheme == HEUN:
            Xs = heun_predict(X, dt, V)
            Vs = heun_predict(V, dt, r1)
            r2 = drag_rhs(velocity(Xs), Vs, tau)
            X, V = heun_correct(X, dt, V, Vs), heun_correct(V, dt, r1, r2)
        elif scheme in (AB2, AB3, AB4):
            q = min(K, hist_len + 1)
            Xn = ab_update(X, dt, [V] + [vh[j] for j in range(q - 1)], q)
            Vn = ab_update(V, dt, [r1] + [rh[j] for j in range(q - 1)], q)
            for j in range(K - 1, 0, -1):
                vh[j] = vh[j - 1]
                rh[j] = rh[j - 1]
            vh[0] = V
            rh[0] = r1
            hist_len = min(hist_len + 1, K)
            X, V = Xn, Vn
        else:
            raise ValueError("unknown scheme")
    return X, V, vh, rh, hist_len


def heun_inertial_two_fields(X, V, vel_now, vel_next, tau: float, dt: float):
    """One Heun step of inertial particles (``advance_inertial``) in a field
    that changes during the step, the stages taking the fields of their own
    times as in ``heun_two_fields``:

        r1 = drag(u(X, t_n), V);  Xs = X + dt*V;  Vs = V + dt*r1;
        r2 = drag(u(Xs, t_n + dt), Vs);
        X <- X + (dt/2)*(V + Vs);  V <- V + (dt/2)*(r1 + r2).

    Returns (X, V)."""
    X = np.array(X, dtype=np.float64)
    V = np.array(V, dtype=np.float64)
    r1 = drag_rhs(vel_now(X), V, tau)
    Xs = heun_predict(X, dt, V)
    Vs = heun_predict(V, dt, r1)
    r2 = drag_rhs(vel_next(Xs), Vs, tau)
    return heun_correct(X, dt, V, Vs), heun_correct(V, dt, r1, r2)


def heun_two_fields(X, vel_now, vel_next, dt: float, gradient_now=None):
    """One Heun step in a field that changes during the step (Eq. "tracers"
    with u = u(x, t)): the first stage takes the velocity of the field at the
    step's start time, the second that of the field at its end time,

        k1 = u(X, t_n);  Xs = X + dt*k1;  k2 = u(Xs, t_n + dt);
        X <- X + (dt/2)*(k1 + k2).

    ``vel_now(X)`` and ``vel_next(X)`` evaluate the two fields;
    ``gradient_now(X) -> (u, grad)`` (optional) replaces vel_now for the first
    stage and its gradient is returned.  Returns (X, grad or None)."""
    X = np.array(X, dtype=np.float64)
    grad = None
    if gradient_now is not None:
        k1, grad = gradient_now(X)
    else:
        k1 = vel_now(X)
    Xs = heun_predict(X, dt, k1)
    k2 = vel_next(Xs)
    return heun_correct(X, dt, k1, k2), grad
