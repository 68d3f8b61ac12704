"""Batched constant-pressure homogeneous reactor step (oracle).

The paper integrates its thermochemistry subsystem, Eq. (1a)-(1b), implicitly with a
stiff solver (Section 2); at a single point with no transport terms that subsystem is
an adiabatic reactor at constant pressure (the homogeneous autoignition of Section
3.1):  x = (T, Y_1..Y_Ns),  dx/dt = f(x) = (dT/dt, dY/dt) from source.py with
dp0/dt = 0.

Jacobian of f, by the chain rule from the Jacobian J of (hrr, w) (jacobian.py) through
rho = p Wbar/(R T) and c_p = sum_k Y_k c_p,k(T)/W_k:

    d rho/dT = -rho/T,   d rho/dY_j = -rho Wbar/W_j,
    d c_p/dT = sum_k Y_k c_p,k'(T)/W_k,   d c_p/dY_j = c_p,j/W_j,
    d(dY_k/dt)/dx = (W_k/rho) (dw_k/dx - w_k (d rho/dx)/rho),
    d(dT/dt)/dx   = (d hrr/dx)/(rho c_p) - (dT/dt) ((d rho/dx)/rho + (d c_p/dx)/c_p).

Step: the two-stage Rosenbrock method ROS2 (Verwer, Spee, Blom and Hundsdorfer, 1999),
L-stable and of order two, applied nsub times with h = dt/nsub and the Jacobian
evaluated once per substep at its start:

    (I - gamma h A) k1 = f(x_n),
    (I - gamma h A) k2 = f(x_n + h k1) - 2 k1,
    x_{n+1} = x_n + (3/2) h k1 + (1/2) h k2,       gamma = 1 + 1/sqrt(2),

with A the Jacobian of f at x_n; the linear systems are solved with numpy's dense
solver (LU with partial pivoting).

Pinned by: complex-step differentiation of f (source_jacobian); the method's own
stability function R(z) = (1 + (1 - 2 gamma) z) / (1 - gamma z)^2 on an isothermal
isomerisation, whose exact solution the step approaches at second order; the
equilibrium state as a fixed point; conservation of sum_k Y_k and of the elements.
"""
from __future__ import annotations

import numpy as np

from .jacobian import jacobian
from .source import chemistry_source
from .thermo import nasa7

GAMMA = 1.0 + 1.0 / np.sqrt(2.0)


def rhs(m, T, p, Y):
    """f(x) as [n, Ns+1]: column 0 dT/dt, columns 1.. dY_k/dt (dp0/dt = 0)."""
    s = chemistry_source(m, T, p, Y)
    return np.concatenate([s["dTdt"][:, None], s["dYdt"]], axis=1)


def source_jacobian(m, T, p, Y):
    """A = df/dx [n, Ns+1, Ns+1], rows (dT/dt, dY_k/dt), columns (T, Y_j)."""
    T = np.asarray(T)
    Y = np.asarray(Y)
    n, ns = Y.shape
    s = chemistry_source(m, T, p, Y)
    J = jacobian(m, T, p, Y)
    rho, cp, w = s["rho"], s["cp_mass"], s["wdot"]
    Wbar = 1.0 / (Y / m.W[None, :]).sum(axis=1)
    cpR, _, _, _ = nasa7(m, T)
    # c_p,k'(T) / R = a2 + 2 a3 T + 3 a4 T^2 + 4 a5 T^3 of the range in use
    low = (np.asarray(T).real[:, None] <= m.t_mid[None, :])
    a = np.where(low[:, :, None], m.a_lo[None, :, :], m.a_hi[None, :, :])
    Tc = T[:, None]
    dcpR = a[:, :, 1] + 2 * a[:, :, 2] * Tc + 3 * a[:, :, 3] * Tc ** 2 + 4 * a[:, :, 4] * Tc ** 3
    drho = np.concatenate([(-rho / T)[:, None], -rho[:, None] * Wbar[:, None] / m.W[None, :]], axis=1)
    dcp = np.concatenate([(Y * m.R * dcpR / m.W[None, :]).sum(axis=1)[:, None], m.R * cpR / m.W[None, :]],
                         axis=1)
    A = np.zeros((n, ns + 1, ns + 1), dtype=np.result_type(T, Y, float))
    A[:, 1:, :] = (m.W[None, :, None] / rho[:, None, None]) * (J[:, 1:, :] - w[:, :, None] * drho[:, None, :]
                                                               / rho[:, None, None])
    A[:, 0, :] = J[:, 0, :] / (rho * cp)[:, None] - s["dTdt"][:, None] * (drho / rho[:, None] + dcp / cp[:, None])
    return A


def ros2_step(m, T, p, Y, dt, nsub=1):
    """(T, Y) after nsub ROS2 substeps of h = dt/nsub each."""
    T = np.array(T, dtype=float)
    Y = np.array(Y, dtype=float)
    n, ns = Y.shape
    h = dt / nsub
    eye = np.eye(ns + 1)[None]
    for _ in range(nsub):
        x = np.concatenate([T[:, None], Y], axis=1)
        A = source_jacobian(m, T, p, Y)
        Mx = eye - GAMMA * h * A
        k1 = np.linalg.solve(Mx, rhs(m, T, p, Y)[:, :, None])[:, :, 0]
        xs = x + h * k1
        k2 = np.linalg.solve(Mx, (rhs(m, xs[:, 0], p, xs[:, 1:]) - 2.0 * k1)[:, :, None])[:, :, 0]
        x = x + 1.5 * h * k1 + 0.5 * h * k2
        T, Y = x[:, 0], x[:, 1:]
    return T, Y
