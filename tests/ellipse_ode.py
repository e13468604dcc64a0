"""Reference for the water-drop test: the semi-axes of an inviscid
incompressible elliptic drop with a linear velocity field (plain numpy)."""
import numpy as np


def ellipse_axes_ode(strain, radius, t_end, nsub):
    """Semi-axes a(t), b(t) of an inviscid incompressible elliptic drop whose
    velocity field stays linear, u = -A x, v = A y, from a circle of radius R
    with A(0) = A0 (the analysis of the water-drop test the paper cites):
    the Euler equations with zero pressure on the ellipse give
    da/dt = -A a, db/dt = A b, dA/dt = A^2 (a^2 - b^2) / (a^2 + b^2).
    Classical RK4 with nsub steps; returns arrays t, a, b."""
    def f(y):
        a, b, A = y
        return np.array([-A * a, A * b, A * A * (a * a - b * b) / (a * a + b * b)])
    h = t_end / nsub
    y = np.array([radius, radius, strain])
    out = [y.copy()]
    for _ in range(nsub):
        k1 = f(y)
        k2 = f(y + 0.5 * h * k1)
        k3 = f(y + 0.5 * h * k2)
        k4 = f(y + h * k3)
        y = y + h / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        out.append(y.copy())
    out = np.array(out)
    return np.linspace(0.0, t_end, nsub + 1), out[:, 0], out[:, 1]
