"""A steady two-dimensional cellular flow for time-order tests of the tracer
schemes (Sec. 4.1.1 reports second order for the two-stage and third order for
the three-stage Runge-Kutta option).

The gas velocity v = (sin(pi x) cos(pi y) + 0.3, -cos(pi x) sin(pi y) + 0.2)
on [0, 2)^2 is sampled at the cell centres of a fine 256^2 grid.  With the
field grid fixed, refining only dt isolates the time error: the reference is
the exact trajectory of the TSC-interpolated field, integrated by an adaptive
eighth-order solver (scipy's DOP853) at a tolerance far below the errors
measured.  (The paper's own one-dimensional test couples dt to the cell size,
so its O(dx^2) sampling error hides the third order; in one dimension the
periodic flow also averages the leading error term of the three-stage scheme
away, which shows as a steeper slope.)
"""

import numpy as np

N = 256
L = 2.0
DX = L / N
T = 3.0
X0 = (0.37 / DX, 0.81 / DX)          # start, in cells


def field():
    c = (np.arange(N) + 0.5) * DX
    xc, yc = np.meshgrid(c, c)        # [j, i]
    vg = np.zeros((3, 1, N, N))
    vg[0, 0] = np.sin(np.pi * xc) * np.cos(np.pi * yc) + 0.3
    vg[1, 0] = -np.cos(np.pi * xc) * np.sin(np.pi * yc) + 0.2
    return vg


def reference(orc, vg):
    """Position (cells) at t = T of the exact trajectory of the interpolated field."""
    from scipy.integrate import solve_ivp
    n = (N, N, 1)

    def rhs(t, y):
        p = [y[0] % N, y[1] % N]
        return [orc.gather(2, n, 2, vg[0], p) / DX, orc.gather(2, n, 2, vg[1], p) / DX]

    sol = solve_ivp(rhs, (0.0, T), list(X0), method="DOP853", rtol=1e-13, atol=1e-9)
    return sol.y[:, -1]


def distance(a, b):
    """Minimum-image distance in length units of two positions in cells."""
    d = (np.asarray(a[:2]) - np.asarray(b[:2]) + N / 2) % N - N / 2
    return float(np.hypot(d[0], d[1])) * DX
