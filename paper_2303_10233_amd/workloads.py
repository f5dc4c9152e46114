"""Seeded synthetic inputs shaped like the paper's test problems.

This module generates inputs only (coordinates, random numbers and the
analytic fields evaluated at nodes); it holds none of the method's arithmetic.
It is the one module shared by the GPU path's tests/benchmarks and the CPU
oracle, so both sides see bit-identical inputs.
"""
import numpy as np


def q2_node_coords(n, x0=0.0, x1=1.0, y0=0.0, y1=1.0):
    """x, y of the (2n+1)^2 Q2 nodes, row-major with x fastest."""
    tx = x0 + (x1 - x0) * np.arange(2 * n + 1) / (2 * n)
    ty = y0 + (y1 - y0) * np.arange(2 * n + 1) / (2 * n)
    X, Y = np.meshgrid(tx, ty, indexing="xy")
    return X.reshape(-1), Y.reshape(-1)


def bump_parameters(seed, nbumps=8, x0=0.0, x1=1.0, y0=0.0, y1=1.0):
    """Centres ~ U(domain), widths ~ U[0.05, 0.2] (scaled with the domain
    side), amplitudes in R^2 ~ N(0, 1), drawn with numpy's PCG64 stream."""
    rng = np.random.default_rng(seed)
    cx = rng.uniform(x0, x1, nbumps)
    cy = rng.uniform(y0, y1, nbumps)
    sig = rng.uniform(0.05, 0.2, nbumps) * (x1 - x0)
    amp = rng.standard_normal((nbumps, 2))
    return cx, cy, sig, amp


def gaussian_bumps(n, seed, x0=0.0, x1=1.0, y0=0.0, y1=1.0, nbumps=8):
    """Nodal forcing f = sum_k a_k exp(-|x - c_k|^2 / (2 s_k^2)) on the Q2
    nodes, layout [f_x (2n+1)^2 | f_y (2n+1)^2]."""
    X, Y = q2_node_coords(n, x0, x1, y0, y1)
    cx, cy, sig, amp = bump_parameters(seed, nbumps, x0, x1, y0, y1)
    fx = np.zeros_like(X)
    fy = np.zeros_like(X)
    for k in range(nbumps):
        g = np.exp(-((X - cx[k]) ** 2 + (Y - cy[k]) ** 2) / (2 * sig[k] ** 2))
        fx += amp[k, 0] * g
        fy += amp[k, 1] * g
    return np.concatenate([fx, fy])


def recirculating_wind(n, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0):
    """Nodal values of w = (2y(1-x^2), -2x(1-y^2)), layout [w_x | w_y]."""
    X, Y = q2_node_coords(n, x0, x1, y0, y1)
    return np.concatenate([2 * Y * (1 - X ** 2), -2 * X * (1 - Y ** 2)])


def uniform_vector(length, seed, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, length)


def ragged_sizes(count=32):
    """Mesh sizes n_i = 32 + 16 (i mod 15) of the ragged cavity batch."""
    return [32 + 16 * (i % 15) for i in range(count)]
