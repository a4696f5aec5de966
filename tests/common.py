"""Shared helpers for the tests: small seeded workloads and comparison utilities."""
import math

import numpy as np

from paper_1006_0532_amd import workloads as W


def box(nx=8, ny=8, *, length=2.0, bottom=W.EDGE_SLIP, top=W.EDGE_SLIP, jitter=0.1,
        stretch=1.0, seed=11, random_diagonals=True):
    """Periodic-in-x box on y in [-1, 1]."""
    return W.channel_mesh(nx, ny, length=length, y0=-1.0, y1=1.0, stretch=stretch,
                          jitter=jitter, seed=seed, bottom=bottom, top=top,
                          random_diagonals=random_diagonals)


def frozen_fields(mesh, *, omega=1.0, r_diag=0.5, mean_u=(0.0, 0.0, 0.0), grad_p=(0.0, 0.0)):
    """Uniform fields with G = 0 and C0 eps clamped to 0 when nu = 0 (wp = eps/2 I)."""
    k = 1.5 * r_diag
    eps = omega * k
    return W.uniform_fields(mesh, grad_p=grad_p, wp=(0.5 * eps,) * 3 + (0.0,) * 3,
                            mean_u=mean_u, mean_omega=omega, rey=(r_diag,) * 3 + (0.0,) * 3)


def edge_distance(frame, e, x, y):
    """Smallest distance of (x, y) to the three edge lines of element e."""
    v = frame[e].reshape(3, 2)
    d = np.inf
    for k in range(3):
        a, b = v[(k + 1) % 3], v[(k + 2) % 3]
        ex, ey = b - a
        L = math.hypot(ex, ey)
        d = min(d, abs((x - a[0]) * ey - (y - a[1]) * ex) / L)
    return d


def shift_periodic(mesh, dx):
    """The same periodic mesh with every node moved by -dx in x (mod the period): an input
    transform that puts a chosen column of nodes on the seam x = 0."""
    L = mesh.period_x
    xy = mesh.xy.copy()
    xy[:, 0] = np.mod(xy[:, 0] - dx, L)
    xy[xy[:, 0] >= L, 0] = 0.0
    return W.Mesh(xy, mesh.tri, mesh.edge_kind, L, dict(mesh.meta))
