"""Seeded synthetic inputs: unstructured triangular meshes and analytic nodal fields.

This module generates *inputs only*.  It holds none of the particle method's
arithmetic (no interpolation, no SDE, no tracking, no statistics), so both the
GPU library and the CPU oracle may consume what it produces.

Workloads follow the structure of the paper's test cases (Sec. 4): a periodic
channel with no-slip walls at y = -1 and y = +1 whose grid is stretched towards
the walls (Sec. 3.7, Sec. 4.1), and a street canyon: a square cavity under a
channel with a free-slip top and periodic in/outflow (Sec. 4.2).  The analytic
nodal fields stand in for the pressure-projection and elliptic-relaxation solves
(Sec. 3.2), which are not part of the particle time step.

Mesh conventions (shared with the C ABI):
  * ``xy``   float64 [n_nodes, 2]
  * ``tri``  int32  [n_elems, 3], counter-clockwise
  * ``edge_kind`` uint8 [n_elems, 3]; edge k is the edge opposite vertex k;
    0 interior, 1 no-slip wall, 2 free-slip wall, 3 periodic.  Only edges that
    belong to a single element are read; shared edges are classified from the
    geometry.
  * ``period_x`` > 0 when x is periodic; nodes then lie in [0, period_x) and the
    elements that straddle the seam reference the nodes at x = 0.
Field conventions: symmetric tensors are stored as (11, 22, 33, 12, 13, 23).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

EDGE_INTERIOR, EDGE_WALL, EDGE_SLIP, EDGE_PERIODIC = 0, 1, 2, 3

# Table 4 constants used on the particle path, plus C_s, C_t of Eq. (25) (Sec. 4.1.2).
TABLE4 = dict(C3=5.0, C4=0.25, CT=6.0, Cw1=0.5, Cw2=0.73, Cs=0.02, Ct=0.7)
# Viscosity and density of the synthetic workloads (the paper quotes only Re_tau).
NU, RHO = 1.0e-4, 1.0
MASTER_SEED = 0x10060532


@dataclass
class Mesh:
    xy: np.ndarray
    tri: np.ndarray
    edge_kind: np.ndarray
    period_x: float
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.tri.shape[0])


@dataclass
class Fields:
    grad_p: np.ndarray      # [n, 2]
    wp: np.ndarray          # [n, 6]  elliptic-relaxation tensor
    mean_u: np.ndarray      # [n, 3]
    mean_omega: np.ndarray  # [n]
    rey: np.ndarray         # [n, 6]  Reynolds stresses <u_i u_j>

    def as_tuple(self):
        return (self.grad_p, self.wp, self.mean_u, self.mean_omega, self.rey)


def model_constants(nu: float = NU, rho: float = RHO) -> dict:
    d = dict(nu=nu, rho=rho)
    d.update(TABLE4)
    return d


# ---------------------------------------------------------------------------------
# structured-topology channel / box generator
# ---------------------------------------------------------------------------------

def _wall_graded_y(ny: int, stretch: float, y0: float, y1: float) -> np.ndarray:
    """Node rows between y0 and y1, geometric in cell size towards both walls.

    ``stretch`` is the ratio between the largest (centre) and smallest (wall)
    cell; with ny/2 cells per half the per-cell ratio is stretch**(1/(ny/2-1)).
    """
    if ny % 2 != 0:
        raise ValueError("ny must be even")
    half = ny // 2
    r = stretch ** (1.0 / (half - 1)) if half > 1 else 1.0
    h = np.array([r ** k for k in range(half)], dtype=np.float64)
    h *= (0.5 * (y1 - y0)) / h.sum()
    y = np.empty(ny + 1, dtype=np.float64)
    y[0] = y0
    for j in range(half):
        y[j + 1] = y[j] + h[j]
    y[half] = 0.5 * (y0 + y1)
    for j in range(half):
        y[ny - j] = y0 + y1 - y[j]
    return y


def channel_mesh(nx: int, ny: int, *, length: float = 2.0 * math.pi, y0: float = -1.0,
                 y1: float = 1.0, stretch: float = 1.1 ** 24, jitter: float = 0.1,
                 seed: int = MASTER_SEED, bottom: int = EDGE_WALL, top: int = EDGE_WALL,
                 periodic: bool = True, random_diagonals: bool = True) -> Mesh:
    """Periodic channel strip of nx*ny quads, each split along a seeded diagonal.

    Nodes: column i (0..nx-1) at x = i*length/nx, rows from ``_wall_graded_y``.
    Interior nodes are jittered by U(-jitter, jitter) of the local spacing: in x by
    the column spacing (the seam column x = 0 keeps x = 0), in y by the smaller of
    the two adjacent row spacings.  Wall rows are not jittered.
    Node id = j*nx + i; element ids run row by row, two per quad.
    """
    rng = np.random.default_rng(seed)
    ys = _wall_graded_y(ny, stretch, y0, y1)
    dx = length / nx
    ncol = nx if periodic else nx + 1
    X = np.empty((ny + 1, ncol), dtype=np.float64)
    Y = np.empty((ny + 1, ncol), dtype=np.float64)
    for j in range(ny + 1):
        X[j, :] = np.arange(ncol, dtype=np.float64) * dx
        Y[j, :] = ys[j]
    jx = rng.uniform(-jitter, jitter, size=(ny + 1, ncol))
    jy = rng.uniform(-jitter, jitter, size=(ny + 1, ncol))
    for j in range(1, ny):
        hmin = min(ys[j] - ys[j - 1], ys[j + 1] - ys[j])
        Y[j, :] += jy[j, :] * hmin
        if periodic:
            X[j, 1:] += jx[j, 1:] * dx
        else:
            X[j, 1:ncol - 1] += jx[j, 1:ncol - 1] * dx
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)

    diag = rng.integers(0, 2, size=(ny, nx)) if random_diagonals else np.zeros((ny, nx), int)
    J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    IP = (I + 1) % ncol if periodic else I + 1
    n00, n10 = J * ncol + I, J * ncol + IP
    n01, n11 = (J + 1) * ncol + I, (J + 1) * ncol + IP
    d0 = (diag == 0)
    t0 = np.where(d0[..., None], np.stack([n00, n10, n11], -1), np.stack([n00, n10, n01], -1))
    t1 = np.where(d0[..., None], np.stack([n00, n11, n01], -1), np.stack([n10, n11, n01], -1))
    tri = np.stack([t0, t1], axis=2).reshape(-1, 3).astype(np.int32)
    # boundary kinds: an edge whose two nodes both lie on the bottom (top) row, or,
    # without periodicity, on the first (last) column
    row = np.arange(xy.shape[0]) // ncol
    col = np.arange(xy.shape[0]) % ncol
    kind = np.zeros(tri.shape, dtype=np.uint8)
    for k in range(3):
        a, b = tri[:, (k + 1) % 3], tri[:, (k + 2) % 3]
        kind[(row[a] == 0) & (row[b] == 0), k] = bottom
        kind[(row[a] == ny) & (row[b] == ny), k] = top
        if not periodic:
            side = (col[a] == col[b]) & ((col[a] == 0) | (col[a] == ncol - 1))
            kind[side, k] = EDGE_SLIP
    return Mesh(xy=xy, tri=tri, edge_kind=kind, period_x=length if periodic else 0.0,
                meta=dict(kind="channel", nx=nx, ny=ny, length=length, y0=y0, y1=y1,
                          stretch=stretch, jitter=jitter, seed=seed))


def channel_fields(mesh: Mesh, *, wp_diag: float = -0.1, r_diag: float = 0.05 ** 2,
                   r12_slope: float = 0.002) -> Fields:
    """Analytic channel fields at the nodes.

    <U> = (1.5 (1 - y^2), 0, 0); grad<P> = (-1, 0);
    <omega> = min(1 + 10 (1 - |y|)^(-1/2), 50) (50 on the walls);
    elliptic-relaxation tensor = wp_diag * I; Reynolds stresses r_diag * I with
    <u v> = r12_slope * y.
    """
    y = mesh.xy[:, 1]
    n = mesh.n_nodes
    grad_p = np.zeros((n, 2))
    grad_p[:, 0] = -1.0
    wp = np.zeros((n, 6))
    wp[:, 0:3] = wp_diag
    mu = np.zeros((n, 3))
    mu[:, 0] = 1.5 * (1.0 - y * y)
    d = 1.0 - np.abs(y)
    with np.errstate(divide="ignore"):
        om = np.where(d > 0, 1.0 + 10.0 / np.sqrt(np.maximum(d, 1e-300)), np.inf)
    om = np.minimum(om, 50.0)
    rey = np.zeros((n, 6))
    rey[:, 0:3] = r_diag
    rey[:, 3] = r12_slope * y
    return Fields(grad_p=grad_p, wp=wp, mean_u=mu, mean_omega=om, rey=rey)


def uniform_fields(mesh: Mesh, *, grad_p=(0.0, 0.0), wp=(-0.1, -0.1, -0.1, 0, 0, 0),
                   mean_u=(0.0, 0.0, 0.0), mean_omega=10.0,
                   rey=(0.0025, 0.0025, 0.0025, 0, 0, 0)) -> Fields:
    n = mesh.n_nodes
    return Fields(grad_p=np.tile(np.asarray(grad_p, float), (n, 1)),
                  wp=np.tile(np.asarray(wp, float), (n, 1)),
                  mean_u=np.tile(np.asarray(mean_u, float), (n, 1)),
                  mean_omega=np.full(n, float(mean_omega)),
                  rey=np.tile(np.asarray(rey, float), (n, 1)))


# ---------------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------------

def init_desc(**kw) -> dict:
    d = dict(ppe=50, u_sigma=0.05, omega_shape=4.0, src_x=math.pi, src_y=0.0, src_r=0.05,
             src_continuous=1, bins=(4, 2, 2), min_per_bin=2, seed=MASTER_SEED, capacity=0)
    d.update(kw)
    return d


def channel_small(nx=40, ny=50, seed=MASTER_SEED):
    """Plain FP64 channel strip: 40x50 quads -> 4000 triangles, 50 particles per element."""
    mesh = channel_mesh(nx, ny, seed=seed)
    return mesh, channel_fields(mesh), model_constants(), init_desc(ppe=50, bins=(4, 2, 2))


def channel_large(nx=400, ny=500, ppe=200, seed=MASTER_SEED):
    """FP64 channel at GPU scale: 400x500 quads -> 4e5 triangles, 200 particles per element.

    The per-cell growth is chosen so that the largest/smallest cell ratio equals the
    small channel's (1.1**24).
    """
    mesh = channel_mesh(nx, ny, seed=seed)
    return mesh, channel_fields(mesh), model_constants(), init_desc(ppe=ppe, bins=(4, 2, 2))


WORKLOADS = {
    "channel_small": dict(fn=channel_small, dt=1e-3, steps=20, control=None),
    "channel_large": dict(fn=channel_large, dt=2e-4, steps=100, control=(150, 250)),
}
