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
# street canyon: square cavity under a periodic channel
# ---------------------------------------------------------------------------------

def _cluster_both(a: float, b: float, n: int, beta: float) -> np.ndarray:
    """n+1 points from a to b, tanh-clustered towards both ends."""
    s = np.arange(n + 1, dtype=np.float64) / n
    xi = 0.5 * (1.0 + np.tanh(beta * (2.0 * s - 1.0)) / math.tanh(beta))
    xi[0], xi[-1] = 0.0, 1.0
    return a + (b - a) * xi


def _cluster_low(a: float, b: float, n: int, beta: float) -> np.ndarray:
    """n+1 points from a to b, tanh-clustered towards a."""
    s = np.arange(n + 1, dtype=np.float64) / n
    xi = 1.0 + np.tanh(beta * (s - 1.0)) / math.tanh(beta)
    xi[0], xi[-1] = 0.0, 1.0
    return a + (b - a) * xi


def _incircle(ax, ay, bx, by, cx, cy, dx, dy):
    """> 0 when d lies inside the circumcircle of the counter-clockwise triangle abc."""
    adx, ady, bdx, bdy, cdx, cdy = ax - dx, ay - dy, bx - dx, by - dy, cx - dx, cy - dy
    return ((adx * adx + ady * ady) * (bdx * cdy - cdx * bdy)
            - (bdx * bdx + bdy * bdy) * (adx * cdy - cdx * ady)
            + (cdx * cdx + cdy * cdy) * (adx * bdy - bdx * ady))


def cavity_mesh(nxh: int, ny_channel: int, ny_cavity: int, *, H: float = 1.0, jitter: float = 0.1,
                beta: float = 1.6, seed: int = MASTER_SEED) -> Mesh:
    """Street canyon: a square H x H cavity (x in [H, 2H], y in [0, H]) under a channel
    of height H (y in [H, 2H]) that is periodic in x over 3H (Sec. 4.2 geometry).

    Node columns: nxh cells across the cavity and 2*nxh across the rest of the period,
    both tanh-clustered towards the cavity's side walls; rows: ny_cavity cells in the
    cavity clustered towards its floor and its top corners, ny_channel cells in the
    channel clustered towards the street level y = H.  Interior nodes are jittered by
    U(-jitter, jitter) of the smaller adjacent spacing (the seam column x = 0, the
    columns x = H, 2H and the rows y = 0, H, 2H stay fixed).  Every quad is split along
    its Delaunay diagonal (one Lawson test per quad; cocircular quads take a seeded
    random diagonal).  Boundaries: no-slip street level, cavity walls and floor;
    free-slip top y = 2H.  About 2 (3 nxh ny_channel + nxh ny_cavity) triangles.
    """
    rng = np.random.default_rng(seed)
    L = 3.0 * H
    cav = _cluster_both(H, 2 * H, nxh, beta)                # [H, 2H]
    out = _cluster_both(2 * H, 4 * H, 2 * nxh, beta)        # [2H, 4H] = [2H, 3H) + [0, H) wrapped
    xs = np.concatenate([out[nxh:2 * nxh] - L, cav[:nxh], out[:nxh]])     # [0, 3H), 3 nxh columns
    ncol, iH, i2H = 3 * nxh, nxh, 2 * nxh
    yc = _cluster_low(H, 2 * H, ny_channel, beta)           # channel rows, y = H first
    yv = _cluster_both(0.0, H, ny_cavity, beta)[::-1]       # cavity rows, y = H first

    # channel block: rows 0..ny_channel, all columns; cavity block: rows 1..ny_cavity of
    # columns iH..i2H
    X = np.tile(xs, (ny_channel + 1, 1))
    Y = np.tile(yc[:, None], (1, ncol))
    ncv = nxh + 1
    XV = np.tile(xs[iH:i2H + 1], (ny_cavity, 1))
    YV = np.tile(yv[1:, None], (1, ncv))

    dxs = np.diff(np.append(xs, L))                        # spacing to the right of each column
    left = np.roll(dxs, 1)
    hx = np.minimum(dxs, left)
    for j in range(1, ny_channel):
        hy = min(yc[j] - yc[j - 1], yc[j + 1] - yc[j])
        cols = np.ones(ncol, bool)
        cols[[0, iH, i2H]] = False
        X[j, cols] += rng.uniform(-jitter, jitter, cols.sum()) * hx[cols]
        Y[j, cols] += rng.uniform(-jitter, jitter, cols.sum()) * hy
    for j in range(ny_cavity - 1):          # cavity rows 1..ny_cavity-1 (row ny_cavity is the floor)
        r = j + 1
        hy = min(yv[r - 1] - yv[r], yv[r] - yv[r + 1])
        inner = slice(1, ncv - 1)
        XV[j, inner] += rng.uniform(-jitter, jitter, ncv - 2) * hx[iH + 1:i2H]
        YV[j, inner] += rng.uniform(-jitter, jitter, ncv - 2) * hy
    xy = np.concatenate([np.stack([X.ravel(), Y.ravel()], 1), np.stack([XV.ravel(), YV.ravel()], 1)])
    base = (ny_channel + 1) * ncol

    quads = []
    # channel quads: lower row j, upper row j+1 (y grows with j)
    J, I = np.meshgrid(np.arange(ny_channel), np.arange(ncol), indexing="ij")
    IP = (I + 1) % ncol
    quads.append(np.stack([J * ncol + I, J * ncol + IP, (J + 1) * ncol + IP, (J + 1) * ncol + I], -1).reshape(-1, 4))

    # cavity quads: upper row r (r = 0 is the channel's street row), lower row r+1
    def vid(r, c):          # c = 0..nxh relative to column iH
        return np.where(r == 0, (iH + c) % ncol, base + (r - 1) * ncv + c)
    R, Cc = np.meshgrid(np.arange(ny_cavity), np.arange(nxh), indexing="ij")
    quads.append(np.stack([vid(R + 1, Cc), vid(R + 1, Cc + 1), vid(R, Cc + 1), vid(R, Cc)], -1).reshape(-1, 4))
    q = np.concatenate(quads).astype(np.int64)

    # unwrap the seam for the geometric tests
    P = xy[q]                                   # [nq, 4, 2]
    span = P[:, :, 0].max(1) - P[:, :, 0].min(1)
    wrap = span > 0.5 * L
    P[wrap, :, 0] = np.where(P[wrap, :, 0] < 0.5 * L, P[wrap, :, 0] + L, P[wrap, :, 0])
    inc = _incircle(P[:, 0, 0], P[:, 0, 1], P[:, 1, 0], P[:, 1, 1], P[:, 2, 0], P[:, 2, 1], P[:, 3, 0], P[:, 3, 1])
    scale = np.abs(P[:, 2, 0] - P[:, 0, 0]) + np.abs(P[:, 2, 1] - P[:, 0, 1])
    tie = np.abs(inc) <= 1e-12 * scale ** 4
    # diagonal 0-2 is Delaunay when vertex 3 is outside the circumcircle of (0, 1, 2)
    use02 = np.where(tie, rng.integers(0, 2, len(q)) == 0, inc <= 0)
    t0 = np.where(use02[:, None], q[:, [0, 1, 2]], q[:, [0, 1, 3]])
    t1 = np.where(use02[:, None], q[:, [0, 2, 3]], q[:, [1, 2, 3]])
    tri = np.stack([t0, t1], 1).reshape(-1, 3).astype(np.int32)

    # boundary edges: edges of one element; the top row is free-slip, everything else no-slip
    e = np.concatenate([np.sort(tri[:, [(k + 1) % 3, (k + 2) % 3]], 1) for k in range(3)])
    key = e[:, 0].astype(np.int64) * xy.shape[0] + e[:, 1]
    _, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
    single = (cnt[inv] == 1).reshape(3, -1).T
    top = (np.arange(xy.shape[0]) >= ny_channel * ncol) & (np.arange(xy.shape[0]) < base)
    kind = np.zeros(tri.shape, np.uint8)
    for k in range(3):
        a, b = tri[:, (k + 1) % 3], tri[:, (k + 2) % 3]
        kind[single[:, k], k] = np.where(top[a] & top[b], EDGE_SLIP, EDGE_WALL)[single[:, k]]
    return Mesh(xy=xy, tri=tri, edge_kind=kind, period_x=L,
                meta=dict(kind="cavity", nxh=nxh, ny_channel=ny_channel, ny_cavity=ny_cavity, H=H,
                          jitter=jitter, beta=beta, seed=seed))


def _wall_distance_cavity(x: np.ndarray, y: np.ndarray, H: float) -> np.ndarray:
    """Distance to the nearest no-slip wall of the street canyon (periodic in x)."""
    L = 3.0 * H
    xm = np.mod(x, L)

    def seg(ax, ay, bx, by):
        best = np.full(x.shape, np.inf)
        for sh in (-L, 0.0, L):
            px, py = xm + sh, y
            vx, vy = bx - ax, by - ay
            t = np.clip(((px - ax) * vx + (py - ay) * vy) / (vx * vx + vy * vy), 0.0, 1.0)
            best = np.minimum(best, np.hypot(px - ax - t * vx, py - ay - t * vy))
        return best
    d = seg(0.0, H, H, H)
    d = np.minimum(d, seg(2 * H, H, 3 * H, H))
    d = np.minimum(d, seg(H, 0.0, H, H))
    d = np.minimum(d, seg(2 * H, 0.0, 2 * H, H))
    return np.minimum(d, seg(H, 0.0, 2 * H, 0.0))


def cavity_fields(mesh: Mesh, *, recirc: float = 0.1, u_tau: float = 0.1, z0: float = 0.01,
                  wp_diag: float = -0.1, r_diag: float = 0.05 ** 2) -> Fields:
    """Analytic street-canyon fields at the nodes.

    In the cavity (y < H) the mean velocity is the recirculation of the stream
    function recirc * sin^2(pi x'/H) sin^2(pi y/H), x' = x - H: <U> = d/dy, <V> = -d/dx.
    Above it a log law <U> = (u_tau / 0.41) ln(1 + (y - H)/z0), <V> = 0, driven by
    grad<P> = (-1, 0) (zero in the cavity).  <omega> = min(1 + 10 d^(-1/2), 50) with d the
    distance to the nearest no-slip wall; elliptic-relaxation tensor wp_diag * I;
    Reynolds stresses r_diag * I.
    """
    H = mesh.meta.get("H", 1.0)
    x, y = mesh.xy[:, 0], mesh.xy[:, 1]
    n = mesh.n_nodes
    above = y >= H
    xp = x - H
    k = math.pi / H
    mu = np.zeros((n, 3))
    mu[:, 0] = np.where(above, (u_tau / 0.41) * np.log1p(np.maximum(y - H, 0.0) / z0),
                        recirc * np.sin(k * xp) ** 2 * k * np.sin(2 * k * y))
    mu[:, 1] = np.where(above, 0.0, -recirc * k * np.sin(2 * k * xp) * np.sin(k * y) ** 2)
    grad_p = np.zeros((n, 2))
    grad_p[above, 0] = -1.0
    wp = np.zeros((n, 6))
    wp[:, 0:3] = wp_diag
    d = _wall_distance_cavity(x, y, H)
    with np.errstate(divide="ignore"):
        om = np.where(d > 0, 1.0 + 10.0 / np.sqrt(np.maximum(d, 1e-300)), np.inf)
    om = np.minimum(om, 50.0)
    rey = np.zeros((n, 6))
    rey[:, 0:3] = r_diag
    return Fields(grad_p=grad_p, wp=wp, mean_u=mu, mean_omega=om, rey=rey)


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


def cavity_small(nxh=20, ny_channel=20, ny_cavity=20, ppe=50, seed=MASTER_SEED):
    """Street canyon for parity: 3 200 triangles, 50 particles per element, source at the
    cavity centre."""
    mesh = cavity_mesh(nxh, ny_channel, ny_cavity, seed=seed)
    return mesh, cavity_fields(mesh), model_constants(), init_desc(ppe=ppe, bins=(4, 2, 2), src_x=1.5,
                                                                     src_y=0.5)


def cavity_large(nxh=250, ny_channel=500, ny_cavity=500, ppe=100, seed=MASTER_SEED):
    """Street canyon at GPU scale: 1e6 triangles, 100 particles per element (1e8)."""
    mesh = cavity_mesh(nxh, ny_channel, ny_cavity, seed=seed)
    return mesh, cavity_fields(mesh), model_constants(), init_desc(ppe=ppe, bins=(4, 2, 2), src_x=1.5,
                                                                     src_y=0.5)


def cavity_huge(nxh=500, ny_channel=1000, ny_cavity=1000, ppe=120, seed=MASTER_SEED):
    """Large street canyon: 4e6 triangles, 120 particles per element (4.8e8), 32 bins."""
    mesh = cavity_mesh(nxh, ny_channel, ny_cavity, seed=seed)
    return mesh, cavity_fields(mesh), model_constants(), init_desc(ppe=ppe, bins=(4, 4, 2), src_x=1.5,
                                                                     src_y=0.5)


def redistribution_test(nx: int = 16, ny: int = 24, *, stretch: float = 50.0, ppe: int = 200,
                        mean0=(1.0, 0.0, 0.0), seed: int = MASTER_SEED):
    """The particle-redistribution test of Sec. 3.7 (Eqs. 46-48) in the form of Eq. (27):
    a periodic strip with free-slip walls whose cells are stretched towards both walls;
    nu = 0, grad<P> = 0 and frozen <omega> = 1, R = 2 I, wp = -1.5 I, so that
    G = (wp - eps/2 I)/k = -I and C0 eps = -2/3 wp:R/k = 2, i.e. dU = -(U - <U>)dt +
    sqrt(2) dW.  Feeding the nodal mean velocity back scaled by alpha gives Eq. (47).
    Particles start with unit-variance Gaussian velocities about mean0."""
    mesh = channel_mesh(nx, ny, length=2.0, y0=-1.0, y1=1.0, stretch=stretch, jitter=0.1, seed=seed,
                        bottom=EDGE_SLIP, top=EDGE_SLIP)
    fields = uniform_fields(mesh, grad_p=(0.0, 0.0), wp=(-1.5, -1.5, -1.5, 0.0, 0.0, 0.0),
                            mean_u=tuple(mean0), mean_omega=1.0, rey=(2.0, 2.0, 2.0, 0.0, 0.0, 0.0))
    init = init_desc(ppe=ppe, u_sigma=1.0, omega_shape=4.0, src_x=1.0, src_y=0.0, src_r=0.2,
                     bins=(4, 2, 2), seed=seed)
    return mesh, fields, model_constants(nu=0.0), init


def batched_problems(n: int = 64, *, tri_range=(1.0e3, 2.0e5), ppe_range=(20, 400), dt: float = 2e-4,
                     seed: int = MASTER_SEED):
    """Independent problems of uneven size for the batched form: triangle counts and
    particles per element log-uniform in the given ranges, channels for even and street
    canyons for odd problem seeds, each problem with its own seed.
    Returns a list of (mesh, fields, model, init, dt)."""
    rng = np.random.default_rng(seed ^ 0xBA7C4ED)
    out = []
    for p in range(n):
        tri = float(np.exp(rng.uniform(math.log(tri_range[0]), math.log(tri_range[1]))))
        ppe = int(round(np.exp(rng.uniform(math.log(ppe_range[0]), math.log(ppe_range[1])))))
        pseed = int(rng.integers(1, 2 ** 62))
        if pseed % 2 == 0:
            ny = max(4, 2 * int(round(math.sqrt(tri / 2.0 / 1.6) / 2.0)))
            nx = max(4, int(round(tri / 2.0 / ny)))
            mesh = channel_mesh(nx, ny, seed=pseed)
            fields = channel_fields(mesh)
            init = init_desc(ppe=ppe, bins=(4, 2, 2), seed=pseed)
        else:
            nxh = max(2, int(round(math.sqrt(tri / 16.0))))
            mesh = cavity_mesh(nxh, 2 * nxh, 2 * nxh, seed=pseed)
            fields = cavity_fields(mesh)
            init = init_desc(ppe=ppe, bins=(4, 2, 2), src_x=1.5, src_y=0.5, seed=pseed)
        out.append((mesh, fields, model_constants(), init, dt))
    return out


WORKLOADS = {
    "channel_small": dict(fn=channel_small, dt=1e-3, steps=20, control=None),
    "channel_large": dict(fn=channel_large, dt=2e-4, steps=100, control=(150, 250)),
    "cavity_small": dict(fn=cavity_small, dt=1e-4, steps=20, control=None),
    "cavity_large": dict(fn=cavity_large, dt=1e-4, steps=200, control=None),
    "cavity_huge": dict(fn=cavity_huge, dt=1e-4, steps=500, control=(90, 150)),
    "batched_64": dict(fn=batched_problems, dt=2e-4, steps=50, control=None),
}
