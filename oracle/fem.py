"""FEM solves on either side of the particle step (Sec. 3.2), written out plainly.

Test infrastructure: only tests, the smoke check and the benchmark's CPU leg use it.

P1 finite elements on the triangles of the grid: element gradients of the shape functions
(Eqs. 39-40), stiffness K_e = A_e grad N_a . grad N_b and consistent mass
M_e = A_e (1 + delta_ab) / 12, assembled into scipy sparse matrices and solved directly.

* Elliptic relaxation, Eq. (12), with the right-hand side of Eqs. (13)-(15), the length
  scale of Eqs. (16)-(17), the wall condition Eq. (59) at no-slip wall nodes and the
  symmetry condition of Sec. 4.1.1 at free-slip nodes (off-diagonal components zero,
  diagonal components natural).  All nine components of wp_ij (row-major ij).
* Stabilised pressure projection, Eq. (33), for the increment dP = <P>^{n+1} - <P>^n
  (natural condition: the increment's wall-normal gradient is zero; the periodic seam is
  shared nodes), the solution with zero sum over the nodes, and the correction of Eq. (31)
  applied with the element gradient of dP.

Readings (each stated where it is used): L is evaluated per element from the averages of
the nodal k and epsilon of its vertices and enters as a constant L^2 per element; C_xi of
Eq. (17) is applied per diagonal component, 1 + 1.3 n_i^2 for wp_ii (no summation) and 1
for the off-diagonal components, with n the outward unit normal of the nearest no-slip wall
edge (midpoint distance, minimum image across the periodic seam, ties to the lowest
element*3+edge); the nodal wall normal of Eq. (59) is the normalised length-weighted sum of
the outward normals of the wall edges at the node; nodal velocity gradients are the plain
averages of the element gradients around the node (the first pass of Sec. 3.4).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# Table 4 constants of the elliptic relaxation model
ELLIPTIC_CONSTANTS = dict(C1=1.85, C2=0.63, CL=0.134, Ceta=72.0, Cv=1.4, gamma5=0.1)

EDGE_WALL, EDGE_SLIP = 1, 2

# statistics columns (nodal statistics of the ensemble)
S_W, S_U, S_OM, S_R = 0, 1, 4, 6


def p1_gradients(frame, area):
    """dN_a/dx and dN_a/dy of the three vertices of every element (Eqs. 39-40)."""
    x = frame[:, 0::2]
    y = frame[:, 1::2]
    bx = np.empty_like(x)
    by = np.empty_like(y)
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        bx[:, a] = (y[:, b] - y[:, c]) / (2.0 * area)
        by[:, a] = (x[:, c] - x[:, b]) / (2.0 * area)
    return bx, by


def element_matrices(frame, area):
    bx, by = p1_gradients(frame, area)
    K = area[:, None, None] * (bx[:, :, None] * bx[:, None, :] + by[:, :, None] * by[:, None, :])
    M = area[:, None, None] * (np.ones((3, 3)) + np.eye(3))[None] / 12.0
    return K, M


def assemble(tri, Ae, nn):
    rows = np.repeat(tri, 3, axis=1).ravel()
    cols = np.tile(tri, (1, 3)).ravel()
    return sp.csr_matrix((Ae.reshape(len(tri), 9).ravel(), (rows, cols)), shape=(nn, nn))


def node_average(tri, elem_vals, nn):
    """Plain average over the elements around each node."""
    ev = elem_vals.reshape(len(tri), -1)
    s = np.zeros((nn, ev.shape[1]))
    c = np.zeros(nn)
    for a in range(3):
        np.add.at(s, tri[:, a], ev)
        np.add.at(c, tri[:, a], 1.0)
    return s / c[:, None]


def wall_geometry(mesh, frame):
    """Nodal outward wall normals (no-slip), no-slip and free-slip node masks, and the
    wall edges (midpoint, outward unit normal) in element-index order."""
    nn = mesh.n_nodes
    tri = mesh.tri
    kind = mesh.edge_kind
    nrm = np.zeros((nn, 2))
    wall = np.zeros(nn, bool)
    slip = np.zeros(nn, bool)
    edges = []
    for e in range(len(tri)):
        for k in range(3):
            if kind[e, k] not in (EDGE_WALL, EDGE_SLIP):
                continue
            a, b = (k + 1) % 3, (k + 2) % 3
            xa, ya = frame[e, 2 * a], frame[e, 2 * a + 1]
            xb, yb = frame[e, 2 * b], frame[e, 2 * b + 1]
            dx, dy = xb - xa, yb - ya
            length = np.hypot(dx, dy)
            out = np.array([dy, -dx]) / length          # right of a->b: outside a CCW element
            if kind[e, k] == EDGE_WALL:
                for v in (tri[e, a], tri[e, b]):
                    nrm[v] += length * out
                    wall[v] = True
                edges.append((0.5 * (xa + xb), 0.5 * (ya + yb), out[0], out[1]))
            else:
                slip[tri[e, a]] = slip[tri[e, b]] = True
    ln = np.linalg.norm(nrm, axis=1)
    nrm[wall] /= ln[wall, None]
    return nrm, wall, slip & ~wall, np.array(edges).reshape(-1, 4)


def nearest_wall_normal(mesh, frame, edges):
    """Outward unit normal of the no-slip wall edge nearest to every element centroid
    (zero when the grid has no no-slip wall)."""
    ne = len(mesh.tri)
    out = np.zeros((ne, 2))
    if len(edges) == 0:
        return out
    cx = frame[:, 0::2].mean(1)
    cy = frame[:, 1::2].mean(1)
    L = mesh.period_x
    for e in range(ne):
        dx = edges[:, 0] - cx[e]
        if L > 0:
            dx = dx - L * np.round(dx / L)
        d2 = dx * dx + (edges[:, 1] - cy[e]) ** 2
        j = int(np.argmin(d2))                        # first minimum: lowest index
        out[e] = edges[j, 2:]
    return out


def _nodal_stats(stats, model):
    if np.isnan(stats[:, :12]).any():
        raise ValueError("statistics missing at some nodes")
    R = np.empty((len(stats), 3, 3))
    r = stats[:, S_R:S_R + 6]
    R[:, 0, 0], R[:, 1, 1], R[:, 2, 2] = r[:, 0], r[:, 1], r[:, 2]
    R[:, 0, 1] = R[:, 1, 0] = r[:, 3]
    R[:, 0, 2] = R[:, 2, 0] = r[:, 4]
    R[:, 1, 2] = R[:, 2, 1] = r[:, 5]
    k = 0.5 * np.trace(R, axis1=1, axis2=2)
    om = stats[:, S_OM]
    eps = om * (k + model["nu"] * model["CT"] ** 2 * om)                 # Eq. (18)
    return R, k, om, eps


def elliptic_rhs(mesh, frame, area, stats, model, consts=ELLIPTIC_CONSTANTS):
    """Nodal right-hand side of Eq. (12), [nn, 3, 3]."""
    R, k, om, eps = _nodal_stats(stats, model)
    tri = mesh.tri
    bx, by = p1_gradients(frame, area)
    U = stats[:, S_U:S_U + 3]
    ge = np.zeros((len(tri), 3, 3))                  # dU_k/dx_l per element, l = 3 is zero
    for c in range(3):
        ge[:, c, 0] = (bx * U[tri, c]).sum(1)
        ge[:, c, 1] = (by * U[tri, c]).sum(1)
    G = node_average(tri, ge.reshape(len(tri), 9), mesh.n_nodes).reshape(-1, 3, 3)
    C1, C2, Cv, g5 = consts["C1"], consts["C2"], consts["Cv"], consts["gamma5"]
    Av = np.minimum(1.0, Cv * np.linalg.det(R) / (2.0 * k / 3.0) ** 3)   # Eq. (14)
    b = R / (2.0 * k)[:, None, None] - np.eye(3)[None] / 3.0             # Eq. (15)
    f = np.zeros_like(R)
    for i in range(3):
        for j in range(3):
            # H_ijkl dU_k/dx_l with H of Eq. (13)
            h = (C2 * Av + g5 / 3.0) * G[:, i, j] - g5 / 3.0 * G[:, j, i]
            h = h + g5 * (b[:, i, :] * G[:, :, j]).sum(1) - g5 * (b[:, i, :] * G[:, j, :]).sum(1)
            f[:, i, j] = k * h + (0.5 * (1.0 - C1) * k * om if i == j else 0.0)
    return f


def length_scale_sq(mesh, frame, stats, model, consts=ELLIPTIC_CONSTANTS):
    """L^2 of Eqs. (16)-(17) per element and component [ne, 3, 3]."""
    _, k, _, eps = _nodal_stats(stats, model)
    tri = mesh.tri
    ke = k[tri].mean(1)
    ee = eps[tri].mean(1)
    _, _, _, edges = wall_geometry(mesh, frame)
    n = nearest_wall_normal(mesh, frame, edges)
    n3 = np.concatenate([n, np.zeros((len(n), 1))], axis=1)
    kol = consts["Ceta"] * (model["nu"] ** 3 / ee) ** 0.25
    L2 = np.empty((len(tri), 3, 3))
    for i in range(3):
        for j in range(3):
            cxi = 1.0 + 1.3 * n3[:, i] ** 2 if i == j else np.ones(len(tri))
            L = consts["CL"] * np.maximum(cxi * ke ** 1.5 / ee, kol)
            L2[:, i, j] = L * L
    return L2


def elliptic_relaxation(mesh, frame, area, stats, model, consts=ELLIPTIC_CONSTANTS):
    """wp_ij at the nodes [nn, 3, 3] from Eq. (12) with the conditions of Eq. (59) and
    Sec. 4.1.1; every component is a separate linear system."""
    nn, tri = mesh.n_nodes, mesh.tri
    K, M = element_matrices(frame, area)
    Mg = assemble(tri, M, nn)
    f = elliptic_rhs(mesh, frame, area, stats, model, consts)
    L2 = length_scale_sq(mesh, frame, stats, model, consts)
    nrm, wall, slip, _ = wall_geometry(mesh, frame)
    _, _, _, eps = _nodal_stats(stats, model)
    n3 = np.concatenate([nrm, np.zeros((nn, 1))], axis=1)
    out = np.zeros((nn, 3, 3))
    for i in range(3):
        for j in range(3):
            A = (Mg + assemble(tri, L2[:, i, j, None, None] * K, nn)).tocsr()
            rhs = Mg @ f[:, i, j]
            fixed = wall | (slip if i != j else np.zeros(nn, bool))
            val = np.zeros(nn)
            val[wall] = -4.5 * eps[wall] * n3[wall, i] * n3[wall, j]          # Eq. (59)
            free = ~fixed
            x = val.copy()
            if free.any():
                Aff = A[free][:, free]
                bf = rhs[free] - A[free][:, fixed] @ val[fixed]
                x[free] = spla.spsolve(Aff.tocsc(), bf)
            out[:, i, j] = x
    return out


def pressure_projection(mesh, frame, area, stats, p_prev, dt, cp=1e-3, rho=1.0):
    """Eq. (33) for dP with zero sum; returns (dP [nn], element gradient of dP [ne, 2])."""
    nn, tri = mesh.n_nodes, mesh.tri
    if np.isnan(stats[:, S_U:S_U + 3]).any():
        raise ValueError("statistics missing at some nodes")
    K, _ = element_matrices(frame, area)
    Kg = assemble(tri, K, nn)
    bx, by = p1_gradients(frame, area)
    U = stats[:, S_U:S_U + 3]
    div = (bx * U[tri, 0]).sum(1) + (by * U[tri, 1]).sum(1)          # div <U>* per element
    D = np.zeros(nn)
    for a in range(3):
        np.add.at(D, tri[:, a], area * div / 3.0)                      # int N_a div <U>*
    # weak form of (1/rho) lap dP = (div <U>* - C_p (1/rho) lap P^n) / dt, with
    # int N_a lap q = -(K q)_a for natural conditions
    b = -(rho / dt) * D - (cp / dt) * (Kg @ p_prev)
    b = b - b.mean()
    # K dP = b with sum(dP) = 0 (K is singular: constants)
    A = sp.bmat([[Kg, np.ones((nn, 1))], [np.ones((1, nn)), None]]).tocsc()
    sol = spla.spsolve(A, np.concatenate([b, [0.0]]))
    dP = sol[:nn]
    g = np.stack([(bx * dP[tri]).sum(1), (by * dP[tri]).sum(1)], axis=1)
    return dP, g


class Projection:
    """Pressure state of an oracle ensemble across repeated projections: P accumulates the
    increments (zero at the start) and the nodal mean-pressure gradient of the grid becomes
    the set-up field plus the nodal average of the element gradients of P."""

    def __init__(self, mesh, grid, grad_p0):
        ex = grid.export()
        self.mesh, self.grid = mesh, grid
        self.frame, self.area = ex["frame"], ex["area"]
        self.P = np.zeros(mesh.n_nodes)
        self.gp0 = np.array(grad_p0, dtype=np.float64).reshape(mesh.n_nodes, 2)

    def apply(self, ens, dt, cp=1e-3, rho=1.0):
        """Eq. (33) from the ensemble's statistics, then Eq. (31) on its particles and nodal
        mean velocity; returns dP."""
        tri, nn = self.mesh.tri, self.mesh.n_nodes
        dP, g = pressure_projection(self.mesh, self.frame, self.area, ens.stats(), self.P, dt, cp, rho)
        scale = dt / rho
        ens.shift_velocities(scale * g, scale * node_average(tri, g, nn))
        self.P = self.P + dP
        bx, by = p1_gradients(self.frame, self.area)
        gP = np.stack([(bx * self.P[tri]).sum(1), (by * self.P[tri]).sum(1)], axis=1)
        self.grid.set_grad_p(self.gp0 + node_average(tri, gP, nn))
        return dP
