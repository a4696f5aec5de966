// Host-side grid construction for libpdfgpu: validation, adjacency, element frames,
// derived fields of the frozen mean velocity, wall lines.  Runs once per grid.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <tuple>

#include "pdf_impl.h"

namespace pdfgpu {

void set_error(const std::string& msg);

namespace {

struct EdgeRef {
    uint64_t key;  // (min node) << 32 | (max node)
    int32_t e;
    int32_t k;
};

// x coordinate of mesh node `node` in the frame of element e (node must be a vertex of e)
double frame_x(const pdf_grid_s& g, const int32_t* tri, int64_t e, int32_t node)
{
    for (int q = 0; q < 3; ++q)
        if (tri[3 * e + q] == node) return g.h_geo[e].x[q];
    return 0.0;
}

}  // namespace

// Element gradient of nodal values q at the vertices (Eqs. 39-40):
// dN/dx = [ -y_CA + y_BA, y_CA, -y_BA ] / (2 A_e), dN/dy = [ x_CA - x_BA, -x_CA, x_BA ] / (2 A_e)
static inline void p1_gradient(const ElemGeo& G, double qa, double qb, double qc, double& gx, double& gy)
{
    const double xba = G.x[1] - G.x[0], xca = G.x[2] - G.x[0];
    const double yba = G.y[1] - G.y[0], yca = G.y[2] - G.y[0];
    const double inv2a = 1.0 / (2.0 * G.area);
    gx = inv2a * ((yba - yca) * qa + yca * qb - yba * qc);
    gy = inv2a * ((xca - xba) * qa - xca * qb + xba * qc);
}

pdf_status build_grid(pdf_grid_s& g, const pdf_mesh_desc& m, const pdf_fields_desc& f)
{
    const int64_t nn = m.n_nodes, ne = m.n_elems;
    const double P = m.period_x;
    if (nn < 3 || ne < 1 || !m.xy || !m.tri || !m.edge_kind || !(P >= 0.0) || !std::isfinite(P) ||
        !f.grad_p || !f.wp || !f.mean_u || !f.mean_omega || !f.rey) {
        set_error("pdf_grid_create: invalid descriptor");
        return PDF_E_INVAL;
    }
    if (ne > (int64_t)INT32_MAX / 3 || nn > (int64_t)INT32_MAX) {
        set_error("pdf_grid_create: mesh too large for 32-bit indices");
        return PDF_E_INVAL;
    }
    const int32_t* tri = m.tri;
    for (int64_t i = 0; i < 3 * ne; ++i)
        if (tri[i] < 0 || tri[i] >= nn) { set_error("pdf_grid_create: node index out of range"); return PDF_E_MESH; }
    for (int64_t i = 0; i < 2 * nn; ++i)
        if (!std::isfinite(m.xy[i])) { set_error("pdf_grid_create: non-finite node coordinate"); return PDF_E_NONFINITE; }

    g.nn = nn;
    g.ne = ne;
    g.period = P;
    g.h_geo.assign(ne, ElemGeo{});

    // element frames; an element straddling the periodic seam has its vertices with
    // x < P/2 moved by +P
    for (int64_t e = 0; e < ne; ++e) {
        ElemGeo& G = g.h_geo[e];
        double lo = INFINITY, hi = -INFINITY;
        for (int k = 0; k < 3; ++k) {
            G.node[k] = tri[3 * e + k];
            G.x[k] = m.xy[2 * (int64_t)G.node[k]];
            G.y[k] = m.xy[2 * (int64_t)G.node[k] + 1];
            lo = std::min(lo, G.x[k]);
            hi = std::max(hi, G.x[k]);
        }
        if (P > 0.0 && hi - lo > 0.5 * P)
            for (int k = 0; k < 3; ++k)
                if (G.x[k] < 0.5 * P) G.x[k] += P;
        G.area = 0.5 * ((G.x[1] - G.x[0]) * (G.y[2] - G.y[0]) - (G.y[1] - G.y[0]) * (G.x[2] - G.x[0]));
        if (!(G.area > 0.0)) { set_error("pdf_grid_create: element not counter-clockwise or degenerate"); return PDF_E_MESH; }
        G.inv_area = 1.0 / G.area;
    }

    // neighbours: sort all directed edges by their node pair
    std::vector<EdgeRef> edges(3 * ne);
    for (int64_t e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) {
            uint32_t a = (uint32_t)tri[3 * e + (k + 1) % 3], b = (uint32_t)tri[3 * e + (k + 2) % 3];
            if (a == b) { set_error("pdf_grid_create: repeated node in element"); return PDF_E_MESH; }
            uint64_t key = ((uint64_t)std::min(a, b) << 32) | std::max(a, b);
            edges[3 * e + k] = EdgeRef{key, (int32_t)e, k};
        }
    std::sort(edges.begin(), edges.end(), [](const EdgeRef& p, const EdgeRef& q) {
        return std::tie(p.key, p.e, p.k) < std::tie(q.key, q.e, q.k);
    });
    for (int64_t e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) { g.h_geo[e].nbr[k] = -1; g.h_geo[e].kind[k] = 255; g.h_geo[e].shift[k] = 0.0; }
    for (size_t i = 0; i < edges.size();) {
        size_t j = i;
        while (j < edges.size() && edges[j].key == edges[i].key) ++j;
        if (j - i > 2) { set_error("pdf_grid_create: edge shared by more than two elements"); return PDF_E_MESH; }
        if (j - i == 2) {
            const EdgeRef &p = edges[i], &q = edges[i + 1];
            g.h_geo[p.e].nbr[p.k] = q.e;
            g.h_geo[q.e].nbr[q.k] = p.e;
            int32_t a = (int32_t)(edges[i].key >> 32);
            double xp = frame_x(g, tri, p.e, a), xq = frame_x(g, tri, q.e, a);
            if (P > 0.0 && std::fabs(xq - xp) > 0.5 * P) {
                g.h_geo[p.e].kind[p.k] = KIND_PERIODIC;
                g.h_geo[p.e].shift[p.k] = xq > xp ? P : -P;
                g.h_geo[q.e].kind[q.k] = KIND_PERIODIC;
                g.h_geo[q.e].shift[q.k] = xp > xq ? P : -P;
            } else {
                g.h_geo[p.e].kind[p.k] = KIND_INTERIOR;
                g.h_geo[q.e].kind[q.k] = KIND_INTERIOR;
            }
        } else {
            const EdgeRef& p = edges[i];
            uint8_t uk = m.edge_kind[3 * (int64_t)p.e + p.k];
            if (uk != KIND_WALL && uk != KIND_SLIP) {
                set_error("pdf_grid_create: boundary edge must be a no-slip or free-slip wall");
                return PDF_E_MESH;
            }
            g.h_geo[p.e].kind[p.k] = uk;
        }
        i = j;
    }

    // elements around each node (ascending element id), stored as element*3 + slot
    g.h_n2e_ptr.assign(nn + 1, 0);
    for (int64_t i = 0; i < 3 * ne; ++i) g.h_n2e_ptr[tri[i] + 1]++;
    for (int64_t n = 0; n < nn; ++n) g.h_n2e_ptr[n + 1] += g.h_n2e_ptr[n];
    g.h_n2e.assign(3 * ne, 0);
    {
        std::vector<int64_t> fill(g.h_n2e_ptr.begin(), g.h_n2e_ptr.end() - 1);
        for (int64_t e = 0; e < ne; ++e)
            for (int k = 0; k < 3; ++k) g.h_n2e[fill[tri[3 * e + k]]++] = (int32_t)(3 * e + k);
    }

    // nodal field records
    g.h_node.assign(nn * NODE_STRIDE, 0.0);
    for (int64_t n = 0; n < nn; ++n) {
        double* r = &g.h_node[n * NODE_STRIDE];
        r[NF_GP] = f.grad_p[2 * n];
        r[NF_GP + 1] = f.grad_p[2 * n + 1];
        for (int q = 0; q < 6; ++q) r[NF_WP + q] = f.wp[6 * n + q];
        for (int q = 0; q < 3; ++q) r[NF_WPT + q] = f.wp[6 * n + 3 + q];   // symmetric input
        for (int q = 0; q < 3; ++q) r[NF_MU + q] = f.mean_u[3 * n + q];
        r[NF_OM] = f.mean_omega[n];
        for (int q = 0; q < 6; ++q) r[NF_RE + q] = f.rey[6 * n + q];
        for (int q = 0; q < NODE_STRIDE; ++q)
            if (!std::isfinite(r[q])) { set_error("pdf_grid_create: non-finite nodal field"); return PDF_E_NONFINITE; }
        if (!(r[NF_OM] > 0.0)) { set_error("pdf_grid_create: mean frequency must be positive"); return PDF_E_NONFINITE; }
        if (!(r[NF_RE] + r[NF_RE + 1] + r[NF_RE + 2] > 0.0)) { set_error("pdf_grid_create: kinetic energy must be positive"); return PDF_E_NONFINITE; }
    }

    // element gradients of <U_i> (Eqs. 39-40)
    for (int64_t e = 0; e < ne; ++e) {
        ElemGeo& G = g.h_geo[e];
        for (int i = 0; i < 3; ++i)
            p1_gradient(G, g.h_node[(int64_t)G.node[0] * NODE_STRIDE + NF_MU + i],
                        g.h_node[(int64_t)G.node[1] * NODE_STRIDE + NF_MU + i],
                        g.h_node[(int64_t)G.node[2] * NODE_STRIDE + NF_MU + i], G.gu[2 * i], G.gu[2 * i + 1]);
    }

    // second derivatives by the two-pass procedure of Sec. 3.4: average the element
    // gradients to the nodes, take the element gradients of those nodal gradients and
    // average again; the Laplacian is d2/dx2 + d2/dy2
    {
        std::vector<double> gn(6 * nn, 0.0), h(6 * ne, 0.0);
        for (int64_t n = 0; n < nn; ++n) {
            const int64_t c = g.h_n2e_ptr[n + 1] - g.h_n2e_ptr[n];
            for (int64_t j = g.h_n2e_ptr[n]; j < g.h_n2e_ptr[n + 1]; ++j)
                for (int q = 0; q < 6; ++q) gn[6 * n + q] += g.h_geo[g.h_n2e[j] / 3].gu[q];
            if (c > 0)
                for (int q = 0; q < 6; ++q) gn[6 * n + q] /= (double)c;
        }
        for (int64_t e = 0; e < ne; ++e) {
            const ElemGeo& G = g.h_geo[e];
            for (int i = 0; i < 3; ++i) {
                double dxx, dxy, dyx, dyy;
                p1_gradient(G, gn[6 * (int64_t)G.node[0] + 2 * i], gn[6 * (int64_t)G.node[1] + 2 * i],
                            gn[6 * (int64_t)G.node[2] + 2 * i], dxx, dxy);
                p1_gradient(G, gn[6 * (int64_t)G.node[0] + 2 * i + 1], gn[6 * (int64_t)G.node[1] + 2 * i + 1],
                            gn[6 * (int64_t)G.node[2] + 2 * i + 1], dyx, dyy);
                h[6 * e + 2 * i] = dxx;
                h[6 * e + 2 * i + 1] = dyy;
            }
        }
        for (int64_t n = 0; n < nn; ++n) {
            const int64_t c = g.h_n2e_ptr[n + 1] - g.h_n2e_ptr[n];
            for (int i = 0; i < 3; ++i) {
                double sxx = 0.0, syy = 0.0;
                for (int64_t j = g.h_n2e_ptr[n]; j < g.h_n2e_ptr[n + 1]; ++j) {
                    sxx += h[6 * (int64_t)(g.h_n2e[j] / 3) + 2 * i];
                    syy += h[6 * (int64_t)(g.h_n2e[j] / 3) + 2 * i + 1];
                }
                g.h_node[n * NODE_STRIDE + NF_LAP + i] = c > 0 ? sxx / (double)c + syy / (double)c : 0.0;
            }
        }
    }

    // wall elements (an edge or a node on a no-slip wall, Sec. 3.8) and their wall line:
    // among the no-slip edges that touch one of the element's nodes, the one whose
    // midpoint is nearest to the centroid (ties: lowest owner*3 + edge)
    {
        std::vector<uint8_t> wnode(nn, 0);
        for (int64_t e = 0; e < ne; ++e)
            for (int k = 0; k < 3; ++k)
                if (g.h_geo[e].kind[k] == KIND_WALL) {
                    wnode[g.h_geo[e].node[(k + 1) % 3]] = 1;
                    wnode[g.h_geo[e].node[(k + 2) % 3]] = 1;
                }
        for (int64_t e = 0; e < ne; ++e) {
            ElemGeo& G = g.h_geo[e];
            G.wall = 0;
            G.wl[0] = G.wl[1] = G.wl[2] = G.wl[3] = 0.0;
            if (!(wnode[G.node[0]] || wnode[G.node[1]] || wnode[G.node[2]])) continue;
            G.wall = 1;
            const double cx = (G.x[0] + G.x[1] + G.x[2]) / 3.0, cy = (G.y[0] + G.y[1] + G.y[2]) / 3.0;
            double best = INFINITY;
            int64_t bestkey = -1;
            for (int v = 0; v < 3; ++v) {
                const int32_t node = G.node[v];
                if (!wnode[node]) continue;
                for (int64_t j = g.h_n2e_ptr[node]; j < g.h_n2e_ptr[node + 1]; ++j) {
                    const int64_t fe = g.h_n2e[j] / 3;
                    const int slot = g.h_n2e[j] % 3;
                    const ElemGeo& F = g.h_geo[fe];
                    const double off = G.x[v] - F.x[slot];   // F's frame -> G's frame
                    for (int k = 0; k < 3; ++k) {
                        if (F.kind[k] != KIND_WALL) continue;
                        const int pa = (k + 1) % 3, pb = (k + 2) % 3;
                        const double ax = F.x[pa] + off, ay = F.y[pa], bx = F.x[pb] + off, by = F.y[pb];
                        const double mx = 0.5 * (ax + bx) - cx, my = 0.5 * (ay + by) - cy;
                        const double d2 = mx * mx + my * my;
                        const int64_t key = 3 * fe + k;
                        if (d2 < best || (d2 == best && key < bestkey)) {
                            const double ex = bx - ax, ey = by - ay, len = std::sqrt(ex * ex + ey * ey);
                            best = d2;
                            bestkey = key;
                            G.wl[0] = ax;
                            G.wl[1] = ay;
                            G.wl[2] = -ey / len;
                            G.wl[3] = ex / len;
                        }
                    }
                }
            }
        }
    }
    return PDF_OK;
}

}  // namespace pdfgpu
