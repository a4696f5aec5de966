// P1 finite-element kernels of the Eulerian solves (Sec. 3.2): elliptic relaxation
// (Eqs. 12-17, 59) and the stabilised pressure projection (Eqs. 30-33) with the velocity
// correction of Eq. (31).
//
// The operators are applied matrix-free by node gather: row n sums, over the elements
// around n (the node->element lists of the grid), the element matrices
// mass * M_e + L^2_e K_e formed from the element's stored K_e = A_e grad N_a . grad N_b and
// A_e / 12 (M_e = A_e (1 + delta_ab) / 12), so every row is owned by one thread, the sums
// run in a fixed order, and no assembled matrix has to be rebuilt when L^2 changes.  Vectors hold NC components per node ([nn][NC]); the components are
// independent systems that share the element reads.
#pragma once
#include "pdf_impl.h"

namespace pdfgpu {

constexpr int FEM_RED_BLOCKS = 256;   // partial sums of the reductions

struct FemOp {
    const ElemGeo* geo;
    const double* ke;     // [ne][8] element matrices of fem_elem_matrices
    const int64_t* n2e_ptr;
    const int32_t* n2e;
    int64_t nn;
    double mass;          // coefficient of M_e
    double stiff;         // coefficient of L^2_e K_e
    const double* L2;     // [ne][4]: L^2 of wp_11, wp_22, wp_33, off-diagonal; null: 1
    const uint16_t* fixed; // [nn] bit c: component c of the node is a Dirichlet entry (its row
                           // gives 0); never null (an all-zero mask for none), so that the
                           // flags are read without a branch
    // assembled form of the nine-component operator (null: matrix-free): the grid's CSR
    // pattern and four coefficient arrays [4][nnz] (L^2 of wp_11, wp_22, wp_33, off-diagonal)
    const int32_t* crp = nullptr;
    const int32_t* ccol = nullptr;
    const double* cval = nullptr;
    int64_t nnz = 0;
};

// cval [4][nnz] = mass M + stiff L^2_g K on the pattern (crp, ccol) of op, summed over the
// elements around each row in the node->element order
void fem_assemble4(const FemOp& op, double* cval, hipStream_t s);

// per element, from its frame coordinates: A_e grad N_a . grad N_b for (a, b) = (0, 0),
// (1, 1), (2, 2), (0, 1), (0, 2), (1, 2) (Eqs. 39-40), then A_e / 12 (the mass matrix is
// A_e (1 + delta_ab) / 12) and one unused slot; the grid's geometry never changes, so this
// is done once
void fem_elem_matrices(const ElemGeo* geo, int64_t ne, double* ke, hipStream_t s);
template <int NC>
void fem_apply(const FemOp& op, const double* x, double* y, hipStream_t s);
template <int NC>
void fem_diag(const FemOp& op, double* d, hipStream_t s);
// out[c] = sum_n a[n][c] b[n][c] (b null: 1), and out[NC + c] = sum_n a2[n][c] b2[n][c]
// when a2 is given; partial holds FEM_RED_BLOCKS x 2NC values; fixed-order sums
template <int NC>
void fem_dot(const double* a, const double* b, const double* a2, const double* b2, int64_t nn, double* partial,
             double* out, hipStream_t s);
// Jacobi-preconditioned CG steps, one independent system per component, with device
// scalars sc = [rz NC][pAp NC][rz_new NC][rr NC][alpha NC][beta NC]; Dirichlet rows keep
// r = z = p = 0
template <int NC>
void fem_cg_init(const double* b, const double* Ax, const double* diag, const uint16_t* fixed, int64_t nn,
                 double* r, double* z, double* p, hipStream_t s);
template <int NC>
void fem_cg_alpha(double* sc, hipStream_t s);
template <int NC>
void fem_cg_xr(const double* sc, const double* p, const double* Ap, const double* diag, const uint16_t* fixed,
               int64_t nn, double* x, double* r, double* z, hipStream_t s);
template <int NC>
void fem_cg_beta(double* sc, hipStream_t s);
template <int NC>
void fem_cg_p(const double* sc, const double* z, int64_t nn, double* p, hipStream_t s);

// elliptic relaxation inputs: nodal right-hand side f [nn][9] of Eq. (12) (Eqs. 13-15,
// nodal velocity gradients as the average of the element gradients around the node),
// Dirichlet values [nn][9] and flags [nn] (Eq. 59 at no-slip nodes, zero off-diagonals at
// free-slip nodes), and L^2 per element [ne][4] (Eqs. 16-17)
struct EllipticConst {
    double C1, C2, CL, Ceta, Cv, gamma5, nu, CT;
};
void fem_elliptic_inputs(const ElemGeo* geo, const int64_t* n2e_ptr, const int32_t* n2e, const double* stats,
                         int64_t nn, int64_t ne, const EllipticConst& c, const uint8_t* wkind, const double* wnrm,
                         const double* enrm, double* f, double* xfix, uint16_t* fixed, double* L2, uint32_t* err,
                         hipStream_t s);
// b = mass-matrix product of f (M f) for the nine components
void fem_mass_rhs(const FemOp& op, const double* f, double* b, hipStream_t s);
// x = Dirichlet value where fixed, else keep x (nine components)
void fem_set_fixed(const double* xfix, const uint16_t* fixed, int64_t nn, double* x, hipStream_t s);

// Assembled stiffness matrix (CSR, one row per node, columns ascending) for the scalar
// pressure system, whose coefficients do not change: y = K p and the block partials of
// p . y in one pass
void fem_csr_apply_dot(const int32_t* row_ptr, const int32_t* col, const double* val, const double* x, int64_t nn,
                       double* y, double* partial, int nblocks, hipStream_t s);
int fem_csr_blocks(int64_t nn);
// CG of one component in two launches per iteration on CG2_BLOCKS workgroups, whose
// reductions are CG2_BLOCKS partials summed again by every workgroup of the next launch
// in one fixed order.  Iteration k: fem_cg2_apply forms beta from the r.z partials
// (part_rz, pairs r.z, r.r per workgroup) and r.z of iteration k - 1 (sc[(k + 1) & 1];
// beta = 0 at k = 0), stores r.z in sc[k & 1], p_k = z + beta p_(k-1) from pold into pnew,
// y = K p_k and the partials of p_k . y (part_py); fem_cg2_update forms alpha and updates
// x, r and z = r / diag with the new r.z and r.r partials.  fem_cg2_dots gives the first
// r.z, r.r partials.
constexpr int CG2_BLOCKS = 1024;
void fem_cg2_apply(const int32_t* row_ptr, const int32_t* col, const double* val, const double* z, const double* pold,
                   double* pnew, int64_t nn, double* y, const double* part_rz, double* part_py, double* sc, int k,
                   hipStream_t s);
void fem_cg2_update(const double* sc, const double* part_py, const double* p, const double* y, const double* diag,
                    int64_t nn, double* x, double* r, double* z, double* part_rz, int k, hipStream_t s);
void fem_cg2_dots(const double* r, const double* z, int64_t nn, double* part_rz, hipStream_t s);
// the update of fem_cg2_update without z and partials, for a preconditioner applied after it
void fem_cg2_update_xr(const double* sc, const double* part_py, const double* p, const double* y, int64_t nn,
                       double* x, double* r, int k, hipStream_t s);
// diag of the CSR matrix
void fem_csr_diag(const int32_t* row_ptr, const int32_t* col, const double* val, int64_t nn, double* d,
                  hipStream_t s);

// nodal wp records (nine components) from the solution [nn][9] (row-major ij)
void fem_store_wp(const double* wp9, int64_t nn, double* node, hipStream_t s);

// pressure projection pieces
// b_a = -(rho/dt) int N_a div <U>* - (cp/dt) (K P)_a over the elements around node a
void fem_pressure_rhs(const FemOp& op, const double* stats, const double* P, double rho, double dt, double cp,
                      double* b, uint32_t* err, hipStream_t s);
// v -= sum / nn (sum given on the device)
void fem_sub_mean(const double* sum, int64_t nn, double* v, hipStream_t s);
// y += a
void fem_add(const double* a, int64_t n, double* y, hipStream_t s);
// count of nodes whose statistics (first 12 values) are not all finite -> *count (added)
void fem_check_stats(const double* stats, int64_t nn, unsigned long long* count, hipStream_t s);
// per element: the gradient of the nodal field q [ne][2]
void fem_elem_grad(const ElemGeo* geo, const double* q, int64_t ne, double* g, hipStream_t s);
// P += dP; nodal mean-pressure gradient record = gp0 + average of the element gradients of P
// around the node; nodal mean velocity of the statistics -= (dt/rho) x average element
// gradient of dP where the node has statistics
void fem_pressure_update(const int64_t* n2e_ptr, const int32_t* n2e, const double* gP, const double* gdP,
                         const double* gp0, int64_t nn, double scale, double* node, double* stats, hipStream_t s);
// outward normal [ne][2] of the no-slip wall edge (edges [nw][4]: midpoint, outward unit
// normal) nearest to each element centroid; zero without wall edges
void fem_nearest_wall(const ElemGeo* geo, int64_t ne, const double* edges, int32_t nw, double period, double* enrm,
                      hipStream_t s);
// particles of element e: U1, U2 -= scale x gdP[e]
template <class R>
void fem_correct_particles(const SoaT<R>& st, const int64_t* nslots, int64_t n_ub, const double* gdP, double scale,
                           hipStream_t s);
}  // namespace pdfgpu
