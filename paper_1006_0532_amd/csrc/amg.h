// Smoothed-aggregation algebraic multigrid for the assembled pressure matrix of Eq. (33)
// (the P1 stiffness matrix of the grid, symmetric positive semi-definite with the
// constants as its null space), used as the preconditioner of its conjugate-gradient
// solve.  The hierarchy is built once on the host from the matrix; the V-cycle runs on
// the device.
//
// Setup, per level (standard smoothed aggregation):
//  - strong couplings |a_ij| >= theta sqrt(a_ii a_jj);
//  - greedy aggregates in node order: a node whose strong neighbours are all free roots
//    an aggregate of itself and them; a node left over joins the aggregate of its
//    strongest aggregated neighbour; what remains roots aggregates again;
//  - tentative prolongator T (the constants of each aggregate) smoothed by one damped
//    Jacobi step, P = (I - omega D^-1 A) T with omega = 4 / (3 lambda), lambda the
//    Gershgorin bound of D^-1 A, so P carries the constants to the constants;
//  - Galerkin coarse matrix P^T A P;
// until at most AMG_COARSE unknowns remain, whose matrix (plus a multiple of the all-ones
// matrix, which makes it definite without changing solutions orthogonal to the constants)
// is inverted densely.
//
// V-cycle (symmetric, so it preconditions CG): one damped Jacobi sweep from zero, the
// residual restricted by P^T, the coarse correction prolonged by P, one damped Jacobi sweep.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace pdfgpu {

constexpr int AMG_COARSE = 400;     // unknowns solved densely
constexpr int AMG_MAX_LEVELS = 16;

struct HostCsr {
    int64_t n = 0, m = 0;           // rows, columns
    std::vector<int32_t> rp, col;   // row pointers [n + 1], columns ascending per row
    std::vector<double> val;
};

struct AmgHostLevel {
    HostCsr A, P, R;                // A on this level; P to it from the next, R = P^T
    std::vector<double> dinv;       // smoother: omega_s / a_ii
};

struct AmgHost {
    std::vector<AmgHostLevel> lv;   // lv[0] holds the fine matrix
    int64_t nc = 0;                 // unknowns of the coarsest level
    std::vector<double> cinv;       // [nc][nc] inverse of its (definite) matrix
};

// Builds the hierarchy of A (square, symmetric, no Dirichlet rows).  Returns false when
// aggregation stalls before the coarse size (the caller keeps Jacobi preconditioning).
bool amg_build(const HostCsr& A, AmgHost& out);

struct DevCsr {
    int64_t n = 0, nnz = 0;
    int32_t* rp = nullptr;
    int32_t* col = nullptr;
    double* val = nullptr;
};

struct AmgDevLevel {
    DevCsr A, P, R;
    double* dinv = nullptr;
    double *b = nullptr, *x = nullptr, *r = nullptr, *t = nullptr;   // [n] work vectors
};

struct AmgDev {
    std::vector<AmgDevLevel> lv;
    int64_t nc = 0;
    double* cinv = nullptr;
    double *cb = nullptr, *cx = nullptr;    // coarsest right-hand side and solution
};

// device copies of the hierarchy; on failure everything allocated is freed
hipError_t amg_upload(const AmgHost& h, AmgDev& d, hipStream_t s);
void amg_free(AmgDev& d);
// z = M^-1 r on level 0 (r, z: [n0] device vectors, z may not alias r)
void amg_vcycle(AmgDev& d, const double* r, double* z, hipStream_t s);

}  // namespace pdfgpu
