// Device pieces of the preconditioned MINRES solve (ris_minres.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace ris {

// Scalar state of one right-hand side (device memory, one row per rhs).
struct MrState {
    double beta, oldb, beta1, beta2, alfa;
    double dbar, epsln, oldeps, phibar;
    double cs, sn, delta, phi, denom;
    double tol, active;
};
constexpr int kMrStride = (int)(sizeof(MrState) / sizeof(double));

// out[k * stride] = sum_i x_k[i] y_k[i] for k < nb (vectors of length n,
// consecutive), two fixed-order stages through partial (bdot_partials doubles).
size_t bdot_partials(long n, int nb);
hipError_t bdot(const double *x, const double *y, long n, int nb, double *partial, double *out, int stride,
                hipStream_t st);
// z_k[i] = r_k[i] / de[i]
hipError_t precond(const double *r, const double *de, double *z, long n, int nb, hipStream_t st);
// state from beta2 = <b, M^-1 b> (already stored in each row)
hipError_t mr_init(MrState *s, int nb, double tol, hipStream_t st);
hipError_t mr_v(const MrState *s, const double *y, double *v, long n, int nb, hipStream_t st);
// y -= (beta / oldb) r1 (second != 0), in place on the matvec result
hipError_t mr_y1(const MrState *s, const double *r1, double *y, long n, int nb, int second, hipStream_t st);
hipError_t mr_y2(const MrState *s, const double *r2, double *y, long n, int nb, hipStream_t st);
hipError_t mr_scal(MrState *s, int nb, hipStream_t st);
hipError_t mr_w(const MrState *s, const double *v, const double *w1, const double *w2, double *w, double *x, long n,
                int nb, hipStream_t st);
hipError_t vsub(const double *a, const double *b, double *d, size_t n, hipStream_t st);
// de[a][i] = max(|e_a - e_i|, kMinGap): the positive diagonal preconditioner
constexpr double kMinGap = 1e-4;
hipError_t orbital_gaps(const double *eps, int nvir, int nocc, double *de, hipStream_t st);

// Eigen-decomposition of a small symmetric m x m matrix A (device, row-major,
// destroyed): on return w[m] holds the eigenvalues ascending and row j of A the
// unit eigenvector of w[j].  work: m * m doubles; cs_buf: max(m, m + 1) doubles.
// One workgroup (cyclic Jacobi, tournament ordering).
hipError_t sym_eig_small(double *A, double *work, int m, double *w, double *cs_buf, hipStream_t st);

// TDA Davidson element steps: unit start vectors V[j][idx[j]] = 1 (V zeroed
// before); Ritz residuals R_j = AX_j - w[j] X_j; the diagonal correction
// t = r / (theta - (e_a - e_i)) with the denominator kept >= kDavFloor in
// magnitude; the plain orbital gaps e_a - e_i.
constexpr double kDavFloor = 1e-8;
hipError_t set_units(double *V, const int *idx, int k, long n, hipStream_t st);
hipError_t ritz_residual(const double *AX, const double *X, const double *w, double *R, long n, int nb,
                         hipStream_t st);
hipError_t davidson_correction(const double *r, double theta, const double *de, double *t, long n, hipStream_t st);
hipError_t orbital_gaps_plain(const double *eps, int nvir, int nocc, double *de, hipStream_t st);

// RS = [[0, R^T/2], [R/2, 0]] and LA = [[0, -L^T/2], [L/2, 0]] as dense
// nmo x nmo matrices (occupied first) from R, L [nvir][nocc].
hipError_t embed_rl(const double *R, const double *L, int nmo, int nocc, double *RS, double *LA, hipStream_t st);

}  // namespace ris
