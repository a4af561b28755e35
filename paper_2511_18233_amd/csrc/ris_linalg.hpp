// Elementwise and reduction helpers of the ris path (ris_linalg.hip).
#pragma once

#include "ris_common.hpp"

namespace ris {

hipError_t fill(double *p, size_t n, double v, hipStream_t st);
hipError_t gather_rows(const double *src, double *dst, const int *perm, int nrow, int ncol, int ld_src,
                       hipStream_t st);
hipError_t scatter_sq(const double *in, double *out, const int *perm, int n, int nb, hipStream_t st);
// out[i][j] = in[perm[i]][perm[j]] for one n x n matrix
hipError_t gather_sq(const double *in, double *out, const int *perm, int n, hipStream_t st);
hipError_t make_rl(const double *X, const double *Y, double *R, double *L, size_t n, hipStream_t st);
hipError_t symmetrize(double *A, int n, int nb, hipStream_t st);
// C_b[i][j] = C_b[j][i] for j > i, b < batch (n x n blocks, leading dimension ldc, batch stride sC):
// completes a symmetric result of which only the lower triangle was formed
hipError_t mirror_lower(double *C, int n, long ldc, long sC, int batch, hipStream_t st);
// out[c][r] = in[r][c] for r < R, c < C (leading dimensions ldi, ldo; not in place)
hipError_t transpose(const double *in, long ldi, double *out, long ldo, int R, int C, hipStream_t st);
// G_b = s (X_b + X_b^T) on the lower triangle of batch n x n blocks (G may alias X)
hipError_t sym_sum_lower(const double *X, double *G, int n, int batch, double s, hipStream_t st);
// V[P][Q] += s (G[P][Q] + G[Q][P]) for P, Q < n; G dense n x n, V with leading dimension ldv
hipError_t add_sym(const double *G, int n, double *V, int ldv, double s, hipStream_t st);
hipError_t add_de(const double *eps, const double *V, double *out, int nvir, int nocc, int nvec, double s,
                  hipStream_t st);
hipError_t axpby(const double *src, double *dst, size_t n, double alpha, double beta, hipStream_t st);
// one o x o source block of a 3 x 3 assembly: base[P*sP + i*si + j*sj] * scale
struct BlockSrc {
    const double *base;
    long sP, si, sj;
    double scale;
};
struct BlockGrid {
    BlockSrc b[3][3][2];  // up to two summed sources per block; base == nullptr means none
};
// W and Wf (either may be null) receive W and a float copy of it.
hipError_t assemble3(const BlockGrid &g, double *W, int o, int nP, hipStream_t st, float *Wf = nullptr);
// Planes (ns bf16 parts of the FP32 values, see plane_ld) of the transposes of
// the same assembly: part p of W_P^T at Wt + p ps + P 3o plane_ld(3o), its row c
// holding column c of W_P (ris_gemm_mp.hip).
hipError_t assemble3_planes(const BlockGrid &g, uint16_t *Wt, int o, int nP, long ps, int ns, hipStream_t st);
// y = (float)x elementwise
hipError_t to_float(const double *x, float *y, size_t n, hipStream_t st);
// out[i0*o0 + i1*o1 + i2*o2] = alpha * in[i0*s0 + i1*s1 + i2*s2] + beta * out over n0 x n1 x n2
hipError_t permute3(const double *in, double *out, int n0, int n1, int n2, long s0, long s1, long s2, long o0,
                    long o1, long o2, hipStream_t st, double alpha = 1.0, double beta = 0.0);
hipError_t reduce_grad(const double *p3, int nshAO, int nshAux, int nout, int NO, const double *p2,
                       const int *atomAO, const int *atomAux, int natm, double *shA, double *shC, double *shP,
                       double scale, int accumulate, double *grad, hipStream_t st);

}  // namespace ris
