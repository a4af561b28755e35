/*
 * ris_test.h -- test-only entry points of libris_hip.so.  They expose building
 * blocks of the hot path (the matrix-core GEMM and its lane layout) so tests
 * can check them in isolation against plain references.  Not part of the
 * production call sequence; same conventions as ris.h (row-major FP64, device
 * pointers, status codes, enqueued on `hip_stream`).
 */
#ifndef RIS_TEST_H
#define RIS_TEST_H

#ifdef __cplusplus
extern "C" {
#endif

/* One matrix-core instruction on one wave, accumulator starting at 0.
 * kind 0: v_mfma_f64_16x16x4f64, lane l supplies a[l], b[l];
 * kind 1: v_mfma_f32_16x16x4f32, lane l supplies a[l], b[l] (rounded to FP32);
 * kind 2: v_mfma_f32_16x16x32_bf16, lane l supplies a[8l..8l+7], b[8l..8l+7]
 *         (rounded to BF16).
 * a, b are device arrays of doubles (64 or 512 values); lane l writes its four
 * result values to out[4 l + i] (device, 256 doubles).  Synchronous. */
int ris_test_mfma_probe(int kind, const double *a, const double *b, double *out);

/* C_z = alpha * op(A_z) op(B_z) + beta * C_z for z < batch (row-major, op(A) is
 * M x K, stored K x M when transA; op(B) is K x N, stored N x K when transB),
 * batch strides sA, sB, sC in elements.  Device pointers; synchronous. */
int ris_test_dgemm(int M, int N, int K, int transA, int transB, double alpha, const double *A, long lda, long sA,
                   const double *B, long ldb, long sB, double beta, double *C, long ldc, long sC, int batch);

/* Same product through the path's reduced-precision GEMM: mode 0 = FP64,
 * 1 = FP32 matrix cores, 2 = split BF16 with three products, 3 = split BF16
 * with six products; FP64 operands and result, FP32 accumulation for modes
 * 1-3.  Synchronous. */
int ris_test_gemm(int mode, int M, int N, int K, int transA, int transB, double alpha, const double *A, long lda,
                  long sA, const double *B, long ldb, long sB, double beta, double *C, long ldc, long sC, int batch);

/* The split-BF16 product on pre-split operands (the kernel of the exchange
 * weights' Y^P and Gamma^P products in the split modes): A (M x K) and B
 * (N x K), FP64 device matrices with leading dimensions lda, ldb, are split
 * into ns = 2 or 3 bf16 parts per element (of fl32(x)), then
 * C = alpha A B^T + beta C (FP64, leading dimension ldc), or with
 * out_planes != 0 (beta 0) the FP32 product is written as ns bf16 parts whose
 * sum in FP64 is returned in C.  kband = w > 0 (K = 3w, B zero in its
 * (1st row, 3rd k) and (3rd row, 1st k) w-blocks) skips those zero blocks;
 * lower != 0 (M == N) computes the 128 x 128 tiles on or below the diagonal
 * only, leaving C's other tiles untouched.  sym2 != 0 (M == N, beta 0, FP64
 * output, no band) computes C = alpha (A B^T + B A^T) in one launch, the
 * form of the exchange weights of a transition between two states.
 * Allocates its own planes; synchronous.  1: invalid arguments, 7: device
 * error. */
int ris_test_pgemm(int ns, int M, int N, int K, double alpha, const double *A, long lda, const double *B, long ldb,
                   double beta, double *C, long ldc, int kband, int lower, int out_planes, int sym2);

/* Eigen-decomposition of a small symmetric m x m matrix by the path's
 * one-workgroup Jacobi kernel (used for Davidson subspaces): A (device,
 * row-major, m x m) is replaced by the eigenvectors as rows, w (device, m)
 * receives the eigenvalues ascending.  Synchronous; allocates its own work. */
int ris_test_sym_eig(int m, double *A, double *w);

/* out[c][r] = in[r][c] for r < R, c < C by the path's LDS-tiled transpose
 * (it forms the H_UO blocks from the H_OU blocks): in (device, leading
 * dimension ldi >= C), out (device, leading dimension ldo >= R, not
 * overlapping in).  Returns 1 on invalid arguments, 7 on a HIP error.
 * Synchronous. */
int ris_test_transpose(const double *in, long ldi, double *out, long ldo, int R, int C);

/* The path's device Boys function F_m(T) = int_0^1 t^2m exp(-T t^2) dt (the
 * table + Taylor + downward recursion below T = 40, the asymptotic F_0 and
 * upward recursion above; it serves every integral kernel): F[i][m] =
 * F_m(T[i]) for m = 0..7.  T (device, n values >= 0), F (device, n x 8).
 * Returns 1 on invalid arguments, 7 on a HIP error.  Synchronous; allocates
 * its own table. */
int ris_test_boys(int n, const double *T, double *F);

#ifdef __cplusplus
}
#endif

#endif /* RIS_TEST_H */
