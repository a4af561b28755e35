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

/* One v_mfma_f64_16x16x4f64 on one wave: lane l supplies a[l] and b[l]
 * (device arrays of 64 doubles, accumulator starts at 0) and writes its four
 * result doubles to out[4 l + i] (device, 256 doubles).  Synchronous. */
int ris_test_mfma_probe(const double *a, const double *b, double *out);

/* C_z = alpha * op(A_z) op(B_z) + beta * C_z for z < batch (row-major, op(A) is
 * M x K, stored K x M when transA; op(B) is K x N, stored N x K when transB),
 * batch strides sA, sB, sC in elements.  Device pointers; synchronous. */
int ris_test_dgemm(int M, int N, int K, int transA, int transB, double alpha, const double *A, long lda, long sA,
                   const double *B, long ldb, long sB, double beta, double *C, long ldc, long sC, int batch);

#ifdef __cplusplus
}
#endif

#endif /* RIS_TEST_H */
