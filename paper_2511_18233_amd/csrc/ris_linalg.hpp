// Elementwise and reduction helpers of the ris path (ris_linalg.hip).
#pragma once

#include "ris_common.hpp"

namespace ris {

hipError_t fill(double *p, size_t n, double v, hipStream_t st);
hipError_t gather_rows(const double *src, double *dst, const int *perm, int nrow, int ncol, int ld_src,
                       hipStream_t st);
hipError_t scatter_sq(const double *in, double *out, const int *perm, int n, int nb, hipStream_t st);
hipError_t make_rl(const double *X, const double *Y, double *R, double *L, size_t n, hipStream_t st);
hipError_t symmetrize(double *A, int n, int nb, hipStream_t st);
hipError_t add_de(const double *eps, const double *V, double *out, int nvir, int nocc, int nvec, double s,
                  hipStream_t st);
hipError_t axpby(const double *src, double *dst, size_t n, double alpha, double beta, hipStream_t st);
hipError_t assemble_w(const double *Hoo, const double *HRou, const double *HLou, const double *HRuo,
                      const double *HLuo, const double *HRuu, const double *HLuu, double *W, int o, int nP,
                      double scale, hipStream_t st);
hipError_t reduce_grad(const double *p3, int nshAO, int nshAux, int nout, int NO, const double *p2,
                       const int *atomAO, const int *atomAux, int natm, double *shA, double *shC, double *shP,
                       double scale, int accumulate, double *grad, hipStream_t st);

}  // namespace ris
