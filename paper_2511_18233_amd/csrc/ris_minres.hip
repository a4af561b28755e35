// Device pieces of the preconditioned MINRES solve of (A+B)^ris Z = rhs:
// batched deterministic dot products, the elementwise vector updates and the
// per-right-hand-side scalar recurrence (Paige and Saunders' MINRES with a
// symmetric positive definite preconditioner).  Every right-hand side k owns a
// row of MrState in device memory; the vector kernels read their
// coefficients from it, so an iteration needs no host round trip.
#include <cmath>

#include "ris_minres.hpp"

namespace ris {
namespace {

inline unsigned nb_of(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

constexpr int kDotThreads = 256;
constexpr int kDotPerThread = 8;
constexpr int kDotChunk = kDotThreads * kDotPerThread;

// partial[k][blk] = sum over the chunk blk of x_k * y_k (fixed order)
__global__ __launch_bounds__(kDotThreads) void k_bdot_partial(const double *__restrict__ x,
                                                              const double *__restrict__ y, long n, int nblk,
                                                              double *__restrict__ partial)
{
    __shared__ double red[kDotThreads];
    const int k = blockIdx.y, blk = blockIdx.x, t = threadIdx.x;
    const double *xk = x + (long)k * n, *yk = y + (long)k * n;
    const long base = (long)blk * kDotChunk;
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kDotPerThread; ++u) {
        const long i = base + (long)u * kDotThreads + t;
        if (i < n) s += xk[i] * yk[i];
    }
    red[t] = s;
    __syncthreads();
    for (int h = kDotThreads / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) partial[(long)k * nblk + blk] = red[0];
}

__global__ void k_bdot_final(const double *__restrict__ partial, int nblk, int nb, double *__restrict__ out,
                             int stride)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nb) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[(long)k * nblk + b];
    out[(long)k * stride] = s;
}

// z_k[i] = r_k[i] / de[i]
__global__ void k_precond(const double *__restrict__ r, const double *__restrict__ de, double *__restrict__ z,
                          long n, int nb)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * nb) return;
    z[idx] = r[idx] / de[idx % n];
}

__global__ void k_mr_init(MrState *st, int nb, double tol)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nb) return;
    MrState &s = st[k];
    const double b1 = sqrt(fmax(s.beta2, 0.0));
    s.beta1 = b1;
    s.beta = b1;
    s.oldb = 0.0;
    s.dbar = 0.0;
    s.epsln = 0.0;
    s.oldeps = 0.0;
    s.phibar = b1;
    s.cs = -1.0;
    s.sn = 0.0;
    s.delta = 0.0;
    s.phi = 0.0;
    s.denom = 0.0;
    s.tol = tol;
    s.active = b1 > 0.0 ? 1.0 : 0.0;
}

// v = y / beta (0 once a right-hand side has stopped)
__global__ void k_mr_v(const MrState *st, const double *__restrict__ y, double *__restrict__ v, long n, int nb)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * nb) return;
    const MrState &s = st[idx / n];
    v[idx] = s.active != 0.0 ? y[idx] / s.beta : 0.0;
}

// y -= (beta / oldb) r1 in place on the matvec result (from the second iteration on)
__global__ void k_mr_y1(const MrState *st, const double *__restrict__ r1, double *__restrict__ y, long n, int nb,
                        int second)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * nb) return;
    const MrState &s = st[idx / n];
    const double c = (second && s.active != 0.0) ? s.beta / s.oldb : 0.0;
    y[idx] -= c * r1[idx];
}

// y -= (alfa / beta) r2
__global__ void k_mr_y2(const MrState *st, const double *__restrict__ r2, double *__restrict__ y, long n, int nb)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * nb) return;
    const MrState &s = st[idx / n];
    const double c = s.active != 0.0 ? s.alfa / s.beta : 0.0;
    y[idx] -= c * r2[idx];
}

// one Lanczos step of the scalar recurrence (Givens rotation of the
// tridiagonal system); stops the right-hand side once the preconditioned
// residual estimate phibar is within tol * beta1
__global__ void k_mr_scal(MrState *st, int nb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nb) return;
    MrState &s = st[k];
    if (s.active == 0.0) {
        s.phi = 0.0;
        s.denom = 0.0;
        s.oldeps = 0.0;
        s.delta = 0.0;
        return;
    }
    s.oldb = s.beta;
    s.beta = sqrt(fmax(s.beta2, 0.0));
    s.oldeps = s.epsln;
    s.delta = s.cs * s.dbar + s.sn * s.alfa;
    const double gbar = s.sn * s.dbar - s.cs * s.alfa;
    s.epsln = s.sn * s.beta;
    s.dbar = -s.cs * s.beta;
    double gamma = hypot(gbar, s.beta);
    if (gamma < 1e-300) gamma = 1e-300;
    s.cs = gbar / gamma;
    s.sn = s.beta / gamma;
    s.phi = s.cs * s.phibar;
    s.phibar = s.sn * s.phibar;
    s.denom = 1.0 / gamma;
    if (s.phibar <= s.tol * s.beta1 || s.beta == 0.0) s.active = 0.0;
}

// w = (v - oldeps w1 - delta w2) denom ; x += phi w
__global__ void k_mr_w(const MrState *st, const double *__restrict__ v, const double *__restrict__ w1,
                       const double *__restrict__ w2, double *__restrict__ w, double *__restrict__ x, long n, int nb)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * nb) return;
    const MrState &s = st[idx / n];
    const double wn = (v[idx] - s.oldeps * w1[idx] - s.delta * w2[idx]) * s.denom;
    w[idx] = wn;
    x[idx] += s.phi * wn;
}

// preconditioner diagonal max(|e_a - e_i|, kMinGap), [a][i] order
__global__ void k_gaps(const double *__restrict__ eps, int nvir, int nocc, double *__restrict__ de)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)nvir * nocc) return;
    const int a = (int)(idx / nocc), i = (int)(idx % nocc);
    de[idx] = fmax(fabs(eps[nocc + a] - eps[i]), kMinGap);
}

// d = a - b
__global__ void k_sub(const double *__restrict__ a, const double *__restrict__ b, double *__restrict__ d, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = a[i] - b[i];
}

}  // namespace

size_t bdot_partials(long n, int nb) { return (size_t)nb * ((n + kDotChunk - 1) / kDotChunk); }

hipError_t bdot(const double *x, const double *y, long n, int nb, double *partial, double *out, int stride,
                hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    const int nblk = (int)((n + kDotChunk - 1) / kDotChunk);
    if (nblk > 0)
        hipLaunchKernelGGL(k_bdot_partial, dim3(nblk, nb), dim3(kDotThreads), 0, st, x, y, n, nblk, partial);
    hipLaunchKernelGGL(k_bdot_final, dim3(nb_of(nb, 64)), dim3(64), 0, st, partial, nblk, nb, out, stride);
    return hipGetLastError();
}

hipError_t precond(const double *r, const double *de, double *z, long n, int nb, hipStream_t st)
{
    if (n * nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_precond, dim3(nb_of((size_t)n * nb, 256)), dim3(256), 0, st, r, de, z, n, nb);
    return hipGetLastError();
}

hipError_t mr_init(MrState *s, int nb, double tol, hipStream_t st)
{
    hipLaunchKernelGGL(k_mr_init, dim3(nb_of(nb, 64)), dim3(64), 0, st, s, nb, tol);
    return hipGetLastError();
}

hipError_t mr_v(const MrState *s, const double *y, double *v, long n, int nb, hipStream_t st)
{
    hipLaunchKernelGGL(k_mr_v, dim3(nb_of((size_t)n * nb, 256)), dim3(256), 0, st, s, y, v, n, nb);
    return hipGetLastError();
}

hipError_t mr_y1(const MrState *s, const double *r1, double *y, long n, int nb, int second, hipStream_t st)
{
    hipLaunchKernelGGL(k_mr_y1, dim3(nb_of((size_t)n * nb, 256)), dim3(256), 0, st, s, r1, y, n, nb, second);
    return hipGetLastError();
}

hipError_t mr_y2(const MrState *s, const double *r2, double *y, long n, int nb, hipStream_t st)
{
    hipLaunchKernelGGL(k_mr_y2, dim3(nb_of((size_t)n * nb, 256)), dim3(256), 0, st, s, r2, y, n, nb);
    return hipGetLastError();
}

hipError_t mr_scal(MrState *s, int nb, hipStream_t st)
{
    hipLaunchKernelGGL(k_mr_scal, dim3(nb_of(nb, 64)), dim3(64), 0, st, s, nb);
    return hipGetLastError();
}

hipError_t mr_w(const MrState *s, const double *v, const double *w1, const double *w2, double *w, double *x, long n,
                int nb, hipStream_t st)
{
    hipLaunchKernelGGL(k_mr_w, dim3(nb_of((size_t)n * nb, 256)), dim3(256), 0, st, s, v, w1, w2, w, x, n, nb);
    return hipGetLastError();
}

hipError_t orbital_gaps(const double *eps, int nvir, int nocc, double *de, hipStream_t st)
{
    if ((long)nvir * nocc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gaps, dim3(nb_of((size_t)nvir * nocc, 256)), dim3(256), 0, st, eps, nvir, nocc, de);
    return hipGetLastError();
}

hipError_t vsub(const double *a, const double *b, double *d, size_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sub, dim3(nb_of(n, 256)), dim3(256), 0, st, a, b, d, n);
    return hipGetLastError();
}

}  // namespace ris

// ---------------------------------------------------------------------------
// Small dense symmetric eigensolver for Davidson subspaces: cyclic Jacobi with
// the round-robin (tournament) ordering, all disjoint rotations of a round in
// parallel, one workgroup, matrices in global memory (m is at most a few
// hundred; the cost is negligible next to one matvec).
namespace ris {
namespace {

constexpr int kJacThreads = 256;

// player j of round r in the circle method over mp (even) players
__device__ __forceinline__ int jac_player(int j, int r, int mp) { return j == 0 ? 0 : ((j - 1 + r) % (mp - 1)) + 1; }

__global__ __launch_bounds__(kJacThreads) void k_jacobi(double *__restrict__ A, double *__restrict__ V, int m,
                                                        double *__restrict__ w, double *__restrict__ cs_buf,
                                                        int max_sweeps)
{
    const int t = threadIdx.x;
    const int mp = m + (m & 1);  // a dummy player pads odd sizes
    const int npair = mp / 2;
    __shared__ double red[kJacThreads];
    __shared__ int stop;
    for (long idx = t; idx < (long)m * m; idx += kJacThreads) V[idx] = (idx / m == idx % m) ? 1.0 : 0.0;
    __syncthreads();
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        // convergence: off-diagonal Frobenius norm against the whole matrix
        double off = 0.0, all = 0.0;
        for (long idx = t; idx < (long)m * m; idx += kJacThreads) {
            const double a = A[idx];
            all += a * a;
            if (idx / m != idx % m) off += a * a;
        }
        red[t] = off;
        __syncthreads();
        for (int h = kJacThreads / 2; h > 0; h >>= 1) {
            if (t < h) red[t] += red[t + h];
            __syncthreads();
        }
        const double offs = red[0];
        __syncthreads();
        red[t] = all;
        __syncthreads();
        for (int h = kJacThreads / 2; h > 0; h >>= 1) {
            if (t < h) red[t] += red[t + h];
            __syncthreads();
        }
        if (t == 0) stop = (offs <= 1e-30 * red[0]) ? 1 : 0;
        __syncthreads();
        if (stop) break;
        for (int r = 0; r < mp - 1; ++r) {
            // rotation of each pair: symmetric 2 x 2 Schur decomposition
            for (int k = t; k < npair; k += kJacThreads) {
                int p = jac_player(k, r, mp), q = jac_player(mp - 1 - k, r, mp);
                if (p > q) { const int x = p; p = q; q = x; }
                double c = 1.0, s = 0.0;
                if (q < m) {
                    const double apq = A[(long)p * m + q];
                    if (apq != 0.0) {
                        const double tau = (A[(long)q * m + q] - A[(long)p * m + p]) / (2.0 * apq);
                        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        s = tt * c;
                    }
                }
                cs_buf[2 * k] = c;
                cs_buf[2 * k + 1] = s;
            }
            __syncthreads();
            // rows p, q of A  (A <- J^T A)
            for (long idx = t; idx < (long)npair * m; idx += kJacThreads) {
                const int k = (int)(idx / m), col = (int)(idx % m);
                int p = jac_player(k, r, mp), q = jac_player(mp - 1 - k, r, mp);
                if (p > q) { const int x = p; p = q; q = x; }
                if (q >= m) continue;
                const double c = cs_buf[2 * k], s = cs_buf[2 * k + 1];
                const double ap = A[(long)p * m + col], aq = A[(long)q * m + col];
                A[(long)p * m + col] = c * ap - s * aq;
                A[(long)q * m + col] = s * ap + c * aq;
            }
            __syncthreads();
            // columns p, q of A and of V  (A <- A J, V <- V J)
            for (long idx = t; idx < (long)npair * m; idx += kJacThreads) {
                const int k = (int)(idx / m), row = (int)(idx % m);
                int p = jac_player(k, r, mp), q = jac_player(mp - 1 - k, r, mp);
                if (p > q) { const int x = p; p = q; q = x; }
                if (q >= m) continue;
                const double c = cs_buf[2 * k], s = cs_buf[2 * k + 1];
                const double ap = A[(long)row * m + p], aq = A[(long)row * m + q];
                A[(long)row * m + p] = c * ap - s * aq;
                A[(long)row * m + q] = s * ap + c * aq;
                const double vp = V[(long)row * m + p], vq = V[(long)row * m + q];
                V[(long)row * m + p] = c * vp - s * vq;
                V[(long)row * m + q] = s * vp + c * vq;
            }
            __syncthreads();
        }
    }
    // eigenvalues ascending; w[j] and the permutation into cs_buf (as doubles)
    if (t == 0) {
        for (int j = 0; j < m; ++j) {
            w[j] = A[(long)j * m + j];
            cs_buf[j] = (double)j;
        }
        for (int i = 1; i < m; ++i) {  // insertion sort (stable)
            const double x = w[i], xi = cs_buf[i];
            int j = i - 1;
            while (j >= 0 && w[j] > x) {
                w[j + 1] = w[j];
                cs_buf[j + 1] = cs_buf[j];
                --j;
            }
            w[j + 1] = x;
            cs_buf[j + 1] = xi;
        }
    }
    __syncthreads();
    // sorted eigenvectors as rows of A: A[j][:] = V[:, perm[j]]
    for (long idx = t; idx < (long)m * m; idx += kJacThreads) {
        const int j = (int)(idx / m), row = (int)(idx % m);
        A[idx] = V[(long)row * m + (int)cs_buf[j]];
    }
}

}  // namespace

hipError_t sym_eig_small(double *A, double *work, int m, double *w, double *cs_buf, hipStream_t st)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(kJacThreads), 0, st, A, work, m, w, cs_buf, 60);
    return hipGetLastError();
}

}  // namespace ris

// ---------------------------------------------------------------------------
// Element kernels of the TDA Davidson iteration.
namespace ris {
namespace {

__global__ void k_set_units(double *__restrict__ V, const int *__restrict__ idx, int k, long n)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < k) V[(long)j * n + idx[j]] = 1.0;
}

// R_j = AX_j - w[j] X_j
__global__ void k_ritz_res(const double *__restrict__ AX, const double *__restrict__ X, const double *__restrict__ w,
                           double *__restrict__ R, long n, int nb)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * nb) return;
    R[idx] = AX[idx] - w[idx / n] * X[idx];
}

// t = r / (theta - d), the denominator kept at least kDavFloor away from 0
__global__ void k_dav_corr(const double *__restrict__ r, double theta, const double *__restrict__ de,
                           double *__restrict__ t, long n)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = theta - de[i];
    if (fabs(d) < kDavFloor) d = d < 0.0 ? -kDavFloor : kDavFloor;
    t[i] = r[i] / d;
}

// de[a][i] = e_a - e_i (unfloored: the Davidson shift uses the plain gaps)
__global__ void k_gaps_plain(const double *__restrict__ eps, int nvir, int nocc, double *__restrict__ de)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)nvir * nocc) return;
    de[idx] = eps[nocc + (int)(idx / nocc)] - eps[(int)(idx % nocc)];
}

}  // namespace

hipError_t set_units(double *V, const int *idx, int k, long n, hipStream_t st)
{
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_units, dim3(nb_of(k, 64)), dim3(64), 0, st, V, idx, k, n);
    return hipGetLastError();
}

hipError_t ritz_residual(const double *AX, const double *X, const double *w, double *R, long n, int nb,
                         hipStream_t st)
{
    if (n * nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ritz_res, dim3(nb_of((size_t)n * nb, 256)), dim3(256), 0, st, AX, X, w, R, n, nb);
    return hipGetLastError();
}

hipError_t davidson_correction(const double *r, double theta, const double *de, double *t, long n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dav_corr, dim3(nb_of((size_t)n, 256)), dim3(256), 0, st, r, theta, de, t, n);
    return hipGetLastError();
}

hipError_t orbital_gaps_plain(const double *eps, int nvir, int nocc, double *de, hipStream_t st)
{
    if ((long)nvir * nocc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gaps_plain, dim3(nb_of((size_t)nvir * nocc, 256)), dim3(256), 0, st, eps, nvir, nocc, de);
    return hipGetLastError();
}

}  // namespace ris

extern "C" int ris_test_sym_eig(int m, double *A, double *w)
{
    if (m < 0 || (m > 0 && (!A || !w))) return 1;
    if (m == 0) return 0;
    double *work = nullptr, *cs = nullptr;
    if (hipMalloc(&work, sizeof(double) * m * m) != hipSuccess) return 3;
    if (hipMalloc(&cs, sizeof(double) * (m + 2)) != hipSuccess) {
        (void)hipFree(work);
        return 3;
    }
    const hipError_t e = ris::sym_eig_small(A, work, m, w, cs, 0);
    const hipError_t s = hipDeviceSynchronize();
    (void)hipFree(work);
    (void)hipFree(cs);
    return (e != hipSuccess || s != hipSuccess) ? 7 : 0;
}

// ---------------------------------------------------------------------------
// Dense MO-basis transition densities (occupied first):
//   RS = [[0, R^T/2], [R/2, 0]],  LA = [[0, -L^T/2], [L/2, 0]]
namespace ris {
namespace {
__global__ void k_embed_rl(const double *__restrict__ R, const double *__restrict__ L, int nmo, int nocc,
                           double *__restrict__ RS, double *__restrict__ LA)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)nmo * nmo) return;
    const int p = (int)(idx / nmo), q = (int)(idx % nmo);
    double rs = 0.0, la = 0.0;
    if (p < nocc && q >= nocc) {
        const long e = (long)(q - nocc) * nocc + p;
        rs = 0.5 * R[e];
        la = -0.5 * L[e];
    } else if (p >= nocc && q < nocc) {
        const long e = (long)(p - nocc) * nocc + q;
        rs = 0.5 * R[e];
        la = 0.5 * L[e];
    }
    RS[idx] = rs;
    LA[idx] = la;
}
}  // namespace

hipError_t embed_rl(const double *R, const double *L, int nmo, int nocc, double *RS, double *LA, hipStream_t st)
{
    hipLaunchKernelGGL(k_embed_rl, dim3(nb_of((size_t)nmo * nmo, 256)), dim3(256), 0, st, R, L, nmo, nocc, RS, LA);
    return hipGetLastError();
}
}  // namespace ris
