// Small dense linear algebra and elementwise kernels for the ris path (FP64).
//
// The auxiliary metric M = (P|Q) is factored as M = L L^T (blocked
// right-looking Cholesky: 64-wide diagonal blocks factored in LDS, panel
// triangular solve, trailing update on the matrix-core GEMM), then
// M^-1 = L^-T L^-1 is formed from the triangular inverse (Sec. 2.2 uses M^-1
// in the RI kernel and -M^-1 M^x M^-1 in its derivative).
#include "ris_common.hpp"
#include "ris_linalg.hpp"

namespace ris {
namespace {

constexpr int NB = 64;

// Factor the NB x NB (or smaller) diagonal block at (k0, k0) in LDS.
// A pivot below 1e-13 of the original diagonal entry (Morig) counts as a
// failure: the metric is then numerically singular.
__global__ __launch_bounds__(256) void k_potrf_diag(double *A, const double *Morig, int n, int k0, int b, int *info)
{
    __shared__ double T[NB][NB + 1];
    __shared__ int bad;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < b * b; idx += blockDim.x) {
        const int i = idx / b, j = idx % b;
        T[i][j] = A[(size_t)(k0 + i) * n + k0 + j];
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int k = 0; k < b; ++k) {
        if (tid == 0) {
            const double d = T[k][k];
            const double ref = Morig ? Morig[(size_t)(k0 + k) * n + k0 + k] : 0.0;
            if (!(d > 1e-13 * ref) || !(d > 0.0)) {
                bad = k0 + k + 1;
            } else {
                T[k][k] = sqrt(d);
            }
        }
        __syncthreads();
        if (bad) break;
        const double dk = T[k][k];
        for (int i = k + 1 + tid; i < b; i += blockDim.x) T[i][k] /= dk;
        __syncthreads();
        const int m = b - k - 1;
        for (int idx = tid; idx < m * m; idx += blockDim.x) {
            const int i = k + 1 + idx / m, j = k + 1 + idx % m;
            if (j <= i) T[i][j] -= T[i][k] * T[j][k];
        }
        __syncthreads();
    }
    if (bad) {
        if (tid == 0 && *info == 0) *info = bad;
        return;
    }
    for (int idx = tid; idx < b * b; idx += blockDim.x) {
        const int i = idx / b, j = idx % b;
        A[(size_t)(k0 + i) * n + k0 + j] = (j <= i) ? T[i][j] : 0.0;
    }
}

// Panel: rows r >= k0+b of columns k0..k0+b-1 become A_r L_kk^{-T}
// (forward substitution per row with the factored diagonal block in LDS).
__global__ __launch_bounds__(64) void k_trsm_panel(double *A, int n, int k0, int b, const int *info)
{
    __shared__ double Lk[NB][NB + 1];
    if (*info) return;
    for (int idx = threadIdx.x; idx < b * b; idx += blockDim.x) {
        const int i = idx / b, j = idx % b;
        Lk[i][j] = A[(size_t)(k0 + i) * n + k0 + j];
    }
    __syncthreads();
    const int r = k0 + b + blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double *row = A + (size_t)r * n + k0;
    for (int j = 0; j < b; ++j) {
        double s = row[j];
        for (int l = 0; l < j; ++l) s -= row[l] * Lk[j][l];
        row[j] = s / Lk[j][j];
    }
}

__global__ void k_set_int(int *p, int v) { *p = v; }

__global__ void k_zero_upper(double *A, int n)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * n) return;
    const int i = (int)(idx / n), j = (int)(idx % n);
    if (j > i) A[idx] = 0.0;
}

// inverse of each kTriBlock x kTriBlock diagonal block of L by forward
// substitution: workgroup k owns block k, thread j its column j (X zeroed before)
__global__ void k_tri_inv_diag(const double *__restrict__ L, double *__restrict__ X, int n)
{
    const int r0 = blockIdx.x * kTriBlock, j = threadIdx.x;
    const int nb = min(kTriBlock, n - r0);
    if (j >= nb) return;
    const int cj = r0 + j;
    X[(size_t)cj * n + cj] = 1.0 / L[(size_t)cj * n + cj];
    for (int i = j + 1; i < nb; ++i) {
        const int ri = r0 + i;
        double s = 0.0;
        for (int k = j; k < i; ++k) s += L[(size_t)ri * n + r0 + k] * X[(size_t)(r0 + k) * n + cj];
        X[(size_t)ri * n + cj] = -s / L[(size_t)ri * n + ri];
    }
}

__global__ void k_fill(double *p, size_t n, double v)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// dst[i][:] = src[perm[i]][:]   (rows of length ncol)
__global__ void k_gather_rows(const double *__restrict__ src, double *__restrict__ dst, const int *__restrict__ perm,
                              int nrow, int ncol, int ld_src)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)nrow * ncol) return;
    const int i = (int)(idx / ncol), c = (int)(idx % ncol);
    dst[idx] = src[(size_t)perm[i] * ld_src + c];
}

// out[b][perm[i]][perm[j]] = in[b][i][j]
__global__ void k_scatter_sq(const double *__restrict__ in, double *__restrict__ out, const int *__restrict__ perm,
                             int n, int nb)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long nn = (long)n * n;
    if (idx >= nn * nb) return;
    const long b = idx / nn, r = idx % nn;
    const int i = (int)(r / n), j = (int)(r % n);
    out[b * nn + (long)perm[i] * n + perm[j]] = in[idx];
}

// out[i][j] = in[perm[i]][perm[j]]  (one n x n matrix into the permuted order)
__global__ void k_gather_sq(const double *__restrict__ in, double *__restrict__ out, const int *__restrict__ perm,
                            int n)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * n) return;
    const int i = (int)(idx / n), j = (int)(idx % n);
    out[idx] = in[(long)perm[i] * n + perm[j]];
}

// R = X + s Y, L = X - s Y  (s = 0 when Y is absent)
__global__ void k_rl(const double *__restrict__ X, const double *__restrict__ Y, double *__restrict__ R,
                     double *__restrict__ L, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = X[i], y = Y ? Y[i] : 0.0;
    R[i] = x + y;
    L[i] = x - y;
}

// in-place symmetrisation of nb square matrices: A = (A + A^T)/2
__global__ void k_symmetrize(double *A, int n, int nb)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long nn = (long)n * n;
    if (idx >= nn * nb) return;
    const long b = idx / nn, r = idx % nn;
    const int i = (int)(r / n), j = (int)(r % n);
    if (j <= i) return;
    double *M = A + b * nn;
    const double v = 0.5 * (M[(size_t)i * n + j] + M[(size_t)j * n + i]);
    M[(size_t)i * n + j] = v;
    M[(size_t)j * n + i] = v;
}

// C_b[i][j] = C_b[j][i] for j > i: the strict upper triangle copied from the
// lower one, 32 x 32 tiles through LDS (block (tj, ti, b) writes upper tile
// (ti, tj) from lower tile (tj, ti); 32 x 8 threads)
__global__ void k_mirror_lower(double *__restrict__ C, int n, long ldc, long sC)
{
    __shared__ double t[32][33];
    const int tj = blockIdx.x, ti = blockIdx.y;
    if (tj < ti) return;
    double *M = C + (long)blockIdx.z * sC;
    const int tx = threadIdx.x, ty = threadIdx.y;
#pragma unroll
    for (int k = 0; k < 32; k += 8) {
        const int r = tj * 32 + ty + k, col = ti * 32 + tx;
        if (r < n && col < n) t[ty + k][tx] = M[(long)r * ldc + col];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 32; k += 8) {
        const int r = ti * 32 + ty + k, col = tj * 32 + tx;
        if (r < n && col < n && col > r) M[(long)r * ldc + col] = t[tx][ty + k];
    }
}

// out[c][r] = in[r][c] for r < R, c < C through a 32 x 32 LDS tile (both
// sides coalesced); row tiles strided over the y grid
__global__ void k_transpose(const double *__restrict__ in, long ldi, double *__restrict__ out, long ldo, int R, int C)
{
    __shared__ double t[32][33];
    const int tx = threadIdx.x, ty = threadIdx.y, c0 = blockIdx.x * 32;
    const int nrt = (R + 31) / 32;
    for (int rt = blockIdx.y; rt < nrt; rt += gridDim.y) {
        const int r0 = rt * 32;
#pragma unroll
        for (int k = 0; k < 32; k += 8) {
            const int r = r0 + ty + k, col = c0 + tx;
            if (r < R && col < C) t[ty + k][tx] = in[(long)r * ldi + col];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 32; k += 8) {
            const int col = c0 + ty + k, r = r0 + tx;
            if (r < R && col < C) out[(long)col * ldo + r] = t[tx][ty + k];
        }
        __syncthreads();
    }
}

// G_b[r][c] = s (X_b[r][c] + X_b[c][r]) on the lower triangle (c <= r) of n x n
// blocks b (batch stride sB): 32 x 32 tiles on or below the diagonal, the
// mirrored tile staged through LDS so that both reads are coalesced.  Only
// lower tiles are written and only the block's own and its mirrored tile are
// read, so G may alias X.
__global__ void k_sym_sum_lower(const double *__restrict__ X, double *__restrict__ G, int n, long sB, double s)
{
    __shared__ double t[32][33];
    const int tj = blockIdx.x, ti = blockIdx.y;
    if (tj > ti) return;
    const double *Xb = X + (long)blockIdx.z * sB;
    double *Gb = G + (long)blockIdx.z * sB;
    const int tx = threadIdx.x, ty = threadIdx.y;
#pragma unroll
    for (int k = 0; k < 32; k += 8) {
        const int r = tj * 32 + ty + k, col = ti * 32 + tx;
        if (r < n && col < n) t[ty + k][tx] = Xb[(long)r * n + col];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 32; k += 8) {
        const int r = ti * 32 + ty + k, col = tj * 32 + tx;
        if (r < n && col < n && col <= r) Gb[(long)r * n + col] = s * (Xb[(long)r * n + col] + t[tx][ty + k]);
    }
}

// V[P][Q] += s (G[P][Q] + G[Q][P]) over n x n (G dense n x n, V leading dim ldv)
__global__ void k_add_sym(const double *__restrict__ G, int n, double *__restrict__ V, int ldv, double s)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * n) return;
    const int p = (int)(idx / n), q = (int)(idx % n);
    V[(size_t)p * ldv + q] += s * (G[(size_t)p * n + q] + G[(size_t)q * n + p]);
}

// out[k][a][i] += s_de * (eps[nocc+a] - eps[i]) * V[k][a][i]
__global__ void k_add_de(const double *__restrict__ eps, const double *__restrict__ V, double *__restrict__ out,
                         int nvir, int nocc, int nvec, double s_de)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long per = (long)nvir * nocc;
    if (idx >= per * nvec) return;
    const long r = idx % per;
    const int a = (int)(r / nocc), i = (int)(r % nocc);
    out[idx] += s_de * (eps[nocc + a] - eps[i]) * V[idx];
}

// dst = alpha * src (+ dst if accumulate)
__global__ void k_axpby(const double *__restrict__ src, double *__restrict__ dst, size_t n, double alpha, double beta)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    dst[i] = alpha * src[i] + (beta == 0.0 ? 0.0 : beta * dst[i]);
}

// Assemble nP matrices of (3o x 3o) from a 3 x 3 grid of o x o blocks; block
// (bi, bj) is the sum of up to two strided sources
//   src[P][i][j] = base[P * sP + i * si + j * sj] * scale   (base null = 0).
// grid: (3 column blocks x chunks of 256 columns, 3o rows, nP); the column
// block, hence the source descriptors, is uniform per workgroup
__global__ __launch_bounds__(256) void k_assemble3(BlockGrid g, double *__restrict__ W, float *__restrict__ Wf, int o)
{
    // one workgroup per (row, P): the row's three column blocks in turn, so a
    // block's sources are the same for every thread; a missing source is read
    // from a present one with factor 0 (or the block is zero), so the loads
    // need no branch
    const int n3 = 3 * o;
    const int row = blockIdx.x, P = blockIdx.y;
    const int bi = row / o, i = row - bi * o;
    const long rbase = ((long)P * n3 + row) * n3;
    for (int bj = 0; bj < 3; ++bj) {
        const BlockSrc s0 = g.b[bi][bj][0], s1 = g.b[bi][bj][1];
        const long at0 = rbase + (long)bj * o;
        if (!s0.base && !s1.base) {
            for (int j = threadIdx.x; j < o; j += blockDim.x) {
                if (W) W[at0 + j] = 0.0;
                if (Wf) Wf[at0 + j] = 0.0f;
            }
            continue;
        }
        const BlockSrc a = s0.base ? s0 : s1;
        const BlockSrc b = s1.base ? s1 : a;
        const double ca = s0.base ? s0.scale : 0.0;
        const double cb = s1.base ? s1.scale : 0.0;
        const double *pa = a.base + P * a.sP + (long)i * a.si;
        const double *pb = b.base + P * b.sP + (long)i * b.si;
        for (int j = threadIdx.x; j < o; j += blockDim.x) {
            const double v = ca * pa[(long)j * a.sj] + cb * pb[(long)j * b.sj];
            if (W) W[at0 + j] = v;
            if (Wf) Wf[at0 + j] = (float)v;
        }
    }
}

__global__ void k_to_float(const double *__restrict__ x, float *__restrict__ y, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (float)x[i];
}

// out[i0*o0 + i1*o1 + i2*o2] = alpha * in[i0*s0 + i1*s1 + i2*s2] (+ beta * out) over n0 x n1 x n2;
// the element index is split with divisions of type I (32-bit when the
// element count fits)
template <typename I>
__global__ void k_permute3(const double *__restrict__ in, double *__restrict__ out, int n0, int n1, int n2,
                           long s0, long s1, long s2, long o0, long o1, long o2, double alpha, double beta)
{
    const I idx = (I)blockIdx.x * (I)blockDim.x + (I)threadIdx.x;
    if ((long)idx >= (long)n0 * n1 * n2) return;
    const I i2 = idx % (I)n2, r = idx / (I)n2;
    const I i1 = r % (I)n1, i0 = r / (I)n1;
    double *d = out + (long)i0 * o0 + (long)i1 * o1 + (long)i2 * o2;
    const double v = alpha * in[(long)i0 * s0 + (long)i1 * s1 + (long)i2 * s2];
    *d = (beta == 0.0) ? v : v + beta * *d;
}

// Reduce the triplet partials into per-shell sums (fixed order).
// p3: [nshAO][nshAux][3][NO][6]; shA[sa][o][3] = sum_{sc, lb} dA; shC[sc][o][3] = sum_{sa, lb} dC
__global__ void k_reduce_p3_a(const double *__restrict__ p3, int nshAO, int nshAux, int nout, int NO,
                              double *__restrict__ shA)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nshAO * nout * 3) return;
    const int sa = idx / (nout * 3), o = (idx / 3) % nout, d = idx % 3;
    double s = 0.0;
    for (int sc = 0; sc < nshAux; ++sc)
        for (int lb = 0; lb < 3; ++lb) s += p3[((((size_t)sa * nshAux + sc) * 3 + lb) * NO + o) * 6 + d];
    shA[idx] = s;
}
__global__ void k_reduce_p3_c(const double *__restrict__ p3, int nshAO, int nshAux, int nout, int NO,
                              double *__restrict__ shC)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nshAux * nout * 3) return;
    const int sc = idx / (nout * 3), o = (idx / 3) % nout, d = idx % 3;
    double s = 0.0;
    for (int sa = 0; sa < nshAO; ++sa)
        for (int lb = 0; lb < 3; ++lb) s += p3[((((size_t)sa * nshAux + sc) * 3 + lb) * NO + o) * 6 + 3 + d];
    shC[idx] = s;
}
// p2: [nshAux][2][nout][3] -> shP[sp][o][3]
__global__ void k_reduce_p2(const double *__restrict__ p2, int nshAux, int nout, double *__restrict__ shP)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nshAux * nout * 3) return;
    const int sp = idx / (nout * 3), o = (idx / 3) % nout, d = idx % 3;
    shP[idx] = p2[(((size_t)sp * 2 + 0) * nout + o) * 3 + d] + p2[(((size_t)sp * 2 + 1) * nout + o) * 3 + d];
}
// grad[o0 + o][X][d] (+)= sum over shells on atom X of the per-shell sums
__global__ void k_atoms(const double *__restrict__ shA, const int *__restrict__ atomA, int nshA,
                        const double *__restrict__ shC, const int *__restrict__ atomC, int nshC,
                        const double *__restrict__ shP, int natm, int nout, double scale, int accumulate,
                        double *__restrict__ grad)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= natm * nout * 3) return;
    const int o = idx / (natm * 3), X = (idx / 3) % natm, d = idx % 3;
    double s = 0.0;
    for (int sa = 0; sa < nshA; ++sa)
        if (atomA[sa] == X) s += shA[((size_t)sa * nout + o) * 3 + d];
    for (int sc = 0; sc < nshC; ++sc)
        if (atomC[sc] == X) s += shC[((size_t)sc * nout + o) * 3 + d] + (shP ? shP[((size_t)sc * nout + o) * 3 + d] : 0.0);
    grad[idx] = (accumulate ? grad[idx] : 0.0) + scale * s;
}

inline unsigned nblk(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t cholesky(double *A, const double *Morig, int n, int *info, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, st, info, 0);
    hipError_t e = hipSuccess;
    for (int k0 = 0; k0 < n; k0 += NB) {
        const int b = (n - k0 < NB) ? n - k0 : NB;
        hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, st, A, Morig, n, k0, b, info);
        const int rest = n - k0 - b;
        if (rest > 0) {
            hipLaunchKernelGGL(k_trsm_panel, dim3(nblk(rest, 64)), dim3(64), 0, st, A, n, k0, b, info);
            GemmArgs g{};
            g.M = rest; g.N = rest; g.K = b;
            g.transA = false; g.transB = true;
            g.alpha = -1.0; g.beta = 1.0;
            g.A = A + (size_t)(k0 + b) * n + k0; g.lda = n;
            g.B = A + (size_t)(k0 + b) * n + k0; g.ldb = n;
            g.C = A + (size_t)(k0 + b) * n + k0 + b; g.ldc = n;
            g.batch = 1; g.nred = 1;
            e = dgemm(g, st);
            if (e != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL(k_zero_upper, dim3(nblk((size_t)n * n, 256)), dim3(256), 0, st, A, n);
    return hipGetLastError();
}

hipError_t tri_inverse(const double *L, double *Linv, int n, double *tmp, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipError_t e = fill(Linv, (size_t)n * n, 0.0, st);
    if (e != hipSuccess) return e;
    const int nb = (n + kTriBlock - 1) / kTriBlock;
    hipLaunchKernelGGL(k_tri_inv_diag, dim3(nb), dim3(kTriBlock), 0, st, L, Linv, n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // block rows below: X[i, :i] = -X_ii (L[i, :i] X[:i, :i])
    for (int i = 1; i < nb; ++i) {
        const int r0 = i * kTriBlock, rows = std::min(kTriBlock, n - r0);
        GemmArgs g{};
        g.M = rows; g.N = r0; g.K = r0; g.alpha = 1.0; g.beta = 0.0;
        g.A = L + (size_t)r0 * n; g.lda = n; g.B = Linv; g.ldb = n; g.C = tmp; g.ldc = r0;
        g.batch = 1; g.nred = 1;
        if ((e = dgemm(g, st)) != hipSuccess) return e;
        GemmArgs h{};
        h.M = rows; h.N = r0; h.K = rows; h.alpha = -1.0; h.beta = 0.0;
        h.A = Linv + (size_t)r0 * n + r0; h.lda = n; h.B = tmp; h.ldb = r0; h.C = Linv + (size_t)r0 * n; h.ldc = n;
        h.batch = 1; h.nred = 1;
        if ((e = dgemm(h, st)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t fill(double *p, size_t n, double v, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(nblk(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t gather_rows(const double *src, double *dst, const int *perm, int nrow, int ncol, int ld_src, hipStream_t st)
{
    hipLaunchKernelGGL(k_gather_rows, dim3(nblk((size_t)nrow * ncol, 256)), dim3(256), 0, st, src, dst, perm, nrow,
                       ncol, ld_src);
    return hipGetLastError();
}

hipError_t scatter_sq(const double *in, double *out, const int *perm, int n, int nb, hipStream_t st)
{
    hipLaunchKernelGGL(k_scatter_sq, dim3(nblk((size_t)n * n * nb, 256)), dim3(256), 0, st, in, out, perm, n, nb);
    return hipGetLastError();
}

hipError_t gather_sq(const double *in, double *out, const int *perm, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_gather_sq, dim3(nblk((size_t)n * n, 256)), dim3(256), 0, st, in, out, perm, n);
    return hipGetLastError();
}

hipError_t make_rl(const double *X, const double *Y, double *R, double *L, size_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_rl, dim3(nblk(n, 256)), dim3(256), 0, st, X, Y, R, L, n);
    return hipGetLastError();
}

hipError_t symmetrize(double *A, int n, int nb, hipStream_t st)
{
    hipLaunchKernelGGL(k_symmetrize, dim3(nblk((size_t)n * n * nb, 256)), dim3(256), 0, st, A, n, nb);
    return hipGetLastError();
}

hipError_t mirror_lower(double *C, int n, long ldc, long sC, int batch, hipStream_t st)
{
    if (n <= 1 || batch <= 0) return hipSuccess;
    if (batch > 65535) return hipErrorInvalidValue;
    const int nt = (n + 31) / 32;
    hipLaunchKernelGGL(k_mirror_lower, dim3(nt, nt, batch), dim3(32, 8), 0, st, C, n, ldc, sC);
    return hipGetLastError();
}

hipError_t transpose(const double *in, long ldi, double *out, long ldo, int R, int C, hipStream_t st)
{
    if (R <= 0 || C <= 0) return hipSuccess;
    const int nct = (C + 31) / 32, nrt = (R + 31) / 32;
    hipLaunchKernelGGL(k_transpose, dim3(nct, std::min(nrt, 65535)), dim3(32, 8), 0, st, in, ldi, out, ldo, R, C);
    return hipGetLastError();
}

hipError_t sym_sum_lower(const double *X, double *G, int n, int batch, double s, hipStream_t st)
{
    if (n <= 0 || batch <= 0) return hipSuccess;
    if (batch > 65535) return hipErrorInvalidValue;
    const int nt = (n + 31) / 32;
    hipLaunchKernelGGL(k_sym_sum_lower, dim3(nt, nt, batch), dim3(32, 8), 0, st, X, G, n, (long)n * n, s);
    return hipGetLastError();
}

hipError_t add_sym(const double *G, int n, double *V, int ldv, double s, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_add_sym, dim3(nblk((size_t)n * n, 256)), dim3(256), 0, st, G, n, V, ldv, s);
    return hipGetLastError();
}

hipError_t add_de(const double *eps, const double *V, double *out, int nvir, int nocc, int nvec, double s,
                  hipStream_t st)
{
    hipLaunchKernelGGL(k_add_de, dim3(nblk((size_t)nvir * nocc * nvec, 256)), dim3(256), 0, st, eps, V, out, nvir,
                       nocc, nvec, s);
    return hipGetLastError();
}

hipError_t axpby(const double *src, double *dst, size_t n, double alpha, double beta, hipStream_t st)
{
    hipLaunchKernelGGL(k_axpby, dim3(nblk(n, 256)), dim3(256), 0, st, src, dst, n, alpha, beta);
    return hipGetLastError();
}

hipError_t to_float(const double *x, float *y, size_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_float, dim3(nblk(n, 256)), dim3(256), 0, st, x, y, n);
    return hipGetLastError();
}

hipError_t assemble3(const BlockGrid &g, double *W, int o, int nP, hipStream_t st, float *Wf)
{
    if (o <= 0 || nP <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_assemble3, dim3(3 * o, nP), dim3(256), 0, st, g, W, Wf, o);
    return hipGetLastError();
}

hipError_t permute3(const double *in, double *out, int n0, int n1, int n2, long s0, long s1, long s2, long o0,
                    long o1, long o2, hipStream_t st, double alpha, double beta)
{
    const size_t n = (size_t)n0 * n1 * n2;
    if (n == 0) return hipSuccess;
    if (n + 256 < (size_t)0x7fffffff)
        hipLaunchKernelGGL(k_permute3<unsigned>, dim3(nblk(n, 256)), dim3(256), 0, st, in, out, n0, n1, n2, s0, s1,
                           s2, o0, o1, o2, alpha, beta);
    else
        hipLaunchKernelGGL(k_permute3<long>, dim3(nblk(n, 256)), dim3(256), 0, st, in, out, n0, n1, n2, s0, s1, s2,
                           o0, o1, o2, alpha, beta);
    return hipGetLastError();
}

hipError_t reduce_grad(const double *p3, int nshAO, int nshAux, int nout, int NO, const double *p2,
                       const int *atomAO, const int *atomAux, int natm, double *shA, double *shC, double *shP,
                       double scale, int accumulate, double *grad, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_p3_a, dim3(nblk((size_t)nshAO * nout * 3, 64)), dim3(64), 0, st, p3, nshAO, nshAux,
                       nout, NO, shA);
    hipLaunchKernelGGL(k_reduce_p3_c, dim3(nblk((size_t)nshAux * nout * 3, 64)), dim3(64), 0, st, p3, nshAO,
                       nshAux, nout, NO, shC);
    if (p2)
        hipLaunchKernelGGL(k_reduce_p2, dim3(nblk((size_t)nshAux * nout * 3, 64)), dim3(64), 0, st, p2, nshAux,
                           nout, shP);
    hipLaunchKernelGGL(k_atoms, dim3(nblk((size_t)natm * nout * 3, 64)), dim3(64), 0, st, shA, atomAO, nshAO, shC,
                       atomAux, nshAux, p2 ? shP : nullptr, natm, nout, scale, accumulate, grad);
    return hipGetLastError();
}

}  // namespace ris

extern "C" int ris_test_transpose(const double *in, long ldi, double *out, long ldo, int R, int C)
{
    if (R < 0 || C < 0 || !in || !out || in == out || ldi < C || ldo < R) return 1;
    if (ris::transpose(in, ldi, out, ldo, R, C, 0) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return 7;
    return 0;
}
