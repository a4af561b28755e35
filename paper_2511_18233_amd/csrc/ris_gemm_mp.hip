// Reduced-precision GEMMs for the exchange-weight contractions (FP64 in HBM,
// reduced precision on the matrix cores, FP32 accumulation, FP64 out).
//
//   mode 1 (FP32): operands rounded to FP32, v_mfma_f32_16x16x4f32 (the
//          matrix-core GEMM of ris_gemm.hip in its FP32 flavour).
//   mode 2 (split BF16, three products): x32 = fl32(x), hi = bf16(x32),
//          lo = bf16(x32 - hi); a.b ~ hi_a hi_b + hi_a lo_b + lo_a hi_b with
//          v_mfma_f32_16x16x32_bf16 (the lo_a lo_b term, ~2^-16 relative, is
//          dropped).
//
// Same contract as the FP64 dgemm (batch, batch-reduce, transposes, alpha,
// beta) and the same XCD-aware tile order.  Lane layouts (checked by the probe
// tests): FP32 16x16x4 as FP64 (A[l%16][l/16], B[l/16][l%16]); BF16 16x16x32
// lane l holds A[l%16][8(l/16)+s], B[8(l/16)+s][l%16], s = 0..7; both write
// D[4(l/16) + e][l%16] to accumulator element e (rows in blocks of four, unlike
// the interleaved rows of the FP64 instruction).
#include <algorithm>

#include "ris_common.hpp"

namespace ris {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int BM = 128, BN = 128;
constexpr int NXCD = 8;
constexpr int GROUP_M = 2;

__device__ __forceinline__ void tile_of(int b, int total, int tm, int tn, int &z, int &mt, int &nt)
{
    const int q = total / NXCD, r = total % NXCD;
    const int xcd = b % NXCD, local = b / NXCD;
    const int lin = (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + local;
    const int per = tm * tn;
    z = lin / per;
    const int t = lin % per;
    const int gsz = GROUP_M * tn;
    const int g = t / gsz, tg = t % gsz;
    const int m0 = g * GROUP_M;
    const int gm = min(GROUP_M, tm - m0);
    mt = m0 + tg % gm;
    nt = tg / gm;
}

// ----------------------------------------------------------- split BF16 --
constexpr int BK2 = 32;
constexpr int PAD2 = 8;  // bf16 elements; keeps 16-byte alignment of each row

__device__ __forceinline__ void split_bf16(double x, __bf16 &hi, __bf16 &lo)
{
    const float f = (float)x;
    hi = (__bf16)f;
    lo = (__bf16)(f - (float)hi);
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_bgemm3(int M, int N, int K, double alpha, const double *__restrict__ A,
                                                long lda, long sA, long sAr, const double *__restrict__ B, long ldb,
                                                long sB, long sBr, double beta, double *__restrict__ C, long ldc,
                                                long sC, int nred, int tm, int tn, int total)
{
    // k-contiguous tiles: a lane's 8 consecutive k of one row are one 16-byte read
    __shared__ __attribute__((aligned(16))) __bf16 Ah[2][BM][BK2 + PAD2];
    __shared__ __attribute__((aligned(16))) __bf16 Al[2][BM][BK2 + PAD2];
    __shared__ __attribute__((aligned(16))) __bf16 Bh[2][BN][BK2 + PAD2];
    __shared__ __attribute__((aligned(16))) __bf16 Bl[2][BN][BK2 + PAD2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    int bz, mt, nt;
    tile_of(blockIdx.x, total, tm, tn, bz, mt, nt);
    const int m0 = mt * BM, n0 = nt * BN;
    A += (long)bz * sA;
    B += (long)bz * sB;
    C += (long)bz * sC;
    v4f acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    double ra[16], rb[16];
    const int ktiles = (K + BK2 - 1) / BK2;
    const int niter = ktiles * nred;
    // element q of a thread's share: (row, k) of the 128 x 32 tile
    auto load = [&](int it) {
        const int r = it / ktiles, k0 = (it % ktiles) * BK2;
        const double *Ar = A + (long)r * sAr;
        const double *Br = B + (long)r * sBr;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            if (!TA) {  // 32 threads per row along k
                const int k = tid & 31, m = (tid >> 5) + 8 * q, gm = m0 + m, gk = k0 + k;
                ra[q] = (gm < M && gk < K) ? Ar[(long)gm * lda + gk] : 0.0;
            } else {    // 128 threads per k along m
                const int m = tid & 127, k = (tid >> 7) + 2 * q, gm = m0 + m, gk = k0 + k;
                ra[q] = (gm < M && gk < K) ? Ar[(long)gk * lda + gm] : 0.0;
            }
            if (!TB) {
                const int n = tid & 127, k = (tid >> 7) + 2 * q, gn = n0 + n, gk = k0 + k;
                rb[q] = (gn < N && gk < K) ? Br[(long)gk * ldb + gn] : 0.0;
            } else {
                const int k = tid & 31, n = (tid >> 5) + 8 * q, gn = n0 + n, gk = k0 + k;
                rb[q] = (gn < N && gk < K) ? Br[(long)gn * ldb + gk] : 0.0;
            }
        }
    };
    auto store = [&](int stg) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            __bf16 h, l;
            split_bf16(ra[q], h, l);
            if (!TA) {
                const int k = tid & 31, m = (tid >> 5) + 8 * q;
                Ah[stg][m][k] = h;
                Al[stg][m][k] = l;
            } else {
                const int m = tid & 127, k = (tid >> 7) + 2 * q;
                Ah[stg][m][k] = h;
                Al[stg][m][k] = l;
            }
            split_bf16(rb[q], h, l);
            if (!TB) {
                const int n = tid & 127, k = (tid >> 7) + 2 * q;
                Bh[stg][n][k] = h;
                Bl[stg][n][k] = l;
            } else {
                const int k = tid & 31, n = (tid >> 5) + 8 * q;
                Bh[stg][n][k] = h;
                Bl[stg][n][k] = l;
            }
        }
    };
    if (niter > 0) {
        load(0);
        store(0);
    }
    __syncthreads();
    const int kofs = 8 * (lane >> 4);
    for (int it = 0; it < niter; ++it) {
        const int cur = it & 1;
        if (it + 1 < niter) load(it + 1);
        v8bf ah[4], al[4], bh[4], bl[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = wm * 64 + i * 16 + (lane & 15);
            ah[i] = *(const v8bf *)&Ah[cur][m][kofs];
            al[i] = *(const v8bf *)&Al[cur][m][kofs];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = wn * 64 + j * 16 + (lane & 15);
            bh[j] = *(const v8bf *)&Bh[cur][n][kofs];
            bl[j] = *(const v8bf *)&Bl[cur][n][kofs];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
            }
        if (it + 1 < niter) store(cur ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + e;
                if (row < M && col < N) {
                    double *cp = C + (long)row * ldc + col;
                    const double v = alpha * (double)acc[i][j][e];
                    *cp = (beta == 0.0) ? v : v + beta * *cp;
                }
            }
        }
}

}  // namespace

hipError_t gemm_mp(const GemmArgs &g, int mode, hipStream_t st)
{
    if (mode == 0 || mode == 1) return gemm_kc(g, mode, 0, st);
    if (g.ftypes) return hipErrorInvalidValue;  // FP32-stored operands: FP32 kernel only
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
    if (g.lower) return hipErrorInvalidValue;  // lower-tile mode: FP64 / FP32 kernel only
    const int tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
    const long total = (long)tm * tn * g.batch;
    if (total > 0x7fffffffL) return hipErrorInvalidValue;
    dim3 grid((unsigned)total);
    const int nred = g.nred > 0 ? g.nred : 1;
#define RIS_MP_LAUNCH(KERN, TA, TB)                                                                                \
    hipLaunchKernelGGL((KERN<TA, TB>), grid, dim3(256), 0, st, g.M, g.N, g.K, g.alpha, g.A, g.lda, g.strideA,      \
                       g.strideAr, g.B, g.ldb, g.strideB, g.strideBr, g.beta, g.C, g.ldc, g.strideC, nred, tm, tn, \
                       (int)total)
    if (!g.transA && !g.transB) RIS_MP_LAUNCH(k_bgemm3, false, false);
    else if (g.transA && !g.transB) RIS_MP_LAUNCH(k_bgemm3, true, false);
    else if (!g.transA && g.transB) RIS_MP_LAUNCH(k_bgemm3, false, true);
    else RIS_MP_LAUNCH(k_bgemm3, true, true);
#undef RIS_MP_LAUNCH
    return hipGetLastError();
}

}  // namespace ris

extern "C" int ris_test_gemm(int mode, int M, int N, int K, int transA, int transB, double alpha, const double *A,
                             long lda, long sA, const double *B, long ldb, long sB, double beta, double *C, long ldc,
                             long sC, int batch)
{
    if (M < 0 || N < 0 || K < 0 || batch < 0 || !A || !B || !C || mode < 0 || mode > 2) return 1;
    ris::GemmArgs g{};
    g.M = M; g.N = N; g.K = K;
    g.transA = transA != 0; g.transB = transB != 0;
    g.alpha = alpha; g.beta = beta;
    g.A = A; g.lda = lda; g.strideA = sA;
    g.B = B; g.ldb = ldb; g.strideB = sB;
    g.C = C; g.ldc = ldc; g.strideC = sC;
    g.batch = batch; g.nred = 1;
    if (ris::gemm_mp(g, mode, 0) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return 7;
    return 0;
}
