// FP64 GEMM on the CDNA4 matrix cores: v_mfma_f64_16x16x4f64.
//
// C_b = alpha * sum_{r < nred} op(A_{b,r}) op(B_{b,r}) + beta * C_b, row-major.
// Block tile 128 x 128 x 16, 256 threads = 4 waves in a 2 x 2 arrangement,
// each wave owning a 64 x 64 sub-tile = 4 x 4 MFMA tiles (16 accumulators of
// four doubles).  Operand tiles are staged k-major in LDS so every MFMA
// fragment read is 16 consecutive doubles; the next k-slab is prefetched into
// registers while the current one is consumed.
//
// MFMA 16x16x4 f64 lane layout (wave64): A fragment lane l holds
// A[l % 16][l / 16], B fragment lane l holds B[l / 16][l % 16], and the four
// accumulator values of lane l are D[4 i + l / 16][l % 16], i = 0..3 (rows
// interleaved across the four lane groups; checked by the layout probe test).
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "ris_common.hpp"

namespace ris {
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
namespace {

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int PAD = 2;    // LDS row padding (doubles) against bank conflicts on the transposing stores
constexpr int NXCD = 8;   // accelerator complex dies on MI355X, each with its own L2
constexpr int GROUP_M = 2;  // m-tiles swept together so their A panels stay in L2

// Linear workgroup id -> (batch, m-tile, n-tile).  Workgroups are dispatched
// round-robin over the XCDs, so id b runs on XCD b % 8; remapping gives each
// XCD one contiguous range of tiles.  Inside a batch the tiles are walked in
// groups of GROUP_M m-tiles with the n-tile as the slower index, so one B
// panel serves GROUP_M consecutive tiles and the group's A panels stay hot.
__device__ __forceinline__ void tile_of(int b, int total, int tm, int tn, bool lower, const int *tiles, int &z,
                                        int &mt, int &nt)
{
    const int q = total / NXCD, r = total % NXCD;
    const int xcd = b % NXCD, local = b / NXCD;
    const int lin = (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + local;
    if (tiles) {  // an explicit list of tn tiles (mt << 16 | nt) per batch entry
        z = lin / tn;
        const int pk = tiles[lin - z * tn];
        mt = pk >> 16;
        nt = pk & 0xffff;
        return;
    }
    if (lower) {  // tiles (mt >= nt) of a square tm x tm grid, row by row
        const int per = tm * (tm + 1) / 2;
        z = lin / per;
        const int t = lin % per;
        int m = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while (m * (m + 1) / 2 > t) --m;
        while ((m + 1) * (m + 2) / 2 <= t) ++m;
        mt = m;
        nt = t - m * (m + 1) / 2;
        return;
    }
    const int per = tm * tn;
    z = lin / per;
    const int t = lin % per;
    const int gsz = GROUP_M * tn;                  // tiles per full group
    const int g = t / gsz, tg = t % gsz;
    const int m0 = g * GROUP_M;
    const int gm = min(GROUP_M, tm - m0);          // rows in this (possibly short) group
    mt = m0 + tg % gm;
    nt = tg / gm;
}

// element at a uniform base plus a 32-bit element offset (byte offset < 2^32)
template <typename E>
__device__ __forceinline__ double ld_off(const E *base, int off)
{
    return (double)*reinterpret_cast<const E *>(reinterpret_cast<const char *>(base) +
                                                ((unsigned)off * (unsigned)sizeof(E)));
}

// Matrix-core flavours of the one kernel below:
//   MODE 0: FP64 operands in LDS, v_mfma_f64_16x16x4f64, k-slab 16;
//   MODE 1: operands rounded to FP32 in LDS, v_mfma_f32_16x16x4f32 with FP32
//           accumulation, k-slab 32 (same matrix-core time per slab, since
//           the FP32 instruction runs at twice the FP64 rate).
// The FP32 instruction leaves D[4 (l/16) + e][l % 16] in accumulator element
// e of lane l (rows in blocks of four), the FP64 one D[4 e + l/16][l % 16].
template <int MODE> struct MfmaCfg;
template <> struct MfmaCfg<0> {
    typedef double T;
    typedef v4d V;
    static constexpr int BKm = 16;
    static __device__ __forceinline__ V mfma(T a, T b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ __forceinline__ int row(int lane, int e) { return 4 * e + (lane >> 4); }
};
template <> struct MfmaCfg<1> {
    typedef float T;
    typedef v4f V;
    static constexpr int BKm = 32;
    static __device__ __forceinline__ V mfma(T a, T b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ __forceinline__ int row(int lane, int e) { return 4 * (lane >> 4) + e; }
};

// Main loop per k-slab: the next slab's global loads are issued at the top,
// the matrix-core work of the current slab runs from LDS, and the next slab
// is written to the other LDS buffer before one barrier.  Loads use clamped
// addresses and a 0/1 factor instead of per-element branches, so a slab is
// one basic block and the scheduler can interleave the memory instructions
// with the MFMAs of the slab (group barriers below); two waves per SIMD (256
// unified registers each) keep the matrix cores fed.
//
// alpha scales the A slabs on their way to LDS and, unless BETA, the
// accumulators are stored as they are (arithmetic on them in the epilogue
// makes the compiler stage all of them through registers at once).
//
// EA, EB, EC: element types of A, B and C in memory (double, or float for the
// FP32 flavour's intermediates, which it rounds to FP32 anyway).
template <int MODE, bool TA, bool TB, bool BETA, typename EA = double, typename EB = double, typename EC = double>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_gemm(
    int M, int N, int K, double alpha, const EA *__restrict__ A, long lda, long sA, long sAr,
    const EB *__restrict__ B, long ldb, long sB, long sBr, double beta, EC *__restrict__ C, long ldc, long sC,
    int nred, int tm, int tn, int total, int kc, bool lower, const int *__restrict__ tiles)
{
    typedef MfmaCfg<MODE> Cfg;
    typedef typename Cfg::T T;
    constexpr int SK = Cfg::BKm;       // k-slab depth
    constexpr int NQ = BM * SK / 256;  // elements per thread per operand and slab
    constexpr int KF = SK;             // threads per row in the k-fast staging pattern
    __shared__ T As[2][SK][BM + PAD];
    __shared__ T Bs[2][SK][BN + PAD];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    int bz, mt, nt;
    tile_of(blockIdx.x, total, tm, tn, lower, tiles, bz, mt, nt);
    const int m0 = mt * BM, n0 = nt * BN;
    // kc > 0: split-K, the batch index selects the k-range [bz*kc, bz*kc + kc);
    // kc < 0: banded K of width w = -kc (column tiles inside the first or the
    // third block of w columns skip the zero third or first block of B's rows)
    int kbeg = 0, kend = K;
    if (kc > 0) {
        kbeg = bz * kc;
        kend = min(K, kbeg + kc);
    } else if (kc < 0) {
        if (n0 >= -2 * kc) kbeg = -kc;
        if (n0 + BN <= -kc) kend = min(K, -2 * kc);
    }
    A += (long)bz * sA;
    B += (long)bz * sB;
    C += (long)bz * sC;

    typename Cfg::V acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[i][j][e] = 0;

    // staging patterns (element q of a thread):
    //   k-fast (A not transposed / B transposed): k = tid % SK, row = tid / SK + (256 / SK) q
    //   m/n-fast (A transposed / B not transposed): col = tid & 127, k = (tid >> 7) + 2 q
    const int kf = tid % KF, rf = tid / KF;
    constexpr int RSTEP = 256 / KF;
    const int cf = tid & 127, kr = tid >> 7;
    // Addresses: a uniform panel base (scalar registers) plus a 32-bit
    // per-thread element offset, clamped into the operand so every load is
    // valid; out-of-range elements are zeroed by a 0/1 factor (a product, not
    // a select, so the compiler keeps the loads unconditional).  The launcher
    // guarantees that every byte offset fits 32 bits (scalar base + 32-bit
    // vector offset addressing).
    // staged values and their factors: FP32 for float operands (no FP64
    // arithmetic on them), FP64 otherwise
    typedef typename std::conditional<std::is_same<EA, float>::value, float, double>::type RA;
    typedef typename std::conditional<std::is_same<EB, float>::value, float, double>::type RB;
    int offA[NQ], offB[NQ];
    RA mA[NQ];
    RB mB[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int gm = m0 + rf + RSTEP * q, gn = n0 + rf + RSTEP * q;
        mA[q] = gm < M ? RA(1) : RA(0);
        mB[q] = gn < N ? RB(1) : RB(0);
        offA[q] = (min(gm, M - 1) - m0) * (int)lda;
        offB[q] = (min(gn, N - 1) - n0) * (int)ldb;
    }
    const RA mAc = m0 + cf < M ? RA(1) : RA(0);
    const RB mBc = n0 + cf < N ? RB(1) : RB(0);
    const int cA = min(m0 + cf, M - 1) - m0, cB = min(n0 + cf, N - 1) - n0;
    const RA ralpha = (RA)alpha;

    RA ra[NQ];
    RB rb[NQ];
    const int ktiles = (kend - kbeg + SK - 1) / SK;
    const int niter = ktiles * nred;

    auto load = [&](int it) {
        const int r = it / ktiles;
        const int k0 = kbeg + (it % ktiles) * SK;
        // panel bases: k-fast operands start at row m0 / n0, the others at row k0
        const EA *pA = A + (long)r * sAr + (TA ? (long)k0 * lda + m0 : (long)m0 * lda);
        const EB *pB = B + (long)r * sBr + (TB ? (long)n0 * ldb : (long)k0 * ldb + n0);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            if (!TA) {
                const int gk = k0 + kf;
                const RA x = (RA)ld_off(pA, offA[q] + min(gk, kend - 1));
                ra[q] = x * (gk < kend ? mA[q] : RA(0));
            } else {
                const int gk = k0 + kr + 2 * q;
                const RA x = (RA)ld_off(pA, (min(gk, kend - 1) - k0) * (int)lda + cA);
                ra[q] = x * (gk < kend ? mAc : RA(0));
            }
            if (!TB) {
                const int gk = k0 + kr + 2 * q;
                const RB x = (RB)ld_off(pB, (min(gk, kend - 1) - k0) * (int)ldb + cB);
                rb[q] = x * (gk < kend ? mBc : RB(0));
            } else {
                const int gk = k0 + kf;
                const RB x = (RB)ld_off(pB, offB[q] + min(gk, kend - 1));
                rb[q] = x * (gk < kend ? mB[q] : RB(0));
            }
        }
    };
    auto store = [&](int stg) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const T x = (T)(ra[q] * ralpha), y = (T)rb[q];
            if (!TA) As[stg][kf][rf + RSTEP * q] = x;
            else As[stg][kr + 2 * q][cf] = x;
            if (!TB) Bs[stg][kr + 2 * q][cf] = y;
            else Bs[stg][kf][rf + RSTEP * q] = y;
        }
    };

    // A wave whose 64 x 64 sub-tile holds nothing that is stored skips its
    // fragment reads, MFMAs and stores (it still stages its share of the
    // operands): the sub-tile past the last row or column of a ragged tile, and
    // in the lower-tile mode the strictly upper sub-tile of a diagonal tile.
    const bool act = m0 + wm * 64 < M && n0 + wn * 64 < N && !(lower && mt == nt && wm < wn);
    if (niter > 0) {
        load(0);
        store(0);
    }
    __syncthreads();
    // one k-slab; ACT: with the matrix-core work
    auto slab = [&](int it, auto act_tag) {
        constexpr bool ACT = decltype(act_tag)::value;
        const int cur = it & 1;
        // next slab (the last iteration reloads its own slab: in bounds, never read)
        load(min(it + 1, niter - 1));
        if constexpr (ACT) {
#pragma unroll
            for (int kk = 0; kk < SK; kk += 4) {
                T fa[4], fb[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) fa[i] = As[cur][kk + (lane >> 4)][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
                for (int j = 0; j < 4; ++j) fb[j] = Bs[cur][kk + (lane >> 4)][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = Cfg::mfma(fa[i], fb[j], acc[i][j]);
            }
        }
        // the other buffer was last read in iteration it-1, before the barrier that ended it
        store(cur ^ 1);
        if constexpr (ACT) {
            // schedule: fragment reads of the first k-step, then the global loads
            // one per MFMA, the remaining fragment reads one per MFMA, and the LDS
            // writes one per MFMA over the last MFMAs of the slab
            constexpr int NMF = 16 * (SK / 4), NLD = 2 * NQ, NDR = 8 * (SK / 4), NDW = 2 * NQ;
#pragma unroll
            for (int u = 0; u < 8; ++u) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
#pragma unroll
            for (int u = 0; u < NLD; ++u) {
                __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            }
#pragma unroll
            for (int u = 0; u < NDR - 8; ++u) {
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            }
#pragma unroll
            for (int u = 0; u < NMF - NLD - (NDR - 8) - NDW; ++u) __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
#pragma unroll
            for (int u = 0; u < NDW; ++u) {
                __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            }
        }
        __syncthreads();
    };
    if (act) {
        for (int it = 0; it < niter; ++it) slab(it, std::true_type{});
    } else {
        for (int it = 0; it < niter; ++it) slab(it, std::false_type{});
        return;
    }

#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = m0 + wm * 64 + i * 16 + Cfg::row(lane, e);
                if (row < M && col < N) {
                    EC *cp = C + (long)row * ldc + col;
                    if constexpr (BETA) *cp = (EC)((double)acc[i][j][e] + beta * (double)*cp);
                    else *cp = (EC)acc[i][j][e];
                }
            }
        }
}

}  // namespace

// Launch of the matrix-core GEMM (mode 0 FP64, 1 FP32); kc > 0: split-K ranges.
hipError_t gemm_kc(const GemmArgs &g, int mode, int kc, hipStream_t st)
{
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
    if (mode != 0 && mode != 1) return hipErrorInvalidValue;
    if (g.kband > 0) {
        if (kc != 0 || g.transB || g.lower || g.K != 3 * g.kband) return hipErrorInvalidValue;
        kc = -g.kband;
    }
    const int tm = (g.M + BM - 1) / BM;
    int tn = (g.N + BN - 1) / BN;
    if (g.lower && (g.M != g.N || kc > 0)) return hipErrorInvalidValue;
    long total = g.lower ? (long)tm * (tm + 1) / 2 * g.batch : (long)tm * tn * g.batch;
    if (g.tiles) {  // an explicit list of lower tiles: tn carries its length
        if (!g.lower || g.ntiles <= 0) return hipErrorInvalidValue;
        tn = g.ntiles;
        total = (long)g.ntiles * g.batch;
    }
    if (total > 0x7fffffffL) return hipErrorInvalidValue;
    // every operand byte offset from a panel base must fit 32 bits.  A k-fast
    // operand (A untransposed, B transposed) spans the rows of its tile; when
    // its rows are too long for a full tile, the product is issued in row
    // (column) slices short enough for 32-bit offsets.
    const long SKm = mode == 0 ? 16 : 32;
    auto fits = [](long span) { return 8 * span < (1L << 32); };
    if (!g.transA && !fits((std::min<long>(BM, g.M) - 1) * g.lda + g.K)) {
        long r = BM - 1;
        while (r > 1 && !fits((r - 1) * g.lda + g.K)) --r;
        if (g.lower || !fits((r - 1) * g.lda + g.K)) return hipErrorInvalidValue;
        const size_t szA = (g.ftypes & kF32A) ? 4 : 8, szC = (g.ftypes & kF32C) ? 4 : 8;
        for (long m0 = 0; m0 < g.M; m0 += r) {
            GemmArgs s = g;
            s.kband = 0;  // carried by kc from here on
            s.M = (int)std::min<long>(r, g.M - m0);
            s.A = (const double *)((const char *)g.A + (size_t)m0 * g.lda * szA);
            s.C = (double *)((char *)g.C + (size_t)m0 * g.ldc * szC);
            const hipError_t e = gemm_kc(s, mode, kc, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    if (g.transB && !fits((std::min<long>(BN, g.N) - 1) * g.ldb + g.K)) {
        long r = BN - 1;
        while (r > 1 && !fits((r - 1) * g.ldb + g.K)) --r;
        if (g.lower || !fits((r - 1) * g.ldb + g.K)) return hipErrorInvalidValue;
        const size_t szB = (g.ftypes & kF32B) ? 4 : 8, szC = (g.ftypes & kF32C) ? 4 : 8;
        for (long n0 = 0; n0 < g.N; n0 += r) {
            GemmArgs s = g;
            s.kband = 0;
            s.N = (int)std::min<long>(r, g.N - n0);
            s.B = (const double *)((const char *)g.B + (size_t)n0 * g.ldb * szB);
            s.C = (double *)((char *)g.C + (size_t)n0 * szC);
            const hipError_t e = gemm_kc(s, mode, kc, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    const long spanA = g.transA ? (SKm - 1) * g.lda + g.M : (std::min<long>(BM, g.M) - 1) * g.lda + g.K;
    const long spanB = g.transB ? (std::min<long>(BN, g.N) - 1) * g.ldb + g.K : (SKm - 1) * g.ldb + g.N;
    if (!fits(spanA) || !fits(spanB)) return hipErrorInvalidValue;
    if (g.ftypes != 0) {
        // FP32-stored operands: the two products that build Gamma in the FP32 mode
        const int nred0 = g.nred > 0 ? g.nred : 1;
        dim3 grid0((unsigned)total);
        if (mode != 1 || kc > 0) return hipErrorInvalidValue;
        if (g.ftypes == (kF32A | kF32B | kF32C) && !g.transA && !g.transB && g.beta == 0.0)
            hipLaunchKernelGGL((k_gemm<1, false, false, false, float, float, float>), grid0, dim3(256), 0, st, g.M, g.N,
                               g.K, g.alpha, (const float *)g.A, g.lda, g.strideA, g.strideAr, (const float *)g.B, g.ldb,
                               g.strideB, g.strideBr, g.beta, (float *)g.C, g.ldc, g.strideC, nred0, tm, tn, (int)total,
                               kc, g.lower, g.tiles);
        else if (g.ftypes == (kF32A | kF32B) && !g.transA && g.transB && g.beta == 0.0)
            hipLaunchKernelGGL((k_gemm<1, false, true, false, float, float, double>), grid0, dim3(256), 0, st, g.M, g.N,
                               g.K, g.alpha, (const float *)g.A, g.lda, g.strideA, g.strideAr, (const float *)g.B, g.ldb,
                               g.strideB, g.strideBr, g.beta, g.C, g.ldc, g.strideC, nred0, tm, tn, (int)total, kc,
                               g.lower, g.tiles);
        else if (g.ftypes == (kF32A | kF32B) && !g.transA && g.transB)
            hipLaunchKernelGGL((k_gemm<1, false, true, true, float, float, double>), grid0, dim3(256), 0, st, g.M, g.N,
                               g.K, g.alpha, (const float *)g.A, g.lda, g.strideA, g.strideAr, (const float *)g.B, g.ldb,
                               g.strideB, g.strideBr, g.beta, g.C, g.ldc, g.strideC, nred0, tm, tn, (int)total, kc,
                               g.lower, g.tiles);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
    dim3 grid((unsigned)total);
    const int nred = g.nred > 0 ? g.nred : 1;
#define RIS_GEMM_LAUNCH1(MODE, TA, TB, BETA)                                                                     \
    hipLaunchKernelGGL((k_gemm<MODE, TA, TB, BETA>), grid, dim3(256), 0, st, g.M, g.N, g.K, g.alpha, g.A, g.lda,  \
                       g.strideA, g.strideAr, g.B, g.ldb, g.strideB, g.strideBr, g.beta, g.C, g.ldc, g.strideC,     \
                       nred, tm, tn, (int)total, kc, g.lower, g.tiles);
#define RIS_GEMM_LAUNCH2(MODE, TA, TB)                                                                           \
    if (g.beta != 0.0) { RIS_GEMM_LAUNCH1(MODE, TA, TB, true) } else { RIS_GEMM_LAUNCH1(MODE, TA, TB, false) }
#define RIS_GEMM_LAUNCH(MODE)                                                                                    \
    if (!g.transA && !g.transB) { RIS_GEMM_LAUNCH2(MODE, false, false) }                                         \
    else if (g.transA && !g.transB) { RIS_GEMM_LAUNCH2(MODE, true, false) }                                      \
    else if (!g.transA && g.transB) { RIS_GEMM_LAUNCH2(MODE, false, true) }                                      \
    else { RIS_GEMM_LAUNCH2(MODE, true, true) }
    if (mode == 0) { RIS_GEMM_LAUNCH(0) }
    else { RIS_GEMM_LAUNCH(1) }
#undef RIS_GEMM_LAUNCH
#undef RIS_GEMM_LAUNCH1
#undef RIS_GEMM_LAUNCH2
    return hipGetLastError();
}

hipError_t dgemm_kc(const GemmArgs &g, int kc, hipStream_t st) { return gemm_kc(g, 0, kc, st); }

hipError_t dgemm(const GemmArgs &g, hipStream_t st) { return dgemm_kc(g, 0, st); }

}  // namespace ris

// ---------------------------------------------------------------- tests --
namespace {
typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf_t __attribute__((ext_vector_type(8)));

// kind 0: v_mfma_f64_16x16x4f64 (1 value per lane); kind 1: v_mfma_f32_16x16x4f32
// (1 value per lane); kind 2: v_mfma_f32_16x16x32_bf16 (8 values per lane).
__global__ __launch_bounds__(64) void k_mfma_probe(int kind, const double *a, const double *b, double *out)
{
    const int lane = threadIdx.x;
    if (kind == 0) {
        ris::v4d acc = ris::v4d{0.0, 0.0, 0.0, 0.0};
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[lane], b[lane], acc, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) out[4 * lane + e] = acc[e];
    } else if (kind == 1) {
        v4f_t acc = v4f_t{0.f, 0.f, 0.f, 0.f};
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32((float)a[lane], (float)b[lane], acc, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) out[4 * lane + e] = acc[e];
    } else {
        v8bf_t av, bv;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            av[i] = (__bf16)(float)a[8 * lane + i];
            bv[i] = (__bf16)(float)b[8 * lane + i];
        }
        v4f_t acc = v4f_t{0.f, 0.f, 0.f, 0.f};
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) out[4 * lane + e] = acc[e];
    }
}
}  // namespace

extern "C" int ris_test_mfma_probe(int kind, const double *a, const double *b, double *out)
{
    if (!a || !b || !out || kind < 0 || kind > 2) return 1;
    hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, 0, kind, a, b, out);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) return 7;
    return 0;
}

extern "C" int ris_test_dgemm(int M, int N, int K, int transA, int transB, double alpha, const double *A, long lda,
                              long sA, const double *B, long ldb, long sB, double beta, double *C, long ldc, long sC,
                              int batch)
{
    if (M < 0 || N < 0 || K < 0 || batch < 0 || !A || !B || !C) return 1;
    ris::GemmArgs g{};
    g.M = M; g.N = N; g.K = K;
    g.transA = transA != 0; g.transB = transB != 0;
    g.alpha = alpha; g.beta = beta;
    g.A = A; g.lda = lda; g.strideA = sA;
    g.B = B; g.ldb = ldb; g.strideB = sB;
    g.C = C; g.ldc = ldc; g.strideC = sC;
    g.batch = batch; g.nred = 1;
    if (ris::dgemm(g, 0) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return 7;
    return 0;
}

// ------------------------------------------------------------ split-K --
// C = alpha op(A) op(B) + beta C for a GEMM with a small M x N output and a
// long K: K is cut into nsplit ranges, each range writes its partial product
// to ws[z][M][N]; a second kernel sums the partials in a fixed order.
namespace {
// A workgroup of 256 takes 32 consecutive elements: thread (g, e) sums the
// partials z = g, g + 8, ... of element e (a wave reads 32 consecutive
// elements of two partials), then the 8 group sums are added in order.
__global__ __launch_bounds__(256) void k_splitk_reduce(const double *__restrict__ ws, int nsplit, int M, int N,
                                                       double beta, double *__restrict__ C, long ldc)
{
    __shared__ double part[8][32];
    const long tot = (long)M * N;
    const int e = threadIdx.x & 31, grp = threadIdx.x >> 5;
    const long idx = (long)blockIdx.x * 32 + e;
    double s = 0.0;
    if (idx < tot)
        for (int z = grp; z < nsplit; z += 8) s += ws[(size_t)z * tot + idx];
    part[grp][e] = s;
    __syncthreads();
    if (grp == 0 && idx < tot) {
        double v = part[0][e];
#pragma unroll
        for (int k = 1; k < 8; ++k) v += part[k][e];
        const int m = (int)(idx / N), n = (int)(idx % N);
        double *cp = C + (long)m * ldc + n;
        *cp = (beta == 0.0) ? v : v + beta * *cp;
    }
}
}  // namespace

namespace ris {

hipError_t gemm_splitk(const GemmArgs &g, int mode, int nsplit, double *ws, hipStream_t st)
{
    if (nsplit <= 1 || g.batch != 1 || g.nred > 1) return gemm_mp(g, mode, st);
    const int kc = ((g.K + nsplit - 1) / nsplit + 31) / 32 * 32;  // multiple of both k-slab depths
    const int used = (g.K + kc - 1) / kc;
    // one launch: batch index = k-range, partial products into ws[z][M][N]
    GemmArgs p = g;
    p.batch = used;
    p.strideA = 0;
    p.strideB = 0;
    p.beta = 0.0;
    p.C = ws;
    p.ldc = g.N;
    p.strideC = (long)g.M * g.N;
    hipError_t e = mode >= 2 ? bgemm_kc(p, kc, st, mode == 2 ? 2 : 3) : gemm_kc(p, mode, kc, st);
    if (e != hipSuccess) return e;
    const long tot = (long)g.M * g.N;
    if ((tot + 31) / 32 > 0x7fffffffL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((tot + 31) / 32)), dim3(256), 0, st, ws, used, g.M, g.N,
                       g.beta, g.C, g.ldc);
    return hipGetLastError();
}

hipError_t dgemm_splitk(const GemmArgs &g, int nsplit, double *ws, hipStream_t st)
{
    return gemm_splitk(g, 0, nsplit, ws, st);
}

int balanced_splits(long tiles, int smax)
{
    // workgroup slots: 256 CUs x 2 resident workgroups
    constexpr double kSlots = 512.0;
    if (tiles >= 4 * (long)kSlots) return 1;
    int best = 1;
    double beff = 0.0;
    for (int sp = 1; sp <= smax; ++sp) {
        const double w = (double)tiles * sp / kSlots;
        const double eff = w / std::ceil(w);
        if (eff > beff + 1e-9) {
            beff = eff;
            best = sp;
        }
        if (eff >= 0.95) break;
    }
    return best;
}
}  // namespace ris
