// Reduced-precision GEMMs for the exchange-weight contractions (FP64 in HBM,
// reduced precision on the matrix cores, FP32 accumulation, FP64 out).
//
//   mode 1 (FP32): operands rounded to FP32, v_mfma_f32_16x16x4f32 (the
//          matrix-core GEMM of ris_gemm.hip in its FP32 flavour).
//   mode 2 (split BF16, three products): x32 = fl32(x), hi = bf16(x32),
//          lo = bf16(x32 - hi); a.b ~ hi_a hi_b + hi_a lo_b + lo_a hi_b with
//          v_mfma_f32_16x16x32_bf16 (the lo_a lo_b term, ~2^-16 relative, is
//          dropped).
//   mode 3 (split BF16, six products): the three-way split x32 = hi + mid + lo
//          (mid = bf16(x32 - hi), lo = bf16(x32 - hi - mid), which holds all
//          24 bits of x32) and the six products whose order is at most 2^-16:
//          hi.hi + hi.mid + mid.hi + hi.lo + lo.hi + mid.mid (mid.lo, lo.mid
//          and lo.lo, 2^-24 and below, are dropped).
//
// k_bgemm3 has the same contract as the FP64 dgemm (batch, batch-reduce,
// transposes, alpha, beta) and the same XCD-aware tile order; k_pgemm runs the
// split modes' two products of every output (Y^P = F_I W^P, Gamma^P) on
// operands kept pre-split in HBM (PGemmArgs).  Lane layouts (checked by the probe
// tests): FP32 16x16x4 as FP64 (A[l%16][l/16], B[l/16][l%16]); BF16 16x16x32
// lane l holds A[l%16][8(l/16)+s], B[8(l/16)+s][l%16], s = 0..7; both write
// D[4(l/16) + e][l%16] to accumulator element e (rows in blocks of four, unlike
// the interleaved rows of the FP64 instruction).
#include <algorithm>
#include <type_traits>

#include "ris_common.hpp"
#include "ris_linalg.hpp"

namespace ris {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int BM = 128, BN = 128;
constexpr int NXCD = 8;
constexpr int GROUP_M = 2;
constexpr int BK2 = 32;  // k-slab: one v_mfma_f32_16x16x32_bf16 step
constexpr int PAD2 = 8;  // bf16 elements; keeps 16-byte alignment of each LDS row

// Linear workgroup id -> (batch, m-tile, n-tile): each XCD walks one
// contiguous range; lower: the tiles mt >= nt of a square grid, row by row;
// otherwise groups of GROUP_M m-tiles with the n-tile as the slower index.
__device__ __forceinline__ void tile_of(int b, int total, int tm, int tn, bool lower, const int *tiles, int &z,
                                        int &mt, int &nt, int group = GROUP_M)
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
    if (lower) {
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
    const int gsz = group * tn;
    const int g = t / gsz, tg = t % gsz;
    const int m0 = g * group;
    const int gm = min(group, tm - m0);
    mt = m0 + tg % gm;
    nt = tg / gm;
}

// element at a uniform base plus a 32-bit element offset (byte offset < 2^32)
template <typename E>
__device__ __forceinline__ E ldo(const E *base, int off)
{
    return *reinterpret_cast<const E *>(reinterpret_cast<const char *>(base) + ((unsigned)off * (unsigned)sizeof(E)));
}

// x32 = fl32(x) * s split into NS bf16 parts: p[0] = bf16(x32), p[k] = bf16 of
// what the earlier parts leave (each difference is exact in FP32); s is a 0/1
// mask, or alpha
template <int NS, typename E>
__device__ __forceinline__ void split_bf16(E x, float s, __bf16 (&p)[NS])
{
    float f = (float)x * s;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        p[k] = (__bf16)f;
        f -= (float)p[k];
    }
}

// ----------------------------------------------------------- split BF16 --
// 128 x 128 tiles, 4 waves of 64 x 64, k-slabs of 32.  Every thread owns 8
// pairs of consecutive k: along rows for a k-fast operand (16 lanes sweep 32
// consecutive k of one row, so each load instruction reads whole rows) and
// along the m- / n-index for the other (64 lanes sweep 64 consecutive
// columns).  Loads are clamped into the operand and zeroed by a 0/1 factor
// (one basic block per slab); each pair's hi and lo parts go to LDS as one
// 32-bit word each, laid out [row][k] so a lane reads its MFMA fragment (8
// consecutive k of one row) as one 16-byte vector.  The three products run
// product-major over the 16 accumulators, so consecutive MFMAs never depend
// on each other.  alpha scales A before the split; lower-tile, split-K
// (batch index = k-range) and batch-reduce as in the FP64 kernel.
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));

// Parts of A and B in product u: NS = 2: hi.lo, lo.hi, hi.hi;
// NS = 3: hi.lo, lo.hi, mid.mid, hi.mid, mid.hi, hi.hi (smallest first).
template <int NS>
__device__ constexpr int part_a(int u)
{
    return NS == 2 ? (u == 1 ? 1 : 0) : (u == 1 ? 2 : (u == 2 || u == 4) ? 1 : 0);
}
template <int NS>
__device__ constexpr int part_b(int u)
{
    return NS == 2 ? (u == 0 ? 1 : 0) : (u == 0 ? 2 : (u == 2 || u == 3) ? 1 : 0);
}

//
// EA, EB, EC: element types in memory (double, or float for operands that are
// already FP32, which the split rounds to first anyway: same result).
// NS: parts per operand (2: three products, 3: six products).
template <int NS, bool TA, bool TB, bool BETA, typename EA = double, typename EB = double, typename EC = double>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_bgemm3(
    int M, int N, int K, double alpha, const EA *__restrict__ A, long lda, long sA, long sAr,
    const EB *__restrict__ B, long ldb, long sB, long sBr, double beta, EC *__restrict__ C, long ldc, long sC,
    int nred, int tm, int tn, int total, int kc, bool lower, const int *__restrict__ tiles)
{
    static_assert(NS == 2 || NS == 3, "two or three parts per operand");
    static_assert(BM == BN, "A and B part tiles share one LDS shape");
    // parts [0, NS) of A and [NS, 2 NS) of B, two stages each: [part][stage][row][k]
    __shared__ __attribute__((aligned(16))) __bf16 S[2 * NS][2][BM][BK2 + PAD2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    int bz, mt, nt;
    tile_of(blockIdx.x, total, tm, tn, lower, tiles, bz, mt, nt);
    const int m0 = mt * BM, n0 = nt * BN;
    // kc > 0: split-K range of the batch index; kc < 0: banded K of width -kc
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

    v4f acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    // k-fast share: k-pair 2 (tid & 15), rows (tid >> 4) + 16 q;
    // m-fast share: column tid & 127, k-pairs 2 (tid >> 7) + 4 q   (q < 8)
    const int kp = 2 * (tid & 15), rk = tid >> 4;
    const int cm = tid & 127, km = 2 * (tid >> 7);
    int offA[8], offB[8];
    unsigned vA = 0, vB = 0;  // bit q: row rk + 16 q inside the operand
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int ra = m0 + rk + 16 * q, rb = n0 + rk + 16 * q;
        vA |= (ra < M ? 1u : 0u) << q;
        vB |= (rb < N ? 1u : 0u) << q;
        offA[q] = (min(ra, M - 1) - m0) * (int)lda;
        offB[q] = (min(rb, N - 1) - n0) * (int)ldb;
    }
    const bool vAc = m0 + cm < M, vBc = n0 + cm < N;
    const int cA = min(m0 + cm, M - 1) - m0, cB = min(n0 + cm, N - 1) - n0;
    const float falpha = (float)alpha;

    EA xa[8][2];
    EB xb[8][2];
    float fa[8][2], fb[8][2];  // 0/1 validity (times alpha for A), applied in FP32 at the split
    const int ktiles = (kend - kbeg + BK2 - 1) / BK2;
    const int niter = ktiles * nred;

    auto load = [&](int it) {
        const int r = it / ktiles;
        const int k0 = kbeg + (it % ktiles) * BK2;
        const EA *pA = A + (long)r * sAr + (TA ? (long)k0 * lda + m0 : (long)m0 * lda);
        const EB *pB = B + (long)r * sBr + (TB ? (long)n0 * ldb : (long)k0 * ldb + n0);
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                if (!TA) {
                    const int gk = k0 + kp + s;
                    xa[q][s] = ldo(pA, offA[q] + min(gk, kend - 1));
                    fa[q][s] = (gk < kend && (vA >> q & 1u)) ? falpha : 0.0f;
                } else {
                    const int gk = k0 + km + 4 * q + s;
                    xa[q][s] = ldo(pA, (min(gk, kend - 1) - k0) * (int)lda + cA);
                    fa[q][s] = (gk < kend && vAc) ? falpha : 0.0f;
                }
                if (TB) {
                    const int gk = k0 + kp + s;
                    xb[q][s] = ldo(pB, offB[q] + min(gk, kend - 1));
                    fb[q][s] = (gk < kend && (vB >> q & 1u)) ? 1.0f : 0.0f;
                } else {
                    const int gk = k0 + km + 4 * q + s;
                    xb[q][s] = ldo(pB, (min(gk, kend - 1) - k0) * (int)ldb + cB);
                    fb[q][s] = (gk < kend && vBc) ? 1.0f : 0.0f;
                }
            }
    };
    auto store = [&](int stg) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            v2bf pa[NS], pb[NS];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                __bf16 t[NS];
                split_bf16<NS>(xa[q][s], fa[q][s], t);
#pragma unroll
                for (int k = 0; k < NS; ++k) pa[k][s] = t[k];
                split_bf16<NS>(xb[q][s], fb[q][s], t);
#pragma unroll
                for (int k = 0; k < NS; ++k) pb[k][s] = t[k];
            }
            const int arow = TA ? cm : rk + 16 * q, acol = TA ? km + 4 * q : kp;
            const int brow = TB ? rk + 16 * q : cm, bcol = TB ? kp : km + 4 * q;
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                *(v2bf *)&S[k][stg][arow][acol] = pa[k];
                *(v2bf *)&S[NS + k][stg][brow][bcol] = pb[k];
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
        // next slab (the last iteration reloads its own slab: in bounds, never read)
        load(min(it + 1, niter - 1));
        // fragments: part k of A rows / B columns of this wave
        v8bf fa_[NS][4], fb_[NS][4];
#pragma unroll
        for (int i = 0; i < 4; ++i) fa_[0][i] = *(const v8bf *)&S[0][cur][wm * 64 + i * 16 + (lane & 15)][kofs];
#pragma unroll
        for (int j = 0; j < 4; ++j) fb_[1][j] = *(const v8bf *)&S[NS + 1][cur][wn * 64 + j * 16 + (lane & 15)][kofs];
#pragma unroll
        for (int i = 0; i < 4; ++i) fa_[1][i] = *(const v8bf *)&S[1][cur][wm * 64 + i * 16 + (lane & 15)][kofs];
#pragma unroll
        for (int j = 0; j < 4; ++j) fb_[0][j] = *(const v8bf *)&S[NS][cur][wn * 64 + j * 16 + (lane & 15)][kofs];
        if constexpr (NS == 3) {
#pragma unroll
            for (int i = 0; i < 4; ++i) fa_[2][i] = *(const v8bf *)&S[2][cur][wm * 64 + i * 16 + (lane & 15)][kofs];
#pragma unroll
            for (int j = 0; j < 4; ++j) fb_[2][j] = *(const v8bf *)&S[NS + 2][cur][wn * 64 + j * 16 + (lane & 15)][kofs];
        }
        // products (part of A, part of B), smallest first, each over all 16
        // accumulators: hi.lo, lo.hi, hi.hi; or hi.lo, lo.hi, mid.mid, hi.mid, mid.hi, hi.hi
        constexpr int NP = NS == 2 ? 3 : 6;
#pragma unroll
        for (int u = 0; u < NP; ++u)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa_[part_a<NS>(u)][i], fb_[part_b<NS>(u)][j],
                                                                        acc[i][j], 0, 0, 0);
        // the other buffer was last read in iteration it-1, before the barrier that ended it
        store(cur ^ 1);
        if constexpr (NS == 2) {
            // schedule: the fragments of the first product, the other fragment
            // reads and the 32 global loads one per MFMA, and the 32 LDS writes
            // four per MFMA over the last eight MFMAs of the slab
#pragma unroll
            for (int u = 0; u < 8; ++u) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            }
#pragma unroll
            for (int u = 0; u < 32; ++u) {
                __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                __builtin_amdgcn_sched_group_barrier(0x200, 4, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            }
        }
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
                    EC *cp = C + (long)row * ldc + col;
                    if constexpr (BETA) *cp = (EC)((double)acc[i][j][e] + beta * (double)*cp);
                    else *cp = (EC)acc[i][j][e];
                }
            }
        }
}

// ------------------------------------------------ pre-split operands --
// The same products on operands already held as bf16 planes (PGemmArgs),
// both k-fast: 128 x 128 tiles, 4 waves of 64 x 64, k-slabs of 32.  Per slab
// and operand a thread moves 2 ns chunks of 16 bytes (8 consecutive k of one
// row of one part; four threads cover a row's 32 k) from global memory
// through registers into LDS; two register sets keep the loads of slab
// it + 2 in flight while slab it is multiplied.  K and the band bounds are
// multiples of 32 (the planes' padded width, zero past the logical one), so
// every slab is whole and the loop has no tail.  Rows past M or N are read
// clamped and never stored.  LDS rows are swizzled (swz).  The products and
// their order per slab are those of k_bgemm3.  SYM2 (M == N, lda == ldb):
// C = alpha (A B^T + B A^T) in one pass, the k-slabs of A B^T followed by
// those of B A^T (operand bases and part strides swapped) into the same
// accumulators.
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// LDS rows of 32 bf16 (64 bytes, unpadded) hold their four 16-byte chunks in
// the order c ^ swz(r): with it both the fragment reads (lane l: row l % 16,
// chunk l / 16) and the staging writes (lane l: row l / 4, chunk l % 4) are
// free of bank conflicts on gfx950 (measured with the LDS conflict counter;
// plain rows and rows padded to 80 bytes conflict on the reads).
__device__ __forceinline__ int swz(int r) { return (r >> 1) & 3; }

template <int NS, bool OUTP, bool BETA, bool SYM2 = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_pgemm(PGemmArgs g, int tm,
                                                                                          int tn, int total)
{
    // [stage][A, B][part][row][k], 16-byte chunk c of row r at chunk c ^ swz(r)
    __shared__ __attribute__((aligned(16))) uint16_t S[2][2][NS][BM][BK2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    int bz, mt, nt;
    // full grids: groups of 8 m-tiles per sweep of the n-tiles, so a B panel
    // (W^P of the Y product) is fetched once per 8 row panels of A
    tile_of(blockIdx.x, total, tm, tn, g.lower, g.tiles, bz, mt, nt, 8);
    const int m0 = mt * BM, n0 = nt * BN;
    int kbeg = 0, kend = g.K;
    if (g.kband > 0) {  // whole slabs: the bounds rounded outward into B's zero blocks
        const int w = g.kband;
        if (n0 >= 2 * w) kbeg = w & ~(BK2 - 1);
        if (n0 + BN <= w) kend = min(g.K, (2 * w + BK2 - 1) & ~(BK2 - 1));
    }
    const char *A = reinterpret_cast<const char *>(g.A + (long)bz * g.sA);
    const char *B = reinterpret_cast<const char *>(g.B + (long)bz * g.sB);
    const long psA = 2 * g.psA, psB = 2 * g.psB;  // bytes

    // chunk q < 2 of this thread: row 64 q + tid / 4, k-offset kq (stored at
    // kqs: rows 64 q + tid / 4 share their swizzle)
    const int kq = 8 * (tid & 3), kqs = 8 * ((tid & 3) ^ swz(tid >> 2));
    int rq[2];
    unsigned offA[2], offB[2];  // byte offsets of (row, kq) from the operand base
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        rq[q] = 64 * q + (tid >> 2);
        offA[q] = (unsigned)(((long)min(m0 + rq[q], g.M - 1) * g.lda + kq) * 2);
        offB[q] = (unsigned)(((long)min(n0 + rq[q], g.N - 1) * g.ldb + kq) * 2);
    }
    // two register sets of staged chunks: slab it + 2 is loaded while slab it
    // is multiplied and slab it + 1 waits in the other set
    v4u xa[2][NS][2], xb[2][NS][2];
    typedef std::integral_constant<int, 0> S0_;
    typedef std::integral_constant<int, 1> S1_;
    // k-slabs per product (SYM2: two products, nh slabs each)
    const int nh = kend > kbeg ? (kend - kbeg + BK2 - 1) / BK2 : 0;
    // slab s into register set SET (every slab is whole: K and the band
    // bounds are multiples of 32); with SYM2, slabs from nh on are those of
    // B A^T: B's rows at the tile's row offsets (offA, as lda == ldb and
    // M == N) and A's at its column offsets
    auto load_slab = [&](auto set, int s) {
        constexpr int SET = decltype(set)::value;
        const bool sw = SYM2 && s >= nh;
        const long k0 = kbeg + (long)(sw ? s - nh : s) * BK2;
        const char *a = (sw ? B : A) + 2 * k0, *b = (sw ? A : B) + 2 * k0;
        const long pa = sw ? psB : psA, pb = sw ? psA : psB;
#pragma unroll
        for (int p = 0; p < NS; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                xa[SET][p][q] = *reinterpret_cast<const v4u *>(a + p * pa + offA[q]);
                xb[SET][p][q] = *reinterpret_cast<const v4u *>(b + p * pb + offB[q]);
            }
    };
    // set SET into LDS stage SET (slab s sits in set s % 2 and stage s % 2)
    auto store = [&](auto set) {
        constexpr int SET = decltype(set)::value;
#pragma unroll
        for (int p = 0; p < NS; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                *reinterpret_cast<v4u *>(&S[SET][0][p][rq[q]][kqs]) = xa[SET][p][q];
                *reinterpret_cast<v4u *>(&S[SET][1][p][rq[q]][kqs]) = xb[SET][p][q];
            }
    };

    v4f acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    // fragment rows start at multiples of 16, so their swizzle is that of lane & 15
    const int kofs = 8 * ((lane >> 4) ^ swz(lane & 15));
    const int nslab = SYM2 ? 2 * nh : nh;
    // A wave whose 64 x 64 sub-tile holds nothing that is stored skips its
    // fragment reads, MFMAs and stores (it still stages its share of the
    // operands): past the last row or stored column of a ragged tile, and in
    // the lower-tile mode the strictly upper sub-tile of a diagonal tile.
    const bool act = m0 + wm * 64 < g.M && n0 + wn * 64 < (OUTP ? (int)g.ldc : g.N) &&
                     !(g.lower && mt == nt && wm < wn);
    // slab it from LDS stage CUR = it % 2; ACT: with the matrix-core work
    auto slab = [&](int it, auto cur, auto act_tag) {
        constexpr int CUR = decltype(cur)::value;
        constexpr int NXT = 1 - CUR;
        constexpr bool ACT = decltype(act_tag)::value;
        typedef std::integral_constant<int, NXT> N_;
        // slab it + 2 into the set slab it left (stored to LDS one slab ago);
        // its global loads go out first, ahead of this slab's work (the last
        // two slabs reload the last one: in bounds, never stored)
        load_slab(cur, min(it + 2, nslab - 1));
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (ACT) {
            // fragments in the order the products use them: the parts of product 0
            // (hi of A, lo of B), then lo of A and hi of B, then mid (NS = 3)
            v8bf fa_[NS][4], fb_[NS][4];
            constexpr int pa_[3] = {0, NS - 1, 1}, pb_[3] = {NS - 1, 0, 1};
#pragma unroll
            for (int h = 0; h < NS; ++h) {
                const int p = pa_[h], q = pb_[h];
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    fa_[p][i] = *reinterpret_cast<const v8bf *>(&S[CUR][0][p][wm * 64 + i * 16 + (lane & 15)][kofs]);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    fb_[q][j] = *reinterpret_cast<const v8bf *>(&S[CUR][1][q][wn * 64 + j * 16 + (lane & 15)][kofs]);
            }
            constexpr int NP = NS == 2 ? 3 : 6;
#pragma unroll
            for (int u = 0; u < NP; ++u)
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa_[part_a<NS>(u)][i], fb_[part_b<NS>(u)][j],
                                                                            acc[i][j], 0, 0, 0);
        }
        // slab it + 1 into the other stage, last read in slab it - 1 (before
        // the barrier that ended it), after every MFMA of this slab
        __builtin_amdgcn_sched_barrier(0);
        if (it + 1 < nslab) store(N_{});
        __syncthreads();
    };
    if (nslab > 0) {
        load_slab(S0_{}, 0);
        store(S0_{});
        load_slab(S1_{}, min(1, nslab - 1));
    }
    __syncthreads();
    int it = 0;
    if (act) {
        for (; it + 1 < nslab; it += 2) {
            slab(it, S0_{}, std::true_type{});
            slab(it + 1, S1_{}, std::true_type{});
        }
        if (it < nslab) slab(it, S0_{}, std::true_type{});
    } else {
        for (; it + 1 < nslab; it += 2) {
            slab(it, S0_{}, std::false_type{});
            slab(it + 1, S1_{}, std::false_type{});
        }
        if (it < nslab) slab(it, S0_{}, std::false_type{});
        return;
    }

    const float falpha = (float)g.alpha;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + e;
                if constexpr (OUTP) {
                    if (row < g.M && col < g.ldc) {
                        __bf16 t[NS];
                        split_bf16<NS>(acc[i][j][e], col < g.N ? falpha : 0.0f, t);
                        uint16_t *cp = g.Cp + (long)bz * g.sC + (long)row * g.ldc + col;
#pragma unroll
                        for (int p = 0; p < NS; ++p) cp[p * g.psC] = __builtin_bit_cast(uint16_t, t[p]);
                    }
                } else {
                    if (row < g.M && col < g.N) {
                        double *cp = g.C + (long)bz * g.sC + (long)row * g.ldc + col;
                        double v = g.alpha * (double)acc[i][j][e];
                        if constexpr (BETA) v += g.beta * *cp;
                        *cp = v;
                    }
                }
            }
        }
}

// ns bf16 parts of fl32(x) per element (split_bf16), zero in the padding columns
template <int NS>
__global__ void k_split_planes(const double *__restrict__ x, int rows, int cols, long ldx, long sx,
                               uint16_t *__restrict__ dst, long ps, long sdst, long ldp)
{
    const long n = (long)rows * ldp;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int b = blockIdx.y;
    const int r = (int)(idx / ldp), cidx = (int)(idx - (long)r * ldp);
    const double v = cidx < cols ? x[(long)b * sx + (long)r * ldx + cidx] : 0.0;
    __bf16 t[NS];
    split_bf16<NS>(v, 1.0f, t);
    uint16_t *d = dst + (long)b * sdst + idx;
#pragma unroll
    for (int p = 0; p < NS; ++p) d[p * ps] = __builtin_bit_cast(uint16_t, t[p]);
}

// Planes of W^T for a 3 x 3 block assembly (k_assemble3's sources): one
// workgroup per 64 x 64 piece (i0, j0) of one block (bi, bj) and matrix P, so
// the block's source descriptors are uniform; the piece is read into LDS along
// whichever index is contiguous in its first source (rows of a row-major
// block, columns of a transposed one), with clamped indices so the loads need
// no branch, and written along W^T's rows.  A last row of workgroups
// (blockIdx.y == 3 nto) writes the padding columns [3o, plane_ld(3o)) of W^T's
// rows zero.
template <int NS>
__global__ __launch_bounds__(256) void k_assemble3_planes(BlockGrid g, uint16_t *__restrict__ Wt, int o, long ps)
{
    __shared__ float T[64][65];
    const int n3 = 3 * o, nto = (o + 63) >> 6;
    const long ldp = plane_ld(n3);
    const int bj = blockIdx.x / nto, j0 = (blockIdx.x - bj * nto) * 64;
    const int P = blockIdx.z, tid = threadIdx.x;
    uint16_t *const Wp = Wt + (long)P * n3 * ldp;
    if ((int)blockIdx.y == 3 * nto) {
        for (int e = tid; e < 64 * 32; e += 256) {
            const int cc = e >> 5, r = n3 + (e & 31);
            if (j0 + cc < o && r < ldp) {
                uint16_t *d = Wp + (long)(bj * o + j0 + cc) * ldp + r;
#pragma unroll
                for (int p = 0; p < NS; ++p) d[p * ps] = 0;
            }
        }
        return;
    }
    const int bi = blockIdx.y / nto, i0 = (blockIdx.y - bi * nto) * 64;
    const BlockSrc s0 = g.b[bi][bj][0], s1 = g.b[bi][bj][1];
    if (s0.base || s1.base) {
        // a missing source is read from the present one with factor 0
        const BlockSrc a = s0.base ? s0 : s1;
        const BlockSrc b = s1.base ? s1 : a;
        const double ca = s0.base ? s0.scale : 0.0, cb = s1.base ? s1.scale : 0.0;
        const double *pa = a.base + P * a.sP, *pb = b.base + P * b.sP;
        const bool rows = a.sj == 1;
#pragma unroll 4
        for (int k = 0; k < 16; ++k) {
            const int u = 4 * k + (tid >> 6), w = tid & 63;
            const int ii = rows ? u : w, jj = rows ? w : u;
            const long i = min(i0 + ii, o - 1), j = min(j0 + jj, o - 1);
            T[ii][jj] = (float)(ca * pa[i * a.si + j * a.sj] + cb * pb[i * b.si + j * b.sj]);
        }
    } else {
#pragma unroll 4
        for (int k = 0; k < 16; ++k) T[4 * k + (tid >> 6)][tid & 63] = 0.0f;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < 16; ++k) {
        const int cc = 4 * k + (tid >> 6), rr = tid & 63;
        if (j0 + cc < o && i0 + rr < o) {
            __bf16 t[NS];
            split_bf16<NS>(T[rr][cc], 1.0f, t);
            uint16_t *d = Wp + (long)(bj * o + j0 + cc) * ldp + bi * o + i0 + rr;
#pragma unroll
            for (int p = 0; p < NS; ++p) d[p * ps] = __builtin_bit_cast(uint16_t, t[p]);
        }
    }
}

}  // namespace

hipError_t assemble3_planes(const BlockGrid &g, uint16_t *Wt, int o, int nP, long ps, int ns, hipStream_t st)
{
    if (o <= 0 || nP <= 0) return hipSuccess;
    if ((ns != 2 && ns != 3) || nP > 65535) return hipErrorInvalidValue;
    const long nto = (o + 63) / 64;
    dim3 grid((unsigned)(3 * nto), (unsigned)(3 * nto + 1), (unsigned)nP);
    if (ns == 2) hipLaunchKernelGGL(k_assemble3_planes<2>, grid, dim3(256), 0, st, g, Wt, o, ps);
    else hipLaunchKernelGGL(k_assemble3_planes<3>, grid, dim3(256), 0, st, g, Wt, o, ps);
    return hipGetLastError();
}

hipError_t pgemm(const PGemmArgs &g, hipStream_t st)
{
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
    if ((g.ns != 2 && g.ns != 3) || g.K <= 0 || g.K % BK2 || g.lda % 8 || g.ldb % 8 || g.lda < g.K ||
        g.ldb < g.K || g.psA % 8 || g.psB % 8 || g.sA % 8 || g.sB % 8 || !g.A || !g.B ||
        (reinterpret_cast<uintptr_t>(g.A) | reinterpret_cast<uintptr_t>(g.B)) % 16)
        return hipErrorInvalidValue;
    if (g.Cp ? (g.beta != 0.0 || g.lower || g.ldc < g.N || g.C) : !g.C) return hipErrorInvalidValue;
    if (g.sym2 && (g.Cp || g.beta != 0.0 || g.kband > 0 || g.M != g.N || g.lda != g.ldb))
        return hipErrorInvalidValue;
    if (g.kband > 0 && (g.lower || g.K != plane_ld(3L * g.kband))) return hipErrorInvalidValue;
    // 32-bit byte offsets of the rows from the operand base
    if (((long)(g.M - 1) * g.lda + g.K) * 2 >= (1L << 32) || ((long)(g.N - 1) * g.ldb + g.K) * 2 >= (1L << 32))
        return hipErrorInvalidValue;
    const int tm = (g.M + BM - 1) / BM;
    int tn = (g.N + BN - 1) / BN;
    if (g.Cp) tn = (int)((g.ldc + BN - 1) / BN);  // the padding columns are written too
    if (g.lower && g.M != g.N) return hipErrorInvalidValue;
    long total = g.lower ? (long)tm * (tm + 1) / 2 * g.batch : (long)tm * tn * g.batch;
    if (g.tiles) {
        if (!g.lower || g.ntiles <= 0) return hipErrorInvalidValue;
        tn = g.ntiles;
        total = (long)g.ntiles * g.batch;
    }
    if (total > 0x7fffffffL) return hipErrorInvalidValue;
    dim3 grid((unsigned)total);
#define RIS_PG_LAUNCH(NS_, OUTP_, BETA_, SYM2_) \
    hipLaunchKernelGGL((k_pgemm<NS_, OUTP_, BETA_, SYM2_>), grid, dim3(256), 0, st, g, tm, tn, (int)total)
    if (g.ns == 2) {
        if (g.Cp) RIS_PG_LAUNCH(2, true, false, false);
        else if (g.sym2) RIS_PG_LAUNCH(2, false, false, true);
        else if (g.beta != 0.0) RIS_PG_LAUNCH(2, false, true, false);
        else RIS_PG_LAUNCH(2, false, false, false);
    } else {
        if (g.Cp) RIS_PG_LAUNCH(3, true, false, false);
        else if (g.sym2) RIS_PG_LAUNCH(3, false, false, true);
        else if (g.beta != 0.0) RIS_PG_LAUNCH(3, false, true, false);
        else RIS_PG_LAUNCH(3, false, false, false);
    }
#undef RIS_PG_LAUNCH
    return hipGetLastError();
}

hipError_t split_planes(const double *x, int rows, int cols, long ldx, long sx, int batch, uint16_t *dst, long ps,
                        long sdst, int ns, hipStream_t st)
{
    if (rows <= 0 || cols <= 0 || batch <= 0) return hipSuccess;
    if ((ns != 2 && ns != 3) || batch > 65535) return hipErrorInvalidValue;
    const long ldp = plane_ld(cols);
    const long n = (long)rows * ldp;
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)batch);
    if (ns == 2)
        hipLaunchKernelGGL(k_split_planes<2>, grid, dim3(256), 0, st, x, rows, cols, ldx, sx, dst, ps, sdst, ldp);
    else
        hipLaunchKernelGGL(k_split_planes<3>, grid, dim3(256), 0, st, x, rows, cols, ldx, sx, dst, ps, sdst, ldp);
    return hipGetLastError();
}

// Split-BF16 product (ns = 2 parts: mode 2, ns = 3: mode 3); kc > 0: split-K
// ranges (kc a multiple of 32).
template <int NS>
static hipError_t bgemm_ns(const GemmArgs &g, int kc, hipStream_t st)
{
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
    if (g.kband > 0) {  // banded K (see GemmArgs), carried as kc = -kband
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
    // 32-bit offsets from a panel base; k-fast operands with rows too long for
    // a full tile are issued in row (column) slices
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
            const hipError_t e = bgemm_ns<NS>(s, kc, st);
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
            const hipError_t e = bgemm_ns<NS>(s, kc, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    const long spanA = g.transA ? (BK2 - 1) * g.lda + g.M : (std::min<long>(BM, g.M) - 1) * g.lda + g.K;
    const long spanB = g.transB ? (std::min<long>(BN, g.N) - 1) * g.ldb + g.K : (BK2 - 1) * g.ldb + g.N;
    if (!fits(spanA) || !fits(spanB)) return hipErrorInvalidValue;
    dim3 grid((unsigned)total);
    const int nred = g.nred > 0 ? g.nred : 1;
    if (g.ftypes != 0) {
        // FP32-stored operands: Y = F_I W (float in, float out) and Gamma
        // from float Y and F_J (double out, BETA for the second NAC half)
        if (kc > 0) return hipErrorInvalidValue;
        if (g.ftypes == (kF32A | kF32B | kF32C) && !g.transA && !g.transB && g.beta == 0.0)
            hipLaunchKernelGGL((k_bgemm3<NS, false, false, false, float, float, float>), grid, dim3(256), 0, st, g.M, g.N,
                               g.K, g.alpha, (const float *)g.A, g.lda, g.strideA, g.strideAr, (const float *)g.B, g.ldb,
                               g.strideB, g.strideBr, g.beta, (float *)g.C, g.ldc, g.strideC, nred, tm, tn, (int)total,
                               kc, g.lower, g.tiles);
        else if (g.ftypes == (kF32A | kF32B) && !g.transA && g.transB && g.beta == 0.0)
            hipLaunchKernelGGL((k_bgemm3<NS, false, true, false, float, float, double>), grid, dim3(256), 0, st, g.M, g.N,
                               g.K, g.alpha, (const float *)g.A, g.lda, g.strideA, g.strideAr, (const float *)g.B, g.ldb,
                               g.strideB, g.strideBr, g.beta, g.C, g.ldc, g.strideC, nred, tm, tn, (int)total, kc,
                               g.lower, g.tiles);
        else if (g.ftypes == (kF32A | kF32B) && !g.transA && g.transB)
            hipLaunchKernelGGL((k_bgemm3<NS, false, true, true, float, float, double>), grid, dim3(256), 0, st, g.M, g.N,
                               g.K, g.alpha, (const float *)g.A, g.lda, g.strideA, g.strideAr, (const float *)g.B, g.ldb,
                               g.strideB, g.strideBr, g.beta, g.C, g.ldc, g.strideC, nred, tm, tn, (int)total, kc,
                               g.lower, g.tiles);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
#define RIS_B3_LAUNCH1(TA, TB, BETA)                                                                               \
    hipLaunchKernelGGL((k_bgemm3<NS, TA, TB, BETA>), grid, dim3(256), 0, st, g.M, g.N, g.K, g.alpha, g.A, g.lda,        \
                       g.strideA, g.strideAr, g.B, g.ldb, g.strideB, g.strideBr, g.beta, g.C, g.ldc, g.strideC,     \
                       nred, tm, tn, (int)total, kc, g.lower, g.tiles);
#define RIS_B3_LAUNCH2(TA, TB)                                                                                     \
    if (g.beta != 0.0) { RIS_B3_LAUNCH1(TA, TB, true) } else { RIS_B3_LAUNCH1(TA, TB, false) }
    if (!g.transA && !g.transB) { RIS_B3_LAUNCH2(false, false) }
    else if (g.transA && !g.transB) { RIS_B3_LAUNCH2(true, false) }
    else if (!g.transA && g.transB) { RIS_B3_LAUNCH2(false, true) }
    else { RIS_B3_LAUNCH2(true, true) }
#undef RIS_B3_LAUNCH2
#undef RIS_B3_LAUNCH1
    return hipGetLastError();
}

hipError_t bgemm_kc(const GemmArgs &g, int kc, hipStream_t st, int nparts)
{
    if (nparts == 2) return bgemm_ns<2>(g, kc, st);
    if (nparts == 3) return bgemm_ns<3>(g, kc, st);
    return hipErrorInvalidValue;
}

hipError_t gemm_mp(const GemmArgs &g, int mode, hipStream_t st)
{
    if (mode == 0 || mode == 1) return gemm_kc(g, mode, 0, st);
    if (mode != 2 && mode != 3) return hipErrorInvalidValue;
    return bgemm_kc(g, 0, st, mode == 2 ? 2 : 3);
}

}  // namespace ris

extern "C" int ris_test_gemm(int mode, int M, int N, int K, int transA, int transB, double alpha, const double *A,
                             long lda, long sA, const double *B, long ldb, long sB, double beta, double *C, long ldc,
                             long sC, int batch)
{
    if (M < 0 || N < 0 || K < 0 || batch < 0 || !A || !B || !C || mode < 0 || mode > 3) return 1;
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

namespace ris {
namespace {
// sum of the ns parts of each plane element back into FP64 (test entry only)
__global__ void k_planes_sum(const uint16_t *__restrict__ P, long ps, int ns, int rows, int cols, long ldp,
                             double *__restrict__ C, long ldc)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)rows * cols) return;
    const int r = (int)(idx / cols), cidx = (int)(idx - (long)r * cols);
    double v = 0.0;
    for (int p = 0; p < ns; ++p)
        v += (double)(float)__builtin_bit_cast(__bf16, P[p * ps + (long)r * ldp + cidx]);
    C[(long)r * ldc + cidx] = v;
}
}  // namespace
}  // namespace ris

extern "C" int ris_test_pgemm(int ns, int M, int N, int K, double alpha, const double *A, long lda, const double *B,
                              long ldb, double beta, double *C, long ldc, int kband, int lower, int out_planes,
                              int sym2)
{
    using namespace ris;
    if ((ns != 2 && ns != 3) || M <= 0 || N <= 0 || K <= 0 || !A || !B || !C || lda < K || ldb < K || ldc < N ||
        (kband > 0 && K != 3 * kband) || (lower && (M != N || out_planes)) || (out_planes && beta != 0.0) ||
        (sym2 && (M != N || out_planes || beta != 0.0 || kband > 0)))
        return 1;
    const long ldp = plane_ld(K), psa = (long)M * ldp, psb = (long)N * ldp, ldcp = plane_ld(N);
    uint16_t *pa = nullptr, *pb = nullptr, *pc = nullptr;
    int rc = 0;
    if (hipMalloc((void **)&pa, 2 * psa * ns) != hipSuccess || hipMalloc((void **)&pb, 2 * psb * ns) != hipSuccess ||
        (out_planes && hipMalloc((void **)&pc, 2 * (long)M * ldcp * ns) != hipSuccess))
        rc = 7;
    if (!rc && (split_planes(A, M, K, lda, 0, 1, pa, psa, 0, ns, 0) != hipSuccess ||
                split_planes(B, N, K, ldb, 0, 1, pb, psb, 0, ns, 0) != hipSuccess))
        rc = 7;
    if (!rc) {
        PGemmArgs g{};
        g.M = M; g.N = N; g.K = (int)ldp; g.ns = ns;
        g.A = pa; g.lda = ldp; g.psA = psa;
        g.B = pb; g.ldb = ldp; g.psB = psb;
        g.alpha = alpha; g.beta = beta;
        if (out_planes) {
            g.Cp = pc; g.ldc = ldcp; g.psC = (long)M * ldcp;
        } else {
            g.C = C; g.ldc = ldc;
        }
        g.batch = 1; g.kband = kband; g.lower = lower != 0; g.sym2 = sym2 != 0;
        const hipError_t e = pgemm(g, 0);
        if (e == hipErrorInvalidValue) rc = 1;
        else if (e != hipSuccess) rc = 7;
    }
    if (!rc && out_planes) {
        hipLaunchKernelGGL(k_planes_sum, dim3((unsigned)(((long)M * N + 255) / 256)), dim3(256), 0, 0, pc,
                           (long)M * ldcp, ns, M, N, ldcp, C, ldc);
        if (hipGetLastError() != hipSuccess) rc = 7;
    }
    if (hipDeviceSynchronize() != hipSuccess && !rc) rc = 7;
    if (pa) (void)hipFree(pa);
    if (pb) (void)hipFree(pb);
    if (pc) (void)hipFree(pc);
    return rc;
}
