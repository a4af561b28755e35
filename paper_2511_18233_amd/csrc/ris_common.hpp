// Internal declarations shared by the gfx950 kernels and the host library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ris {

constexpr int kMaxAOL = 2;   // AO shells up to d (Cartesian)
constexpr int kMaxAuxL = 1;  // auxiliary shells up to p
// AO shell pairs whose Gaussian product prefactor is below this are skipped
// in the derivative contraction (their integrals and derivatives are below
// roundoff of the kept terms)
constexpr double kDefaultScreen = 1e-15;

__host__ __device__ constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }

// Shell table in structure-of-arrays form (device pointers).
struct ShellTab {
    const double *x, *y, *z;  // centre
    const double *exp;        // exponent
    const double *nrm;        // radial normalisation (2a/pi)^{3/4} (4a)^{l/2}
    const int *atom;          // atom index
    const int *off;           // first function index of the shell
};

// --- Boys function table: F_m(T_k) on T_k = k / kBoysInvStep, k <= kBoysNGrid-1
constexpr int kBoysMaxM = 7;       // highest order needed by any kernel
constexpr int kBoysTaylor = 8;     // Taylor terms (orders kept: 0..kBoysTaylor-1)
constexpr int kBoysCols = kBoysMaxM + kBoysTaylor;  // stored orders 0..kBoysCols-1
constexpr double kBoysInvStep = 16.0;
constexpr double kBoysTMax = 40.0;
constexpr int kBoysNGrid = 641;    // 40 * 16 + 1

// Host: fill tab[k * kBoysCols + m] = F_m(k / 16) (long-double series).
void boys_table_host(double *tab);

// --- kernels launched from the host library (ris_ints.hip / ris_linalg.hip)
struct AuxGeom {
    ShellTab sh;
    int nshell;
    int nfunc;
};

// (P|Q) metric over the auxiliary set, full square [n][n].
hipError_t launch_int2c(const AuxGeom &aux, const double *boys, double *M, hipStream_t st);

// (mu nu|P): X[P][mu][nu] (internal AO order), all J auxiliary shells.
struct AOGeom {
    ShellTab sh;
    int nshell;
    int nao;
    int lbeg[kMaxAOL + 2];  // shells sorted by l: shells of l are [lbeg[l], lbeg[l+1])
};
// With an aux shell range [cs0, cs1) (cs1 < 0: to the last shell) only those
// shells are computed and X row 0 is the first function of shell cs0.
hipError_t launch_int3c(const AOGeom &ao, const AuxGeom &aux, int auxl_beg[kMaxAuxL + 2],
                        const double *boys, double *X, hipStream_t st, int cs0 = 0, int cs1 = -1);

// Fused three-centre derivative contraction (see ris_ints.hip).
struct DerivJob {
    int nout;                  // outputs in this launch (<= kMaxOutChunk)
    const double *gammaK;      // [nout][nK][nao][nao] symmetric K weights (lower triangle read), may be null
    int nK;                    // K functions held by gammaK: J functions [kbeg, kbeg + nK)
    int kbeg;                  // (the K set is the leading s functions of the J set)
    const double *dens;        // [nstate][nao][nao] symmetric AO densities R^S
    const double *cvec;        // [nstate][nJ] c_I = M_J^-1 t_I
    int nJ;
    int stI[8], stJ[8];        // state pair of each output
    double alphaJ;
    double *partial;           // [nshellAO][nshellAux][3][kMaxOutChunk][6] (dA xyz, dC xyz); slots o < nout written
    // AO shell-pair screen (null: every pair): the partners of internal shell sa
    // in class l are pair_idx[pair_ptr[(kMaxAOL+1) sa + l] .. pair_ptr[(kMaxAOL+1) sa + l + 1])
    const int *pair_ptr;
    const int *pair_idx;
    // Optional compact copy of the s-shell weights (null: gammaK and the
    // densities are read in place).  With it, the s-shell classes of the K
    // block run on a second kernel (lanes over the K functions) that reads
    // only the copy.  Layout Gc[o][q][k], k < nK fastest, q = the
    // function pair inside the block of its unordered kept shell pair
    // (nfq function pairs in all, see launch_pack_gamma).  lst_ptr / lst_idx are the
    // partner lists in pair_ptr / pair_idx form (always given, every pair when
    // nothing is screened) and lst_gq[e] = base << 1 | flip for list entry e:
    // the pair's block starts at q = base and is stored with the partner's
    // functions first when flip is set.
    const double *gcomp;
    long nfq;
    const int *lst_ptr;
    const int *lst_idx;
    const int *lst_gq;
};
constexpr int kMaxOutChunk = 4;
// Gc[o][base + ka nb + kb][k] = W_o^k[mu0 + ka][nu0 + kb] for o < nout and
// every unordered kept AO shell pair (a, b) whose b starts at or before a
// (the diagonal block taken from the lower triangle), base = the pair's block
// start, W_o^k = gammaK_o^k + alphaJ (D_I c_J[k] + D_J c_I[k]) the whole weight
// of the s-shell triplets (symmetric).  gammaK: [nout][nK][nao][nao], only the
// lower blocks of kept pairs are read.  The lists (device, built with the pair
// lists):
struct PackLists {
    // pk_ptr[a] .. pk_ptr[a + 1]: a's partners b starting at or before a, by
    // first function (a itself last); pk_base: their block starts
    const int *pk_ptr, *pk_base;
    // pc_ptr[a] .. pc_ptr[a + 1]: the columns of those partners other than a,
    // in order; pc_cn = column * 8 + the partner's function count, pc_qb =
    // block start + the column's index in the partner
    const int *pc_ptr, *pc_cn, *pc_qb;
};
// Fills job.gcomp from job.gammaK (job.nout outputs, job.nK K functions from
// J function job.kbeg), the densities and Coulomb vectors of the job's states.
hipError_t launch_pack_gamma(const AOGeom &ao, const DerivJob &job, const PackLists &pl, hipStream_t st);
// Only the aux shells in [cs0, cs1) (cs1 < 0: to the last shell); partial
// slots of the other shells are left untouched.
hipError_t launch_int3c_deriv(const AOGeom &ao, const AuxGeom &aux, int auxl_beg[kMaxAuxL + 2],
                              const double *boys, const DerivJob &job, hipStream_t st, int cs0 = 0, int cs1 = -1);

// 2c metric derivative contraction: partial2[P shell][out][3] for d/dP.
hipError_t launch_int2c_deriv(const AuxGeom &aux, const double *boys, int nout,
                              const double *W /*[nout][n][n]*/, double *partial2, hipStream_t st);

// Batched / batch-reduced FP64 GEMM on the matrix cores (ris_gemm.hip):
// for b < batch: C_b = alpha * sum_{r < nred} op(A_{b,r}) op(B_{b,r}) + beta * C_b,
// row-major; op(A) is M x K (A stored K x M when transA), op(B) is K x N.
struct GemmArgs {
    int M, N, K;
    bool transA, transB;
    double alpha, beta;
    const double *A;
    long lda, strideA, strideAr;
    const double *B;
    long ldb, strideB, strideBr;
    double *C;
    long ldc, strideC;
    int batch, nred;
    bool lower;  // M == N: compute only the 128 x 128 tiles on or below the diagonal
    // bits kF32A / kF32B / kF32C: that operand is stored as float (FP32 mode only;
    // supported: A, B, C float with no transposes, or A, B float with B transposed)
    int ftypes;
    // kband = w > 0 (K = 3w, B untransposed, no split-K): B's rows and columns
    // are three blocks of w and B is zero in its (3rd row, 1st column) and
    // (1st row, 3rd column) blocks, so a column tile inside the first block
    // reads rows [0, 2w) and one inside the third block rows [w, 3w)
    int kband;
    // lower mode only: compute just these tiles (mt << 16 | nt, mt >= nt; device
    // array of ntiles) of every batch entry instead of all lower tiles
    const int *tiles;
    int ntiles;
};
constexpr int kF32A = 1, kF32B = 2, kF32C = 4;
hipError_t dgemm(const GemmArgs &g, hipStream_t st);
// Same product with K cut into nsplit ranges (batch == 1, nred == 1): partials
// go to ws (nsplit * M * N doubles) and are summed in a fixed order.
hipError_t dgemm_splitk(const GemmArgs &g, int nsplit, double *ws, hipStream_t st);
// Same for every mode of gemm_mp (partials in FP64, summed in a fixed order).
hipError_t gemm_splitk(const GemmArgs &g, int mode, int nsplit, double *ws, hipStream_t st);
// K-split count in [1, smax] that fills whole waves of workgroups best for a
// product of `tiles` 128 x 128 output tiles (1 for large tile counts).
int balanced_splits(long tiles, int smax);
// Same contract with the products on reduced-precision matrix cores (FP64 in
// and out, FP32 accumulation): mode 0 = FP64 (dgemm), 1 = FP32, 2 = split BF16
// with three products, 3 = split BF16 with six products (ris_gemm_mp.hip).
hipError_t gemm_mp(const GemmArgs &g, int mode, hipStream_t st);
// The split-BF16 product alone (nparts 2: three products, 3: six); kc > 0:
// split-K ranges of kc (a multiple of 32).
hipError_t bgemm_kc(const GemmArgs &g, int kc, hipStream_t st, int nparts = 2);
// The matrix-core GEMM itself for mode 0 (FP64) or 1 (FP32); kc > 0 splits K
// into ranges of kc indexed by the batch (ris_gemm.hip).
hipError_t gemm_kc(const GemmArgs &g, int mode, int kc, hipStream_t st);

// Split-BF16 operands kept pre-split ("planes"): the FP32 value x32 of every
// element as ns bf16 parts (ns = 2: hi, lo; ns = 3: hi, mid, lo; the parts of
// the split-BF16 GEMM), part p of a rows x cols matrix at base + p * ps, each
// part rows x plane_ld(cols) with the padding columns zero (the width padded
// to whole k-slabs of 32).
constexpr long plane_ld(long cols) { return (cols + 31) & ~31L; }
// C_b = alpha * A_b B_b^T (+ beta * C_b) for b < batch with both operands
// k-fast planes: A_b M x K, B_b N x K (K a multiple of 32, the padded width).
// Output either FP64 (C, ldc, sC) or, with Cp set, planes of the FP32
// product (Cp, ldc, psC, sC; columns [N, ldc) written zero; beta 0).
// kband = w > 0: B's rows and K are three blocks of w with B zero in its
// (1st row, 3rd k) and (3rd row, 1st k) blocks (see GemmArgs).
struct PGemmArgs {
    int M, N, K, ns;
    const uint16_t *A;
    long lda, psA, sA;
    const uint16_t *B;
    long ldb, psB, sB;
    double alpha, beta;
    double *C;
    uint16_t *Cp;
    long ldc, psC, sC;
    int batch, kband;
    bool lower;
    const int *tiles;
    int ntiles;
    // C = alpha (A B^T + B A^T) (FP64 C, beta 0, M == N, lda == ldb, no band)
    bool sym2;
};
hipError_t pgemm(const PGemmArgs &g, hipStream_t st);
// Planes (ns parts, leading dimension plane_ld(cols), parts ps apart) of the
// batch x rows x cols FP64 matrices x (leading dimension ldx, batch stride sx)
// into dst (batch stride sdst).
hipError_t split_planes(const double *x, int rows, int cols, long ldx, long sx, int batch, uint16_t *dst, long ps,
                        long sdst, int ns, hipStream_t st);

// Dense linear algebra on small matrices (ris_linalg.hip).
// In-place Cholesky of the n x n SPD matrix (lower triangle written, upper
// zeroed); *info (device int) = 0 or the 1-based failing column.  A pivot
// below 1e-13 of Morig's diagonal (the unfactored matrix, may be null) fails.
hipError_t cholesky(double *A, const double *Morig, int n, int *info, hipStream_t st);
// Linv = L^-1 for lower-triangular L (n x n), full matrix written.
// Blocks of kTriBlock rows: diagonal blocks by substitution, the rest by GEMMs;
// tmp holds kTriBlock * n doubles.
constexpr int kTriBlock = 64;
hipError_t tri_inverse(const double *L, double *Linv, int n, double *tmp, hipStream_t st);

}  // namespace ris
