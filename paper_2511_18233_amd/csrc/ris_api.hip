// Host side of the TDDFT-ris hot path: context, device-resident state and the
// five entry points declared in include/ris.h.  Every arithmetic step runs in
// the gfx950 kernels of ris_ints.hip, ris_gemm.hip and ris_linalg.hip on the
// context's stream; this file only sizes buffers, builds shell tables and
// sequences launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <cstdio>
#include <cstdarg>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ris.h"
#include "ris_common.hpp"
#include "ris_linalg.hpp"
#include "ris_minres.hpp"

using namespace ris;

// Fixed device scratch of ris_response_matvec_noalloc (128 MiB).  Each device
// that loads the library holds its own copy until the process ends; host code
// reaches it only through the address hipGetSymbolAddress returns on that
// device (the array's name on the host is a stand-in, not a device address).
static __device__ __align__(256) char scratch[(size_t)128 << 20];

namespace {

constexpr size_t kNoAllocScratchBytes = sizeof(scratch);
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (resolved once per device).
hipError_t scratch_address(int device, void **out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct ris_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    size_t budget = 0;
    size_t held = 0;
    std::string err;
    std::vector<DevBuf> bufs;

    double *boys = nullptr;  // Boys table
    int *info = nullptr;     // Cholesky status (device)
    void *scratch_dev = nullptr;  // this device's fixed scratch (ris_response_matvec_noalloc)

    // ---- aux_build state
    bool have_aux = false;
    int natm = 0, nao = 0, nshAO = 0;
    int nJ = 0, nK = 0, nshJ = 0, nsJ = 0;  // J functions, K functions, J shells, J s-shells
    std::vector<int> h_ao_perm;             // internal AO function -> caller AO function
    std::vector<int> h_ao_atom, h_aux_atom;
    std::vector<int> h_aux_off;             // first J function of each J shell (+ total)
    AOGeom ao{};
    AuxGeom aux{};
    int auxl_beg[kMaxAuxL + 2] = {0, 0, 0};
    int *d_ao_perm = nullptr;
    // the forward integrals of ris_int3c and their MO transforms use a second
    // AO order, the kernels' shell order (by l), so (mu nu|P) rows are written
    // in whole runs; the result is in the MO basis, so only C's rows follow it
    AOGeom ao_int{};
    std::vector<int> h_ao_perm_int;  // integral-order function -> caller function
    int *d_ao_perm_int = nullptr;
    double *MJ = nullptr, *LinvJ = nullptr, *MinvJ = nullptr, *MinvK = nullptr;
    // AO shell-pair screen of the derivative contraction (internal shell order)
    double screen = kDefaultScreen;
    std::vector<double> h_sh_xyz, h_sh_exp;  // [nsh][3], [nsh]
    int *d_pair_ptr = nullptr, *d_pair_idx = nullptr;
    long npair_kept = 0;
    // the 128 x 128 lower tiles of an AO-pair matrix that hold a kept shell
    // pair (mt << 16 | nt): the exchange weights Gamma^P are formed only there
    std::vector<int> h_sh_off;  // first AO function of each internal shell (+ total)
    int *d_gtiles = nullptr;     // lower tiles row by row, then the same tiles column by column
    int *d_gtiles_cm = nullptr;
    int ngtiles = 0;
    double gtile_lower = 0.0;  // elements on or below the diagonal inside those tiles
    // numbering of the compact copy of the exchange weights read by the
    // derivative contraction (build_pairs): block start and orientation per
    // partner-list entry, the lower partners of each shell with their block
    // starts, and the function pairs of all blocks (0: no copy, the weights
    // are read in place)
    int *d_pair_gq = nullptr, *d_pk_ptr = nullptr, *d_pk_sb = nullptr, *d_pk_base = nullptr;
    int *d_pc_ptr = nullptr, *d_pc_cn = nullptr, *d_pc_qb = nullptr;  // the copy's column lists (PackLists)
    long nfq = 0;

    // ---- int3c state
    bool have_int3c = false;
    int nmo = 0, nocc = 0, nvir = 0;
    double alphaJ = 2.0, cx = 0.25;
    int prec = RIS_FP64;  // arithmetic of the exchange-weight contractions
    int prec_tr = RIS_FP64;  // arithmetic of the MO transforms of (mu nu|P)
    double *C = nullptr;    // [nao][nmo] internal AO order
    double *eps = nullptr;  // [nmo]
    double *aiJ = nullptr;   // [nJ][v][o]  raw (ai|P), Coulomb set
    double *coo = nullptr;   // [nK][o][o]  c^P_ij = sum_Q (M_K^-1)_PQ (ij|Q)
    double *cvo = nullptr;   // [v][nK][o]  c^P_aj
    double *cvv = nullptr;   // [v][nK][v]  c^P_ab
    double *roo = nullptr;   // [nK][o][o]  raw (ij|P), exchange set
    int ablock = 0;          // auxiliary functions per block (0: as many as fit)

    // ---- grow-only device regions; after warm-up a request of the same or a
    // smaller size allocates nothing (hipFree would synchronise the device)
    struct Pool {
        void *p = nullptr;
        size_t bytes = 0;
    };
    Pool aux_pool;    // shell tables, permutation, metric and its inverses
    Pool mo_pool;     // orbitals and the MO blocks kept between calls
    Pool out_pool;    // staging of combined gradient + NAC outputs
    Pool zv_pool;     // vectors of the Z-vector solve (the matvec uses the scratch below)
    Pool dv_pool;     // subspace of the TDA Davidson solve
    void *ws = nullptr;  // scratch shared by the calls
    size_t ws_bytes = 0;

    // ---- optional per-stage timing
    struct Mark {
        int stage;
        hipEvent_t a, b;
        double flops, bytes;
    };
    bool prof = false;
    std::vector<Mark> marks;
    std::vector<hipEvent_t> event_pool;
};

namespace {

int fail(ris_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(ctx, expr)                                                                                  \
    do {                                                                                                   \
        hipError_t e_ = (expr);                                                                            \
        if (e_ != hipSuccess) return fail(ctx, RIS_E_DEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                          __FILE__, __LINE__);                                             \
    } while (0)

void *dalloc(ris_ctx *c, size_t bytes, int *st)
{
    *st = RIS_OK;
    if (bytes == 0) bytes = 8;
    if (c->held + bytes > c->budget) {
        *st = fail(c, RIS_E_NOMEM, "allocation of %zu bytes exceeds the HBM budget (%zu of %zu held)", bytes, c->held,
                   c->budget);
        return nullptr;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        *st = fail(c, RIS_E_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
        return nullptr;
    }
    c->held += bytes;
    c->bufs.push_back({p, bytes});
    return p;
}

void dfree(ris_ctx *c, void *p)
{
    if (!p) return;
    for (size_t i = 0; i < c->bufs.size(); ++i)
        if (c->bufs[i].p == p) {
            (void)hipStreamSynchronize(c->stream);
            (void)hipFree(p);
            c->held -= c->bufs[i].bytes;
            c->bufs.erase(c->bufs.begin() + i);
            return;
        }
}

// Region of at least `bytes` (grow-only; contents not preserved when it grows).
char *pool_get(ris_ctx *c, ris_ctx::Pool &pl, size_t bytes, int *st)
{
    *st = RIS_OK;
    if (bytes <= pl.bytes) return (char *)pl.p;
    dfree(c, pl.p);
    pl.p = nullptr;
    pl.bytes = 0;
    pl.p = dalloc(c, bytes, st);
    if (pl.p) pl.bytes = bytes;
    return (char *)pl.p;
}

// Scratch of at least `bytes` shared by all calls of the context.
char *ws_get(ris_ctx *c, size_t bytes, int *st)
{
    ris_ctx::Pool pl{c->ws, c->ws_bytes};
    char *p = pool_get(c, pl, bytes, st);
    c->ws = pl.p;
    c->ws_bytes = pl.bytes;
    return p;
}

// carve consecutive 256-byte aligned pieces out of a scratch block
struct Carve {
    size_t off = 0;
    size_t take(size_t elems)
    {
        const size_t o = off;
        off += (elems * 8 + 255) / 256 * 256;
        return o;
    }
};

void free_int3c(ris_ctx *c)
{
    c->have_int3c = false;
    c->C = c->eps = c->aiJ = c->coo = c->cvo = c->cvv = c->roo = nullptr;
}

void free_aux(ris_ctx *c)
{
    free_int3c(c);
    c->d_ao_perm = nullptr;
    c->d_ao_perm_int = nullptr;
    c->ao_int = AOGeom{};
    c->d_pair_ptr = c->d_pair_idx = nullptr;
    c->d_gtiles = c->d_gtiles_cm = nullptr;
    c->ngtiles = 0;
    c->d_pair_gq = c->d_pk_ptr = c->d_pk_sb = c->d_pk_base = nullptr;
    c->d_pc_ptr = c->d_pc_cn = c->d_pc_qb = nullptr;
    c->nfq = 0;
    c->MJ = c->LinvJ = c->MinvJ = c->MinvK = nullptr;
    c->ao = AOGeom{};
    c->aux = AuxGeom{};
    c->have_aux = false;
}

hipEvent_t get_event(ris_ctx *c)
{
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// Bracket a launch group with events when profiling is on:
//   hipEvent_t t = stage_begin(c); ...launches...; stage_end(c, t, stage, flops, bytes);
hipEvent_t stage_begin(ris_ctx *c)
{
    if (!c->prof) return nullptr;
    hipEvent_t a = get_event(c);
    (void)hipEventRecord(a, c->stream);
    return a;
}

void stage_end(ris_ctx *c, hipEvent_t a, int stage, double flops, double bytes)
{
    if (!a) return;
    hipEvent_t b = get_event(c);
    (void)hipEventRecord(b, c->stream);
    c->marks.push_back({stage, a, b, flops, bytes});
}

void release_marks(ris_ctx *c)
{
    for (auto &m : c->marks) {
        c->event_pool.push_back(m.a);
        c->event_pool.push_back(m.b);
    }
    c->marks.clear();
}

// Shell table: 5 double arrays + 2 int arrays, bytes needed and upload into dst.
size_t shell_bytes(int n) { return ((size_t)5 * n * 8 + ((size_t)2 * n + 1) * 4 + 255) / 256 * 256; }

int upload_shells(ris_ctx *c, int n, const std::vector<double> &x, const std::vector<double> &y,
                  const std::vector<double> &z, const std::vector<double> &e, const std::vector<double> &nrm,
                  const std::vector<int> &atom, const std::vector<int> &off, char *base, ShellTab *out)
{
    const size_t nd = (size_t)5 * n, ni = (size_t)2 * n + 1;
    std::vector<char> h(nd * 8 + ni * 4);
    double *hd = (double *)h.data();
    memcpy(hd + 0 * n, x.data(), 8 * n);
    memcpy(hd + 1 * n, y.data(), 8 * n);
    memcpy(hd + 2 * n, z.data(), 8 * n);
    memcpy(hd + 3 * n, e.data(), 8 * n);
    memcpy(hd + 4 * n, nrm.data(), 8 * n);
    int *hi = (int *)(hd + nd);
    memcpy(hi, atom.data(), 4 * n);
    memcpy(hi + n, off.data(), 4 * (n + 1));
    HIPCHK(c, hipMemcpyAsync(base, h.data(), h.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const double *d = (const double *)base;
    out->x = d;
    out->y = d + n;
    out->z = d + 2 * n;
    out->exp = d + 3 * n;
    out->nrm = d + 4 * n;
    out->atom = (const int *)(d + nd);
    out->off = out->atom + n;
    return RIS_OK;
}

double radial_norm(double a, int l) { return std::pow(2.0 * a / M_PI, 0.75) * std::pow(4.0 * a, 0.5 * l); }

// plain GEMM helper (no batching)
GemmArgs gm(int M, int N, int K, bool tA, bool tB, double alpha, const double *A, long lda, const double *B, long ldb,
            double beta, double *C, long ldc)
{
    GemmArgs g{};
    g.M = M; g.N = N; g.K = K;
    g.transA = tA; g.transB = tB;
    g.alpha = alpha; g.beta = beta;
    g.A = A; g.lda = lda;
    g.B = B; g.ldb = ldb;
    g.C = C; g.ldc = ldc;
    g.batch = 1; g.nred = 1;
    return g;
}

// The screen's test for an AO shell pair of exponents ea, eb at squared distance r2.
bool pair_kept(double ea, double eb, double r2, double thr)
{
    return thr <= 0.0 || std::exp(-ea * eb / (ea + eb) * r2) >= thr;
}

// Partner lists of the AO shell-pair screen: pair (a, b) is kept when its
// Gaussian product prefactor exp(-a b / (a + b) |A - B|^2) is >= c->screen
// (every pair when the threshold is 0).  Lists are grouped by the partner's
// class so each derivative kernel reads the partners of its own class.
int build_pairs(ris_ctx *c)
{
    const int nsh = c->nshAO, ncls = kMaxAOL + 1;
    std::vector<int> ptr((size_t)ncls * nsh + 1, 0), idx;
    idx.reserve((size_t)nsh * 16);
    const double thr = c->screen;
    const double *X = c->h_sh_xyz.data(), *E = c->h_sh_exp.data();
    for (int a = 0; a < nsh; ++a)
        for (int l = 0; l < ncls; ++l) {
            ptr[(size_t)ncls * a + l] = (int)idx.size();
            for (int b = c->ao.lbeg[l]; b < c->ao.lbeg[l + 1]; ++b) {
                const double dx = X[3 * a] - X[3 * b], dy = X[3 * a + 1] - X[3 * b + 1], dz = X[3 * a + 2] - X[3 * b + 2];
                if (pair_kept(E[a], E[b], dx * dx + dy * dy + dz * dz, thr)) idx.push_back(b);
            }
        }
    ptr[(size_t)ncls * nsh] = (int)idx.size();
    c->npair_kept = (long)idx.size();
    // lower 128-tiles touched by a kept pair (the relation is symmetric)
    const int N = c->nao, T = 128, tm = (N + T - 1) / T;
    const std::vector<int> &off = c->h_sh_off;
    // functions of internal shell i: shells are sorted by l
    auto shell_nf = [&](int i) {
        int l = 0;
        while (i >= c->ao.lbeg[l + 1]) ++l;
        return ncart(l);
    };
    std::vector<char> mark((size_t)tm * tm, 0);
    for (int a = 0; a < nsh; ++a)
        for (size_t q = ptr[(size_t)ncls * a]; q < (size_t)ptr[(size_t)ncls * (a + 1)]; ++q) {
            const int b = idx[q];
            for (int ta = off[a] / T; ta <= (off[a] + shell_nf(a) - 1) / T; ++ta)
                for (int tb = off[b] / T; tb <= (off[b] + shell_nf(b) - 1) / T; ++tb)
                    mark[(size_t)std::max(ta, tb) * tm + std::min(ta, tb)] = 1;
        }
    std::vector<int> tiles;
    double lower = 0.0;
    for (int mt = 0; mt < tm; ++mt)
        for (int nt = 0; nt <= mt; ++nt)
            if (mark[(size_t)mt * tm + nt]) {
                tiles.push_back(mt << 16 | nt);
                const double rows = std::min(N, mt * T + T) - mt * T, cols = std::min(N, nt * T + T) - nt * T;
                lower += mt > nt ? rows * cols : rows * (rows + 1) / 2;
            }
    c->ngtiles = (int)tiles.size();
    c->gtile_lower = lower;
    // the same tiles column by column: launches whose per-P operand is B (the
    // second half of a NAC in the FP32 mode) then meet each of its row panels in
    // consecutive tiles
    std::vector<int> tiles_cm(tiles);
    std::stable_sort(tiles_cm.begin(), tiles_cm.end(), [](int a, int b) { return (a & 0xffff) < (b & 0xffff); });
    tiles.insert(tiles.end(), tiles_cm.begin(), tiles_cm.end());
    c->d_gtiles_cm = c->d_gtiles + c->ngtiles;
    // Compact copy of the exchange weights (the derivative contraction's
    // s-shell classes): each unordered kept pair owns one block of
    // nf(a) nf(b) function pairs, stored in the orientation whose first shell
    // starts later in the AO order (rows >= columns: the lower triangle the
    // weights are formed in), blocks ordered by that shell and then by the
    // partner's first function.  pk: those partners of each shell in that
    // order; gq[e] of list entry e = (a, b): block start << 1, | 1 when a is
    // the earlier shell (its functions then run second in the block).
    std::vector<int> pk_ptr((size_t)nsh + 1, 0), pk_sb, gq(idx.size());
    std::vector<long> pk_base;
    long nfq = 0;
    for (int a = 0; a < nsh; ++a) {
        pk_ptr[a] = (int)pk_sb.size();
        const size_t k0 = pk_sb.size();
        for (size_t q = ptr[(size_t)ncls * a]; q < (size_t)ptr[(size_t)ncls * (a + 1)]; ++q)
            if (off[idx[q]] <= off[a]) pk_sb.push_back(idx[q]);
        std::sort(pk_sb.begin() + k0, pk_sb.end(), [&](int x, int y) { return off[x] < off[y]; });
        for (size_t k = k0; k < pk_sb.size(); ++k) {
            pk_base.push_back(nfq);
            nfq += (long)shell_nf(a) * shell_nf(pk_sb[k]);
        }
    }
    pk_ptr[nsh] = (int)pk_sb.size();
    // block starts are stored as int with the orientation bit
    c->nfq = nfq < (1L << 30) ? nfq : 0;
    if (c->nfq > 0) {
        for (int a = 0; a < nsh; ++a)
            for (size_t q = ptr[(size_t)ncls * a]; q < (size_t)ptr[(size_t)ncls * (a + 1)]; ++q) {
                const int b = idx[q];
                const bool flip = off[a] < off[b];
                const int x = flip ? b : a, y = flip ? a : b;
                const auto beg = pk_sb.begin() + pk_ptr[x], end = pk_sb.begin() + pk_ptr[x + 1];
                const auto it = std::lower_bound(beg, end, y, [&](int s, int t) { return off[s] < off[t]; });
                if (it == end || *it != y) return fail(c, RIS_E_INVALID, "internal: shell-pair lists not symmetric");
                gq[q] = (int)(pk_base[it - pk_sb.begin()] << 1) | (flip ? 1 : 0);
            }
        std::vector<int> base32(pk_base.begin(), pk_base.end());
        // the columns of each shell's earlier partners (its own block apart)
        std::vector<int> pc_ptr((size_t)nsh + 1, 0), pc_cn, pc_qb;
        for (int a = 0; a < nsh; ++a) {
            pc_ptr[a] = (int)pc_cn.size();
            if (pk_ptr[a + 1] == pk_ptr[a] || pk_sb[pk_ptr[a + 1] - 1] != a)
                return fail(c, RIS_E_INVALID, "internal: shell %d is not its own last partner", a);
            for (int k = pk_ptr[a]; k < pk_ptr[a + 1] - 1; ++k) {
                const int b = pk_sb[k], nb = shell_nf(b);
                for (int kb = 0; kb < nb; ++kb) {
                    pc_cn.push_back((off[b] + kb) * 8 + nb);
                    pc_qb.push_back((int)(pk_base[k] + kb));
                }
            }
        }
        pc_ptr[nsh] = (int)pc_cn.size();
        HIPCHK(c, hipMemcpyAsync(c->d_pc_ptr, pc_ptr.data(), 4 * pc_ptr.size(), hipMemcpyHostToDevice, c->stream));
        if (!pc_cn.empty()) {
            HIPCHK(c, hipMemcpyAsync(c->d_pc_cn, pc_cn.data(), 4 * pc_cn.size(), hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(c->d_pc_qb, pc_qb.data(), 4 * pc_qb.size(), hipMemcpyHostToDevice, c->stream));
        }
        if (!gq.empty())
            HIPCHK(c, hipMemcpyAsync(c->d_pair_gq, gq.data(), 4 * gq.size(), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->d_pk_ptr, pk_ptr.data(), 4 * pk_ptr.size(), hipMemcpyHostToDevice, c->stream));
        if (!pk_sb.empty()) {
            HIPCHK(c, hipMemcpyAsync(c->d_pk_sb, pk_sb.data(), 4 * pk_sb.size(), hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(c->d_pk_base, base32.data(), 4 * base32.size(), hipMemcpyHostToDevice,
                                     c->stream));
        }
        // the copies read from host vectors: finish them before those go
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    HIPCHK(c, hipMemcpyAsync(c->d_pair_ptr, ptr.data(), 4 * ptr.size(), hipMemcpyHostToDevice, c->stream));
    if (!idx.empty())
        HIPCHK(c, hipMemcpyAsync(c->d_pair_idx, idx.data(), 4 * idx.size(), hipMemcpyHostToDevice, c->stream));
    if (!tiles.empty())
        HIPCHK(c, hipMemcpyAsync(c->d_gtiles, tiles.data(), 4 * tiles.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RIS_OK;
}

}  // namespace

// Reverse Cuthill-McKee order of the atoms on the graph that joins two atoms
// when the Gaussian product of their most diffuse shells, exp(-a b / (a + b)
// |A - B|^2), is at least 1e-15 (a fixed threshold: the order does not depend
// on the screen setting).  BFS from an unvisited atom of least degree,
// neighbours by increasing degree, then reversed: a narrow band for chains and
// other extended molecules.
static std::vector<int> atom_band_order(const ris_mol *mol)
{
    const int n = mol->natm;
    std::vector<double> amin(n, 1e300);
    for (int s = 0; s < mol->nshell; ++s) amin[mol->shell_atom[s]] = std::min(amin[mol->shell_atom[s]], mol->shell_exp[s]);
    std::vector<std::vector<int>> nb(n);
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            if (amin[i] > 1e299 || amin[j] > 1e299) continue;  // an atom without AO shells
            double r2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                const double t = mol->xyz[3 * i + d] - mol->xyz[3 * j + d];
                r2 += t * t;
            }
            if (std::exp(-amin[i] * amin[j] / (amin[i] + amin[j]) * r2) >= 1e-15) {
                nb[i].push_back(j);
                nb[j].push_back(i);
            }
        }
    std::vector<int> deg(n);
    for (int i = 0; i < n; ++i) deg[i] = (int)nb[i].size();
    auto by_degree = [&](int a, int b) { return deg[a] != deg[b] ? deg[a] < deg[b] : a < b; };
    for (auto &v : nb) std::sort(v.begin(), v.end(), by_degree);
    std::vector<int> out;
    out.reserve(n);
    std::vector<char> seen(n, 0);
    while ((int)out.size() < n) {
        int start = -1;
        for (int i = 0; i < n; ++i)
            if (!seen[i] && (start < 0 || by_degree(i, start))) start = i;
        size_t head = out.size();
        out.push_back(start);
        seen[start] = 1;
        while (head < out.size()) {
            const int u = out[head++];
            for (int w : nb[u])
                if (!seen[w]) {
                    seen[w] = 1;
                    out.push_back(w);
                }
        }
    }
    std::reverse(out.begin(), out.end());
    return out;
}

// ---- sizes of every device region, shared by the calls and ris_request_bytes
struct Dims {
    int N, nmo, o, v, nJ, nK, nshAO, nshJ, natm;
    long nfq;  // function pairs of the compact exchange-weight copy (0: none)
};

struct MoLayout {
    size_t oC, oCI, oE, oA, oOO, oVO, oVV, oROO, total;
};
MoLayout mo_layout(const Dims &d)
{
    Carve pv;
    MoLayout L;
    const long vo = (long)d.v * d.o;
    L.oC = pv.take((size_t)d.N * d.nmo);
    L.oCI = pv.take((size_t)d.N * d.nmo);  // C rows in the integral order (forward transforms)
    L.oE = pv.take(d.nmo);
    L.oA = pv.take((size_t)d.nJ * vo);
    L.oOO = pv.take((size_t)d.nK * d.o * d.o);
    L.oVO = pv.take((size_t)d.nK * vo);
    L.oVV = pv.take((size_t)d.nK * d.v * d.v);
    L.oROO = pv.take((size_t)d.nK * d.o * d.o);
    L.total = pv.off;
    return L;
}

// (mu nu|P) of one block of nb auxiliary functions and its half-transformed
// Z; after the blocks the same region serves the M_K^-1 fits by rows a.
struct Int3cWs {
    size_t oX, oZ, total;
};
Int3cWs int3c_ws(const Dims &d, int nb)
{
    Carve cv;
    Int3cWs L;
    const size_t NN = (size_t)d.N * d.N;
    L.oX = cv.take((size_t)nb * NN);
    L.oZ = cv.take((size_t)nb * d.N * std::max(d.o, d.v));
    L.total = cv.off;
    return L;
}

// K-split of the long-K Coulomb products t = V (ai|P)^T (K = nvir nocc, a few
// output rows): 512 ranges fill the 256 CUs twice over, also when (ai|P) rows
// are long enough that the product goes out in column slices of one tile each
constexpr int kSplitV = 512;
struct MatvecWs {
    size_t ot, oT, oU, oSK, total;
};
constexpr int kMatvecChunk = 10;  // vectors whose exchange terms share one GEMM
// K-split of the exchange products U (v x chunk*o output, K = nK v or o nK)
int matvec_u_splits(const Dims &d, int chunk)
{
    return balanced_splits((long)((d.v + 127) / 128) * ((chunk * d.o + 127) / 128), 8);
}

MatvecWs matvec_ws(const Dims &d, int nvec, int chunk = kMatvecChunk)
{
    Carve cv;
    MatvecWs L;
    chunk = std::max(1, std::min(nvec, chunk));
    const long vo = (long)d.v * d.o, oo = (long)d.o * d.o;
    L.ot = cv.take((size_t)nvec * d.nJ * 2);
    L.oT = cv.take((size_t)chunk * d.nK * std::max(vo, oo));  // T (exchange A) or S (exchange B)
    L.oU = cv.take((size_t)chunk * vo);                        // [a][k][i] product before the permuted add
    // split-K partials of t = V (ai|P)^T and of the exchange products U
    L.oSK = cv.take(std::max((size_t)kSplitV * nvec * d.nJ,
                             (size_t)matvec_u_splits(d, chunk) * d.v * chunk * d.o));
    L.total = cv.off;
    return L;
}

constexpr int kDavMaxSpace = 256;  // largest Davidson subspace (the Jacobi eigensolver's size)
// K-split of the Gram products of V_PQ (nK x nK output, K = o^2): about 1024
// workgroups over its 128 x 128 tiles
int vpq_splits(int nK)
{
    const int t = (nK + 127) / 128;
    return std::max(1, std::min(256, 1024 / (t * t)));
}
// doubles holding a reduced-precision copy of a rows x cols FP64 matrix: float
// (FP32 mode) or the bf16 planes of the split modes (up to three 2-byte parts
// per element of the padded width plane_ld(cols))
size_t xcopy_doubles(size_t rows, long cols)
{
    return std::max((rows * cols + 1) / 2, (rows * plane_ld(cols) * 3 + 3) / 4);
}

struct ContractWs {
    size_t oR, oL, oRLT, oF, oD, otT, ocv, oTall, oHUO, oHOU, oHUU, oW, oHc, oY, oG, oV2, oSK, op3, op2, oshA, oshC,
        oshP, oFf, oWf, oGc, total;
};
ContractWs contract_ws(const Dims &d, int ns)
{
    Carve cv;
    ContractWs L;
    const long vo = (long)d.v * d.o, NN = (long)d.N * d.N, o3 = 3L * d.o, oo = (long)d.o * d.o;
    const long w2 = 2L * ns * d.o;
    const int NO = kMaxOutChunk;
    L.oR = cv.take((size_t)ns * vo);
    L.oL = cv.take((size_t)ns * vo);
    L.oRLT = cv.take((size_t)d.v * w2);
    L.oF = cv.take((size_t)ns * d.N * o3);
    L.oD = cv.take((size_t)ns * NN);
    L.otT = cv.take((size_t)ns * d.nJ);
    L.ocv = cv.take((size_t)ns * d.nJ);
    L.oTall = cv.take((size_t)d.v * d.nK * w2);
    L.oHUO = cv.take((size_t)w2 * d.nK * d.o);
    L.oHOU = cv.take((size_t)d.nK * d.o * w2);
    L.oHUU = cv.take((size_t)2 * d.nK * oo);
    L.oW = cv.take((size_t)d.nK * o3 * o3);
    // gathered H_UO / H_OU blocks ([P][i][j], four of them) and G of the metric weights
    L.oHc = cv.take((size_t)4 * d.nK * oo + (size_t)d.nK * d.nK);
    L.oY = cv.take(std::max((size_t)d.nK * d.N * o3, xcopy_doubles((size_t)d.nK * d.N, o3)));
    // reduced-precision copies of F_s and W^P (W^P transposed in the planes)
    L.oFf = cv.take(xcopy_doubles((size_t)ns * d.N, o3));
    L.oWf = cv.take(xcopy_doubles((size_t)d.nK * o3, o3));
    L.oG = cv.take((size_t)NO * d.nK * NN);
    // compact copy of the kept lower blocks of Gamma, K function fastest
    L.oGc = cv.take((size_t)NO * d.nfq * d.nK);
    L.oV2 = cv.take((size_t)NO * d.nJ * d.nJ);
    L.oSK = cv.take(std::max((size_t)kSplitV * ns * d.nJ, (size_t)vpq_splits(d.nK) * d.nK * d.nK));
    L.op3 = cv.take((size_t)d.nshAO * d.nshJ * 3 * NO * 6);
    L.op2 = cv.take((size_t)d.nshJ * 2 * NO * 3);
    L.oshA = cv.take((size_t)d.nshAO * NO * 3);
    L.oshC = cv.take((size_t)d.nshJ * NO * 3);
    L.oshP = cv.take((size_t)d.nshJ * NO * 3);
    L.total = cv.off;
    return L;
}

// Scratch of the contraction blocked over the exchange (K) functions: the
// per-state factors, per output the H_OU blocks of its two states for all P,
// and per block of nb functions Tall, H_UU, W (+ float copy), Y and Gamma.
struct ContractBlkWs {
    size_t oR, oL, oRLT, oF, oFf, oD, otT, ocv, oHI0, oHI1, oHJ0, oHJ1, oTR, oG1, oV2, oSK, op3, op2, oshA, oshC, oshP,
        oTall, oHUU, oW, oWf, oY, oG, oGc, oOut, total;
};
ContractBlkWs contract_blk_ws(const Dims &d, int ns, int nb)
{
    Carve cv;
    ContractBlkWs L;
    const long vo = (long)d.v * d.o, NN = (long)d.N * d.N, o3 = 3L * d.o, oo = (long)d.o * d.o;
    const long w2 = 2L * ns * d.o;
    L.oR = cv.take((size_t)ns * vo);
    L.oL = cv.take((size_t)ns * vo);
    L.oRLT = cv.take((size_t)d.v * w2);
    L.oF = cv.take((size_t)ns * d.N * o3);
    L.oFf = cv.take(xcopy_doubles((size_t)ns * d.N, o3));
    L.oD = cv.take((size_t)ns * NN);
    L.otT = cv.take((size_t)ns * d.nJ);
    L.ocv = cv.take((size_t)ns * d.nJ);
    L.oHI0 = cv.take((size_t)d.nK * oo);
    L.oHI1 = cv.take((size_t)d.nK * oo);
    L.oHJ0 = cv.take((size_t)d.nK * oo);
    L.oHJ1 = cv.take((size_t)d.nK * oo);
    L.oTR = cv.take((size_t)d.nK * oo);
    L.oG1 = cv.take((size_t)kMaxOutChunk * d.nK * d.nK);
    L.oV2 = cv.take((size_t)kMaxOutChunk * d.nJ * d.nJ);
    L.oOut = cv.take((size_t)kMaxOutChunk * d.natm * 3);
    L.oSK = cv.take(std::max((size_t)kSplitV * ns * d.nJ, (size_t)vpq_splits(d.nK) * d.nK * d.nK));
    L.op3 = cv.take((size_t)d.nshAO * d.nshJ * 3 * kMaxOutChunk * 6);
    L.op2 = cv.take((size_t)d.nshJ * 2 * kMaxOutChunk * 3);
    L.oshA = cv.take((size_t)d.nshAO * kMaxOutChunk * 3);
    L.oshC = cv.take((size_t)d.nshJ * kMaxOutChunk * 3);
    L.oshP = cv.take((size_t)d.nshJ * kMaxOutChunk * 3);
    L.oTall = cv.take((size_t)nb * d.v * 2 * d.o);
    L.oHUU = cv.take((size_t)2 * nb * oo);
    L.oW = cv.take((size_t)nb * o3 * o3);
    L.oWf = cv.take(xcopy_doubles((size_t)nb * o3, o3));
    L.oY = cv.take(std::max((size_t)nb * d.N * o3, xcopy_doubles((size_t)nb * d.N, o3)));
    L.oG = cv.take((size_t)nb * NN);
    L.oGc = cv.take((size_t)d.nfq * nb);  // compact copy of the block's Gamma (one output)
    L.total = cv.off;
    return L;
}

struct AuxLayout {
    size_t oAO, oAX, oP, oMJ, oLJ, oIJ, oIK, oPP, oPI, oPQ, oGT, oOI, oPJ, total;
};
AuxLayout aux_layout(int nsh, int nshJ, int nao, int nJ, int nK)
{
    Carve cv;
    AuxLayout L;
    L.oAO = cv.take(shell_bytes(nsh) / 8 + 1);
    L.oAX = cv.take(shell_bytes(nshJ) / 8 + 1);
    L.oP = cv.take(nao / 2 + 1);
    L.oOI = cv.take(nsh / 2 + 1);   // integral-order first functions (ints)
    L.oPJ = cv.take(nao / 2 + 1);   // integral-order permutation (ints)
    L.oMJ = cv.take((size_t)nJ * nJ);
    L.oLJ = cv.take((size_t)nJ * nJ);
    L.oIJ = cv.take((size_t)nJ * nJ);
    L.oIK = cv.take((size_t)nK * nK);
    // screened pair lists sized for the unscreened worst case (ints, 2 per slot)
    L.oPP = cv.take(((size_t)(kMaxAOL + 1) * nsh + 2) / 2);
    L.oPI = cv.take(((size_t)nsh * nsh + 1) / 2);
    // numbering of the compact exchange-weight copy (ints): a block start per
    // list entry, the earlier partners of each shell (pointers, shells, block
    // starts) and their columns (pointers, two lists of at most nsh * nao:
    // a shell's earlier partners hold at most nao functions)
    L.oPQ = cv.take(((size_t)2 * nsh * nsh + 4 * (size_t)nsh + 4 + 2 * (size_t)nsh * nao) / 2 + 1);
    // lower-tile list of the AO-pair matrix (ints, 2 per slot)
    const size_t tm = (size_t)(nao + 127) / 128;
    L.oGT = cv.take((tm * (tm + 1) + 1) / 2);  // two orders of the list
    L.total = cv.off;
    return L;
}

Dims ctx_dims(const ris_ctx *c)
{
    return Dims{c->nao, c->nmo, c->nocc, c->nvir, c->nJ, c->nK, c->nshAO, c->nshJ, c->natm, c->nfq};
}

// ========================================================================
extern "C" {

int ris_ctx_create(ris_ctx **out, int device, void *hip_stream, size_t hbm_budget)
{
    if (!out) return RIS_E_INVALID;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return RIS_E_DEVICE;
    if (device < 0 || device >= ndev) return RIS_E_INVALID;
    if (hipSetDevice(device) != hipSuccess) return RIS_E_DEVICE;
    ris_ctx *c = new ris_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        delete c;
        return RIS_E_DEVICE;
    }
    c->budget = hbm_budget ? hbm_budget : (size_t)(0.9 * (double)fr);
    // the fixed scratch of the allocation-free matvec, resolved with the device current
    if (scratch_address(device, &c->scratch_dev) != hipSuccess) {
        delete c;
        return RIS_E_DEVICE;
    }
    int st;
    c->boys = (double *)dalloc(c, sizeof(double) * kBoysNGrid * kBoysCols, &st);
    c->info = (int *)dalloc(c, 64, &st);
    if (!c->boys || !c->info) {
        ris_ctx_destroy(c);
        return RIS_E_NOMEM;
    }
    std::vector<double> tab((size_t)kBoysNGrid * kBoysCols);
    boys_table_host(tab.data());
    if (hipMemcpy(c->boys, tab.data(), tab.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
        ris_ctx_destroy(c);
        return RIS_E_DEVICE;
    }
    *out = c;
    return RIS_OK;
}

void ris_ctx_destroy(ris_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto &b : c->bufs) (void)hipFree(b.p);
    release_marks(c);
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    delete c;
}

size_t ris_plan_bytes(const ris_mol *mol, const ris_aux_opts *opts, int nmo, int nocc, int nstate, int nvec, int nout,
                      int aux_block)
{
    if (!mol || !opts || mol->natm <= 0 || mol->nshell <= 0 || nocc <= 0 || nmo <= nocc || aux_block < 0) return 0;
    int nao = 0, nheavy = 0;
    for (int s = 0; s < mol->nshell; ++s) nao += ncart(mol->shell_l[s]);
    for (int a = 0; a < mol->natm; ++a) nheavy += (mol->Z[a] > 1);
    const int natm = mol->natm;
    const int nshJ = natm + (opts->j_p_on_heavy ? nheavy : 0);
    const int nJ = natm + (opts->j_p_on_heavy ? 3 * nheavy : 0);
    // function pairs of the unordered AO shell pairs the default screen keeps
    long nfq = 0;
    for (int a = 0; a < mol->nshell; ++a)
        for (int b = 0; b <= a; ++b) {
            const double *A = mol->xyz + 3 * mol->shell_atom[a], *B = mol->xyz + 3 * mol->shell_atom[b];
            const double r2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) + (A[2] - B[2]) * (A[2] - B[2]);
            if (pair_kept(mol->shell_exp[a], mol->shell_exp[b], r2, kDefaultScreen))
                nfq += (long)ncart(mol->shell_l[a]) * ncart(mol->shell_l[b]);
        }
    const Dims d{nao, nmo, nocc, nmo - nocc, nJ, natm, mol->shell_l ? mol->nshell : 0, nshJ, natm,
                 nfq < (1L << 30) ? nfq : 0};
    size_t ws;
    if (aux_block == 0) {
        ws = int3c_ws(d, d.nJ).total;
        if (nvec > 0) ws = std::max(ws, matvec_ws(d, nvec).total);
        if (nstate > 0) ws = std::max(ws, contract_ws(d, nstate).total);
    } else {
        ws = int3c_ws(d, std::max(3, std::min(aux_block, d.nJ))).total;
        if (nvec > 0) ws = std::max(ws, matvec_ws(d, nvec, 1).total);
        if (nstate > 0) ws = std::max(ws, contract_blk_ws(d, nstate, std::min(aux_block, d.nK)).total);
    }
    ws = std::max(ws, sizeof(double) * (size_t)kTriBlock * nJ);  // metric inverse in ris_aux_build
    const size_t fixed = (size_t)8 * kBoysNGrid * kBoysCols + 64;
    return fixed + aux_layout(mol->nshell, nshJ, nao, nJ, natm).total + mo_layout(d).total + ws +
           (size_t)8 * std::max(nout, 0) * natm * 3;
}

size_t ris_request_bytes(const ris_mol *mol, const ris_aux_opts *opts, int nmo, int nocc, int nstate, int nvec,
                         int nout)
{
    return ris_plan_bytes(mol, opts, nmo, nocc, nstate, nvec, nout, 0);
}

int ris_zvector_solve(ris_ctx *c, int nrhs, const double *rhs, double *Z, double tol, int maxit, int *iters,
                      double *rel_resid)
{
    if (!c) return RIS_E_INVALID;
    c->err.clear();
    if (iters) *iters = 0;
    if (rel_resid) *rel_resid = 0.0;
    if (!c->have_int3c) return fail(c, RIS_E_ORDER, "ris_zvector_solve before ris_int3c");
    if (nrhs < 0 || maxit < 0) return fail(c, RIS_E_INVALID, "nrhs and maxit must be >= 0");
    if (!(tol > 0.0 && tol < 1.0)) return fail(c, RIS_E_INVALID, "tol must be in (0, 1)");
    if (nrhs == 0) return RIS_OK;
    if (!rhs || !Z || rhs == Z) return fail(c, RIS_E_INVALID, "null or aliased rhs / Z pointer");
    HIPCHK(c, hipSetDevice(c->device));
    const int o = c->nocc, v = c->nvir, nb = nrhs;
    const long n = (long)v * o;
    const size_t nv = (size_t)nb * n;
    // v, q, r1, r2, yz, w, w1, w2 (nb vectors each), de, dot partials, state rows
    Carve cv;
    size_t ob[8];
    for (int i = 0; i < 8; ++i) ob[i] = cv.take(nv);
    const size_t ode = cv.take(n), opart = cv.take(bdot_partials(n, nb)), ost = cv.take((size_t)nb * kMrStride);
    int stc;
    char *base = pool_get(c, c->zv_pool, cv.off, &stc);
    if (!base) return stc;
    double *buf[8];
    for (int i = 0; i < 8; ++i) buf[i] = (double *)(base + ob[i]);
    double *V = buf[0], *Q = buf[1], *R1 = buf[2], *R2 = buf[3], *YZ = buf[4], *Wv = buf[5], *W1 = buf[6],
           *W2 = buf[7];
    double *de = (double *)(base + ode), *part = (double *)(base + opart);
    MrState *st = (MrState *)(base + ost);
    double *stp = (double *)st;

    // preconditioner e_a - e_i, start: Z = 0, r2 = rhs, y = M^-1 rhs, beta1^2 = <rhs, y>
    HIPCHK(c, orbital_gaps(c->eps, v, o, de, c->stream));
    HIPCHK(c, fill(Z, nv, 0.0, c->stream));
    HIPCHK(c, fill(Wv, nv, 0.0, c->stream));
    HIPCHK(c, fill(W1, nv, 0.0, c->stream));
    HIPCHK(c, fill(W2, nv, 0.0, c->stream));
    HIPCHK(c, fill(R1, nv, 0.0, c->stream));
    HIPCHK(c, hipMemcpyAsync(R2, rhs, nv * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, precond(R2, de, YZ, n, nb, c->stream));
    HIPCHK(c, bdot(R2, YZ, n, nb, part, stp + offsetof(MrState, beta2) / sizeof(double), kMrStride, c->stream));
    HIPCHK(c, mr_init(st, nb, tol, c->stream));

    std::vector<MrState> hs(nb);
    int it = 0;
    bool all_done = false;
    HIPCHK(c, hipMemcpyAsync(hs.data(), st, sizeof(MrState) * nb, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    all_done = std::all_of(hs.begin(), hs.end(), [](const MrState &x) { return x.active == 0.0; });
    while (!all_done && it < maxit) {
        ++it;
        HIPCHK(c, mr_v(st, YZ, V, n, nb, c->stream));
        {
            const int sm = ris_response_matvec(c, RIS_OP_APB, nb, V, Q);
            if (sm != RIS_OK) return sm;
        }
        HIPCHK(c, mr_y1(st, R1, Q, n, nb, it >= 2 ? 1 : 0, c->stream));
        HIPCHK(c, bdot(V, Q, n, nb, part, stp + offsetof(MrState, alfa) / sizeof(double), kMrStride, c->stream));
        HIPCHK(c, mr_y2(st, R2, Q, n, nb, c->stream));
        std::swap(R1, R2);  // r1 <- r2
        std::swap(R2, Q);   // r2 <- y; the old r1 buffer receives the next matvec
        HIPCHK(c, precond(R2, de, YZ, n, nb, c->stream));
        HIPCHK(c, bdot(R2, YZ, n, nb, part, stp + offsetof(MrState, beta2) / sizeof(double), kMrStride, c->stream));
        HIPCHK(c, mr_scal(st, nb, c->stream));
        // w1 <- w2, w2 <- w, w <- (v - oldeps w1 - delta w2) denom, x += phi w
        double *nw = W1;
        W1 = W2;
        W2 = Wv;
        Wv = nw;
        HIPCHK(c, mr_w(st, V, W1, W2, Wv, Z, n, nb, c->stream));
        HIPCHK(c, hipMemcpyAsync(hs.data(), st, sizeof(MrState) * nb, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        all_done = std::all_of(hs.begin(), hs.end(), [](const MrState &x) { return x.active == 0.0; });
    }
    // true residual rhs - (A+B) Z
    {
        const int sm = ris_response_matvec(c, RIS_OP_APB, nb, Z, Q);
        if (sm != RIS_OK) return sm;
    }
    HIPCHK(c, vsub(rhs, Q, R1, nv, c->stream));
    std::vector<double> rr(nb), bb(nb);
    // the dots land in the first nb doubles of two free vector buffers
    HIPCHK(c, bdot(R1, R1, n, nb, part, YZ, 1, c->stream));
    HIPCHK(c, bdot(rhs, rhs, n, nb, part, W1, 1, c->stream));
    HIPCHK(c, hipMemcpyAsync(rr.data(), YZ, sizeof(double) * nb, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(bb.data(), W1, sizeof(double) * nb, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double rel = 0.0;
    for (int k = 0; k < nb; ++k)
        if (bb[k] > 0.0) rel = std::max(rel, std::sqrt(rr[k] / bb[k]));
    if (iters) *iters = it;
    if (rel_resid) *rel_resid = rel;
    if (!all_done) return fail(c, RIS_E_NOCONV, "Z-vector solve: %d iterations, relative residual %.3e", it, rel);
    return RIS_OK;
}

int ris_tda_davidson(ris_ctx *c, int nroots, double tol, int maxit, int max_space, double *omega, double *X,
                     int *iters)
{
    if (!c) return RIS_E_INVALID;
    c->err.clear();
    if (iters) *iters = 0;
    if (!c->have_int3c) return fail(c, RIS_E_ORDER, "ris_tda_davidson before ris_int3c");
    const int o = c->nocc, v = c->nvir;
    const long n = (long)v * o;
    if (nroots <= 0 || nroots > n) return fail(c, RIS_E_INVALID, "nroots must be in [1, nvir*nocc]");
    if (!(tol > 0.0) || maxit <= 0) return fail(c, RIS_E_INVALID, "tol must be > 0 and maxit >= 1");
    if (!omega || !X) return fail(c, RIS_E_INVALID, "null omega or X pointer");
    const long cap = std::min<long>(n, kDavMaxSpace);
    int ms = max_space > 0 ? max_space : (int)std::min<long>(cap, std::max(8 * nroots, 32));
    if (ms > cap || ms < std::min<long>(n, 2L * nroots))
        return fail(c, RIS_E_INVALID, "max_space must be in [min(2 nroots, nvir*nocc), %ld]", cap);
    HIPCHK(c, hipSetDevice(c->device));
    const int k0 = (int)std::min<long>(ms, std::min<long>(n, 2L * nroots));  // start vectors
    // layout: V, AV [ms][n]; Ritz X, AX, residual / corrections R [nroots][n]; H, work [ms][ms]; w, cs [ms + 1];
    // gaps [n]; dot partials; start indices
    Carve cv;
    const size_t oV = cv.take((size_t)ms * n), oAV = cv.take((size_t)ms * n), oX = cv.take((size_t)nroots * n),
                 oAX = cv.take((size_t)nroots * n), oR = cv.take((size_t)nroots * n), oH = cv.take((size_t)ms * ms),
                 oWk = cv.take((size_t)ms * ms), ow = cv.take(ms + 1), ocs = cv.take(ms + 1), ode = cv.take(n),
                 opt = cv.take(bdot_partials(n, std::max(ms, nroots))), onr = cv.take(std::max(ms, nroots)),
                 oid = cv.take((k0 + 1) / 2 + 1);
    // K-split of the subspace products (m x m or 1 x m outputs, K = nvir nocc)
    const int nsk = (int)std::max<long>(1, std::min<long>(256, n / 4096));
    const size_t osk = cv.take((size_t)nsk * ms * ms);
    int stc;
    char *base = pool_get(c, c->dv_pool, cv.off, &stc);
    if (!base) return stc;
    auto D = [&](size_t off) { return (double *)(base + off); };
    double *Vb = D(oV), *AVb = D(oAV), *Xr = D(oX), *AXr = D(oAX), *Rb = D(oR), *H = D(oH), *Wk = D(oWk), *w = D(ow),
           *csb = D(ocs), *de = D(ode), *part = D(opt), *nrm = D(onr);
    int *didx = (int *)(base + oid);
    double *skb = D(osk);

    // start: unit vectors on the k0 smallest orbital-energy gaps
    HIPCHK(c, orbital_gaps_plain(c->eps, v, o, de, c->stream));
    std::vector<double> hde(n);
    HIPCHK(c, hipMemcpyAsync(hde.data(), de, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<int> order(n);
    for (long i = 0; i < n; ++i) order[i] = (int)i;
    std::partial_sort(order.begin(), order.begin() + k0, order.end(),
                      [&](int a, int b) { return hde[a] < hde[b] || (hde[a] == hde[b] && a < b); });
    HIPCHK(c, hipMemcpyAsync(didx, order.data(), sizeof(int) * k0, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, fill(Vb, (size_t)k0 * n, 0.0, c->stream));
    HIPCHK(c, set_units(Vb, didx, k0, n, c->stream));
    int m = k0;
    {
        const int sm = ris_response_matvec(c, RIS_OP_A, m, Vb, AVb);
        if (sm != RIS_OK) return sm;
    }
    std::vector<double> hw(nroots), hn(nroots);
    int it = 0;
    bool conv = false;
    while (it < maxit) {
        ++it;
        // subspace matrix H = V AV^T (symmetrised), its eigenpairs, Ritz pairs
        HIPCHK(c, dgemm_splitk(gm(m, m, (int)n, false, true, 1.0, Vb, n, AVb, n, 0.0, H, m), nsk, skb, c->stream));
        HIPCHK(c, symmetrize(H, m, 1, c->stream));
        HIPCHK(c, sym_eig_small(H, Wk, m, w, csb, c->stream));
        HIPCHK(c, dgemm(gm(nroots, (int)n, m, false, false, 1.0, H, m, Vb, n, 0.0, Xr, n), c->stream));
        HIPCHK(c, dgemm(gm(nroots, (int)n, m, false, false, 1.0, H, m, AVb, n, 0.0, AXr, n), c->stream));
        HIPCHK(c, ritz_residual(AXr, Xr, w, Rb, n, nroots, c->stream));
        HIPCHK(c, bdot(Rb, Rb, n, nroots, part, nrm, 1, c->stream));
        HIPCHK(c, hipMemcpyAsync(hw.data(), w, sizeof(double) * nroots, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(hn.data(), nrm, sizeof(double) * nroots, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        std::vector<int> todo;
        for (int j = 0; j < nroots; ++j)
            if (std::sqrt(std::max(hn[j], 0.0)) > tol) todo.push_back(j);
        if (todo.empty()) {
            conv = true;
            break;
        }
        if (it == maxit) break;
        // corrections of the unconverged roots, in place in R
        for (int j : todo) HIPCHK(c, davidson_correction(Rb + (size_t)j * n, hw[j], de, Rb + (size_t)j * n, n, c->stream));
        // collapse to the Ritz vectors when the new ones would not fit
        if (m + (int)todo.size() > ms) {
            HIPCHK(c, hipMemcpyAsync(Vb, Xr, sizeof(double) * nroots * n, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(AVb, AXr, sizeof(double) * nroots * n, hipMemcpyDeviceToDevice, c->stream));
            m = nroots;
        }
        // append each correction after two Gram-Schmidt passes against the basis
        const int m0 = m;
        for (int j : todo) {
            double *t = Rb + (size_t)j * n;
            HIPCHK(c, bdot(t, t, n, 1, part, nrm, 1, c->stream));
            double before = 0.0;
            HIPCHK(c, hipMemcpyAsync(&before, nrm, sizeof(double), hipMemcpyDeviceToHost, c->stream));
            for (int pass = 0; pass < 2; ++pass) {
                HIPCHK(c, dgemm_splitk(gm(1, m, (int)n, false, true, 1.0, t, n, Vb, n, 0.0, csb, m), nsk, skb,
                                       c->stream));
                HIPCHK(c, dgemm(gm(1, (int)n, m, false, false, -1.0, csb, m, Vb, n, 1.0, t, n), c->stream));
            }
            HIPCHK(c, bdot(t, t, n, 1, part, nrm, 1, c->stream));
            double after = 0.0;
            HIPCHK(c, hipMemcpyAsync(&after, nrm, sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            if (!(after > 1e-20 * std::max(before, 1e-300)) || m >= ms) continue;  // dependent: dropped
            HIPCHK(c, axpby(t, Vb + (size_t)m * n, n, 1.0 / std::sqrt(after), 0.0, c->stream));
            ++m;
        }
        if (m == m0) break;  // no new direction: the iteration has stalled
        {
            const int sm = ris_response_matvec(c, RIS_OP_A, m - m0, Vb + (size_t)m0 * n, AVb + (size_t)m0 * n);
            if (sm != RIS_OK) return sm;
        }
    }
    HIPCHK(c, hipMemcpyAsync(X, Xr, sizeof(double) * nroots * n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int j = 0; j < nroots; ++j) omega[j] = hw[j];
    if (iters) *iters = it;
    if (!conv) return fail(c, RIS_E_NOCONV, "TDA Davidson: %d iterations without convergence", it);
    return RIS_OK;
}

int ris_zrhs_contract(ris_ctx *c, int nstate, const double *X, const double *Y, int npair, const int *pairs,
                      double *G)
{
    if (!c) return RIS_E_INVALID;
    c->err.clear();
    if (!c->have_int3c) return fail(c, RIS_E_ORDER, "ris_zrhs_contract before ris_int3c");
    if (nstate <= 0 || npair < 0) return fail(c, RIS_E_INVALID, "nstate must be > 0 and npair >= 0");
    if (npair == 0) return RIS_OK;
    if (!X || !pairs || !G) return fail(c, RIS_E_INVALID, "null X, pairs or G pointer");
    std::vector<char> used(nstate, 0);
    for (int k = 0; k < npair; ++k) {
        const int I = pairs[2 * k], J = pairs[2 * k + 1];
        if (I < 0 || J < 0 || I >= nstate || J >= nstate) return fail(c, RIS_E_INVALID, "pair %d out of range", k);
        used[I] = used[J] = 1;
    }
    if (c->nK > c->auxl_beg[1]) return fail(c, RIS_E_UNSUPPORTED, "exchange set is not a run of leading s shells");
    HIPCHK(c, hipSetDevice(c->device));
    const int N = c->nao, nmo = c->nmo, o = c->nocc, v = c->nvir, nJ = c->nJ, nK = c->nK, ns = nstate;
    const long vo = (long)v * o, NN = (long)N * N, MM = (long)nmo * nmo;
    // ---- common part: R, L, U = C_V R, U' = C_V L, Coulomb vectors, the AO
    // matrices g[D] of every used state (t = 0: R^S, t = 1: L^A) and their MO forms
    Carve cv;
    const size_t oR = cv.take((size_t)ns * vo), oL = cv.take((size_t)ns * vo), oUR = cv.take((size_t)ns * N * o),
                 oUL = cv.take((size_t)ns * N * o), otT = cv.take((size_t)ns * nJ), ocv = cv.take((size_t)ns * nJ),
                 oSK = cv.take((size_t)kSplitV * ns * nJ), ogA = cv.take((size_t)ns * 2 * NN),
                 oT1 = cv.take((size_t)N * nmo), ogM = cv.take((size_t)ns * 2 * MM), oEm = cv.take((size_t)4 * MM);
    const size_t common = cv.off;
    // K-split of the exchange products (N x N output, K = (block functions) x nocc)
    const int ksp = balanced_splits((long)((N + 127) / 128) * ((N + 127) / 128), 8);
    // the integral part: all J functions at once, or blocks of nb functions (whole shells)
    auto path_bytes = [&](int nb, bool all) {
        Carve q;
        const long Ko = (long)(all ? nK : nb) * o;
        q.take((size_t)(all ? nJ : nb) * NN);  // raw (mu nu|P) of the J set / of the block
        q.take((size_t)(all ? nK : nb) * NN);  // metric-applied exchange functions C^P
        if (!all) q.take((size_t)nb * NN);     // streamed K blocks
        for (int k = 0; k < 4; ++k) q.take((size_t)N * Ko);
        q.take((size_t)ksp * NN);
        return q.off;
    };
    const size_t other = c->held - c->ws_bytes;
    const size_t wsroom = std::max(c->budget > other ? c->budget - other : 0, c->ws_bytes);
    const bool blocked = (c->ablock > 0 && c->ablock < nK) || common + path_bytes(nK, true) > wsroom;
    int nb = nK;
    if (blocked) {
        nb = std::max(3, c->ablock > 0 ? std::min(c->ablock, nK) : nK);
        while (nb > 3 && common + path_bytes(nb, false) > wsroom) nb = std::max(3, (int)(nb * 0.8));
    }
    const size_t total = common + path_bytes(nb, !blocked);
    int st;
    char *wsb = ws_get(c, total, &st);
    if (!wsb) return st;
    auto P_ = [&](size_t off) { return (double *)(wsb + off); };
    double *R = P_(oR), *L = P_(oL), *UR = P_(oUR), *UL = P_(oUL), *tT = P_(otT), *cvec = P_(ocv), *SK = P_(oSK),
           *gAll = P_(ogA), *T1 = P_(oT1), *gM = P_(ogM), *Em = P_(oEm);
    const double *CO = c->C, *CV = c->C + o;

    HIPCHK(c, make_rl(X, Y, R, L, (size_t)ns * vo, c->stream));
    for (int t = 0; t < 2; ++t) {
        GemmArgs g = gm(N, o, v, false, false, 1.0, CV, nmo, t ? L : R, o, 0.0, t ? UL : UR, o);
        g.batch = ns; g.strideA = 0; g.strideB = vo; g.strideC = (long)N * o;
        HIPCHK(c, dgemm(g, c->stream));
    }
    HIPCHK(c, dgemm_splitk(gm(ns, nJ, (int)vo, false, true, 1.0, R, vo, c->aiJ, vo, 0.0, tT, nJ), kSplitV, SK,
                           c->stream));
    HIPCHK(c, dgemm(gm(ns, nJ, nJ, false, false, 1.0, tT, nJ, c->MinvJ, nJ, 0.0, cvec, nJ), c->stream));
    HIPCHK(c, fill(gAll, (size_t)ns * 2 * NN, 0.0, c->stream));

    // the exchange part of g[D] for the functions [p0, p0 + m) of the K set:
    //   K[D] = sum_P C^P D (mu nu|P) = (Y1 Z2^T +- Z1 Y2^T) / 2,
    //   Z1^P = C^P C_O, Z2^P = (.|P) C_O, Y1^P = C^P U, Y2^P = (.|P) U  ([mu][P][i])
    auto exchange = [&](const double *Cb, const double *Xb, int m, double *Z1, double *Z2, double *Y1, double *Y2,
                        double *SK2) -> int {
        const long Ko = (long)m * o;
        for (int t = 0; t < 2; ++t) {
            GemmArgs g = gm(N, o, N, false, false, 1.0, t ? Xb : Cb, N, CO, nmo, 0.0, t ? Z2 : Z1, Ko);
            g.batch = m; g.strideA = NN; g.strideB = 0; g.strideC = o;
            HIPCHK(c, dgemm(g, c->stream));
        }
        for (int s = 0; s < ns; ++s) {
            if (!used[s]) continue;
            for (int t = 0; t < 2; ++t) {
                const double *U = (t ? UL : UR) + (size_t)s * N * o;
                for (int q = 0; q < 2; ++q) {
                    GemmArgs g = gm(N, o, N, false, false, 1.0, q ? Xb : Cb, N, U, o, 0.0, q ? Y2 : Y1, Ko);
                    g.batch = m; g.strideA = NN; g.strideB = 0; g.strideC = o;
                    HIPCHK(c, dgemm(g, c->stream));
                }
                double *gA = gAll + ((size_t)s * 2 + t) * NN;
                const double sgn = t ? -1.0 : 1.0;
                HIPCHK(c, dgemm_splitk(gm(N, N, (int)Ko, false, true, -0.5 * c->cx, Y1, Ko, Z2, Ko, 1.0, gA, N), ksp,
                                       SK2, c->stream));
                HIPCHK(c, dgemm_splitk(gm(N, N, (int)Ko, false, true, -0.5 * c->cx * sgn, Z1, Ko, Y2, Ko, 1.0, gA,
                                          N), ksp, SK2, c->stream));
            }
        }
        return RIS_OK;
    };
    // Coulomb part alpha_J sum_P c_s,P (mu nu|P) of the J functions [f0, f0 + nf), into gAll[s][0]
    auto coulomb = [&](const double *Xb, int f0, int nf) -> int {
        GemmArgs g = gm(ns, (int)NN, nf, false, false, c->alphaJ, cvec + f0, nJ, Xb, NN, 1.0, gAll, 2 * NN);
        HIPCHK(c, dgemm(g, c->stream));
        return RIS_OK;
    };

    Carve q;
    q.off = common;
    if (!blocked) {
        const long Ko = (long)nK * o;
        double *X3 = P_(q.take((size_t)nJ * NN)), *Bk = P_(q.take((size_t)nK * NN));
        double *Z1 = P_(q.take((size_t)N * Ko)), *Z2 = P_(q.take((size_t)N * Ko)), *Y1 = P_(q.take((size_t)N * Ko)),
               *Y2 = P_(q.take((size_t)N * Ko)), *SK2 = P_(q.take((size_t)ksp * NN));
        HIPCHK(c, launch_int3c(c->ao, c->aux, c->auxl_beg, c->boys, X3, c->stream));
        HIPCHK(c, dgemm(gm(nK, (int)NN, nK, false, false, 1.0, c->MinvK, nK, X3, NN, 0.0, Bk, NN), c->stream));
        if ((st = coulomb(X3, 0, nJ)) != RIS_OK) return st;
        if ((st = exchange(Bk, X3, nK, Z1, Z2, Y1, Y2, SK2)) != RIS_OK) return st;
    } else {
        const long Ko = (long)nb * o;
        double *Xb = P_(q.take((size_t)nb * NN)), *Cb = P_(q.take((size_t)nb * NN)), *Bq = P_(q.take((size_t)nb * NN));
        double *Z1 = P_(q.take((size_t)N * Ko)), *Z2 = P_(q.take((size_t)N * Ko)), *Y1 = P_(q.take((size_t)N * Ko)),
               *Y2 = P_(q.take((size_t)N * Ko)), *SK2 = P_(q.take((size_t)ksp * NN));
        const std::vector<int> &aoff = c->h_aux_off;
        // J shells in blocks of at most nb functions: the Coulomb part
        for (int a = 0; a < c->nshJ;) {
            int b = a + 1;
            while (b < c->nshJ && aoff[b + 1] - aoff[a] <= nb) ++b;
            HIPCHK(c, launch_int3c(c->ao, c->aux, c->auxl_beg, c->boys, Xb, c->stream, a, b));
            if ((st = coulomb(Xb, aoff[a], aoff[b] - aoff[a])) != RIS_OK) return st;
            a = b;
        }
        // K functions (the leading s shells) in blocks of nb: C^P of the block
        // from every K block streamed through Bq, the raw block itself in Xb
        for (int k0 = 0; k0 < nK; k0 += nb) {
            const int m = std::min(nb, nK - k0);
            HIPCHK(c, launch_int3c(c->ao, c->aux, c->auxl_beg, c->boys, Xb, c->stream, k0, k0 + m));
            for (int q0 = 0; q0 < nK; q0 += nb) {
                const int mq = std::min(nb, nK - q0);
                const double *src = Xb;
                if (q0 != k0) {
                    HIPCHK(c, launch_int3c(c->ao, c->aux, c->auxl_beg, c->boys, Bq, c->stream, q0, q0 + mq));
                    src = Bq;
                }
                HIPCHK(c, dgemm(gm(m, (int)NN, mq, false, false, 1.0, c->MinvK + (size_t)k0 * nK + q0, nK, src, NN,
                                   q0 ? 1.0 : 0.0, Cb, NN), c->stream));
            }
            if ((st = exchange(Cb, Xb, m, Z1, Z2, Y1, Y2, SK2)) != RIS_OK) return st;
        }
    }
    // MO forms C^T g[D] C of every used (state, density)
    for (int s = 0; s < ns; ++s) {
        if (!used[s]) continue;
        for (int t = 0; t < 2; ++t) {
            const double *gA = gAll + ((size_t)s * 2 + t) * NN;
            HIPCHK(c, dgemm(gm(N, nmo, N, false, false, 1.0, gA, N, c->C, nmo, 0.0, T1, nmo), c->stream));
            HIPCHK(c, dgemm(gm(nmo, nmo, N, true, false, 1.0, c->C, nmo, T1, nmo, 0.0, gM + ((size_t)s * 2 + t) * MM,
                               nmo), c->stream));
        }
    }
    // per output: 4 [R^S g[R^S]] - 4 [L^A g[L^A]] (I == J), or the four ris terms of Q_IJ
    double *RSI = Em, *LAI = Em + MM, *RSJ = Em + 2 * MM, *LAJ = Em + 3 * MM;
    for (int k = 0; k < npair; ++k) {
        const int I = pairs[2 * k], J = pairs[2 * k + 1];
        double *Gk = G + (size_t)k * MM;
        const double *gRI = gM + ((size_t)I * 2) * MM, *gLI = gM + ((size_t)I * 2 + 1) * MM;
        const double *gRJ = gM + ((size_t)J * 2) * MM, *gLJ = gM + ((size_t)J * 2 + 1) * MM;
        HIPCHK(c, embed_rl(R + (size_t)I * vo, L + (size_t)I * vo, nmo, o, RSI, LAI, c->stream));
        if (I == J) {
            HIPCHK(c, dgemm(gm(nmo, nmo, nmo, false, false, 4.0, RSI, nmo, gRI, nmo, 0.0, Gk, nmo), c->stream));
            HIPCHK(c, dgemm(gm(nmo, nmo, nmo, false, false, -4.0, LAI, nmo, gLI, nmo, 1.0, Gk, nmo), c->stream));
        } else {
            HIPCHK(c, embed_rl(R + (size_t)J * vo, L + (size_t)J * vo, nmo, o, RSJ, LAJ, c->stream));
            HIPCHK(c, dgemm(gm(nmo, nmo, nmo, false, false, 2.0, RSI, nmo, gRJ, nmo, 0.0, Gk, nmo), c->stream));
            HIPCHK(c, dgemm(gm(nmo, nmo, nmo, false, false, -2.0, LAI, nmo, gLJ, nmo, 1.0, Gk, nmo), c->stream));
            HIPCHK(c, dgemm(gm(nmo, nmo, nmo, false, false, 2.0, RSJ, nmo, gRI, nmo, 1.0, Gk, nmo), c->stream));
            HIPCHK(c, dgemm(gm(nmo, nmo, nmo, false, false, -2.0, LAJ, nmo, gLI, nmo, 1.0, Gk, nmo), c->stream));
        }
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RIS_OK;
}

int ris_ctx_set_screening(ris_ctx *c, double threshold, long *kept_pairs)
{
    if (!c) return RIS_E_INVALID;
    c->err.clear();
    if (!(threshold >= 0.0 && threshold < 1.0)) return fail(c, RIS_E_INVALID, "screening threshold must be in [0, 1)");
    HIPCHK(c, hipSetDevice(c->device));
    c->screen = threshold;
    if (c->have_aux) {
        const int sp = build_pairs(c);
        if (sp) return sp;
    }
    if (kept_pairs) *kept_pairs = c->have_aux ? c->npair_kept : -1;
    return RIS_OK;
}

int ris_ctx_set_blocking(ris_ctx *c, int aux_block)
{
    if (!c) return RIS_E_INVALID;
    c->err.clear();
    if (aux_block < 0) return fail(c, RIS_E_INVALID, "aux_block must be >= 0");
    c->ablock = aux_block;
    return RIS_OK;
}

int ris_ctx_set_profiling(ris_ctx *c, int enable)
{
    if (!c) return RIS_E_INVALID;
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    release_marks(c);
    c->prof = enable != 0;
    return RIS_OK;
}

int ris_ctx_stage_stats(ris_ctx *c, int stage, double *ms, double *flops, double *bytes, long *launches)
{
    if (!c || stage < 0 || stage >= RIS_STAGE_COUNT) return RIS_E_INVALID;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double t = 0.0, f = 0.0, by = 0.0;
    long n = 0;
    for (auto &m : c->marks) {
        if (m.stage != stage) continue;
        float e = 0.f;
        HIPCHK(c, hipEventElapsedTime(&e, m.a, m.b));
        t += e;
        f += m.flops;
        by += m.bytes;
        ++n;
    }
    if (ms) *ms = t;
    if (flops) *flops = f;
    if (bytes) *bytes = by;
    if (launches) *launches = n;
    return RIS_OK;
}

int ris_ctx_release(ris_ctx *c)
{
    if (!c) return RIS_E_INVALID;
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    free_aux(c);
    ris_ctx::Pool *pools[] = {&c->aux_pool, &c->mo_pool, &c->out_pool, &c->zv_pool, &c->dv_pool};
    for (ris_ctx::Pool *pl : pools) {
        dfree(c, pl->p);
        pl->p = nullptr;
        pl->bytes = 0;
    }
    dfree(c, c->ws);
    c->ws = nullptr;
    c->ws_bytes = 0;
    return RIS_OK;
}

const char *ris_last_error(const ris_ctx *c) { return c ? c->err.c_str() : "null context"; }

size_t ris_ctx_bytes(const ris_ctx *c) { return c ? c->held : 0; }

// ------------------------------------------------------------------------
int ris_aux_build(ris_ctx *c, const ris_mol *mol, const ris_aux_opts *opts, int *nauxJ, int *nauxK)
{
    if (!c) return RIS_E_INVALID;
    c->err.clear();
    if (!mol || !opts || !mol->Z || !mol->xyz || !mol->shell_atom || !mol->shell_l || !mol->shell_exp ||
        !opts->radius_bohr)
        return fail(c, RIS_E_INVALID, "null molecule or options pointer");
    if (mol->natm <= 0 || mol->nshell <= 0) return fail(c, RIS_E_INVALID, "empty molecule");
    if (!(opts->theta > 0.0)) return fail(c, RIS_E_INVALID, "theta must be > 0");
    HIPCHK(c, hipSetDevice(c->device));
    free_aux(c);

    const int natm = mol->natm, nsh = mol->nshell;
    for (int a = 0; a < natm; ++a) {
        const int z = mol->Z[a];
        if (z < 1 || z > 118) return fail(c, RIS_E_INVALID, "atom %d: Z=%d out of range", a, z);
        if (!(opts->radius_bohr[z] > 0.0)) return fail(c, RIS_E_INVALID, "no radius for Z=%d", z);
    }
    for (int s = 0; s < nsh; ++s) {
        if (mol->shell_atom[s] < 0 || mol->shell_atom[s] >= natm)
            return fail(c, RIS_E_INVALID, "shell %d: atom index out of range", s);
        if (mol->shell_l[s] < 0) return fail(c, RIS_E_INVALID, "shell %d: negative l", s);
        if (mol->shell_l[s] > kMaxAOL) return fail(c, RIS_E_UNSUPPORTED, "shell %d: l=%d > 2", s, mol->shell_l[s]);
        if (!(mol->shell_exp[s] > 0.0)) return fail(c, RIS_E_INVALID, "shell %d: exponent must be > 0", s);
    }

    // --- AO shells sorted by l (stable), internal function offsets, permutation
    std::vector<int> caller_off(nsh + 1, 0);
    for (int s = 0; s < nsh; ++s) caller_off[s + 1] = caller_off[s] + ncart(mol->shell_l[s]);
    const int nao = caller_off[nsh];
    // AO function order of every matrix: atoms in reverse Cuthill-McKee order
    // (each atom's shells in the caller's order), so that the shell pairs the
    // screen keeps, and the 128 x 128 tiles of Gamma^P that hold them, gather
    // near the diagonal.  The kernels' shell tables are sorted by l, and within
    // one l by that atom order, so consecutive shells of a class have
    // increasing first functions (writes and partner reads stay local).
    std::vector<int> fofs(nsh, 0), order;
    {
        const std::vector<int> ord = atom_band_order(mol);
        std::vector<std::vector<int>> by_atom(natm);
        for (int s = 0; s < nsh; ++s) by_atom[mol->shell_atom[s]].push_back(s);
        int g = 0;
        for (int a : ord)
            for (int s : by_atom[a]) {
                fofs[s] = g;
                g += ncart(mol->shell_l[s]);
            }
        for (int l = 0; l <= kMaxAOL; ++l) {
            c->ao.lbeg[l] = (int)order.size();
            for (int a : ord)
                for (int s : by_atom[a])
                    if (mol->shell_l[s] == l) order.push_back(s);
        }
        c->ao.lbeg[kMaxAOL + 1] = nsh;
    }
    std::vector<double> x(nsh), y(nsh), z(nsh), e(nsh), nr(nsh);
    std::vector<int> at(nsh), off(nsh + 1);
    c->h_ao_perm.assign(nao, 0);
    std::vector<int> off_int(nsh + 1, 0);
    c->h_ao_perm_int.assign(nao, 0);
    for (int i = 0, g = 0; i < nsh; ++i) {
        const int sc = order[i], l = mol->shell_l[sc];
        off_int[i] = g;
        for (int k = 0; k < ncart(l); ++k) c->h_ao_perm_int[g + k] = caller_off[sc] + k;
        g += ncart(l);
    }
    off_int[nsh] = nao;
    for (int i = 0; i < nsh; ++i) {
        const int s = order[i], a = mol->shell_atom[s], l = mol->shell_l[s];
        x[i] = mol->xyz[3 * a];
        y[i] = mol->xyz[3 * a + 1];
        z[i] = mol->xyz[3 * a + 2];
        e[i] = mol->shell_exp[s];
        nr[i] = radial_norm(e[i], l);
        at[i] = a;
        off[i] = fofs[s];
        for (int k = 0; k < ncart(l); ++k) c->h_ao_perm[fofs[s] + k] = caller_off[s] + k;
    }
    int f = nao;
    off[nsh] = nao;
    c->h_sh_off = off;
    c->h_sh_xyz.resize(3 * (size_t)nsh);
    for (int i = 0; i < nsh; ++i) {
        c->h_sh_xyz[3 * i] = x[i];
        c->h_sh_xyz[3 * i + 1] = y[i];
        c->h_sh_xyz[3 * i + 2] = z[i];
    }
    c->h_sh_exp = e;
    c->ao.nshell = nsh;
    c->ao.nao = nao;
    c->h_ao_atom = at;

    // --- auxiliary J set: s on every atom, then p on heavy atoms (same exponent)
    std::vector<int> js_atom, jl;
    for (int a = 0; a < natm; ++a) js_atom.push_back(a), jl.push_back(0);
    if (opts->j_p_on_heavy)
        for (int a = 0; a < natm; ++a)
            if (mol->Z[a] > 1) js_atom.push_back(a), jl.push_back(1);
    const int nshJ = (int)js_atom.size();
    std::vector<double> ax(nshJ), ay(nshJ), az(nshJ), ae(nshJ), anr(nshJ);
    std::vector<int> aat(nshJ), aoff(nshJ + 1);
    f = 0;
    for (int i = 0; i < nshJ; ++i) {
        const int a = js_atom[i];
        const double R = opts->radius_bohr[mol->Z[a]];
        ax[i] = mol->xyz[3 * a];
        ay[i] = mol->xyz[3 * a + 1];
        az[i] = mol->xyz[3 * a + 2];
        ae[i] = opts->theta / (R * R);
        anr[i] = radial_norm(ae[i], jl[i]);
        aat[i] = a;
        aoff[i] = f;
        f += ncart(jl[i]);
    }
    aoff[nshJ] = f;
    // one region for the tables, the permutation and the metric matrices
    {
        const AuxLayout AL = aux_layout(nsh, nshJ, nao, f, natm);
        int st0;
        char *base = pool_get(c, c->aux_pool, AL.total, &st0);
        if (!base) return st0;
        int st1 = upload_shells(c, nsh, x, y, z, e, nr, at, off, base + AL.oAO, &c->ao.sh);
        if (st1) return st1;
        st1 = upload_shells(c, nshJ, ax, ay, az, ae, anr, aat, aoff, base + AL.oAX, &c->aux.sh);
        if (st1) return st1;
        c->d_ao_perm = (int *)(base + AL.oP);
        c->d_ao_perm_int = (int *)(base + AL.oPJ);
        HIPCHK(c, hipMemcpyAsync(base + AL.oOI, off_int.data(), 4 * (size_t)(nsh + 1), hipMemcpyHostToDevice,
                                 c->stream));
        c->ao_int = c->ao;  // the same shells, first functions in the integral order
        c->ao_int.sh.off = (const int *)(base + AL.oOI);
        c->MJ = (double *)(base + AL.oMJ);
        c->LinvJ = (double *)(base + AL.oLJ);
        c->MinvJ = (double *)(base + AL.oIJ);
        c->MinvK = (double *)(base + AL.oIK);
        c->d_pair_ptr = (int *)(base + AL.oPP);
        c->d_pair_idx = (int *)(base + AL.oPI);
        c->d_pair_gq = (int *)(base + AL.oPQ);
        c->d_pk_ptr = c->d_pair_gq + (size_t)nsh * nsh;
        c->d_pk_sb = c->d_pk_ptr + nsh + 1;
        c->d_pk_base = c->d_pk_sb + (size_t)nsh * (nsh + 1) / 2;
        c->d_pc_ptr = c->d_pk_base + (size_t)nsh * (nsh + 1) / 2;
        c->d_pc_cn = c->d_pc_ptr + nsh + 1;
        c->d_pc_qb = c->d_pc_cn + (size_t)nsh * nao;
        c->d_gtiles = (int *)(base + AL.oGT);
    }
    c->aux.nshell = nshJ;
    c->aux.nfunc = f;
    c->auxl_beg[0] = 0;
    c->auxl_beg[1] = natm;
    c->auxl_beg[2] = nshJ;
    c->h_aux_atom = aat;
    c->h_aux_off = aoff;
    c->natm = natm;
    c->nao = nao;
    c->nshAO = nsh;
    c->nJ = f;
    c->nK = natm;
    c->nshJ = nshJ;
    c->nsJ = natm;

    HIPCHK(c, hipMemcpyAsync(c->d_ao_perm, c->h_ao_perm.data(), sizeof(int) * nao, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_ao_perm_int, c->h_ao_perm_int.data(), sizeof(int) * nao, hipMemcpyHostToDevice,
                             c->stream));
    {
        const int sp = build_pairs(c);
        if (sp) return sp;
    }

    // --- metric, Cholesky, inverses
    const int nJ = c->nJ, nK = c->nK;
    hipEvent_t t_aux = stage_begin(c);
    HIPCHK(c, launch_int2c(c->aux, c->boys, c->MJ, c->stream));
    // factor a copy (MJ keeps the metric itself)
    HIPCHK(c, hipMemcpyAsync(c->MinvJ, c->MJ, sizeof(double) * nJ * nJ, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, cholesky(c->MinvJ, c->MJ, nJ, c->info, c->stream));
    int info = 0;
    HIPCHK(c, hipMemcpyAsync(&info, c->info, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (info != 0) return fail(c, RIS_E_NOT_PD, "auxiliary metric not positive definite (column %d)", info);
    {
        int stw;
        char *tw = ws_get(c, sizeof(double) * (size_t)kTriBlock * nJ, &stw);
        if (!tw) return stw;
        HIPCHK(c, tri_inverse(c->MinvJ, c->LinvJ, nJ, (double *)tw, c->stream));
    }
    // M_J^-1 = L^-T L^-1 ; M_K = leading nK block, so L_K^-1 = leading block of L_J^-1
    HIPCHK(c, dgemm(gm(nJ, nJ, nJ, true, false, 1.0, c->LinvJ, nJ, c->LinvJ, nJ, 0.0, c->MinvJ, nJ), c->stream));
    HIPCHK(c, dgemm(gm(nK, nK, nK, true, false, 1.0, c->LinvJ, nJ, c->LinvJ, nJ, 0.0, c->MinvK, nK), c->stream));
    stage_end(c, t_aux, RIS_STAGE_AUX, 2.0 * (double)nJ * nJ * nJ + 2.0 * (double)nK * nK * nK, 0.0);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->have_aux = true;
    if (nauxJ) *nauxJ = nJ;
    if (nauxK) *nauxK = nK;
    return RIS_OK;
}

// ------------------------------------------------------------------------
int ris_int3c(ris_ctx *c, const ris_mo *mo, double *dbg)
{
    if (!c) return RIS_E_INVALID;
    c->err.clear();
    if (!c->have_aux) return fail(c, RIS_E_ORDER, "ris_int3c before ris_aux_build");
    if (!mo || !mo->C || !mo->eps) return fail(c, RIS_E_INVALID, "null orbital pointer");
    if (mo->nao != c->nao) return fail(c, RIS_E_INVALID, "nao %d does not match the basis (%d)", mo->nao, c->nao);
    if (mo->nocc <= 0 || mo->nocc >= mo->nmo || mo->nmo > mo->nao)
        return fail(c, RIS_E_INVALID, "need 0 < nocc < nmo <= nao (nocc=%d nmo=%d)", mo->nocc, mo->nmo);
    const int pmode = mo->precision & ~RIS_PREC_TRANSFORMS;
    if (pmode < RIS_FP64 || pmode > RIS_BF16X6)
        return fail(c, RIS_E_UNSUPPORTED, "precision mode %d not built", mo->precision);
    HIPCHK(c, hipSetDevice(c->device));
    free_int3c(c);

    const int N = c->nao, nmo = mo->nmo, o = mo->nocc, v = nmo - o, nJ = c->nJ, nK = c->nK;
    c->nmo = nmo;
    c->nocc = o;
    c->nvir = v;
    c->alphaJ = mo->alpha_J;
    c->cx = mo->c_x;
    c->prec = pmode;
    // arithmetic of the (mu nu|P) -> MO transforms: FP64 unless the flag asks for the mode
    const int tprec = (mo->precision & RIS_PREC_TRANSFORMS) ? pmode : RIS_FP64;
    c->prec_tr = tprec;
    const size_t NN = (size_t)N * N;
    const long vo = (long)v * o;

    const Dims dm = ctx_dims(c);
    const MoLayout ML = mo_layout(dm);
    // auxiliary functions per block: all of them when they fit, else the most
    // that fit beside the kept MO blocks (whole shells, at most 3 functions)
    const size_t other = c->held - c->mo_pool.bytes - c->ws_bytes;  // what stays allocated meanwhile
    const size_t room = c->budget > other + ML.total ? c->budget - other - ML.total : 0;
    const size_t wsroom = std::max(room, c->ws_bytes);
    int nbf = nJ;
    while (nbf > 3 && int3c_ws(dm, nbf).total > wsroom) nbf = std::max(3, (int)(nbf * 0.8));
    if (c->ablock > 0) nbf = std::min(nbf, std::max(3, c->ablock));
    const Int3cWs IW = int3c_ws(dm, nbf);
    if (other + ML.total + std::max(IW.total, c->ws_bytes) > c->budget)
        return fail(c, RIS_E_NOMEM, "int3c needs %.2f GB (persistent %.2f GB); budget %.2f GB, %.2f GB held",
                    (ML.total + IW.total) / 1e9, ML.total / 1e9, c->budget / 1e9, other / 1e9);
    int st;
    {
        char *pb = pool_get(c, c->mo_pool, ML.total, &st);
        if (!pb) return st;
        c->C = (double *)(pb + ML.oC);
        c->eps = (double *)(pb + ML.oE);
        c->aiJ = (double *)(pb + ML.oA);
        c->coo = (double *)(pb + ML.oOO);
        c->cvo = (double *)(pb + ML.oVO);
        c->cvv = (double *)(pb + ML.oVV);
        c->roo = (double *)(pb + ML.oROO);
    }
    char *wsb = ws_get(c, IW.total, &st);
    if (!wsb) return st;
    double *X = (double *)(wsb + IW.oX), *Z = (double *)(wsb + IW.oZ);
    const size_t tmp_el = IW.total / 8;  // the whole region as scratch for the fits

    // C rows into the matrix order of the contraction, and into the integral
    // order of the forward transforms (the kernels' shell order)
    double *Cint = (double *)((char *)c->C - ML.oC + ML.oCI);
    HIPCHK(c, gather_rows(mo->C, c->C, c->d_ao_perm, N, nmo, nmo, c->stream));
    HIPCHK(c, gather_rows(mo->C, Cint, c->d_ao_perm_int, N, nmo, nmo, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->eps, mo->eps, 8 * nmo, hipMemcpyDeviceToDevice, c->stream));

    const double *CO = Cint, *CV = Cint + o;
    const long oo = (long)o * o;
    // blocks of whole J shells [cs0, cs1) = functions [f0, f1); the K set is
    // the leading nK (s) functions, so a block holds K functions only below nK
    std::vector<int> shf(c->nshJ + 1, 0);
    for (int sh = 0; sh < c->nshJ; ++sh) shf[sh + 1] = shf[sh] + (sh < c->auxl_beg[1] ? 1 : 3);
    for (int cs0 = 0; cs0 < c->nshJ;) {
        int cs1 = cs0;
        while (cs1 < c->nshJ && shf[cs1 + 1] - shf[cs0] <= nbf) ++cs1;
        const int f0 = shf[cs0], nb = shf[cs1] - f0, nbk = std::max(0, std::min(f0 + nb, nK) - f0);
        // (mu nu|P) for the block
        hipEvent_t t_int = stage_begin(c);
        HIPCHK(c, launch_int3c(c->ao_int, c->aux, c->auxl_beg, c->boys, X, c->stream, cs0, cs1));
        stage_end(c, t_int, RIS_STAGE_INT3C, 0.0, 8.0 * (double)nb * NN);
        if (dbg) HIPCHK(c, scatter_sq(X, dbg + (size_t)f0 * NN, c->d_ao_perm_int, N, nb, c->stream));
        hipEvent_t t_mo = stage_begin(c);
        // Z^P = X^P C_O  [nb][N][o]
        GemmArgs g = gm(N, o, N, false, false, 1.0, X, N, CO, nmo, 0.0, Z, o);
        g.batch = nb; g.strideA = NN; g.strideB = 0; g.strideC = (long)N * o;
        HIPCHK(c, gemm_mp(g, tprec, c->stream));
        // (ai|P) = C_V^T Z^P  [nJ][v][o]
        g = gm(v, o, N, true, false, 1.0, CV, nmo, Z, o, 0.0, c->aiJ + (size_t)f0 * vo, o);
        g.batch = nb; g.strideA = 0; g.strideB = (long)N * o; g.strideC = vo;
        HIPCHK(c, gemm_mp(g, tprec, c->stream));
        if (nbk > 0) {
            // raw (ij|P) = C_O^T Z^P of the exchange set  [nK][o][o]
            g = gm(o, o, N, true, false, 1.0, CO, nmo, Z, o, 0.0, c->roo + (size_t)f0 * oo, o);
            g.batch = nbk; g.strideA = 0; g.strideB = (long)N * o; g.strideC = oo;
            HIPCHK(c, gemm_mp(g, tprec, c->stream));
            // raw (ab|P) = C_V^T (X^P C_V) into the c_vv storage as [a][P][b]
            g = gm(N, v, N, false, false, 1.0, X, N, CV, nmo, 0.0, Z, v);
            g.batch = nbk; g.strideA = NN; g.strideB = 0; g.strideC = (long)N * v;
            HIPCHK(c, gemm_mp(g, tprec, c->stream));
            g = gm(v, v, N, true, false, 1.0, CV, nmo, Z, v, 0.0, c->cvv + (size_t)f0 * v, (long)nK * v);
            g.batch = nbk; g.strideA = 0; g.strideB = (long)N * v; g.strideC = v;
            g.lower = true;  // (ab|P) is symmetric in a, b: lower tiles, then mirrored
            HIPCHK(c, gemm_mp(g, tprec, c->stream));
            HIPCHK(c, mirror_lower(c->cvv + (size_t)f0 * v, v, (long)nK * v, v, nbk, c->stream));
        }
        stage_end(c, t_mo, RIS_STAGE_MO,
                  2.0 * nb * ((double)N * N * o + (double)N * v * o) +
                      2.0 * nbk * ((double)N * o * o + (double)N * N * v + (double)N * v * v),
                  0.0);
        cs0 = cs1;
    }
    hipEvent_t t_fit = stage_begin(c);
    double *tmp = (double *)wsb;
    // c_oo = M_K^-1 (ij|.)
    HIPCHK(c, dgemm(gm(nK, (int)oo, nK, false, false, 1.0, c->MinvK, nK, c->roo, oo, 0.0, c->coo, oo), c->stream));
    // c_vv[a] = M_K^-1 (a.|.) in place, rows a in chunks through the scratch
    {
        const int ac = (int)std::max<size_t>(1, std::min<size_t>(v, tmp_el / ((size_t)nK * v)));
        for (int a0 = 0; a0 < v; a0 += ac) {
            const int na = std::min(ac, v - a0);
            double *blk = c->cvv + (size_t)a0 * nK * v;
            GemmArgs g = gm(nK, v, nK, false, false, 1.0, c->MinvK, nK, blk, v, 0.0, tmp, v);
            g.batch = na; g.strideA = 0; g.strideB = (long)nK * v; g.strideC = (long)nK * v;
            HIPCHK(c, dgemm(g, c->stream));
            HIPCHK(c, hipMemcpyAsync(blk, tmp, (size_t)na * nK * v * 8, hipMemcpyDeviceToDevice, c->stream));
        }
    }
    // c_vo[a] = M_K^-1 (a.|.) of the exchange set as [a][P][j], rows a in chunks
    {
        const int ac = (int)std::max<size_t>(1, std::min<size_t>(v, tmp_el / ((size_t)nK * o)));
        for (int a0 = 0; a0 < v; a0 += ac) {
            const int na = std::min(ac, v - a0);
            HIPCHK(c, permute3(c->aiJ + (size_t)a0 * o, tmp, na, nK, o, o, vo, 1, (long)nK * o, o, 1, c->stream));
            GemmArgs g = gm(nK, o, nK, false, false, 1.0, c->MinvK, nK, tmp, o, 0.0, c->cvo + (size_t)a0 * nK * o, o);
            g.batch = na; g.strideA = 0; g.strideB = (long)nK * o; g.strideC = (long)nK * o;
            HIPCHK(c, dgemm(g, c->stream));
        }
    }
    stage_end(c, t_fit, RIS_STAGE_MO, 2.0 * (double)nK * nK * ((double)o * o + (double)v * o + (double)v * v), 0.0);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->have_int3c = true;
    return RIS_OK;
}

// ------------------------------------------------------------------------
// Parts per element of the split-BF16 modes (0: no planes)
static int plane_parts(const ris_ctx *c)
{
    return c->prec == RIS_BF16X3 ? 2 : c->prec == RIS_BF16X6 ? 3 : 0;
}

// Argument checks shared by both matvec entry points.
static int matvec_check(ris_ctx *c, int op, int nvec, const double *V, double *out)
{
    if (!c) return RIS_E_INVALID;
    c->err.clear();
    if (!c->have_int3c) return fail(c, RIS_E_ORDER, "ris_response_matvec before ris_int3c");
    if (op < RIS_OP_A || op > RIS_OP_AMB) return fail(c, RIS_E_INVALID, "unknown operator %d", op);
    if (nvec < 0) return fail(c, RIS_E_INVALID, "nvec < 0");
    if (nvec == 0) return RIS_OK;
    if (!V || !out || V == out) return fail(c, RIS_E_INVALID, "null or aliased vector pointer");
    return RIS_OK;
}

// The matvec itself on the scratch wsb (laid out by matvec_ws(nvec, chunk)).
// timed: bracket it with the stage events (the allocation-free entry point
// records none, so it creates no events either).
static int matvec_run(ris_ctx *c, int op, int nvec, const double *V, double *out, char *wsb, int chunk, bool timed)
{
    const int o = c->nocc, v = c->nvir, nJ = c->nJ, nK = c->nK;
    const long vo = (long)v * o, oo = (long)o * o;
    // coefficients of Delta, J, K_A, K_B for A, B, A+B, A-B
    static const double cDe[4] = {1, 0, 1, 1}, cJ[4] = {1, 1, 2, 0}, cKA[4] = {1, 0, 1, 1}, cKB[4] = {0, 1, 1, -1};
    const MatvecWs MW = matvec_ws(ctx_dims(c), nvec, chunk);
    double *t = (double *)(wsb + MW.ot), *cc = t + (size_t)nvec * nJ, *T = (double *)(wsb + MW.oT),
           *U = (double *)(wsb + MW.oU), *SKm = (double *)(wsb + MW.oSK);
    hipEvent_t t_mv = timed ? stage_begin(c) : nullptr;
    // Coulomb: t = V (ai|P)^T (tiny output, K = nvir*nocc: split-K) ; cc = t M_J^-1 ; out = cJ alpha_J cc (ai|P)
    HIPCHK(c, dgemm_splitk(gm(nvec, nJ, (int)vo, false, true, 1.0, V, vo, c->aiJ, vo, 0.0, t, nJ), kSplitV, SKm,
                           c->stream));
    HIPCHK(c, dgemm(gm(nvec, nJ, nJ, false, false, 1.0, t, nJ, c->MinvJ, nJ, 0.0, cc, nJ), c->stream));
    HIPCHK(c, dgemm(gm(nvec, (int)vo, nJ, false, false, cJ[op] * c->alphaJ, cc, nJ, c->aiJ, vo, 0.0, out, vo),
                    c->stream));
    if (cDe[op] != 0.0) HIPCHK(c, add_de(c->eps, V, out, v, o, nvec, cDe[op], c->stream));
    // K-split of U within the partials region (sized in matvec_ws for full chunks)
    const size_t skcap = std::max((size_t)kSplitV * nvec * nJ, (size_t)matvec_u_splits(ctx_dims(c), chunk) * v * chunk * o);
    for (int k0 = 0; k0 < nvec; k0 += chunk) {
        const int nv = std::min(chunk, nvec - k0);
        const int usplit = (int)std::min((size_t)matvec_u_splits(ctx_dims(c), nv), skcap / ((size_t)v * nv * o));
        const double *Vk = V + (size_t)k0 * vo;
        double *ok = out + (size_t)k0 * vo;
        const long nvo = (long)nv * o;  // columns (k, i) of the chunk
        // the exchange terms pair the fitted c^P of one index pair with the raw
        // (pq|P) of the other: sum_PQ (pq|P) (M_K^-1)_PQ (rs|Q) = sum_P c^P_pq (rs|P)
        if (cKA[op] != 0.0) {
            // T[P][b][k][i] = sum_j V_k[b][j] (ij|P); in the split modes on bf16
            // planes of V's chunk and of (ij|P) (both k-fast), formed in the
            // split-K region, which the U product below only fills afterwards
            const int np = plane_parts(c);
            const long ldo = plane_ld(o);
            const size_t pr = (size_t)nK * o * ldo, pv = (size_t)nv * v * ldo;
            if (np && (pr + pv) * 2 * np <= skcap * 8 && (long)pr * 2 < (1L << 32) && (long)pv * 2 < (1L << 32)) {
                uint16_t *PR = (uint16_t *)SKm, *PV = PR + pr * np;
                HIPCHK(c, split_planes(c->roo, nK * o, o, o, 0, 1, PR, (long)pr, 0, np, c->stream));
                HIPCHK(c, split_planes(Vk, nv * v, o, o, 0, 1, PV, (long)pv, 0, np, c->stream));
                for (int k = 0; k < nv; ++k) {
                    PGemmArgs p{};
                    p.M = v; p.N = o; p.K = (int)ldo; p.ns = np;
                    p.A = PV + (size_t)k * v * ldo; p.lda = ldo; p.psA = (long)pv; p.sA = 0;
                    p.B = PR; p.ldb = ldo; p.psB = (long)pr; p.sB = (long)o * ldo;
                    p.alpha = 1.0;
                    p.C = T + (size_t)k * o; p.ldc = nvo; p.sC = (long)v * nvo;
                    p.batch = nK;
                    HIPCHK(c, pgemm(p, c->stream));
                }
            } else {
                for (int k = 0; k < nv; ++k) {
                    GemmArgs g = gm(v, o, o, false, true, 1.0, Vk + k * vo, o, c->roo, o, 0.0, T + (size_t)k * o, nvo);
                    g.batch = nK; g.strideA = 0; g.strideB = oo; g.strideC = (long)v * nvo;
                    HIPCHK(c, gemm_mp(g, c->prec, c->stream));
                }
            }
            // U[a][(k,i)] = sum_{(P,b)} c^P_ab T[(P,b)][(k,i)];  out_k[a][i] -= c_x U[a][k][i]
            HIPCHK(c, gemm_splitk(gm(v, (int)nvo, nK * v, false, false, 1.0, c->cvv, (long)nK * v, T, nvo, 0.0, U, nvo),
                                  c->prec, usplit, SKm, c->stream));
            HIPCHK(c, permute3(U, ok, nv, v, o, o, nvo, 1, vo, o, 1, c->stream, -cKA[op] * c->cx, 1.0));
        }
        if (cKB[op] != 0.0) {
            // S[P][j][k][i] = sum_b V_k[b][j] (bi|P)
            for (int k = 0; k < nv; ++k) {
                GemmArgs g = gm(o, o, v, true, false, 1.0, Vk + k * vo, o, c->aiJ, o, 0.0, T + (size_t)k * o, nvo);
                g.batch = nK; g.strideA = 0; g.strideB = vo; g.strideC = (long)o * nvo;
                HIPCHK(c, gemm_mp(g, c->prec, c->stream));
            }
            // U[a][(k,i)] = sum_{(P,j)} c^P_aj S[(P,j)][(k,i)];  out_k[a][i] -= c_x U[a][k][i]
            HIPCHK(c, gemm_splitk(gm(v, (int)nvo, nK * o, false, false, 1.0, c->cvo, (long)nK * o, T, nvo, 0.0, U, nvo),
                                  c->prec, usplit, SKm, c->stream));
            HIPCHK(c, permute3(U, ok, nv, v, o, o, nvo, 1, vo, o, 1, c->stream, -cKB[op] * c->cx, 1.0));
        }
    }
    {
        const double fJ = 4.0 * (double)vo * nJ + 2.0 * (double)nJ * nJ;
        const double fA = 2.0 * nK * ((double)v * o * o + (double)v * v * o);
        const double fB = 4.0 * nK * (double)v * o * o;
        stage_end(c, t_mv, RIS_STAGE_MATVEC,
                  nvec * ((cJ[op] != 0 ? fJ : 0.0) + (cKA[op] != 0 ? fA : 0.0) + (cKB[op] != 0 ? fB : 0.0)), 0.0);
    }
    return RIS_OK;
}

int ris_response_matvec(ris_ctx *c, int op, int nvec, const double *V, double *out)
{
    int st = matvec_check(c, op, nvec, V, out);
    if (st != RIS_OK || nvec == 0) return st;
    HIPCHK(c, hipSetDevice(c->device));
    // vectors per exchange chunk: as many (up to kMatvecChunk) as the budget allows
    const size_t other = c->held - c->ws_bytes;
    const size_t wsroom = std::max(c->budget > other ? c->budget - other : 0, c->ws_bytes);
    int chunk = std::min(nvec, kMatvecChunk);
    while (chunk > 1 && matvec_ws(ctx_dims(c), nvec, chunk).total > wsroom) --chunk;
    char *wsb = ws_get(c, matvec_ws(ctx_dims(c), nvec, chunk).total, &st);
    if (!wsb) return st;
    st = matvec_run(c, op, nvec, V, out, wsb, chunk, true);
    if (st != RIS_OK) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RIS_OK;
}

int ris_response_matvec_noalloc(ris_ctx *c, int op, int nvec, const double *V, double *out)
{
    int st = matvec_check(c, op, nvec, V, out);
    if (st != RIS_OK || nvec == 0) return st;
    if (!c->scratch_dev) return fail(c, RIS_E_DEVICE, "fixed scratch of the device was not resolved");
    HIPCHK(c, hipSetDevice(c->device));
    // the largest exchange chunk whose scratch fits the fixed array
    int chunk = std::min(nvec, kMatvecChunk);
    while (chunk > 1 && matvec_ws(ctx_dims(c), nvec, chunk).total > kNoAllocScratchBytes) --chunk;
    const size_t need = matvec_ws(ctx_dims(c), nvec, chunk).total;
    if (need > kNoAllocScratchBytes)
        return fail(c, RIS_E_NOMEM,
                    "ris_response_matvec_noalloc: %d vectors need %zu bytes of scratch; the fixed scratch holds %zu "
                    "(use fewer vectors or ris_response_matvec)",
                    nvec, need, kNoAllocScratchBytes);
    // every buffer of the matvec is written before it is read: nothing to clear
    return matvec_run(c, op, nvec, V, out, (char *)c->scratch_dev, chunk, false);
}

// The reduced-precision copy of the per-state factors F (ns x N x 3o): float
// in the FP32 mode, bf16 planes (part stride ns N plane_ld(3o)) in the split modes.
static hipError_t reduced_f(ris_ctx *c, const double *F, int ns, float *Ff)
{
    const long o3 = 3L * c->nocc, N = c->nao, ldp = plane_ld(o3);
    if (c->prec == RIS_FP32) return to_float(F, Ff, (size_t)ns * N * o3, c->stream);
    if (const int np = plane_parts(c))
        return split_planes(F, (int)N, (int)o3, o3, N * o3, ns, (uint16_t *)Ff, ns * N * ldp, N * ldp, np, c->stream);
    return hipSuccess;
}

// state s of reduced_f's copy
static const float *f_state(const ris_ctx *c, const float *Ff, int s)
{
    const long o3 = 3L * c->nocc, N = c->nao;
    if (plane_parts(c)) return (const float *)((const uint16_t *)Ff + s * N * plane_ld(o3));
    return Ff + s * N * o3;
}

// W^P for nP exchange functions: FP64 (W) in the FP64 mode, float (Wf) in the
// FP32 mode, planes of W^P transposed (in Wf's region) in the split modes.
static hipError_t assemble_w(ris_ctx *c, const BlockGrid &gw, double *W, float *Wf, int nP)
{
    const int o = c->nocc;
    if (c->prec == RIS_FP64) return assemble3(gw, W, o, nP, c->stream, nullptr);
    if (c->prec == RIS_FP32) return assemble3(gw, nullptr, o, nP, c->stream, Wf);
    const long o3 = 3L * o;
    return assemble3_planes(gw, (uint16_t *)Wf, o, nP, nP * o3 * plane_ld(o3), plane_parts(c), c->stream);
}

// Planes the split modes keep from the per-state stage for the H_UU products:
// (R,L)^T (w2 rows (t,s,i), k = a) and, per P, Tall^P^T (w2 rows (t,s,j),
// k = a, P stride w2 ld), both of leading dimension ld with parts prl / ptall
// apart.  tall == nullptr: the stage ran on FP64 or float operands.
struct StatePlanes {
    const uint16_t *rl = nullptr, *tall = nullptr;
    long ld = 0, prl = 0, ptall = 0;
};

// The per-state products of the split modes on bf16 planes:
//   Tall^P[(t,s,j)][a] = sum_b (R,L)_s[b][j] c_vv^P[a][b]   (as planes, for H_UU),
//   HOU[(P,i)][(t,s,j)] = sum_b c_vo^P[b][i] (R,L)_s[b][j]   (FP64).
// c_vv (rows (a,P), k = b), c_vo^T and (R,L)^T are split into the scratch
// (room bytes, free during this stage), except (R,L)^T, which goes with the
// Tall planes into Tall's region (tallroom bytes; H_UU reads both later), and
// multiplied by the plane kernel, whose staging schedule runs these K = v
// products at a higher rate than splitting the FP64 operands inside the loop.
// Returns false, having done nothing, when the mode keeps FP64 or FP32
// operands or the planes do not fit (the caller then takes gemm_mp).
static bool state_products_on_planes(ris_ctx *c, int v, int o, int nK, long w2, const double *RLT, char *tallreg,
                                     size_t tallroom, double *HOU, char *scratch, size_t room, StatePlanes *sp,
                                     hipError_t *err)
{
    *err = hipSuccess;
    const int np = plane_parts(c);
    if (!np || v <= 0 || o <= 0 || nK <= 0 || w2 <= 0) return false;
    const long ldp = plane_ld(v), rows = (long)v * nK, rows2 = (long)nK * o;
    const size_t bA = (size_t)rows * ldp * 2 * np, bA2 = (size_t)rows2 * ldp * 2 * np, bB = (size_t)w2 * ldp * 2 * np;
    const size_t bTP = (size_t)nK * w2 * ldp * 2 * np;
    const size_t bT = (size_t)std::max(rows2, w2) * v * 8;  // FP64 staging of c_vo^T, then of (R,L)^T
    // the plane kernel's 32-bit row offsets (c_vv's rows of one P lie nK rows apart) and int sizes
    if (bA + bA2 + bT > room || bTP + bB > tallroom || rows * ldp * 2 >= (1L << 32) ||
        rows2 * ldp * 2 >= (1L << 32) || rows >= (1L << 31) || w2 >= (1L << 31))
        return false;
    uint16_t *PA = (uint16_t *)scratch, *PA2 = PA + (size_t)rows * ldp * np;
    double *XT = (double *)(PA2 + (size_t)rows2 * ldp * np);
    uint16_t *TP = (uint16_t *)tallreg, *PB = TP + (size_t)nK * w2 * ldp * np;
    // stream order keeps the two uses of XT apart
    hipError_t e = split_planes(c->cvv, (int)rows, v, v, 0, 1, PA, rows * ldp, 0, np, c->stream);
    if (e == hipSuccess) e = transpose(c->cvo, rows2, XT, v, v, (int)rows2, c->stream);
    if (e == hipSuccess) e = split_planes(XT, (int)rows2, v, v, 0, 1, PA2, rows2 * ldp, 0, np, c->stream);
    if (e == hipSuccess) e = transpose(RLT, w2, XT, v, v, (int)w2, c->stream);
    if (e == hipSuccess) e = split_planes(XT, (int)w2, v, v, 0, 1, PB, w2 * ldp, 0, np, c->stream);
    if (e == hipSuccess) {
        // batch P: (R,L)^T against c_vv's rows (a, P), written as planes with
        // the padding columns [v, ldp) zero
        PGemmArgs p{};
        p.M = (int)w2; p.N = v; p.K = (int)ldp; p.ns = np;
        p.A = PB; p.lda = ldp; p.psA = w2 * ldp; p.sA = 0;
        p.B = PA; p.ldb = (long)nK * ldp; p.psB = rows * ldp; p.sB = ldp;
        p.alpha = 1.0;
        p.Cp = TP; p.ldc = ldp; p.psC = (long)nK * w2 * ldp; p.sC = w2 * ldp;
        p.batch = nK;
        e = pgemm(p, c->stream);
    }
    if (e == hipSuccess) {
        PGemmArgs p{};
        p.M = (int)rows2; p.N = (int)w2; p.K = (int)ldp; p.ns = np;
        p.A = PA2; p.lda = ldp; p.psA = rows2 * ldp;
        p.B = PB; p.ldb = ldp; p.psB = w2 * ldp;
        p.alpha = 1.0;
        p.C = HOU; p.ldc = w2;
        p.batch = 1;
        e = pgemm(p, c->stream);
    }
    sp->rl = PB; sp->tall = TP; sp->ld = ldp; sp->prl = w2 * ldp; sp->ptall = (long)nK * w2 * ldp;
    *err = e;
    return true;
}

// Y^P = F_I W^P and the exchange weights Gamma^P for nP auxiliary functions:
// Gamma^P = -2 c_x Y^P F_I^T (same state) or -c_x (Y^P F_J^T + F_J Y^P^T).
// Only the lower tiles of each symmetric Gamma^P are formed (and the lower
// triangle read).  FI, FJ: the FP64 factors; FfI, FfJ: their
// reduced copies (reduced_f; in the split modes the planes of state I and J,
// part stride fps); W / Wf as assemble_w leaves them; Y3 holds Y^P (FP64,
// float or planes).
static int gamma_products(ris_ctx *c, int N, int o, int nP, const double *FI, const double *FJ, const float *FfI,
                          const float *FfJ, long fps, const double *W, const float *Wf, double *Y3, double *Gk,
                          bool same)
{
    const long o3 = 3L * o, NN = (long)N * N;
    const int np = plane_parts(c);
    // one timed group per GEMM launch; a lower-tile launch does
    // nP N (N + 1) 3o flops and moves Y, F_J (reduced in the reduced modes)
    // and the lower half of Gamma (always double)
    // only the lower tiles that hold a kept AO shell pair (the derivative
    // contraction reads Gamma nowhere else); the flops and bytes counted are
    // those of the lower-triangle elements inside them
    const double fl_low = 2.0 * nP * c->gtile_lower * o3;
    const double ein = c->prec == RIS_FP64 ? 8.0 : np ? 2.0 * np : 4.0;
    const double by_low = ein * ((double)nP * N * o3 + (double)N * o3) + 8.0 * nP * c->gtile_lower;
    if (np) {
        // split modes on the planes: A and B k-fast, K the padded width
        const long ldp = plane_ld(o3), yps = nP * N * ldp;
        const uint16_t *PI = (const uint16_t *)FfI, *PJ = (const uint16_t *)FfJ, *PW = (const uint16_t *)Wf;
        uint16_t *PY = (uint16_t *)Y3;
        PGemmArgs p{};
        p.M = N; p.N = (int)o3; p.K = (int)ldp; p.ns = np;
        p.A = PI; p.lda = ldp; p.psA = fps; p.sA = 0;
        p.B = PW; p.ldb = ldp; p.psB = nP * o3 * ldp; p.sB = o3 * ldp;
        p.alpha = 1.0;
        p.Cp = PY; p.ldc = ldp; p.psC = yps; p.sC = N * ldp;
        p.batch = nP; p.kband = o;
        hipEvent_t t_y = stage_begin(c);
        HIPCHK(c, pgemm(p, c->stream));
        stage_end(c, t_y, RIS_STAGE_YW, 2.0 * (double)nP * N * o3 * o3, 0.0);
        // Y^P F_J^T, and for two states + F_J Y^P^T in the same launch (sym2)
        p = PGemmArgs{};
        p.M = N; p.N = N; p.K = (int)ldp; p.ns = np;
        p.A = PY; p.lda = ldp; p.psA = yps; p.sA = N * ldp;
        p.B = PJ; p.ldb = ldp; p.psB = fps; p.sB = 0;
        p.alpha = (same ? -2.0 : -1.0) * c->cx;
        p.sym2 = !same;
        p.C = Gk; p.ldc = N; p.sC = NN;
        p.batch = nP; p.lower = true; p.tiles = c->d_gtiles; p.ntiles = c->ngtiles;
        hipEvent_t t_g = stage_begin(c);
        HIPCHK(c, pgemm(p, c->stream));
        // the two-product launch reads each operand twice
        stage_end(c, t_g, RIS_STAGE_GAMMA, (same ? 1.0 : 2.0) * fl_low,
                  by_low + (same ? 0.0 : ein * ((double)nP * N * o3 + (double)N * o3)));
        return RIS_OK;
    }
    // FP64 and FP32 modes: F, W and Y as double or float (FP32 rounds them first)
    const bool f32 = c->prec == RIS_FP32;
    float *Y3f = (float *)Y3;
    GemmArgs g = gm(N, (int)o3, (int)o3, false, false, 1.0, FI, o3, W, o3, 0.0, Y3, o3);
    g.batch = nP; g.strideA = 0; g.strideB = o3 * o3; g.strideC = (long)N * o3;
    // W^P (rows / cols [U_R, C_O, U_L]) is zero in its (U_L, U_R) and (U_R, U_L)
    // blocks: column tiles inside the U_R block need rows [0, 2o) of W, those
    // inside the U_L block rows [o, 3o)
    g.kband = o;
    if (f32) {
        g.A = (const double *)FfI;
        g.B = (const double *)Wf;
        g.C = (double *)Y3f;
        g.ftypes = kF32A | kF32B | kF32C;
    }
    hipEvent_t t_y = stage_begin(c);
    HIPCHK(c, gemm_mp(g, c->prec, c->stream));
    stage_end(c, t_y, RIS_STAGE_YW, 2.0 * (double)nP * N * o3 * o3, 0.0);
    if (same) {
        g = gm(N, N, (int)o3, false, true, -2.0 * c->cx, Y3, o3, FJ, o3, 0.0, Gk, N);
        g.batch = nP; g.strideA = (long)N * o3; g.strideB = 0; g.strideC = NN; g.lower = true;
        g.tiles = c->d_gtiles; g.ntiles = c->ngtiles;
        if (f32) {
            g.A = (const double *)Y3f;
            g.B = (const double *)FfJ;
            g.ftypes = kF32A | kF32B;
        }
        hipEvent_t t_g = stage_begin(c);
        HIPCHK(c, gemm_mp(g, c->prec, c->stream));
        stage_end(c, t_g, RIS_STAGE_GAMMA, fl_low, by_low);
    } else {
        g = gm(N, N, (int)o3, false, true, -c->cx, Y3, o3, FJ, o3, 0.0, Gk, N);
        g.batch = nP; g.strideA = (long)N * o3; g.strideB = 0; g.strideC = NN; g.lower = true;
        g.tiles = c->d_gtiles; g.ntiles = c->ngtiles;
        if (f32) {
            g.A = (const double *)Y3f;
            g.B = (const double *)FfJ;
            g.ftypes = kF32A | kF32B;
        }
        hipEvent_t t_g = stage_begin(c);
        HIPCHK(c, gemm_mp(g, c->prec, c->stream));
        stage_end(c, t_g, RIS_STAGE_GAMMA, fl_low, by_low);
        g = gm(N, N, (int)o3, false, true, -c->cx, FJ, o3, Y3, o3, 1.0, Gk, N);
        g.batch = nP; g.strideA = 0; g.strideB = (long)N * o3; g.strideC = NN; g.lower = true;
        g.tiles = f32 ? c->d_gtiles_cm : c->d_gtiles; g.ntiles = c->ngtiles;
        if (f32) {
            g.A = (const double *)FfJ;
            g.B = (const double *)Y3f;
            g.ftypes = kF32A | kF32B;
        }
        t_g = stage_begin(c);
        HIPCHK(c, gemm_mp(g, c->prec, c->stream));
        // the accumulating launch also reads the lower half of Gamma
        stage_end(c, t_g, RIS_STAGE_GAMMA, fl_low, by_low + 8.0 * nP * c->gtile_lower);
    }
    return RIS_OK;
}

// The same contraction with the exchange (K) functions taken in blocks of nb,
// for problems whose all-P intermediates do not fit: one output at a time, and
// for each block Tall^P = c_vv^P (R, L)_J, H_UU^P, W^P, Y^P and Gamma^P, then
// the derivative contraction of the block's auxiliary shells.  The metric
// weights need all P at once; with W^P and H^P written out in their blocks
//   V_PQ = sum_kl H^P_kl W^Q_kl = (G + G^T)_PQ / 4,
//   G_PQ = <H_RUU^P + H_LUU^P, c_oo^Q> + <H_RUO^P, H_ROU^Q> - <H_LUO^P, H_LOU^Q>
// (<.,.> the elementwise inner product over (i, j)), which needs only the
// H_OU blocks of the two states over all P and the block's H_UU.
// The derivative contraction reads the weights of its s-shell classes from
// the compact copy Gc (when the pair blocks are numbered): set the job up for
// it, and fill it from the job's Gamma, densities and Coulomb vectors before
// the launch.
static void set_compact(const ris_ctx *c, DerivJob &job, double *Gc)
{
    if (c->nfq <= 0) return;
    job.gcomp = Gc;
    job.nfq = c->nfq;
    job.lst_ptr = c->d_pair_ptr;
    job.lst_idx = c->d_pair_idx;
    job.lst_gq = c->d_pair_gq;
}
static hipError_t pack_compact(const ris_ctx *c, const DerivJob &job)
{
    return launch_pack_gamma(c->ao, job, PackLists{c->d_pk_ptr, c->d_pk_base, c->d_pc_ptr, c->d_pc_cn, c->d_pc_qb},
                             c->stream);
}

static int contract_pairs_blocked(ris_ctx *c, int nstate, const double *X, const double *Y, int npair,
                                  const int *pI, const int *pJ, double *outg, int nb)
{
    const int N = c->nao, nmo = c->nmo, o = c->nocc, v = c->nvir, nJ = c->nJ, nK = c->nK, natm = c->natm;
    const long vo = (long)v * o, NN = (long)N * N, o3 = 3L * o, oo = (long)o * o;
    const int ns = nstate;
    const long w2 = 2L * ns * o;
    const int nsplit = vpq_splits(nK);
    // doubles in the split-K partials region (the SK region of contract_blk_ws)
    const size_t skcap = std::max((size_t)kSplitV * ns * nJ, (size_t)nsplit * nK * nK);
    if (nK > c->auxl_beg[1]) return fail(c, RIS_E_UNSUPPORTED, "exchange set is not a run of leading s shells");
    const ContractBlkWs CW = contract_blk_ws(ctx_dims(c), ns, nb);
    int st;
    char *wsb = ws_get(c, CW.total, &st);
    if (!wsb) return st;
    auto P_ = [&](size_t off) { return (double *)(wsb + off); };
    double *R = P_(CW.oR), *L = P_(CW.oL), *RLT = P_(CW.oRLT), *F = P_(CW.oF), *D = P_(CW.oD), *tT = P_(CW.otT),
           *cvec = P_(CW.ocv), *HI0 = P_(CW.oHI0), *HI1 = P_(CW.oHI1), *HJ0 = P_(CW.oHJ0), *HJ1 = P_(CW.oHJ1),
           *TR = P_(CW.oTR), *G1 = P_(CW.oG1), *V2 = P_(CW.oV2), *SK = P_(CW.oSK), *p3 = P_(CW.op3),
           *p2 = P_(CW.op2), *shA = P_(CW.oshA), *shC = P_(CW.oshC), *shP = P_(CW.oshP), *Tall = P_(CW.oTall),
           *HUU = P_(CW.oHUU), *W = P_(CW.oW), *Y3 = P_(CW.oY), *G = P_(CW.oG), *Gc = P_(CW.oGc);
    // reduced-precision copies of F and W^P (reduced_f, assemble_w)
    float *Ff = (float *)(wsb + CW.oFf), *Wf = (float *)(wsb + CW.oWf);
    const double *CO = c->C, *CV = c->C + o;

    // ---- per-state factors (as in the unblocked contraction)
    hipEvent_t t_h = stage_begin(c);
    HIPCHK(c, make_rl(X, Y, R, L, (size_t)ns * vo, c->stream));
    HIPCHK(c, permute3(R, RLT, v, ns, o, o, vo, 1, w2, o, 1, c->stream));
    HIPCHK(c, permute3(L, RLT + (size_t)ns * o, v, ns, o, o, vo, 1, w2, o, 1, c->stream));
    {
        GemmArgs g = gm(N, o, v, false, false, 1.0, CV, nmo, R, o, 0.0, F, o3);
        g.batch = ns; g.strideA = 0; g.strideB = vo; g.strideC = (long)N * o3;
        HIPCHK(c, dgemm(g, c->stream));
        g = gm(N, o, v, false, false, 1.0, CV, nmo, L, o, 0.0, F + 2 * o, o3);
        g.batch = ns; g.strideA = 0; g.strideB = vo; g.strideC = (long)N * o3;
        HIPCHK(c, dgemm(g, c->stream));
        for (int s = 0; s < ns; ++s)
            HIPCHK(c, hipMemcpy2DAsync(F + (size_t)s * N * o3 + o, o3 * 8, CO, (size_t)nmo * 8, (size_t)o * 8, N,
                                       hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, reduced_f(c, F, ns, Ff));
        g = gm(N, N, o, false, true, 1.0, F, o3, CO, nmo, 0.0, D, N);
        g.batch = ns; g.strideA = (long)N * o3; g.strideB = 0; g.strideC = NN;
        HIPCHK(c, dgemm(g, c->stream));
        HIPCHK(c, symmetrize(D, N, ns, c->stream));
        HIPCHK(c, dgemm_splitk(gm(ns, nJ, (int)vo, false, true, 1.0, R, vo, c->aiJ, vo, 0.0, tT, nJ), kSplitV, SK,
                               c->stream));
        HIPCHK(c, dgemm(gm(ns, nJ, nJ, false, false, 1.0, tT, nJ, c->MinvJ, nJ, 0.0, cvec, nJ), c->stream));
    }
    stage_end(c, t_h, RIS_STAGE_HBLK, 2.0 * ns * ((double)N * N * o) + 4.0 * ns * (double)N * v * o, 0.0);

    auto blk = [](const double *b, long sP, long si, long sj, double sc) { return BlockSrc{b, sP, si, sj, sc}; };
    auto sc = [](BlockSrc b, double f) { b.scale *= f; return b; };
    const BlockSrc none{nullptr, 0, 0, 0, 0.0};
    // Outputs that share the state J share the per-block Tall^P = c_vv^P (R, L)_J
    // and the H_OU blocks of J: a group holds outputs with one J and at most one
    // other state I (a gradient J with the NAC (I, J), say), up to kMaxOutChunk.
    std::vector<std::vector<int>> groups;
    {
        std::vector<char> done(npair, 0);
        for (int k = 0; k < npair; ++k) {
            if (done[k]) continue;
            const int J = pJ[k];
            int other = pI[k] != J ? pI[k] : -1;
            std::vector<int> gq;
            for (int k2 = k; k2 < npair && (int)gq.size() < kMaxOutChunk; ++k2) {
                if (done[k2] || pJ[k2] != J) continue;
                const int I2 = pI[k2];
                if (I2 != J) {
                    if (other < 0) other = I2;
                    if (I2 != other) continue;
                }
                gq.push_back(k2);
                done[k2] = 1;
            }
            groups.push_back(gq);
        }
    }
    double *Gout = P_(CW.oOut);
    for (const std::vector<int> &gq : groups) {
        const int r = (int)gq.size(), J = pJ[gq[0]];
        int Io = -1;  // the group's state other than J, if any
        for (int q = 0; q < r; ++q)
            if (pI[gq[q]] != J) Io = pI[gq[q]];
        // H_OU^P of a state s and t = R, L: [P][i][j] = sum_b c_vo^P[b][i] (R, L)_s[b][j]
        hipEvent_t t_u = stage_begin(c);
        double *HJt[2] = {HJ0, HJ1}, *HOt[2] = {HI0, HI1};
        for (int t = 0; t < 2; ++t) {
            HIPCHK(c, gemm_mp(gm(nK * o, o, v, true, false, 1.0, c->cvo, (long)nK * o, RLT + (size_t)(t * ns + J) * o,
                                 w2, 0.0, HJt[t], o), c->prec, c->stream));
            if (Io >= 0)
                HIPCHK(c, gemm_mp(gm(nK * o, o, v, true, false, 1.0, c->cvo, (long)nK * o,
                                     RLT + (size_t)(t * ns + Io) * o, w2, 0.0, HOt[t], o), c->prec, c->stream));
        }
        stage_end(c, t_u, RIS_STAGE_HBLK, (Io >= 0 ? 8.0 : 4.0) * (double)nK * o * v * o, 0.0);
        HIPCHK(c, fill(p3, (size_t)c->nshAO * c->nshJ * 3 * kMaxOutChunk * 6, 0.0, c->stream));
        DerivJob job{};
        job.nout = 1;
        job.dens = D;
        job.cvec = cvec;
        job.nJ = nJ;
        job.alphaJ = c->alphaJ;
        job.pair_ptr = c->screen > 0.0 ? c->d_pair_ptr : nullptr;
        job.pair_idx = c->d_pair_idx;
        set_compact(c, job, Gc);
        for (int p0 = 0; p0 < nK; p0 += nb) {
            const int m = std::min(nb, nK - p0);
            hipEvent_t t_b = stage_begin(c);
            for (int t = 0; t < 2; ++t) {
                // Tall^P[a][(t, j)] = sum_b c_vv^P[a][b] (R, L)_J[b][j] for P in the block
                GemmArgs g = gm(v, o, v, false, false, 1.0, c->cvv + (size_t)p0 * v, (long)nK * v,
                                RLT + (size_t)(t * ns + J) * o, w2, 0.0, Tall + (size_t)t * o, 2L * o);
                g.batch = m; g.strideA = v; g.strideB = 0; g.strideC = (long)v * 2 * o;
                HIPCHK(c, gemm_mp(g, c->prec, c->stream));
            }
            stage_end(c, t_b, RIS_STAGE_HBLK, 4.0 * (double)m * v * v * o, 0.0);
            for (int q = 0; q < r; ++q) {
                const int I = pI[gq[q]];
                double *const *HIt = I == J ? HJt : HOt;
                hipEvent_t t_q = stage_begin(c);
                for (int t = 0; t < 2; ++t) {
                    // H_UU^P(t) = (R, L)_I^T Tall^P(t)  (symmetric for a gradient: lower tiles + mirror)
                    GemmArgs g = gm(o, o, v, true, false, 1.0, RLT + (size_t)(t * ns + I) * o, w2, Tall + (size_t)t * o,
                                    2L * o, 0.0, HUU + (size_t)t * m * oo, o);
                    g.batch = m; g.strideA = 0; g.strideB = (long)v * 2 * o; g.strideC = oo;
                    g.lower = I == J;
                    HIPCHK(c, gemm_mp(g, c->prec, c->stream));
                    if (I == J) HIPCHK(c, mirror_lower(HUU + (size_t)t * m * oo, o, o, oo, m, c->stream));
                }
                stage_end(c, t_q, RIS_STAGE_HBLK, 4.0 * (double)m * oo * v, 0.0);
                // exchange weights W^P of the block (rows / cols [U_R, C_O, U_L])
                hipEvent_t t_yw = stage_begin(c);
                const BlockSrc Hoo = blk(c->coo + (size_t)p0 * oo, oo, o, 1, 1.0);
                const BlockSrc HRuo = blk(HIt[0] + (size_t)p0 * oo, oo, 1, o, 1.0);
                const BlockSrc HLuo = blk(HIt[1] + (size_t)p0 * oo, oo, 1, o, 1.0);
                const BlockSrc HRou = blk(HJt[0] + (size_t)p0 * oo, oo, o, 1, 1.0);
                const BlockSrc HLou = blk(HJt[1] + (size_t)p0 * oo, oo, o, 1, 1.0);
                const BlockSrc HRuu = blk(HUU, oo, o, 1, 1.0);
                const BlockSrc HLuu = blk(HUU + (size_t)m * oo, oo, o, 1, 1.0);
                BlockGrid gw{};
                gw.b[0][0][0] = sc(Hoo, 0.25);  gw.b[0][1][0] = sc(HRou, 0.25);  gw.b[0][2][0] = none;
                gw.b[1][0][0] = sc(HRuo, 0.25); gw.b[1][1][0] = sc(HRuu, 0.25);  gw.b[1][2][0] = sc(HLuo, -0.25);
                gw.b[1][1][1] = sc(HLuu, 0.25);
                gw.b[2][0][0] = none;           gw.b[2][1][0] = sc(HLou, -0.25); gw.b[2][2][0] = sc(Hoo, 0.25);
                HIPCHK(c, assemble_w(c, gw, W, Wf, m));
                stage_end(c, t_yw, RIS_STAGE_YW, 0.0, 8.0 * 9.0 * (double)oo * m);
                // G rows of the block: <H_RUU^P + H_LUU^P, c_oo^Q>
                double *G1q = G1 + (size_t)q * nK * nK;
                hipEvent_t t_v = stage_begin(c);
                // K-split for about 1024 workgroups over the block's m x nK tiles, within the partials region
                const long tmn = (long)((m + 127) / 128) * ((nK + 127) / 128);
                const int bsplit = (int)std::max(1L, std::min({256L, 1024L / tmn, (long)(skcap / ((size_t)m * nK))}));
                for (int t = 0; t < 2; ++t)
                    HIPCHK(c, gemm_splitk(gm(m, nK, (int)oo, false, true, 1.0, HUU + (size_t)t * m * oo, oo, c->coo,
                                             oo, t ? 1.0 : 0.0, G1q + (size_t)p0 * nK, nK), c->prec, bsplit, SK,
                                          c->stream));
                stage_end(c, t_v, RIS_STAGE_VPQ, 4.0 * (double)m * nK * oo, 0.0);
                const int rr = gamma_products(c, N, o, m, F + (size_t)I * N * o3, F + (size_t)J * N * o3,
                                              f_state(c, Ff, I), f_state(c, Ff, J), ns * N * plane_ld(o3), W, Wf,
                                              Y3, G, I == J);
                if (rr != RIS_OK) return rr;
                // derivative contraction over the block's (s) shells, Coulomb part
                // included, into the partial slot q of the group
                job.gammaK = G;
                job.nK = m;
                job.kbeg = p0;
                job.partial = p3 + 6 * q;
                for (int u = 0; u < kMaxOutChunk; ++u) {
                    job.stI[u] = I;
                    job.stJ[u] = J;
                }
                hipEvent_t t_d = stage_begin(c);
                if (job.gcomp) HIPCHK(c, pack_compact(c, job));
                HIPCHK(c, launch_int3c_deriv(c->ao, c->aux, c->auxl_beg, c->boys, job, c->stream, p0, p0 + m));
                stage_end(c, t_d, RIS_STAGE_DERIV, 0.0, 8.0 * (double)m * NN);
            }
        }
        for (int q = 0; q < r; ++q) {
            const int I = pI[gq[q]];
            double *const *HIt = I == J ? HJt : HOt;
            job.partial = p3 + 6 * q;
            for (int u = 0; u < kMaxOutChunk; ++u) {
                job.stI[u] = I;
                job.stJ[u] = J;
            }
            // the remaining auxiliary shells carry the Coulomb part only
            if (nK < c->nshJ) {
                job.gammaK = nullptr;
                job.nK = 0;
                job.kbeg = 0;
                hipEvent_t t_d = stage_begin(c);
                HIPCHK(c, launch_int3c_deriv(c->ao, c->aux, c->auxl_beg, c->boys, job, c->stream, nK, c->nshJ));
                stage_end(c, t_d, RIS_STAGE_DERIV, 0.0, 0.0);
            }
            // metric weights: W2 = -alpha_J c_I c_J^T + c_x (G + G^T) / 4
            double *G1q = G1 + (size_t)q * nK * nK, *V2q = V2 + (size_t)q * nJ * nJ;
            hipEvent_t t_v = stage_begin(c);
            // G += <H_RUO^P, H_ROU^Q> - <H_LUO^P, H_LOU^Q>  (H_UO^P[i][j] = H_OU(I)^P[j][i])
            for (int t = 0; t < 2; ++t) {
                HIPCHK(c, permute3(HIt[t], TR, nK, o, o, oo, 1, o, oo, o, 1, c->stream));
                HIPCHK(c, gemm_splitk(gm(nK, nK, (int)oo, false, true, t ? -1.0 : 1.0, TR, oo, HJt[t], oo, 1.0, G1q,
                                         nK), c->prec, nsplit, SK, c->stream));
            }
            HIPCHK(c, dgemm(gm(nJ, nJ, 1, true, false, -c->alphaJ, cvec + (size_t)I * nJ, nJ, cvec + (size_t)J * nJ,
                               nJ, 0.0, V2q, nJ), c->stream));
            HIPCHK(c, add_sym(G1q, nK, V2q, nJ, 0.25 * c->cx, c->stream));
            stage_end(c, t_v, RIS_STAGE_VPQ, 4.0 * (double)nK * nK * oo, 0.0);
        }
        HIPCHK(c, fill(p2, (size_t)c->nshJ * 2 * r * 3, 0.0, c->stream));
        HIPCHK(c, launch_int2c_deriv(c->aux, c->boys, r, V2, p2, c->stream));
        HIPCHK(c, reduce_grad(p3, c->nshAO, c->nshJ, r, kMaxOutChunk, p2, c->ao.sh.atom, c->aux.sh.atom, natm, shA,
                              shC, shP, 1.0, 0, Gout, c->stream));
        for (int q = 0; q < r; ++q)
            HIPCHK(c, hipMemcpyAsync(outg + (size_t)gq[q] * natm * 3, Gout + (size_t)q * natm * 3, 8 * (size_t)natm * 3,
                                     hipMemcpyDeviceToDevice, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RIS_OK;
}

// ------------------------------------------------------------------------
// Gradients / NAC numerators for a list of state pairs (I, J):
//   out[k] = d/dR [ alpha_J sum (mn|ls)_J R^S_I R^S_J - c_x sum (ml|ns)_K (R^S_I R^S_J + L^A_I L^A_J) ]
// with the exchange weights Gamma^P = D_I C^P D_J^T built from the rank-3o
// factors F_s = [C_V R_s, C_O, C_V L_s]: Gamma^P = F_I W^P F_J^T.
static int contract_pairs(ris_ctx *c, int nstate, const double *X, const double *Y, int npair, const int *pI,
                          const int *pJ, double *outg)
{
    HIPCHK(c, hipSetDevice(c->device));
    const int N = c->nao, nmo = c->nmo, o = c->nocc, v = c->nvir, nJ = c->nJ, nK = c->nK, natm = c->natm;
    const long vo = (long)v * o, NN = (long)N * N, o3 = 3L * o, oo = (long)o * o;
    const int ns = nstate;
    const long w2 = 2L * ns * o;  // columns of RLT / Tall: (t, s, i)
    const int NO = kMaxOutChunk;
    const int nsplit = vpq_splits(nK);
    const ContractWs CW = contract_ws(ctx_dims(c), ns);
    {
        // blocked over the exchange functions when forced or when the all-P
        // intermediates do not fit; the largest block that fits otherwise
        const size_t other = c->held - c->ws_bytes;
        const size_t wsroom = std::max(c->budget > other ? c->budget - other : 0, c->ws_bytes);
        if ((c->ablock > 0 && c->ablock < nK) || CW.total > wsroom) {
            int nb = nK;
            while (nb > 1 && contract_blk_ws(ctx_dims(c), ns, nb).total > wsroom) nb = std::max(1, (int)(nb * 0.8));
            // whole 128-row tiles for the block's rows of the Gram matrix
            if (nb > 128) nb = nb / 128 * 128;
            if (c->ablock > 0) nb = std::min(nb, c->ablock);
            return contract_pairs_blocked(c, nstate, X, Y, npair, pI, pJ, outg, nb);
        }
    }
    int st;
    char *wsb = ws_get(c, CW.total, &st);
    if (!wsb) return st;
    auto P_ = [&](size_t off) { return (double *)(wsb + off); };
    double *R = P_(CW.oR), *L = P_(CW.oL), *RLT = P_(CW.oRLT), *F = P_(CW.oF), *D = P_(CW.oD), *tT = P_(CW.otT),
           *cvec = P_(CW.ocv), *Tall = P_(CW.oTall), *HUO = P_(CW.oHUO), *HOU = P_(CW.oHOU), *HUU = P_(CW.oHUU),
           *W = P_(CW.oW), *Hc = P_(CW.oHc), *Y3 = P_(CW.oY), *G = P_(CW.oG), *V2 = P_(CW.oV2), *SK = P_(CW.oSK),
           *p3 = P_(CW.op3), *p2 = P_(CW.op2), *shA = P_(CW.oshA), *shC = P_(CW.oshC), *shP = P_(CW.oshP),
           *Gc = P_(CW.oGc);
    // FP32 and split-BF16 modes: F, W and Y stored as float for the two products
    // that build Gamma (both kernels round the operands to FP32 first: same results)
    // reduced-precision copies of F and W^P (reduced_f, assemble_w)
    float *Ff = (float *)(wsb + CW.oFf), *Wf = (float *)(wsb + CW.oWf);
    const double *CO = c->C, *CV = c->C + o;

    // ---- per-state intermediates
    StatePlanes sp;  // split modes: the planes H_UU reads (none: FP64 or float operands)
    hipEvent_t t_h = stage_begin(c);
    HIPCHK(c, make_rl(X, Y, R, L, (size_t)ns * vo, c->stream));
    // RLT[a][t][s][i] = (R, L)_s[a][i]
    HIPCHK(c, permute3(R, RLT, v, ns, o, o, vo, 1, w2, o, 1, c->stream));
    HIPCHK(c, permute3(L, RLT + (size_t)ns * o, v, ns, o, o, vo, 1, w2, o, 1, c->stream));
    {
        // F_s = [C_V R_s, C_O, C_V L_s]  (N x 3o)
        GemmArgs g = gm(N, o, v, false, false, 1.0, CV, nmo, R, o, 0.0, F, o3);
        g.batch = ns; g.strideA = 0; g.strideB = vo; g.strideC = (long)N * o3;
        HIPCHK(c, dgemm(g, c->stream));
        g = gm(N, o, v, false, false, 1.0, CV, nmo, L, o, 0.0, F + 2 * o, o3);
        g.batch = ns; g.strideA = 0; g.strideB = vo; g.strideC = (long)N * o3;
        HIPCHK(c, dgemm(g, c->stream));
        for (int s = 0; s < ns; ++s)
            HIPCHK(c, hipMemcpy2DAsync(F + (size_t)s * N * o3 + o, o3 * 8, CO, (size_t)nmo * 8, (size_t)o * 8, N,
                                       hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, reduced_f(c, F, ns, Ff));
        // D_s = sym(U_Rs C_O^T) = R^S_s
        g = gm(N, N, o, false, true, 1.0, F, o3, CO, nmo, 0.0, D, N);
        g.batch = ns; g.strideA = (long)N * o3; g.strideB = 0; g.strideC = NN;
        HIPCHK(c, dgemm(g, c->stream));
        HIPCHK(c, symmetrize(D, N, ns, c->stream));
        // c_s = M_J^-1 t_s, t_s[P] = sum_ai (ai|P) R_s[a][i]
        HIPCHK(c, dgemm_splitk(gm(ns, nJ, (int)vo, false, true, 1.0, R, vo, c->aiJ, vo, 0.0, tT, nJ), kSplitV, SK,
                               c->stream));
        HIPCHK(c, dgemm(gm(ns, nJ, nJ, false, false, 1.0, tT, nJ, c->MinvJ, nJ, 0.0, cvec, nJ), c->stream));
        // Tall[(a,P)][(t,s,j)] = sum_b c_vv^P[a][b] (R,L)_s[b][j]
        // HOU[(P,i)][(t,s,j)] = sum_b c_vo^P[b][i] (R,L)_s[b][j]  (= H_OU blocks)
        // (split modes: on planes, Tall transposed per P as planes in its own region, the
        // other operands in Gamma's region, not in use until the exchange weights)
        hipError_t te;
        if (state_products_on_planes(c, v, o, nK, w2, RLT, (char *)Tall, (size_t)v * nK * w2 * 8, HOU, (char *)G,
                                     (size_t)NO * nK * NN * 8, &sp, &te)) {
            HIPCHK(c, te);
        } else {
            HIPCHK(c, gemm_mp(gm(v * nK, (int)w2, v, false, false, 1.0, c->cvv, v, RLT, w2, 0.0, Tall, w2), c->prec,
                              c->stream));
            HIPCHK(c, gemm_mp(gm(nK * o, (int)w2, v, true, false, 1.0, c->cvo, (long)nK * o, RLT, w2, 0.0, HOU, w2),
                              c->prec, c->stream));
        }
        // HUO[(t,s,i)][(P,j)] = HOU[(P,j)][(t,s,i)]  (H_UO^P of a state is the transpose of its H_OU^P)
        HIPCHK(c, transpose(HOU, w2, HUO, (long)nK * o, nK * o, (int)w2, c->stream));
    }
    stage_end(c, t_h, RIS_STAGE_HBLK,
              2.0 * (double)v * nK * w2 * v + 2.0 * (double)w2 * nK * o * v + 2.0 * ns * ((double)N * N * o) +
                  4.0 * ns * (double)N * v * o,
              0.0);

    auto blk = [](const double *b, long sP, long si, long sj, double sc) { return BlockSrc{b, sP, si, sj, sc}; };
    for (int k0 = 0; k0 < npair; k0 += NO) {
        const int nb = std::min(NO, npair - k0);
        DerivJob job{};
        job.nout = nb;
        job.gammaK = G;
        job.nK = nK;
        job.dens = D;
        job.cvec = cvec;
        job.nJ = nJ;
        job.alphaJ = c->alphaJ;
        job.partial = p3;
        job.pair_ptr = c->screen > 0.0 ? c->d_pair_ptr : nullptr;
        job.pair_idx = c->d_pair_idx;
        set_compact(c, job, Gc);
        for (int k = 0; k < NO; ++k) {
            const int kk = k0 + std::min(k, nb - 1);
            job.stI[k] = pI[kk];
            job.stJ[k] = pJ[kk];
        }
        for (int k = 0; k < nb; ++k) {
            const int I = pI[k0 + k], J = pJ[k0 + k];
            hipEvent_t t_u = stage_begin(c);
            // H_UU^P = (R,L)_I^T Tall^P_{(R,L) J}  (symmetric for a gradient: lower tiles + mirror)
            for (int t = 0; t < 2; ++t) {
                if (sp.tall) {
                    PGemmArgs p{};
                    p.M = o; p.N = o; p.K = (int)sp.ld; p.ns = plane_parts(c);
                    p.A = sp.rl + (size_t)(t * ns + I) * o * sp.ld; p.lda = sp.ld; p.psA = sp.prl; p.sA = 0;
                    p.B = sp.tall + (size_t)(t * ns + J) * o * sp.ld; p.ldb = sp.ld; p.psB = sp.ptall;
                    p.sB = w2 * sp.ld;
                    p.alpha = 1.0;
                    p.C = HUU + (size_t)t * nK * oo; p.ldc = o; p.sC = oo;
                    p.batch = nK; p.lower = I == J;
                    HIPCHK(c, pgemm(p, c->stream));
                } else {
                    GemmArgs g = gm(o, o, v, true, false, 1.0, RLT + (size_t)(t * ns + I) * o, w2,
                                    Tall + (size_t)(t * ns + J) * o, (long)nK * w2, 0.0, HUU + (size_t)t * nK * oo, o);
                    g.batch = nK; g.strideA = 0; g.strideB = w2; g.strideC = oo;
                    g.lower = I == J;
                    HIPCHK(c, gemm_mp(g, c->prec, c->stream));
                }
                if (I == J) HIPCHK(c, mirror_lower(HUU + (size_t)t * nK * oo, o, o, oo, nK, c->stream));
            }
            stage_end(c, t_u, RIS_STAGE_HBLK, 4.0 * (double)nK * oo * v, 0.0);
            const BlockSrc Hoo = blk(c->coo, oo, o, 1, 1.0);
            const BlockSrc HRuo = blk(HUO + (size_t)I * o * nK * o, o, (long)nK * o, 1, 1.0);
            const BlockSrc HLuo = blk(HUO + (size_t)(ns + I) * o * nK * o, o, (long)nK * o, 1, 1.0);
            const BlockSrc HRou = blk(HOU + (size_t)J * o, o * w2, w2, 1, 1.0);
            const BlockSrc HLou = blk(HOU + (size_t)(ns + J) * o, o * w2, w2, 1, 1.0);
            const BlockSrc HRuu = blk(HUU, oo, o, 1, 1.0);
            const BlockSrc HLuu = blk(HUU + (size_t)nK * oo, oo, o, 1, 1.0);
            const BlockSrc none{nullptr, 0, 0, 0, 0.0};
            auto sc = [](BlockSrc b, double f) { b.scale *= f; return b; };
            // exchange weights W^P (rows/cols [U_R, C_O, U_L]) from D = (U C_O^T +- C_O U^T)/2
            hipEvent_t t_yw = stage_begin(c);
            BlockGrid gw{};
            gw.b[0][0][0] = sc(Hoo, 0.25);  gw.b[0][1][0] = sc(HRou, 0.25);  gw.b[0][2][0] = none;
            gw.b[1][0][0] = sc(HRuo, 0.25); gw.b[1][1][0] = sc(HRuu, 0.25);  gw.b[1][2][0] = sc(HLuo, -0.25);
            gw.b[1][1][1] = sc(HLuu, 0.25);
            gw.b[2][0][0] = none;           gw.b[2][1][0] = sc(HLou, -0.25); gw.b[2][2][0] = sc(Hoo, 0.25);
            HIPCHK(c, assemble_w(c, gw, W, Wf, nK));
            stage_end(c, t_yw, RIS_STAGE_YW, 0.0, 8.0 * 9.0 * (double)oo * nK);
            hipEvent_t t_v = stage_begin(c);
            // metric weights: W2 = -alpha_J c_I c_J^T + c_x V with V_PQ = sum_kl H^P_kl W^Q_kl
            // = (G + G^T)_PQ / 4, G_PQ = <H_RUU^P + H_LUU^P, c_oo^Q> + <H_RUO^P, H_ROU^Q>
            // - <H_LUO^P, H_LOU^Q> (elementwise inner products over (i, j); the
            // H blocks gathered into [P][i][j] order in the H region)
            double *V2k = V2 + (size_t)k * nJ * nJ;
            double *Ru = Hc, *Rc = Hc + (size_t)nK * oo, *Lu = Hc + 2 * (size_t)nK * oo, *Lc = Hc + 3 * (size_t)nK * oo,
                   *Gm = Hc + 4 * (size_t)nK * oo;
            HIPCHK(c, permute3(HUO + (size_t)I * o * nK * o, Ru, nK, o, o, o, (long)nK * o, 1, oo, o, 1, c->stream));
            HIPCHK(c, permute3(HUO + (size_t)(ns + I) * o * nK * o, Lu, nK, o, o, o, (long)nK * o, 1, oo, o, 1,
                               c->stream));
            HIPCHK(c, permute3(HOU + (size_t)J * o, Rc, nK, o, o, (long)o * w2, w2, 1, oo, o, 1, c->stream));
            HIPCHK(c, permute3(HOU + (size_t)(ns + J) * o, Lc, nK, o, o, (long)o * w2, w2, 1, oo, o, 1, c->stream));
            const double *gA[4] = {HUU, HUU + (size_t)nK * oo, Ru, Lu}, *gB[4] = {c->coo, c->coo, Rc, Lc};
            for (int u = 0; u < 4; ++u)
                HIPCHK(c, gemm_splitk(gm(nK, nK, (int)oo, false, true, u == 3 ? -1.0 : 1.0, gA[u], oo, gB[u], oo,
                                         u ? 1.0 : 0.0, Gm, nK), c->prec, nsplit, SK, c->stream));
            HIPCHK(c, dgemm(gm(nJ, nJ, 1, true, false, -c->alphaJ, cvec + (size_t)I * nJ, nJ, cvec + (size_t)J * nJ,
                               nJ, 0.0, V2k, nJ), c->stream));
            HIPCHK(c, add_sym(Gm, nK, V2k, nJ, 0.25 * c->cx, c->stream));
            stage_end(c, t_v, RIS_STAGE_VPQ, 8.0 * (double)nK * nK * oo, 0.0);
            // Y^P = F_I W^P ; Gamma^P from Y^P and F_J
            double *Gk = G + (size_t)k * nK * NN;
            {
                const int r = gamma_products(c, N, o, nK, F + (size_t)I * N * o3, F + (size_t)J * N * o3,
                                             f_state(c, Ff, I), f_state(c, Ff, J), ns * N * plane_ld(o3), W, Wf,
                                             Y3, Gk, I == J);
                if (r != RIS_OK) return r;
            }
        }
        // three-centre derivative contraction + metric derivative, reduced into atoms
        HIPCHK(c, fill(p3, (size_t)c->nshAO * c->nshJ * 3 * NO * 6, 0.0, c->stream));
        hipEvent_t t_d = stage_begin(c);
        if (job.gcomp) HIPCHK(c, pack_compact(c, job));
        HIPCHK(c, launch_int3c_deriv(c->ao, c->aux, c->auxl_beg, c->boys, job, c->stream));
        stage_end(c, t_d, RIS_STAGE_DERIV, 0.0, 8.0 * (double)nb * nK * NN);
        HIPCHK(c, fill(p2, (size_t)c->nshJ * 2 * nb * 3, 0.0, c->stream));
        HIPCHK(c, launch_int2c_deriv(c->aux, c->boys, nb, V2, p2, c->stream));
        HIPCHK(c, reduce_grad(p3, c->nshAO, c->nshJ, nb, NO, p2, c->ao.sh.atom, c->aux.sh.atom, natm, shA, shC, shP,
                              1.0, 0, outg + (size_t)k0 * natm * 3, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RIS_OK;
}

// ------------------------------------------------------------------------
// Extra density pairs (ris_extra_pair): pair e adds to its output the nuclear
// derivative, at fixed symmetric D1, D2 (internal AO order), of
//   cJ sum (mn|ls)_J D1_mn D2_ls - cK sum (ml|ns)_K D1_mn D2_ls.
// Coulomb: t_x[P] = sum (mn|P) D_x,mn, c_x = M_J^-1 t_x; weights cJ (D1 c2_P + D2 c1_P)
// on (mn|P)^xi and -cJ c1 c2^T on M_J^xi.  Exchange: with C^P = sum_Q (M_K^-1)_PQ (Q|..)
// and X^P = D1 C^P D2, weights -cK (X^P + X^P^T) on (mn|P)^xi and cK V on M_K^xi,
// V_PQ = <X^P, C^Q> = sum_R <X^P, (R|..)> (M_K^-1)_RQ.  The AO integrals are
// recomputed in blocks of whole shells of at most nb functions: once over the
// J shells for t and, per block of exchange functions, once for C^P of the
// block and once per pair for its rows of V (a block already in place is not
// recomputed, so a single block costs one evaluation).
struct ExtraWs {
    size_t oD, ot, oc, ocs, oSK, oV2, oV, oVr, op3, op2, oshA, oshC, oshP, oG, oCb, oUb, oXb, oBq, oGc, total;
};
// K-split of the Gram-type products V = X B^T (m x nq output, K = nao^2): about
// 1024 workgroups over the output tiles
static int extra_vsplit(int m, int n)
{
    const long t = (long)((m + 127) / 128) * ((n + 127) / 128);
    return (int)std::max(1L, std::min(256L, 1024L / t));
}
static ExtraWs extra_ws(const Dims &d, int ne, int nb)
{
    Carve cv;
    ExtraWs L;
    const size_t NN = (size_t)d.N * d.N, NO = kMaxOutChunk;
    L.oD = cv.take((size_t)2 * ne * NN);
    L.ot = cv.take((size_t)2 * ne * d.nJ);
    L.oc = cv.take((size_t)2 * ne * d.nJ);
    L.ocs = cv.take((size_t)2 * ne * d.nJ);
    // split-K partials: t (2ne x nb per range) and V (at most 1024 x 128^2 over all ranges, or nb^2 unsplit)
    L.oSK = cv.take(std::max({(size_t)kSplitV * 2 * ne * nb, (size_t)1024 * 128 * 128, (size_t)nb * nb}));
    L.oV2 = cv.take(NO * d.nJ * d.nJ);
    L.oV = cv.take(NO * d.nK * d.nK);
    L.oVr = cv.take((size_t)nb * d.nK);
    L.op3 = cv.take((size_t)d.nshAO * d.nshJ * 3 * NO * 6);
    L.op2 = cv.take((size_t)d.nshJ * 2 * NO * 3);
    L.oshA = cv.take((size_t)d.nshAO * NO * 3);
    L.oshC = cv.take((size_t)d.nshJ * NO * 3);
    L.oshP = cv.take((size_t)d.nshJ * NO * 3);
    L.oG = cv.take(NO * d.natm * 3);
    L.oCb = cv.take((size_t)nb * NN);
    L.oUb = cv.take((size_t)nb * NN);
    L.oXb = cv.take((size_t)nb * NN);
    L.oBq = cv.take((size_t)nb * NN);
    L.oGc = cv.take((size_t)d.nfq * nb);  // compact copy of a block's exchange weights (one pair)
    L.total = cv.off;
    return L;
}

static int contract_extra(ris_ctx *c, int ne, const ris_extra_pair *ex, const int *eout, double *outg)
{
    const int N = c->nao, nJ = c->nJ, nK = c->nK, natm = c->natm, NO = kMaxOutChunk;
    const long NN = (long)N * N;
    if (nK > c->auxl_beg[1]) return fail(c, RIS_E_UNSUPPORTED, "exchange set is not a run of leading s shells");
    const Dims dm = ctx_dims(c);
    // the largest block of auxiliary functions (at least one p shell) that fits
    const size_t other = c->held - c->ws_bytes;
    const size_t wsroom = std::max(c->budget > other ? c->budget - other : 0, c->ws_bytes);
    int nb = std::max(nK, 3);
    if (c->ablock > 0) nb = std::min(nb, c->ablock);
    nb = std::max(nb, 3);
    while (nb > 3 && extra_ws(dm, ne, nb).total > wsroom) nb = std::max(3, (int)(nb * 0.8));
    const ExtraWs EW = extra_ws(dm, ne, nb);
    int st;
    char *wsb = ws_get(c, EW.total, &st);
    if (!wsb) return st;
    auto P_ = [&](size_t off) { return (double *)(wsb + off); };
    double *Dx = P_(EW.oD), *t = P_(EW.ot), *cr = P_(EW.oc), *cs = P_(EW.ocs), *SK = P_(EW.oSK), *V2 = P_(EW.oV2),
           *Vk = P_(EW.oV), *Vr = P_(EW.oVr), *p3 = P_(EW.op3), *p2 = P_(EW.op2), *shA = P_(EW.oshA),
           *shC = P_(EW.oshC), *shP = P_(EW.oshP), *Gt = P_(EW.oG), *Cb = P_(EW.oCb), *Ub = P_(EW.oUb),
           *Xb = P_(EW.oXb), *Bq = P_(EW.oBq), *Gc = P_(EW.oGc);
    const std::vector<int> &aoff = c->h_aux_off;

    // densities in the internal AO order, symmetrised: Dx[2e] = D1 of pair e, Dx[2e+1] = D2
    for (int e = 0; e < ne; ++e)
        for (int x = 0; x < 2; ++x) {
            double *Dd = Dx + (size_t)(2 * e + x) * NN;
            HIPCHK(c, gather_sq(x ? ex[e].D2 : ex[e].D1, Dd, c->d_ao_perm, N, c->stream));
            HIPCHK(c, symmetrize(Dd, N, 1, c->stream));
        }
    // blocks of whole J shells [a, b) holding at most nb functions
    auto shell_blocks = [&](int s0, int s1) {
        std::vector<std::pair<int, int>> bl;
        for (int a = s0; a < s1;) {
            int b = a + 1;
            while (b < s1 && aoff[b + 1] - aoff[a] <= nb) ++b;
            bl.push_back({a, b});
            a = b;
        }
        return bl;
    };
    // (mn|P) of the J shells [a, b) in Bq (row 0 = first function of shell a)
    int bq_a = -1, bq_b = -1;
    auto int3c_block = [&](int a, int b) -> hipError_t {
        if (a == bq_a && b == bq_b) return hipSuccess;
        bq_a = a;
        bq_b = b;
        return launch_int3c(c->ao, c->aux, c->auxl_beg, c->boys, Bq, c->stream, a, b);
    };

    // Coulomb vectors of every extra density: t = D (mn|P)^T over the J set, c = t M_J^-1
    for (auto [a, b] : shell_blocks(0, c->nshJ)) {
        const int f0 = aoff[a], nf = aoff[b] - aoff[a];
        HIPCHK(c, int3c_block(a, b));
        HIPCHK(c, dgemm_splitk(gm(2 * ne, nf, (int)NN, false, true, 1.0, Dx, NN, Bq, NN, 0.0, t + f0, nJ), kSplitV,
                               SK, c->stream));
    }
    HIPCHK(c, dgemm(gm(2 * ne, nJ, nJ, false, false, 1.0, t, nJ, c->MinvJ, nJ, 0.0, cr, nJ), c->stream));

    DerivJob job{};
    job.dens = Dx;
    job.cvec = cs;
    job.nJ = nJ;
    job.alphaJ = 1.0;  // cJ is carried by the scaled Coulomb vectors cs
    job.pair_ptr = c->screen > 0.0 ? c->d_pair_ptr : nullptr;
    job.pair_idx = c->d_pair_idx;
    set_compact(c, job, Gc);
    const auto kblocks = shell_blocks(0, nK);  // the K functions: the leading s shells, one function each
    for (int e0 = 0; e0 < ne; e0 += NO) {
        const int r = std::min(NO, ne - e0);
        for (int q = 0; q < r; ++q) {
            const int e = e0 + q;
            HIPCHK(c, axpby(cr + (size_t)2 * e * nJ, cs + (size_t)2 * e * nJ, (size_t)2 * nJ, ex[e].cJ, 0.0,
                            c->stream));
        }
        HIPCHK(c, fill(p3, (size_t)c->nshAO * c->nshJ * 3 * NO * 6, 0.0, c->stream));
        for (auto [k0, k1] : kblocks) {
            const int m = k1 - k0;
            // C^P = sum_Q (M_K^-1)_PQ (Q|..) for P in the block
            for (auto [q0, q1] : kblocks) {
                HIPCHK(c, int3c_block(q0, q1));
                HIPCHK(c, dgemm(gm(m, (int)NN, q1 - q0, false, false, 1.0, c->MinvK + (size_t)k0 * nK + q0, nK, Bq,
                                   NN, q0 ? 1.0 : 0.0, Cb, NN), c->stream));
            }
            for (int q = 0; q < r; ++q) {
                const int e = e0 + q;
                const double *D1 = Dx + (size_t)2 * e * NN, *D2 = D1 + NN;
                // X^P = D1 C^P D2
                GemmArgs g = gm(N, N, N, false, false, 1.0, D1, N, Cb, N, 0.0, Ub, N);
                g.batch = m; g.strideA = 0; g.strideB = NN; g.strideC = NN;
                HIPCHK(c, dgemm(g, c->stream));
                g = gm(N, N, N, false, false, 1.0, Ub, N, D2, N, 0.0, Xb, N);
                g.batch = m; g.strideA = NN; g.strideB = 0; g.strideC = NN;
                HIPCHK(c, dgemm(g, c->stream));
                // the block's rows of V: Vr[P][R] = <X^P, (R|..)>, V[P][Q] = sum_R Vr[P][R] (M_K^-1)_RQ
                for (auto [q0, q1] : kblocks) {
                    HIPCHK(c, int3c_block(q0, q1));
                    HIPCHK(c, dgemm_splitk(gm(m, q1 - q0, (int)NN, false, true, 1.0, Xb, NN, Bq, NN, 0.0, Vr + q0, nK),
                                           extra_vsplit(m, q1 - q0), SK, c->stream));
                }
                HIPCHK(c, dgemm(gm(m, nK, nK, false, false, 1.0, Vr, nK, c->MinvK, nK, 0.0,
                                   Vk + ((size_t)q * nK + k0) * nK, nK), c->stream));
                // exchange weights of the block on the lower triangle: -cK (X^P + X^P^T)
                HIPCHK(c, sym_sum_lower(Xb, Ub, N, m, -ex[e].cK, c->stream));
                // derivative contraction over the block's shells, Coulomb part included, into slot q
                job.nout = 1;
                job.gammaK = Ub;
                job.nK = m;
                job.kbeg = k0;
                job.partial = p3 + 6 * q;
                for (int u = 0; u < NO; ++u) {
                    job.stI[u] = 2 * e;
                    job.stJ[u] = 2 * e + 1;
                }
                if (job.gcomp) HIPCHK(c, pack_compact(c, job));
                HIPCHK(c, launch_int3c_deriv(c->ao, c->aux, c->auxl_beg, c->boys, job, c->stream, k0, k1));
            }
        }
        // the remaining (p) shells carry the Coulomb part only
        if (nK < c->nshJ) {
            job.nout = r;
            job.gammaK = nullptr;
            job.nK = 0;
            job.kbeg = 0;
            job.partial = p3;
            for (int u = 0; u < NO; ++u) {
                const int e = e0 + std::min(u, r - 1);
                job.stI[u] = 2 * e;
                job.stJ[u] = 2 * e + 1;
            }
            HIPCHK(c, launch_int3c_deriv(c->ao, c->aux, c->auxl_beg, c->boys, job, c->stream, nK, c->nshJ));
        }
        // metric weights: W2 = -cJ c1 c2^T + cK V (V on the leading K block)
        for (int q = 0; q < r; ++q) {
            const int e = e0 + q;
            double *V2q = V2 + (size_t)q * nJ * nJ;
            HIPCHK(c, dgemm(gm(nJ, nJ, 1, true, false, -ex[e].cJ, cr + (size_t)2 * e * nJ, nJ,
                               cr + (size_t)(2 * e + 1) * nJ, nJ, 0.0, V2q, nJ), c->stream));
            HIPCHK(c, add_sym(Vk + (size_t)q * nK * nK, nK, V2q, nJ, 0.5 * ex[e].cK, c->stream));
        }
        HIPCHK(c, fill(p2, (size_t)c->nshJ * 2 * r * 3, 0.0, c->stream));
        HIPCHK(c, launch_int2c_deriv(c->aux, c->boys, r, V2, p2, c->stream));
        HIPCHK(c, reduce_grad(p3, c->nshAO, c->nshJ, r, NO, p2, c->ao.sh.atom, c->aux.sh.atom, natm, shA, shC, shP,
                              1.0, 0, Gt, c->stream));
        // added into the outputs in pair order (deterministic)
        for (int q = 0; q < r; ++q)
            HIPCHK(c, axpby(Gt + (size_t)q * natm * 3, outg + (size_t)eout[e0 + q] * natm * 3, (size_t)natm * 3, 1.0,
                            1.0, c->stream));
    }
    return RIS_OK;
}

int ris_grad_nac_contract(ris_ctx *c, int nstate, const double *X, const double *Y, int nsel, const int *sel,
                          double *grad, int npair, const int *pairs, const double *omega, double *nac, int nextra,
                          const ris_extra_pair *extra)
{
    if (!c) return RIS_E_INVALID;
    c->err.clear();
    if (!c->have_int3c) return fail(c, RIS_E_ORDER, "gradient/NAC call before ris_int3c");
    if (nstate <= 0 || nsel < 0 || npair < 0 || nextra < 0 || !X || (nsel > 0 && (!sel || !grad)) ||
        (npair > 0 && (!pairs || !nac)) || (nextra > 0 && !extra))
        return fail(c, RIS_E_INVALID, "bad gradient/NAC arguments");
    const int nout = nsel + npair;
    std::vector<int> pI(nout), pJ(nout);
    for (int k = 0; k < nsel; ++k) {
        if (sel[k] < 0 || sel[k] >= nstate) return fail(c, RIS_E_INVALID, "sel[%d]=%d out of range", k, sel[k]);
        pI[k] = pJ[k] = sel[k];
    }
    for (int k = 0; k < npair; ++k) {
        pI[nsel + k] = pairs[2 * k];
        pJ[nsel + k] = pairs[2 * k + 1];
        if (pI[nsel + k] < 0 || pI[nsel + k] >= nstate || pJ[nsel + k] < 0 || pJ[nsel + k] >= nstate)
            return fail(c, RIS_E_INVALID, "pair %d out of range", k);
    }
    std::vector<int> eout(nextra);
    for (int e = 0; e < nextra; ++e) {
        if (extra[e].out < 0 || extra[e].out >= nout)
            return fail(c, RIS_E_INVALID, "extra pair %d names output %d of %d", e, extra[e].out, nout);
        if (!extra[e].D1 || !extra[e].D2) return fail(c, RIS_E_INVALID, "extra pair %d: null density", e);
        if (!std::isfinite(extra[e].cJ) || !std::isfinite(extra[e].cK))
            return fail(c, RIS_E_INVALID, "extra pair %d: coefficient not finite", e);
        eout[e] = extra[e].out;
    }
    if (nout == 0) return RIS_OK;
    int st;
    double *out = nullptr;
    const size_t per = (size_t)c->natm * 3;
    if (nsel > 0 && npair > 0) {
        out = (double *)pool_get(c, c->out_pool, 8 * per * nout, &st);
        if (!out) return st;
    } else {
        out = nsel > 0 ? grad : nac;
    }
    st = contract_pairs(c, nstate, X, Y, nout, pI.data(), pJ.data(), out);
    if (st == RIS_OK && nextra > 0) st = contract_extra(c, nextra, extra, eout.data(), out);
    if (st == RIS_OK && nsel > 0 && npair > 0) {
        HIPCHK(c, hipMemcpyAsync(grad, out, 8 * per * nsel, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(nac, out + per * nsel, 8 * per * npair, hipMemcpyDeviceToDevice, c->stream));
    }
    if (st) return st;
    bool degenerate = false;
    if (omega) {
        for (int k = 0; k < npair; ++k) {
            const double gap = omega[pJ[nsel + k]] - omega[pI[nsel + k]];
            if (std::fabs(gap) < 1e-12) {
                degenerate = true;
                continue;
            }
            HIPCHK(c, axpby(nac + (size_t)k * per, nac + (size_t)k * per, per, 1.0 / gap, 0.0, c->stream));
        }
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (degenerate) return fail(c, RIS_E_DEGENERATE, "degenerate state pair: numerator left undivided");
    return RIS_OK;
}

int ris_grad_contract(ris_ctx *c, int nstate, const double *X, const double *Y, int nsel, const int *sel, int nextra,
                      const ris_extra_pair *extra, double *grad)
{
    if (!c) return RIS_E_INVALID;
    if (nsel > 0 && !sel) return fail(c, RIS_E_INVALID, "null selection");
    return ris_grad_nac_contract(c, nstate, X, Y, nsel, sel, grad, 0, nullptr, nullptr, nullptr, nextra, extra);
}

int ris_nac_contract(ris_ctx *c, int nstate, const double *X, const double *Y, int npair, const int *pairs,
                     int nextra, const ris_extra_pair *extra, const double *omega, double *nac)
{
    if (!c) return RIS_E_INVALID;
    return ris_grad_nac_contract(c, nstate, X, Y, 0, nullptr, nullptr, npair, pairs, omega, nac, nextra, extra);
}

int ris_density_ao(ris_ctx *c, int kind, int nstate, const double *X, const double *Y, int I, int J, const double *Z,
                   double *D)
{
    if (!c) return RIS_E_INVALID;
    c->err.clear();
    if (!c->have_int3c) return fail(c, RIS_E_ORDER, "ris_density_ao before ris_int3c");
    if (kind < RIS_DENS_GROUND || kind > RIS_DENS_RELAXED) return fail(c, RIS_E_INVALID, "unknown density %d", kind);
    if (!D) return fail(c, RIS_E_INVALID, "null output");
    if (kind != RIS_DENS_GROUND) {
        if (!X || nstate <= 0 || I < 0 || J < 0 || I >= nstate || J >= nstate)
            return fail(c, RIS_E_INVALID, "bad amplitudes or state index (I=%d, J=%d, nstate=%d)", I, J, nstate);
        if (kind == RIS_DENS_RELAXED && !Z) return fail(c, RIS_E_INVALID, "relaxed density without Z");
    }
    HIPCHK(c, hipSetDevice(c->device));
    const int N = c->nao, nmo = c->nmo, o = c->nocc, v = c->nvir;
    const long vo = (long)v * o, NN = (long)N * N;
    Carve cv;
    const size_t oM = cv.take(NN), o1 = cv.take((size_t)N * std::max(v, o)), o2 = cv.take((size_t)N * std::max(v, o));
    int st;
    char *wsb = ws_get(c, cv.off, &st);
    if (!wsb) return st;
    double *M = (double *)(wsb + oM), *T1 = (double *)(wsb + o1), *T2 = (double *)(wsb + o2);
    const double *CO = c->C, *CV = c->C + o;
    if (kind == RIS_DENS_GROUND) {
        HIPCHK(c, dgemm(gm(N, N, o, false, true, 1.0, CO, nmo, CO, nmo, 0.0, M, N), c->stream));
    } else {
        const double *XI = X + (size_t)I * vo, *XJ = X + (size_t)J * vo;
        // occupied block: -C_O (X_J^T X_I + Y_I^T Y_J) C_O^T = -(X_J C_O^T)^T (X_I C_O^T) - (Y_I C_O^T)^T (Y_J C_O^T)
        for (int y = 0; y < (Y ? 2 : 1); ++y) {
            const double *A = y ? Y + (size_t)I * vo : XJ, *B = y ? Y + (size_t)J * vo : XI;
            HIPCHK(c, dgemm(gm(v, N, o, false, true, 1.0, A, o, CO, nmo, 0.0, T1, N), c->stream));
            HIPCHK(c, dgemm(gm(v, N, o, false, true, 1.0, B, o, CO, nmo, 0.0, T2, N), c->stream));
            HIPCHK(c, dgemm(gm(N, N, v, true, false, -1.0, T1, N, T2, N, y ? 1.0 : 0.0, M, N), c->stream));
        }
        // virtual block: C_V (X_I X_J^T + Y_J Y_I^T) C_V^T = (C_V X_I)(C_V X_J)^T + (C_V Y_J)(C_V Y_I)^T
        for (int y = 0; y < (Y ? 2 : 1); ++y) {
            const double *A = y ? Y + (size_t)J * vo : XI, *B = y ? Y + (size_t)I * vo : XJ;
            HIPCHK(c, dgemm(gm(N, o, v, false, false, 1.0, CV, nmo, A, o, 0.0, T1, o), c->stream));
            HIPCHK(c, dgemm(gm(N, o, v, false, false, 1.0, CV, nmo, B, o, 0.0, T2, o), c->stream));
            HIPCHK(c, dgemm(gm(N, N, o, false, true, 1.0, T1, o, T2, o, 1.0, M, N), c->stream));
        }
        if (kind == RIS_DENS_RELAXED) {
            // + C_V Z C_O^T (symmetrised below with the rest)
            HIPCHK(c, dgemm(gm(N, o, v, false, false, 1.0, CV, nmo, Z, o, 0.0, T1, o), c->stream));
            HIPCHK(c, dgemm(gm(N, N, o, false, true, 1.0, T1, o, CO, nmo, 1.0, M, N), c->stream));
        }
    }
    HIPCHK(c, symmetrize(M, N, 1, c->stream));
    HIPCHK(c, scatter_sq(M, D, c->d_ao_perm, N, 1, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RIS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------
// Boys table on the host: F_m(k/16) by the all-positive series
// F_m(T) = e^{-T} sum_j (2T)^j / ((2m+1)(2m+3)...(2m+2j+1)) in long double.
void ris::boys_table_host(double *tab)
{
    for (int k = 0; k < kBoysNGrid; ++k) {
        const long double T = (long double)k / kBoysInvStep;
        const long double et = expl(-T);
        for (int m = 0; m < kBoysCols; ++m) {
            long double term = 1.0L / (2 * m + 1), sum = term;
            for (int j = 1; j < 2000; ++j) {
                term *= 2.0L * T / (2 * m + 2 * j + 1);
                sum += term;
                if (term < 1e-22L * sum) break;
            }
            tab[(size_t)k * kBoysCols + m] = (double)(et * sum);
        }
    }
}
