// Host side of the TDDFT-ris hot path: context, device-resident state and the
// five entry points declared in include/ris.h.  Every arithmetic step runs in
// the gfx950 kernels of ris_ints.hip, ris_gemm.hip and ris_linalg.hip on the
// context's stream; this file only sizes buffers, builds shell tables and
// sequences launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdarg>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ris.h"
#include "ris_common.hpp"
#include "ris_linalg.hpp"

using namespace ris;

namespace {

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

    // ---- aux_build state
    bool have_aux = false;
    int natm = 0, nao = 0, nshAO = 0;
    int nJ = 0, nK = 0, nshJ = 0, nsJ = 0;  // J functions, K functions, J shells, J s-shells
    std::vector<int> h_ao_perm;             // internal AO function -> caller AO function
    std::vector<int> h_ao_atom, h_aux_atom;
    AOGeom ao{};
    AuxGeom aux{};
    int auxl_beg[kMaxAuxL + 2] = {0, 0, 0};
    int *d_ao_perm = nullptr;
    double *MJ = nullptr, *LinvJ = nullptr, *MinvJ = nullptr, *MinvK = nullptr;

    // ---- int3c state
    bool have_int3c = false;
    int nmo = 0, nocc = 0, nvir = 0;
    double alphaJ = 2.0, cx = 0.25;
    double *C = nullptr;    // [nao][nmo] internal AO order
    double *eps = nullptr;  // [nmo]
    double *aiJ = nullptr;  // [nJ][v][o] raw (ai|P)
    double *rawoo = nullptr, *rawvv = nullptr;        // [nK][o][o], [nK][v][v]
    double *coo = nullptr, *cvo = nullptr, *cvv = nullptr;  // metric-applied K blocks
    std::vector<void *> int3c_allocs;
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
            hipStreamSynchronize(c->stream);
            hipFree(p);
            c->held -= c->bufs[i].bytes;
            c->bufs.erase(c->bufs.begin() + i);
            return;
        }
}

void free_int3c(ris_ctx *c)
{
    for (void *p : c->int3c_allocs) dfree(c, p);
    c->int3c_allocs.clear();
    c->have_int3c = false;
    c->C = c->eps = c->aiJ = c->rawoo = c->rawvv = c->coo = c->cvo = c->cvv = nullptr;
}

void free_aux(ris_ctx *c)
{
    free_int3c(c);
    for (void *p : {(void *)c->d_ao_perm, (void *)c->MJ, (void *)c->LinvJ, (void *)c->MinvJ, (void *)c->MinvK,
                    (void *)c->ao.sh.x, (void *)c->aux.sh.x})
        dfree(c, p);
    c->d_ao_perm = nullptr;
    c->MJ = c->LinvJ = c->MinvJ = c->MinvK = nullptr;
    c->ao = AOGeom{};
    c->aux = AuxGeom{};
    c->have_aux = false;
}

// Upload a shell table: 5 double arrays + 2 int arrays in one allocation.
int upload_shells(ris_ctx *c, int n, const std::vector<double> &x, const std::vector<double> &y,
                  const std::vector<double> &z, const std::vector<double> &e, const std::vector<double> &nrm,
                  const std::vector<int> &atom, const std::vector<int> &off, ShellTab *out)
{
    const size_t nd = (size_t)5 * n, ni = (size_t)2 * n + 1;
    int st;
    char *base = (char *)dalloc(c, nd * 8 + ni * 4, &st);
    if (!base) return st;
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

}  // namespace

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
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    for (auto &b : c->bufs) hipFree(b.p);
    delete c;
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
    std::vector<int> order;
    for (int l = 0; l <= kMaxAOL; ++l) {
        c->ao.lbeg[l] = (int)order.size();
        for (int s = 0; s < nsh; ++s)
            if (mol->shell_l[s] == l) order.push_back(s);
    }
    c->ao.lbeg[kMaxAOL + 1] = nsh;
    std::vector<double> x(nsh), y(nsh), z(nsh), e(nsh), nr(nsh);
    std::vector<int> at(nsh), off(nsh + 1);
    c->h_ao_perm.assign(nao, 0);
    int f = 0;
    for (int i = 0; i < nsh; ++i) {
        const int s = order[i], a = mol->shell_atom[s], l = mol->shell_l[s];
        x[i] = mol->xyz[3 * a];
        y[i] = mol->xyz[3 * a + 1];
        z[i] = mol->xyz[3 * a + 2];
        e[i] = mol->shell_exp[s];
        nr[i] = radial_norm(e[i], l);
        at[i] = a;
        off[i] = f;
        for (int k = 0; k < ncart(l); ++k) c->h_ao_perm[f + k] = caller_off[s] + k;
        f += ncart(l);
    }
    off[nsh] = f;
    int st = upload_shells(c, nsh, x, y, z, e, nr, at, off, &c->ao.sh);
    if (st) return st;
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
    st = upload_shells(c, nshJ, ax, ay, az, ae, anr, aat, aoff, &c->aux.sh);
    if (st) return st;
    c->aux.nshell = nshJ;
    c->aux.nfunc = f;
    c->auxl_beg[0] = 0;
    c->auxl_beg[1] = natm;
    c->auxl_beg[2] = nshJ;
    c->h_aux_atom = aat;
    c->natm = natm;
    c->nao = nao;
    c->nshAO = nsh;
    c->nJ = f;
    c->nK = natm;
    c->nshJ = nshJ;
    c->nsJ = natm;

    c->d_ao_perm = (int *)dalloc(c, sizeof(int) * nao, &st);
    if (!c->d_ao_perm) return st;
    HIPCHK(c, hipMemcpyAsync(c->d_ao_perm, c->h_ao_perm.data(), sizeof(int) * nao, hipMemcpyHostToDevice, c->stream));

    // --- metric, Cholesky, inverses
    const int nJ = c->nJ, nK = c->nK;
    c->MJ = (double *)dalloc(c, sizeof(double) * nJ * nJ, &st);
    if (!c->MJ) return st;
    c->LinvJ = (double *)dalloc(c, sizeof(double) * nJ * nJ, &st);
    if (!c->LinvJ) return st;
    c->MinvJ = (double *)dalloc(c, sizeof(double) * nJ * nJ, &st);
    if (!c->MinvJ) return st;
    c->MinvK = (double *)dalloc(c, sizeof(double) * nK * nK, &st);
    if (!c->MinvK) return st;
    HIPCHK(c, launch_int2c(c->aux, c->boys, c->MJ, c->stream));
    // factor a copy (MJ keeps the metric itself)
    HIPCHK(c, hipMemcpyAsync(c->MinvJ, c->MJ, sizeof(double) * nJ * nJ, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, cholesky(c->MinvJ, c->MJ, nJ, c->info, c->stream));
    int info = 0;
    HIPCHK(c, hipMemcpyAsync(&info, c->info, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (info != 0) return fail(c, RIS_E_NOT_PD, "auxiliary metric not positive definite (column %d)", info);
    HIPCHK(c, tri_inverse(c->MinvJ, c->LinvJ, nJ, c->stream));
    // M_J^-1 = L^-T L^-1 ; M_K = leading nK block, so L_K^-1 = leading block of L_J^-1
    HIPCHK(c, dgemm(gm(nJ, nJ, nJ, true, false, 1.0, c->LinvJ, nJ, c->LinvJ, nJ, 0.0, c->MinvJ, nJ), c->stream));
    HIPCHK(c, dgemm(gm(nK, nK, nK, true, false, 1.0, c->LinvJ, nJ, c->LinvJ, nJ, 0.0, c->MinvK, nK), c->stream));
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
    if (mo->precision != RIS_FP64) return fail(c, RIS_E_UNSUPPORTED, "precision mode %d not built", mo->precision);
    HIPCHK(c, hipSetDevice(c->device));
    free_int3c(c);

    const int N = c->nao, nmo = mo->nmo, o = mo->nocc, v = nmo - o, nJ = c->nJ, nK = c->nK;
    c->nmo = nmo;
    c->nocc = o;
    c->nvir = v;
    c->alphaJ = mo->alpha_J;
    c->cx = mo->c_x;
    const size_t NN = (size_t)N * N;

    // persistent: C, eps, aiJ, rawoo, rawvv, coo, cvo, cvv ; scratch: X, Z
    const size_t persist = 8 * ((size_t)N * nmo + nmo + (size_t)nJ * v * o + (size_t)nK * o * o * 2 +
                                (size_t)nK * v * v * 2 + (size_t)nK * v * o);
    const size_t scratch = 8 * ((size_t)nJ * NN + (size_t)nJ * N * std::max(o, 1) + (size_t)nK * N * v);
    if (c->held + persist + scratch > c->budget)
        return fail(c, RIS_E_NOMEM, "int3c needs %.2f GB (persistent %.2f GB); budget %.2f GB, %.2f GB held",
                    (persist + scratch) / 1e9, persist / 1e9, c->budget / 1e9, c->held / 1e9);
    int st;
    auto take = [&](size_t elems) -> double * {
        double *p = (double *)dalloc(c, elems * 8, &st);
        if (p) c->int3c_allocs.push_back(p);
        return p;
    };
    if (!(c->C = take((size_t)N * nmo)) || !(c->eps = take(nmo)) || !(c->aiJ = take((size_t)nJ * v * o)) ||
        !(c->rawoo = take((size_t)nK * o * o)) || !(c->rawvv = take((size_t)nK * v * v)) ||
        !(c->coo = take((size_t)nK * o * o)) || !(c->cvo = take((size_t)nK * v * o)) ||
        !(c->cvv = take((size_t)nK * v * v)))
        return st;
    double *X = (double *)dalloc(c, 8 * (size_t)nJ * NN, &st);
    if (!X) return st;
    double *Z = (double *)dalloc(c, 8 * std::max((size_t)nJ * N * o, (size_t)nK * N * v), &st);
    if (!Z) {
        dfree(c, X);
        return st;
    }

    // C rows into the internal (l-sorted) AO order
    HIPCHK(c, gather_rows(mo->C, c->C, c->d_ao_perm, N, nmo, nmo, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->eps, mo->eps, 8 * nmo, hipMemcpyDeviceToDevice, c->stream));

    // (mu nu|P)
    HIPCHK(c, launch_int3c(c->ao, c->aux, c->auxl_beg, c->boys, X, c->stream));
    if (dbg) HIPCHK(c, scatter_sq(X, dbg, c->d_ao_perm, N, nJ, c->stream));

    const double *CO = c->C, *CV = c->C + o;
    // Z^P = X^P C_O  [nJ][N][o]
    GemmArgs g = gm(N, o, N, false, false, 1.0, X, N, CO, nmo, 0.0, Z, o);
    g.batch = nJ; g.strideA = NN; g.strideB = 0; g.strideC = (long)N * o;
    HIPCHK(c, dgemm(g, c->stream));
    // (ai|P) = C_V^T Z^P  [nJ][v][o]
    g = gm(v, o, N, true, false, 1.0, CV, nmo, Z, o, 0.0, c->aiJ, o);
    g.batch = nJ; g.strideA = 0; g.strideB = (long)N * o; g.strideC = (long)v * o;
    HIPCHK(c, dgemm(g, c->stream));
    // (ij|P) = C_O^T Z^P, K functions only  [nK][o][o]
    g = gm(o, o, N, true, false, 1.0, CO, nmo, Z, o, 0.0, c->rawoo, o);
    g.batch = nK; g.strideA = 0; g.strideB = (long)N * o; g.strideC = (long)o * o;
    HIPCHK(c, dgemm(g, c->stream));
    // (ab|P) = C_V^T (X^P C_V), K functions only  [nK][v][v]
    g = gm(N, v, N, false, false, 1.0, X, N, CV, nmo, 0.0, Z, v);
    g.batch = nK; g.strideA = NN; g.strideB = 0; g.strideC = (long)N * v;
    HIPCHK(c, dgemm(g, c->stream));
    g = gm(v, v, N, true, false, 1.0, CV, nmo, Z, v, 0.0, c->rawvv, v);
    g.batch = nK; g.strideA = 0; g.strideB = (long)N * v; g.strideC = (long)v * v;
    HIPCHK(c, dgemm(g, c->stream));
    // metric-applied exchange blocks c^P = sum_Q (M_K^-1)_PQ (..|Q)
    HIPCHK(c, dgemm(gm(nK, o * o, nK, false, false, 1.0, c->MinvK, nK, c->rawoo, (long)o * o, 0.0, c->coo,
                       (long)o * o), c->stream));
    HIPCHK(c, dgemm(gm(nK, v * o, nK, false, false, 1.0, c->MinvK, nK, c->aiJ, (long)v * o, 0.0, c->cvo,
                       (long)v * o), c->stream));
    HIPCHK(c, dgemm(gm(nK, v * v, nK, false, false, 1.0, c->MinvK, nK, c->rawvv, (long)v * v, 0.0, c->cvv,
                       (long)v * v), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dfree(c, Z);
    dfree(c, X);
    c->have_int3c = true;
    return RIS_OK;
}

// ------------------------------------------------------------------------
int ris_response_matvec(ris_ctx *c, int op, int nvec, const double *V, double *out)
{
    if (!c) return RIS_E_INVALID;
    c->err.clear();
    if (!c->have_int3c) return fail(c, RIS_E_ORDER, "ris_response_matvec before ris_int3c");
    if (op < RIS_OP_A || op > RIS_OP_AMB) return fail(c, RIS_E_INVALID, "unknown operator %d", op);
    if (nvec < 0) return fail(c, RIS_E_INVALID, "nvec < 0");
    if (nvec == 0) return RIS_OK;
    if (!V || !out || V == out) return fail(c, RIS_E_INVALID, "null or aliased vector pointer");
    HIPCHK(c, hipSetDevice(c->device));
    const int o = c->nocc, v = c->nvir, nJ = c->nJ, nK = c->nK;
    const long vo = (long)v * o;
    // coefficients of Delta, J, K_A, K_B for A, B, A+B, A-B
    static const double cDe[4] = {1, 0, 1, 1}, cJ[4] = {1, 1, 2, 0}, cKA[4] = {1, 0, 1, 1}, cKB[4] = {0, 1, 1, -1};
    int st;
    double *t = (double *)dalloc(c, 8 * (size_t)nvec * nJ * 2, &st);
    if (!t) return st;
    double *T = (double *)dalloc(c, 8 * (size_t)nK * std::max(vo, (long)o * o), &st);
    if (!T) {
        dfree(c, t);
        return st;
    }
    double *cc = t + (size_t)nvec * nJ;
    // Coulomb: t = V (ai|P)^T ; cc = t M_J^-1 ; out = cJ alpha_J cc (ai|P)
    HIPCHK(c, dgemm(gm(nvec, nJ, (int)vo, false, true, 1.0, V, vo, c->aiJ, vo, 0.0, t, nJ), c->stream));
    HIPCHK(c, dgemm(gm(nvec, nJ, nJ, false, false, 1.0, t, nJ, c->MinvJ, nJ, 0.0, cc, nJ), c->stream));
    HIPCHK(c, dgemm(gm(nvec, (int)vo, nJ, false, false, cJ[op] * c->alphaJ, cc, nJ, c->aiJ, vo, 0.0, out, vo),
                    c->stream));
    if (cDe[op] != 0.0) HIPCHK(c, add_de(c->eps, V, out, v, o, nvec, cDe[op], c->stream));
    for (int k = 0; k < nvec; ++k) {
        const double *Vk = V + (size_t)k * vo;
        double *ok = out + (size_t)k * vo;
        if (cKA[op] != 0.0) {
            // T^P[b][i] = sum_j V[b][j] c_oo^P[i][j] ; out[a][i] -= c_x sum_P sum_b (ab|P) T^P[b][i]
            GemmArgs g = gm(v, o, o, false, true, 1.0, Vk, o, c->coo, o, 0.0, T, o);
            g.batch = nK; g.strideA = 0; g.strideB = (long)o * o; g.strideC = vo;
            HIPCHK(c, dgemm(g, c->stream));
            g = gm(v, o, v, false, false, -cKA[op] * c->cx, c->rawvv, v, T, o, 1.0, ok, o);
            g.nred = nK; g.strideAr = (long)v * v; g.strideBr = vo;
            HIPCHK(c, dgemm(g, c->stream));
        }
        if (cKB[op] != 0.0) {
            // S^P[i][j] = sum_b c_vo^P[b][i] V[b][j] ; out[a][i] -= c_x sum_P sum_j (aj|P) S^P[i][j]
            GemmArgs g = gm(o, o, v, true, false, 1.0, c->cvo, o, Vk, o, 0.0, T, o);
            g.batch = nK; g.strideA = vo; g.strideB = 0; g.strideC = (long)o * o;
            HIPCHK(c, dgemm(g, c->stream));
            g = gm(v, o, o, false, true, -cKB[op] * c->cx, c->aiJ, o, T, o, 1.0, ok, o);
            g.nred = nK; g.strideAr = vo; g.strideBr = (long)o * o;
            HIPCHK(c, dgemm(g, c->stream));
        }
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dfree(c, T);
    dfree(c, t);
    return RIS_OK;
}

// ------------------------------------------------------------------------
// Gradient / NAC numerators for a list of state pairs (I, J):
//   out[k] = d/dR [ alpha_J sum (mn|ls)_J R^S_I R^S_J - c_x sum (ml|ns)_K (R^S_I R^S_J + L^A_I L^A_J) ]
static int contract_pairs(ris_ctx *c, int nstate, const double *X, const double *Y, int npair, const int *pI,
                          const int *pJ, double *outg)
{
    HIPCHK(c, hipSetDevice(c->device));
    const int N = c->nao, nmo = c->nmo, o = c->nocc, v = c->nvir, nJ = c->nJ, nK = c->nK, natm = c->natm;
    const long vo = (long)v * o, NN = (long)N * N, o3 = 3L * o;
    const int NO = kMaxOutChunk;
    int st;
    std::vector<void *> tmp;
    auto take = [&](size_t elems) -> double * {
        double *p = (double *)dalloc(c, elems * 8, &st);
        if (p) tmp.push_back(p);
        return p;
    };
    auto cleanup = [&]() {
        for (void *p : tmp) dfree(c, p);
    };
    double *R, *L, *F, *D, *tT, *cvec, *H, *Tm, *W, *Y3, *G, *V2, *p3, *p2, *shA, *shC, *shP;
    if (!(R = take((size_t)nstate * vo)) || !(L = take((size_t)nstate * vo)) || !(F = take((size_t)nstate * N * o3)) ||
        !(D = take((size_t)nstate * NN)) || !(tT = take((size_t)nstate * nJ)) || !(cvec = take((size_t)nstate * nJ)) ||
        !(H = take((size_t)6 * nK * o * o)) || !(Tm = take((size_t)nK * vo)) || !(W = take((size_t)nK * o3 * o3)) ||
        !(Y3 = take((size_t)nK * N * o3)) || !(G = take((size_t)NO * nK * NN)) || !(V2 = take((size_t)NO * nJ * nJ)) ||
        !(p3 = take((size_t)c->nshAO * c->nshJ * 3 * NO * 6)) || !(p2 = take((size_t)c->nshJ * 2 * NO * 3)) ||
        !(shA = take((size_t)c->nshAO * NO * 3)) || !(shC = take((size_t)c->nshJ * NO * 3)) ||
        !(shP = take((size_t)c->nshJ * NO * 3))) {
        cleanup();
        return st;
    }
    const double *CO = c->C, *CV = c->C + o;
    HIPCHK(c, make_rl(X, Y, R, L, (size_t)nstate * vo, c->stream));
    // F_s = [C_V R_s, C_V L_s, C_O]  (N x 3o)
    {
        GemmArgs g = gm(N, o, v, false, false, 1.0, CV, nmo, R, o, 0.0, F, o3);
        g.batch = nstate; g.strideA = 0; g.strideB = vo; g.strideC = (long)N * o3;
        HIPCHK(c, dgemm(g, c->stream));
        g = gm(N, o, v, false, false, 1.0, CV, nmo, L, o, 0.0, F + o, o3);
        g.batch = nstate; g.strideA = 0; g.strideB = vo; g.strideC = (long)N * o3;
        HIPCHK(c, dgemm(g, c->stream));
        for (int s = 0; s < nstate; ++s)
            HIPCHK(c, hipMemcpy2DAsync(F + (size_t)s * N * o3 + 2 * o, o3 * 8, CO, (size_t)nmo * 8, (size_t)o * 8, N,
                                       hipMemcpyDeviceToDevice, c->stream));
        // D_s = sym(U_Rs C_O^T) = R^S_s
        g = gm(N, N, o, false, true, 1.0, F, o3, CO, nmo, 0.0, D, N);
        g.batch = nstate; g.strideA = (long)N * o3; g.strideB = 0; g.strideC = NN;
        HIPCHK(c, dgemm(g, c->stream));
        HIPCHK(c, symmetrize(D, N, nstate, c->stream));
        // c_s = M_J^-1 t_s, t_s[P] = sum_ai (ai|P) R_s[a][i]
        HIPCHK(c, dgemm(gm(nstate, nJ, (int)vo, false, true, 1.0, R, vo, c->aiJ, vo, 0.0, tT, nJ), c->stream));
        HIPCHK(c, dgemm(gm(nstate, nJ, nJ, false, false, 1.0, tT, nJ, c->MinvJ, nJ, 0.0, cvec, nJ), c->stream));
    }
    double *Hoo = c->coo;
    double *HRuo = H, *HLuo = H + (size_t)nK * o * o, *HRou = H + 2 * (size_t)nK * o * o,
           *HLou = H + 3 * (size_t)nK * o * o, *HRuu = H + 4 * (size_t)nK * o * o, *HLuu = H + 5 * (size_t)nK * o * o;
    const long oo = (long)o * o;

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
        for (int k = 0; k < NO; ++k) {
            const int kk = k0 + std::min(k, nb - 1);
            job.stI[k] = pI[kk];
            job.stJ[k] = pJ[kk];
        }
        for (int k = 0; k < nb; ++k) {
            const int I = pI[k0 + k], J = pJ[k0 + k];
            const double *RI = R + (size_t)I * vo, *RJ = R + (size_t)J * vo;
            const double *LI = L + (size_t)I * vo, *LJ = L + (size_t)J * vo;
            // H_UO = R_I^T c_vo^P ; H_OU = c_vo^P^T R_J (o x o per P); same with L
            auto hb = [&](const double *A, bool tA, long sA, const double *B, bool tB, long sB, double *Cm) {
                (void)tB;
                GemmArgs g = gm(o, o, v, tA, false, 1.0, A, o, B, o, 0.0, Cm, o);
                g.batch = nK; g.strideA = sA; g.strideB = sB; g.strideC = oo;
                return dgemm(g, c->stream);
            };
            HIPCHK(c, hb(RI, true, 0, c->cvo, false, vo, HRuo));
            HIPCHK(c, hb(LI, true, 0, c->cvo, false, vo, HLuo));
            HIPCHK(c, hb(c->cvo, true, vo, RJ, false, 0, HRou));
            HIPCHK(c, hb(c->cvo, true, vo, LJ, false, 0, HLou));
            // H_UU = R_I^T (c_vv^P R_J)
            for (int rl = 0; rl < 2; ++rl) {
                const double *SI = rl ? LI : RI, *SJ = rl ? LJ : RJ;
                GemmArgs g = gm(v, o, v, false, false, 1.0, c->cvv, v, SJ, o, 0.0, Tm, o);
                g.batch = nK; g.strideA = (long)v * v; g.strideB = 0; g.strideC = vo;
                HIPCHK(c, dgemm(g, c->stream));
                HIPCHK(c, hb(SI, true, 0, Tm, false, vo, rl ? HLuu : HRuu));
            }
            // W^P (3o x 3o), Y^P = F_I W^P, Gamma^P = -2 c_x Y^P F_J^T
            HIPCHK(c, assemble_w(Hoo, HRou, HLou, HRuo, HLuo, HRuu, HLuu, W, o, nK, 1.0, c->stream));
            GemmArgs g = gm(N, (int)o3, (int)o3, false, false, 1.0, F + (size_t)I * N * o3, o3, W, o3, 0.0, Y3, o3);
            g.batch = nK; g.strideA = 0; g.strideB = o3 * o3; g.strideC = (long)N * o3;
            HIPCHK(c, dgemm(g, c->stream));
            double *Gk = G + (size_t)k * nK * NN;
            g = gm(N, N, (int)o3, false, true, -2.0 * c->cx, Y3, o3, F + (size_t)J * N * o3, o3, 0.0, Gk, N);
            g.batch = nK; g.strideA = (long)N * o3; g.strideB = 0; g.strideC = NN;
            HIPCHK(c, dgemm(g, c->stream));
            if (I != J) HIPCHK(c, symmetrize(Gk, N, nK, c->stream));
            // metric weights: W2 = -alpha_J c_I c_J^T (J set) + c_x V (K block),
            // V_PQ = sum_kl H^P_kl W^Q_kl over the nonzero exchange blocks
            double *V2k = V2 + (size_t)k * nJ * nJ;
            HIPCHK(c, dgemm(gm(nJ, nJ, 1, true, false, -c->alphaJ, cvec + (size_t)I * nJ, nJ, cvec + (size_t)J * nJ,
                               nJ, 0.0, V2k, nJ), c->stream));
            const double q = 0.25 * c->cx;
            struct Term { const double *a; const double *b; double s; };
            const Term terms[] = {{HRuu, Hoo, q},   {HLuu, Hoo, q},   {HRuo, HRou, q}, {HLuo, HLou, -q},
                                  {HRou, HRuo, q},  {HLou, HLuo, -q}, {Hoo, HRuu, q},  {Hoo, HLuu, q}};
            for (const Term &tm : terms)
                HIPCHK(c, dgemm(gm(nK, nK, (int)oo, false, true, tm.s, tm.a, oo, tm.b, oo, 1.0, V2k, nJ), c->stream));
        }
        // three-centre derivative contraction + metric derivative, reduced into atoms
        HIPCHK(c, fill(p3, (size_t)c->nshAO * c->nshJ * 3 * NO * 6, 0.0, c->stream));
        HIPCHK(c, launch_int3c_deriv(c->ao, c->aux, c->auxl_beg, c->boys, job, c->stream));
        HIPCHK(c, fill(p2, (size_t)c->nshJ * 2 * nb * 3, 0.0, c->stream));
        HIPCHK(c, launch_int2c_deriv(c->aux, c->boys, nb, V2, p2, c->stream));
        // the deriv kernel indexes partials with stride NO; pass NO for p3, nb outputs
        HIPCHK(c, reduce_grad(p3, c->nshAO, c->nshJ, nb, NO, p2, c->ao.sh.atom, c->aux.sh.atom, natm, shA, shC, shP,
                              1.0, 0, outg + (size_t)k0 * natm * 3, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    cleanup();
    return RIS_OK;
}

int ris_grad_contract(ris_ctx *c, int nstate, const double *X, const double *Y, int nsel, const int *sel, double *grad)
{
    if (!c) return RIS_E_INVALID;
    c->err.clear();
    if (!c->have_int3c) return fail(c, RIS_E_ORDER, "ris_grad_contract before ris_int3c");
    if (nstate <= 0 || nsel < 0 || !X || (nsel > 0 && (!sel || !grad)))
        return fail(c, RIS_E_INVALID, "bad gradient arguments");
    std::vector<int> pI(nsel), pJ(nsel);
    for (int k = 0; k < nsel; ++k) {
        if (sel[k] < 0 || sel[k] >= nstate) return fail(c, RIS_E_INVALID, "sel[%d]=%d out of range", k, sel[k]);
        pI[k] = pJ[k] = sel[k];
    }
    if (nsel == 0) return RIS_OK;
    return contract_pairs(c, nstate, X, Y, nsel, pI.data(), pJ.data(), grad);
}

int ris_nac_contract(ris_ctx *c, int nstate, const double *X, const double *Y, int npair, const int *pairs,
                     const double *omega, double *nac)
{
    if (!c) return RIS_E_INVALID;
    c->err.clear();
    if (!c->have_int3c) return fail(c, RIS_E_ORDER, "ris_nac_contract before ris_int3c");
    if (nstate <= 0 || npair < 0 || !X || (npair > 0 && (!pairs || !nac)))
        return fail(c, RIS_E_INVALID, "bad NAC arguments");
    std::vector<int> pI(npair), pJ(npair);
    for (int k = 0; k < npair; ++k) {
        pI[k] = pairs[2 * k];
        pJ[k] = pairs[2 * k + 1];
        if (pI[k] < 0 || pI[k] >= nstate || pJ[k] < 0 || pJ[k] >= nstate)
            return fail(c, RIS_E_INVALID, "pair %d out of range", k);
    }
    if (npair == 0) return RIS_OK;
    int st = contract_pairs(c, nstate, X, Y, npair, pI.data(), pJ.data(), nac);
    if (st || !omega) return st;
    bool degenerate = false;
    for (int k = 0; k < npair; ++k) {
        const double gap = omega[pJ[k]] - omega[pI[k]];
        if (std::fabs(gap) < 1e-12) {
            degenerate = true;
            continue;
        }
        HIPCHK(c, axpby(nac + (size_t)k * c->natm * 3, nac + (size_t)k * c->natm * 3, (size_t)c->natm * 3, 1.0 / gap,
                        0.0, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (degenerate) return fail(c, RIS_E_DEGENERATE, "degenerate state pair: numerator left undivided");
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
