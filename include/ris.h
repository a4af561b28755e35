/*
 * ris.h -- C ABI of the MI355X (gfx950) TDDFT-ris gradient / derivative-coupling
 * hot path.
 *
 * Method (arXiv 2511.18233): the TDDFT-ris kernel replaces both two-electron
 * integrals of the response matrices by a resolution of the identity over a
 * minimal auxiliary basis, g^ris_{pq,sr} = sum_AB (pq|A)(M_J^-1)_AB (B|sr)
 * - c_x sum_AB (pr|A)(M_K^-1)_AB (B|sq) with M_AB = (A|B), and drops f_xc
 * (Sec. 2.2, eqs. ris and g_modified).  The ris term of the excited-state
 * gradient and of the NAC numerator is <g^{ris,(xi)}; Gamma_IJ> with
 * Gamma_IJ = {R^S_I, R^S_J} + {L^A_I, L^A_J} (Sec. 2.2, eqs. gI_xi_ris and
 * gIJ_xi_ris; Appendix A.1), evaluated with the three-term derivative of the
 * RI four-index object (last equation of Sec. 2.2).
 *
 * Conventions used by every call:
 *   - FP64, row-major, atomic units (Bohr, Hartree).
 *   - AO basis: uncontracted Cartesian Gaussians, one primitive per shell,
 *     each Cartesian component normalised to one; l <= 2 with component order
 *     x,y,z and xx,xy,xz,yy,yz,zz; AO index = shells in the caller's order.
 *   - Auxiliary basis built by ris_aux_build: J (Coulomb) set = one s function
 *     on every atom (atom order) followed, if requested, by one p shell
 *     (x,y,z) on every atom with Z > 1 (atom order); K (exchange) set = the s
 *     functions, i.e. the first natm J functions.  One exponent per atom,
 *     theta / R_A^2 (Sec. 2.2: one Gaussian per angular momentum per atom;
 *     Sec. 4: s+p for Coulomb, s for exchange).
 *   - Amplitude arrays are [nstate][nvir][nocc] (index a*nocc + i).
 *   - Large arrays (C, eps, V, out, X, Y, grad, nac, dbg) are DEVICE pointers
 *     on the context's device; small tables (ris_mol, ris_aux_opts, sel,
 *     pairs, omega) are HOST pointers.  The caller owns every buffer it
 *     passes; the context owns all of its internal device state.
 *   - All device work is enqueued on the stream given at ris_ctx_create.
 *     Each declaration states whether the call synchronises that stream
 *     before returning: the calls that read a device result on the host
 *     (Cholesky status, convergence tests) or hand back buffers the caller
 *     may free at once do; ris_response_matvec_noalloc does not.
 *   - Errors: a status code is returned and a message is kept for
 *     ris_last_error; nothing is thrown across the ABI.  After an error the
 *     outputs of that call are undefined.
 *   - Calls on one context must not overlap; any host thread may make them,
 *     one at a time.  Contexts are independent of each other.
 */
#ifndef RIS_H
#define RIS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum ris_status {
    RIS_OK = 0,
    RIS_E_INVALID = 1,      /* bad argument, shape or pointer */
    RIS_E_UNSUPPORTED = 2,  /* AO l > 2, or a precision mode not built */
    RIS_E_NOMEM = 3,        /* request exceeds the context's HBM budget */
    RIS_E_NOT_PD = 4,       /* auxiliary metric not positive definite */
    RIS_E_DEGENERATE = 5,   /* |omega_J - omega_I| < 1e-12 (numerator still written) */
    RIS_E_ORDER = 6,        /* calls out of order (aux_build -> int3c -> others) */
    RIS_E_DEVICE = 7,       /* HIP runtime error */
    RIS_E_NOCONV = 8        /* iterative solve stopped at its iteration limit */
};

/* Arithmetic of the exchange-weight contractions (the products that build
 * Gamma^P, its MO-space blocks and V_PQ) and of the exchange part of the
 * matvecs.  Integrals, every metric solve (M^-1 applications), the Coulomb
 * part, the extra density pairs and all gradient accumulation stay FP64 in
 * every mode; the MO transforms of (mu nu|P) too, unless RIS_PREC_TRANSFORMS
 * is or-ed into the mode.
 *   RIS_FP64   : FP64 matrix cores.
 *   RIS_FP32   : FP32 matrix cores, FP32 accumulation.
 *   RIS_BF16X3 : split BF16 (x32 = fl32(x) ~ hi + lo), three products
 *                hi.hi + hi.lo + lo.hi on BF16 matrix cores, FP32 accumulation
 *                (about 16 bits of each operand).
 *   RIS_BF16X6 : three-way split BF16 (x32 = hi + mid + lo, all 24 bits), the
 *                six products down to order 2^-16, FP32 accumulation.
 *   RIS_PREC_TRANSFORMS : flag; the (ai|P), (ij|P) and (ab|P) transforms of
 *                (mu nu|P) also run in the mode (the M^-1 fits stay FP64). */
enum ris_precision { RIS_FP64 = 0, RIS_FP32 = 1, RIS_BF16X3 = 2, RIS_BF16X6 = 3, RIS_PREC_TRANSFORMS = 16 };

/* Response operators of the Casida problem (Sec. 2.1, eqs. casida, A_matrix,
 * B_matrix): A, B, A+B, A-B with the ris kernel. */
enum ris_op { RIS_OP_A = 0, RIS_OP_B = 1, RIS_OP_APB = 2, RIS_OP_AMB = 3 };

typedef struct ris_ctx ris_ctx;

/* Molecule and AO basis (host pointers, copied during the call). */
typedef struct {
    int natm;
    const int *Z;             /* [natm] nuclear charges (1..118) */
    const double *xyz;        /* [natm][3] Bohr */
    int nshell;
    const int *shell_atom;    /* [nshell] atom of each AO shell */
    const int *shell_l;       /* [nshell] 0..2 */
    const double *shell_exp;  /* [nshell] Gaussian exponent > 0 */
} ris_mol;

/* Minimal auxiliary basis options (host pointers, copied). */
typedef struct {
    double theta;               /* exponent rule alpha_A = theta / R_A^2 */
    const double *radius_bohr;  /* [119] radius R_A by Z, Bohr (> 0 for every Z used) */
    int j_p_on_heavy;           /* 1: add a p shell on every Z > 1 atom to the J set */
} ris_aux_opts;

/* Orbitals and kernel parameters (C, eps are device pointers). */
typedef struct {
    int nao;            /* must equal the AO count of the molecule */
    int nmo;            /* number of MOs (columns of C), nocc < nmo <= nao */
    int nocc;           /* occupied orbitals are columns 0..nocc-1 */
    const double *C;    /* [nao][nmo] device */
    const double *eps;  /* [nmo] device, orbital energies */
    double alpha_J;     /* Coulomb factor (closed-shell singlet: 2) */
    double c_x;         /* exact-exchange fraction (Sec. 2.1, eq. g_integral) */
    int precision;      /* enum ris_precision, optionally | RIS_PREC_TRANSFORMS */
} ris_mo;

/* Create a context on `device` (HIP ordinal) that enqueues on `hip_stream`
 * (a hipStream_t, NULL = the legacy default stream).  hbm_budget bounds the
 * bytes the context may allocate (0 = 90% of the device's free memory).
 * Returns RIS_E_DEVICE if HIP cannot be initialised. */
int ris_ctx_create(ris_ctx **out, int device, void *hip_stream, size_t hbm_budget);

/* Release every device buffer of the context (synchronises its stream). */
void ris_ctx_destroy(ris_ctx *ctx);

/* Message of the last failing call on this context ("" if none). */
const char *ris_last_error(const ris_ctx *ctx);

/* Bytes of device memory the context currently holds. */
size_t ris_ctx_bytes(const ris_ctx *ctx);

/* Free every device region the context holds for a request (basis tables,
 * metric, MO blocks, scratch), keeping only what ris_ctx_create made; the
 * next call must be ris_aux_build.  For a scheduler that needs an idle
 * context's memory for another request.  Synchronises the context's stream. */
int ris_ctx_release(ris_ctx *ctx);

/* Peak device bytes a context holds for one request of this molecule with
 * nmo orbitals (nocc occupied), nstate amplitude vectors, matvecs of up to
 * nvec vectors and nout gradient/NAC outputs (0 for any of the three if that
 * call is not made).  The sizing is the one the calls themselves use, so a
 * scheduler can admit requests by HBM footprint.  The geometry and exponents
 * enter through the AO shell pairs the default screen keeps (the derivative
 * contraction holds a copy of the exchange weights of those pairs): a
 * molecule given with all atoms at one point is sized for every pair, an
 * upper bound.  Host-only, no device work; returns 0 for invalid input. */
size_t ris_request_bytes(const ris_mol *mol, const ris_aux_opts *opts, int nmo, int nocc, int nstate, int nvec,
                         int nout);

/* The same sizing for the blocked path (ris_ctx_set_blocking): the peak
 * device bytes when the auxiliary functions are taken in blocks of at most
 * aux_block (at least one whole shell for the integrals) and the matvec
 * exchange terms one vector at a time; aux_block = 0 gives the unblocked
 * sizing of ris_request_bytes.  A context whose budget holds this many bytes
 * completes the request: the calls fall back to blocks of this size or larger
 * when the unblocked scratch does not fit.  Host-only; 0 for invalid input. */
size_t ris_plan_bytes(const ris_mol *mol, const ris_aux_opts *opts, int nmo, int nocc, int nstate, int nvec,
                      int nout, int aux_block);

/* Instrumented stages of the path (for ris_ctx_stage_stats). */
enum ris_stage {
    RIS_STAGE_INT3C = 0,   /* (mu nu|P) integral kernels of ris_int3c */
    RIS_STAGE_MO = 1,      /* MO-transform and metric GEMMs of ris_int3c */
    RIS_STAGE_MATVEC = 2,  /* one whole ris_response_matvec call */
    RIS_STAGE_HBLK = 3,    /* MO-space exchange blocks of one gradient/NAC output */
    RIS_STAGE_GAMMA = 4,   /* one AO back-transform GEMM launch of Gamma^P = (F_I W^P) F_J^T (lower tiles;
                              a NAC output takes two) */
    RIS_STAGE_DERIV = 5,   /* fused three-centre derivative contraction, one output chunk */
    RIS_STAGE_AUX = 6,     /* one whole ris_aux_build (metric, Cholesky, inverses) */
    RIS_STAGE_YW = 7,      /* Y^P = F_I W^P of one output (W assembly included) */
    RIS_STAGE_VPQ = 8,     /* metric weights V_PQ of one output */
    RIS_STAGE_COUNT = 9
};

/* ris-approximated Z-vector solve (Sec. 4.2: the ris kernel also in the
 * (A+B) matrix of the Z-vector equation, eq. Z_vector of Sec. 2.1): solves
 * (A+B)^ris Z_k = rhs_k for k < nrhs with the same (A+B) as
 * ris_response_matvec(RIS_OP_APB) in the context's precision mode.  Method:
 * MINRES (the operator is symmetric; it need not be positive definite for
 * model orbitals) preconditioned by the orbital-energy differences
 * max(|e_a - e_i|, 1e-4), all right-hand sides advanced together (one
 * batched matvec per iteration), the scalar recurrences on the device.
 * rhs: [nrhs][nvir][nocc] device, read only; Z: [nrhs][nvir][nocc] device,
 * overwritten (the start vector is 0), must not alias rhs.  A right-hand side
 * stops when its preconditioned residual estimate falls to tol times its
 * initial value (0 < tol < 1).  iters (may be NULL) receives the iterations
 * run; rel_resid (may be NULL) the largest true relative residual
 * ||rhs_k - (A+B) Z_k|| / ||rhs_k|| after the solve (one extra matvec).
 * Returns RIS_E_NOCONV if maxit iterations end before every right-hand side
 * has stopped (Z holds the last iterate), RIS_E_ORDER before ris_int3c.
 * Synchronous (the convergence test reads the residuals on the host). */
int ris_zvector_solve(ris_ctx *ctx, int nrhs, const double *rhs, double *Z, double tol, int maxit, int *iters,
                      double *rel_resid);

/* ris terms of the right-hand side of the Z-vector equation and of W
 * (Appendix A.3, eqs. g_I_pp_ris and g_IJ_pp_ris): for each output pair
 * (I, J) the MO-basis matrix
 *   I == J: 4 [R^S_I g^ris[R^S_I]] - 4 [L^A_I g^ris[L^A_I]]
 *   I != J: 2 [R^S_I g^ris[R^S_J]] - 2 [L^A_I g^ris[L^A_J]]
 *         + 2 [R^S_J g^ris[R^S_I]] - 2 [L^A_J g^ris[L^A_I]]
 * with R^S = [[0, R^T/2], [R/2, 0]], L^A = [[0, -L^T/2], [L/2, 0]] in the MO
 * basis (occupied first), R = X + Y, L = X - Y, and
 * g^ris[D]_mn = alpha_J sum (mn|ls)_J D_ls - c_x sum (ml|ns)_K D_ls.
 * The Z-vector right-hand side takes its VO block minus the transposed OV
 * block (eq. Z_vector of Sec. 2.1), W its OO and VV blocks.  FP64 in every
 * precision mode.  X, Y: [nstate][nvir][nocc] device (Y = NULL: TDA);
 * pairs: host [npair][2]; G: device [npair][nmo][nmo], rows and columns in
 * the MO order of ris_int3c's C.  Recomputes (mu nu|P) into the context's
 * scratch (nJ nao^2 doubles).  RIS_E_ORDER before ris_int3c.  Synchronises the
 * context's stream before returning. */
int ris_zrhs_contract(ris_ctx *ctx, int nstate, const double *X, const double *Y, int npair, const int *pairs,
                      double *G);

/* TDA-ris excitation energies (Sec. 2.1, eq. casida with B = 0; the ris
 * kernel of Sec. 2.2 in A): the nroots lowest eigenpairs of the symmetric
 * A^ris by block Davidson on ris_response_matvec(RIS_OP_A) in the context's
 * precision mode.  Start vectors: unit vectors on the 2 nroots smallest
 * orbital-energy gaps; corrections r / (theta - (e_a - e_i)); subspace
 * eigenproblem on the device (one-workgroup Jacobi); the subspace collapses
 * to the Ritz vectors when it would exceed max_space (0 = min(nvir nocc,
 * max(8 nroots, 32)); at most 256 and at least min(2 nroots, nvir nocc)).
 * A root is converged when its residual norm ||A x - w x|| <= tol.
 * omega: host [nroots], ascending; X: device [nroots][nvir][nocc], unit
 * vectors (sign arbitrary but reproducible).  iters (may be NULL): iterations
 * run.  RIS_E_NOCONV after maxit iterations or when no new direction is left
 * (omega and X hold the last Ritz pairs), RIS_E_ORDER before ris_int3c.
 * Synchronous (omega is a host array). */
int ris_tda_davidson(ris_ctx *ctx, int nroots, double tol, int maxit, int max_space, double *omega, double *X,
                     int *iters);

/* AO shell-pair screen of the three-centre derivative contraction (the
 * (mu nu|P)^xi term of the three-term RI derivative, last equation of
 * Sec. 2.2; the screen itself is an implementation choice: a pair whose
 * Gaussian product is negligible contributes nothing above roundoff).
 * A pair of shells with exponents a, b on centres
 * A, B is skipped when exp(-a b / (a + b) |A - B|^2) < threshold; 0 keeps
 * every pair.  Default 1e-15.  Takes effect at once (the lists are rebuilt if
 * the molecule is already set) and stays for later ris_aux_build calls.
 * kept_pairs (may be NULL) receives the number of ordered shell pairs kept,
 * or -1 before the first ris_aux_build.  RIS_E_INVALID unless 0 <= threshold < 1. */
int ris_ctx_set_screening(ris_ctx *ctx, double threshold, long *kept_pairs);

/* Memory blocking over the auxiliary index (the paper batches its
 * density-fitting tensors along the AO or auxiliary dimension, Sec. 3; the
 * block sizes here are an implementation choice).  aux_block > 0 caps the
 * auxiliary functions per block: ris_int3c computes (mu nu|P) and its MO
 * transforms one block of whole J shells at a time (at least one shell), and
 * the gradient / NAC calls take the exchange (K) functions in blocks of at most
 * aux_block, one output at a time.  0 (default): the unblocked path whenever
 * its scratch fits the HBM budget, else the largest blocks that fit.  The
 * results agree with the unblocked path to rounding (only the order of the
 * metric-weight sums changes).  Takes effect from the next call.
 * RIS_E_INVALID if aux_block < 0. */
int ris_ctx_set_blocking(ris_ctx *ctx, int aux_block);

/* Turn per-stage timing on (1) or off (0); either way the counters reset.
 * When on, each instrumented launch group is bracketed by HIP events on the
 * context's stream (no extra synchronisation inside the calls). */
int ris_ctx_set_profiling(ris_ctx *ctx, int enable);

/* Accumulated device time (ms, from the events), algorithmic FLOPs and
 * algorithmic HBM bytes, and the number of timed launch groups of a stage
 * since profiling was last enabled.  Synchronises the context's stream.
 * Any output pointer may be NULL. */
int ris_ctx_stage_stats(ris_ctx *ctx, int stage, double *ms, double *flops, double *bytes, long *launches);

/* Minimal ris auxiliary basis and its Coulomb metric (Sec. 2.2).
 * Builds the AO shell tables and the J and K auxiliary sets, evaluates
 * M_PQ = (P|Q) on the device, factors M = L L^T (FP64 Cholesky) and forms
 * M^-1 for both sets.  Writes the J and K function counts.  Synchronous
 * (the Cholesky positivity check is read back).  RIS_E_NOT_PD if a metric
 * is not positive definite (e.g. two atoms on the same spot); RIS_E_UNSUPPORTED
 * for AO l > 2.  Invalidates previous ris_int3c state. */
int ris_aux_build(ris_ctx *ctx, const ris_mol *mol, const ris_aux_opts *opts,
                  int *nauxJ, int *nauxK);

/* Three-centre integrals (mu nu|P) over the J set (Sec. 2.2, eq. g_modified)
 * and their MO blocks (Sec. 3, reduced MO storage): (ai|P) for every J
 * function, and (ij|P), (ab|P) for the K functions, plus the metric-applied
 * blocks sum_Q (M_K^-1)_PQ (pq|Q).  mo->C and mo->eps are copied.  If
 * dbg_int3c is not NULL it receives (mu nu|P) as [nauxJ][nao][nao] in the
 * caller's AO order (device pointer).  RIS_E_ORDER before ris_aux_build,
 * RIS_E_NOMEM if the tensors exceed the budget.  Synchronises the context's
 * stream before returning. */
int ris_int3c(ris_ctx *ctx, const ris_mo *mo, double *dbg_int3c);

/* ris response matrix-vector products (Sec. 2.1, eqs. A_matrix, B_matrix
 * with K = g^ris): for each of nvec vectors V[v][o] (device, [nvec][nvir][nocc])
 *   (A V)_ai = (e_a - e_i) V_ai + alpha_J sum_bj (ai|bj)_J V_bj - c_x sum_bj (ab|ij)_K V_bj
 *   (B V)_ai =                     alpha_J sum_bj (ai|bj)_J V_bj - c_x sum_bj (aj|bi)_K V_bj
 * op selects A, B, A+B or A-B; out has V's shape (device, may not alias V).
 * Synchronises the context's stream before returning. */
int ris_response_matvec(ris_ctx *ctx, int op, int nvec, const double *V, double *out);

/* Allocation-free ris_response_matvec, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving or solver loops,
 * harnesses that forbid hipMalloc.  Same operators, arguments, layouts and
 * results as ris_response_matvec (the same kernels), but its intermediates
 * live in a fixed 128 MiB device array that the library holds on every device
 * it runs on until the process ends; the call makes no hipMalloc / hipFree and
 * no other allocation, and records no profiling events.  Returns RIS_E_NOMEM,
 * with the bytes needed in ris_last_error, when even one vector per exchange
 * chunk needs more scratch than that (the intermediates grow as
 * nK nvir nocc, so roughly molecules above 70 atoms of the chain workloads);
 * the context's own state (MO blocks, metric) must already exist (ris_int3c).
 * Returns once the work is enqueued on the context's stream (no
 * synchronisation).  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, other contexts, other host threads) race
 * and must be serialised by the caller.  Nothing in the array needs to start
 * at zero; it keeps the last call's contents. */
int ris_response_matvec_noalloc(ris_ctx *ctx, int op, int nvec, const double *V, double *out);

/* One extra density pair of a gradient / NAC output: the <g^(xi); {D, P}>
 * terms of Sec. 2.2 (eqs. gI_xi_ris and gIJ_xi_ris), in which the ground-state
 * density D meets the relaxed density P_I = T_II + Z^S of a gradient or
 * P_IJ = T_IJ + Z~^S of a coupling (Appendix A.1 eq. T, Appendix A.2), taken
 * here over the same ris auxiliary sets as the transition densities (the
 * full density-fitting basis is not part of this path).  The pair adds to
 * output `out` the nuclear derivative, at fixed D1 and D2, of
 *     cJ sum (mn|ls)_J D1_mn D2_ls - cK sum (ml|ns)_K D1_mn D2_ls
 * with (pq|rs)_X = sum_PQ (pq|P)(M_X^-1)_PQ(Q|rs), the three-term RI
 * derivative included.  D1 and D2 are device [nao][nao] arrays in the
 * caller's AO order, read only; they are taken as symmetric (the call uses
 * (D + D^T)/2, which is the matrix itself for the densities above).  The
 * extra pairs run in FP64 in every precision mode.  ris_density_ao builds D,
 * T_IJ and P_IJ on the device. */
typedef struct {
    int out;            /* output index: into sel (gradients) or pairs (NACs);
                           ris_grad_nac_contract counts the nsel gradients first */
    const double *D1;   /* [nao][nao] device */
    const double *D2;   /* [nao][nao] device */
    double cJ;          /* Coulomb coefficient */
    double cK;          /* exchange coefficient */
} ris_extra_pair;

/* ris part of excited-state gradients (Sec. 2.2, eq. gI_xi_ris): for each
 * selected state I = sel[k], grad[k][A][x] = d/dA_x <g^ris; Gamma_II> at fixed
 * AO transition densities R^S_I, L^A_I built from R_I = X_I + Y_I and
 * L_I = X_I - Y_I (Appendix A.1), including the (P|Q) metric derivative,
 * plus the derivatives of the extra pairs that name output k (nextra may be
 * 0 and extra NULL).
 * X, Y: [nstate][nvir][nocc] device; Y = NULL means TDA (Y = 0, Sec. 3).
 * grad: [nsel][natm][3] device, Ha/Bohr (dE/dR, not a force).
 * Synchronises the context's stream before returning. */
int ris_grad_contract(ris_ctx *ctx, int nstate, const double *X, const double *Y,
                      int nsel, const int *sel, int nextra, const ris_extra_pair *extra, double *grad);

/* ris part of NACs between excited states (Sec. 2.2, eq. gIJ_xi_ris): for
 * each pair (I, J) = (pairs[2k], pairs[2k+1]) writes the numerator
 * d/dA_x <g^ris; Gamma_IJ> (plus the extra pairs that name output k) to
 * nac[k][A][x] (device, Ha/Bohr); if omega (host, [nstate]) is given the
 * whole numerator is divided by (omega_J - omega_I) (1/Bohr).  Returns
 * RIS_E_DEGENERATE (after writing the numerator) if any gap is below 1e-12.
 * Synchronises the context's stream before returning. */
int ris_nac_contract(ris_ctx *ctx, int nstate, const double *X, const double *Y,
                     int npair, const int *pairs, int nextra, const ris_extra_pair *extra,
                     const double *omega, double *nac);

/* Gradients and NAC numerators in one call (Sec. 2.2, eqs. gI_xi_ris and
 * gIJ_xi_ris): same outputs and errors as ris_grad_contract followed by
 * ris_nac_contract on the same amplitudes, but the per-state intermediates
 * (AO transition-density factors and their exchange blocks) are built once
 * for all outputs.  Either list may be empty (its pointers may then be NULL).
 * extra[e].out counts the nsel gradients first, then the npair couplings.
 * Synchronises the context's stream before returning. */
int ris_grad_nac_contract(ris_ctx *ctx, int nstate, const double *X, const double *Y,
                          int nsel, const int *sel, double *grad,
                          int npair, const int *pairs, const double *omega, double *nac,
                          int nextra, const ris_extra_pair *extra);

/* AO densities for the extra pairs (device, FP64, every precision mode):
 *   RIS_DENS_GROUND     : D = C_O C_O^T, the occupied projector (the MO
 *                         matrix diag(1_occ, 0) of Appendix A.3 in the AO basis);
 *   RIS_DENS_DIFFERENCE : T_IJ = C (gamma + gamma^T)/2 C^T with
 *                         gamma_oo = -(X_J^T X_I + Y_I^T Y_J),
 *                         gamma_vv = X_I X_J^T + Y_J Y_I^T (Appendix A.1, eq. T);
 *   RIS_DENS_RELAXED    : T_IJ + Z^S, Z^S = (C_V Z C_O^T + C_O Z^T C_V^T)/2
 *                         (Appendix A.2: P_I = T_II + Z^S, P_IJ = T_IJ + Z~^S).
 * X, Y: [nstate][nvir][nocc] device (Y = NULL: TDA), I, J < nstate (ignored
 * for the ground density, as are X, Y and Z); Z: [nvir][nocc] device (the
 * relaxed density only); D: [nao][nao] device, caller AO order, overwritten.
 * Uses the orbitals given to ris_int3c (RIS_E_ORDER before it).
 * Synchronises the context's stream before returning. */
enum ris_density { RIS_DENS_GROUND = 0, RIS_DENS_DIFFERENCE = 1, RIS_DENS_RELAXED = 2 };
int ris_density_ao(ris_ctx *ctx, int kind, int nstate, const double *X, const double *Y, int I, int J,
                   const double *Z, double *D);

#ifdef __cplusplus
}
#endif

#endif /* RIS_H */
