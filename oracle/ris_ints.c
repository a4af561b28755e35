/*
 * CPU ORACLE -- test infrastructure only.  Plain FP64 Gaussian integrals for
 * the TDDFT-ris response path.  Only tests/, the smoke check and the bench's
 * CPU-baseline leg may load this library; the product path never does.
 *
 * Integrals follow the textbook McMurchie-Davidson scheme (McMurchie and
 * Davidson 1978; Helgaker, Jorgensen, Olsen, "Molecular Electronic-Structure
 * Theory", ch. 9): Hermite expansion coefficients E^{ij}_t of Gaussian
 * products, Hermite Coulomb integrals R_{tuv} from the Boys function, and
 *
 *   (ab|c) = 2 pi^{5/2} / (p q sqrt(p+q)) sum_{tuv} E^{ab}_{tuv}
 *            sum_{tau nu phi} (-1)^{tau+nu+phi} E^{c}_{tau nu phi}
 *            R_{t+tau, u+nu, v+phi}(p q/(p+q), P - C)
 *
 * The paper defines the RI three-centre integrals (pq|A) and the metric
 * M_AB = (A|B) (Sec. 2.2, eq. g_modified); their nuclear derivatives enter the
 * three-term derivative of the RI four-index object (Sec. 2.2, last equation).
 * Derivatives here are taken for EVERY centre explicitly by differentiating the
 * Gaussian itself, d/dA_x x_A^i e^{-a x_A^2} = 2a x_A^{i+1} e - i x_A^{i-1} e,
 * so translational invariance is a genuine check and not built in.
 *
 * Basis functions are Cartesian, each component normalised to one; component
 * order x,y,z and xx,xy,xz,yy,yz,zz.  Every shell is one primitive.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXL1D 5          /* 1D index range 0..4 (l<=3 plus one derivative) */
#define MAXT (2 * MAXL1D) /* Hermite index range */
#define MAXLR 10          /* R table edge */

static const int NCART[4] = {1, 3, 6, 10};
static const int CART[4][10][3] = {
    {{0, 0, 0}},
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
    {{2, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}},
    {{3, 0, 0}, {2, 1, 0}, {2, 0, 1}, {1, 2, 0}, {1, 1, 1}, {1, 0, 2}, {0, 3, 0}, {0, 2, 1}, {0, 1, 2}, {0, 0, 3}},
};

/* ---------------------------------------------------------------- Boys --- */
/* F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt.
 * Small/moderate T: the all-positive series
 *   F_m(T) = e^{-T} sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1))
 * for the top order, then the downward recursion F_m = (2T F_{m+1} + e^{-T})/(2m+1).
 * Large T: F_0 = (1/2) sqrt(pi/T) erf(sqrt T) and the upward recursion
 * F_{m+1} = ((2m+1) F_m - e^{-T}) / (2T), which is stable there. */
void oracle_boys(int mmax, double T, double *F)
{
    if (T < 35.0) {
        double et = exp(-T);
        double term = 1.0 / (2 * mmax + 1), sum = term;
        for (int k = 1; k < 400; ++k) {
            term *= 2.0 * T / (2 * mmax + 2 * k + 1);
            sum += term;
            if (term < 1e-18 * sum) break;
        }
        F[mmax] = et * sum;
        for (int m = mmax - 1; m >= 0; --m) F[m] = (2.0 * T * F[m + 1] + et) / (2 * m + 1);
    } else {
        double et = exp(-T);
        F[0] = 0.5 * sqrt(M_PI / T) * erf(sqrt(T));
        for (int m = 0; m < mmax; ++m) F[m + 1] = ((2 * m + 1) * F[m] - et) / (2.0 * T);
    }
}

static double dfact(int n)
{
    double r = 1.0;
    while (n > 1) { r *= n; n -= 2; }
    return r;
}

double oracle_cart_norm(double a, int lx, int ly, int lz)
{
    int l = lx + ly + lz;
    return pow(2.0 * a / M_PI, 0.75) * pow(4.0 * a, 0.5 * l) /
           sqrt(dfact(2 * lx - 1) * dfact(2 * ly - 1) * dfact(2 * lz - 1));
}

/* ------------------------------------------------- Hermite coefficients --- */
/* E[i][j][t] for the 1D product x_A^i x_B^j e^{-a x_A^2 - b x_B^2}.
 * b = 0 with j = 0 gives the expansion of a single Gaussian. */
typedef double Etab[MAXL1D][MAXL1D][MAXT + 1];

static void hermite_E(int imax, int jmax, double a, double b, double Ax, double Bx, Etab E)
{
    double p = a + b, mu = a * b / p;
    double Xab = Ax - Bx;
    double Xpa = -b / p * Xab, Xpb = a / p * Xab;
    memset(E, 0, sizeof(Etab));
    E[0][0][0] = exp(-mu * Xab * Xab);
    for (int i = 0; i <= imax; ++i) {
        for (int j = 0; j <= jmax; ++j) {
            if (i == 0 && j == 0) continue;
            for (int t = 0; t <= i + j; ++t) {
                double v;
                if (i > 0) {
                    v = Xpa * E[i - 1][j][t];
                    if (t > 0) v += E[i - 1][j][t - 1] / (2.0 * p);
                    if (t + 1 <= i - 1 + j) v += (t + 1) * E[i - 1][j][t + 1];
                } else {
                    v = Xpb * E[i][j - 1][t];
                    if (t > 0) v += E[i][j - 1][t - 1] / (2.0 * p);
                    if (t + 1 <= i + j - 1) v += (t + 1) * E[i][j - 1][t + 1];
                }
                E[i][j][t] = v;
            }
        }
    }
}

/* ------------------------------------------- Hermite Coulomb integrals --- */
typedef double Rtab[MAXLR][MAXLR][MAXLR];

/* R_{tuv} = R^0_{tuv}(alpha, X, Y, Z) for t+u+v <= L, via
 *   R^n_{000} = (-2 alpha)^n F_n(alpha |PC|^2)
 *   R^n_{t+1,u,v} = t R^{n+1}_{t-1,u,v} + X R^{n+1}_{t,u,v}   (likewise u, v) */
static void hermite_R(int L, double alpha, double X, double Y, double Z, Rtab R)
{
    static __thread double Rn[MAXLR + 1][MAXLR][MAXLR][MAXLR];
    double F[MAXLR + 1];
    oracle_boys(L, alpha * (X * X + Y * Y + Z * Z), F);
    for (int n = 0; n <= L; ++n) Rn[n][0][0][0] = pow(-2.0 * alpha, n) * F[n];
    for (int n = L - 1; n >= 0; --n) {
        int lmax = L - n;
        for (int s = 1; s <= lmax; ++s)
            for (int t = 0; t <= s; ++t)
                for (int u = 0; u <= s - t; ++u) {
                    int v = s - t - u;
                    double r;
                    if (t > 0) {
                        r = X * Rn[n + 1][t - 1][u][v];
                        if (t > 1) r += (t - 1) * Rn[n + 1][t - 2][u][v];
                    } else if (u > 0) {
                        r = Y * Rn[n + 1][t][u - 1][v];
                        if (u > 1) r += (u - 1) * Rn[n + 1][t][u - 2][v];
                    } else {
                        r = Z * Rn[n + 1][t][u][v - 1];
                        if (v > 1) r += (v - 1) * Rn[n + 1][t][u][v - 2];
                    }
                    Rn[n][t][u][v] = r;
                }
    }
    for (int t = 0; t <= L; ++t)
        for (int u = 0; u <= L - t; ++u)
            for (int v = 0; v <= L - t - u; ++v) R[t][u][v] = Rn[0][t][u][v];
}

/* -------------------------------------------- one unnormalised integral --- */
/* Tables for one shell triplet (a on A, b on B, c on C). */
typedef struct {
    Etab Ex, Ey, Ez;    /* pair a,b */
    Etab Cx, Cy, Cz;    /* single Gaussian c */
    Rtab R;
    double pref;
} trip_t;

static void trip_setup(trip_t *T, int la, int lb, int lc, int extra,
                       double a, const double *A, double b, const double *B,
                       double c, const double *C)
{
    double p = a + b;
    hermite_E(la + extra, lb + extra, a, b, A[0], B[0], T->Ex);
    hermite_E(la + extra, lb + extra, a, b, A[1], B[1], T->Ey);
    hermite_E(la + extra, lb + extra, a, b, A[2], B[2], T->Ez);
    hermite_E(lc + extra, 0, c, 0.0, C[0], C[0], T->Cx);
    hermite_E(lc + extra, 0, c, 0.0, C[1], C[1], T->Cy);
    hermite_E(lc + extra, 0, c, 0.0, C[2], C[2], T->Cz);
    double P[3];
    for (int d = 0; d < 3; ++d) P[d] = (a * A[d] + b * B[d]) / p;
    double alpha = p * c / (p + c);
    hermite_R(la + lb + lc + extra, alpha, P[0] - C[0], P[1] - C[1], P[2] - C[2], T->R);
    T->pref = 2.0 * pow(M_PI, 2.5) / (p * c * sqrt(p + c));
}

/* (x^i y^j z^k | x^.. | x^..) with the triplet tables; negative index -> 0 */
static double trip_int(const trip_t *T, const int *ia, const int *ib, const int *ic)
{
    for (int d = 0; d < 3; ++d)
        if (ia[d] < 0 || ib[d] < 0 || ic[d] < 0) return 0.0;
    double s = 0.0;
    for (int t = 0; t <= ia[0] + ib[0]; ++t) {
        double ex = T->Ex[ia[0]][ib[0]][t];
        if (ex == 0.0) continue;
        for (int u = 0; u <= ia[1] + ib[1]; ++u) {
            double ey = T->Ey[ia[1]][ib[1]][u];
            if (ey == 0.0) continue;
            for (int v = 0; v <= ia[2] + ib[2]; ++v) {
                double ez = T->Ez[ia[2]][ib[2]][v];
                if (ez == 0.0) continue;
                double inner = 0.0;
                for (int tau = 0; tau <= ic[0]; ++tau)
                    for (int nu = 0; nu <= ic[1]; ++nu)
                        for (int phi = 0; phi <= ic[2]; ++phi) {
                            double ec = T->Cx[ic[0]][0][tau] * T->Cy[ic[1]][0][nu] * T->Cz[ic[2]][0][phi];
                            if (ec == 0.0) continue;
                            double sg = ((tau + nu + phi) & 1) ? -1.0 : 1.0;
                            inner += sg * ec * T->R[t + tau][u + nu][v + phi];
                        }
                s += ex * ey * ez * inner;
            }
        }
    }
    return T->pref * s;
}

/* d/dX_d of the unnormalised Gaussian with exponent e and powers l[] at X:
 * 2e * (l + 1_d) - l_d * (l - 1_d).  which = 0,1,2 selects the function. */
static double trip_deriv(const trip_t *T, const int *ia, const int *ib, const int *ic,
                         int which, int d, double e)
{
    int up[3][3], dn[3][3];
    for (int k = 0; k < 3; ++k) {
        up[0][k] = dn[0][k] = ia[k];
        up[1][k] = dn[1][k] = ib[k];
        up[2][k] = dn[2][k] = ic[k];
    }
    up[which][d] += 1;
    dn[which][d] -= 1;
    double v = 2.0 * e * trip_int(T, up[0], up[1], up[2]);
    int l = (which == 0 ? ia : which == 1 ? ib : ic)[d];
    if (l > 0) v -= l * trip_int(T, dn[0], dn[1], dn[2]);
    return v;
}

/* ---------------------------------------------------------- public API --- */
/* Shell lists: centre xyz [n][3], l [n], exponent [n]; offsets computed here. */
static void offsets(int n, const int *l, int *off)
{
    off[0] = 0;
    for (int s = 0; s < n; ++s) off[s + 1] = off[s] + NCART[l[s]];
}

/* (mu nu | P) for all AO pairs and aux functions: out[naux][nao][nao] */
void oracle_int3c(int nao_sh, const double *ao_xyz, const int *ao_l, const double *ao_e,
                  int naux_sh, const double *aux_xyz, const int *aux_l, const double *aux_e,
                  double *out)
{
    int *ao_off = malloc(sizeof(int) * (nao_sh + 1));
    int *ax_off = malloc(sizeof(int) * (naux_sh + 1));
    offsets(nao_sh, ao_l, ao_off);
    offsets(naux_sh, aux_l, ax_off);
    int nao = ao_off[nao_sh];
#pragma omp parallel for schedule(dynamic)
    for (int sa = 0; sa < nao_sh; ++sa) {
        trip_t *T = malloc(sizeof(trip_t));
        for (int sb = 0; sb < nao_sh; ++sb)
            for (int sc = 0; sc < naux_sh; ++sc) {
                trip_setup(T, ao_l[sa], ao_l[sb], aux_l[sc], 0, ao_e[sa], ao_xyz + 3 * sa,
                           ao_e[sb], ao_xyz + 3 * sb, aux_e[sc], aux_xyz + 3 * sc);
                for (int ca = 0; ca < NCART[ao_l[sa]]; ++ca)
                    for (int cb = 0; cb < NCART[ao_l[sb]]; ++cb)
                        for (int cc = 0; cc < NCART[aux_l[sc]]; ++cc) {
                            const int *ia = CART[ao_l[sa]][ca], *ib = CART[ao_l[sb]][cb],
                                      *ic = CART[aux_l[sc]][cc];
                            double nrm = oracle_cart_norm(ao_e[sa], ia[0], ia[1], ia[2]) *
                                         oracle_cart_norm(ao_e[sb], ib[0], ib[1], ib[2]) *
                                         oracle_cart_norm(aux_e[sc], ic[0], ic[1], ic[2]);
                            out[((size_t)(ax_off[sc] + cc) * nao + ao_off[sa] + ca) * nao +
                                ao_off[sb] + cb] = nrm * trip_int(T, ia, ib, ic);
                        }
            }
        free(T);
    }
    free(ao_off);
    free(ax_off);
}

/* (P|Q) over aux functions: out[naux][naux] */
void oracle_int2c(int naux_sh, const double *aux_xyz, const int *aux_l, const double *aux_e,
                  double *out)
{
    int *off = malloc(sizeof(int) * (naux_sh + 1));
    offsets(naux_sh, aux_l, off);
    int n = off[naux_sh];
    static const int zero3[3] = {0, 0, 0};
    trip_t *T = malloc(sizeof(trip_t));
    for (int sp = 0; sp < naux_sh; ++sp)
        for (int sq = 0; sq < naux_sh; ++sq) {
            /* bra = single Gaussian P: treat as pair (P, s-function with exponent 0) */
            trip_setup(T, aux_l[sp], 0, aux_l[sq], 0, aux_e[sp], aux_xyz + 3 * sp, 0.0,
                       aux_xyz + 3 * sp, aux_e[sq], aux_xyz + 3 * sq);
            for (int cp = 0; cp < NCART[aux_l[sp]]; ++cp)
                for (int cq = 0; cq < NCART[aux_l[sq]]; ++cq) {
                    const int *ip = CART[aux_l[sp]][cp], *iq = CART[aux_l[sq]][cq];
                    double nrm = oracle_cart_norm(aux_e[sp], ip[0], ip[1], ip[2]) *
                                 oracle_cart_norm(aux_e[sq], iq[0], iq[1], iq[2]);
                    out[(size_t)(off[sp] + cp) * n + off[sq] + cq] = nrm * trip_int(T, ip, zero3, iq);
                }
        }
    free(T);
    free(off);
}

/* Gradient contraction of the three-centre derivatives:
 *   grad[o][X][d] += sum_{mu nu P} W[o][P][mu][nu] * d(mu nu|P)/dX_d
 * with every centre differentiated explicitly.  ao_atom / aux_atom map shells
 * to atoms.  If atom_mask is non-NULL, only triplets touching a masked atom are
 * evaluated and only masked atoms receive contributions. */
void oracle_int3c_grad(int nao_sh, const double *ao_xyz, const int *ao_l, const double *ao_e,
                       const int *ao_atom, int naux_sh, const double *aux_xyz, const int *aux_l,
                       const double *aux_e, const int *aux_atom, int natm, int nout,
                       const double *W, const unsigned char *atom_mask, double *grad)
{
    int *ao_off = malloc(sizeof(int) * (nao_sh + 1));
    int *ax_off = malloc(sizeof(int) * (naux_sh + 1));
    offsets(nao_sh, ao_l, ao_off);
    offsets(naux_sh, aux_l, ax_off);
    size_t nao = ao_off[nao_sh], naux = ax_off[naux_sh];
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double *part = calloc((size_t)nth * nout * natm * 3, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *g = part + (size_t)tid * nout * natm * 3;
        trip_t *T = malloc(sizeof(trip_t));
#pragma omp for schedule(dynamic)
        for (int sa = 0; sa < nao_sh; ++sa)
            for (int sb = 0; sb < nao_sh; ++sb)
                for (int sc = 0; sc < naux_sh; ++sc) {
                    int at[3] = {ao_atom[sa], ao_atom[sb], aux_atom[sc]};
                    if (atom_mask && !atom_mask[at[0]] && !atom_mask[at[1]] && !atom_mask[at[2]]) continue;
                    trip_setup(T, ao_l[sa], ao_l[sb], aux_l[sc], 1, ao_e[sa], ao_xyz + 3 * sa,
                               ao_e[sb], ao_xyz + 3 * sb, aux_e[sc], aux_xyz + 3 * sc);
                    double ex[3] = {ao_e[sa], ao_e[sb], aux_e[sc]};
                    for (int ca = 0; ca < NCART[ao_l[sa]]; ++ca)
                        for (int cb = 0; cb < NCART[ao_l[sb]]; ++cb)
                            for (int cc = 0; cc < NCART[aux_l[sc]]; ++cc) {
                                const int *ia = CART[ao_l[sa]][ca], *ib = CART[ao_l[sb]][cb],
                                          *ic = CART[aux_l[sc]][cc];
                                double nrm = oracle_cart_norm(ao_e[sa], ia[0], ia[1], ia[2]) *
                                             oracle_cart_norm(ao_e[sb], ib[0], ib[1], ib[2]) *
                                             oracle_cart_norm(aux_e[sc], ic[0], ic[1], ic[2]);
                                size_t P = ax_off[sc] + cc, mu = ao_off[sa] + ca, nu = ao_off[sb] + cb;
                                for (int which = 0; which < 3; ++which) {
                                    if (atom_mask && !atom_mask[at[which]]) continue;
                                    for (int d = 0; d < 3; ++d) {
                                        double dv = nrm * trip_deriv(T, ia, ib, ic, which, d, ex[which]);
                                        for (int o = 0; o < nout; ++o)
                                            g[((size_t)o * natm + at[which]) * 3 + d] +=
                                                W[(((size_t)o * naux + P) * nao + mu) * nao + nu] * dv;
                                    }
                                }
                            }
                }
        free(T);
    }
    for (int t = 0; t < nth; ++t)
        for (size_t k = 0; k < (size_t)nout * natm * 3; ++k) grad[k] += part[(size_t)t * nout * natm * 3 + k];
    free(part);
    free(ao_off);
    free(ax_off);
}

/* grad[o][X][d] += sum_{PQ} W[o][P][Q] d(P|Q)/dX_d, both centres explicit. */
void oracle_int2c_grad(int naux_sh, const double *aux_xyz, const int *aux_l, const double *aux_e,
                       const int *aux_atom, int natm, int nout, const double *W, double *grad)
{
    int *off = malloc(sizeof(int) * (naux_sh + 1));
    offsets(naux_sh, aux_l, off);
    size_t n = off[naux_sh];
    trip_t *T = malloc(sizeof(trip_t));
    static const int zero[3] = {0, 0, 0};
    for (int sp = 0; sp < naux_sh; ++sp)
        for (int sq = 0; sq < naux_sh; ++sq) {
            trip_setup(T, aux_l[sp], 0, aux_l[sq], 1, aux_e[sp], aux_xyz + 3 * sp, 0.0,
                       aux_xyz + 3 * sp, aux_e[sq], aux_xyz + 3 * sq);
            for (int cp = 0; cp < NCART[aux_l[sp]]; ++cp)
                for (int cq = 0; cq < NCART[aux_l[sq]]; ++cq) {
                    const int *ip = CART[aux_l[sp]][cp], *iq = CART[aux_l[sq]][cq];
                    double nrm = oracle_cart_norm(aux_e[sp], ip[0], ip[1], ip[2]) *
                                 oracle_cart_norm(aux_e[sq], iq[0], iq[1], iq[2]);
                    size_t P = off[sp] + cp, Q = off[sq] + cq;
                    for (int d = 0; d < 3; ++d) {
                        double dP = nrm * trip_deriv(T, ip, zero, iq, 0, d, aux_e[sp]);
                        double dQ = nrm * trip_deriv(T, ip, zero, iq, 2, d, aux_e[sq]);
                        for (int o = 0; o < nout; ++o) {
                            double w = W[((size_t)o * n + P) * n + Q];
                            grad[((size_t)o * natm + aux_atom[sp]) * 3 + d] += w * dP;
                            grad[((size_t)o * natm + aux_atom[sq]) * 3 + d] += w * dQ;
                        }
                    }
                }
        }
    free(T);
    free(off);
}
