// Gaussian integrals of the ris auxiliary expansion on gfx950 (FP64 VALU).
//
// The RI kernel of TDDFT-ris needs the three-centre integrals (mu nu|P), the
// metric (P|Q) (Sec. 2.2, eq. g_modified) and their nuclear derivatives (the
// three-term RI derivative at the end of Sec. 2.2).  Every shell is a single
// Cartesian primitive, so each integral is one McMurchie-Davidson expansion:
//   (ab|c) = 2 pi^{5/2} / (p q sqrt(p+q)) exp(-mu |AB|^2)
//            sum_T E^{ab}_T Lambda^c_T,
//   Lambda^s_T = R_T,  Lambda^{p_k}_T = -R_{T+1_k} / (2q),
// with Hermite coefficients E (recurrence over the Gaussian product) and
// Hermite Coulomb integrals R_{tuv}(alpha, P-C) (recurrence over the Boys
// function).  Derivatives used:
//   d/dA_d (ab|c): E_x replaced by 2a E_{i+1} - i E_{i-1} in direction d,
//   d/dC_d (ab|c) = -sum_T E^{ab}_T Lambda^c_{T+1_d}  (R depends on P-C only),
//   d/dB = -d/dA - d/dC (translational invariance of the integral).
// All angular loops are unrolled at compile time per (la, lb, lc) class so the
// recurrence tables live in registers.
#include <algorithm>
#include <utility>
#include <vector>

#include "ris_boys.hpp"
#include "ris_common.hpp"

namespace ris {
namespace {

template <typename F, int... Is>
__device__ __forceinline__ void sfor_impl(F &&f, std::integer_sequence<int, Is...>)
{
    (f(std::integral_constant<int, Is>{}), ...);
}
// compile-time loop: f(integral_constant<int, 0..N-1>)
template <int N, typename F>
__device__ __forceinline__ void sfor(F &&f)
{
    sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// power of direction d in Cartesian component c of angular momentum l
// (order x,y,z and xx,xy,xz,yy,yz,zz)
__host__ __device__ constexpr int cpow(int l, int c, int d)
{
    return l == 0 ? 0
         : l == 1 ? (c == d ? 1 : 0)
         : d == 0 ? (c == 0 ? 2 : (c == 1 || c == 2) ? 1 : 0)
         : d == 1 ? (c == 1 ? 1 : c == 3 ? 2 : c == 4 ? 1 : 0)
                  : (c == 2 ? 1 : c == 4 ? 1 : c == 5 ? 2 : 0);
}
// 1/sqrt((2lx-1)!!(2ly-1)!!(2lz-1)!!) for the component
__host__ __device__ constexpr double cnorm(int l, int c)
{
    return (l == 2 && (c == 0 || c == 3 || c == 5)) ? 0.57735026918962576451 : 1.0;
}

// packed index of R_{tuv}: level s = t+u+v, then (u+v), then v
__host__ __device__ constexpr int ridx(int t, int u, int v)
{
    return (t + u + v) * (t + u + v + 1) * (t + u + v + 2) / 6 + (u + v) * (u + v + 1) / 2 + v;
}
__host__ __device__ constexpr int rsize(int L) { return (L + 1) * (L + 2) * (L + 3) / 6; }

// Hermite coefficients of one direction, E[i][j][t], i <= I, j <= J, without
// the exp(-mu X_AB^2) factor (applied once per shell pair).
template <int I, int J>
struct Herm {
    double e[I + 1][J + 1][I + J + 1];
};

template <int I, int J>
__device__ __forceinline__ void herm_build(double xpa, double xpb, double inv2p, Herm<I, J> &H)
{
    sfor<I + 1>([&](auto ii) {
        sfor<J + 1>([&](auto jj) {
            sfor<I + J + 1>([&](auto tt) { H.e[ii][jj][tt] = 0.0; });
        });
    });
    H.e[0][0][0] = 1.0;
    sfor<I>([&](auto im) {  // i = im + 1, j = 0
        constexpr int i = im + 1;
        sfor<i + 1>([&](auto tt) {
            constexpr int t = tt;
            double v = 0.0;
            if constexpr (t > 0) v += inv2p * H.e[i - 1][0][t - 1];
            if constexpr (t <= i - 1) v += xpa * H.e[i - 1][0][t];
            if constexpr (t + 1 <= i - 1) v += (t + 1) * H.e[i - 1][0][t + 1];
            H.e[i][0][t] = v;
        });
    });
    sfor<J>([&](auto jm) {
        constexpr int j = jm + 1;
        sfor<I + 1>([&](auto ii) {
            constexpr int i = ii;
            sfor<i + j + 1>([&](auto tt) {
                constexpr int t = tt;
                double v = 0.0;
                if constexpr (t > 0) v += inv2p * H.e[i][j - 1][t - 1];
                if constexpr (t <= i + j - 1) v += xpb * H.e[i][j - 1][t];
                if constexpr (t + 1 <= i + j - 1) v += (t + 1) * H.e[i][j - 1][t + 1];
                H.e[i][j][t] = v;
            });
        });
    });
}

// R_{tuv} for t+u+v <= L into r[ridx], in place from level n = L down to 0.
template <int L>
__device__ __forceinline__ void hermite_r(double alpha, double X, double Y, double Z,
                                          const double *__restrict__ boys, double (&r)[rsize(L)])
{
    double F[L + 1];
    boys_eval<L>(alpha * (X * X + Y * Y + Z * Z), boys, F);
    const double m2a = -2.0 * alpha;
    double pw[L + 1];
    pw[0] = 1.0;
    sfor<L>([&](auto n) { pw[n + 1] = pw[n] * m2a; });
    r[0] = pw[L] * F[L];
    sfor<L>([&](auto nn) {
        constexpr int n = L - 1 - nn;  // level n, entries with sum <= L - n
        sfor<L - n>([&](auto ss) {
            constexpr int s = L - n - ss;  // descending s
            sfor<s + 1>([&](auto tt) {
                constexpr int t = s - tt;
                sfor<s - t + 1>([&](auto uu) {
                    constexpr int u = s - t - uu;
                    constexpr int v = s - t - u;
                    double val;
                    if constexpr (t > 0) {
                        val = X * r[ridx(t - 1, u, v)];
                        if constexpr (t > 1) val += (t - 1) * r[ridx(t - 2, u, v)];
                    } else if constexpr (u > 0) {
                        val = Y * r[ridx(t, u - 1, v)];
                        if constexpr (u > 1) val += (u - 1) * r[ridx(t, u - 2, v)];
                    } else {
                        val = Z * r[ridx(t, u, v - 1)];
                        if constexpr (v > 1) val += (v - 1) * r[ridx(t, u, v - 2)];
                    }
                    r[ridx(t, u, v)] = val;
                });
            });
        });
        r[0] = pw[n] * F[n];
    });
}

// sum_{t,u,v} ex[t] ey[u] ez[v] R[t+SX][u+SY][v+SZ] for compile-time extents
template <int NX, int NY, int NZ, int SX, int SY, int SZ, int RS>
__device__ __forceinline__ double hsum(const double *ex, const double *ey, const double *ez,
                                       const double (&r)[RS])
{
    double acc = 0.0;
    sfor<NX>([&](auto t) {
        double ay = 0.0;
        sfor<NY>([&](auto u) {
            double az = 0.0;
            sfor<NZ>([&](auto v) { az += ez[v] * r[ridx(t + SX, u + SY, v + SZ)]; });
            ay += ey[u] * az;
        });
        acc += ex[t] * ay;
    });
    return acc;
}

struct PairGeo {
    double a, b, p, xpa[3], xpb[3], P[3], kab;
};

__device__ __forceinline__ PairGeo pair_geo(const ShellTab &S, int sa, int sb)
{
    PairGeo g;
    const double A[3] = {S.x[sa], S.y[sa], S.z[sa]};
    const double B[3] = {S.x[sb], S.y[sb], S.z[sb]};
    g.a = S.exp[sa];
    g.b = S.exp[sb];
    g.p = g.a + g.b;
    const double ip = 1.0 / g.p;
    double ab2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        g.P[d] = (g.a * A[d] + g.b * B[d]) * ip;
        g.xpa[d] = g.P[d] - A[d];
        g.xpb[d] = g.P[d] - B[d];
        ab2 += (A[d] - B[d]) * (A[d] - B[d]);
    }
    g.kab = exp(-g.a * g.b * ip * ab2);
    return g;
}

constexpr double kTwoPi52 = 34.98683665524972497;  // 2 pi^{5/2}

// ------------------------------------------------------------------------
// (mu nu|P): one thread per ordered shell triplet of the class.
template <int LA, int LB, int LC>
__global__ __launch_bounds__(128) void k_int3c(ShellTab ao, int nao, int a0, int na, int b0, int nb,
                                               ShellTab aux, int c0, int nc, int pofs,
                                               const double *__restrict__ boys, double *__restrict__ X)
{
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (long)na * nb * nc) return;
    const int sb = b0 + (int)(tid % nb);
    const long r1 = tid / nb;
    const int sa = a0 + (int)(r1 % na);
    const int sc = c0 + (int)(r1 / na);

    constexpr int L = LA + LB + LC;
    const PairGeo g = pair_geo(ao, sa, sb);
    const double c = aux.exp[sc];
    const double PC[3] = {g.P[0] - aux.x[sc], g.P[1] - aux.y[sc], g.P[2] - aux.z[sc]};
    const double alpha = g.p * c / (g.p + c);
    double r[rsize(L)];
    hermite_r<L>(alpha, PC[0], PC[1], PC[2], boys, r);
    const double inv2p = 0.5 / g.p;
    Herm<LA, LB> Ex, Ey, Ez;
    herm_build<LA, LB>(g.xpa[0], g.xpb[0], inv2p, Ex);
    herm_build<LA, LB>(g.xpa[1], g.xpb[1], inv2p, Ey);
    herm_build<LA, LB>(g.xpa[2], g.xpb[2], inv2p, Ez);
    const double pref = kTwoPi52 / (g.p * c * sqrt(g.p + c)) * g.kab * ao.nrm[sa] * ao.nrm[sb] * aux.nrm[sc];
    const double cfac = (LC == 1) ? -0.5 / c : 1.0;
    const int mu0 = ao.off[sa], nu0 = ao.off[sb], P0 = aux.off[sc];
    sfor<ncart(LC)>([&](auto kc) {
        constexpr int sx = cpow(LC, kc, 0), sy = cpow(LC, kc, 1), sz = cpow(LC, kc, 2);
        sfor<ncart(LA)>([&](auto ka) {
            constexpr int ix = cpow(LA, ka, 0), iy = cpow(LA, ka, 1), iz = cpow(LA, ka, 2);
            double *row = X + ((size_t)(P0 - pofs + kc) * nao + (mu0 + ka)) * nao + nu0;
            sfor<ncart(LB)>([&](auto kb) {
                constexpr int jx = cpow(LB, kb, 0), jy = cpow(LB, kb, 1), jz = cpow(LB, kb, 2);
                const double v = hsum<ix + jx + 1, iy + jy + 1, iz + jz + 1, sx, sy, sz>(
                    Ex.e[ix][jx], Ey.e[iy][jy], Ez.e[iz][jz], r);
                row[kb] = pref * cfac * cnorm(LA, ka) * cnorm(LB, kb) * v;
            });
        });
    });
}

// ------------------------------------------------------------------------
// Fused derivative contraction.  One wave per (A shell, C shell); lanes walk
// the B shells of class LB.  For every ordered triplet and output o
//   w_o = alphaJ (D_I[mu nu] c_J[P] + D_J[mu nu] c_I[P]) + GammaK_o[P][mu nu]
//   accA_o[d] += 2 w_o d(mu nu|P)/dA_d,  accC_o[d] += w_o d(mu nu|P)/dC_d
// (weights symmetric in mu nu, so the bra-2 derivative folds into the factor
// 2 on bra 1 over ordered pairs).  The wave sum is written to
// partial[sa][sc][LB][o][6] for a deterministic reduction afterwards.
//
// G > 1: a wave takes G consecutive C shells of the class, lane l working on
// C shell l % G and every G-th partner (short screened partner lists, as for
// d shells, would otherwise leave most lanes idle); the sums are reduced
// over the lanes of each C shell.
template <int LA, int LB, int LC, int NO, int G>
__global__ __launch_bounds__(64) void k_int3c_deriv(ShellTab ao, int nao, int a0, int na, int b0, int nb,
                                                    ShellTab aux, int c0, int nc, int nshAux,
                                                    const double *__restrict__ boys, DerivJob job)
{
    // Waves are dispatched round-robin over the 8 XCDs; remap so each XCD walks
    // a contiguous range with the C shell fastest: waves resident together on
    // one XCD share the A shell and reuse its density rows from that XCD's L2.
    const int ncg = (nc + G - 1) / G;
    const int total = na * ncg;
    if ((int)blockIdx.x >= total) return;
    int lin;
    {
        const int q = total / 8, r = total % 8, x = blockIdx.x % 8, local = blockIdx.x / 8;
        lin = (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + local;
    }
    const int lane = threadIdx.x;
    const int sa = a0 + lin / ncg;
    const int cl = lane % G, csh = (lin % ncg) * G + cl;
    const bool cvalid = csh < nc;
    const int sc = c0 + min(csh, nc - 1);

    constexpr int L = LA + LB + LC + 1;
    const double Ax = ao.x[sa], Ay = ao.y[sa], Az = ao.z[sa];
    const double c = aux.exp[sc];
    const double Cx = aux.x[sc], Cy = aux.y[sc], Cz = aux.z[sc];
    const int mu0 = ao.off[sa], P0 = aux.off[sc];
    // K functions are the leading (s) J functions; gammaK holds [kbeg, kbeg + nK)
    const bool inK = P0 >= job.kbeg && P0 < job.kbeg + job.nK;
    const size_t nao2 = (size_t)nao * nao;
    // Every load below is issued on every lane and for every output slot
    // (slots past nout read the last output's data, C shells outside the K
    // block a density element scaled by 0): a load under a branch, even a
    // uniform one, is waited for on its own.
    const bool kin = LC == 0 && inK && job.gammaK;
    const double kf = kin ? 1.0 : 0.0;
    const double *gK = kin ? job.gammaK + (size_t)(P0 - job.kbeg) * nao2 : job.dens;
    const size_t gKo = kin ? (size_t)job.nK * nao2 : 0;
    const int olast = max(job.nout - 1, 0);

    double acc[NO][6];
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int k = 0; k < 6; ++k) acc[o][k] = 0.0;

    double cI[NO][ncart(LC)], cJ[NO][ncart(LC)];
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int k = 0; k < ncart(LC); ++k) {
            cI[o][k] = job.cvec[(size_t)job.stI[o] * job.nJ + P0 + k];
            cJ[o][k] = job.cvec[(size_t)job.stJ[o] * job.nJ + P0 + k];
        }

    // partners of sa in class LB: all of them, or the screened list
    int cnt = nb;
    const int *lst = nullptr;
    if (job.pair_ptr) {
        const int q0 = job.pair_ptr[(kMaxAOL + 1) * sa + LB];
        cnt = job.pair_ptr[(kMaxAOL + 1) * sa + LB + 1] - q0;
        lst = job.pair_idx + q0;
    }
    if (!cvalid) cnt = 0;  // lanes past the last C shell of the class
    for (int ib = lane / G; ib < cnt; ib += 64 / G) {
        const int sb = lst ? lst[ib] : b0 + ib;
        const double a = ao.exp[sa], b = ao.exp[sb];
        const double p = a + b, ip = 1.0 / p;
        const double Bx = ao.x[sb], By = ao.y[sb], Bz = ao.z[sb];
        const double P[3] = {(a * Ax + b * Bx) * ip, (a * Ay + b * By) * ip, (a * Az + b * Bz) * ip};
        const double ab2 = (Ax - Bx) * (Ax - Bx) + (Ay - By) * (Ay - By) + (Az - Bz) * (Az - Bz);
        const double kab = exp(-a * b * ip * ab2);
        const double alpha = p * c / (p + c);
        double r[rsize(L)];
        hermite_r<L>(alpha, P[0] - Cx, P[1] - Cy, P[2] - Cz, boys, r);
        const double inv2p = 0.5 * ip;
        Herm<LA + 1, LB> Ex, Ey, Ez;
        herm_build<LA + 1, LB>(P[0] - Ax, P[0] - Bx, inv2p, Ex);
        herm_build<LA + 1, LB>(P[1] - Ay, P[1] - By, inv2p, Ey);
        herm_build<LA + 1, LB>(P[2] - Az, P[2] - Bz, inv2p, Ez);
        const double pref = kTwoPi52 / (p * c * sqrt(p + c)) * kab * ao.nrm[sa] * ao.nrm[sb] * aux.nrm[sc];
        const double cfac = (LC == 1) ? -0.5 / c : 1.0;
        const int nu0 = ao.off[sb];
        const double twoa = 2.0 * a;

        sfor<ncart(LA)>([&](auto ka) {
            constexpr int ix = cpow(LA, ka, 0), iy = cpow(LA, ka, 1), iz = cpow(LA, ka, 2);
            sfor<ncart(LB)>([&](auto kb) {
                constexpr int jx = cpow(LB, kb, 0), jy = cpow(LB, kb, 1), jz = cpow(LB, kb, 2);
                const double *ex = Ex.e[ix][jx];
                const double *ey = Ey.e[iy][jy];
                const double *ez = Ez.e[iz][jz];
                // derivative coefficients 2a E_{i+1} - i E_{i-1} per direction
                double dx[ix + jx + 2], dy[iy + jy + 2], dz[iz + jz + 2];
                sfor<ix + jx + 2>([&](auto t) {
                    double v = twoa * Ex.e[ix + 1][jx][t];
                    if constexpr (ix > 0 && t <= ix - 1 + jx) v -= ix * Ex.e[ix - 1][jx][t];
                    dx[t] = v;
                });
                sfor<iy + jy + 2>([&](auto t) {
                    double v = twoa * Ey.e[iy + 1][jy][t];
                    if constexpr (iy > 0 && t <= iy - 1 + jy) v -= iy * Ey.e[iy - 1][jy][t];
                    dy[t] = v;
                });
                sfor<iz + jz + 2>([&](auto t) {
                    double v = twoa * Ez.e[iz + 1][jz][t];
                    if constexpr (iz > 0 && t <= iz - 1 + jz) v -= iz * Ez.e[iz - 1][jz][t];
                    dz[t] = v;
                });
                constexpr int NX = ix + jx + 1, NY = iy + jy + 1, NZ = iz + jz + 1;
                const size_t mn = (size_t)(mu0 + ka) * nao + nu0 + kb;
                // the symmetric K weights are read from their lower triangle (row >= column)
                const size_t mnl = (mu0 + ka >= nu0 + kb) ? mn : (size_t)(nu0 + kb) * nao + mu0 + ka;
                // Coulomb densities of this (mu, nu): loaded once for all auxiliary components
                double dI[NO], dJ[NO];
#pragma unroll
                for (int o = 0; o < NO; ++o) {
                    if constexpr (LB == 2 && LC == 1) {
                        // these classes spill: loads and sums held back by the
                        // output test keep fewer values live and measured faster
                        dI[o] = (o < job.nout) ? job.alphaJ * job.dens[(size_t)job.stI[o] * nao2 + mn] : 0.0;
                        dJ[o] = (o < job.nout) ? job.alphaJ * job.dens[(size_t)job.stJ[o] * nao2 + mn] : 0.0;
                    } else {
                        dI[o] = job.alphaJ * job.dens[(size_t)job.stI[o] * nao2 + mn];
                        dJ[o] = job.alphaJ * job.dens[(size_t)job.stJ[o] * nao2 + mn];
                    }
                }
                sfor<ncart(LC)>([&](auto kc) {
                    constexpr int sx = cpow(LC, kc, 0), sy = cpow(LC, kc, 1), sz = cpow(LC, kc, 2);
                    const double f = pref * cfac * cnorm(LA, ka) * cnorm(LB, kb);
                    double dA[3], dC[3];
                    dA[0] = f * hsum<NX + 1, NY, NZ, sx, sy, sz>(dx, ey, ez, r);
                    dA[1] = f * hsum<NX, NY + 1, NZ, sx, sy, sz>(ex, dy, ez, r);
                    dA[2] = f * hsum<NX, NY, NZ + 1, sx, sy, sz>(ex, ey, dz, r);
                    dC[0] = -f * hsum<NX, NY, NZ, sx + 1, sy, sz>(ex, ey, ez, r);
                    dC[1] = -f * hsum<NX, NY, NZ, sx, sy + 1, sz>(ex, ey, ez, r);
                    dC[2] = -f * hsum<NX, NY, NZ, sx, sy, sz + 1>(ex, ey, ez, r);
#pragma unroll
                    for (int o = 0; o < NO; ++o) {
                        if constexpr (LB == 2 && LC == 1)
                            if (o >= job.nout) continue;
                        double w = dI[o] * cJ[o][kc] + dJ[o] * cI[o][kc];
                        // K functions are s shells: one component
                        if constexpr (LC == 0) w += kf * gK[(size_t)min(o, olast) * gKo + mnl];
                        const double w2 = 2.0 * w;
                        acc[o][0] += w2 * dA[0];
                        acc[o][1] += w2 * dA[1];
                        acc[o][2] += w2 * dA[2];
                        acc[o][3] += w * dC[0];
                        acc[o][4] += w * dC[1];
                        acc[o][5] += w * dC[2];
                    }
                });
            });
        });
    }
    // reduction over the lanes of each C shell (fixed order, deterministic)
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            double v = acc[o][k];
#pragma unroll
            for (int off = 32; off >= G; off >>= 1) v += __shfl_xor(v, off, 64);
            acc[o][k] = v;
        }
    if (lane < G && cvalid) {
        // only the job's outputs: the partial slots of other outputs are left as they are
        double *dst = job.partial + (((size_t)sa * nshAux + sc) * (kMaxAOL + 1) + LB) * NO * 6;
#pragma unroll
        for (int o = 0; o < NO; ++o)
            if (o < job.nout) {
#pragma unroll
                for (int k = 0; k < 6; ++k) dst[o * 6 + k] = acc[o][k];
            }
    }
}

// ------------------------------------------------------------------------
// The exchange weights gammaK are the bulk of what the contraction reads, and
// in place (lanes over B partners) every lane reads its own scattered element,
// half of them across rows.  Their s-shell classes can instead run on a copy
// with the K function fastest: k_pack_gamma copies the lower block of every
// kept shell pair into Gc[o][q][k]; k_int3c_deriv_k then takes one A shell
// and 16 consecutive K functions per wave, its four quarter-waves walking
// different B partners, so the 16 lanes of a quarter read 16 consecutive k of
// one function pair (one 128-byte line) and share its density elements.

// One workgroup per (output, A shell a, 64 consecutive k).  For each row mu
// of a, the columns of a's kept partners that start before a (the flattened
// list pc: column * 8 + the partner's function count, and the block start
// + column index) go through LDS 64 at a time: each wave reads a contiguous
// row segment of one plane k, then each wave writes one column's 64 values of
// k as a contiguous run.  The diagonal block (a, a) is copied element by
// element from the lower triangle afterwards.  What is stored is the whole
// weight of the s-shell triplets, the Coulomb part added on the way:
//   Gamma_o^k[mu nu] + alphaJ (D_I[mu nu] c_J[k] + D_J[mu nu] c_I[k])
// (symmetric in mu nu like Gamma; the density elements are the same for
// all lanes).
constexpr int kPackCols = 64;
__global__ __launch_bounds__(256) void k_pack_gamma(const int *__restrict__ off, int lb1, int lb2, int nsh, int nao,
                                                    int nK, const double *__restrict__ G,
                                                    const int *__restrict__ pk_ptr, const int *__restrict__ pk_base,
                                                    const int *__restrict__ pc_ptr, const int *__restrict__ pc_cn,
                                                    const int *__restrict__ pc_qb, long nfq, double *__restrict__ Gc,
                                                    DerivJob job)
{
    __shared__ double tile[64][kPackCols + 1];  // [k][column]; odd row stride: column reads by k are conflict-free
    const int ngrp = (nK + 63) / 64;
    const int g = blockIdx.x % ngrp;
    const int a = (blockIdx.x / ngrp) % nsh;
    const int o = blockIdx.x / (ngrp * nsh);
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int k0 = g * 64, nk = min(64, nK - k0);
    const size_t nn = (size_t)nao * nao;
    const double *Gb = G + ((size_t)o * nK + k0) * nn;  // plane k0 + kl at Gb + kl * nn
    double *Go = Gc + (size_t)o * nfq * nK + k0;
    const int na = ncart(a >= lb2 ? 2 : (a >= lb1 ? 1 : 0));
    const int mu0 = off[a], j0 = pc_ptr[a], j1 = pc_ptr[a + 1];
    // Coulomb factors of this lane's K function (J function kbeg + k)
    const int kc = job.kbeg + k0 + min(lane, nk - 1);
    const double cJa = job.alphaJ * job.cvec[(size_t)job.stJ[o] * job.nJ + kc];
    const double cIa = job.alphaJ * job.cvec[(size_t)job.stI[o] * job.nJ + kc];
    const double *DI = job.dens + (size_t)job.stI[o] * nn, *DJ = job.dens + (size_t)job.stJ[o] * nn;
    for (int ka = 0; ka < na; ++ka) {
        const size_t row = (size_t)(mu0 + ka) * nao;
        for (int jc = j0; jc < j1; jc += kPackCols) {
            const int nc = min(kPackCols, j1 - jc);
            {
                // all 16 loads of the wave in flight together: plane and
                // column clamped into range, the extra rows of the tile unused
                const int col = pc_cn[jc + min(lane, nc - 1)] >> 3;
                double v[16];
#pragma unroll
                for (int i = 0; i < 16; ++i) v[i] = Gb[(size_t)min(wv + 4 * i, nk - 1) * nn + row + col];
#pragma unroll
                for (int i = 0; i < 16; ++i) tile[wv + 4 * i][lane] = v[i];
            }
            __syncthreads();
            if (lane < nk)
                for (int c = wv; c < nc; c += 4) {
                    const int cn = pc_cn[jc + c];
                    const long q = (long)pc_qb[jc + c] + (long)ka * (cn & 7);
                    const size_t mn = row + (cn >> 3);
                    Go[(size_t)q * nK + lane] = tile[lane][c] + DI[mn] * cJa + DJ[mn] * cIa;
                }
            __syncthreads();
        }
    }
    // the diagonal block: the last partner in a's list, its upper elements
    // taken from the lower triangle
    const long qd = pk_base[pk_ptr[a + 1] - 1];
    if (lane < nk)
        for (int e = wv; e < na * na; e += 4) {
            const int ka = e / na, kb = e % na;
            const size_t mn = (size_t)(mu0 + max(ka, kb)) * nao + mu0 + min(ka, kb);
            Go[(size_t)(qd + e) * nK + lane] = Gb[lane * nn + mn] + DI[mn] * cJa + DJ[mn] * cIa;
        }
}

// The s-shell (LC = 0) classes of the K block on the copy: the same triplet
// terms as k_int3c_deriv, a wave per (A shell, 16 K functions), lane l on
// K function l % 16 and every fourth partner from l / 16; each lane owns the
// partial slot of its (A shell, C shell) after the sum over its quarters.
template <int LA, int LB, int NO>
__global__ __launch_bounds__(64) void k_int3c_deriv_k(ShellTab ao, int nao, int a0, int na, ShellTab aux, int c0,
                                                      int nc, int nshAux, const double *__restrict__ boys,
                                                      DerivJob job)
{
    constexpr int QL = 16, NQ = 64 / QL;
    const int ncg = (nc + QL - 1) / QL;
    const int total = na * ncg;
    if ((int)blockIdx.x >= total) return;
    int lin;
    {
        // each XCD walks a contiguous range, the C-shell group fastest
        const int q = total / 8, r = total % 8, x = blockIdx.x % 8, local = blockIdx.x / 8;
        lin = (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + local;
    }
    const int lane = threadIdx.x, slot = lane / QL;
    const int sa = a0 + lin / ncg;
    const int ci = (lin % ncg) * QL + lane % QL;
    const bool cvalid = ci < nc;
    const int sc = c0 + min(ci, nc - 1);

    constexpr int L = LA + LB + 1;
    const double Ax = ao.x[sa], Ay = ao.y[sa], Az = ao.z[sa];
    const double c = aux.exp[sc];
    const double Cx = aux.x[sc], Cy = aux.y[sc], Cz = aux.z[sc];
    const int P0 = aux.off[sc];
    const int kk = P0 - job.kbeg;  // position in the K block (the launcher checks the range)

    double acc[NO][6];
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int k = 0; k < 6; ++k) acc[o][k] = 0.0;
    const double *gk = job.gcomp + kk;
    const size_t gstride = (size_t)job.nfq * job.nK;  // one output's copy
    // loads on every lane and output slot (past nout: the last output's
    // data), never under a branch (see k_int3c_deriv)
    const int olast = max(job.nout - 1, 0);

    const int e0 = job.lst_ptr[(kMaxAOL + 1) * sa + LB];
    const int cnt = cvalid ? job.lst_ptr[(kMaxAOL + 1) * sa + LB + 1] - e0 : 0;
    for (int ib = slot; ib < cnt; ib += NQ) {
        const int sb = job.lst_idx[e0 + ib];
        const int gq = job.lst_gq[e0 + ib];
        const long gbase = gq >> 1;
        const bool flip = gq & 1;
        const double a = ao.exp[sa], b = ao.exp[sb];
        const double p = a + b, ip = 1.0 / p;
        const double Bx = ao.x[sb], By = ao.y[sb], Bz = ao.z[sb];
        const double P[3] = {(a * Ax + b * Bx) * ip, (a * Ay + b * By) * ip, (a * Az + b * Bz) * ip};
        const double ab2 = (Ax - Bx) * (Ax - Bx) + (Ay - By) * (Ay - By) + (Az - Bz) * (Az - Bz);
        const double kab = exp(-a * b * ip * ab2);
        const double alpha = p * c / (p + c);
        double r[rsize(L)];
        hermite_r<L>(alpha, P[0] - Cx, P[1] - Cy, P[2] - Cz, boys, r);
        const double inv2p = 0.5 * ip;
        Herm<LA + 1, LB> Ex, Ey, Ez;
        herm_build<LA + 1, LB>(P[0] - Ax, P[0] - Bx, inv2p, Ex);
        herm_build<LA + 1, LB>(P[1] - Ay, P[1] - By, inv2p, Ey);
        herm_build<LA + 1, LB>(P[2] - Az, P[2] - Bz, inv2p, Ez);
        const double pref = kTwoPi52 / (p * c * sqrt(p + c)) * kab * ao.nrm[sa] * ao.nrm[sb] * aux.nrm[sc];
        const double twoa = 2.0 * a;

        sfor<ncart(LA)>([&](auto ka) {
            constexpr int ix = cpow(LA, ka, 0), iy = cpow(LA, ka, 1), iz = cpow(LA, ka, 2);
            sfor<ncart(LB)>([&](auto kb) {
                constexpr int jx = cpow(LB, kb, 0), jy = cpow(LB, kb, 1), jz = cpow(LB, kb, 2);
                const double *ex = Ex.e[ix][jx];
                const double *ey = Ey.e[iy][jy];
                const double *ez = Ez.e[iz][jz];
                double dx[ix + jx + 2], dy[iy + jy + 2], dz[iz + jz + 2];
                sfor<ix + jx + 2>([&](auto t) {
                    double v = twoa * Ex.e[ix + 1][jx][t];
                    if constexpr (ix > 0 && t <= ix - 1 + jx) v -= ix * Ex.e[ix - 1][jx][t];
                    dx[t] = v;
                });
                sfor<iy + jy + 2>([&](auto t) {
                    double v = twoa * Ey.e[iy + 1][jy][t];
                    if constexpr (iy > 0 && t <= iy - 1 + jy) v -= iy * Ey.e[iy - 1][jy][t];
                    dy[t] = v;
                });
                sfor<iz + jz + 2>([&](auto t) {
                    double v = twoa * Ez.e[iz + 1][jz][t];
                    if constexpr (iz > 0 && t <= iz - 1 + jz) v -= iz * Ez.e[iz - 1][jz][t];
                    dz[t] = v;
                });
                constexpr int NX = ix + jx + 1, NY = iy + jy + 1, NZ = iz + jz + 1;
                const long q = gbase + (flip ? (long)kb * ncart(LA) + ka : (long)ka * ncart(LB) + kb);
                const double f = pref * cnorm(LA, ka) * cnorm(LB, kb);
                double dA[3], dC[3];
                dA[0] = f * hsum<NX + 1, NY, NZ, 0, 0, 0>(dx, ey, ez, r);
                dA[1] = f * hsum<NX, NY + 1, NZ, 0, 0, 0>(ex, dy, ez, r);
                dA[2] = f * hsum<NX, NY, NZ + 1, 0, 0, 0>(ex, ey, dz, r);
                dC[0] = -f * hsum<NX, NY, NZ, 1, 0, 0>(ex, ey, ez, r);
                dC[1] = -f * hsum<NX, NY, NZ, 0, 1, 0>(ex, ey, ez, r);
                dC[2] = -f * hsum<NX, NY, NZ, 0, 0, 1>(ex, ey, ez, r);
#pragma unroll
                for (int o = 0; o < NO; ++o) {
                    // the whole weight, Coulomb part included (k_pack_gamma)
                    const double w = gk[(size_t)min(o, olast) * gstride + (size_t)q * job.nK];
                    const double w2 = 2.0 * w;
                    acc[o][0] += w2 * dA[0];
                    acc[o][1] += w2 * dA[1];
                    acc[o][2] += w2 * dA[2];
                    acc[o][3] += w * dC[0];
                    acc[o][4] += w * dC[1];
                    acc[o][5] += w * dC[2];
                }
            });
        });
    }
    // the four quarters of a K function, in a fixed order
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            double v = acc[o][k];
            v += __shfl_xor(v, 32, 64);
            v += __shfl_xor(v, 16, 64);
            acc[o][k] = v;
        }
    if (slot == 0 && cvalid) {
        double *dst = job.partial + (((size_t)sa * nshAux + sc) * (kMaxAOL + 1) + LB) * NO * 6;
#pragma unroll
        for (int o = 0; o < NO; ++o)
            if (o < job.nout) {
#pragma unroll
                for (int k = 0; k < 6; ++k) dst[o * 6 + k] = acc[o][k];
            }
    }
}

// ------------------------------------------------------------------------
// (P|Q) and its derivative for single-Gaussian auxiliary shells (l <= 1):
//   (P|Q) = 2 pi^{5/2}/(a b sqrt(a+b)) sum E^P_T (-1)^{|T'|} E^Q_{T'} R_{T+T'}(ab/(a+b), P-Q),
// E^s = 1, E^{p_k} = 1/(2e) at T = 1_k; d/dP_d shifts R by 1_d.
template <int LP, int LQ, bool DERIV>
__device__ __forceinline__ void aux_pair(const ShellTab &S, int sp, int sq, const double *boys,
                                         double (&val)[ncart(LP)][ncart(LQ)][DERIV ? 3 : 1])
{
    constexpr int L = LP + LQ + (DERIV ? 1 : 0);
    const double a = S.exp[sp], b = S.exp[sq];
    const double X = S.x[sp] - S.x[sq], Y = S.y[sp] - S.y[sq], Z = S.z[sp] - S.z[sq];
    double r[rsize(L)];
    hermite_r<L>(a * b / (a + b), X, Y, Z, boys, r);
    const double pref = kTwoPi52 / (a * b * sqrt(a + b)) * S.nrm[sp] * S.nrm[sq] *
                        (LP == 1 ? 0.5 / a : 1.0) * (LQ == 1 ? -0.5 / b : 1.0);
    sfor<ncart(LP)>([&](auto kp) {
        sfor<ncart(LQ)>([&](auto kq) {
            constexpr int tx = cpow(LP, kp, 0) + cpow(LQ, kq, 0);
            constexpr int ty = cpow(LP, kp, 1) + cpow(LQ, kq, 1);
            constexpr int tz = cpow(LP, kp, 2) + cpow(LQ, kq, 2);
            if constexpr (DERIV) {
                val[kp][kq][0] = pref * r[ridx(tx + 1, ty, tz)];
                val[kp][kq][1] = pref * r[ridx(tx, ty + 1, tz)];
                val[kp][kq][2] = pref * r[ridx(tx, ty, tz + 1)];
            } else {
                val[kp][kq][0] = pref * r[ridx(tx, ty, tz)];
            }
        });
    });
}

template <int LP, int LQ>
__global__ __launch_bounds__(128) void k_int2c(ShellTab S, int n, int p0, int np, int q0, int nq,
                                               const double *__restrict__ boys, double *__restrict__ M)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= np * nq) return;
    const int sq = q0 + tid % nq, sp = p0 + tid / nq;
    double v[ncart(LP)][ncart(LQ)][1];
    aux_pair<LP, LQ, false>(S, sp, sq, boys, v);
#pragma unroll
    for (int i = 0; i < ncart(LP); ++i)
#pragma unroll
        for (int j = 0; j < ncart(LQ); ++j) M[(size_t)(S.off[sp] + i) * n + S.off[sq] + j] = v[i][j][0];
}

// partial2[sp][LQ][o][3] = sum_{Q shells of class LQ} (W_PQ + W_QP) d(P|Q)/dP
template <int LP, int LQ>
__global__ __launch_bounds__(64) void k_int2c_deriv(ShellTab S, int n, int p0, int np, int q0, int nq,
                                                    const double *__restrict__ boys, int nout,
                                                    const double *__restrict__ W, double *__restrict__ part)
{
    const int sp = p0 + blockIdx.x;
    if (blockIdx.x >= np) return;
    const int lane = threadIdx.x;
    const int o = blockIdx.y;
    double acc[3] = {0.0, 0.0, 0.0};
    const double *Wo = W + (size_t)o * n * n;
    for (int iq = lane; iq < nq; iq += 64) {
        const int sq = q0 + iq;
        double v[ncart(LP)][ncart(LQ)][3];
        aux_pair<LP, LQ, true>(S, sp, sq, boys, v);
#pragma unroll
        for (int i = 0; i < ncart(LP); ++i)
#pragma unroll
            for (int j = 0; j < ncart(LQ); ++j) {
                const int P = S.off[sp] + i, Q = S.off[sq] + j;
                const double w = Wo[(size_t)P * n + Q] + Wo[(size_t)Q * n + P];
                acc[0] += w * v[i][j][0];
                acc[1] += w * v[i][j][1];
                acc[2] += w * v[i][j][2];
            }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double v = acc[k];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        acc[k] = v;
    }
    if (lane == 0) {
        double *dst = part + (((size_t)sp * (kMaxAuxL + 1) + LQ) * nout + o) * 3;
        dst[0] = acc[0];
        dst[1] = acc[1];
        dst[2] = acc[2];
    }
}

}  // namespace

// ------------------------------------------------------------------ hosts --
hipError_t launch_int2c(const AuxGeom &aux, const double *boys, double *M, hipStream_t st)
{
    // auxiliary shells: s shells first, then p shells (contiguous classes)
    int ns = 0;
    // count s shells: offsets equal shell index for the leading s block
    // (the host passes classes through AuxGeom.nshell and nfunc)
    ns = 3 * aux.nshell - aux.nfunc;  // nfunc = ns + 3 (nshell - ns)
    ns /= 2;
    const int np = aux.nshell - ns;
    const int n = aux.nfunc;
    auto go = [&](auto kern, int p0, int npp, int q0, int nqq) {
        if (npp == 0 || nqq == 0) return;
        const int tot = npp * nqq;
        hipLaunchKernelGGL(kern, dim3((tot + 127) / 128), dim3(128), 0, st, aux.sh, n, p0, npp, q0, nqq, boys, M);
    };
    go(k_int2c<0, 0>, 0, ns, 0, ns);
    go(k_int2c<0, 1>, 0, ns, ns, np);
    go(k_int2c<1, 0>, ns, np, 0, ns);
    go(k_int2c<1, 1>, ns, np, ns, np);
    return hipGetLastError();
}

hipError_t launch_int2c_deriv(const AuxGeom &aux, const double *boys, int nout, const double *W,
                              double *part, hipStream_t st)
{
    const int ns = (3 * aux.nshell - aux.nfunc) / 2;
    const int np = aux.nshell - ns;
    const int n = aux.nfunc;
    auto go = [&](auto kern, int p0, int npp, int q0, int nqq) {
        if (npp == 0 || nqq == 0) return;
        hipLaunchKernelGGL(kern, dim3(npp, nout), dim3(64), 0, st, aux.sh, n, p0, npp, q0, nqq, boys, nout, W, part);
    };
    go(k_int2c_deriv<0, 0>, 0, ns, 0, ns);
    go(k_int2c_deriv<0, 1>, 0, ns, ns, np);
    go(k_int2c_deriv<1, 0>, ns, np, 0, ns);
    go(k_int2c_deriv<1, 1>, ns, np, ns, np);
    return hipGetLastError();
}

namespace {
// aux shells of class LC inside [cs0, cs1)
template <int LC>
bool class_range(const int *auxl_beg, int cs0, int cs1, int *c0, int *nc)
{
    const int lo = std::max(auxl_beg[LC], cs0), hi = std::min(auxl_beg[LC + 1], cs1);
    *c0 = lo;
    *nc = hi - lo;
    return hi > lo;
}

template <int LA, int LB, int LC>
void int3c_one(const AOGeom &ao, const AuxGeom &aux, const int *auxl_beg, int cs0, int cs1, int pofs,
               const double *boys, double *X, hipStream_t st)
{
    const int a0 = ao.lbeg[LA], na = ao.lbeg[LA + 1] - a0;
    const int b0 = ao.lbeg[LB], nb = ao.lbeg[LB + 1] - b0;
    int c0, nc;
    if (!class_range<LC>(auxl_beg, cs0, cs1, &c0, &nc)) return;
    const long tot = (long)na * nb * nc;
    if (tot == 0) return;
    hipLaunchKernelGGL((k_int3c<LA, LB, LC>), dim3((unsigned)((tot + 127) / 128)), dim3(128), 0, st, ao.sh,
                       ao.nao, a0, na, b0, nb, aux.sh, c0, nc, pofs, boys, X);
}

template <int LA, int LB, int LC>
void deriv_one(const AOGeom &ao, const AuxGeom &aux, const int *auxl_beg, int cs0, int cs1, const double *boys,
               const DerivJob &job, hipStream_t st)
{
    const int a0 = ao.lbeg[LA], na = ao.lbeg[LA + 1] - a0;
    const int b0 = ao.lbeg[LB], nb = ao.lbeg[LB + 1] - b0;
    int c0, nc;
    if (!class_range<LC>(auxl_beg, cs0, cs1, &c0, &nc)) return;
    if (na == 0 || nb == 0) return;
    if constexpr (LC == 0) {
        if (job.gcomp) {
            // K block on its copy (launch_int3c_deriv checked the range)
            hipLaunchKernelGGL((k_int3c_deriv_k<LA, LB, kMaxOutChunk>), dim3(na * ((nc + 15) / 16)), dim3(64), 0, st,
                               ao.sh, ao.nao, a0, na, aux.sh, c0, nc, aux.nshell, boys, job);
            return;
        }
    }
    // d-shell partner lists are short: four C shells per wave there
    constexpr int G = LB == 2 ? 4 : (LB == 1 ? 2 : 1);
    hipLaunchKernelGGL((k_int3c_deriv<LA, LB, LC, kMaxOutChunk, G>), dim3(na * ((nc + G - 1) / G)), dim3(64), 0, st,
                       ao.sh, ao.nao, a0, na, b0, nb, aux.sh, c0, nc, aux.nshell, boys, job);
}

// first function of aux shell cs (shells sorted by l, ncart(l) functions each)
int aux_func_off(const int *auxl_beg, int cs)
{
    int f = 0;
    for (int l = 0; l <= kMaxAuxL; ++l) {
        const int lo = auxl_beg[l], hi = auxl_beg[l + 1];
        f += ncart(l) * (std::min(std::max(cs, lo), hi) - lo);
    }
    return f;
}
}  // namespace

hipError_t launch_int3c(const AOGeom &ao, const AuxGeom &aux, int auxl_beg[kMaxAuxL + 2], const double *boys,
                        double *X, hipStream_t st, int cs0, int cs1)
{
    if (cs1 < 0) cs1 = aux.nshell;
    if (cs0 < 0 || cs0 > cs1 || cs1 > aux.nshell) return hipErrorInvalidValue;
    if (cs0 == cs1) return hipSuccess;
    // the block's first function is row 0 of X
    const int pofs = aux_func_off(auxl_beg, cs0);
    int3c_one<0, 0, 0>(ao, aux, auxl_beg, cs0, cs1, pofs, boys, X, st);
    int3c_one<0, 1, 0>(ao, aux, auxl_beg, cs0, cs1, pofs, boys, X, st);
    int3c_one<0, 2, 0>(ao, aux, auxl_beg, cs0, cs1, pofs, boys, X, st);
    int3c_one<1, 0, 0>(ao, aux, auxl_beg, cs0, cs1, pofs, boys, X, st);
    int3c_one<1, 1, 0>(ao, aux, auxl_beg, cs0, cs1, pofs, boys, X, st);
    int3c_one<1, 2, 0>(ao, aux, auxl_beg, cs0, cs1, pofs, boys, X, st);
    int3c_one<2, 0, 0>(ao, aux, auxl_beg, cs0, cs1, pofs, boys, X, st);
    int3c_one<2, 1, 0>(ao, aux, auxl_beg, cs0, cs1, pofs, boys, X, st);
    int3c_one<2, 2, 0>(ao, aux, auxl_beg, cs0, cs1, pofs, boys, X, st);
    int3c_one<0, 0, 1>(ao, aux, auxl_beg, cs0, cs1, pofs, boys, X, st);
    int3c_one<0, 1, 1>(ao, aux, auxl_beg, cs0, cs1, pofs, boys, X, st);
    int3c_one<0, 2, 1>(ao, aux, auxl_beg, cs0, cs1, pofs, boys, X, st);
    int3c_one<1, 0, 1>(ao, aux, auxl_beg, cs0, cs1, pofs, boys, X, st);
    int3c_one<1, 1, 1>(ao, aux, auxl_beg, cs0, cs1, pofs, boys, X, st);
    int3c_one<1, 2, 1>(ao, aux, auxl_beg, cs0, cs1, pofs, boys, X, st);
    int3c_one<2, 0, 1>(ao, aux, auxl_beg, cs0, cs1, pofs, boys, X, st);
    int3c_one<2, 1, 1>(ao, aux, auxl_beg, cs0, cs1, pofs, boys, X, st);
    int3c_one<2, 2, 1>(ao, aux, auxl_beg, cs0, cs1, pofs, boys, X, st);
    return hipGetLastError();
}

hipError_t launch_int3c_deriv(const AOGeom &ao, const AuxGeom &aux, int auxl_beg[kMaxAuxL + 2],
                              const double *boys, const DerivJob &job, hipStream_t st, int cs0, int cs1)
{
    if (cs1 < 0) cs1 = aux.nshell;
    if (cs0 < 0 || cs0 > cs1 || cs1 > aux.nshell) return hipErrorInvalidValue;
    if (job.gcomp) {
        // the copy serves the s shells of the range (a range of p shells
        // only carries the Coulomb part): all of them must be K functions of
        // the block (s shells hold one function each)
        int c0, nc;
        if (class_range<0>(auxl_beg, cs0, cs1, &c0, &nc) &&
            (!job.gammaK || !job.lst_ptr || !job.lst_idx || !job.lst_gq || job.nfq <= 0 || c0 < job.kbeg ||
             c0 + nc > job.kbeg + job.nK || auxl_beg[0] != 0))
            return hipErrorInvalidValue;
    }
    deriv_one<0, 0, 0>(ao, aux, auxl_beg, cs0, cs1, boys, job, st);
    deriv_one<0, 1, 0>(ao, aux, auxl_beg, cs0, cs1, boys, job, st);
    deriv_one<0, 2, 0>(ao, aux, auxl_beg, cs0, cs1, boys, job, st);
    deriv_one<1, 0, 0>(ao, aux, auxl_beg, cs0, cs1, boys, job, st);
    deriv_one<1, 1, 0>(ao, aux, auxl_beg, cs0, cs1, boys, job, st);
    deriv_one<1, 2, 0>(ao, aux, auxl_beg, cs0, cs1, boys, job, st);
    deriv_one<2, 0, 0>(ao, aux, auxl_beg, cs0, cs1, boys, job, st);
    deriv_one<2, 1, 0>(ao, aux, auxl_beg, cs0, cs1, boys, job, st);
    deriv_one<2, 2, 0>(ao, aux, auxl_beg, cs0, cs1, boys, job, st);
    deriv_one<0, 0, 1>(ao, aux, auxl_beg, cs0, cs1, boys, job, st);
    deriv_one<0, 1, 1>(ao, aux, auxl_beg, cs0, cs1, boys, job, st);
    deriv_one<0, 2, 1>(ao, aux, auxl_beg, cs0, cs1, boys, job, st);
    deriv_one<1, 0, 1>(ao, aux, auxl_beg, cs0, cs1, boys, job, st);
    deriv_one<1, 1, 1>(ao, aux, auxl_beg, cs0, cs1, boys, job, st);
    deriv_one<1, 2, 1>(ao, aux, auxl_beg, cs0, cs1, boys, job, st);
    deriv_one<2, 0, 1>(ao, aux, auxl_beg, cs0, cs1, boys, job, st);
    deriv_one<2, 1, 1>(ao, aux, auxl_beg, cs0, cs1, boys, job, st);
    deriv_one<2, 2, 1>(ao, aux, auxl_beg, cs0, cs1, boys, job, st);
    return hipGetLastError();
}

hipError_t launch_pack_gamma(const AOGeom &ao, const DerivJob &job, const PackLists &pl, hipStream_t st)
{
    const int nout = job.nout, nK = job.nK;
    if (nout <= 0 || nK <= 0 || ao.nshell <= 0) return hipSuccess;
    if (nout > kMaxOutChunk || job.nfq <= 0 || !job.gammaK || !job.gcomp || !job.dens || !job.cvec)
        return hipErrorInvalidValue;
    const long blocks = (long)nout * ao.nshell * ((nK + 63) / 64);
    hipLaunchKernelGGL(k_pack_gamma, dim3((unsigned)blocks), dim3(256), 0, st, ao.sh.off, ao.lbeg[1], ao.lbeg[2],
                       ao.nshell, ao.nao, nK, job.gammaK, pl.pk_ptr, pl.pk_base, pl.pc_ptr, pl.pc_cn, pl.pc_qb,
                       job.nfq, const_cast<double *>(job.gcomp), job);
    return hipGetLastError();
}

}  // namespace ris

// ------------------------------------------------------------------------
// Test probe of the device Boys function: F[i][m] = F_m(T[i]) for m <= 7.
namespace {
__global__ void k_boys_probe(int n, const double *__restrict__ T, const double *__restrict__ tab,
                             double *__restrict__ F)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double f[ris::kBoysMaxM + 1];
    ris::boys_eval<ris::kBoysMaxM>(T[i], tab, f);
#pragma unroll
    for (int m = 0; m <= ris::kBoysMaxM; ++m) F[(size_t)i * (ris::kBoysMaxM + 1) + m] = f[m];
}
}  // namespace

extern "C" int ris_test_boys(int n, const double *T, double *F)
{
    if (n < 0 || (n > 0 && (!T || !F))) return 1;
    if (n == 0) return 0;
    std::vector<double> tab((size_t)ris::kBoysNGrid * ris::kBoysCols);
    ris::boys_table_host(tab.data());
    double *dtab = nullptr;
    if (hipMalloc(&dtab, tab.size() * sizeof(double)) != hipSuccess) return 7;
    int rc = 0;
    if (hipMemcpy(dtab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) rc = 7;
    if (!rc) {
        hipLaunchKernelGGL(k_boys_probe, dim3((n + 255) / 256), dim3(256), 0, 0, n, T, dtab, F);
        if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) rc = 7;
    }
    (void)hipFree(dtab);
    return rc;
}
