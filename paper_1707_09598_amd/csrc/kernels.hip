// kernels.hip -- gfx950 kernels of the sparse-grid isogeometric solver and
// the C-ABI entry points that launch them.
//
//   k_tables      Cox-de Boor values/derivatives at the Gauss points of every
//                 level (eq. Bsp), geometry basis tables
//   k_assemble    per Gauss point: NURBS map F (eq. F-B-splines), Jacobian,
//                 a, f, operator coefficients a w |det DF| DF^-1 DF^-T and the
//                 load density (Galerkin form of Problem 1)
//   k_rhs         load vector b_j = sum_q f w |det DF| phi_j
//   k_solve       persistent refinement + fast-diagonalisation PCG over all
//                 component grids (grid-wide barrier between phases)
//   k_combine     u_sg(xi) = sum_i c_i u_i(xi), eq. (TD-combi-tec), FP64
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "device.hpp"
#include "plan.hpp"

using namespace igasg;

#define HIP_OK(call)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) {                                                             \
            set_error("%s failed: %s", #call, hipGetErrorString(e_));                      \
            return IGA_ERR_DEVICE;                                                          \
        }                                                                                   \
    } while (0)

namespace igasg {

// ===========================================================================
// fields
// ===========================================================================
struct FieldDev {
    int kind;
    double prm[4];
    const double* data;
    int n[3];
};

__device__ __forceinline__ void sincos_coef(const double* prm, const double* x, double* a, double* da) {
    const double tp = 6.283185307179586476925;
    double sx, cx, sy, cy;
    sincos(tp * (x[0] + prm[1]), &sx, &cx);
    sincos(tp * x[1], &sy, &cy);
    *a = 1.0 + prm[0] * sx * cy;
    da[0] = tp * prm[0] * cx * cy;
    da[1] = -tp * prm[0] * sx * sy;
}

__device__ double field_eval(const FieldDev& F, int dim, const double* x) {
    const double pi = 3.141592653589793238463;
    switch (F.kind) {
        case IGA_FIELD_CONST:
            return F.prm[0];
        case IGA_FIELD_SINPROD: {
            double v = F.prm[0];
            for (int k = 0; k < dim; ++k) v *= sin(pi * x[k]);
            return v;
        }
        case IGA_FIELD_SINCOS: {
            double a, da[2];
            sincos_coef(F.prm, x, &a, da);
            return a;
        }
        case IGA_FIELD_ANNULUS_RHS: {
            // u = P(s) x y^2, s = x^2 + y^2, P(s) = -(s-1)(s-4)
            double X = x[0], Y = x[1], s = X * X + Y * Y;
            double Pv = -(s - 1.0) * (s - 4.0), dP = 5.0 - 2.0 * s, ddP = -2.0;
            double ux = Y * Y * (2.0 * X * X * dP + Pv);
            double uy = 2.0 * X * Y * (Y * Y * dP + Pv);
            double lap = 16.0 * X * Y * Y * dP + 4.0 * X * Y * Y * s * ddP + 2.0 * X * Pv;
            double a, da[2];
            sincos_coef(F.prm, x, &a, da);
            return -(a * lap + da[0] * ux + da[1] * uy);
        }
        case IGA_FIELD_POLY_RHS: {
            double q[3], dq[3];
            for (int k = 0; k < dim; ++k) {
                q[k] = x[k] * (1.0 - x[k]);
                dq[k] = 1.0 - 2.0 * x[k];
            }
            double g[3], lap = 0.0;
            for (int k = 0; k < dim; ++k) {
                double rest = 1.0;
                for (int j = 0; j < dim; ++j)
                    if (j != k) rest *= q[j];
                g[k] = dq[k] * rest;
                lap -= 2.0 * rest;
            }
            double a, da[2];
            sincos_coef(F.prm, x, &a, da);
            return -(a * lap + da[0] * g[0] + da[1] * g[1]);
        }
        case IGA_FIELD_GRID3D: {
            int i[3];
            double t[3];
            for (int k = 0; k < 3; ++k) {
                int n = F.n[k];
                double s = x[k] * (n - 1);
                int ii = static_cast<int>(floor(s));
                ii = ii < 0 ? 0 : (ii > n - 2 ? n - 2 : ii);
                i[k] = ii;
                t[k] = s - ii;
            }
            double v = 0.0;
            for (int c = 0; c < 2; ++c)
                for (int b = 0; b < 2; ++b)
                    for (int a = 0; a < 2; ++a) {
                        double wt = (a ? t[0] : 1 - t[0]) * (b ? t[1] : 1 - t[1]) * (c ? t[2] : 1 - t[2]);
                        int64_t idx = (i[0] + a) + static_cast<int64_t>(F.n[0]) * ((i[1] + b) + static_cast<int64_t>(F.n[1]) * (i[2] + c));
                        v += wt * F.data[idx];
                    }
            return v;
        }
        case IGA_FIELD_CORNER: {
            double r = sqrt(x[0] * x[0] + x[1] * x[1]);
            if (r == 0.0) return 0.0;
            double th = atan2(x[1], x[0]);
            if (th < 0) th += 2.0 * pi;
            return pow(r, 2.0 / 3.0) * sin(2.0 * th / 3.0);
        }
        case IGA_FIELD_AFFINE: {
            double v = F.prm[0];
            for (int k = 0; k < dim; ++k) v += F.prm[1 + k] * x[k];
            return v;
        }
        default:
            return __builtin_nan("");
    }
}

// ===========================================================================
// K1: basis tables at the Gauss points of every (patch, direction, level)
// ===========================================================================
__global__ void __launch_bounds__(kBlock) k_tables(Params P) {
    const int ti = blockIdx.y;
    const Tab1D T = P.tabs[ti];
    const int q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= T.Q) return;
    double* dp = const_cast<double*>(P.dpool);
    int* ip = const_cast<int*>(P.ipool);
    const int nq = P.nq, p = P.p;
    const int e = q / nq, j = q - e * nq;
    const double* brk = dp + T.oBrk;
    const double a = brk[e], b = brk[e + 1];
    const double xq = a + 0.5 * (b - a) * (P.gx[j] + 1.0);
    const double wq = 0.5 * (b - a) * P.gw[j];
    double N[kMaxPg + 1], dN[kMaxPg + 1];
    d_basis_funs(p, dp + T.oKn, p + e * T.m, xq, N, dN);
    for (int r = 0; r <= p; ++r) {
        dp[T.oB + static_cast<int64_t>(q) * (p + 1) + r] = N[r];
        dp[T.oD + static_cast<int64_t>(q) * (p + 1) + r] = dN[r];
    }
    const double* gk = dp + T.oGkn;
    int sg = d_find_interval(T.pg, T.ngk, gk, xq);
    d_basis_funs(T.pg, gk, sg, xq, N, dN);
    for (int r = 0; r <= T.pg; ++r) {
        dp[T.oBg + static_cast<int64_t>(q) * (T.pg + 1) + r] = N[r];
        dp[T.oDg + static_cast<int64_t>(q) * (T.pg + 1) + r] = dN[r];
    }
    ip[T.oGs + q] = sg - T.pg;
    dp[T.oXq + q] = xq;
    dp[T.oWq + q] = wq;
}

// ===========================================================================
// K2: assembly at the Gauss points
// ===========================================================================
__device__ __forceinline__ int grid_of_qp(const Params& P, int g0, int g1, int64_t gq) {
    int lo = g0, hi = g1 - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (P.grids[mid].qp_off <= gq) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Geometry at a tensor Gauss point from the per-direction geometry tables:
// homogeneous sums X_c = sum w P_c B, W = sum w B and their derivatives.
__device__ __forceinline__ void geom_at(const Params& P, const Grid& g, const int* qk, double* x,
                                        double DF[3][3], double* W, double* dW) {
    const int d = P.dim, pt = g.patch;
    const double* Bg[3];
    const double* Dg[3];
    int f[3] = {0, 0, 0}, pg[3] = {0, 0, 0};
    for (int k = 0; k < d; ++k) {
        const Tab1D& T = P.tabs[g.tab[k]];
        pg[k] = T.pg;
        Bg[k] = P.dpool + T.oBg + static_cast<int64_t>(qk[k]) * (T.pg + 1);
        Dg[k] = P.dpool + T.oDg + static_cast<int64_t>(qk[k]) * (T.pg + 1);
        f[k] = P.ipool[T.oGs + qk[k]];
    }
    double Xh[4] = {0, 0, 0, 0}, dXh[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    const double* C = P.ctrl + P.ctrl_off[pt];
    const int n0 = P.gn[pt][0], n1 = P.gn[pt][1];
    const int lim2 = d > 2 ? pg[2] : 0;
    for (int c = 0; c <= lim2; ++c)
        for (int b = 0; b <= pg[1]; ++b)
            for (int a = 0; a <= pg[0]; ++a) {
                double v[3] = {Bg[0][a], Bg[1][b], d > 2 ? Bg[2][c] : 1.0};
                double dv[3] = {Dg[0][a], Dg[1][b], d > 2 ? Dg[2][c] : 0.0};
                int64_t idx = (f[0] + a) + static_cast<int64_t>(n0) * ((f[1] + b) + static_cast<int64_t>(n1) * (d > 2 ? f[2] + c : 0));
                const double* cp = C + idx * 4;
                double B = v[0] * v[1] * v[2];
                double dB[3] = {dv[0] * v[1] * v[2], v[0] * dv[1] * v[2], v[0] * v[1] * dv[2]};
                for (int t = 0; t < 4; ++t) {
                    Xh[t] += cp[t] * B;
                    for (int k = 0; k < d; ++k) dXh[k][t] += cp[t] * dB[k];
                }
            }
    *W = Xh[3];
    for (int c = 0; c < d; ++c) {
        x[c] = Xh[c] / Xh[3];
        for (int k = 0; k < d; ++k) DF[c][k] = (dXh[k][c] - x[c] * dXh[k][3]) / Xh[3];
    }
    for (int k = 0; k < d; ++k) dW[k] = dXh[k][3];
}

__global__ void __launch_bounds__(kBlock) k_assemble(Params P, FieldDev fa, FieldDev ff, int g0, int g1,
                                                    int* err) {
    const int64_t q0 = P.grids[g0].qp_off;
    const int64_t q1 = P.grids[g1 - 1].qp_off + P.grids[g1 - 1].nqp;
    const int d = P.dim;
    for (int64_t gq = q0 + blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; gq < q1;
         gq += static_cast<int64_t>(gridDim.x) * kBlock) {
        const int gi = grid_of_qp(P, g0, g1, gq);
        const Grid& g = P.grids[gi];
        const int64_t l = gq - g.qp_off;
        int qk[3];
        qk[0] = static_cast<int>(l % g.Q[0]);
        qk[1] = static_cast<int>((l / g.Q[0]) % g.Q[1]);
        qk[2] = static_cast<int>(l / (static_cast<int64_t>(g.Q[0]) * g.Q[1]));
        double x[3] = {0, 0, 0}, DF[3][3], W, dW[3] = {0, 0, 0};
        geom_at(P, g, qk, x, DF, &W, dW);
        double wq = 1.0;
        for (int k = 0; k < d; ++k) wq *= P.dpool[P.tabs[g.tab[k]].oWq + qk[k]];
        double det, inv[3][3];
        if (d == 2) {
            det = DF[0][0] * DF[1][1] - DF[0][1] * DF[1][0];
            inv[0][0] = DF[1][1] / det;
            inv[0][1] = -DF[0][1] / det;
            inv[1][0] = -DF[1][0] / det;
            inv[1][1] = DF[0][0] / det;
        } else {
            det = DF[0][0] * (DF[1][1] * DF[2][2] - DF[1][2] * DF[2][1]) -
                  DF[0][1] * (DF[1][0] * DF[2][2] - DF[1][2] * DF[2][0]) +
                  DF[0][2] * (DF[1][0] * DF[2][1] - DF[1][1] * DF[2][0]);
            inv[0][0] = (DF[1][1] * DF[2][2] - DF[1][2] * DF[2][1]) / det;
            inv[0][1] = (DF[0][2] * DF[2][1] - DF[0][1] * DF[2][2]) / det;
            inv[0][2] = (DF[0][1] * DF[1][2] - DF[0][2] * DF[1][1]) / det;
            inv[1][0] = (DF[1][2] * DF[2][0] - DF[1][0] * DF[2][2]) / det;
            inv[1][1] = (DF[0][0] * DF[2][2] - DF[0][2] * DF[2][0]) / det;
            inv[1][2] = (DF[0][2] * DF[1][0] - DF[0][0] * DF[1][2]) / det;
            inv[2][0] = (DF[1][0] * DF[2][1] - DF[1][1] * DF[2][0]) / det;
            inv[2][1] = (DF[0][1] * DF[2][0] - DF[0][0] * DF[2][1]) / det;
            inv[2][2] = (DF[0][0] * DF[1][1] - DF[0][1] * DF[1][0]) / det;
        }
        if (!(det > 0.0)) atomicOr(err, 1);
        const double av = field_eval(fa, d, x);
        const double fv = field_eval(ff, d, x);
        const double s = av * wq * fabs(det);
        // parametric coefficients Gp = a w |det| DF^-1 DF^-T (symmetric)
        double Gp[3][3];
        for (int i = 0; i < d; ++i)
            for (int j = i; j < d; ++j) {
                double t = 0.0;
                for (int k = 0; k < d; ++k) t += inv[i][k] * inv[j][k];
                Gp[i][j] = Gp[j][i] = s * t;
            }
        const int64_t nqp = g.nqp;
        double* G = P.G64 + g.qp_off * P.ncompG + l;
        float* G32 = P.G32 + g.qp_off * P.ncompG + l;
        int c = 0;
        if (P.rational[g.patch]) {
            // phi = B/W: grad phi = grad B / W - B grad W / W^2, so the form acts
            // on (v, grad v) of v = sum c B through T = [-grad W / W^2, I / W]
            double gw[3], Ggw[3];
            for (int k = 0; k < d; ++k) gw[k] = dW[k] / (W * W);
            for (int i = 0; i < d; ++i) {
                Ggw[i] = 0.0;
                for (int k = 0; k < d; ++k) Ggw[i] += Gp[i][k] * gw[k];
            }
            double g00 = 0.0;
            for (int k = 0; k < d; ++k) g00 += gw[k] * Ggw[k];
            double H[4][4];
            H[0][0] = g00;
            for (int i = 0; i < d; ++i) {
                H[0][i + 1] = H[i + 1][0] = -Ggw[i] / W;
                for (int j = 0; j < d; ++j) H[i + 1][j + 1] = Gp[i][j] / (W * W);
            }
            for (int i = 0; i <= d; ++i)
                for (int j = i; j <= d; ++j, ++c) {
                    G[c * nqp] = H[i][j];
                    G32[c * nqp] = static_cast<float>(H[i][j]);
                }
        } else {
            for (int i = 0; i < d; ++i)
                for (int j = i; j < d; ++j, ++c) {
                    G[c * nqp] = Gp[i][j];
                    G32[c * nqp] = static_cast<float>(Gp[i][j]);
                }
        }
        P.Fq[g.qp_off + l] = fv * wq * fabs(det) / W;
    }
}

// Element range touching interior unknowns [a, b) of one direction.
__device__ __forceinline__ void d_elem_range(int a, int b, int p, int m, int E, int* elo, int* ehi) {
    int lo_basis = a + 1, hi_basis = b;
    int lo = (lo_basis - p <= 0) ? 0 : (lo_basis - p + m - 1) / m;
    int hi = hi_basis / m;
    *elo = lo < 0 ? 0 : lo;
    *ehi = hi > E - 1 ? E - 1 : hi;
}

// Load vector: b_i = sum over Gauss points of the supporting elements of
// B_i(q) Fq(q) (Fq = f w |det DF| / W), one thread per unknown.
__global__ void __launch_bounds__(kBlock) k_rhs(Params P, int g0, int g1) {
    const int64_t i0 = P.grids[g0].dof_off;
    const int64_t i1 = P.grids[g1 - 1].dof_off + P.grids[g1 - 1].ndof;
    const int p = P.p, nq = P.nq, d = P.dim;
    for (int64_t gi = i0 + blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; gi < i1;
         gi += static_cast<int64_t>(gridDim.x) * kBlock) {
        int lo = g0, hi = g1 - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (P.grids[mid].dof_off <= gi) lo = mid;
            else hi = mid - 1;
        }
        const Grid& g = P.grids[lo];
        int64_t l = gi - g.dof_off;
        int I[3];
        I[0] = static_cast<int>(l % g.ni[0]) + 1;
        I[1] = static_cast<int>((l / g.ni[0]) % g.ni[1]) + 1;
        I[2] = static_cast<int>(l / (static_cast<int64_t>(g.ni[0]) * g.ni[1])) + 1;
        int elo[3] = {0, 0, 0}, ehi[3] = {0, 0, 0};
        const double* B[3] = {nullptr, nullptr, nullptr};
        int m[3] = {1, 1, 1};
        for (int k = 0; k < d; ++k) {
            const Tab1D& T = P.tabs[g.tab[k]];
            d_elem_range(I[k] - 1, I[k], p, T.m, T.E, &elo[k], &ehi[k]);
            B[k] = P.dpool + T.oB;
            m[k] = T.m;
        }
        const double* F = P.Fq + g.qp_off;
        double s3 = 0.0;
        const int e3lo = d > 2 ? elo[2] : 0, e3hi = d > 2 ? ehi[2] : 0, nq3 = d > 2 ? nq : 1;
        for (int e3 = e3lo; e3 <= e3hi; ++e3)
            for (int j3 = 0; j3 < nq3; ++j3) {
                int q3 = e3 * nq + j3;
                double w3 = d > 2 ? B[2][static_cast<int64_t>(q3) * (p + 1) + (I[2] - e3 * m[2])] : 1.0;
                if (d <= 2) q3 = 0;
                double s2 = 0.0;
                for (int e2 = elo[1]; e2 <= ehi[1]; ++e2)
                    for (int j2 = 0; j2 < nq; ++j2) {
                        int q2 = e2 * nq + j2;
                        double w2 = B[1][static_cast<int64_t>(q2) * (p + 1) + (I[1] - e2 * m[1])];
                        double s1 = 0.0;
                        const double* Fr = F + (static_cast<int64_t>(q3) * g.Q[1] + q2) * g.Q[0];
                        for (int e1 = elo[0]; e1 <= ehi[0]; ++e1)
                            for (int j1 = 0; j1 < nq; ++j1) {
                                int q1 = e1 * nq + j1;
                                s1 += B[0][static_cast<int64_t>(q1) * (p + 1) + (I[0] - e1 * m[0])] * Fr[q1];
                            }
                        s2 += w2 * s1;
                    }
                s3 += w3 * s2;
            }
        P.b[gi] = s3;
    }
}

// ===========================================================================
// operator application (2D): one workgroup per tile of unknowns; the
// elements touching the tile are recomputed (halo), element outputs are staged
// in LDS and summed per owned unknown in a fixed order (no atomics).
// ===========================================================================
struct OpIO {
    const double* in_a;   // input (or z)
    const double* in_b;   // added as beta * in_b (or nullptr)
    double beta;
    double* out_in;       // owned part of in_a + beta in_b is written here (or nullptr)
    double* out;          // A x (or b - A x when rhs != nullptr)
    const double* rhs;
    double* part;         // per-tile partial: in.(A in) or ||b - A x||^2 (or nullptr)
    int lowp;             // 1: FP32 coefficients and arithmetic
};

template <int PP, bool RAT, typename T>
__device__ __forceinline__ void elem_apply_2d(const double* X, int nh1, int x1, int x2, const double* B1,
                                              const double* D1, const double* B2, const double* D2,
                                              const T* G, int64_t nqp, int64_t qrow0, int Q1, double* Y) {
    constexpr int NQ = PP + 1;
    T c[PP + 1][PP + 1], y[PP + 1][PP + 1];
#pragma unroll
    for (int a2 = 0; a2 <= PP; ++a2)
#pragma unroll
        for (int a1 = 0; a1 <= PP; ++a1) {
            c[a1][a2] = static_cast<T>(X[(x2 + a2) * nh1 + x1 + a1]);
            y[a1][a2] = T(0);
        }
#pragma unroll
    for (int j2 = 0; j2 < NQ; ++j2) {
        T b2[PP + 1], d2[PP + 1];
#pragma unroll
        for (int a = 0; a <= PP; ++a) {
            b2[a] = static_cast<T>(B2[j2 * (PP + 1) + a]);
            d2[a] = static_cast<T>(D2[j2 * (PP + 1) + a]);
        }
        T tb[PP + 1], td[PP + 1], sb[PP + 1], sd[PP + 1];
#pragma unroll
        for (int a1 = 0; a1 <= PP; ++a1) {
            T u = T(0), v = T(0);
#pragma unroll
            for (int a2 = 0; a2 <= PP; ++a2) {
                u += b2[a2] * c[a1][a2];
                v += d2[a2] * c[a1][a2];
            }
            tb[a1] = u;
            td[a1] = v;
            sb[a1] = T(0);
            sd[a1] = T(0);
        }
        const T* Gr = G + qrow0 + static_cast<int64_t>(j2) * Q1;
#pragma unroll
        for (int j1 = 0; j1 < NQ; ++j1) {
            T b1[PP + 1], d1[PP + 1];
#pragma unroll
            for (int a = 0; a <= PP; ++a) {
                b1[a] = static_cast<T>(B1[j1 * (PP + 1) + a]);
                d1[a] = static_cast<T>(D1[j1 * (PP + 1) + a]);
            }
            T v0 = T(0), v1 = T(0), v2 = T(0);
#pragma unroll
            for (int a1 = 0; a1 <= PP; ++a1) {
                if (RAT) v0 += b1[a1] * tb[a1];
                v1 += d1[a1] * tb[a1];
                v2 += b1[a1] * td[a1];
            }
            T F0 = T(0), F1, F2;
            if (RAT) {
                T g00 = Gr[j1], g01 = Gr[nqp + j1], g02 = Gr[2 * nqp + j1];
                T g11 = Gr[3 * nqp + j1], g12 = Gr[4 * nqp + j1], g22 = Gr[5 * nqp + j1];
                F0 = g00 * v0 + g01 * v1 + g02 * v2;
                F1 = g01 * v0 + g11 * v1 + g12 * v2;
                F2 = g02 * v0 + g12 * v1 + g22 * v2;
            } else {
                T g11 = Gr[j1], g12 = Gr[nqp + j1], g22 = Gr[2 * nqp + j1];
                F1 = g11 * v1 + g12 * v2;
                F2 = g12 * v1 + g22 * v2;
            }
#pragma unroll
            for (int a1 = 0; a1 <= PP; ++a1) {
                sb[a1] += (RAT ? b1[a1] * F0 : T(0)) + d1[a1] * F1;
                sd[a1] += b1[a1] * F2;
            }
        }
#pragma unroll
        for (int a2 = 0; a2 <= PP; ++a2)
#pragma unroll
            for (int a1 = 0; a1 <= PP; ++a1) y[a1][a2] += b2[a2] * sb[a1] + d2[a2] * sd[a1];
    }
#pragma unroll
    for (int a2 = 0; a2 <= PP; ++a2)
#pragma unroll
        for (int a1 = 0; a1 <= PP; ++a1) Y[a1 + (PP + 1) * a2] = static_cast<double>(y[a1][a2]);
}

template <int PP>
__device__ void op_tile_2d(const Params& P, const Grid& g, int tile, const OpIO& io, double* lds) {
    const int p = PP;
    const Tab1D& T1 = P.tabs[g.tab[0]];
    const Tab1D& T2 = P.tabs[g.tab[1]];
    const int m1 = T1.m, m2 = T2.m;
    const int t1 = tile % g.ntd[0], t2 = tile / g.ntd[0];
    const int a1 = t1 * g.tile[0], b1 = min(g.ni[0], a1 + g.tile[0]);
    const int a2 = t2 * g.tile[1], b2 = min(g.ni[1], a2 + g.tile[1]);
    int el1, eh1, el2, eh2;
    d_elem_range(a1, b1, p, m1, g.E[0], &el1, &eh1);
    d_elem_range(a2, b2, p, m2, g.E[1], &el2, &eh2);
    const int ne1 = eh1 - el1 + 1, ne2 = eh2 - el2 + 1;
    const int hl1 = el1 * m1 - 1, hl2 = el2 * m2 - 1;           // interior index of halo start
    const int nh1 = eh1 * m1 + p - 1 - hl1 + 1, nh2 = eh2 * m2 + p - 1 - hl2 + 1;
    double* X = lds;
    double* Y = lds + nh1 * nh2;
    double* red = Y + ne1 * ne2 * (p + 1) * (p + 1);
    const int64_t off = g.dof_off;
    const int n1 = g.ni[0], n2 = g.ni[1];
    for (int idx = threadIdx.x; idx < nh1 * nh2; idx += kBlock) {
        int i1 = hl1 + idx % nh1, i2 = hl2 + idx / nh1;
        double v = 0.0;
        if (i1 >= 0 && i1 < n1 && i2 >= 0 && i2 < n2) {
            int64_t gi = off + static_cast<int64_t>(i2) * n1 + i1;
            v = io.in_a[gi];
            if (io.in_b) v += io.beta * io.in_b[gi];
            if (io.out_in && i1 >= a1 && i1 < b1 && i2 >= a2 && i2 < b2) io.out_in[gi] = v;
        }
        X[idx] = v;
    }
    __syncthreads();
    const int nqp1 = P.nq * (p + 1);
    const int64_t nqp = g.nqp;
    for (int el = threadIdx.x; el < ne1 * ne2; el += kBlock) {
        int e1 = el1 + el % ne1, e2 = el2 + el / ne1;
        const double* B1 = P.dpool + T1.oB + static_cast<int64_t>(e1) * nqp1;
        const double* D1 = P.dpool + T1.oD + static_cast<int64_t>(e1) * nqp1;
        const double* B2 = P.dpool + T2.oB + static_cast<int64_t>(e2) * nqp1;
        const double* D2 = P.dpool + T2.oD + static_cast<int64_t>(e2) * nqp1;
        const int x1 = e1 * m1 - 1 - hl1, x2 = e2 * m2 - 1 - hl2;
        const int64_t qrow0 = static_cast<int64_t>(e2) * P.nq * g.Q[0] + static_cast<int64_t>(e1) * P.nq;
        double* Ye = Y + el * (p + 1) * (p + 1);
        const bool rat = P.rational[g.patch] != 0;
        if (io.lowp) {
            const float* G = P.G32 + g.qp_off * P.ncompG;
            if (rat) elem_apply_2d<PP, true, float>(X, nh1, x1, x2, B1, D1, B2, D2, G, nqp, qrow0, g.Q[0], Ye);
            else elem_apply_2d<PP, false, float>(X, nh1, x1, x2, B1, D1, B2, D2, G, nqp, qrow0, g.Q[0], Ye);
        } else {
            const double* G = P.G64 + g.qp_off * P.ncompG;
            if (rat) elem_apply_2d<PP, true, double>(X, nh1, x1, x2, B1, D1, B2, D2, G, nqp, qrow0, g.Q[0], Ye);
            else elem_apply_2d<PP, false, double>(X, nh1, x1, x2, B1, D1, B2, D2, G, nqp, qrow0, g.Q[0], Ye);
        }
    }
    __syncthreads();
    const int w1 = b1 - a1, nown = w1 * (b2 - a2);
    double dot = 0.0;
    for (int o = threadIdx.x; o < nown; o += kBlock) {
        const int i1 = a1 + o % w1, i2 = a2 + o / w1;
        const int I1 = i1 + 1, I2 = i2 + 1;
        int lo1, hi1, lo2, hi2;
        d_elem_range(i1, i1 + 1, p, m1, g.E[0], &lo1, &hi1);
        d_elem_range(i2, i2 + 1, p, m2, g.E[1], &lo2, &hi2);
        double s = 0.0;
        for (int e2 = lo2; e2 <= hi2; ++e2)
            for (int e1 = lo1; e1 <= hi1; ++e1) {
                int el = (e2 - el2) * ne1 + (e1 - el1);
                s += Y[el * (p + 1) * (p + 1) + (I1 - e1 * m1) + (p + 1) * (I2 - e2 * m2)];
            }
        const int64_t gi = off + static_cast<int64_t>(i2) * n1 + i1;
        if (io.rhs) {
            s = io.rhs[gi] - s;
            dot += s * s;
        } else {
            dot += X[(i2 - hl2) * nh1 + (i1 - hl1)] * s;
        }
        io.out[gi] = s;
    }
    if (io.part) {
        double t = wg_sum(dot, red);
        if (threadIdx.x == 0) *io.part = t;
    }
    __syncthreads();
}

// ===========================================================================
// fast diagonalisation: z = (U1 (x) U2) diag(1/(c1 l1 + c2 l2)) (U1 (x) U2)^T r
// as mode products (workgroup GEMMs with split K)
// ===========================================================================
// C(b, m, n) = sum_k A(b, m, k) B(b, k, n); operands in LDS or global memory.
template <typename TA, typename TB, typename TC>
__device__ void wg_gemm(int nbat, int M, int N, int K, const TA* A, int64_t sAb, int64_t sAm, int64_t sAk,
                        const TB* B, int64_t sBb, int64_t sBk, int64_t sBn, double* C, int64_t sCb,
                        int64_t sCm, int64_t sCn, double* red) {
    const int O = nbat * M * N;
    auto ld = [](auto* p, int64_t i) -> TC {
        using V = typename std::remove_cv<typename std::remove_pointer<decltype(p)>::type>::type;
        if constexpr (std::is_same<V, uint16_t>::value) return static_cast<TC>(bf16_to_f32(p[i]));
        else return static_cast<TC>(p[i]);
    };
    if (O * 2 >= kBlock || K <= 8) {
        for (int o = threadIdx.x; o < O; o += kBlock) {
            const int n = o % N, mb = o / N, m = mb % M, b = mb / M;
            const TA* a = A + b * sAb + m * sAm;
            const TB* bb = B + b * sBb + n * sBn;
            TC s = TC(0);
            for (int k = 0; k < K; ++k) s += ld(a, k * sAk) * ld(bb, k * sBk);
            C[b * sCb + m * sCm + n * sCn] = static_cast<double>(s);
        }
        __syncthreads();
        return;
    }
    int S = kBlock / O;
    if (S > (K + 3) / 4) S = (K + 3) / 4;
    const int kc = (K + S - 1) / S;
    const int o = threadIdx.x % O, sl = threadIdx.x / O;
    if (sl < S) {
        const int n = o % N, mb = o / N, m = mb % M, b = mb / M;
        const TA* a = A + b * sAb + m * sAm;
        const TB* bb = B + b * sBb + n * sBn;
        TC s = TC(0);
        const int k1 = min(K, (sl + 1) * kc);
        for (int k = sl * kc; k < k1; ++k) s += ld(a, k * sAk) * ld(bb, k * sBk);
        red[sl * O + o] = static_cast<double>(s);
    }
    __syncthreads();
    if (threadIdx.x < O) {
        const int n = o % N, mb = o / N, m = mb % M, b = mb / M;
        double s = 0.0;
        for (int t = 0; t < S; ++t) s += red[t * O + o];
        C[b * sCb + m * sCm + n * sCn] = s;
    }
    __syncthreads();
}

// U tables for one precision: element-type pointers to U and U^T of a Tab1D.
template <typename TU>
__device__ __forceinline__ const TU* u_ptr(const Params& P, const Tab1D& T, bool trans);
template <>
__device__ __forceinline__ const double* u_ptr<double>(const Params& P, const Tab1D& T, bool trans) {
    return P.dpool + (trans ? T.oUT : T.oU);
}
template <>
__device__ __forceinline__ const float* u_ptr<float>(const Params& P, const Tab1D& T, bool trans) {
    return P.fpool + (trans ? T.oUT32 : T.oU32);
}
template <>
__device__ __forceinline__ const uint16_t* u_ptr<uint16_t>(const Params& P, const Tab1D& T, bool trans) {
    return P.hpool + (trans ? T.oUT16 : T.oU16);
}

struct FdIO {
    const double* r_old;  // full grid input
    const double* q;      // r = r_old - alpha q when q != nullptr
    double alpha;
    double* r_out;        // owned part of r written here (or nullptr)
    double* dvec;         // dvec += alpha * pvec on owned part (or nullptr)
    const double* pvec;
    double* part;         // ||r_owned||^2 (forward) or r_owned . z_owned (backward)
    double* rt;           // transformed vector (grid-sized)
    double* z;            // backward output
    const double* rdot;   // backward: dot partner (or nullptr)
    int prec;             // 0 FP64, 1 FP32, 2 BF16 factors
};

// Owned index set of a block: unknowns whose index along g.big lies in the block.
__device__ __forceinline__ bool owned_2d(const Grid& g, int blk, int i1, int i2) {
    const int ib = g.big == 0 ? i1 : i2;
    return ib >= blk * g.blk && ib < min(g.ni[g.big], (blk + 1) * g.blk);
}

template <typename TU, typename TC>
__device__ void fd_fwd_2d(const Params& P, const Grid& g, int blk, const FdIO& io, double* lds) {
    const int n1 = g.ni[0], n2 = g.ni[1], n = n1 * n2;
    const Tab1D& T1 = P.tabs[g.tab[0]];
    const Tab1D& T2 = P.tabs[g.tab[1]];
    double* R = lds;
    double* S = lds + n;
    double* red = S + n;      // kBlock doubles of split-K / reduction scratch
    const int64_t off = g.dof_off;
    double nrm = 0.0;
    for (int i = threadIdx.x; i < n; i += kBlock) {
        double v = io.r_old[off + i];
        if (io.q) v -= io.alpha * io.q[off + i];
        R[i] = v;
        const int i1 = i % n1, i2 = i / n1;
        if (owned_2d(g, blk, i1, i2)) {
            if (io.r_out) io.r_out[off + i] = v;
            if (io.dvec) io.dvec[off + i] += io.alpha * io.pvec[off + i];
            nrm += v * v;
        }
    }
    if (io.part) {
        double t = wg_sum(nrm, red);
        if (threadIdx.x == 0) *io.part = t;
    }
    __syncthreads();
    const int k0 = blk * g.blk;
    const int bs = min(g.blk, g.ni[g.big] - k0);
    double* Out = red + kBlock;  // block of the transformed vector
    const double* lam1 = P.dpool + T1.oLam;
    const double* lam2 = P.dpool + T2.oLam;
    if (g.big == 0) {
        // S[k2][i1] = sum_i2 UT2[k2][i2] R[i2][i1]
        wg_gemm<TU, double, TC>(1, n2, n1, n2, u_ptr<TU>(P, T2, true), 0, n2, 1, R, 0, n1, 1, S, 0, n1, 1, red);
        // Rt[k2][k1] = sum_i1 S[k2][i1] U1[i1][k1], k1 in block
        wg_gemm<double, TU, TC>(1, n2, bs, n1, S, 0, n1, 1, u_ptr<TU>(P, T1, false) + k0, 0, n1, 1, Out, 0, bs,
                                1, red);
        for (int o = threadIdx.x; o < n2 * bs; o += kBlock) {
            const int k2 = o / bs, kk = o % bs, k1 = k0 + kk;
            io.rt[off + static_cast<int64_t>(k2) * n1 + k1] = Out[o] / (g.fdc[0] * lam1[k1] + g.fdc[1] * lam2[k2]);
        }
    } else {
        // S[i2][k1] = sum_i1 R[i2][i1] U1[i1][k1]
        wg_gemm<double, TU, TC>(1, n2, n1, n1, R, 0, n1, 1, u_ptr<TU>(P, T1, false), 0, n1, 1, S, 0, n1, 1, red);
        // Rt[k2][k1] = sum_i2 UT2[k2][i2] S[i2][k1], k2 in block
        wg_gemm<TU, double, TC>(1, bs, n1, n2, u_ptr<TU>(P, T2, true) + static_cast<int64_t>(k0) * n2, 0, n2, 1, S,
                                0, n1, 1, Out, 0, n1, 1, red);
        for (int o = threadIdx.x; o < bs * n1; o += kBlock) {
            const int kk = o / n1, k1 = o % n1, k2 = k0 + kk;
            io.rt[off + static_cast<int64_t>(k2) * n1 + k1] = Out[o] / (g.fdc[0] * lam1[k1] + g.fdc[1] * lam2[k2]);
        }
    }
    __syncthreads();
}

template <typename TU, typename TC>
__device__ void fd_bwd_2d(const Params& P, const Grid& g, int blk, const FdIO& io, double* lds) {
    const int n1 = g.ni[0], n2 = g.ni[1], n = n1 * n2;
    const Tab1D& T1 = P.tabs[g.tab[0]];
    const Tab1D& T2 = P.tabs[g.tab[1]];
    double* Rt = lds;
    double* Tm = lds + n;
    double* red = Tm + n;     // kBlock doubles of split-K / reduction scratch
    const int64_t off = g.dof_off;
    for (int i = threadIdx.x; i < n; i += kBlock) Rt[i] = io.rt[off + i];
    __syncthreads();
    const int k0 = blk * g.blk;
    const int bs = min(g.blk, g.ni[g.big] - k0);
    double* Out = red + kBlock;
    double dot = 0.0;
    if (g.big == 0) {
        // T[i2][k1] = sum_k2 U2[i2][k2] Rt[k2][k1]
        wg_gemm<TU, double, TC>(1, n2, n1, n2, u_ptr<TU>(P, T2, false), 0, n2, 1, Rt, 0, n1, 1, Tm, 0, n1, 1, red);
        // Z[i2][i1] = sum_k1 T[i2][k1] UT1[k1][i1], i1 in block
        wg_gemm<double, TU, TC>(1, n2, bs, n1, Tm, 0, n1, 1, u_ptr<TU>(P, T1, true) + k0, 0, n1, 1, Out, 0, bs, 1,
                                red);
        for (int o = threadIdx.x; o < n2 * bs; o += kBlock) {
            const int i2 = o / bs, i1 = k0 + o % bs;
            const int64_t gi = off + static_cast<int64_t>(i2) * n1 + i1;
            io.z[gi] = Out[o];
            if (io.rdot) dot += io.rdot[gi] * Out[o];
        }
    } else {
        // T[k2][i1] = sum_k1 Rt[k2][k1] UT1[k1][i1]
        wg_gemm<double, TU, TC>(1, n2, n1, n1, Rt, 0, n1, 1, u_ptr<TU>(P, T1, true), 0, n1, 1, Tm, 0, n1, 1, red);
        // Z[i2][i1] = sum_k2 U2[i2][k2] T[k2][i1], i2 in block
        wg_gemm<TU, double, TC>(1, bs, n1, n2, u_ptr<TU>(P, T2, false) + static_cast<int64_t>(k0) * n2, 0, n2, 1,
                                Tm, 0, n1, 1, Out, 0, n1, 1, red);
        for (int o = threadIdx.x; o < bs * n1; o += kBlock) {
            const int i2 = k0 + o / n1, i1 = o % n1;
            const int64_t gi = off + static_cast<int64_t>(i2) * n1 + i1;
            io.z[gi] = Out[o];
            if (io.rdot) dot += io.rdot[gi] * Out[o];
        }
    }
    if (io.part) {
        double t = wg_sum(dot, red);
        if (threadIdx.x == 0) *io.part = t;
    }
    __syncthreads();
}

__device__ void fd_fwd(const Params& P, const Grid& g, int blk, const FdIO& io, double* lds) {
    if (io.prec == 0) fd_fwd_2d<double, double>(P, g, blk, io, lds);
    else if (io.prec == 1) fd_fwd_2d<float, float>(P, g, blk, io, lds);
    else fd_fwd_2d<uint16_t, float>(P, g, blk, io, lds);
}

__device__ void fd_bwd(const Params& P, const Grid& g, int blk, const FdIO& io, double* lds) {
    if (io.prec == 0) fd_bwd_2d<double, double>(P, g, blk, io, lds);
    else if (io.prec == 1) fd_bwd_2d<float, float>(P, g, blk, io, lds);
    else fd_bwd_2d<uint16_t, float>(P, g, blk, io, lds);
}

// ===========================================================================
// grid-wide barrier (all workgroups co-resident: cooperative launch)
// ===========================================================================
__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned nwg) {
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        unsigned arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nwg - 1) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&bar[1], gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen)
                __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// ===========================================================================
// persistent refinement + PCG over all component grids
//
// One sweep = three phases separated by grid-wide barriers:
//   1 operator   ITER: p = z + beta p, q = A p (inner precision), p.q
//                RESID: r = b - A x (FP64), ||r||^2
//   2 update     ITER: alpha, d += alpha p, r -= alpha q, FD forward of r
//                XUPD: x += d, d = 0;  RESID: FD forward of r
//   3 commit     FD backward -> z, r.z; next state written by block 0
// Convergence tests use the preconditioned residual r.P^-1 r (relative to
// b.P^-1 b for the FP64 outer test, to its value at the start of an inner
// solve for the inner test); they are evaluated identically by every task of
// a grid from the same partial sums, so all tasks take the same decision.
// ===========================================================================
struct SolveArgs {
    int op_b, op_e, fd_b, fd_e;   // task ranges
    int ndone_target;             // grids in this launch
    int prec;                     // inner precision (IGA_PREC_*)
    int maxit, max_refine, max_sweeps;
    double tol2, tol_in2;
};

__device__ __forceinline__ double* part_ptr(const Params& P, int kind, int parity) {
    return P.part + static_cast<int64_t>(kind * 2 + parity) * P.part_stride;
}
enum { PK_PQ = 0, PK_RES = 1, PK_RR = 2, PK_RZ = 3 };
enum { ACT_SKIP = 0, ACT_RESID, ACT_ITER, ACT_XUPD, ACT_DONE };

struct Decision {
    int act, status;
    double rho, rhob, rho0;
};

__device__ Decision decide(const Params& P, const SolveArgs& A, const Grid& g, const GState& st, int nxt,
                           double* red) {
    Decision D;
    D.status = GS_OK;
    D.rho = 0.0;
    D.rhob = st.rhob;
    D.rho0 = st.rho0;
    if (st.stage == STAGE_DONE) {
        D.act = ACT_SKIP;
        return D;
    }
    if (st.stage == STAGE_RESID) {
        D.act = ACT_RESID;
        return D;
    }
    if (st.stage == STAGE_XUPD) {
        D.act = ACT_XUPD;
        return D;
    }
    const double rho = sum_partials(part_ptr(P, PK_RZ, nxt) + g.blk_off, g.nblk, red);
    D.rho = rho;
    if (!isfinite(rho) || rho < 0.0) {
        D.act = ACT_DONE;
        D.status = GS_BREAKDOWN;
    } else if (st.it == 0) {
        const double rhob = st.refine == 1 ? rho : st.rhob;
        D.rhob = rhob;
        if (rho <= A.tol2 * rhob) {
            D.act = ACT_DONE;
            D.status = GS_OK;
        } else if (st.refine > A.max_refine) {
            D.act = ACT_DONE;
            D.status = GS_MAXIT;
        } else {
            D.act = ACT_ITER;
            D.rho0 = rho;
        }
    } else if (rho <= A.tol_in2 * st.rho0 || st.it >= A.maxit) {
        D.act = ACT_XUPD;
    } else {
        D.act = ACT_ITER;
    }
    return D;
}

template <int PP>
__global__ void __launch_bounds__(kBlock) k_solve(Params P, SolveArgs A) {
    extern __shared__ double lds[];
    double* red = lds;
    const unsigned nwg = gridDim.x;
    const int64_t N = P.ndof_total;
    const int lowp = A.prec != IGA_PREC_FP64;
    const int fdprec = A.prec == IGA_PREC_FP64 ? 0 : (A.prec == IGA_PREC_FP32 ? 1 : 2);
    for (int sweep = 0; sweep < A.max_sweeps; ++sweep) {
        const int cur = sweep & 1, nxt = cur ^ 1;
        GState* S0 = P.st2 + cur * P.ngrid;
        GState* S1 = P.st2 + nxt * P.ngrid;
        double* r_new = P.r2 + cur * N;
        double* r_old = P.r2 + nxt * N;
        double* p_new = P.p2 + cur * N;
        double* p_old = P.p2 + nxt * N;
        // ---------------- phase 1: operator -------------------------------------
        for (int t = A.op_b + blockIdx.x; t < A.op_e; t += nwg) {
            const Task tk = P.optask[t];
            const Grid& g = P.grids[tk.grid];
            const GState st = S0[tk.grid];
            if (st.stage == STAGE_DONE) {
                if (tk.local == 0 && threadIdx.x == 0) S1[tk.grid] = st;  // carry forward
                continue;
            }
            const Decision D = decide(P, A, g, st, nxt, red);
            OpIO io;
            if (D.act == ACT_ITER) {
                io.in_a = P.z;
                io.in_b = p_old;
                io.beta = st.it == 0 ? 0.0 : D.rho / st.rho;
                io.out_in = p_new;
                io.out = P.q;
                io.rhs = nullptr;
                io.part = part_ptr(P, PK_PQ, cur) + g.tile_off + tk.local;
                io.lowp = lowp;
            } else if (D.act == ACT_RESID) {
                io.in_a = P.x;
                io.in_b = nullptr;
                io.beta = 0.0;
                io.out_in = nullptr;
                io.out = r_new;
                io.rhs = P.b;
                io.part = part_ptr(P, PK_RES, cur) + g.tile_off + tk.local;
                io.lowp = 0;
            } else {
                continue;
            }
            op_tile_2d<PP>(P, g, tk.local, io, lds);
        }
        grid_barrier(P.bar, nwg);
        // ---------------- phase 2: update + FD forward ---------------------------
        for (int t = A.fd_b + blockIdx.x; t < A.fd_e; t += nwg) {
            const Task tk = P.fdtask[t];
            const Grid& g = P.grids[tk.grid];
            const GState st = S0[tk.grid];
            if (st.stage == STAGE_DONE) continue;
            const Decision D = decide(P, A, g, st, nxt, red);
            const int n1 = g.ni[0];
            if (D.act == ACT_XUPD) {
                for (int i = threadIdx.x; i < g.ndof; i += kBlock) {
                    if (!owned_2d(g, tk.local, i % n1, i / n1)) continue;
                    const int64_t k = g.dof_off + i;
                    P.x[k] += P.d[k];
                    P.d[k] = 0.0;
                }
                continue;
            }
            FdIO io;
            io.rt = P.rt;
            io.prec = fdprec;
            io.z = nullptr;
            io.rdot = nullptr;
            io.part = part_ptr(P, PK_RR, cur) + g.blk_off + tk.local;
            if (D.act == ACT_ITER) {
                const double pq = sum_partials(part_ptr(P, PK_PQ, cur) + g.tile_off, g.ntile, red);
                if (!(pq > 0.0) || !isfinite(D.rho / pq)) continue;  // breakdown: committed in phase 3
                io.alpha = D.rho / pq;
                io.r_old = r_old;
                io.q = P.q;
                io.r_out = r_new;
                io.dvec = P.d;
                io.pvec = p_new;
            } else if (D.act == ACT_RESID) {
                io.alpha = 0.0;
                io.r_old = r_new;
                io.q = nullptr;
                io.r_out = nullptr;
                io.dvec = nullptr;
                io.pvec = nullptr;
            } else {
                continue;
            }
            fd_fwd(P, g, tk.local, io, lds);
        }
        grid_barrier(P.bar, nwg);
        // ---------------- phase 3: FD backward and commit ---------------------------
        for (int t = A.fd_b + blockIdx.x; t < A.fd_e; t += nwg) {
            const Task tk = P.fdtask[t];
            const int gi = tk.grid;
            const Grid& g = P.grids[gi];
            const GState st = S0[gi];
            if (st.stage == STAGE_DONE) continue;
            const Decision D = decide(P, A, g, st, nxt, red);
            GState ns = st;
            bool run_bwd = false, finish = false;
            if (D.act == ACT_ITER) {
                const double pq = sum_partials(part_ptr(P, PK_PQ, cur) + g.tile_off, g.ntile, red);
                ns.rhob = D.rhob;
                ns.rho0 = D.rho0;
                if (!(pq > 0.0) || !isfinite(D.rho / pq)) {
                    ns.stage = STAGE_DONE;
                    ns.status = GS_BREAKDOWN;
                    ns.total_it += st.it;
                    finish = true;
                } else {
                    ns.stage = STAGE_ITER;
                    ns.it = st.it + 1;
                    ns.rho = D.rho;
                    run_bwd = true;
                }
            } else if (D.act == ACT_XUPD) {
                ns.stage = STAGE_RESID;
                ns.total_it += st.it;
                ns.prelres = D.rhob > 0.0 ? sqrt(D.rho / D.rhob) : 0.0;
            } else if (D.act == ACT_RESID) {
                const double rn2 = sum_partials(part_ptr(P, PK_RES, cur) + g.tile_off, g.ntile, red);
                const double bn2 = st.refine == 0 ? rn2 : st.bn2;
                ns.bn2 = bn2;
                ns.relres = bn2 > 0.0 ? sqrt(rn2 / bn2) : 0.0;
                ns.stage = STAGE_ITER;
                ns.it = 0;
                ns.refine = st.refine + 1;
                run_bwd = true;
            } else if (D.act == ACT_DONE) {
                ns.stage = STAGE_DONE;
                ns.status = D.status;
                ns.rhob = D.rhob;
                ns.prelres = D.rhob > 0.0 ? sqrt(D.rho / D.rhob) : 0.0;
                finish = true;
            }
            if (run_bwd) {
                FdIO io;
                io.rt = P.rt;
                io.z = P.z;
                io.rdot = r_new;
                io.prec = fdprec;
                io.part = part_ptr(P, PK_RZ, cur) + g.blk_off + tk.local;
                fd_bwd(P, g, tk.local, io, lds);
            }
            if (tk.local == 0 && threadIdx.x == 0) {
                S1[gi] = ns;
                if (finish) atomicAdd(&P.bar[2], 1u);
            }
            __syncthreads();
        }
        grid_barrier(P.bar, nwg);
        const unsigned done = __hip_atomic_load(&P.bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (static_cast<int>(done) >= A.ndone_target) break;
    }
}

// Reset solver state and vectors of a grid range before a solve.
__global__ void __launch_bounds__(kBlock) k_solve_init(Params P, int g0, int g1, int64_t i0, int64_t i1) {
    const int64_t N = P.ndof_total;
    for (int64_t i = i0 + blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < i1;
         i += static_cast<int64_t>(gridDim.x) * kBlock) {
        P.x[i] = 0.0;
        P.d[i] = 0.0;
        P.z[i] = 0.0;
        P.p2[i] = 0.0;
        P.p2[N + i] = 0.0;
    }
    if (blockIdx.x == 0) {
        for (int g = g0 + threadIdx.x; g < g1; g += kBlock) {
            GState s;
            s.rho = 0.0;
            s.rho0 = 0.0;
            s.rhob = 0.0;
            s.bn2 = 0.0;
            s.relres = 0.0;
            s.prelres = 0.0;
            s.stage = STAGE_RESID;
            s.it = 0;
            s.total_it = 0;
            s.refine = 0;
            s.status = GS_RUNNING;
            s.pad = 0;
            P.st2[g] = s;
            P.st2[P.ngrid + g] = s;
        }
        if (threadIdx.x == 0) {
            P.bar[0] = 0u;
            P.bar[2] = 0u;
        }
    }
}

// Standalone operator / preconditioner launches (test hooks).
template <int PP>
__global__ void __launch_bounds__(kBlock) k_apply_op(Params P, int gi, OpIO io) {
    extern __shared__ double lds[];
    const Grid& g = P.grids[gi];
    OpIO a = io;
    a.part = nullptr;
    for (int t = blockIdx.x; t < g.ntile; t += gridDim.x) op_tile_2d<PP>(P, g, t, a, lds);
}
__global__ void __launch_bounds__(kBlock) k_apply_fd_fwd(Params P, int gi, FdIO io) {
    extern __shared__ double lds[];
    const Grid& g = P.grids[gi];
    for (int t = blockIdx.x; t < g.nblk; t += gridDim.x) fd_fwd(P, g, t, io, lds);
}
__global__ void __launch_bounds__(kBlock) k_apply_fd_bwd(Params P, int gi, FdIO io) {
    extern __shared__ double lds[];
    const Grid& g = P.grids[gi];
    for (int t = blockIdx.x; t < g.nblk; t += gridDim.x) fd_bwd(P, g, t, io, lds);
}

// ===========================================================================
// combination / evaluation: u(xi) = sum_c coef_c (sum_j x_j B_j(xi)) / W(xi)
// ===========================================================================
__global__ void __launch_bounds__(kBlock) k_combine(Params P, const double* xi, const int* patch, int64_t n,
                                                   double* u, int g0, int g1, int use_coef) {
    const int d = P.dim, p = P.p;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock) {
        double xv[3] = {0, 0, 0};
        for (int k = 0; k < d; ++k) {
            double t = xi[i * d + k];
            xv[k] = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
        }
        const int pt = patch ? patch[i] : 0;
        // weight function W(xi) of the geometry
        double W = 1.0;
        if (P.rational[pt]) {
            double Ng[3][kMaxPg + 1];
            int fg[3] = {0, 0, 0};
            int pgk[3] = {0, 0, 0};
            for (int k = 0; k < d; ++k) {
                const Tab1D& T = P.tabs[P.grids[g0].tab[k]];
                const double* gk = P.dpool + T.oGkn;
                pgk[k] = T.pg;
                int s = d_find_interval(T.pg, T.ngk, gk, xv[k]);
                d_basis_funs(T.pg, gk, s, xv[k], Ng[k], nullptr);
                fg[k] = s - T.pg;
            }
            W = 0.0;
            const double* C = P.ctrl + P.ctrl_off[pt];
            const int lim2 = d > 2 ? pgk[2] : 0;
            for (int c = 0; c <= lim2; ++c)
                for (int b = 0; b <= pgk[1]; ++b)
                    for (int a = 0; a <= pgk[0]; ++a) {
                        int64_t idx = (fg[0] + a) + static_cast<int64_t>(P.gn[pt][0]) *
                                                        ((fg[1] + b) + static_cast<int64_t>(P.gn[pt][1]) * (d > 2 ? fg[2] + c : 0));
                        W += C[idx * 4 + 3] * Ng[0][a] * Ng[1][b] * (d > 2 ? Ng[2][c] : 1.0);
                    }
        }
        double acc = 0.0;
        for (int gi = g0; gi < g1; ++gi) {
            const Grid& g = P.grids[gi];
            if (g.patch != pt) continue;
            double N[3][kMaxPg + 1];
            int f[3] = {0, 0, 0};
            for (int k = 0; k < d; ++k) {
                const Tab1D& T = P.tabs[g.tab[k]];
                int e;
                if (T.uniform) {
                    e = static_cast<int>(xv[k] * T.E);
                    e = e > T.E - 1 ? T.E - 1 : e;
                } else {
                    const double* brk = P.dpool + T.oBrk;
                    int lo = 0, hi = T.E;
                    while (hi - lo > 1) {
                        int mid = (lo + hi) >> 1;
                        if (xv[k] < brk[mid]) hi = mid;
                        else lo = mid;
                    }
                    e = lo;
                }
                d_basis_funs(p, P.dpool + T.oKn, p + e * T.m, xv[k], N[k], nullptr);
                f[k] = e * T.m - 1;  // interior index of the first local function
            }
            double v = 0.0;
            const double* X = P.x + g.dof_off;
            const int lim2 = d > 2 ? p : 0;
            for (int c = 0; c <= lim2; ++c) {
                const int i3 = d > 2 ? f[2] + c : 0;
                if (i3 < 0 || i3 >= g.ni[2]) continue;
                for (int b = 0; b <= p; ++b) {
                    const int i2 = f[1] + b;
                    if (i2 < 0 || i2 >= g.ni[1]) continue;
                    for (int a = 0; a <= p; ++a) {
                        const int i1 = f[0] + a;
                        if (i1 < 0 || i1 >= g.ni[0]) continue;
                        v += X[i1 + static_cast<int64_t>(g.ni[0]) * (i2 + static_cast<int64_t>(g.ni[1]) * i3)] *
                             N[0][a] * N[1][b] * (d > 2 ? N[2][c] : 1.0);
                    }
                }
            }
            acc += (use_coef ? g.ccoef : 1.0) * (v / W);
        }
        u[i] = acc;
    }
}

Params make_params(iga_sg_plan_s* P) {
    Params K;
    std::memset(&K, 0, sizeof(K));
    char* base = static_cast<char*>(P->ws);
    const Layout& L = P->lay;
    K.tabs = reinterpret_cast<const Tab1D*>(base + L.tabs);
    K.grids = reinterpret_cast<const Grid*>(base + L.grids);
    K.dpool = reinterpret_cast<const double*>(base + L.dpool);
    K.ipool = reinterpret_cast<const int*>(base + L.ipool);
    K.fpool = reinterpret_cast<const float*>(base + L.fpool);
    K.hpool = reinterpret_cast<const uint16_t*>(base + L.hpool);
    K.ctrl = reinterpret_cast<const double*>(base + L.ctrl);
    for (int pt = 0; pt < static_cast<int>(P->patches.size()); ++pt) {
        K.ctrl_off[pt] = P->ctrl_off[pt];
        for (int k = 0; k < P->dim; ++k) {
            K.gdeg[pt][k] = P->patches[pt].degree[k];
            K.gn[pt][k] = static_cast<int>(P->patches[pt].knots[k].size()) - P->patches[pt].degree[k] - 1;
        }
        for (int k = P->dim; k < 3; ++k) K.gn[pt][k] = 1;
        bool rat = false;
        for (double w : P->patches[pt].weights)
            if (w != P->patches[pt].weights[0]) rat = true;
        K.rational[pt] = rat ? 1 : 0;
    }
    K.dim = P->dim;
    K.p = P->p;
    K.nq = P->nq;
    K.ncompG = P->ncompG;
    K.ngrid = static_cast<int>(P->grids.size());
    K.nop = static_cast<int>(P->optask.size());
    K.nfd = static_cast<int>(P->fdtask.size());
    K.nqp_total = P->nqp_total;
    K.ndof_total = P->ndof_total;
    K.G64 = reinterpret_cast<double*>(base + L.G64);
    K.G32 = reinterpret_cast<float*>(base + L.G32);
    K.Fq = reinterpret_cast<double*>(base + L.Fq);
    K.b = reinterpret_cast<double*>(base + L.b);
    K.x = reinterpret_cast<double*>(base + L.x);
    K.d = reinterpret_cast<double*>(base + L.d);
    K.r2 = reinterpret_cast<double*>(base + L.r2);
    K.z = reinterpret_cast<double*>(base + L.z);
    K.p2 = reinterpret_cast<double*>(base + L.p2);
    K.q = reinterpret_cast<double*>(base + L.q);
    K.rt = reinterpret_cast<double*>(base + L.rt);
    K.st2 = reinterpret_cast<GState*>(base + L.st2);
    K.part = reinterpret_cast<double*>(base + L.part);
    K.part_stride = static_cast<int64_t>(std::max(P->optask.size(), P->fdtask.size()));
    K.optask = reinterpret_cast<const Task*>(base + L.optask);
    K.fdtask = reinterpret_cast<const Task*>(base + L.fdtask);
    K.bar = reinterpret_cast<unsigned*>(base + L.bar);
    for (int i = 0; i < P->nq && i < 8; ++i) {
        K.gx[i] = P->gauss_x[i];
        K.gw[i] = P->gauss_w[i];
    }
    return K;
}

const void* solve_kernel(int p) {
    switch (p) {
        case 1: return reinterpret_cast<const void*>(k_solve<1>);
        case 2: return reinterpret_cast<const void*>(k_solve<2>);
        case 3: return reinterpret_cast<const void*>(k_solve<3>);
        default: return reinterpret_cast<const void*>(k_solve<4>);
    }
}

}  // namespace igasg

// ===========================================================================
// C ABI
// ===========================================================================
namespace {

FieldDev to_dev(const iga_field* f) {
    FieldDev F;
    std::memset(&F, 0, sizeof(F));
    F.kind = f ? f->kind : IGA_FIELD_NONE;
    if (f) {
        for (int i = 0; i < 4; ++i) F.prm[i] = f->prm[i];
        F.data = f->data_dev;
        for (int k = 0; k < 3; ++k) F.n[k] = f->n[k];
    }
    return F;
}

bool field_ok(const iga_field* f, int dim) {
    if (!f) return false;
    if (f->kind < IGA_FIELD_CONST || f->kind > IGA_FIELD_AFFINE) return false;
    if (f->kind == IGA_FIELD_GRID3D && (dim != 3 || !f->data_dev || f->n[0] < 2 || f->n[1] < 2 || f->n[2] < 2))
        return false;
    return true;
}

int blocks_for(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    return static_cast<int>(std::min<int64_t>(std::max<int64_t>(b, 1), 65535));
}

}  // namespace

extern "C" {

iga_status iga_sg_bind(iga_sg_plan P, void* ws, size_t bytes, void* stream) {
    if (!P || !ws) {
        set_error("null plan or workspace");
        return IGA_ERR_INVALID_ARG;
    }
    if (bytes < P->lay.total) {
        set_error("workspace too small: %zu < %zu bytes", bytes, P->lay.total);
        return IGA_ERR_OUT_OF_MEMORY;
    }
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) {
        set_error("workspace must be 256-byte aligned");
        return IGA_ERR_INVALID_ARG;
    }
    P->ws = ws;
    P->ws_bytes = bytes;
    P->stream = stream;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(ws);
    const Layout& L = P->lay;
    HIP_OK(hipMemcpyAsync(base + L.tabs, P->tabs.data(), sizeof(Tab1D) * P->tabs.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(base + L.grids, P->grids.data(), sizeof(Grid) * P->grids.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(base + L.dpool, P->dpool.data(), sizeof(double) * P->dpool.size(), hipMemcpyHostToDevice, st));
    if (!P->ipool.empty())
        HIP_OK(hipMemcpyAsync(base + L.ipool, P->ipool.data(), sizeof(int) * P->ipool.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(base + L.fpool, P->fpool.data(), sizeof(float) * P->fpool.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(base + L.hpool, P->hpool.data(), sizeof(uint16_t) * P->hpool.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(base + L.ctrl, P->ctrl.data(), sizeof(double) * P->ctrl.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(base + L.optask, P->optask.data(), sizeof(Task) * P->optask.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(base + L.fdtask, P->fdtask.data(), sizeof(Task) * P->fdtask.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemsetAsync(base + L.bar, 0, 256, st));
    Params K = make_params(P);
    int maxQ = 0;
    for (const Tab1D& T : P->tabs) maxQ = std::max(maxQ, T.Q);
    dim3 grid((maxQ + kBlock - 1) / kBlock, static_cast<unsigned>(P->tabs.size()));
    hipLaunchKernelGGL(k_tables, grid, dim3(kBlock), 0, st, K);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(st));
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, dev));
    P->num_cu = prop.multiProcessorCount;
    int occ = 0;
    HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, solve_kernel(P->p), kBlock, P->lds_bytes));
    P->max_wg = std::max(1, occ) * P->num_cu;
    for (int i = 0; i < 8; ++i)
        if (!P->ev[i]) HIP_OK(hipEventCreate(reinterpret_cast<hipEvent_t*>(&P->ev[i])));
    P->bound = true;
    P->assembled = false;
    P->solved = false;
    return IGA_OK;
}

iga_status iga_sg_assemble(iga_sg_plan P, const iga_field* f, const iga_field* a, const iga_field* g) {
    if (!P) {
        set_error("null plan");
        return IGA_ERR_INVALID_ARG;
    }
    if (!P->bound) {
        set_error("iga_sg_assemble before iga_sg_bind");
        return IGA_ERR_STATE;
    }
    if (!field_ok(f, P->dim) || !field_ok(a, P->dim)) {
        set_error("invalid f or a field");
        return IGA_ERR_INVALID_ARG;
    }
    if (g && g->kind != IGA_FIELD_NONE) {
        set_error("nonhomogeneous Dirichlet data is not supported by the GPU path");
        return IGA_ERR_INVALID_ARG;
    }
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    Params K = make_params(P);
    int* err = reinterpret_cast<int*>(reinterpret_cast<char*>(P->ws) + P->lay.bar + 64);
    HIP_OK(hipMemsetAsync(err, 0, sizeof(int), st));
    const int ng = static_cast<int>(P->grids.size());
    hipLaunchKernelGGL(k_assemble, dim3(blocks_for(P->nqp_total)), dim3(kBlock), 0, st, K, to_dev(a), to_dev(f), 0,
                       ng, err);
    HIP_OK(hipGetLastError());
    hipLaunchKernelGGL(k_rhs, dim3(blocks_for(P->ndof_total)), dim3(kBlock), 0, st, K, 0, ng);
    HIP_OK(hipGetLastError());
    P->assembled = true;
    P->solved = false;
    return IGA_OK;
}

iga_status iga_sg_solve(iga_sg_plan P, const iga_sg_solve_opts* o, iga_sg_report* rep) {
    if (!P || !o) {
        set_error("null argument");
        return IGA_ERR_INVALID_ARG;
    }
    if (!P->assembled) {
        set_error("iga_sg_solve before iga_sg_assemble");
        return IGA_ERR_STATE;
    }
    if (o->precision < IGA_PREC_FP64 || o->precision > IGA_PREC_BF16FD || !(o->tol > 0) || o->maxit < 1) {
        set_error("invalid solve options");
        return IGA_ERR_INVALID_ARG;
    }
    if (P->dim != 2) {
        set_error("the GPU solve path currently supports dim = 2");
        return IGA_ERR_INVALID_ARG;
    }
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    Params K = make_params(P);
    const int ng = static_cast<int>(P->grids.size());
    SolveArgs A;
    A.prec = o->precision;
    A.maxit = o->maxit;
    A.max_refine = o->precision == IGA_PREC_FP64 ? std::max(1, o->max_refine > 0 ? o->max_refine : 3)
                                                 : std::max(1, o->max_refine);
    A.tol2 = o->tol * o->tol;
    // FP64: the inner test equals the outer one; mixed: loose inner tolerance
    double ti = o->precision == IGA_PREC_FP64 ? o->tol : (o->tol_inner > 0 ? o->tol_inner : 1e-4);
    A.tol_in2 = ti * ti;
    A.max_sweeps = (A.maxit + 2) * (A.max_refine + 1) + 4;
    const size_t lds = P->lds_bytes;
    hipEvent_t e0 = static_cast<hipEvent_t>(P->ev[0]), e1 = static_cast<hipEvent_t>(P->ev[1]);
    if (o->timing) HIP_OK(hipEventRecord(e0, st));
    auto launch = [&](int g0, int g1, int opb, int ope, int fdb, int fde) -> iga_status {
        const int64_t i0 = P->grids[g0].dof_off;
        const int64_t i1 = P->grids[g1 - 1].dof_off + P->grids[g1 - 1].ndof;
        hipLaunchKernelGGL(k_solve_init, dim3(blocks_for(i1 - i0)), dim3(kBlock), 0, st, K, g0, g1, i0, i1);
        HIP_OK(hipGetLastError());
        A.op_b = opb;
        A.op_e = ope;
        A.fd_b = fdb;
        A.fd_e = fde;
        A.ndone_target = g1 - g0;
        int want = std::max(ope - opb, fde - fdb);
        if (o->workgroups > 0) want = o->workgroups;
        int nwg = std::max(1, std::min(want, P->max_wg));
        void* args[] = {&K, &A};
        HIP_OK(hipLaunchCooperativeKernel(solve_kernel(P->p), dim3(nwg), dim3(kBlock), args,
                                          static_cast<unsigned>(lds), st));
        return IGA_OK;
    };
    if (o->batched) {
        iga_status s = launch(0, ng, 0, static_cast<int>(P->optask.size()), 0, static_cast<int>(P->fdtask.size()));
        if (s != IGA_OK) return s;
    } else {
        for (int gi = 0; gi < ng; ++gi) {
            const Grid& g = P->grids[gi];
            iga_status s = launch(gi, gi + 1, g.tile_off, g.tile_off + g.ntile, g.blk_off, g.blk_off + g.nblk);
            if (s != IGA_OK) return s;
        }
    }
    if (o->timing) {
        HIP_OK(hipEventRecord(e1, st));
    }
    P->solved = true;
    const bool need_state = rep != nullptr;
    if (!need_state && !o->timing) return IGA_OK;
    std::vector<GState> both(2 * static_cast<size_t>(ng)), stv(ng);
    HIP_OK(hipMemcpyAsync(both.data(), reinterpret_cast<char*>(P->ws) + P->lay.st2, sizeof(GState) * 2 * ng,
                          hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    for (int gi = 0; gi < ng; ++gi) {
        const GState& a = both[gi];
        const GState& b = both[ng + gi];
        // the buffer written last holds the final state: DONE wins, else the later one
        if (a.stage == STAGE_DONE && b.stage != STAGE_DONE) stv[gi] = a;
        else if (b.stage == STAGE_DONE && a.stage != STAGE_DONE) stv[gi] = b;
        else stv[gi] = (a.total_it + a.it + 2 * a.refine >= b.total_it + b.it + 2 * b.refine) ? a : b;
    }
    iga_status ret = IGA_OK;
    int total = 0;
    for (int gi = 0; gi < ng; ++gi) {
        const GState& s = stv[gi];
        // the state buffer of the parity last written holds DONE for finished grids
        total += s.total_it;
        if (s.stage != STAGE_DONE || s.status == GS_MAXIT || s.status == GS_RUNNING) {
            if (ret == IGA_OK) ret = IGA_ERR_NOT_CONVERGED;
        }
        if (s.status == GS_BREAKDOWN) ret = IGA_ERR_BREAKDOWN;
    }
    if (rep) {
        rep->ncomp = P->ncomp;
        rep->total_iters = total;
        for (int gi = 0; gi < ng; ++gi) {
            const GState& s = stv[gi];
            const int c = P->grids[gi].comp;
            if (rep->iters) rep->iters[c] = s.total_it;
            if (rep->refinements) rep->refinements[c] = s.refine;
            if (rep->relres) rep->relres[c] = s.relres;
            if (rep->prelres) rep->prelres[c] = s.prelres;
            if (rep->status) rep->status[c] = s.stage == STAGE_DONE ? s.status : GS_MAXIT;
        }
        if (o->timing) {
            float ms = 0.0f;
            HIP_OK(hipEventElapsedTime(&ms, e0, e1));
            rep->kernel_ms[1] = ms;
        }
    }
    if (ret == IGA_ERR_NOT_CONVERGED) set_error("some component did not reach the tolerance");
    if (ret == IGA_ERR_BREAKDOWN) set_error("CG breakdown in some component");
    return ret;
}

iga_status iga_sg_combine(iga_sg_plan P, const double* xi, const int* patch, int64_t n, double* u) {
    if (!P || (n > 0 && (!xi || !u)) || n < 0) {
        set_error("invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    if (!P->solved) {
        set_error("iga_sg_combine before iga_sg_solve");
        return IGA_ERR_STATE;
    }
    if (n == 0) return IGA_OK;
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    Params K = make_params(P);
    hipLaunchKernelGGL(k_combine, dim3(blocks_for(n)), dim3(kBlock), 0, st, K, xi, patch, n, u, 0,
                       static_cast<int>(P->grids.size()), 1);
    HIP_OK(hipGetLastError());
    return IGA_OK;
}

iga_status iga_sg_eval(iga_sg_plan P, int comp, const double* xi, const int* patch, int64_t n, double* u) {
    if (!P || comp < 0 || comp >= P->ncomp || (n > 0 && (!xi || !u)) || n < 0) {
        set_error("invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    if (!P->solved) {
        set_error("iga_sg_eval before iga_sg_solve");
        return IGA_ERR_STATE;
    }
    if (n == 0) return IGA_OK;
    int g0 = -1, g1 = -1;
    for (int gi = 0; gi < static_cast<int>(P->grids.size()); ++gi)
        if (P->grids[gi].comp == comp) {
            if (g0 < 0) g0 = gi;
            g1 = gi + 1;
        }
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    Params K = make_params(P);
    hipLaunchKernelGGL(k_combine, dim3(blocks_for(n)), dim3(kBlock), 0, st, K, xi, patch, n, u, g0, g1, 0);
    HIP_OK(hipGetLastError());
    return IGA_OK;
}

iga_status iga_sg_coeffs(iga_sg_plan P, int comp, double* out) {
    if (!P || comp < 0 || comp >= P->ncomp || !out) {
        set_error("invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    if (!P->solved) {
        set_error("iga_sg_coeffs before iga_sg_solve");
        return IGA_ERR_STATE;
    }
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    Params K = make_params(P);
    for (const Grid& g : P->grids)
        if (g.comp == comp)
            HIP_OK(hipMemcpyAsync(out, K.x + g.dof_off, sizeof(double) * g.ndof, hipMemcpyDeviceToDevice, st));
    return IGA_OK;
}

iga_status iga_sg_rhs(iga_sg_plan P, int comp, double* out) {
    if (!P || comp < 0 || comp >= P->ncomp || !out) {
        set_error("invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    if (!P->assembled) {
        set_error("iga_sg_rhs before iga_sg_assemble");
        return IGA_ERR_STATE;
    }
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    Params K = make_params(P);
    for (const Grid& g : P->grids)
        if (g.comp == comp)
            HIP_OK(hipMemcpyAsync(out, K.b + g.dof_off, sizeof(double) * g.ndof, hipMemcpyDeviceToDevice, st));
    return IGA_OK;
}

iga_status iga_sg_apply(iga_sg_plan P, int comp, int which, const double* x, double* y) {
    if (!P || comp < 0 || comp >= P->ncomp || !x || !y || which < 0 || which > 4) {
        set_error("invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    if (!P->assembled) {
        set_error("iga_sg_apply before iga_sg_assemble");
        return IGA_ERR_STATE;
    }
    if (P->dim != 2) {
        set_error("iga_sg_apply currently supports dim = 2");
        return IGA_ERR_INVALID_ARG;
    }
    int gi = -1;
    for (int i = 0; i < static_cast<int>(P->grids.size()); ++i)
        if (P->grids[i].comp == comp) gi = i;
    const Grid& g = P->grids[gi];
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    Params K = make_params(P);
    // the hooks read/write the caller's vectors shifted to the grid's offset
    const double* xs = x - g.dof_off;
    double* ys = y - g.dof_off;
    if (which <= 1) {
        OpIO io;
        io.in_a = xs;
        io.in_b = nullptr;
        io.beta = 0.0;
        io.out_in = nullptr;
        io.out = ys;
        io.rhs = nullptr;
        io.part = nullptr;
        io.lowp = which;
        switch (P->p) {
            case 1: hipLaunchKernelGGL(k_apply_op<1>, dim3(g.ntile), dim3(kBlock), P->lds_bytes, st, K, gi, io); break;
            case 2: hipLaunchKernelGGL(k_apply_op<2>, dim3(g.ntile), dim3(kBlock), P->lds_bytes, st, K, gi, io); break;
            case 3: hipLaunchKernelGGL(k_apply_op<3>, dim3(g.ntile), dim3(kBlock), P->lds_bytes, st, K, gi, io); break;
            default: hipLaunchKernelGGL(k_apply_op<4>, dim3(g.ntile), dim3(kBlock), P->lds_bytes, st, K, gi, io); break;
        }
        HIP_OK(hipGetLastError());
    } else {
        FdIO io;
        std::memset(&io, 0, sizeof(io));
        io.r_old = xs;
        io.rt = K.rt;
        io.z = ys;
        io.prec = which - 2;
        hipLaunchKernelGGL(k_apply_fd_fwd, dim3(g.nblk), dim3(kBlock), P->lds_bytes, st, K, gi, io);
        HIP_OK(hipGetLastError());
        hipLaunchKernelGGL(k_apply_fd_bwd, dim3(g.nblk), dim3(kBlock), P->lds_bytes, st, K, gi, io);
        HIP_OK(hipGetLastError());
    }
    return IGA_OK;
}

void iga_sg_destroy(iga_sg_plan P) {
    if (!P) return;
    for (int i = 0; i < 8; ++i)
        if (P->ev[i]) (void)hipEventDestroy(static_cast<hipEvent_t>(P->ev[i]));
    delete P;
}

}  // extern "C"
