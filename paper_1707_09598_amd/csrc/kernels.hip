// kernels.hip -- gfx950 kernels of the sparse-grid isogeometric solver and
// the C-ABI entry points that launch them.
//
//   k_tables      Cox-de Boor values/derivatives at the Gauss points of every
//                 level (eq. Bsp), geometry basis tables
//   k_assemble    per Gauss point: NURBS map F (eq. F-B-splines), Jacobian,
//                 a, f, operator coefficients a w |det DF| DF^-1 DF^-T and the
//                 load density (Galerkin form of Problem 1)
//   k_elemloc     per element and local basis function: its load and
//                 operator-diagonal sums over the element's Gauss points
//   k_gather      load vector b_j = sum_q f w |det DF| phi_j and the
//                 preconditioner scaling from the operator diagonal
//   k_solve       persistent refinement + fast-diagonalisation PCG over all
//                 component grids (grid-wide barrier between phases)
//   k_combine     u_sg(xi) = sum_i c_i u_i(xi), eq. (TD-combi-tec), FP64
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "device.hpp"
#include "iga_nn.h"
#include "plan.hpp"
#include "solve.hpp"

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

constexpr int kTraceSweeps = 4096;

// ===========================================================================
// fields
// ===========================================================================
struct FieldDev {
    int kind;
    double prm[4];
    const double* data;
    int n[3];
    int64_t sample_stride;  // elements between the data of consecutive samples
};
// The field of one grid's coefficient sample.
__device__ __forceinline__ FieldDev field_of_sample(FieldDev f, int sample) {
    if (f.data) f.data += sample * f.sample_stride;
    return f;
}

__device__ __forceinline__ void sincos_coef(const double* prm, const double* x, double* a, double* da) {
    const double tp = 6.283185307179586476925;
    double sx, cx, sy, cy;
    sincos(tp * (x[0] + prm[1]), &sx, &cx);
    sincos(tp * x[1], &sy, &cy);
    *a = 1.0 + prm[0] * sx * cy;
    da[0] = tp * prm[0] * cx * cy;
    da[1] = -tp * prm[0] * sx * sy;
}

__device__ __forceinline__ double field_eval(const FieldDev& F, int dim, const double* x) {
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

// Field of a kind fixed at compile time (the switch of field_eval folds to
// one branch, which keeps the register use of the assembly kernels low);
// K < 0: the kind is read at run time.
template <int K>
__device__ __forceinline__ double field_eval_k(const FieldDev& F, int dim, const double* x) {
    if constexpr (K < 0) {
        return field_eval(F, dim, x);
    } else {
        FieldDev G = F;
        G.kind = K;
        return field_eval(G, dim, x);
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
// Grid of a Gauss point / of an unknown in [g0, g1): binary search over the
// grid offsets; over all grids of several samples, over the grids of one
// sample after the sample is found from the per-sample totals.
__device__ __forceinline__ int grid_of_qp(const Params& P, int g0, int g1, int64_t gq) {
    int base = 0;
    if (g0 == 0 && g1 == P.ngrid && P.ngrid1 < P.ngrid) {
        const int smp = static_cast<int>(gq / P.nqp1);
        base = smp * P.ngrid1;
        g0 = base;
        g1 = base + P.ngrid1;
    }
    int lo = g0, hi = g1 - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (P.grids[mid].qp_off <= gq) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}
// The same for all lanes of a wavefront at once: the grid of the first active
// lane's point is searched with wavefront-uniform indices (one search per
// wavefront), lanes whose point lies outside that grid search their own.
__device__ __forceinline__ int grid_of_qp_w(const Params& P, int g0, int g1, int64_t gq) {
    const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(gq));
    const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(static_cast<uint64_t>(gq) >> 32));
    const int64_t q0 = static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
    const int gw = grid_of_qp(P, g0, g1, q0);
    const Grid& G = P.grids[gw];
    if (gq >= G.qp_off && gq < G.qp_off + G.nqp) return gw;
    return grid_of_qp(P, g0, g1, gq);
}
__device__ __forceinline__ int grid_of_dof(const Params& P, int g0, int g1, int64_t gi) {
    if (g0 == 0 && g1 == P.ngrid && P.ngrid1 < P.ngrid) {
        const int smp = static_cast<int>(gi / P.ndof1);
        g0 = smp * P.ngrid1;
        g1 = g0 + P.ngrid1;
    }
    int lo = g0, hi = g1 - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (P.grids[mid].dof_off <= gi) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Geometry at a tensor Gauss point from the per-direction geometry tables:
// homogeneous sums X_c = sum w P_c B, W = sum w B and their derivatives.
template <int DIM>
__device__ __forceinline__ void geom_at(const Params& P, const Grid& g, const int* qk, double* x,
                                        double DF[3][3], double* W, double* dW) {
    constexpr int d = DIM;
    const int pt = g.patch;
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

template <int KA, int KF, int DIM>
__global__ void __launch_bounds__(kBlock) k_assemble(Params P, FieldDev fa, FieldDev ff, int g0, int g1,
                                                    int* err) {
    const int64_t q0 = P.grids[g0].qp_off;
    const int64_t q1 = P.grids[g1 - 1].qp_off + P.grids[g1 - 1].nqp;
    constexpr int d = DIM;
    for (int64_t gq = q0 + blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; gq < q1;
         gq += static_cast<int64_t>(gridDim.x) * kBlock) {
        const int gi = grid_of_qp_w(P, g0, g1, gq);
        const Grid& g = P.grids[gi];
        // storage index l of the point; lt its index in the tensor order of
        // the grid's Gauss points (fields sampled at the points).  2D: the
        // same.  3D: element-major, l = ((element * NQ + j3) * NQ + j2) * NQ + j1
        // with the elements direction 1 fastest, so that the coefficients of
        // an element (and of one of its layers) are contiguous for the
        // operator and the element sums
        const int64_t l = gq - g.qp_off;
        int64_t lt = l;
        int qk[3];
        if constexpr (DIM == 3) {
            const int nq = P.p + 1, nq2 = nq * nq;
            const int64_t e = l / (nq2 * nq);
            const int r = static_cast<int>(l - e * nq2 * nq);
            const int64_t e23 = e / g.E[0];
            qk[0] = static_cast<int>(e - e23 * g.E[0]) * nq + r % nq;
            qk[1] = static_cast<int>(e23 % g.E[1]) * nq + (r / nq) % nq;
            qk[2] = static_cast<int>(e23 / g.E[1]) * nq + r / nq2;
            lt = (static_cast<int64_t>(qk[2]) * g.Q[1] + qk[1]) * g.Q[0] + qk[0];
        } else {
            qk[0] = static_cast<int>(l % g.Q[0]);
            qk[1] = static_cast<int>((l / g.Q[0]) % g.Q[1]);
            qk[2] = 0;
        }
        double x[3] = {0, 0, 0}, DF[3][3], W, dW[3] = {0, 0, 0};
        geom_at<DIM>(P, g, qk, x, DF, &W, dW);
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
        // a field sampled at the Gauss points holds its value at the point's
        // index in the tensor order
        const double av = fa.kind == IGA_FIELD_QP_SAMPLES ? fa.data[g.qp_off + lt]
                                                          : field_eval_k<KA>(field_of_sample(fa, g.sample), d, x);
        const double fv = ff.kind == IGA_FIELD_QP_SAMPLES ? ff.data[g.qp_off + lt]
                                                          : field_eval_k<KF>(field_of_sample(ff, g.sample), d, x);
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


// ---------------------------------------------------------------------------
// Load vector and diagonal of the operator, element by element.
//
// Every Gauss point lies in one element and contributes to the (p+1)^d basis
// functions that are nonzero there.  k_elemloc visits each element once: lane
// a of the element's lane group takes local basis function
// B_a = B_{a0}(xi_0) B_{a1}(xi_1) [B_{a2}(xi_2)] and sums over the element's
// Gauss points
//   bl(a) = sum_q Fq(q) B_a(q)                      (Fq = f w |det DF| / W)
//   dl(a) = sum_q sum_uv G_uv(q) f_u(q) f_v(q)      (f = grad B_a, or
//           (B_a, grad B_a) for the rational form; both orders for u != v)
// with the element's coefficients staged once in LDS and read by every lane
// of the group.  The sums are stored structure-of-arrays by local index,
// loc[a][element] (dl) and loc[nloc + a][element] (bl), so that the gather
// reads them with consecutive unknowns on consecutive elements.
//
// k_gather, one thread per unknown: b_i = sum of bl over the elements of the
// support of B_i, A_ii likewise from dl, in a fixed element order (bitwise
// reproducible), and the preconditioner scaling s_i = sqrt(P_ii / A_ii) with
// P = sum_k K_k (x) prod_{l != k} M_l the pencil of the 1D matrices, so that
// S P S has the diagonal of A.
// ---------------------------------------------------------------------------
template <int DIM, int PP>
struct ElemShape {
    static constexpr int NQ = PP + 1;                                          // Gauss points = local functions per direction
    static constexpr int NLOC = DIM == 2 ? NQ * NQ : NQ * NQ * NQ;             // per element
    static constexpr int NLP = NLOC <= 4 ? 4 : NLOC <= 8 ? 8 : NLOC <= 16 ? 16 : NLOC <= 32 ? 32 : 64;
    static constexpr int EPW = 64 / NLP;                                       // elements per wavefront
    static constexpr int LPL = (NLOC + 63) / 64;                               // local functions per lane
};

// The Gauss-point sums are evaluated by sum factorisation: with f_u f_v a
// product of one 1D factor per direction (B B, B D or D D of the local
// function's 1D value B and derivative D, by whether u and v differentiate in
// that direction; a single B for the load), each coefficient's sum over the
// element's NQ^d points is d successive contractions over one direction,
//   T_k(a_0..a_k, q_{k+1}..) = sum_j W_k(a_k, j) T_{k-1}(a_0..a_{k-1}, j, q_{k+1}..),
// NQ multiply-adds per coefficient and stage for each lane, the stages
// exchanged through LDS.  Position pos of a lane group is the tensor index
// with direction 0 fastest (local function index after the last stage).
template <int DIM, int PP, bool RAT>
__global__ void __launch_bounds__(kBlock) k_elemloc(Params P) {
    using SH = ElemShape<DIM, PP>;
    constexpr int NQ = SH::NQ, NLOC = SH::NLOC, NLP = SH::NLP, EPW = SH::EPW, LPL = SH::LPL;
    constexpr int NE = DIM + (RAT ? 1 : 0);      // entries of f: (value,) d/dxi_0, ..
    constexpr int NC = NE * (NE + 1) / 2;        // stored coefficients per Gauss point
    constexpr int NT = NC + 1;                   // + load density
    constexpr int WAVES = kBlock / 64;
    __shared__ double sh[WAVES][EPW][NLOC][NT];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = lane / NLP, la = lane % NLP;
    const int64_t nelem = P.nelem;
    // 1D factor of entry e in direction k: derivative when e differentiates in k
    auto is_d = [](int e, int k) { return RAT ? e == k + 1 : e == k; };
    for (int64_t blk0 = static_cast<int64_t>(blockIdx.x) * WAVES * EPW; blk0 < nelem;
         blk0 += static_cast<int64_t>(gridDim.x) * WAVES * EPW) {
        const int64_t el = blk0 + wave * EPW + slot;
        const bool live = el < nelem;
        int gi = 0, ek[3] = {0, 0, 0};
        double Bv[LPL][DIM][NQ], Dv[LPL][DIM][NQ];
        double (*T)[NT] = sh[wave][slot];
        if (live) {
            gi = grid_of_qp_w(P, 0, P.ngrid, el * NLOC);
            const Grid& g = P.grids[gi];
            const int64_t rel = el - g.qp_off / NLOC;  // element index in the grid
            int64_t r = rel;
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                ek[k] = static_cast<int>(r % g.E[k]);
                r /= g.E[k];
            }
            const int64_t nqp = g.nqp;
            const int64_t qbase = g.qp_off + ek[0] * NQ + static_cast<int64_t>(g.Q[0]) *
                                      (ek[1] * NQ + (DIM > 2 ? static_cast<int64_t>(g.Q[1]) * ek[2] * NQ : 0));
#pragma unroll
            for (int s = 0; s < LPL; ++s) {
                const int pos = la + 64 * s;
                if (pos < NLOC) {
                    const int dg[3] = {pos % NQ, (pos / NQ) % NQ, DIM > 2 ? pos / (NQ * NQ) : 0};
                    // stage Gauss point pos of the element (off-diagonal coefficients doubled)
                    // storage index: tensor order (2D), element-major (3D)
                    const int64_t lq = DIM == 3 ? g.qp_off + rel * NLOC + pos
                                                : qbase + dg[0] + static_cast<int64_t>(g.Q[0]) * (dg[1] + static_cast<int64_t>(g.Q[1]) * dg[2]);
                    const double* G = P.G64 + g.qp_off * NC + (lq - g.qp_off);
                    int c = 0;
#pragma unroll
                    for (int u = 0; u < NE; ++u)
#pragma unroll
                        for (int v = u; v < NE; ++v, ++c) {
                            const double gv = G[c * nqp];
                            T[pos][c] = u == v ? gv : 2.0 * gv;
                        }
                    T[pos][NC] = P.Fq[lq];
                    // 1D values of local function dg[k] of direction k at the element's points
#pragma unroll
                    for (int k = 0; k < DIM; ++k) {
                        const Tab1D& Tb = P.tabs[g.tab[k]];
#pragma unroll
                        for (int j = 0; j < NQ; ++j) {
                            const int64_t t = static_cast<int64_t>(ek[k] * NQ + j) * NQ + dg[k];
                            Bv[s][k][j] = P.dpool[Tb.oB + t];
                            Dv[s][k][j] = P.dpool[Tb.oD + t];
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            __syncthreads();  // the previous stage's values are in LDS
            double out[LPL][NT];
            if (live) {
#pragma unroll
                for (int s = 0; s < LPL; ++s) {
                    const int pos = la + 64 * s;
                    if (pos < NLOC) {
                        constexpr int st[3] = {1, NQ, NQ * NQ};
                        const int base = pos - ((pos / st[k]) % NQ) * st[k];  // digit k cleared
#pragma unroll
                        for (int c = 0; c < NT; ++c) out[s][c] = 0.0;
#pragma unroll
                        for (int j = 0; j < NQ; ++j) {
                            const double* in = T[base + j * st[k]];
                            const double b = Bv[s][k][j], dv = Dv[s][k][j];
                            const double w[3] = {b * b, b * dv, dv * dv};
                            int c = 0;
#pragma unroll
                            for (int u = 0; u < NE; ++u)
#pragma unroll
                                for (int v = u; v < NE; ++v, ++c) out[s][c] += w[is_d(u, k) + is_d(v, k)] * in[c];
                            out[s][NC] += b * in[NC];
                        }
                    }
                }
            }
            __syncthreads();  // every lane has read this stage's inputs
            if (live) {
#pragma unroll
                for (int s = 0; s < LPL; ++s) {
                    const int pos = la + 64 * s;
                    if (pos < NLOC) {
                        if (k + 1 < DIM) {
#pragma unroll
                            for (int c = 0; c < NT; ++c) T[pos][c] = out[s][c];
                        } else {
                            double dl = 0.0;
#pragma unroll
                            for (int c = 0; c < NC; ++c) dl += out[s][c];
                            P.loc[static_cast<int64_t>(pos) * nelem + el] = dl;
                            P.loc[static_cast<int64_t>(NLOC + pos) * nelem + el] = out[s][NC];
                        }
                    }
                }
            }
        }
        __syncthreads();  // LDS free for the next elements
    }
}

template <int DIM, int PP>
__global__ void __launch_bounds__(kBlock) k_gather(Params P) {
    constexpr int NQ = PP + 1;
    constexpr int NLOC = ElemShape<DIM, PP>::NLOC;
    const int64_t nelem = P.nelem;
    for (int64_t gi = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; gi < P.ndof_total;
         gi += static_cast<int64_t>(gridDim.x) * kBlock) {
        const Grid& g = P.grids[grid_of_dof(P, 0, P.ngrid, gi)];
        int64_t l = gi - g.dof_off;
        int ik[3] = {0, 0, 0}, elo[3] = {0, 0, 0}, ehi[3] = {0, 0, 0}, mk[3] = {1, 1, 1}, lk[3] = {1, 1, 1};
        double pd = 0.0, md[3] = {1.0, 1.0, 1.0}, kd[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            ik[k] = static_cast<int>(l % g.ni[k]);
            l /= g.ni[k];
            const Tab1D& T = P.tabs[g.tab[k]];
            d_elem_range(ik[k], ik[k] + 1, PP, T.m, g.E[k], T.lo, &elo[k], &ehi[k]);
            mk[k] = T.m;
            lk[k] = T.lo;
            kd[k] = P.dpool[T.oKd + ik[k]];
            md[k] = P.dpool[T.oMd + ik[k]];
        }
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            double t = g.fdc[k] * kd[k];
#pragma unroll
            for (int j = 0; j < DIM; ++j)
                if (j != k) t *= md[j];
            pd += t;
        }
        const int64_t e0 = g.qp_off / NLOC;
        double ad = 0.0, bb = 0.0;
        for (int c2 = elo[2]; c2 <= ehi[2]; ++c2) {
            const int a2 = DIM > 2 ? ik[2] + lk[2] - c2 * mk[2] : 0;
            for (int c1 = elo[1]; c1 <= ehi[1]; ++c1) {
                const int a1 = ik[1] + lk[1] - c1 * mk[1];
                const int64_t row = e0 + g.E[0] * (c1 + static_cast<int64_t>(g.E[1]) * c2);
                for (int c0 = elo[0]; c0 <= ehi[0]; ++c0) {
                    const int a = (ik[0] + lk[0] - c0 * mk[0]) + NQ * (a1 + NQ * a2);
                    const int64_t el = row + c0;
                    ad += P.loc[static_cast<int64_t>(a) * nelem + el];
                    bb += P.loc[static_cast<int64_t>(NLOC + a) * nelem + el];
                }
            }
        }
        P.b[gi] = bb;
        P.fdscale[gi] = ad > 0.0 && pd > 0.0 ? sqrt(pd / ad) : 1.0;
    }
}

// log a at the Greville point of every interior unknown (feature of the
// learned preconditioner): xi*_k = (t_{j+1} + ... + t_{j+p}) / p for basis
// j = i_k + 1 of direction k, mapped through F.
template <int KA>
__global__ void __launch_bounds__(kBlock) k_loga(Params P, FieldDev fa, int g0, int g1) {
    const int64_t i0 = P.grids[g0].dof_off;
    const int64_t i1 = P.grids[g1 - 1].dof_off + P.grids[g1 - 1].ndof;
    const int p = P.p, d = P.dim;
    for (int64_t gi = i0 + blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; gi < i1;
         gi += static_cast<int64_t>(gridDim.x) * kBlock) {
        const int lo = grid_of_dof(P, g0, g1, gi);
        const Grid& g = P.grids[lo];
        int64_t l = gi - g.dof_off;
        double xi[3] = {0, 0, 0};
        int ik[3] = {0, 0, 0};
        for (int k = 0; k < d; ++k) {
            ik[k] = static_cast<int>(l % g.ni[k]);
            l /= g.ni[k];
            const Tab1D& T = P.tabs[g.tab[k]];
            const double* kn = P.dpool + T.oKn;
            double s = 0.0;
            for (int m = 1; m <= p; ++m) s += kn[ik[k] + T.lo + m];
            xi[k] = s / p;
        }
        // geometry map F(xi) = sum w P B / sum w B from the coarse geometry
        const int pt = g.patch;
        double Ng[3][kMaxPg + 1];
        int fg[3] = {0, 0, 0}, pgk[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
#pragma unroll
            for (int a = 0; a <= kMaxPg; ++a) Ng[k][a] = a == 0 ? 1.0 : 0.0;
            if (k < d) {
                const Tab1D& T = P.tabs[g.tab[k]];
                const double* gk = P.dpool + T.oGkn;
                pgk[k] = T.pg;
                const int sp = d_find_interval(T.pg, T.ngk, gk, xi[k]);
                d_basis_funs_m<kMaxPg>(T.pg, gk, sp, xi[k], Ng[k], nullptr);
                fg[k] = sp - T.pg;
            }
        }
        double Xh[4] = {0, 0, 0, 0};
        const double* C = P.ctrl + P.ctrl_off[pt];
#pragma unroll
        for (int c = 0; c <= kMaxPg; ++c) {
            if (c > pgk[2]) break;
#pragma unroll
            for (int b = 0; b <= kMaxPg; ++b) {
                if (b > pgk[1]) break;
#pragma unroll
                for (int a = 0; a <= kMaxPg; ++a) {
                    if (a > pgk[0]) break;
                    const int64_t idx = (fg[0] + a) + static_cast<int64_t>(P.gn[pt][0]) *
                                                          ((fg[1] + b) + static_cast<int64_t>(P.gn[pt][1]) * (fg[2] + c));
                    const double B = Ng[0][a] * Ng[1][b] * Ng[2][c];
#pragma unroll
                    for (int t = 0; t < 4; ++t) Xh[t] += C[idx * 4 + t] * B;
                }
            }
        }
        double x[3] = {0, 0, 0};
        for (int k = 0; k < d; ++k) x[k] = Xh[k] / Xh[3];
        P.loga[gi] = fa.kind == IGA_FIELD_QP_SAMPLES ? 0.0 : log(field_eval_k<KA>(field_of_sample(fa, g.sample), d, x));
    }
}

// Physical Gauss points F(xi_q) and weights w_q |det DF(xi_q)| of every grid.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_quad_points(Params P, double* xq, double* wq) {
    constexpr int d = DIM;
    for (int64_t gq = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; gq < P.nqp_total;
         gq += static_cast<int64_t>(gridDim.x) * kBlock) {
        const int gi = grid_of_qp(P, 0, P.ngrid, gq);
        const Grid& g = P.grids[gi];
        const int64_t l = gq - g.qp_off;
        int qk[3];
        qk[0] = static_cast<int>(l % g.Q[0]);
        qk[1] = static_cast<int>((l / g.Q[0]) % g.Q[1]);
        qk[2] = static_cast<int>(l / (static_cast<int64_t>(g.Q[0]) * g.Q[1]));
        double x[3] = {0, 0, 0}, DF[3][3], W, dW[3] = {0, 0, 0};
        geom_at<DIM>(P, g, qk, x, DF, &W, dW);
        for (int k = 0; k < d; ++k) xq[gq * d + k] = x[k];
        if (wq) {
            double w = 1.0;
            for (int k = 0; k < d; ++k) w *= P.dpool[P.tabs[g.tab[k]].oWq + qk[k]];
            const double det = d == 2 ? DF[0][0] * DF[1][1] - DF[0][1] * DF[1][0]
                                      : DF[0][0] * (DF[1][1] * DF[2][2] - DF[1][2] * DF[2][1]) -
                                            DF[0][1] * (DF[1][0] * DF[2][2] - DF[1][2] * DF[2][0]) +
                                            DF[0][2] * (DF[1][0] * DF[2][1] - DF[1][1] * DF[2][0]);
            wq[gq] = w * fabs(det);
        }
    }
}

// Packs the network's FP32 weights w[co][ci][t] into the BF16 layout of the
// solve's convolutions, Wp[co][t][ci] per layer with co rounded up to 16 and
// ci to 8 (zero-filled); one thread per packed element.
__global__ void __launch_bounds__(kBlock) k_nn_pack(Params P) {
    const int ch[4] = {3, P.nn_ch[1], P.nn_ch[2], 1};
    int64_t base_w = 0, base_p = 0;
    for (int l = 0; l < 3; ++l) {
        const int cin = ch[l], cout = ch[l + 1], cip = nn_pad8(cin);
        const int64_t np = nn_packed_layer(cin, cout);
        for (int64_t e = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; e < np;
             e += static_cast<int64_t>(gridDim.x) * kBlock) {
            const int ci = static_cast<int>(e % cip);
            const int t = static_cast<int>((e / cip) % 27);
            const int co = static_cast<int>(e / (static_cast<int64_t>(cip) * 27));
            const float v = (co < cout && ci < cin) ? P.nn[base_w + (static_cast<int64_t>(co) * cin + ci) * 27 + t] : 0.0f;
            reinterpret_cast<__bf16*>(P.nnw_rw)[base_p + e] = static_cast<__bf16>(v);
        }
        base_w += static_cast<int64_t>(cout) * cin * 27 + cout;
        base_p += np;
    }
}

// Clears the assembly error flag.
__global__ void k_clear_flag(int* flag) {
    if (threadIdx.x == 0) *flag = 0;
}

// Reset solver state and vectors of a grid range before a solve; the first
// sweep's active task lists are the launch's task ranges.
__global__ void __launch_bounds__(kBlock) k_solve_init(Params P, int g0, int g1, int64_t i0, int64_t i1,
                                                      int op_b, int op_e, int fd_b, int fd_e) {
    const int64_t N = P.ndof_total;
    for (int64_t i = i0 + blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < i1;
         i += static_cast<int64_t>(gridDim.x) * kBlock) {
        P.x[i] = 0.0;
        P.d[i] = 0.0;
        P.z[i] = 0.0;
        P.p2[i] = 0.0;
        P.p2[N + i] = 0.0;
    }
    for (int t = blockIdx.x * kBlock + threadIdx.x; t < op_e - op_b || t < fd_e - fd_b; t += gridDim.x * kBlock) {
        if (t < op_e - op_b) P.oplist[t] = P.optask[op_b + t];
        if (t < fd_e - fd_b) P.fdlist[t] = P.fdtask[fd_b + t];
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
            s.op64 = 0;
            P.st2[g] = s;
            P.st2[P.ngrid + g] = s;
        }
        if (threadIdx.x == 0) {
            P.bar[kBarDone] = 0u;
            P.bar[kBarCount] = 0u;
            P.bar[kBarNext] = 0u;
        }
        if (threadIdx.x < kBarGroups) P.bar[kBarGroup + kBarStride * threadIdx.x] = 0u;
        if (threadIdx.x == 0) {
            P.bar[kBarOpLen] = static_cast<unsigned>(op_e - op_b);
            P.bar[kBarOpLen + 1] = 0u;
            P.bar[kBarFdLen] = static_cast<unsigned>(fd_e - fd_b);
            P.bar[kBarFdLen + 1] = 0u;
        }
    }
}

// Standalone operator / preconditioner launches (test hooks).  Same LDS
// layout as the solve kernel: context, task descriptions, work arrays.
template <int PP>
__global__ void __launch_bounds__(kBlock) k_apply_op(Params P, int gi, OpIO io) {
    extern __shared__ double lds_all[];
    TaskMeta* M = reinterpret_cast<TaskMeta*>(reinterpret_cast<char*>(lds_all) + kCtxBytes);
    double* lds = reinterpret_cast<double*>(reinterpret_cast<char*>(lds_all) + kSolveLdsHead);
    meta_fill(P, Task{gi, 0}, M);
    OpIO a = io;
    a.part = nullptr;
    for (int t = blockIdx.x; t < M->g.ntile; t += gridDim.x) {
        if (P.dim == 3) op_tile_3d<PP>(P, M->g, M->t[0], M->t[1], M->t[2], t, a, lds);
        else op_tile_2d<PP>(P, M->g, M->t[0], M->t[1], t, a, lds);
    }
}
__global__ void __launch_bounds__(kBlock) k_apply_fd(Params P, int gi, FdIO io, int fwd) {
    extern __shared__ double lds_all[];
    TaskMeta* M = reinterpret_cast<TaskMeta*>(reinterpret_cast<char*>(lds_all) + kCtxBytes);
    double* lds = reinterpret_cast<double*>(reinterpret_cast<char*>(lds_all) + kSolveLdsHead);
    meta_fill(P, Task{gi, 0}, M);
    for (int t = blockIdx.x; t < M->g.nblk; t += gridDim.x) {
        if (io.prec == 0) fd_apply_block<0>(P, *M, t, io, lds, fwd != 0);
        else if (io.prec == 1) fd_apply_block<1>(P, *M, t, io, lds, fwd != 0);
        else fd_apply_block<2>(P, *M, t, io, lds, fwd != 0);
    }
}

// ===========================================================================
// combination / evaluation: u(xi) = sum_c coef_c (sum_j x_j B_j(xi)) / W(xi)
// ===========================================================================
// Cox-de Boor recursion on a uniform open knot vector with simple interior
// knots (t_i = clamp(i - PP, 0, E) / E), in units of one knot span: with
// X = x E and element e (span e + PP) the differences x - t and t - x become
// X minus an integer, and every denominator t_{i+j} - t_i is an integer
// count c of spans (1 <= c <= PP, at least the element itself), so the
// divisions become products with 1 / c.
template <int PP>
__device__ __forceinline__ void uniform_basis(double X, int e, int E, double* N) {
    double left[PP + 1], right[PP + 1];
    N[0] = 1.0;
#pragma unroll
    for (int j = 1; j <= PP; ++j) {
        left[j] = X - static_cast<double>(max(e + 1 - j, 0));
        right[j] = static_cast<double>(min(e + j, E)) - X;
        double saved = 0.0;
#pragma unroll
        for (int r = 0; r < j; ++r) {
            const int c = min(e + r + 1, E) - max(e + 1 - j + r, 0);
            // 1 / c for c in 1..4: 2^-(c/2) for c = 1, 2, 4 (exact), 1/3 by a select
            const double rc = c == 3 ? 1.0 / 3.0 : ldexp(1.0, -(c >> 1));
            const double tmp = N[r] * rc;
            N[r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        N[j] = saved;
    }
}
static_assert(kMaxP <= 4, "uniform_basis holds reciprocals of span counts up to 4");

// Basis functions of degree PP that are nonzero at x in direction k of a
// grid, and the interior index of the first of them.  UNI: the table is
// uniform with simple interior knots (checked by the host for every grid).
template <int PP, bool UNI>
__device__ __forceinline__ int comb_basis(const Params& P, const Tab1D& T, double x, double* N) {
    int e;
    if (UNI || T.uniform) {
        const double X = x * T.E;
        e = static_cast<int>(X);
        e = e > T.E - 1 ? T.E - 1 : e;
        if (UNI || T.m == 1) {
            uniform_basis<PP>(X, e, T.E, N);
            return e - T.lo;
        }
    } else {
        const double* brk = P.dpool + T.oBrk;
        int lo = 0, hi = T.E;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (x < brk[mid]) hi = mid;
            else lo = mid;
        }
        e = lo;
    }
    d_basis_funs_m<PP>(PP, P.dpool + T.oKn, PP + e * T.m, x, N, nullptr);
    return e * T.m - T.lo;
}

// u(xi) = sum over the grids g0..g1 of the point's patch of c_g u_g(xi)
// (c_g = 1 without use_coef), one thread per point; on a rational patch the
// sum of the B-spline parts is divided once by the weight W(xi).  The basis
// values of a direction are kept while consecutive grids share its table;
// functions outside a grid's interior set get weight zero and a clamped
// index, so the coefficient gathers run without branches.
template <int PP, int DIM, bool UNI>
__global__ void __launch_bounds__(kBlock) k_combine(Params P, const double* xi, const int* patch, int64_t n,
                                                   double* u, int g0, int g1, int use_coef) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock) {
        double xv[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const double t = xi[i * DIM + k];
            xv[k] = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
        }
        const int pt = patch ? patch[i] : 0;
        // weight function W(xi) of the geometry
        double W = 1.0;
        if (P.rational[pt]) {
            double Ng[3][kMaxPg + 1];
            int fg[3] = {0, 0, 0};
            int pgk[3] = {0, 0, 0};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
#pragma unroll
                for (int a = 0; a <= kMaxPg; ++a) Ng[k][a] = a == 0 ? 1.0 : 0.0;
                if (k < DIM) {
                    int gp = g0;  // a grid of the point's patch (its tables hold the patch geometry)
                    while (gp < g1 - 1 && P.grids[gp].patch != pt) ++gp;
                    const Tab1D& T = P.tabs[P.grids[gp].tab[k]];
                    const double* gk = P.dpool + T.oGkn;
                    pgk[k] = T.pg;
                    const int s = d_find_interval(T.pg, T.ngk, gk, xv[k]);
                    d_basis_funs_m<kMaxPg>(T.pg, gk, s, xv[k], Ng[k], nullptr);
                    fg[k] = s - T.pg;
                }
            }
            W = 0.0;
            const double* C = P.ctrl + P.ctrl_off[pt];
#pragma unroll
            for (int c = 0; c <= kMaxPg; ++c) {
                if (c > pgk[2]) break;
#pragma unroll
                for (int b = 0; b <= kMaxPg; ++b) {
                    if (b > pgk[1]) break;
#pragma unroll
                    for (int a = 0; a <= kMaxPg; ++a) {
                        if (a > pgk[0]) break;
                        const int64_t idx = (fg[0] + a) + static_cast<int64_t>(P.gn[pt][0]) *
                                                              ((fg[1] + b) + static_cast<int64_t>(P.gn[pt][1]) * (fg[2] + c));
                        W += C[idx * 4 + 3] * Ng[0][a] * Ng[1][b] * Ng[2][c];
                    }
                }
            }
        }
        double acc = 0.0;
        double N[DIM][PP + 1];
        int ix[DIM][PP + 1];
        int ctab[DIM];
        double Nf[DIM][PP + 1];  // unmasked values and first basis index (Dirichlet lift, 2D)
        int Jf[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) ctab[k] = -1;
        for (int gi = g0; gi < g1; ++gi) {
            const Grid& g = P.grids[gi];
            // the basis update depends on the grid only (uniform over the
            // wavefront); the patch test comes after it
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                if (g.tab[k] == ctab[k]) continue;
                ctab[k] = g.tab[k];
                const int f = comb_basis<PP, UNI>(P, P.tabs[g.tab[k]], xv[k], N[k]);
                const int ni = g.ni[k];
                Jf[k] = f + P.tabs[g.tab[k]].lo;
#pragma unroll
                for (int a = 0; a <= PP; ++a) {
                    const int j = f + a;
                    const bool in = j >= 0 && j < ni;
                    Nf[k][a] = N[k][a];
                    N[k][a] = in ? N[k][a] : 0.0;
                    ix[k][a] = j < 0 ? 0 : (j >= ni ? ni - 1 : j);
                }
            }
            if (g.patch != pt) continue;
            const double* X = P.x + g.dof_off;
            double v = 0.0;
#pragma unroll
            for (int c = 0; c <= (DIM > 2 ? PP : 0); ++c) {
#pragma unroll
                for (int b = 0; b <= PP; ++b) {
                    const int64_t row = static_cast<int64_t>(g.ni[0]) *
                                        (ix[1][b] + (DIM > 2 ? static_cast<int64_t>(g.ni[1]) * ix[2][c] : 0));
                    const double* Xr = X + row;
                    double vb = 0.0;
#pragma unroll
                    for (int a = 0; a <= PP; ++a) vb += Xr[ix[0][a]] * N[0][a];
                    v += vb * N[1][b] * (DIM > 2 ? N[2][c] : 1.0);
                }
            }
            if (DIM == 2 && P.lift) {
                // the lift's boundary coefficients (zero at the unknowns)
                const double* Lg = P.lift + g.lift_off;
#pragma unroll
                for (int b = 0; b <= PP; ++b) {
                    double vb = 0.0;
#pragma unroll
                    for (int a = 0; a <= PP; ++a) vb += Lg[(Jf[0] + a) + static_cast<int64_t>(g.nb[0]) * (Jf[DIM - 1] + b)] * Nf[0][a];
                    v += vb * Nf[DIM - 1][b];
                }
            }
            acc += use_coef ? g.ccoef * v : v;
        }
        u[i] = acc / W;
    }
}

// Geometry of patch pt at parametric point xv from the coarse NURBS (tables
// T[k] of any grid of the patch): weight W, its parametric gradient dW and
// the Jacobian DF of F = sum w P B / W (quotient rule), FP64.
template <int DIM>
__device__ __forceinline__ void point_geom(const Params& P, const Tab1D* const* T, int pt, const double* xv,
                                           double* W, double* dW, double DF[DIM][DIM], double* xo = nullptr) {
    double Ng[3][kMaxPg + 1], dNg[3][kMaxPg + 1];
    int fg[3] = {0, 0, 0}, pgk[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
        for (int a = 0; a <= kMaxPg; ++a) {
            Ng[k][a] = a == 0 ? 1.0 : 0.0;
            dNg[k][a] = 0.0;
        }
        if (k < DIM) {
            const double* gk = P.dpool + T[k]->oGkn;
            pgk[k] = T[k]->pg;
            const int s = d_find_interval(T[k]->pg, T[k]->ngk, gk, xv[k]);
            d_basis_funs_m<kMaxPg>(T[k]->pg, gk, s, xv[k], Ng[k], dNg[k]);
            fg[k] = s - T[k]->pg;
        }
    }
    double Xh[4] = {0, 0, 0, 0}, dXh[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    const double* C = P.ctrl + P.ctrl_off[pt];
#pragma unroll
    for (int c = 0; c <= kMaxPg; ++c) {
        if (c > pgk[2]) break;
#pragma unroll
        for (int b = 0; b <= kMaxPg; ++b) {
            if (b > pgk[1]) break;
#pragma unroll
            for (int a = 0; a <= kMaxPg; ++a) {
                if (a > pgk[0]) break;
                const int64_t idx = (fg[0] + a) + static_cast<int64_t>(P.gn[pt][0]) *
                                                      ((fg[1] + b) + static_cast<int64_t>(P.gn[pt][1]) * (fg[2] + c));
                const double v[3] = {Ng[0][a], Ng[1][b], Ng[2][c]};
                const double dv[3] = {dNg[0][a], dNg[1][b], dNg[2][c]};
                const double B = v[0] * v[1] * v[2];
                const double dB[3] = {dv[0] * v[1] * v[2], v[0] * dv[1] * v[2], v[0] * v[1] * dv[2]};
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const double cp = C[idx * 4 + t];
                    Xh[t] += cp * B;
#pragma unroll
                    for (int k = 0; k < DIM; ++k) dXh[k][t] += cp * dB[k];
                }
            }
        }
    }
    *W = Xh[3];
#pragma unroll
    for (int k = 0; k < DIM; ++k) dW[k] = dXh[k][3];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        const double x = Xh[c] / Xh[3];
        if (xo) xo[c] = x;
#pragma unroll
        for (int k = 0; k < DIM; ++k) DF[c][k] = (dXh[k][c] - x * dXh[k][3]) / Xh[3];
    }
}

// ===========================================================================
// Dirichlet lift (2D, polynomial patches): the boundary coefficients of
// u_D = sum over the Dirichlet functions of c_j phi_j.  The two end functions
// of a Dirichlet side interpolate g at the patch corners (open knots); the
// others are the L2 projection of g on the side's trace space with the ends
// fixed: M c = (g, B) - M_corner c_corner with the side's 1D mass matrix in
// arc length, one workgroup per (grid, side), the band of M assembled row by
// row in LDS (each thread one function, over the elements of its support),
// then a banded Cholesky solve by one thread.  Values go to the grid's full
// coefficient array (direction 1 fastest); the others stay 0.
// ===========================================================================
template <int PP>
__global__ void __launch_bounds__(kBlock) k_lift_edges(Params P, FieldDev fg) {
    extern __shared__ double lsh[];
    const int gi = blockIdx.x, sd = blockIdx.y;
    const Grid& g = P.grids[gi];
    const int k = sd / 2, t = 1 - k;  // fixed and running directions
    const Tab1D& Tk = P.tabs[g.tab[k]];
    const Tab1D& Tt = P.tabs[g.tab[t]];
    const Tab1D* Tg[2] = {P.tabs + g.tab[0], P.tabs + g.tab[1]};
    if (sd == 0 && threadIdx.x == 0) {
        // a vertex between two interfaces of this patch that carries Dirichlet
        // data elsewhere (fixed unknown): its value interpolates g as well
        for (int e = 0; e < 4; ++e) {
            if (g.pin[e] < 0) continue;
            double xi[2] = {static_cast<double>(e & 1), static_cast<double>(e >> 1)}, x[2], W, dW[2], DF[2][2];
            point_geom<2>(P, Tg, g.patch, xi, &W, dW, DF, x);
            const int64_t idx = ((e & 1) ? g.nb[0] - 1 : 0) + static_cast<int64_t>(g.nb[0]) * ((e >> 1) ? g.nb[1] - 1 : 0);
            P.lift_rw[g.lift_off + idx] = field_eval(field_of_sample(fg, g.sample), 2, x);
        }
    }
    const int hik = Tk.nb - Tk.lo - Tk.ni;
    if ((sd % 2 == 0 && Tk.lo == 0) || (sd % 2 == 1 && hik == 0)) return;  // interface side
    const int n = Tt.nb, m = n - 2;
    const int jfix = (sd % 2) ? Tk.nb - 1 : 0;
    double* Lb = lsh;                            // [m][PP + 1]: M[i][i - d]
    double* rhs = lsh + static_cast<size_t>(m) * (PP + 1);
    double* cv = rhs + m;                        // corner values
    if (threadIdx.x < 2) {
        double xi[2], x[2], W, dW[2], DF[2][2];
        xi[k] = static_cast<double>(sd % 2);
        xi[t] = static_cast<double>(threadIdx.x);
        point_geom<2>(P, Tg, g.patch, xi, &W, dW, DF, x);
        cv[threadIdx.x] = field_eval(field_of_sample(fg, g.sample), 2, x);
    }
    __syncthreads();
    const int mult = Tt.m, nq = P.nq;
    for (int i = 1 + threadIdx.x; i <= m; i += kBlock) {
        double row[2 * PP + 1], b = 0.0;
#pragma unroll
        for (int j = 0; j <= 2 * PP; ++j) row[j] = 0.0;
        // elements e whose functions e mult .. e mult + p include i
        const int e0 = max(0, (i - PP + mult - 1) / mult), e1 = min(Tt.E - 1, i / mult);
        for (int e = e0; e <= e1; ++e) {
            const int a = i - e * mult;
            for (int q = 0; q < nq; ++q) {
                const int qq = e * nq + q;
                const double* Nq = P.dpool + Tt.oB + static_cast<int64_t>(qq) * (PP + 1);
                double xi[2], x[2], W, dW[2], DF[2][2];
                xi[k] = static_cast<double>(sd % 2);
                xi[t] = P.dpool[Tt.oXq + qq];
                point_geom<2>(P, Tg, g.patch, xi, &W, dW, DF, x);
                const double ds = sqrt(DF[0][t] * DF[0][t] + DF[1][t] * DF[1][t]) * P.dpool[Tt.oWq + qq];
                const double gv = field_eval(field_of_sample(fg, g.sample), 2, x);
                b += gv * Nq[a] * ds;
#pragma unroll
                for (int c = 0; c <= PP; ++c) {
                    const int j = e * mult + c;
                    row[j - i + PP] += Nq[a] * Nq[c] * ds;
                }
            }
        }
        // fixed end values move to the right-hand side
#pragma unroll
        for (int c = 0; c <= 2 * PP; ++c) {
            const int j = i - PP + c;
            if (j == 0) b -= row[c] * cv[0];
            if (j == n - 1) b -= row[c] * cv[1];
        }
        rhs[i - 1] = b;
#pragma unroll
        for (int dd = 0; dd <= PP; ++dd) Lb[static_cast<size_t>(i - 1) * (PP + 1) + dd] = row[PP - dd];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // banded Cholesky M = L L^T in place (L[i][i - d] at Lb[i][d]), then
        // the two triangular solves
        for (int i = 0; i < m; ++i) {
            for (int dd = min(PP, i); dd >= 1; --dd) {
                const int j = i - dd;
                double v = Lb[i * (PP + 1) + dd];
                for (int kk = 1; kk <= PP - dd && j - kk >= 0; ++kk)
                    v -= Lb[i * (PP + 1) + dd + kk] * Lb[j * (PP + 1) + kk];
                Lb[i * (PP + 1) + dd] = v / Lb[j * (PP + 1)];
            }
            double v = Lb[i * (PP + 1)];
            for (int dd = 1; dd <= min(PP, i); ++dd) v -= Lb[i * (PP + 1) + dd] * Lb[i * (PP + 1) + dd];
            Lb[i * (PP + 1)] = sqrt(v);
        }
        for (int i = 0; i < m; ++i) {
            double v = rhs[i];
            for (int dd = 1; dd <= min(PP, i); ++dd) v -= Lb[i * (PP + 1) + dd] * rhs[i - dd];
            rhs[i] = v / Lb[i * (PP + 1)];
        }
        for (int i = m - 1; i >= 0; --i) {
            double v = rhs[i];
            for (int dd = 1; dd <= PP && i + dd < m; ++dd) v -= Lb[(i + dd) * (PP + 1) + dd] * rhs[i + dd];
            rhs[i] = v / Lb[i * (PP + 1)];
        }
    }
    __syncthreads();
    double* L = P.lift_rw + g.lift_off;
    for (int j = threadIdx.x; j < n; j += kBlock) {
        const double v = j == 0 ? cv[0] : (j == n - 1 ? cv[1] : rhs[j - 1]);
        const int64_t idx = k == 0 ? jfix + static_cast<int64_t>(Tk.nb) * j : j + static_cast<int64_t>(Tt.nb) * jfix;
        L[idx] = v;
    }
}

// Load vector correction of the lift, -a(u_D, phi_a) for every local
// function a of every element (2D, polynomial map): per Gauss point the
// parametric gradient of u_D from the element's (p+1)^2 lift coefficients,
// its flux G grad u_D, and the sum of the flux against grad B_a, added to the
// element-local load sums before the gather.  One thread per element.
template <int PP>
__global__ void __launch_bounds__(kBlock) k_lift_rhs(Params P) {
    constexpr int NQ = PP + 1, NLOC = NQ * NQ;
    for (int64_t el = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; el < P.nelem;
         el += static_cast<int64_t>(gridDim.x) * kBlock) {
        const int gi = grid_of_qp(P, 0, P.ngrid, el * NLOC);
        const Grid& g = P.grids[gi];
        const int64_t le = el - g.qp_off / NLOC;
        const int e0 = static_cast<int>(le % g.E[0]), e1 = static_cast<int>(le / g.E[0]);
        const Tab1D& T0 = P.tabs[g.tab[0]];
        const Tab1D& T1 = P.tabs[g.tab[1]];
        const double* L = P.lift + g.lift_off;
        double c[NQ][NQ];
        bool any = false;
#pragma unroll
        for (int b = 0; b < NQ; ++b)
#pragma unroll
            for (int a = 0; a < NQ; ++a) {
                c[a][b] = L[(e0 * T0.m + a) + static_cast<int64_t>(T0.nb) * (e1 * T1.m + b)];
                any = any || c[a][b] != 0.0;
            }
        if (!any) continue;
        double out[NQ][NQ];
#pragma unroll
        for (int b = 0; b < NQ; ++b)
#pragma unroll
            for (int a = 0; a < NQ; ++a) out[a][b] = 0.0;
        for (int q1 = 0; q1 < NQ; ++q1)
            for (int q0 = 0; q0 < NQ; ++q0) {
                const int Q0 = e0 * NQ + q0, Q1 = e1 * NQ + q1;
                const double* B0 = P.dpool + T0.oB + static_cast<int64_t>(Q0) * NQ;
                const double* D0 = P.dpool + T0.oD + static_cast<int64_t>(Q0) * NQ;
                const double* B1 = P.dpool + T1.oB + static_cast<int64_t>(Q1) * NQ;
                const double* D1 = P.dpool + T1.oD + static_cast<int64_t>(Q1) * NQ;
                double u0 = 0.0, u1 = 0.0;  // parametric gradient of u_D
#pragma unroll
                for (int b = 0; b < NQ; ++b)
#pragma unroll
                    for (int a = 0; a < NQ; ++a) {
                        u0 += c[a][b] * D0[a] * B1[b];
                        u1 += c[a][b] * B0[a] * D1[b];
                    }
                const int64_t qi = g.qp_off + static_cast<int64_t>(Q1) * g.Q[0] + Q0;
                const int64_t nqp = g.nqp;
                const double* G = P.G64 + g.qp_off * P.ncompG + (qi - g.qp_off);
                const double f0 = G[0] * u0 + G[nqp] * u1, f1 = G[nqp] * u0 + G[2 * nqp] * u1;
#pragma unroll
                for (int b = 0; b < NQ; ++b)
#pragma unroll
                    for (int a = 0; a < NQ; ++a) out[a][b] -= f0 * D0[a] * B1[b] + f1 * B0[a] * D1[b];
            }
        // element-local load sums: loc[NLOC + a][element]
#pragma unroll
        for (int b = 0; b < NQ; ++b)
#pragma unroll
            for (int a = 0; a < NQ; ++a) P.loc[static_cast<int64_t>(NLOC + a + NQ * b) * P.nelem + el] += out[a][b];
    }
}

// Full coefficient arrays of grids g0..g1 (every basis function, direction 1
// fastest, one grid after another): the lift's boundary values plus the
// unknowns at their basis functions.
__global__ void __launch_bounds__(kBlock) k_full_coeffs(Params P, int g0, int g1, double* out) {
    int64_t base = 0;
    for (int gi = g0; gi < g1; ++gi) {
        const Grid& g = P.grids[gi];
        const int n0 = g.nb[0], n1 = g.nb[1], n2 = g.nb[2];
        const int lo0 = P.tabs[g.tab[0]].lo, lo1 = P.tabs[g.tab[1]].lo;
        const int lo2 = P.dim > 2 ? P.tabs[g.tab[2]].lo : 0;
        const int64_t nt = static_cast<int64_t>(n0) * n1 * n2;
        for (int64_t j = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; j < nt;
             j += static_cast<int64_t>(gridDim.x) * kBlock) {
            const int j0 = static_cast<int>(j % n0), j1 = static_cast<int>((j / n0) % n1),
                      j2 = static_cast<int>(j / (static_cast<int64_t>(n0) * n1));
            const int i0 = j0 - lo0, i1 = j1 - lo1, i2 = j2 - lo2;
            double v = (P.lift && P.dim == 2) ? P.lift[g.lift_off + j] : 0.0;
            if (i0 >= 0 && i0 < g.ni[0] && i1 >= 0 && i1 < g.ni[1] && i2 >= 0 && i2 < g.ni[2])
                v += P.x[g.dof_off + i0 + static_cast<int64_t>(g.ni[0]) * (i1 + static_cast<int64_t>(g.ni[1]) * i2)];
            out[base + j] = v;
        }
        base += nt;
    }
}

// Detail norms: workgroup b forms Delta_b(x_i) = sum_z (-1)^|z| u_(b-z)(x_i)
// from the grid values vals[grid][i] (the table nb[b][z] names grid b - z,
// -1 for a negative level) and sums w_i Delta_b(x_i)^2 over the points in a
// fixed order (thread-strided partial sums, then the workgroup tree).
__global__ void __launch_bounds__(kBlock) k_detail_norms(const double* vals, const double* wq, int64_t n,
                                                         const int* nb, int nz, double* out) {
    __shared__ double red[kWaves];
    const int b = blockIdx.x;
    int g[8];
    double sg[8];
    for (int z = 0; z < 8; ++z) {
        g[z] = z < nz ? nb[b * 8 + z] : -1;
        sg[z] = (__popc(z) & 1) ? -1.0 : 1.0;
    }
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        double dv = 0.0;
        for (int z = 0; z < nz; ++z)
            if (g[z] >= 0) dv += sg[z] * vals[static_cast<int64_t>(g[z]) * n + i];
        acc += wq[i] * dv * dv;
    }
    const double t = wg_sum(acc, red);
    if (threadIdx.x == 0) out[b] = sqrt(t);
}

// Clears the lift arrays (a kernel, so that the assembly can be captured).
__global__ void __launch_bounds__(kBlock) k_zero(double* v, int64_t n) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock)
        v[i] = 0.0;
}

// grad_i = grad sum over the grids g0..g1 of the point's patch of c_g u_g at
// xi_i (c_g = 1 without use_coef), physical coordinates: with v the sum of
// the B-spline parts (discrete basis B / W), grad_xi (v / W) =
// (grad_xi v - (v / W) grad_xi W) / W and grad_x = DF^-T grad_xi, FP64.  One
// thread per point; general Cox-de Boor values and derivatives (any knots).
template <int PP, int DIM>
__global__ void __launch_bounds__(kBlock) k_combine_grad(Params P, const double* xi, const int* patch, int64_t n,
                                                        double* grad, int g0, int g1, int use_coef) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock) {
        double xv[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const double t = xi[i * DIM + k];
            xv[k] = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
        }
        const int pt = patch ? patch[i] : 0;
        int gp = g0;  // a grid of the point's patch (its tables hold the patch geometry)
        while (gp < g1 - 1 && P.grids[gp].patch != pt) ++gp;
        const Tab1D* Tg[3] = {nullptr, nullptr, nullptr};
#pragma unroll
        for (int k = 0; k < DIM; ++k) Tg[k] = P.tabs + P.grids[gp].tab[k];
        double W, dW[DIM], DF[DIM][DIM];
        point_geom<DIM>(P, Tg, pt, xv, &W, dW, DF);
        double acc = 0.0, accd[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) accd[k] = 0.0;
        for (int gi = g0; gi < g1; ++gi) {
            const Grid& g = P.grids[gi];
            if (g.patch != pt) continue;
            double N[DIM][PP + 1], dN[DIM][PP + 1], Nf[DIM][PP + 1], dNf[DIM][PP + 1];
            int ix[DIM][PP + 1], Jf[DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                const Tab1D& T = P.tabs[g.tab[k]];
                const double* brk = P.dpool + T.oBrk;
                int lo = 0, hi = T.E;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (xv[k] < brk[mid]) hi = mid;
                    else lo = mid;
                }
                d_basis_funs_m<PP>(PP, P.dpool + T.oKn, PP + lo * T.m, xv[k], N[k], dN[k]);
                const int f = lo * T.m - T.lo;  // unknown index of the first nonzero function
                Jf[k] = lo * T.m;
#pragma unroll
                for (int a = 0; a <= PP; ++a) {
                    Nf[k][a] = N[k][a];
                    dNf[k][a] = dN[k][a];
                }
#pragma unroll
                for (int a = 0; a <= PP; ++a) {
                    const int j = f + a;
                    const bool in = j >= 0 && j < g.ni[k];
                    N[k][a] = in ? N[k][a] : 0.0;
                    dN[k][a] = in ? dN[k][a] : 0.0;
                    ix[k][a] = j < 0 ? 0 : (j >= g.ni[k] ? g.ni[k] - 1 : j);
                }
            }
            const double* X = P.x + g.dof_off;
            double v = 0.0, dv[DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) dv[k] = 0.0;
#pragma unroll
            for (int c = 0; c <= (DIM > 2 ? PP : 0); ++c) {
#pragma unroll
                for (int b = 0; b <= PP; ++b) {
                    const int64_t row = static_cast<int64_t>(g.ni[0]) *
                                        (ix[1][b] + (DIM > 2 ? static_cast<int64_t>(g.ni[1]) * ix[2][c] : 0));
                    const double* Xr = X + row;
                    double vb = 0.0, db = 0.0;
#pragma unroll
                    for (int a = 0; a <= PP; ++a) {
                        vb += Xr[ix[0][a]] * N[0][a];
                        db += Xr[ix[0][a]] * dN[0][a];
                    }
                    const double n2 = DIM > 2 ? N[2][c] : 1.0;
                    v += vb * N[1][b] * n2;
                    dv[0] += db * N[1][b] * n2;
                    dv[1] += vb * dN[1][b] * n2;
                    if (DIM > 2) dv[DIM - 1] += vb * N[1][b] * dN[2][c];
                }
            }
            if (DIM == 2 && P.lift) {
                // the lift's boundary coefficients (zero at the unknowns)
                const double* Lg = P.lift + g.lift_off;
#pragma unroll
                for (int b = 0; b <= PP; ++b)
#pragma unroll
                    for (int a = 0; a <= PP; ++a) {
                        const double cl = Lg[(Jf[0] + a) + static_cast<int64_t>(g.nb[0]) * (Jf[DIM - 1] + b)];
                        v += cl * Nf[0][a] * Nf[DIM - 1][b];
                        dv[0] += cl * dNf[0][a] * Nf[DIM - 1][b];
                        dv[DIM - 1] += cl * Nf[0][a] * dNf[DIM - 1][b];
                    }
            }
            const double cf = use_coef ? g.ccoef : 1.0;
            acc += cf * v;
#pragma unroll
            for (int k = 0; k < DIM; ++k) accd[k] += cf * dv[k];
        }
        const double u = acc / W;
        double gh[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) gh[k] = (accd[k] - u * dW[k]) / W;
        // grad_x = DF^-T gh: solve DF^T y = gh by the adjugate
        double y[DIM];
        if constexpr (DIM == 2) {
            const double det = DF[0][0] * DF[1][1] - DF[0][1] * DF[1][0];
            // DF^-T = [[DF11, -DF10], [-DF01, DF00]] / det
            y[0] = (DF[1][1] * gh[0] - DF[1][0] * gh[1]) / det;
            y[1] = (-DF[0][1] * gh[0] + DF[0][0] * gh[1]) / det;
        } else {
            double cof[3][3];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int r1 = (r + 1) % 3, r2 = (r + 2) % 3, c1 = (c + 1) % 3, c2 = (c + 2) % 3;
                    cof[r][c] = DF[r1][c1] * DF[r2][c2] - DF[r1][c2] * DF[r2][c1];
                }
            const double det = DF[0][0] * cof[0][0] + DF[0][1] * cof[0][1] + DF[0][2] * cof[0][2];
            // (DF^-1)[k][c] = cof[c][k] / det, so (DF^-T gh)_c = sum_k cof[c][k] gh_k / det
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                double t = 0.0;
#pragma unroll
                for (int k = 0; k < DIM; ++k) t += cof[c][k] * gh[k];
                y[c] = t / det;
            }
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c) grad[i * DIM + c] = y[c];
    }
}

inline int blocks_for_n(int64_t n) {
    const int64_t b = (n + kBlock - 1) / kBlock;
    return static_cast<int>(std::min<int64_t>(std::max<int64_t>(b, 1), 65535));
}

// Assembly kernels specialised for the field kinds of the workloads
// (coefficient: constant, sin-cos, 3D grid; load: constant, sine product,
// annulus right-hand side), the run-time switch for any other combination.
template <int KA, int DIM>
hipError_t launch_assemble_f(int kf, dim3 grid, hipStream_t st, const Params& K, const FieldDev& fa,
                             const FieldDev& ff, int ng, int* err) {
    switch (kf) {
        case IGA_FIELD_CONST: hipLaunchKernelGGL((k_assemble<KA, IGA_FIELD_CONST, DIM>), grid, dim3(kBlock), 0, st, K, fa, ff, 0, ng, err); break;
        case IGA_FIELD_SINPROD: hipLaunchKernelGGL((k_assemble<KA, IGA_FIELD_SINPROD, DIM>), grid, dim3(kBlock), 0, st, K, fa, ff, 0, ng, err); break;
        case IGA_FIELD_ANNULUS_RHS: hipLaunchKernelGGL((k_assemble<KA, IGA_FIELD_ANNULUS_RHS, DIM>), grid, dim3(kBlock), 0, st, K, fa, ff, 0, ng, err); break;
        default: hipLaunchKernelGGL((k_assemble<KA, -1, DIM>), grid, dim3(kBlock), 0, st, K, fa, ff, 0, ng, err); break;
    }
    return hipGetLastError();
}
template <int DIM>
hipError_t launch_assemble_d(int ka, int kf, dim3 grid, hipStream_t st, const Params& K, const FieldDev& fa,
                             const FieldDev& ff, int ng, int* err) {
    switch (ka) {
        case IGA_FIELD_CONST: return launch_assemble_f<IGA_FIELD_CONST, DIM>(kf, grid, st, K, fa, ff, ng, err);
        case IGA_FIELD_SINCOS: return launch_assemble_f<IGA_FIELD_SINCOS, DIM>(kf, grid, st, K, fa, ff, ng, err);
        case IGA_FIELD_GRID3D: return launch_assemble_f<IGA_FIELD_GRID3D, DIM>(kf, grid, st, K, fa, ff, ng, err);
        default: return launch_assemble_f<-1, DIM>(kf, grid, st, K, fa, ff, ng, err);
    }
}
hipError_t launch_assemble(int dim, int ka, int kf, dim3 grid, hipStream_t st, const Params& K, const FieldDev& fa,
                           const FieldDev& ff, int ng, int* err) {
    return dim == 2 ? launch_assemble_d<2>(ka, kf, grid, st, K, fa, ff, ng, err)
                    : launch_assemble_d<3>(ka, kf, grid, st, K, fa, ff, ng, err);
}
// Element-local sums and their gather (load vector, preconditioner scaling),
// specialised by dimension, degree and the rational form of the coefficients.
template <int DIM, int PP>
void launch_loadiag_p(bool rat, bool lift, hipStream_t st, const Params& K, int dblocks) {
    constexpr int64_t epb = (kBlock / 64) * ElemShape<DIM, PP>::EPW;  // elements per workgroup
    const int eblocks = static_cast<int>(std::min<int64_t>(std::max<int64_t>((K.nelem + epb - 1) / epb, 1), 65535));
    if (rat) hipLaunchKernelGGL((k_elemloc<DIM, PP, true>), dim3(eblocks), dim3(kBlock), 0, st, K);
    else hipLaunchKernelGGL((k_elemloc<DIM, PP, false>), dim3(eblocks), dim3(kBlock), 0, st, K);
    if constexpr (DIM == 2)
        if (lift) hipLaunchKernelGGL((k_lift_rhs<PP>), dim3(blocks_for_n(K.nelem)), dim3(kBlock), 0, st, K);
    hipLaunchKernelGGL((k_gather<DIM, PP>), dim3(dblocks), dim3(kBlock), 0, st, K);
}
template <int DIM>
void launch_loadiag_d(int p, bool rat, bool lift, hipStream_t st, const Params& K, int dblocks) {
    switch (p) {
        case 1: launch_loadiag_p<DIM, 1>(rat, lift, st, K, dblocks); break;
        case 2: launch_loadiag_p<DIM, 2>(rat, lift, st, K, dblocks); break;
        case 3: launch_loadiag_p<DIM, 3>(rat, lift, st, K, dblocks); break;
        default: launch_loadiag_p<DIM, 4>(rat, lift, st, K, dblocks); break;
    }
}
// element-local sums, the lift's load correction (when lift), the gather
hipError_t launch_loadiag(int dim, int p, bool rat, bool lift, hipStream_t st, const Params& K, int dblocks) {
    if (dim == 2) launch_loadiag_d<2>(p, rat, lift, st, K, dblocks);
    else launch_loadiag_d<3>(p, rat, lift, st, K, dblocks);
    return hipGetLastError();
}
hipError_t launch_lift_edges(int p, dim3 grid, size_t lds, hipStream_t st, const Params& K, const FieldDev& fg) {
    switch (p) {
        case 1: hipLaunchKernelGGL(k_lift_edges<1>, grid, dim3(kBlock), lds, st, K, fg); break;
        case 2: hipLaunchKernelGGL(k_lift_edges<2>, grid, dim3(kBlock), lds, st, K, fg); break;
        case 3: hipLaunchKernelGGL(k_lift_edges<3>, grid, dim3(kBlock), lds, st, K, fg); break;
        default: hipLaunchKernelGGL(k_lift_edges<4>, grid, dim3(kBlock), lds, st, K, fg); break;
    }
    return hipGetLastError();
}
hipError_t launch_loga(int ka, dim3 grid, hipStream_t st, const Params& K, const FieldDev& fa, int ng) {
    switch (ka) {
        case IGA_FIELD_CONST: hipLaunchKernelGGL((k_loga<IGA_FIELD_CONST>), grid, dim3(kBlock), 0, st, K, fa, 0, ng); break;
        case IGA_FIELD_SINCOS: hipLaunchKernelGGL((k_loga<IGA_FIELD_SINCOS>), grid, dim3(kBlock), 0, st, K, fa, 0, ng); break;
        case IGA_FIELD_GRID3D: hipLaunchKernelGGL((k_loga<IGA_FIELD_GRID3D>), grid, dim3(kBlock), 0, st, K, fa, 0, ng); break;
        default: hipLaunchKernelGGL((k_loga<-1>), grid, dim3(kBlock), 0, st, K, fa, 0, ng); break;
    }
    return hipGetLastError();
}

template <int PP>
void launch_combine_p(int dim, bool uni, int blocks, hipStream_t st, const Params& K, const double* xi,
                      const int* patch, int64_t n, double* u, int g0, int g1, int use_coef) {
    const dim3 grid(blocks), block(kBlock);
    if (dim == 2 && uni) hipLaunchKernelGGL((k_combine<PP, 2, true>), grid, block, 0, st, K, xi, patch, n, u, g0, g1, use_coef);
    else if (dim == 2) hipLaunchKernelGGL((k_combine<PP, 2, false>), grid, block, 0, st, K, xi, patch, n, u, g0, g1, use_coef);
    else if (uni) hipLaunchKernelGGL((k_combine<PP, 3, true>), grid, block, 0, st, K, xi, patch, n, u, g0, g1, use_coef);
    else hipLaunchKernelGGL((k_combine<PP, 3, false>), grid, block, 0, st, K, xi, patch, n, u, g0, g1, use_coef);
}
hipError_t launch_combine_grad(int dim, int p, int blocks, hipStream_t st, const Params& K, const double* xi,
                               const int* patch, int64_t n, double* grad, int g0, int g1, int use_coef) {
    const dim3 grid(blocks), block(kBlock);
#define IGASG_CG(PP)                                                                                              \
    if (dim == 2) hipLaunchKernelGGL((k_combine_grad<PP, 2>), grid, block, 0, st, K, xi, patch, n, grad, g0, g1, use_coef); \
    else hipLaunchKernelGGL((k_combine_grad<PP, 3>), grid, block, 0, st, K, xi, patch, n, grad, g0, g1, use_coef);
    switch (p) {
        case 1: IGASG_CG(1) break;
        case 2: IGASG_CG(2) break;
        case 3: IGASG_CG(3) break;
        default: IGASG_CG(4) break;
    }
#undef IGASG_CG
    return hipGetLastError();
}
hipError_t launch_combine(int dim, int p, bool uni, int blocks, hipStream_t st, const Params& K, const double* xi,
                          const int* patch, int64_t n, double* u, int g0, int g1, int use_coef) {
    switch (p) {
        case 1: launch_combine_p<1>(dim, uni, blocks, st, K, xi, patch, n, u, g0, g1, use_coef); break;
        case 2: launch_combine_p<2>(dim, uni, blocks, st, K, xi, patch, n, u, g0, g1, use_coef); break;
        case 3: launch_combine_p<3>(dim, uni, blocks, st, K, xi, patch, n, u, g0, g1, use_coef); break;
        default: launch_combine_p<4>(dim, uni, blocks, st, K, xi, patch, n, u, g0, g1, use_coef); break;
    }
    return hipGetLastError();
}

Params make_params(iga_sg_plan_s* P, bool lowp_fd) {
    Params K;
    std::memset(&K, 0, sizeof(K));
    char* base = static_cast<char*>(P->ws);
    const Layout& L = P->lay;
    K.tabs = reinterpret_cast<const Tab1D*>(base + L.tabs);
    K.grids = reinterpret_cast<const Grid*>(base + (lowp_fd ? L.grids_lp : L.grids));
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
    K.lift_rw = P->nlift > 0 ? reinterpret_cast<double*>(base + L.lift) : nullptr;
    K.lift = P->lifted ? K.lift_rw : nullptr;
    K.mp = P->patches.size() > 1 ? 1 : 0;
    K.dim = P->dim;
    K.p = P->p;
    K.nq = P->nq;
    K.ncompG = P->ncompG;
    K.ngrid = static_cast<int>(P->grids.size());
    K.ngrid1 = K.ngrid / P->nsamples;
    K.nqp1 = P->nqp_total / P->nsamples;
    K.ndof1 = P->ndof_total / P->nsamples;
    K.nop = static_cast<int>(P->optask.size());
    K.nfd = static_cast<int>((lowp_fd ? P->fdtask_lp : P->fdtask).size());
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
    K.part_stride = static_cast<int64_t>(std::max(P->optask.size(), std::max(P->fdtask.size(), P->fdtask_lp.size())));
    K.optask = reinterpret_cast<const Task*>(base + L.optask);
    K.fdtask = reinterpret_cast<const Task*>(base + (lowp_fd ? L.fdtask_lp : L.fdtask));
    K.bar = reinterpret_cast<unsigned*>(base + L.bar);
    K.loga = reinterpret_cast<double*>(base + L.loga);
    K.fdscale = reinterpret_cast<double*>(base + L.fdscale);
    K.loc = reinterpret_cast<double*>(base + L.loc);
    K.gmeta = reinterpret_cast<const TaskMeta*>(base + (lowp_fd ? L.gmeta_lp : L.gmeta));
    K.oplist = reinterpret_cast<Task*>(base + L.oplist);
    K.fdlist = reinterpret_cast<Task*>(base + L.fdlist);
    K.op_cap = static_cast<int>(P->optask.size());
    K.fd_cap = static_cast<int>(std::max(P->fdtask.size(), P->fdtask_lp.size()));
    {
        int64_t nloc = 1;
        for (int k = 0; k < P->dim; ++k) nloc *= P->nq;
        K.nelem = P->nqp_total / nloc;
    }
    K.nn = P->nn;
    for (int i = 0; i < 4; ++i) K.nn_ch[i] = P->nn_ch[i];
    K.nnw_rw = reinterpret_cast<uint16_t*>(base + L.nnw);
    K.nnw = K.nnw_rw;
    K.nn_head = P->nn_head;
    for (int i = 0; i < P->nq && i < 8; ++i) {
        K.gx[i] = P->gauss_x[i];
        K.gw[i] = P->gauss_w[i];
    }
    return K;
}

// k_solve<PP, *> lives in one translation unit per degree (solve_p*.hip)
const void* solve_kernel_p1(int prec, int dim, int narrow, int grid);
const void* solve_kernel_p2(int prec, int dim, int narrow, int grid);
const void* solve_kernel_p3(int prec, int dim, int narrow, int grid);
const void* solve_kernel_p4(int prec, int dim, int narrow, int grid);

// The persistent solve in 3D comes in two builds: 512-thread workgroups
// (8 wavefronts, 256 VGPRs with about 1 KB per lane of spills) and 256-thread
// workgroups (narrow: one workgroup per CU with the whole register file, no
// spills).  The narrow build is faster when every workgroup has many tasks
// per phase (several coefficient samples in one launch), the wide one when a
// task's work is spread over few tasks (a single sample, the learned
// correction's convolutions).  2D uses the wide build.
int solve_threads(int dim, int narrow) { return dim == 3 && narrow ? kBlockSolve3 : kBlock; }

// grid: the whole-grid solve k_solve_grid built for 1 or 2 workgroups per CU
// (0: the cooperative k_solve)
const void* solve_kernel(int p, int prec, int dim, int narrow = 0, int grid = 0) {
    switch (p) {
        case 1: return solve_kernel_p1(prec, dim, narrow, grid);
        case 2: return solve_kernel_p2(prec, dim, narrow, grid);
        case 3: return solve_kernel_p3(prec, dim, narrow, grid);
        default: return solve_kernel_p4(prec, dim, narrow, grid);
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
        F.sample_stride = f->sample_stride;
    }
    return F;
}

bool field_ok(const iga_field* f, int dim) {
    if (!f) return false;
    if (f->kind < IGA_FIELD_CONST || f->kind > IGA_FIELD_QP_SAMPLES) return false;
    if (f->kind == IGA_FIELD_QP_SAMPLES && !f->data_dev) return false;
    if (f->kind == IGA_FIELD_GRID3D && (dim != 3 || !f->data_dev || f->n[0] < 2 || f->n[1] < 2 || f->n[2] < 2))
        return false;
    return true;
}

// Instance index of a grid: component c of sample s is s * ncomp + c.
int instance_of(const iga_sg_plan_s* P, const Grid& g) { return g.sample * P->ncomp + g.comp; }
int ninstances(const iga_sg_plan_s* P) { return P->ncomp * P->nsamples; }

// Every solution table of grids g0..g1 is uniform with simple interior knots.
bool uniform_tables(const iga_sg_plan_s* P, int g0, int g1) {
    for (int gi = g0; gi < g1; ++gi)
        for (int k = 0; k < P->dim; ++k) {
            const Tab1D& T = P->tabs[P->grids[gi].tab[k]];
            if (!T.uniform || T.m != 1) return false;
        }
    return true;
}

// Inner precision a solve runs with: FP32 / BF16 factors hold the 1D
// eigen-decompositions only while max lambda / min lambda stays below about
// 1 / (FP32 precision); strongly graded knots exceed that (the L-shape with
// exponent 3 at level 4: 6e7) and the mixed modes then diverge, so the solve
// runs in FP64 and the report says so.
constexpr double kLowpLamRatio = 1e7;
int effective_precision(const iga_sg_plan_s* P, int prec) {
    return prec != IGA_PREC_FP64 && P->lam_ratio > kLowpLamRatio ? IGA_PREC_FP64 : prec;
}

int blocks_for(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    return static_cast<int>(std::min<int64_t>(std::max<int64_t>(b, 1), 65535));
}

}  // namespace

// Workspace of iga_sg_bind_static: one array per device, held until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it only stands in for the symbol); the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kStaticWorkspaceBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};       // device address of scratch, per device
uint64_t g_static_gen[kMaxDevices] = {};    // static bindings made on each device so far

// A plan bound to the static workspace stays usable until another plan binds
// the same device's array.
iga_status check_workspace(const iga_sg_plan_s* P) {
    if (P->static_dev < 0) return IGA_OK;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_gen[P->static_dev] != P->static_gen) {
        set_error("the static workspace of device %d was bound to another plan since this plan's "
                  "iga_sg_bind_static", P->static_dev);
        return IGA_ERR_STATE;
    }
    return IGA_OK;
}

iga_status bind_impl(iga_sg_plan P, void* ws, size_t bytes, void* stream);

}  // namespace

iga_status igasg::workspace_ok(const iga_sg_plan_s* P) { return check_workspace(P); }

extern "C" {

iga_status iga_sg_bind(iga_sg_plan P, void* ws, size_t bytes, void* stream) {
    if (!P || !ws) {
        set_error("null plan or workspace");
        return IGA_ERR_INVALID_ARG;
    }
    const iga_status s = bind_impl(P, ws, bytes, stream);
    if (s == IGA_OK) P->static_dev = -1;
    return s;
}

iga_status iga_sg_bind_static(iga_sg_plan P, void* stream) {
    if (!P) {
        set_error("null plan");
        return IGA_ERR_INVALID_ARG;
    }
    if (P->lay.total > kStaticWorkspaceBytes) {
        set_error("plan needs %zu bytes of workspace, the static workspace holds %zu", P->lay.total,
                  kStaticWorkspaceBytes);
        return IGA_ERR_OUT_OF_MEMORY;
    }
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d beyond the %d devices the static workspace serves", dev, kMaxDevices);
        return IGA_ERR_DEVICE;
    }
    uint64_t gen = 0;
    void* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (!g_static_ptr[dev]) {
            void* a = nullptr;
            HIP_OK(hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));
            g_static_ptr[dev] = a;
        }
        ptr = g_static_ptr[dev];
        gen = ++g_static_gen[dev];
    }
    P->static_dev = -1;  // until the binding is complete
    const iga_status s = bind_impl(P, ptr, kStaticWorkspaceBytes, stream);
    if (s != IGA_OK) return s;
    P->static_dev = dev;
    P->static_gen = gen;
    return IGA_OK;
}

}  // extern "C"

namespace {

iga_status bind_impl(iga_sg_plan P, void* ws, size_t bytes, void* stream) {
    if (bytes < P->lay.total) {
        set_error("workspace too small: %zu < %zu bytes", bytes, P->lay.total);
        return IGA_ERR_OUT_OF_MEMORY;
    }
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) {
        set_error("workspace must be 256-byte aligned");
        return IGA_ERR_INVALID_ARG;
    }
    // a captured step holds the previous workspace's addresses
    if (P->gexec) {
        (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(P->gexec));
        P->gexec = nullptr;
    }
    P->bound = false;
    P->ws = ws;
    P->ws_bytes = bytes;
    P->stream = stream;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(ws);
    const Layout& L = P->lay;
    HIP_OK(hipMemcpyAsync(base + L.tabs, P->tabs.data(), sizeof(Tab1D) * P->tabs.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(base + L.grids, P->grids.data(), sizeof(Grid) * P->grids.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(base + L.grids_lp, P->grids_lp.data(), sizeof(Grid) * P->grids_lp.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(base + L.dpool, P->dpool.data(), sizeof(double) * P->dpool.size(), hipMemcpyHostToDevice, st));
    if (!P->ipool.empty())
        HIP_OK(hipMemcpyAsync(base + L.ipool, P->ipool.data(), sizeof(int) * P->ipool.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(base + L.fpool, P->fpool.data(), sizeof(float) * P->fpool.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(base + L.hpool, P->hpool.data(), sizeof(uint16_t) * P->hpool.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(base + L.ctrl, P->ctrl.data(), sizeof(double) * P->ctrl.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(base + L.optask, P->optask.data(), sizeof(Task) * P->optask.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(base + L.fdtask, P->fdtask.data(), sizeof(Task) * P->fdtask.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(base + L.fdtask_lp, P->fdtask_lp.data(), sizeof(Task) * P->fdtask_lp.size(), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemsetAsync(base + L.bar, 0, 256, st));
    {
        // every grid's description with its 1D tables, one record per grid, so
        // that a solve task reads its description in one contiguous copy
        for (int lp = 0; lp < 2; ++lp) {
            const std::vector<Grid>& gv = lp ? P->grids_lp : P->grids;
            std::vector<TaskMeta>& mv = lp ? P->gmeta_lp : P->gmeta;
            mv.assign(gv.size(), TaskMeta());
            for (size_t gi = 0; gi < gv.size(); ++gi) {
                TaskMeta& M = mv[gi];
                std::memset(&M, 0, sizeof(M));
                M.g = gv[gi];
                for (int k = 0; k < kMaxDim; ++k)
                    if (gv[gi].tab[k] >= 0) M.t[k] = P->tabs[gv[gi].tab[k]];
                M.grid = static_cast<int>(gi);
                M.local = 0;
            }
            HIP_OK(hipMemcpyAsync(base + (lp ? L.gmeta_lp : L.gmeta), mv.data(), sizeof(TaskMeta) * mv.size(),
                                  hipMemcpyHostToDevice, st));
        }
    }
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
    if (P->lds_bytes > prop.sharedMemPerBlock) {
        set_error("plan needs %zu bytes of LDS per workgroup, the device offers %zu", P->lds_bytes,
                  static_cast<size_t>(prop.sharedMemPerBlock));
        return IGA_ERR_DEVICE;
    }
    // kernels that take the plan's LDS size: allow dynamic LDS beyond 64 KiB
    {
        const void* ks[] = {reinterpret_cast<const void*>(k_apply_op<1>), reinterpret_cast<const void*>(k_apply_op<2>),
                            reinterpret_cast<const void*>(k_apply_op<3>), reinterpret_cast<const void*>(k_apply_op<4>),
                            reinterpret_cast<const void*>(k_apply_fd)};
        for (const void* k : ks)
            HIP_OK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(P->lds_bytes)));
        for (int prec : {IGA_PREC_FP64, IGA_PREC_FP32, IGA_PREC_BF16FD})
            for (int narrow = 0; narrow <= (P->dim == 3 ? 1 : 0); ++narrow)
                for (int grid = 0; grid <= 2; ++grid)
                    HIP_OK(hipFuncSetAttribute(solve_kernel(P->p, prec, P->dim, narrow, grid),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               static_cast<int>(P->lds_bytes)));
    }
    // persistent width: workgroups resident at once for every build of the solve
    int occ = 1 << 20;
    for (int prec : {IGA_PREC_FP64, IGA_PREC_FP32, IGA_PREC_BF16FD})
        for (int narrow = 0; narrow <= (P->dim == 3 ? 1 : 0); ++narrow) {
            int o = 0;
            HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, solve_kernel(P->p, prec, P->dim, narrow),
                                                                solve_threads(P->dim, narrow), P->lds_bytes));
            occ = std::min(occ, o);
        }
    P->max_wg = std::max(1, occ) * P->num_cu;
    P->bound = true;
    P->assembled = false;
    P->solved = false;
    return IGA_OK;
}

}  // namespace

extern "C" {

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
    const bool lift = g && g->kind != IGA_FIELD_NONE;
    if (lift && (P->dim != 2 || P->rational_any || !field_ok(g, P->dim) || g->kind == IGA_FIELD_GRID3D ||
                 g->kind == IGA_FIELD_QP_SAMPLES)) {
        set_error("Dirichlet data: two-dimensional plans with polynomial maps and an analytic field");
        return IGA_ERR_INVALID_ARG;
    }
    size_t lift_lds = 0;
    if (lift) {
        int nmax = 0;
        for (const Grid& gr : P->grids) nmax = std::max(nmax, std::max(gr.nb[0], gr.nb[1]));
        lift_lds = sizeof(double) * (static_cast<size_t>(nmax) * (P->p + 2) + 2);
        if (lift_lds > static_cast<size_t>(kLdsLimit)) {
            set_error("Dirichlet data: a side of %d basis functions exceeds the LDS of the projection", nmax);
            return IGA_ERR_INVALID_ARG;
        }
    }
    if (const iga_status ws = check_workspace(P)) return ws;
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    Params K = make_params(P);
    int* err = reinterpret_cast<int*>(reinterpret_cast<char*>(P->ws) + P->lay.bar + 64);
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, st, err);  // a kernel, so that the step can be captured
    const int ng = static_cast<int>(P->grids.size());
    HIP_OK(launch_assemble(P->dim, a ? a->kind : IGA_FIELD_NONE, f ? f->kind : IGA_FIELD_NONE,
                           dim3(blocks_for(P->nqp_total)), st, K, to_dev(a), to_dev(f), ng, err));
    if (lift) {
        // boundary coefficients of the lift, then its load correction with the
        // element-local sums
        hipLaunchKernelGGL(k_zero, dim3(blocks_for(P->nlift)), dim3(kBlock), 0, st, K.lift_rw, P->nlift);
        HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(k_lift_edges<1>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lift_lds)));
        HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(k_lift_edges<2>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lift_lds)));
        HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(k_lift_edges<3>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lift_lds)));
        HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(k_lift_edges<4>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lift_lds)));
        HIP_OK(launch_lift_edges(P->p, dim3(ng, 4), lift_lds, st, K, to_dev(g)));
        K.lift = K.lift_rw;
    }
    // element-local sums (one lane group per element), then one thread per unknown
    HIP_OK(launch_loadiag(P->dim, P->p, P->ncompG == (P->dim == 2 ? 6 : 10), lift, st, K, blocks_for(P->ndof_total)));
    P->lifted = lift;
    HIP_OK(launch_loga(a ? a->kind : IGA_FIELD_NONE, dim3(blocks_for(P->ndof_total)), st, K, to_dev(a), ng));
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
    if (o->precision < IGA_PREC_FP64 || o->precision > IGA_PREC_BF16FD || !(o->tol > 0) || o->maxit < 1 ||
        o->schedule < 0 || o->schedule > 4) {
        set_error("invalid solve options");
        return IGA_ERR_INVALID_ARG;
    }
    if (const iga_status ws = check_workspace(P)) return ws;
    // a full tensor grid too large for one workgroup (or schedule 4): whole-device kernels
    if (P->streamed || o->schedule == 4) {
        if (P->xfer_off.empty() || P->grids.size() != 1 || o->precond != 0 || o->plain_fd) {
            set_error("schedule 4 (whole-device kernels) solves the single grid of a full tensor plan of one "
                      "patch and one sample with the scaled fast diagonalisation");
            return IGA_ERR_INVALID_ARG;
        }
        return fg_solve_plain(P, o, rep);
    }
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    // a mixed mode is declined where FP32 factors cannot hold the 1D pencils
    const int prec = effective_precision(P, o->precision);
    const bool lp = prec != IGA_PREC_FP64;  // FD blocking of the factor precision
    Params K = make_params(P, lp);
    if (o->plain_fd) K.fdscale = nullptr;  // unscaled pencil
    const std::vector<Grid>& grids = lp ? P->grids_lp : P->grids;
    const size_t nfd = (lp ? P->fdtask_lp : P->fdtask).size();
    const int ng = static_cast<int>(P->grids.size());
    SolveArgs A;
    A.prec = prec;
    A.maxit = o->maxit;
    A.max_refine = prec == IGA_PREC_FP64 ? std::max(1, o->max_refine > 0 ? o->max_refine : 3)
                                                 : std::max(1, o->max_refine);
    A.tol2 = o->tol * o->tol;
    // FP64: the inner test equals the outer one; mixed: loose inner tolerance
    double ti = prec == IGA_PREC_FP64 ? o->tol : (o->tol_inner > 0 ? o->tol_inner : 1e-4);
    A.tol_in2 = ti * ti;
    A.max_sweeps = (A.maxit + 2) * (A.max_refine + 1) + 4;
    A.continue_cg = o->continue_cg != 0 && prec != IGA_PREC_FP64;
    A.learned = o->precond == 1 ? 1 : 0;
    A.learned_iters = o->learned_iters > 0 ? o->learned_iters : 0;
    if (A.learned && (P->dim != 3 || !P->nn)) {
        set_error("learned preconditioning needs a three-dimensional plan and an attached network");
        return IGA_ERR_INVALID_ARG;
    }
    if (A.learned) {
        // the network's weights in the BF16 layout of the solve's convolutions
        hipLaunchKernelGGL(k_nn_pack, dim3(64), dim3(kBlock), 0, st, K);
        HIP_OK(hipGetLastError());
    }
    char* trbase = reinterpret_cast<char*>(P->ws) + P->lay.trace;
    A.trace = o->timing >= 2 ? reinterpret_cast<unsigned long long*>(trbase) : nullptr;
    A.trace_sweeps = kTraceSweeps;
    if (A.trace) HIP_OK(hipMemsetAsync(trbase, 0, sizeof(unsigned long long) * (1 + 6 * kTraceSweeps), st));
    const size_t lds = P->lds_bytes;
    if (o->timing)  // timing events are created on first use (a solve without timing creates nothing)
        for (int i = 0; i < 2; ++i)
            if (!P->ev[i]) HIP_OK(hipEventCreate(reinterpret_cast<hipEvent_t*>(&P->ev[i])));
    hipEvent_t e0 = static_cast<hipEvent_t>(P->ev[0]), e1 = static_cast<hipEvent_t>(P->ev[1]);
    if (o->timing) HIP_OK(hipEventRecord(e0, st));
    // Whole-grid solve (one workgroup per grid, no grid barrier) for a batched
    // launch whose grids are each a few tasks: forced by schedule 3, chosen
    // when every grid has one FD block and at most four operator tiles.
    bool whole = false;
    const int npat = static_cast<int>(P->patches.size());
    if (o->schedule == 3 && npat > 1) {
        set_error("the whole-grid schedule solves one patch grid per workgroup: not for several patches");
        return IGA_ERR_INVALID_ARG;
    }
    if (o->batched && npat == 1) {
        bool small = true;
        for (const Grid& g : grids) small = small && g.nblk == 1 && g.ntile <= 4;
        whole = o->schedule == 3 || (o->schedule == 0 && small);
    }
    auto launch = [&](int g0, int g1, int opb, int ope, int fdb, int fde) -> iga_status {
        const int64_t i0 = P->grids[g0].dof_off;
        const int64_t i1 = P->grids[g1 - 1].dof_off + P->grids[g1 - 1].ndof;
        hipLaunchKernelGGL(k_solve_init, dim3(blocks_for(i1 - i0)), dim3(kBlock), 0, st, K, g0, g1, i0, i1, opb, ope,
                           fdb, fde);
        HIP_OK(hipGetLastError());
        A.op_b = opb;
        A.op_e = ope;
        A.fd_b = fdb;
        A.fd_e = fde;
        A.ndone_target = (g1 - g0) / npat;  // solver-state groups
        int want = std::max(ope - opb, fde - fdb);
        if (o->workgroups > 0) want = o->workgroups;
        int nwg = std::max(1, std::min(want, P->max_wg));
        // at most one task per workgroup and phase: round robin over the
        // launch's tasks with their descriptions cached for the launch; more:
        // round robin over the per-sweep lists of the grids still iterating
        // (annulus w=10: FP32-class 245 FD tasks, static 2.73 against 2.85 ms;
        // FP64-class 453, lists 3.19 against 3.41 ms)
        A.active = (ope - opb > nwg || fde - fdb > nwg) ? 1 : 0;
        if (o->schedule == 1) A.active = 0;
        if (o->schedule == 2) A.active = 1;
        // 3D with more tasks than workgroups (and no learned correction, whose
        // convolutions want the wide workgroup): the narrow build (64
        // random-field samples: FP64 57 -> 46 ms, mixed 48 -> 44 ms).  The
        // choice depends on the launch alone, not on a forced schedule, so
        // both schedules of one launch run the same build and agree bitwise.
        const int narrow = P->dim == 3 && (ope - opb > nwg || fde - fdb > nwg) && !A.learned ? 1 : 0;
        void* args[] = {&K, &A};
        if (whole) {
            // whole-grid solve: a plain launch of as many workgroups as are
            // resident at once (they take the grids from a counter)
            const int nar = P->dim == 3 && !A.learned ? 1 : 0;
            const size_t ldsg = A.learned ? lds : P->lds_plain;  // no activations without the network
            // the two-workgroup build where two fit a CU by LDS, in the mixed
            // modes (random-field batch of 256 samples, FP32 inner solve, tile
            // 256: 77.7 against 107 ms; its FP64 operator spills, so plain
            // FP64 keeps the one-workgroup build)
            int waves = 1;
            if (prec != IGA_PREC_FP64) {
                int occ2 = 0;
                HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &occ2, solve_kernel(P->p, prec, P->dim, nar, 2), solve_threads(P->dim, nar), ldsg));
                if (occ2 >= 2) waves = 2;
            }
            const void* fk = solve_kernel(P->p, prec, P->dim, nar, waves);
            int occg = 0;
            HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occg, fk, solve_threads(P->dim, nar), ldsg));
            int nw = std::max(1, std::min(fde - fdb, std::max(1, occg) * P->num_cu));
            if (o->workgroups > 0) nw = std::min(nw, o->workgroups);
            HIP_OK(hipLaunchKernel(fk, dim3(nw), dim3(solve_threads(P->dim, nar)), args, ldsg, st));
            P->last_solve_coop = 0;
            return IGA_OK;
        }
        HIP_OK(hipLaunchCooperativeKernel(solve_kernel(P->p, prec, P->dim, narrow), dim3(nwg),
                                          dim3(solve_threads(P->dim, narrow)), args, static_cast<unsigned>(lds), st));
        P->last_solve_coop = 1;
        return IGA_OK;
    };
    if (o->batched) {
        iga_status s = launch(0, ng, 0, static_cast<int>(P->optask.size()), 0, static_cast<int>(nfd));
        if (s != IGA_OK) return s;
    } else {
        // one launch per solver-state group (a grid, or the patch grids of a component)
        for (int gi = 0; gi < ng; gi += npat) {
            const Grid& g = grids[gi];
            iga_status s = launch(gi, gi + npat, g.gtile_off, g.gtile_off + g.gntile, g.gblk_off, g.gblk_off + g.gnblk);
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
    int geom_err = 0;  // the assembly's flag: a non-positive det DF at some Gauss point
    HIP_OK(hipMemcpyAsync(&geom_err, reinterpret_cast<char*>(P->ws) + P->lay.bar + 64, sizeof(int),
                          hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (geom_err) {
        set_error("the geometry map has a non-positive Jacobian determinant at a Gauss point");
        return IGA_ERR_GEOMETRY;
    }
    for (int gi = 0; gi < ng; ++gi) {
        const int sg = P->grids[gi].state;  // the grid's solver-state group
        const GState& a = both[sg];
        const GState& b = both[ng + sg];
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
        if (P->grids[gi].state == gi) total += s.total_it;  // once per group
        if (s.stage != STAGE_DONE || s.status == GS_MAXIT || s.status == GS_RUNNING) {
            if (ret == IGA_OK) ret = IGA_ERR_NOT_CONVERGED;
        }
        if (s.status == GS_BREAKDOWN) ret = IGA_ERR_BREAKDOWN;
    }
    if (rep) {
        rep->ncomp = ninstances(P);
        rep->total_iters = total;
        rep->precision = prec;
        rep->lam_ratio = P->lam_ratio;
        for (int gi = 0; gi < ng; ++gi) {
            const GState& s = stv[gi];
            const int c = instance_of(P, P->grids[gi]);
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
        if (A.trace && o->batched) {
            std::vector<unsigned long long> tr(1 + 6 * kTraceSweeps);
            unsigned sweeps = 0;
            HIP_OK(hipMemcpy(tr.data(), A.trace, sizeof(unsigned long long) * tr.size(), hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(&sweeps, reinterpret_cast<char*>(P->ws) + P->lay.bar + 4 * kBarSweeps, sizeof(unsigned),
                             hipMemcpyDeviceToHost));
            const int ns = std::min<int>(static_cast<int>(sweeps), kTraceSweeps);
            rep->sweeps = static_cast<int>(sweeps);
            double acc[6] = {0, 0, 0, 0, 0, 0};
            for (int s = 0; s < ns; ++s) {
                for (int ph = 0; ph < 3; ++ph) {
                    unsigned long long prev = (ph == 0) ? (s == 0 ? tr[0] : tr[1 + 6 * (s - 1) + 2]) : tr[1 + 6 * s + ph - 1];
                    acc[ph] += static_cast<double>(tr[1 + 6 * s + ph] - prev);
                    acc[3 + ph] += static_cast<double>(tr[1 + 6 * s + 3 + ph]);
                }
            }
            for (int i = 0; i < 6; ++i) rep->phase_us[i] = ns > 0 ? acc[i] / ns * 0.01 : 0.0;  // 100 MHz
        }
    }
    if (ret == IGA_ERR_NOT_CONVERGED) set_error("some component did not reach the tolerance");
    if (ret == IGA_ERR_BREAKDOWN) set_error("CG breakdown in some component");
    return ret;
}

iga_status iga_sg_combine(iga_sg_plan P, const double* xi, const int* patch, int64_t n, double* u, double* grad) {
    if (!P || (n > 0 && (!xi || !u)) || n < 0) {
        set_error("invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    if (!P->solved) {
        set_error("iga_sg_combine before iga_sg_solve");
        return IGA_ERR_STATE;
    }
    if (const iga_status ws = check_workspace(P)) return ws;
    if (n == 0) return IGA_OK;
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    Params K = make_params(P);
    // the grids of a sample are contiguous (sample-major); sample s writes u + s n
    const int gps = static_cast<int>(P->grids.size()) / P->nsamples;
    for (int smp = 0; smp < P->nsamples; ++smp) {
        HIP_OK(launch_combine(P->dim, P->p, uniform_tables(P, smp * gps, (smp + 1) * gps), blocks_for(n), st, K, xi, patch, n,
                              u + smp * n, smp * gps, (smp + 1) * gps, 1));
        if (grad)
            HIP_OK(launch_combine_grad(P->dim, P->p, blocks_for(n), st, K, xi, patch, n, grad + smp * n * P->dim,
                                       smp * gps, (smp + 1) * gps, 1));
    }
    HIP_OK(hipGetLastError());
    return IGA_OK;
}

iga_status iga_sg_eval(iga_sg_plan P, int comp, const double* xi, const int* patch, int64_t n, double* u,
                       double* grad) {
    if (!P || comp < 0 || comp >= ninstances(P) || (n > 0 && (!xi || !u)) || n < 0) {
        set_error("invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    if (!P->solved) {
        set_error("iga_sg_eval before iga_sg_solve");
        return IGA_ERR_STATE;
    }
    if (const iga_status ws = check_workspace(P)) return ws;
    if (n == 0) return IGA_OK;
    int g0 = -1, g1 = -1;
    for (int gi = 0; gi < static_cast<int>(P->grids.size()); ++gi)
        if (instance_of(P, P->grids[gi]) == comp) {
            if (g0 < 0) g0 = gi;
            g1 = gi + 1;
        }
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    Params K = make_params(P);
    HIP_OK(launch_combine(P->dim, P->p, uniform_tables(P, g0, g1), blocks_for(n), st, K, xi, patch, n, u, g0, g1, 0));
    if (grad) HIP_OK(launch_combine_grad(P->dim, P->p, blocks_for(n), st, K, xi, patch, n, grad, g0, g1, 0));
    HIP_OK(hipGetLastError());
    return IGA_OK;
}

iga_status iga_sg_quad_points(iga_sg_plan P, double* xq, double* wq, int64_t cap, int64_t* nq) {
    if (!P || !nq) {
        set_error("invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    *nq = P->nqp_total;
    if (!xq || cap < P->nqp_total) return IGA_OK;
    if (!P->bound) {
        set_error("iga_sg_quad_points before iga_sg_bind");
        return IGA_ERR_STATE;
    }
    if (const iga_status ws = check_workspace(P)) return ws;
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    Params K = make_params(P);
    if (P->dim == 2) hipLaunchKernelGGL(k_quad_points<2>, dim3(blocks_for(P->nqp_total)), dim3(kBlock), 0, st, K, xq, wq);
    else hipLaunchKernelGGL(k_quad_points<3>, dim3(blocks_for(P->nqp_total)), dim3(kBlock), 0, st, K, xq, wq);
    HIP_OK(hipGetLastError());
    return IGA_OK;
}

iga_status iga_sg_detail_norms(iga_sg_plan P, const double* xi, const double* wq, int64_t n, double* vals,
                               double* norms) {
    if (!P || n < 0 || (n > 0 && (!xi || !wq || !vals)) || !norms) {
        set_error("invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    if (P->detail_off < 0 || P->patches.size() != 1 || P->nsamples != 1) {
        set_error("iga_sg_detail_norms needs a plan of one patch and one sample built from an index set "
                  "with keep_all");
        return IGA_ERR_INVALID_ARG;
    }
    if (!P->solved) {
        set_error("iga_sg_detail_norms before iga_sg_solve");
        return IGA_ERR_STATE;
    }
    if (const iga_status ws = check_workspace(P)) return ws;
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    Params K = make_params(P);
    const int ng = static_cast<int>(P->grids.size());
    for (int g = 0; g < ng && n > 0; ++g)
        HIP_OK(launch_combine(P->dim, P->p, uniform_tables(P, g, g + 1), blocks_for(n), st, K, xi, nullptr, n,
                              vals + static_cast<int64_t>(g) * n, g, g + 1, 0));
    hipLaunchKernelGGL(k_detail_norms, dim3(ng), dim3(kBlock), 0, st, vals, wq, n, K.ipool + P->detail_off,
                       1 << P->dim, norms);
    HIP_OK(hipGetLastError());
    return IGA_OK;
}

iga_status iga_sg_coeffs(iga_sg_plan P, int comp, double* out) {
    if (!P || comp < 0 || comp >= ninstances(P) || !out) {
        set_error("invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    if (!P->solved) {
        set_error("iga_sg_coeffs before iga_sg_solve");
        return IGA_ERR_STATE;
    }
    if (const iga_status ws = check_workspace(P)) return ws;
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    Params K = make_params(P);
    int64_t o = 0;  // the patch grids of a component one after another
    for (const Grid& g : P->grids)
        if (instance_of(P, g) == comp) {
            HIP_OK(hipMemcpyAsync(out + o, K.x + g.dof_off, sizeof(double) * g.ndof, hipMemcpyDeviceToDevice, st));
            o += g.ndof;
        }
    return IGA_OK;
}

iga_status iga_sg_coeffs_full(iga_sg_plan P, int comp, double* out) {
    if (!P || comp < 0 || comp >= ninstances(P) || !out) {
        set_error("invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    if (!P->solved) {
        set_error("iga_sg_coeffs_full before iga_sg_solve");
        return IGA_ERR_STATE;
    }
    if (const iga_status ws = check_workspace(P)) return ws;
    int g0 = -1, g1 = -1;
    int64_t nt = 0;
    for (int gi = 0; gi < static_cast<int>(P->grids.size()); ++gi)
        if (instance_of(P, P->grids[gi]) == comp) {
            if (g0 < 0) g0 = gi;
            g1 = gi + 1;
            const Grid& g = P->grids[gi];
            nt += static_cast<int64_t>(g.nb[0]) * g.nb[1] * g.nb[2];
        }
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    Params K = make_params(P);
    hipLaunchKernelGGL(k_full_coeffs, dim3(blocks_for(nt / std::max(1, g1 - g0))), dim3(kBlock), 0, st, K, g0, g1, out);
    HIP_OK(hipGetLastError());
    return IGA_OK;
}

iga_status iga_sg_loga(iga_sg_plan P, int comp, double* out) {
    if (!P || comp < 0 || comp >= ninstances(P) || !out) {
        set_error("invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    if (!P->assembled) {
        set_error("iga_sg_loga before iga_sg_assemble");
        return IGA_ERR_STATE;
    }
    if (const iga_status ws = check_workspace(P)) return ws;
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    Params K = make_params(P);
    int64_t o = 0;  // the patch grids of a component one after another
    for (const Grid& g : P->grids)
        if (instance_of(P, g) == comp) {
            HIP_OK(hipMemcpyAsync(out + o, K.loga + g.dof_off, sizeof(double) * g.ndof, hipMemcpyDeviceToDevice, st));
            o += g.ndof;
        }
    return IGA_OK;
}

iga_status iga_sg_set_network(iga_sg_plan P, const int* channels, int nlayers, const float* params_dev, int head) {
    if (!P) {
        set_error("null plan");
        return IGA_ERR_INVALID_ARG;
    }
    // a captured step holds the previous network's address
    if (P->gexec && params_dev != P->nn) {
        (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(P->gexec));
        P->gexec = nullptr;
    }
    if (!params_dev) {
        P->nn = nullptr;
        return IGA_OK;
    }
    if (P->dim != 3 || !channels || nlayers != 3 || channels[0] != 3 || channels[3] != 1 || channels[1] < 1 ||
        channels[1] > kNnMaxH1 || channels[2] < 1 || channels[2] > kNnMaxH2) {
        set_error("the learned preconditioner takes 3 layers, channels 3 -> h1 -> h2 -> 1 (h1 <= %d, h2 <= %d), "
                  "3D plans", kNnMaxH1, kNnMaxH2);
        return IGA_ERR_INVALID_ARG;
    }
    if (head < 0 || head > 1) {
        set_error("network head must be 0 (additive) or 1 (log-scale)");
        return IGA_ERR_INVALID_ARG;
    }
    P->nn = params_dev;
    for (int i = 0; i < 4; ++i) P->nn_ch[i] = channels[i];
    P->nn_head = head;
    return IGA_OK;
}

iga_status iga_sg_rhs(iga_sg_plan P, int comp, double* out) {
    if (!P || comp < 0 || comp >= ninstances(P) || !out) {
        set_error("invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    if (!P->assembled) {
        set_error("iga_sg_rhs before iga_sg_assemble");
        return IGA_ERR_STATE;
    }
    if (const iga_status ws = check_workspace(P)) return ws;
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    Params K = make_params(P);
    int64_t o = 0;  // the patch grids of a component one after another
    for (const Grid& g : P->grids)
        if (instance_of(P, g) == comp) {
            HIP_OK(hipMemcpyAsync(out + o, K.b + g.dof_off, sizeof(double) * g.ndof, hipMemcpyDeviceToDevice, st));
            o += g.ndof;
        }
    return IGA_OK;
}

iga_status iga_sg_set_rhs(iga_sg_plan P, int comp, const double* b) {
    if (!P || comp < 0 || comp >= ninstances(P) || !b) {
        set_error("invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    if (!P->assembled) {
        set_error("iga_sg_set_rhs before iga_sg_assemble");
        return IGA_ERR_STATE;
    }
    if (const iga_status ws = check_workspace(P)) return ws;
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    Params K = make_params(P);
    int64_t o = 0;
    for (const Grid& g : P->grids)
        if (instance_of(P, g) == comp) {
            HIP_OK(hipMemcpyAsync(K.b + g.dof_off, b + o, sizeof(double) * g.ndof, hipMemcpyDeviceToDevice, st));
            o += g.ndof;
        }
    P->solved = false;
    return IGA_OK;
}

iga_status iga_sg_apply(iga_sg_plan P, int comp, int which, const double* x, double* y) {
    if (!P || comp < 0 || comp >= ninstances(P) || !x || !y || which < 0 || which > 6) {
        set_error("invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    if (P->patches.size() > 1) {
        set_error("iga_sg_apply acts on one patch grid: not for several patches");
        return IGA_ERR_INVALID_ARG;
    }
    if (!P->assembled) {
        set_error("iga_sg_apply before iga_sg_assemble");
        return IGA_ERR_STATE;
    }
    if (const iga_status ws = check_workspace(P)) return ws;
    int gi = -1;
    for (int i = 0; i < static_cast<int>(P->grids.size()); ++i)
        if (instance_of(P, P->grids[i]) == comp) gi = i;
    if (P->streamed && which >= 2 && which != 5) {
        set_error("iga_sg_apply: the fast diagonalisation of a grid solved by whole-device kernels has no "
                  "block tasks");
        return IGA_ERR_INVALID_ARG;
    }
    const bool lp = which == 3 || which == 4;  // FD with FP32/BF16 factors uses their blocking
    const Grid& g = (lp ? P->grids_lp : P->grids)[gi];
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    Params K = make_params(P, lp);
    // the hooks read/write the caller's vectors shifted to the grid's offset
    const double* xs = x - g.dof_off;
    double* ys = y - g.dof_off;
    if (which <= 1 || which == 5) {
        OpIO io;
        io.in_a = xs;
        io.in_b = nullptr;
        io.beta = 0.0;
        io.out_in = nullptr;
        io.out = ys;
        io.rhs = which == 5 ? K.b : nullptr;  // residual b - A x
        io.part = nullptr;
        io.lowp = which == 1 ? 1 : 0;
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
        io.prec = which == 6 ? 0 : which - 2;
        io.scale = which == 6 ? K.fdscale : nullptr;
        hipLaunchKernelGGL(k_apply_fd, dim3(g.nblk), dim3(kBlock), P->lds_bytes, st, K, gi, io, 1);
        HIP_OK(hipGetLastError());
        hipLaunchKernelGGL(k_apply_fd, dim3(g.nblk), dim3(kBlock), P->lds_bytes, st, K, gi, io, 0);
        HIP_OK(hipGetLastError());
    }
    return IGA_OK;
}

iga_status iga_sg_graph_capture(iga_sg_plan P, const iga_field* f, const iga_field* a, const iga_sg_solve_opts* o) {
    if (!P || !o) {
        set_error("null argument");
        return IGA_ERR_INVALID_ARG;
    }
    if (!P->bound) {
        set_error("iga_sg_graph_capture before iga_sg_bind");
        return IGA_ERR_STATE;
    }
    if (o->timing) {
        set_error("timing reports are not available for a captured step");
        return IGA_ERR_INVALID_ARG;
    }
    if (const iga_status ws = check_workspace(P)) return ws;
    if (P->streamed || o->schedule == 4) {
        set_error("graph capture records the persistent solve: not for whole-device full-grid solves");
        return IGA_ERR_INVALID_ARG;
    }
    hipStream_t st = static_cast<hipStream_t>(P->stream);
    if (!st) {
        set_error("graph capture needs a plan bound to a created stream, not the default stream");
        return IGA_ERR_STATE;
    }
    if (P->gexec) {
        HIP_OK(hipGraphExecDestroy(static_cast<hipGraphExec_t>(P->gexec)));
        P->gexec = nullptr;
    }
    HIP_OK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    iga_status s = iga_sg_assemble(P, f, a, nullptr);
    if (s == IGA_OK) s = iga_sg_solve(P, o, nullptr);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);  // always leave capture mode
    if (s != IGA_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        if (s == IGA_OK) {
            set_error("hipStreamEndCapture failed: %s", hipGetErrorString(e));
            s = IGA_ERR_DEVICE;
        }
        return s;
    }
    // The persistent solve needs all its workgroups resident at once (grid
    // barrier): its captured node is marked cooperative, as the direct
    // launch is.
    size_t nn = 0;
    hipError_t ge = hipGraphGetNodes(g, nullptr, &nn);
    std::vector<hipGraphNode_t> nodes(nn);
    if (ge == hipSuccess && nn) ge = hipGraphGetNodes(g, nodes.data(), &nn);
    const void* fsolve = solve_kernel(P->p, effective_precision(P, o->precision), P->dim, 0);
    const void* fsolve_narrow = solve_kernel(P->p, effective_precision(P, o->precision), P->dim, 1);
    // the whole-grid solve is a plain kernel node: nothing to mark
    const int want_marked = !P->last_solve_coop ? 0
                            : (o->batched ? 1 : static_cast<int>(P->grids.size() / P->patches.size()));
    int marked = 0;
    for (size_t i = 0; ge == hipSuccess && i < nn; ++i) {
        hipGraphNodeType t;
        ge = hipGraphNodeGetType(nodes[i], &t);
        if (ge != hipSuccess || t != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams kp;
        ge = hipGraphKernelNodeGetParams(nodes[i], &kp);
        if (ge != hipSuccess || (kp.func != fsolve && kp.func != fsolve_narrow)) continue;
        hipLaunchAttributeValue v;
        std::memset(&v, 0, sizeof(v));
        v.cooperative = 1;
        ge = hipGraphKernelNodeSetAttribute(nodes[i], hipKernelNodeAttributeCooperative, &v);
        ++marked;
    }
    hipGraphExec_t ex = nullptr;
    if (ge == hipSuccess && marked == want_marked)
        ge = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    else if (ge == hipSuccess)
        ge = hipErrorInvalidValue;
    (void)hipGraphDestroy(g);
    if (ge != hipSuccess) {
        set_error("graph of the step not built (%s, %d solve nodes marked)", hipGetErrorString(ge), marked);
        return IGA_ERR_DEVICE;
    }
    P->gexec = ex;
    return IGA_OK;
}

iga_status iga_sg_graph_launch(iga_sg_plan P) {
    if (!P) {
        set_error("null plan");
        return IGA_ERR_INVALID_ARG;
    }
    if (!P->gexec) {
        set_error("no captured step: iga_sg_graph_launch before iga_sg_graph_capture, or after a bind or a "
                  "network change released it");
        return IGA_ERR_STATE;
    }
    if (const iga_status ws = check_workspace(P)) return ws;
    HIP_OK(hipGraphLaunch(static_cast<hipGraphExec_t>(P->gexec), static_cast<hipStream_t>(P->stream)));
    P->assembled = true;
    P->solved = true;
    return IGA_OK;
}

void iga_sg_destroy(iga_sg_plan P) {
    if (!P) return;
    if (P->gexec) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(P->gexec));
    for (int i = 0; i < 8; ++i)
        if (P->ev[i]) (void)hipEventDestroy(static_cast<hipEvent_t>(P->ev[i]));
    delete P;
}

}  // extern "C"
