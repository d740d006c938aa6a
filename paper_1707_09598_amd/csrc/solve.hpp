// solve.hpp -- device code of the persistent sparse-grid solve: matrix-free
// operator tiles, fast-diagonalisation transforms, the grid-wide barrier and
// the refinement / PCG state machine (kernel template k_solve).  Included by
// the translation units that instantiate k_solve for one spline degree each
// and by kernels.hip for the single-operation kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <type_traits>

#include "common.hpp"
#include "device.hpp"
#include "iga_sg.h"

namespace igasg {

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
    int isum = 0;         // several patches: in_a summed across interfaces (iface_add)
};

// Several patches (2D): a vector assembled patch by patch (an operator
// output, a preconditioned residual) holds at an interface unknown the
// contribution of its own patch only.  iface_add returns x (the value at
// unknown (i1, i2) of grid g) plus the partner's value from the neighbouring
// patch's grid, and 0 at a fixed vertex; other unknowns keep x.  Both
// copies of an interface unknown form the same sum (addition commutes), so
// the copies stay equal.
__device__ __forceinline__ bool iface_pinned(const Grid& g, int lin) {
    return g.pin[0] == lin || g.pin[1] == lin || g.pin[2] == lin || g.pin[3] == lin;
}
// side of grid g whose interface holds unknown (i1, i2), or -1
__device__ __forceinline__ int iface_side(const Grid& g, int i1, int i2) {
    if ((g.nbr_on & 1) && i1 == 0) return 0;
    if ((g.nbr_on & 2) && i1 == g.ni[0] - 1) return 1;
    if ((g.nbr_on & 4) && i2 == 0) return 2;
    if ((g.nbr_on & 8) && i2 == g.ni[1] - 1) return 3;
    return -1;
}
__device__ __forceinline__ double iface_add(const Grid& g, const double* v, int i1, int i2, double x) {
    if (!g.nbr_on) return x;
    if (iface_pinned(g, i1 + g.ni[0] * i2)) return 0.0;
    const int sd = iface_side(g, i1, i2);
    if (sd < 0) return x;
    const int t = sd < 2 ? i2 : i1;
    return x + v[g.dof_off + g.nbr_base[sd] + static_cast<int64_t>(g.nbr_stride[sd]) * t];
}

// One row j2 of Gauss points of one element, by sum factorisation: the
// element's (p+1)^2 output contributions from that row,
//   y[a1][a2] = sum_j1 B2[j2][a2] (B1[j1][a1] F0 + D1[j1][a1] F1) + D2[j2][a2] B1[j1][a1] F2,
// with (F0, F1, F2) = G (v, dv/dxi1, dv/dxi2) at the point (the rational basis
// adds the value component F0; G holds the symmetric coefficient matrix).
template <int PP, bool RAT, typename T>
__device__ __forceinline__ void elem_row_2d(const double* X, int nh1, int x1, int x2, const double* B1,
                                            const double* D1, const double* B2r, const double* D2r, const T* Gr,
                                            int64_t nqp, T (&y)[PP + 1][PP + 1]) {
    constexpr int NQ = PP + 1;
    T b2[PP + 1], d2[PP + 1], tb[PP + 1], td[PP + 1], sb[PP + 1], sd[PP + 1];
#pragma unroll
    for (int a = 0; a <= PP; ++a) {
        b2[a] = static_cast<T>(B2r[a]);
        d2[a] = static_cast<T>(D2r[a]);
    }
#pragma unroll
    for (int a1 = 0; a1 <= PP; ++a1) {
        T u = T(0), v = T(0);
#pragma unroll
        for (int a2 = 0; a2 <= PP; ++a2) {
            const T c = static_cast<T>(X[(x2 + a2) * nh1 + x1 + a1]);
            u += b2[a2] * c;
            v += d2[a2] * c;
        }
        tb[a1] = u;
        td[a1] = v;
        sb[a1] = T(0);
        sd[a1] = T(0);
    }
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
            const T g00 = Gr[j1], g01 = Gr[nqp + j1], g02 = Gr[2 * nqp + j1];
            const T g11 = Gr[3 * nqp + j1], g12 = Gr[4 * nqp + j1], g22 = Gr[5 * nqp + j1];
            F0 = g00 * v0 + g01 * v1 + g02 * v2;
            F1 = g01 * v0 + g11 * v1 + g12 * v2;
            F2 = g02 * v0 + g12 * v1 + g22 * v2;
        } else {
            const T g11 = Gr[j1], g12 = Gr[nqp + j1], g22 = Gr[2 * nqp + j1];
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
        for (int a1 = 0; a1 <= PP; ++a1) y[a1][a2] = b2[a2] * sb[a1] + d2[a2] * sd[a1];
}

template <int PP>
__device__ __forceinline__ void op_tile_2d(const Params& P, const Grid& g, const Tab1D& T1, const Tab1D& T2,
                                           int tile, const OpIO& io, double* lds) {
    const int p = PP;
    const int m1 = T1.m, m2 = T2.m;
    const int t1 = tile % g.ntd[0], t2 = tile / g.ntd[0];
    const int a1 = t1 * g.tile[0], b1 = min(g.ni[0], a1 + g.tile[0]);
    const int a2 = t2 * g.tile[1], b2 = min(g.ni[1], a2 + g.tile[1]);
    int el1, eh1, el2, eh2;
    d_elem_range(a1, b1, p, m1, g.E[0], T1.lo, &el1, &eh1);
    d_elem_range(a2, b2, p, m2, g.E[1], T2.lo, &el2, &eh2);
    const int ne1 = eh1 - el1 + 1, ne2 = eh2 - el2 + 1;
    const int hl1 = el1 * m1 - T1.lo, hl2 = el2 * m2 - T2.lo;   // unknown index of halo start
    // halo: unknowns hl .. (last basis function of the last element) - lo
    const int nh1 = eh1 * m1 + p - T1.lo - hl1 + 1, nh2 = eh2 * m2 + p - T2.lo - hl2 + 1;
    double* X = lds;
    double* Y = lds + nh1 * nh2;
    double* red = Y + ne1 * ne2 * (p + 1) * (p + 1);
    const int64_t off = g.dof_off;
    const int n1 = g.ni[0], n2 = g.ni[1];
    const FDiv dh(nh1);
    for (int idx = threadIdx.x; idx < nh1 * nh2; idx += kBlock) {
        int r1;
        const int q1 = dh.div(idx, &r1);
        int i1 = hl1 + r1, i2 = hl2 + q1;
        double v = 0.0;
        if (i1 >= 0 && i1 < n1 && i2 >= 0 && i2 < n2) {
            int64_t gi = off + static_cast<int64_t>(i2) * n1 + i1;
            v = io.in_a[gi];
            if (io.isum) v = iface_add(g, io.in_a, i1, i2, v);
            if (io.in_b) v += io.beta * io.in_b[gi];
            if (io.out_in && i1 >= a1 && i1 < b1 && i2 >= a2 && i2 < b2) io.out_in[gi] = v;
        }
        X[idx] = v;
    }
    __syncthreads();
    // items: (element, row j2 of Gauss points), NG lanes per element (NG the
    // power of two >= p+1); the rows of an element are summed over its lanes
    // in a fixed order (group_reduce_scatter), lane j2 keeping the outputs of
    // a2 = j2
    constexpr int NQ = PP + 1;
    constexpr int NG = NQ <= 2 ? 2 : (NQ <= 4 ? 4 : 8);
    const int nqp1 = NQ * NQ;
    const int64_t nqp = g.nqp;
    const FDiv de(ne1);
    const bool rat = P.rational[g.patch] != 0;
    const int nitem = ne1 * ne2 * NG;
    for (int it = threadIdx.x; it < nitem; it += kBlock) {
        const int el = it / NG, j2 = it & (NG - 1);
        int r1;
        const int q1 = de.div(el, &r1);
        const int e1 = el1 + r1, e2 = el2 + q1;
        const int x1 = e1 * m1 - T1.lo - hl1, x2 = e2 * m2 - T2.lo - hl2;
        const int jr = j2 < NQ ? j2 : 0;
        const double* B1 = P.dpool + T1.oB + static_cast<int64_t>(e1) * nqp1;
        const double* D1 = P.dpool + T1.oD + static_cast<int64_t>(e1) * nqp1;
        const double* B2r = P.dpool + T2.oB + static_cast<int64_t>(e2) * nqp1 + jr * NQ;
        const double* D2r = P.dpool + T2.oD + static_cast<int64_t>(e2) * nqp1 + jr * NQ;
        const int64_t qrow = static_cast<int64_t>(e2 * NQ + jr) * g.Q[0] + static_cast<int64_t>(e1) * NQ;
        double yv[NQ];
        if (io.lowp) {
            float y[NQ][NQ];
            const float* Gr = P.G32 + g.qp_off * P.ncompG + qrow;
            if (rat) elem_row_2d<PP, true, float>(X, nh1, x1, x2, B1, D1, B2r, D2r, Gr, nqp, y);
            else elem_row_2d<PP, false, float>(X, nh1, x1, x2, B1, D1, B2r, D2r, Gr, nqp, y);
#pragma unroll
            for (int a1 = 0; a1 < NQ; ++a1) {
                float c[NG];
#pragma unroll
                for (int a2 = 0; a2 < NG; ++a2) c[a2] = a2 < NQ && j2 < NQ ? y[a1][a2] : 0.0f;
                yv[a1] = static_cast<double>(group_reduce_scatter<NG>(c, j2));
            }
        } else {
            double y[NQ][NQ];
            const double* Gr = P.G64 + g.qp_off * P.ncompG + qrow;
            if (rat) elem_row_2d<PP, true, double>(X, nh1, x1, x2, B1, D1, B2r, D2r, Gr, nqp, y);
            else elem_row_2d<PP, false, double>(X, nh1, x1, x2, B1, D1, B2r, D2r, Gr, nqp, y);
#pragma unroll
            for (int a1 = 0; a1 < NQ; ++a1) {
                double c[NG];
#pragma unroll
                for (int a2 = 0; a2 < NG; ++a2) c[a2] = a2 < NQ && j2 < NQ ? y[a1][a2] : 0.0;
                yv[a1] = group_reduce_scatter<NG>(c, j2);
            }
        }
        // lane j2 holds the outputs of a2 = j2 summed over the element's rows
        if (j2 < NQ) {
            double* Ye = Y + el * nqp1 + NQ * j2;
#pragma unroll
            for (int a1 = 0; a1 < NQ; ++a1) Ye[a1] = yv[a1];
        }
    }
    __syncthreads();
    const int w1 = b1 - a1, nown = w1 * (b2 - a2);
    double dot = 0.0;
    const FDiv dw(w1);
    for (int o = threadIdx.x; o < nown; o += kBlock) {
        int r1;
        const int q1 = dw.div(o, &r1);
        const int i1 = a1 + r1, i2 = a2 + q1;
        const int I1 = i1 + T1.lo, I2 = i2 + T2.lo;
        int lo1, hi1, lo2, hi2;
        d_elem_range(i1, i1 + 1, p, m1, g.E[0], T1.lo, &lo1, &hi1);
        d_elem_range(i2, i2 + 1, p, m2, g.E[1], T2.lo, &lo2, &hi2);
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

// ---------------------------------------------------------------------------
// operator application (3D).  Items are (element, layer j3 of Gauss points);
// one item computes the element's (p+1)^3 output contributions of its layer by
// sum factorisation through the directions 3, 2, 1 and back; the NG lanes of
// an element add their layers in a fixed order (group_reduce_scatter, DPP
// lane exchanges), lane j3 keeping the outputs of a3 = j3.
// ---------------------------------------------------------------------------
template <int PP, bool RAT, typename T, typename TX>
__device__ __forceinline__ void elem_layer_3d(const TX* X, int nh1, int nh2, int x1, int x2, int x3,
                                              const double* B1, const double* D1, const double* B2,
                                              const double* D2, const double* B3r, const double* D3r,
                                              const T* Gl, int64_t nqp, int Q1, T (&Zb)[PP + 1][PP + 1],
                                              T (&Zd)[PP + 1][PP + 1], T (&b3)[PP + 1], T (&d3)[PP + 1]) {
    constexpr int NQ = PP + 1;
    T tb[PP + 1][PP + 1], td[PP + 1][PP + 1];
#pragma unroll
    for (int a = 0; a <= PP; ++a) {
        b3[a] = static_cast<T>(B3r[a]);
        d3[a] = static_cast<T>(D3r[a]);
    }
    // contract direction 3: tb = sum_a3 b3 c, td = sum_a3 d3 c
#pragma unroll
    for (int a2 = 0; a2 <= PP; ++a2)
#pragma unroll
        for (int a1 = 0; a1 <= PP; ++a1) {
            T u = T(0), v = T(0);
#pragma unroll
            for (int a3 = 0; a3 <= PP; ++a3) {
                const T c = static_cast<T>(X[((x3 + a3) * nh2 + x2 + a2) * nh1 + x1 + a1]);
                u += b3[a3] * c;
                v += d3[a3] * c;
            }
            tb[a1][a2] = u;
            td[a1][a2] = v;
            Zb[a1][a2] = T(0);
            Zd[a1][a2] = T(0);
        }
    // one row j2 at a time (not unrolled): bounds the loads in flight and the registers
#pragma unroll 1
    for (int j2 = 0; j2 < NQ; ++j2) {
        T b2[PP + 1], d2[PP + 1];
#pragma unroll
        for (int a = 0; a <= PP; ++a) {
            b2[a] = static_cast<T>(B2[j2 * NQ + a]);
            d2[a] = static_cast<T>(D2[j2 * NQ + a]);
        }
        // contract direction 2
        T ub[PP + 1], u2[PP + 1], u3[PP + 1];
#pragma unroll
        for (int a1 = 0; a1 <= PP; ++a1) {
            T s0 = T(0), s2 = T(0), s3 = T(0);
#pragma unroll
            for (int a2 = 0; a2 <= PP; ++a2) {
                s0 += b2[a2] * tb[a1][a2];
                s2 += d2[a2] * tb[a1][a2];
                s3 += b2[a2] * td[a1][a2];
            }
            ub[a1] = s0;
            u2[a1] = s2;
            u3[a1] = s3;
        }
        T w0[PP + 1], w2[PP + 1], w3[PP + 1];
#pragma unroll
        for (int a1 = 0; a1 <= PP; ++a1) w0[a1] = w2[a1] = w3[a1] = T(0);
        const T* Gr = Gl + static_cast<int64_t>(j2) * Q1;
#pragma unroll
        for (int j1 = 0; j1 < NQ; ++j1) {
            T b1[PP + 1], d1[PP + 1];
#pragma unroll
            for (int a = 0; a <= PP; ++a) {
                b1[a] = static_cast<T>(B1[j1 * NQ + a]);
                d1[a] = static_cast<T>(D1[j1 * NQ + a]);
            }
            T v0 = T(0), v1 = T(0), v2 = T(0), v3 = T(0);
#pragma unroll
            for (int a1 = 0; a1 <= PP; ++a1) {
                if (RAT) v0 += b1[a1] * ub[a1];
                v1 += d1[a1] * ub[a1];
                v2 += b1[a1] * u2[a1];
                v3 += b1[a1] * u3[a1];
            }
            T F0 = T(0), F1, F2, F3;
            if (RAT) {
                const T g00 = Gr[j1], g01 = Gr[nqp + j1], g02 = Gr[2 * nqp + j1], g03 = Gr[3 * nqp + j1];
                const T g11 = Gr[4 * nqp + j1], g12 = Gr[5 * nqp + j1], g13 = Gr[6 * nqp + j1];
                const T g22 = Gr[7 * nqp + j1], g23 = Gr[8 * nqp + j1], g33 = Gr[9 * nqp + j1];
                F0 = g00 * v0 + g01 * v1 + g02 * v2 + g03 * v3;
                F1 = g01 * v0 + g11 * v1 + g12 * v2 + g13 * v3;
                F2 = g02 * v0 + g12 * v1 + g22 * v2 + g23 * v3;
                F3 = g03 * v0 + g13 * v1 + g23 * v2 + g33 * v3;
            } else {
                const T g11 = Gr[j1], g12 = Gr[nqp + j1], g13 = Gr[2 * nqp + j1];
                const T g22 = Gr[3 * nqp + j1], g23 = Gr[4 * nqp + j1], g33 = Gr[5 * nqp + j1];
                F1 = g11 * v1 + g12 * v2 + g13 * v3;
                F2 = g12 * v1 + g22 * v2 + g23 * v3;
                F3 = g13 * v1 + g23 * v2 + g33 * v3;
            }
#pragma unroll
            for (int a1 = 0; a1 <= PP; ++a1) {
                w0[a1] += (RAT ? b1[a1] * F0 : T(0)) + d1[a1] * F1;  // tested by B2 B3 (value in 2, 3)
                w2[a1] += b1[a1] * F2;                               // tested by D2 B3
                w3[a1] += b1[a1] * F3;                               // tested by B2 D3
            }
        }
#pragma unroll
        for (int a2 = 0; a2 <= PP; ++a2)
#pragma unroll
            for (int a1 = 0; a1 <= PP; ++a1) {
                Zb[a1][a2] += b2[a2] * w0[a1] + d2[a2] * w2[a1];
                Zd[a1][a2] += b2[a2] * w3[a1];
            }
    }
}

// The FP64 element layer of the residual sweeps with fewer live registers:
// instead of accumulating the (p+1)^2 x 2 partial sums Zb, Zd over the rows
// j2 and expanding them by the direction-3 factors at the end, each row's
// contributions are expanded, summed over the element's NG layer lanes in the
// same order and added to the element's outputs Ye in LDS at once (lane j3
// accumulates the outputs of a3 = j3; the rows in order, so the sums are
// reproducible).  Same
// arithmetic as elem_layer_3d followed by the expansion, grouped by rows.
template <int PP, bool RAT>
__device__ __forceinline__ void elem_layer_3d_rows(const double* X, int nh1, int nh2, int x1, int x2, int x3,
                                                   const double* B1, const double* D1, const double* B2,
                                                   const double* D2, const double* B3r, const double* D3r,
                                                   const double* Gl, int64_t nqp, int Q1, int j3, double* Ye) {
    constexpr int NQ = PP + 1;
    constexpr int NG = NQ <= 2 ? 2 : (NQ <= 4 ? 4 : 8);
    double tb[PP + 1][PP + 1], td[PP + 1][PP + 1], b3[PP + 1], d3[PP + 1];
#pragma unroll
    for (int a = 0; a <= PP; ++a) {
        b3[a] = B3r[a];
        d3[a] = D3r[a];
    }
#pragma unroll
    for (int a2 = 0; a2 <= PP; ++a2)
#pragma unroll
        for (int a1 = 0; a1 <= PP; ++a1) {
            double u = 0.0, v = 0.0;
#pragma unroll
            for (int a3 = 0; a3 <= PP; ++a3) {
                const double c = X[((x3 + a3) * nh2 + x2 + a2) * nh1 + x1 + a1];
                u += b3[a3] * c;
                v += d3[a3] * c;
            }
            tb[a1][a2] = u;
            td[a1][a2] = v;
        }
#pragma unroll 1
    for (int j2 = 0; j2 < NQ; ++j2) {
        double b2[PP + 1], d2[PP + 1];
#pragma unroll
        for (int a = 0; a <= PP; ++a) {
            b2[a] = B2[j2 * NQ + a];
            d2[a] = D2[j2 * NQ + a];
        }
        double ub[PP + 1], u2[PP + 1], u3[PP + 1];
#pragma unroll
        for (int a1 = 0; a1 <= PP; ++a1) {
            double s0 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
            for (int a2 = 0; a2 <= PP; ++a2) {
                s0 += b2[a2] * tb[a1][a2];
                s2 += d2[a2] * tb[a1][a2];
                s3 += b2[a2] * td[a1][a2];
            }
            ub[a1] = s0;
            u2[a1] = s2;
            u3[a1] = s3;
        }
        double w0[PP + 1], w2[PP + 1], w3[PP + 1];
#pragma unroll
        for (int a1 = 0; a1 <= PP; ++a1) w0[a1] = w2[a1] = w3[a1] = 0.0;
        const double* Gr = Gl + static_cast<int64_t>(j2) * Q1;
#pragma unroll 1
        for (int j1 = 0; j1 < NQ; ++j1) {
            double b1[PP + 1], d1[PP + 1];
#pragma unroll
            for (int a = 0; a <= PP; ++a) {
                b1[a] = B1[j1 * NQ + a];
                d1[a] = D1[j1 * NQ + a];
            }
            double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
#pragma unroll
            for (int a1 = 0; a1 <= PP; ++a1) {
                if (RAT) v0 += b1[a1] * ub[a1];
                v1 += d1[a1] * ub[a1];
                v2 += b1[a1] * u2[a1];
                v3 += b1[a1] * u3[a1];
            }
            double F0 = 0.0, F1, F2, F3;
            if (RAT) {
                const double g00 = Gr[j1], g01 = Gr[nqp + j1], g02 = Gr[2 * nqp + j1], g03 = Gr[3 * nqp + j1];
                const double g11 = Gr[4 * nqp + j1], g12 = Gr[5 * nqp + j1], g13 = Gr[6 * nqp + j1];
                const double g22 = Gr[7 * nqp + j1], g23 = Gr[8 * nqp + j1], g33 = Gr[9 * nqp + j1];
                F0 = g00 * v0 + g01 * v1 + g02 * v2 + g03 * v3;
                F1 = g01 * v0 + g11 * v1 + g12 * v2 + g13 * v3;
                F2 = g02 * v0 + g12 * v1 + g22 * v2 + g23 * v3;
                F3 = g03 * v0 + g13 * v1 + g23 * v2 + g33 * v3;
            } else {
                const double g11 = Gr[j1], g12 = Gr[nqp + j1], g13 = Gr[2 * nqp + j1];
                const double g22 = Gr[3 * nqp + j1], g23 = Gr[4 * nqp + j1], g33 = Gr[5 * nqp + j1];
                F1 = g11 * v1 + g12 * v2 + g13 * v3;
                F2 = g12 * v1 + g22 * v2 + g23 * v3;
                F3 = g13 * v1 + g23 * v2 + g33 * v3;
            }
#pragma unroll
            for (int a1 = 0; a1 <= PP; ++a1) {
                w0[a1] += (RAT ? b1[a1] * F0 : 0.0) + d1[a1] * F1;
                w2[a1] += b1[a1] * F2;
                w3[a1] += b1[a1] * F3;
            }
        }
        // this row's share of the outputs, summed over the layer lanes; lane
        // j3 keeps and accumulates the outputs of a3 = j3
#pragma unroll
        for (int a2 = 0; a2 < NQ; ++a2)
#pragma unroll
            for (int a1 = 0; a1 < NQ; ++a1) {
                double c[NG];
#pragma unroll
                for (int a3 = 0; a3 < NG; ++a3)
                    c[a3] = a3 < NQ && j3 < NQ
                                ? b3[a3] * (b2[a2] * w0[a1] + d2[a2] * w2[a1]) + d3[a3] * (b2[a2] * w3[a1])
                                : 0.0;
                const double v = group_reduce_scatter<NG>(c, j3);
                if (j3 < NQ) {
                    double* y = Ye + a1 + NQ * (a2 + NQ * j3);
                    *y = j2 == 0 ? v : *y + v;
                }
                // one output at a time: keeps the scheduler from interleaving
                // all of them, which would exceed the register budget
                __builtin_amdgcn_sched_barrier(0);
            }
    }
}

// ROWS64: the FP64 element layers by rows (elem_layer_3d_rows), for builds
// whose register budget the accumulating form exceeds (two workgroups per
// CU); the FP64-only solve keeps the accumulating form (fewer shuffles).
template <int PP, bool ROWS64 = false>
__device__ __forceinline__ void op_tile_3d(const Params& P, const Grid& g, const Tab1D& T1, const Tab1D& T2,
                                           const Tab1D& T3, int tile, const OpIO& io, double* lds) {
    constexpr int NQ = PP + 1;
    constexpr int NG = NQ <= 2 ? 2 : (NQ <= 4 ? 4 : 8);
    constexpr int NE = NQ * NQ * NQ;
    const int p = PP;
    const int m1 = T1.m, m2 = T2.m, m3 = T3.m;
    int r12;
    const int t3 = FDiv(g.ntd[0] * g.ntd[1]).div(tile, &r12);
    int t1;
    const int t2 = FDiv(g.ntd[0]).div(r12, &t1);
    const int a1 = t1 * g.tile[0], b1 = min(g.ni[0], a1 + g.tile[0]);
    const int a2 = t2 * g.tile[1], b2 = min(g.ni[1], a2 + g.tile[1]);
    const int a3 = t3 * g.tile[2], b3 = min(g.ni[2], a3 + g.tile[2]);
    int el1, eh1, el2, eh2, el3, eh3;
    d_elem_range(a1, b1, p, m1, g.E[0], T1.lo, &el1, &eh1);
    d_elem_range(a2, b2, p, m2, g.E[1], T2.lo, &el2, &eh2);
    d_elem_range(a3, b3, p, m3, g.E[2], T3.lo, &el3, &eh3);
    const int ne1 = eh1 - el1 + 1, ne2 = eh2 - el2 + 1, ne3 = eh3 - el3 + 1;
    const int hl1 = el1 * m1 - T1.lo, hl2 = el2 * m2 - T2.lo, hl3 = el3 * m3 - T3.lo;
    const int nh1 = eh1 * m1 + p - T1.lo - hl1 + 1, nh2 = eh2 * m2 + p - T2.lo - hl2 + 1,
              nh3 = eh3 * m3 + p - T3.lo - hl3 + 1;
    double* X = lds;
    double* Y = lds + nh1 * nh2 * nh3;
    double* red = Y + ne1 * ne2 * ne3 * NE;
    // FP32 element arithmetic: an FP32 copy of the halo block after red
    float* Xf = reinterpret_cast<float*>(red + kWaves);
    const int64_t off = g.dof_off;
    const int n1 = g.ni[0], n2 = g.ni[1], n3 = g.ni[2];
    {
        const FDiv dh1(nh1), dh12(nh1 * nh2);
        for (int idx = threadIdx.x; idx < nh1 * nh2 * nh3; idx += kBlock) {
            int r, q1;
            const int q2 = dh12.div(idx, &r);
            q1 = dh1.div(r, &r);
            const int i1 = hl1 + r, i2 = hl2 + q1, i3 = hl3 + q2;
            double v = 0.0;
            if (i1 >= 0 && i1 < n1 && i2 >= 0 && i2 < n2 && i3 >= 0 && i3 < n3) {
                const int64_t gi = off + (static_cast<int64_t>(i3) * n2 + i2) * n1 + i1;
                v = io.in_a[gi];
                if (io.in_b) v += io.beta * io.in_b[gi];
                if (io.out_in && i1 >= a1 && i1 < b1 && i2 >= a2 && i2 < b2 && i3 >= a3 && i3 < b3)
                    io.out_in[gi] = v;
            }
            X[idx] = v;
            if (io.lowp) Xf[idx] = static_cast<float>(v);
        }
    }
    __syncthreads();
    const int nqp1 = NQ * NQ;
    const int64_t nqp = g.nqp;
    const FDiv de1(ne1), de12(ne1 * ne2);
    const bool rat = P.rational[g.patch] != 0;
    const int nitem = ne1 * ne2 * ne3 * NG;
    for (int it = threadIdx.x; it < nitem; it += kBlock) {
        const int el = it / NG, j3 = it & (NG - 1);
        int r, q1;
        const int q2 = de12.div(el, &r);
        q1 = de1.div(r, &r);
        const int e1 = el1 + r, e2 = el2 + q1, e3 = el3 + q2;
        const int x1 = e1 * m1 - T1.lo - hl1, x2 = e2 * m2 - T2.lo - hl2, x3 = e3 * m3 - T3.lo - hl3;
        const int jr = j3 < NQ ? j3 : 0;
        const double* B1 = P.dpool + T1.oB + static_cast<int64_t>(e1) * nqp1;
        const double* D1 = P.dpool + T1.oD + static_cast<int64_t>(e1) * nqp1;
        const double* B2 = P.dpool + T2.oB + static_cast<int64_t>(e2) * nqp1;
        const double* D2 = P.dpool + T2.oD + static_cast<int64_t>(e2) * nqp1;
        const double* B3r = P.dpool + T3.oB + static_cast<int64_t>(e3) * nqp1 + jr * NQ;
        const double* D3r = P.dpool + T3.oD + static_cast<int64_t>(e3) * nqp1 + jr * NQ;
        // coefficients of layer jr of the element (element-major storage: the
        // layer's NQ x NQ points contiguous, direction 1 fastest)
        const int64_t ql = ((static_cast<int64_t>(e3) * g.E[1] + e2) * g.E[0] + e1) * NE + jr * NQ * NQ;
        double* Ye = Y + el * NE;
        // the layers' shares of output (a1, a2, a3) summed over the NG lanes
        // of the element; lane j3 keeps and writes the outputs of a3 = j3
        auto finish = [&](auto& Zb, auto& Zd, auto& b3v, auto& d3v) {
            using TV = typename std::remove_reference<decltype(b3v[0])>::type;
#pragma unroll
            for (int a2 = 0; a2 < NQ; ++a2)
#pragma unroll
                for (int a1 = 0; a1 < NQ; ++a1) {
                    TV c[NG];
#pragma unroll
                    for (int a3 = 0; a3 < NG; ++a3)
                        c[a3] = a3 < NQ && j3 < NQ ? b3v[a3] * Zb[a1][a2] + d3v[a3] * Zd[a1][a2] : TV(0);
                    const TV v = group_reduce_scatter<NG>(c, j3);
                    if (j3 < NQ) Ye[a1 + NQ * (a2 + NQ * j3)] = static_cast<double>(v);
                }
        };
        if (io.lowp) {
            float Zb[NQ][NQ], Zd[NQ][NQ], b3v[NQ], d3v[NQ];
            const float* Gl = P.G32 + g.qp_off * P.ncompG + ql;
            if (rat) elem_layer_3d<PP, true, float>(Xf, nh1, nh2, x1, x2, x3, B1, D1, B2, D2, B3r, D3r, Gl, nqp, NQ, Zb, Zd, b3v, d3v);
            else elem_layer_3d<PP, false, float>(Xf, nh1, nh2, x1, x2, x3, B1, D1, B2, D2, B3r, D3r, Gl, nqp, NQ, Zb, Zd, b3v, d3v);
            finish(Zb, Zd, b3v, d3v);
        } else {
            const double* Gl = P.G64 + g.qp_off * P.ncompG + ql;
            if constexpr (ROWS64) {
                if (rat) elem_layer_3d_rows<PP, true>(X, nh1, nh2, x1, x2, x3, B1, D1, B2, D2, B3r, D3r, Gl, nqp, NQ, j3, Ye);
                else elem_layer_3d_rows<PP, false>(X, nh1, nh2, x1, x2, x3, B1, D1, B2, D2, B3r, D3r, Gl, nqp, NQ, j3, Ye);
            } else {
                double Zb[NQ][NQ], Zd[NQ][NQ], b3v[NQ], d3v[NQ];
                if (rat) elem_layer_3d<PP, true, double>(X, nh1, nh2, x1, x2, x3, B1, D1, B2, D2, B3r, D3r, Gl, nqp, NQ, Zb, Zd, b3v, d3v);
                else elem_layer_3d<PP, false, double>(X, nh1, nh2, x1, x2, x3, B1, D1, B2, D2, B3r, D3r, Gl, nqp, NQ, Zb, Zd, b3v, d3v);
                finish(Zb, Zd, b3v, d3v);
            }
        }
    }
    __syncthreads();
    const int w1 = b1 - a1, w2 = b2 - a2, nown = w1 * w2 * (b3 - a3);
    double dot = 0.0;
    const FDiv dw1(w1), dw12(w1 * w2);
    for (int o = threadIdx.x; o < nown; o += kBlock) {
        int r, q1;
        const int q2 = dw12.div(o, &r);
        q1 = dw1.div(r, &r);
        const int i1 = a1 + r, i2 = a2 + q1, i3 = a3 + q2;
        int lo1, hi1, lo2, hi2, lo3, hi3;
        d_elem_range(i1, i1 + 1, p, m1, g.E[0], T1.lo, &lo1, &hi1);
        d_elem_range(i2, i2 + 1, p, m2, g.E[1], T2.lo, &lo2, &hi2);
        d_elem_range(i3, i3 + 1, p, m3, g.E[2], T3.lo, &lo3, &hi3);
        // the contributions of the support's elements, e3 and e2 outer, e1 inner
        // (at most NQ elements a direction); the e1 run unrolled to NQ with the
        // elements past hi1 adding 0, so that its loads are issued together
        double s = 0.0;
        const int d1 = hi1 - lo1;
        for (int e3 = lo3; e3 <= hi3; ++e3)
            for (int e2 = lo2; e2 <= hi2; ++e2) {
                const int el = ((e3 - el3) * ne2 + (e2 - el2)) * ne1 + (lo1 - el1);
                const int base = el * NE + (i1 + T1.lo - lo1 * m1) +
                                 NQ * ((i2 + T2.lo - e2 * m2) + NQ * (i3 + T3.lo - e3 * m3));
#pragma unroll
                for (int t1 = 0; t1 < NQ; ++t1) {
                    // element lo1 + t1: element index + 1, local index - m1
                    const double v = Y[t1 <= d1 ? base + t1 * (NE - m1) : base];
                    s += t1 <= d1 ? v : 0.0;
                }
            }
        const int64_t gi = off + (static_cast<int64_t>(i3) * n2 + i2) * n1 + i1;
        if (io.rhs) {
            s = io.rhs[gi] - s;
            dot += s * s;
        } else {
            dot += X[((i3 - hl3) * nh2 + (i2 - hl2)) * nh1 + (i1 - hl1)] * s;
        }
        io.out[gi] = s;
    }
    if (io.part) {
        const double t = wg_sum(dot, red);
        if (threadIdx.x == 0) *io.part = t;
    }
    __syncthreads();
}

// ===========================================================================
// fast diagonalisation: z = (U1 (x) U2) diag(1/(c1 l1 + c2 l2)) (U1 (x) U2)^T r
// as mode products
// ===========================================================================
// C[m][n] = sum_k A(m, k) B(k, n) on the matrix cores, operands addressed by
// strides (A(m, k) = A[m sAm + k sAk], ...), nb independent products at batch
// strides.  Each wavefront takes 16 x 16 output tiles in turn and walks K in
// steps of 4 with the 16x16x4 MFMA (FP64 for TC = double, FP32 for TC =
// float), two accumulator chains (even and odd steps) in flight; with BF16
// factors (an operand of type uint16_t) in steps of 32 with the 16x16x32 BF16
// MFMA, the other operand rounded to BF16 and the products accumulated in
// FP32 (lane l supplies A(16 t_m + l % 16, k + 8 (l / 16) + j) and
// B(k + 8 (l / 16) + j, 16 t_n + l % 16), j < 8).  Lane l supplies A(16 t_m + l % 16, k + l / 16) and
// B(k + l / 16, 16 t_n + l % 16); out-of-range operands are zero.  The
// accumulation order is fixed, so results are reproducible.  E (optional):
// each output multiplied by E at the output's index in C (a diagonal scaling
// in the epilogue).  Ends with a workgroup barrier.
typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef double v4d_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
template <typename TC> struct Mfma;
template <> struct Mfma<double> {
    using V = v4d_t;
    static __device__ __forceinline__ V step(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // row of accumulator entry r held by a lane (its column is lane % 16)
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mfma<float> {
    using V = v4f_t;
    static __device__ __forceinline__ V step(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <typename TC, typename T>
__device__ __forceinline__ TC mm_ld(const T* p, int i) {
    if constexpr (std::is_same<T, uint16_t>::value) return static_cast<TC>(bf16_to_f32(p[i]));
    else return static_cast<TC>(p[i]);
}
template <typename TA, typename TB, typename TC>
__device__ __forceinline__ void mfma_gemm(int M, int N, int K, const TA* A, int sAm, int sAk, const TB* B, int sBk,
                                          int sBn, double* C, int sCm, int sCn, int nb = 1, int sAb = 0,
                                          int sBb = 0, int sCb = 0, double* red = nullptr,
                                          const double* E = nullptr) {
    using MF = Mfma<TC>;
    using V = typename MF::V;
    constexpr bool kBf = std::is_same<TA, uint16_t>::value || std::is_same<TB, uint16_t>::value;
    // Small FP64/FP32 products (K <= 64 and at most 64 multiply-adds per
    // thread of the workgroup): one output per thread on the vector units, in
    // the same precision TC, with K in order.  The short directions of the
    // component grids (2 to about 33 unknowns) would leave the 16 x 16
    // matrix-core tiles mostly padding and spend the product on operand
    // staging and the split-K reduction; long contractions (a long direction
    // of a 2D grid, full grids) stay on the matrix cores.
    if (!kBf && K <= 64 && static_cast<int64_t>(M) * N * nb * K <= 64 * kBlock) {
        const int mn = M * N, tot = mn * nb;
        const FDiv dmn(mn), dn(N);
        for (int o = threadIdx.x; o < tot; o += kBlock) {
            int r, n;
            const int bt = dmn.div(o, &r);
            const int m = dn.div(r, &n);
            const TA* Ar = A + bt * sAb + m * sAm;
            const TB* Bc = B + bt * sBb + n * sBn;
            TC acc = TC(0);
            for (int k = 0; k < K; ++k) acc = fma(mm_ld<TC>(Ar, k * sAk), mm_ld<TC>(Bc, k * sBk), acc);
            const int ci = bt * sCb + m * sCm + n * sCn;
            C[ci] = E ? static_cast<double>(acc) * E[ci] : static_cast<double>(acc);
        }
        __syncthreads();
        return;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int tm = (M + 15) >> 4, tn = (N + 15) >> 4, tmn = tm * tn, units = tmn * nb;
    // fewer tiles than wavefronts: K is cut into ks slices whose partial tiles
    // are summed in slice order through red (ks * M * N <= kBigRed doubles)
    int ks = 1;
    if (red && nb == 1)
        while (2 * ks * units <= kWaves && 2 * ks * M * N <= kBigRed && K >= 16 * ks) ks *= 2;
    const int kc = kBf ? (((K + ks - 1) / ks + 31) & ~31) : (((K + ks - 1) / ks + 7) & ~7);
    for (int w = wave; w < units * ks; w += kWaves) {  // uniform per wavefront
        const int u = w / ks, sl = w - u * ks;
        const int bt = u / tmn, t = u - bt * tmn;
        const int ti = t / tn, tj = t - ti * tn;
        const TA* Ab = A + bt * sAb;
        const TB* Bb = B + bt * sBb;
        double* Cb = C + bt * sCb;
        const int i = 16 * ti + li, j = 16 * tj + li;
        const bool iv = i < M, jv = j < N;
        const int kb0 = sl * kc, kb1 = min(K, kb0 + kc);
        V acc0 = {TC(0), TC(0), TC(0), TC(0)};
        V acc1 = acc0;
        if constexpr (kBf) {
            static_assert(std::is_same<TC, float>::value, "BF16 products accumulate in FP32");
            for (int k0 = kb0; k0 < kb1; k0 += 32) {
                bf16x8_t av, bv;
#pragma unroll
                for (int jj = 0; jj < 8; ++jj) {
                    const int k = k0 + 8 * lk + jj;
                    const bool kin = k < kb1;
                    av[jj] = static_cast<__bf16>(iv && kin ? mm_ld<float>(Ab, i * sAm + k * sAk) : 0.0f);
                    bv[jj] = static_cast<__bf16>(jv && kin ? mm_ld<float>(Bb, k * sBk + j * sBn) : 0.0f);
                }
                acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc0, 0, 0, 0);
            }
        } else
        for (int k0 = kb0; k0 < kb1; k0 += 8) {
            const int ka = k0 + lk, kb = k0 + 4 + lk;
            const TC a0 = iv && ka < kb1 ? mm_ld<TC>(Ab, i * sAm + ka * sAk) : TC(0);
            const TC b0 = jv && ka < kb1 ? mm_ld<TC>(Bb, ka * sBk + j * sBn) : TC(0);
            const TC a1 = iv && kb < kb1 ? mm_ld<TC>(Ab, i * sAm + kb * sAk) : TC(0);
            const TC b1 = jv && kb < kb1 ? mm_ld<TC>(Bb, kb * sBk + j * sBn) : TC(0);
            acc0 = MF::step(a0, b0, acc0);
            acc1 = MF::step(a1, b1, acc1);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ii = 16 * ti + MF::row(lane, r);
            if (ii < M && jv) {
                const double v = static_cast<double>(acc0[r] + acc1[r]);
                if (ks == 1) Cb[ii * sCm + j * sCn] = E ? v * E[bt * sCb + ii * sCm + j * sCn] : v;
                else red[(sl * M + ii) * N + j] = v;
            }
        }
    }
    __syncthreads();
    if (ks > 1) {
        const FDiv dN(N);
        for (int o = threadIdx.x; o < M * N; o += kBlock) {
            int n;
            const int m = dN.div(o, &n);
            double v = 0.0;
            for (int sl = 0; sl < ks; ++sl) v += red[sl * M * N + o];
            C[m * sCm + n * sCn] = E ? v * E[m * sCm + n * sCn] : v;
        }
        __syncthreads();
    }
}

__device__ __forceinline__ double load_val(const double* p, int i) { return p[i]; }
__device__ __forceinline__ float load_val(const float* p, int i) { return p[i]; }
__device__ __forceinline__ float load_val(const uint16_t* p, int i) { return bf16_to_f32(p[i]); }

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
    const double* scale;  // diagonal scaling s (z = s P^-1 (s r)), or nullptr
    // several patches (2D): interface sums of q (or of the residual in q),
    // fixed vertices kept at 0, interface unknowns weighted 1/2 in ||r||^2
    int mp = 0;
    int resq = 0;         // residual sweep: the patch-local residual b - A x is in q
    // learned preconditioner (3D backward transform only)
    int learned;
    const double* rold;   // previous residual: part2 = z . rold (flexible CG)
    double* part2;
    double* part3 = nullptr;  // r . z_FD of the plain preconditioner (learned solves: the stopping test)
    // 3D, one workgroup per grid: the forward transform leaves its output
    // (times 1 / lambda) in LDS and the residual in the backward transform's
    // dot-partner slot, so that the backward transform of the same workgroup
    // follows without reloading them (rt is then not written)
    int keep = 0;
};


// 16-byte units of the factor tables (CPL elements each).  The slab of a
// blocked long direction is copied to LDS by 16-byte lanes, thread t taking
// row t / (blk / CPL) and column group t % (blk / CPL) of each pass of
// kBlock * CPL / blk rows, which lays it out row-major, [long index][blk].
template <typename TU> struct VecU;
template <> struct VecU<double> {
    static constexpr int CPL = 2;
    using Raw = double2;
};
template <> struct VecU<float> {
    static constexpr int CPL = 4;
    using Raw = float4;
};
template <> struct VecU<uint16_t> {
    static constexpr int CPL = 8;
    using Raw = uint4;
};

// Direct global -> LDS copies (gfx950 global_load_lds): each active lane of
// a wavefront moves SIZE bytes from its own global address to
// lds_wave_base + lane * SIZE (SIZE 4 or 16 bytes); lds_wave_base is uniform
// over the wavefront.
// The copies bypass registers, so a task issues all of them back to back.
__device__ __forceinline__ void g2l4(const void* src, void* lds_wave_base) {
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds_wave_base, 4, 0, 0);
}
__device__ __forceinline__ void g2l16(const void* src, void* lds_wave_base) {
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds_wave_base, 16, 0, 0);
}
// Wait for this wavefront's outstanding copies, then for the workgroup.
__device__ __forceinline__ void g2l_wait_sync() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}
// dst[i] = src[i], i < n (FP64 values moved as dwords: 8-byte copies do not exist)
__device__ __forceinline__ void g2l_vec(const double* src, int n, double* dst) {
    const int wave = threadIdx.x >> 6, nd = 2 * n;
    const uint32_t* s = reinterpret_cast<const uint32_t*>(src);
    uint32_t* d = reinterpret_cast<uint32_t*>(dst);
    for (int base = 0; base < nd; base += kBlock)
        if (base + static_cast<int>(threadIdx.x) < nd) g2l4(s + base + threadIdx.x, d + base + wave * 64);
}
// bytes (a multiple of 16) copied as 16-byte chunks
__device__ __forceinline__ void g2l_bytes(const void* src, int bytes, void* dst) {
    const int wave = threadIdx.x >> 6, nc = bytes >> 4;
    const char* s = static_cast<const char*>(src);
    char* d = static_cast<char*>(dst);
    for (int base = 0; base < nc; base += kBlock)
        if (base + static_cast<int>(threadIdx.x) < nc)
            g2l16(s + 16 * (base + threadIdx.x), d + 16 * (base + wave * 64));
}

// Block geometry of FD task blk of a 2D grid.  Owned unknowns (index along
// the long direction inside the block) are enumerated o < nown in the order
// of the block outputs: long direction fastest for big == 0, short direction
// fastest (contiguous) for big == 1.
struct FdBlock {
    int n1, n2, n, big, nbig, nsm, k0, bs, nown;
    bool wide, sbig;  // wide: the block's slab of the long factor is staged in LDS
    FDiv dbs;
    __device__ explicit FdBlock(const Grid& g, int blk)
        : n1(g.ni[0]), n2(g.ni[1]), n(g.ni[0] * g.ni[1]), big(g.big), nbig(g.ni[g.big]), nsm(g.ni[1 - g.big]),
          k0(blk * g.blk), bs(min(g.blk, g.ni[g.big] - blk * g.blk)), nown(0), wide(g.nblk > 1 && g.fdstage >= 0),
          sbig(g.nblk <= 1 && g.fdstage != 0), dbs(min(g.blk, g.ni[g.big] - blk * g.blk)) {
        nown = nsm * bs;
    }
    __device__ __forceinline__ int gi(int o) const {
        if (big == 0) {
            int kk;
            const int i2 = dbs.div(o, &kk);
            return i2 * n1 + k0 + kk;
        }
        return k0 * n1 + o;
    }
};
// owned gather: dst[o] = src[gi(o)], o < nown (as dwords)
__device__ __forceinline__ void g2l_owned(const double* src, const FdBlock& B, double* dst) {
    const int wave = threadIdx.x >> 6, nd = 2 * B.nown;
    const uint32_t* s = reinterpret_cast<const uint32_t*>(src);
    uint32_t* d = reinterpret_cast<uint32_t*>(dst);
    for (int base = 0; base < nd; base += kBlock) {
        const int w = base + threadIdx.x;
        if (w < nd) g2l4(s + 2 * B.gi(w >> 1) + (w & 1), d + base + wave * 64);
    }
}

// LDS pointers of an FD task for factor element type TU.
template <typename TU>
struct FdLds {
    double *R, *S, *red, *Out, *Own;
    TU *Us, *Ub;
    typename VecU<TU>::Raw* Slab;
    int rows, ldu_s, ldu_b;
};
template <typename TU>
__device__ __forceinline__ FdLds<TU> fd_lds(const TaskMeta& M, double* lds) {
    const Grid& g = M.g;
    const int ls = M.t[1 - g.big].ldu, lb = M.t[g.big].ldu;
    const FdLayout Y = fd_layout(g, ls, lb, sizeof(TU));
    char* base = reinterpret_cast<char*>(lds);
    FdLds<TU> L;
    L.R = reinterpret_cast<double*>(base + Y.R);
    L.S = reinterpret_cast<double*>(base + Y.S);
    L.red = reinterpret_cast<double*>(base + Y.red);
    L.Out = reinterpret_cast<double*>(base + Y.Out);
    L.Own = reinterpret_cast<double*>(base + Y.Own);
    L.Us = reinterpret_cast<TU*>(base + Y.Us);
    L.Ub = reinterpret_cast<TU*>(base + Y.Ub);
    L.Slab = reinterpret_cast<typename VecU<TU>::Raw*>(base + Y.Slab);
    L.rows = Y.rows;
    L.ldu_s = ls;
    L.ldu_b = lb;
    return L;
}

template <typename TU>
__device__ __forceinline__ void fd_factor_ptrs(const Params& P, const TaskMeta& M, bool fwd, const TU** Us,
                                               const TU** Ub, const TU** Ubig) {
    // forward: short factor transposed (big == 0: UT2; big == 1: U1), long factor U (block columns);
    // backward: short factor (big == 0: U2; big == 1: UT1), long factor U^T (block columns);
    // single-block long factor as consumed by the second product
    const Tab1D& T1 = M.t[0];
    const Tab1D& T2 = M.t[1];
    if (M.g.big == 0) {
        *Us = u_ptr<TU>(P, T2, fwd);
        *Ub = u_ptr<TU>(P, T1, !fwd);
        *Ubig = u_ptr<TU>(P, T1, !fwd);
    } else {
        *Us = u_ptr<TU>(P, T1, !fwd);
        *Ub = u_ptr<TU>(P, T2, fwd);
        *Ubig = u_ptr<TU>(P, T2, !fwd);
    }
}

// Issue the copies of the factors an FD task reads: the short-direction
// factor, the long one of a single-block grid, the slab of a blocked grid.
template <typename TU>
__device__ __forceinline__ void fd_issue_factors(const Params& P, const TaskMeta& M, const FdBlock& B, bool fwd,
                                                 const FdLds<TU>& L) {
    const TU *Us, *Ub, *Ubig;
    fd_factor_ptrs<TU>(P, M, fwd, &Us, &Ub, &Ubig);
    g2l_bytes(Us, B.nsm * L.ldu_s * static_cast<int>(sizeof(TU)), L.Us);
    if (B.sbig) g2l_bytes(Ub, B.nbig * L.ldu_b * static_cast<int>(sizeof(TU)), L.Ub);
    if (B.wide) {
        constexpr int CPL = VecU<TU>::CPL;
        const int lpr = M.g.blk / CPL;  // lanes per row segment (power of two)
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        const int rpw = 64 / lpr, rpt = kWaves * rpw;
        const int jc = (lane & (lpr - 1)) * CPL;
        const int r0 = wave * rpw + lane / lpr;
        if (jc < B.bs) {
            const TU* ub = Ubig + B.k0 + jc;
            for (int s = 0; s < L.rows; ++s) {
                const int k = r0 + s * rpt;
                if (k < B.nbig) g2l16(ub + static_cast<int64_t>(k) * L.ldu_b, L.Slab + s * kBlock + wave * 64);
            }
        }
    }
}

// Issue the copies of a forward task: r (and q) over the grid, owned p, d and
// 1 / lambda, the factors.
template <typename TU>
__device__ __forceinline__ void fd_issue_fwd(const Params& P, const TaskMeta& M, int blk, const double* r_src,
                                             const double* q_src, const double* p_src, const double* d_src,
                                             double* lds) {
    const Grid& g = M.g;
    const FdBlock B(g, blk);
    const FdLds<TU> L = fd_lds<TU>(M, lds);
    const int64_t off = g.dof_off;
    g2l_vec(r_src + off, B.n, L.R);
    if (q_src) g2l_vec(q_src + off, B.n, L.S);
    if (p_src) g2l_owned(p_src + off, B, L.Own);
    if (d_src) g2l_owned(d_src + off, B, L.Own + B.nown);
    g2l_owned(P.dpool + g.oDinv, B, L.Own + 2 * B.nown);
    fd_issue_factors<TU>(P, M, B, true, L);
}

template <typename TU>
__device__ __forceinline__ void fd_issue_bwd(const Params& P, const TaskMeta& M, int blk, const double* rt_src,
                                             const double* rdot, double* lds) {
    const Grid& g = M.g;
    const FdBlock B(g, blk);
    const FdLds<TU> L = fd_lds<TU>(M, lds);
    const int64_t off = g.dof_off;
    g2l_vec(rt_src + off, B.n, L.R);
    if (rdot) g2l_owned(rdot + off, B, L.Own);
    fd_issue_factors<TU>(P, M, B, false, L);
}

// Forward transform of one FD block, after fd_issue_fwd and g2l_wait_sync:
//   r = r_old - alpha q (grid, LDS), owned: r_out = r, d += alpha p,
//   part = ||r_owned||^2, Rt = (U1 (x) U2)^T r on the block times 1 / lambda.
template <typename TU, typename TC>
__device__ __forceinline__ void fd_fwd_run(const Params& P, const TaskMeta& M, int blk, const FdIO& io,
                                           double* lds) {
    const Grid& g = M.g;
    const FdBlock B(g, blk);
    const FdLds<TU> L = fd_lds<TU>(M, lds);
    const int64_t off = g.dof_off;
    const int n1 = B.n1, n2 = B.n2;
    const TU *Us, *Ub, *Ubig;
    fd_factor_ptrs<TU>(P, M, true, &Us, &Ub, &Ubig);
    if (io.mp) {
        // interface sums of q (r = r_old - alpha q) or of the residual itself
        const FDiv d1(n1);
        for (int i = threadIdx.x; i < B.n; i += kBlock) {
            int i1;
            const int i2 = d1.div(i, &i1);
            const double qv = iface_add(g, io.q, i1, i2, L.S[i]);
            const double v = io.resq ? qv : L.R[i] - io.alpha * qv;
            L.S[i] = v;
            // Neumann-Neumann weights: an interface unknown's residual is
            // shared half and half by the two patch solves (and so is their
            // correction, in the backward transform)
            const double wv = iface_side(g, i1, i2) >= 0 ? 0.5 : 1.0;
            L.R[i] = (io.scale ? v * io.scale[off + i] : v) * wv;
        }
    } else if (io.scale) {
        // the update in S (written out below), the scaled residual s r in R
        for (int i = threadIdx.x; i < B.n; i += kBlock) {
            const double v = io.q ? L.R[i] - io.alpha * L.S[i] : L.R[i];
            L.S[i] = v;
            L.R[i] = v * io.scale[off + i];
        }
    } else if (io.q) {
        for (int i = threadIdx.x; i < B.n; i += kBlock) L.R[i] -= io.alpha * L.S[i];
    }
    __syncthreads();
    const double* Ru = (io.scale || io.mp) ? L.S : L.R;
    const double* Pw = L.Own;
    const double* Dw = L.Own + B.nown;
    const double* Iw = L.Own + 2 * B.nown;
    double nrm = 0.0;
    for (int o = threadIdx.x; o < B.nown; o += kBlock) {
        const int gi = B.gi(o);
        const double v = Ru[gi];
        if (io.r_out) io.r_out[off + gi] = v;
        if (io.dvec) io.dvec[off + gi] = Dw[o] + io.alpha * Pw[o];
        // an interface unknown has a copy in both patches: half weight each
        const double wgt = io.mp && iface_side(g, gi % n1, gi / n1) >= 0 ? 0.5 : 1.0;
        nrm += wgt * v * v;
    }
    if (io.part) {
        const double t = wg_sum(nrm, L.red);
        if (threadIdx.x == 0) *io.part = t;
    }
    __syncthreads();
    const int k0 = B.k0, bs = B.bs, ls = L.ldu_s, lb = L.ldu_b;
    if (B.big == 0) {
        // S[k2][i1] = sum_i2 UT2[k2][i2] R[i2][i1]
        mfma_gemm<TU, double, TC>(n2, n1, n2, L.Us, ls, 1, L.R, n1, 1, L.S, n1, 1, 1, 0, 0, 0, L.red);
        // Rt[k2][k1] = sum_i1 S[k2][i1] U1[i1][k1], k1 in block
        if (B.wide)
            mfma_gemm<double, TU, TC>(n2, bs, n1, L.S, n1, 1, reinterpret_cast<const TU*>(L.Slab), g.blk, 1, L.Out, bs, 1, 1, 0, 0, 0, L.red);
        else if (B.sbig)
            mfma_gemm<double, TU, TC>(n2, bs, n1, L.S, n1, 1, L.Ub + k0, lb, 1, L.Out, bs, 1, 1, 0, 0, 0, L.red);
        else
            mfma_gemm<double, TU, TC>(n2, bs, n1, L.S, n1, 1, Ubig + k0, lb, 1, L.Out, bs, 1, 1, 0, 0, 0, L.red);
    } else {
        // S[i2][k1] = sum_i1 R[i2][i1] U1[i1][k1]
        mfma_gemm<double, TU, TC>(n2, n1, n1, L.R, n1, 1, L.Us, ls, 1, L.S, n1, 1, 1, 0, 0, 0, L.red);
        // Rt[k2][k1] = sum_i2 U2[i2][k2] S[i2][k1], k2 in block
        if (B.wide)
            mfma_gemm<double, TU, TC>(n1, bs, n2, L.S, 1, n1, reinterpret_cast<const TU*>(L.Slab), g.blk, 1, L.Out, 1, n1, 1, 0, 0, 0, L.red);
        else if (B.sbig)
            mfma_gemm<TU, double, TC>(bs, n1, n2, L.Ub + static_cast<int64_t>(k0) * lb, lb, 1, L.S, n1, 1, L.Out, n1, 1, 1, 0, 0, 0, L.red);
        else
            mfma_gemm<TU, double, TC>(bs, n1, n2, Ub + static_cast<int64_t>(k0) * lb, lb, 1, L.S, n1, 1, L.Out, n1, 1, 1, 0, 0, 0, L.red);
    }
    for (int o = threadIdx.x; o < B.nown; o += kBlock) io.rt[off + B.gi(o)] = L.Out[o] * Iw[o];
    __syncthreads();
}

// Backward transform of one FD block, after fd_issue_bwd and g2l_wait_sync:
// z = (U1 (x) U2) Rt on the block; part = rdot . z over the block.
template <typename TU, typename TC>
__device__ __forceinline__ void fd_bwd_run(const Params& P, const TaskMeta& M, int blk, const FdIO& io,
                                           double* lds) {
    const Grid& g = M.g;
    const FdBlock B(g, blk);
    const FdLds<TU> L = fd_lds<TU>(M, lds);
    const int64_t off = g.dof_off;
    const int n1 = B.n1, n2 = B.n2;
    const TU *Us, *Ub, *Ubig;
    fd_factor_ptrs<TU>(P, M, false, &Us, &Ub, &Ubig);
    double* Rt = L.R;
    double* Tm = L.S;
    const int k0 = B.k0, bs = B.bs, ls = L.ldu_s, lb = L.ldu_b;
    if (B.big == 0) {
        // T[i2][k1] = sum_k2 U2[i2][k2] Rt[k2][k1]
        mfma_gemm<TU, double, TC>(n2, n1, n2, L.Us, ls, 1, Rt, n1, 1, Tm, n1, 1, 1, 0, 0, 0, L.red);
        // Z[i2][i1] = sum_k1 T[i2][k1] UT1[k1][i1], i1 in block
        if (B.wide)
            mfma_gemm<double, TU, TC>(n2, bs, n1, Tm, n1, 1, reinterpret_cast<const TU*>(L.Slab), g.blk, 1, L.Out, bs, 1, 1, 0, 0, 0, L.red);
        else if (B.sbig)
            mfma_gemm<double, TU, TC>(n2, bs, n1, Tm, n1, 1, L.Ub + k0, lb, 1, L.Out, bs, 1, 1, 0, 0, 0, L.red);
        else
            mfma_gemm<double, TU, TC>(n2, bs, n1, Tm, n1, 1, Ubig + k0, lb, 1, L.Out, bs, 1, 1, 0, 0, 0, L.red);
    } else {
        // T[k2][i1] = sum_k1 Rt[k2][k1] UT1[k1][i1]
        mfma_gemm<double, TU, TC>(n2, n1, n1, Rt, n1, 1, L.Us, ls, 1, Tm, n1, 1, 1, 0, 0, 0, L.red);
        // Z[i2][i1] = sum_k2 UT2[k2][i2] T[k2][i1], i2 in block
        if (B.wide)
            mfma_gemm<double, TU, TC>(n1, bs, n2, Tm, 1, n1, reinterpret_cast<const TU*>(L.Slab), g.blk, 1, L.Out, 1, n1, 1, 0, 0, 0, L.red);
        else if (B.sbig)
            mfma_gemm<TU, double, TC>(bs, n1, n2, L.Ub + static_cast<int64_t>(k0) * lb, lb, 1, Tm, n1, 1, L.Out, n1, 1, 1, 0, 0, 0, L.red);
        else
            mfma_gemm<TU, double, TC>(bs, n1, n2, Ub + static_cast<int64_t>(k0) * lb, lb, 1, Tm, n1, 1, L.Out, n1, 1, 1, 0, 0, 0, L.red);
    }
    double dot = 0.0;
    const double* Rd = L.Own;
    for (int o = threadIdx.x; o < B.nown; o += kBlock) {
        const int64_t gi = off + B.gi(o);
        double zv = io.scale ? L.Out[o] * io.scale[gi] : L.Out[o];
        if (io.mp) {
            const int lo = B.gi(o);
            if (iface_pinned(g, lo)) zv = 0.0;  // a fixed vertex stays at its value
            else if (iface_side(g, lo % n1, lo / n1) >= 0) zv *= 0.5;  // Neumann-Neumann weight
        }
        io.z[gi] = zv;
        if (io.rdot) dot += Rd[o] * zv;
    }
    if (io.part) {
        const double t = wg_sum(dot, L.red);
        if (threadIdx.x == 0) *io.part = t;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// 3D fast diagonalisation: one task per grid, the three factors staged in LDS,
// six mode products (mfma_gemm; the middle one batched over direction 3).
// ---------------------------------------------------------------------------
template <typename TU>
struct Fd3Lds {
    double *R, *S, *T, *red, *Own;
    const TU *U1, *U2, *U3;  // LDS copies, or the tables in global memory when not staged
    int ld1, ld2, ld3;
};
template <typename TU>
__device__ __forceinline__ Fd3Lds<TU> fd3_lds(const Params& P, const TaskMeta& M, double* lds) {
    const int ld[3] = {M.t[0].ldu, M.t[1].ldu, M.t[2].ldu};
    const FdLayout Y = fd_layout_3d(M.g, ld, sizeof(TU));
    char* base = reinterpret_cast<char*>(lds);
    Fd3Lds<TU> L;
    L.R = reinterpret_cast<double*>(base + Y.R);
    L.S = reinterpret_cast<double*>(base + Y.S);
    L.T = reinterpret_cast<double*>(base + Y.Out);
    L.red = reinterpret_cast<double*>(base + Y.red);
    L.Own = reinterpret_cast<double*>(base + Y.Own);
    const int st = M.g.fdstage;
    L.U1 = (st & 1) ? reinterpret_cast<const TU*>(base + Y.Us) : u_ptr<TU>(P, M.t[0], false);
    L.U2 = (st & 2) ? reinterpret_cast<const TU*>(base + Y.Ub) : u_ptr<TU>(P, M.t[1], false);
    L.U3 = (st & 4) ? reinterpret_cast<const TU*>(base + Y.Slab) : u_ptr<TU>(P, M.t[2], false);
    L.ld1 = ld[0];
    L.ld2 = ld[1];
    L.ld3 = ld[2];
    return L;
}
template <typename TU>
__device__ __forceinline__ void fd3_issue_factors(const Params& P, const TaskMeta& M, const Fd3Lds<TU>& L) {
    const int us = static_cast<int>(sizeof(TU));
    const int st = M.g.fdstage;
    if (st & 1) g2l_bytes(u_ptr<TU>(P, M.t[0], false), M.g.ni[0] * L.ld1 * us, const_cast<TU*>(L.U1));
    if (st & 2) g2l_bytes(u_ptr<TU>(P, M.t[1], false), M.g.ni[1] * L.ld2 * us, const_cast<TU*>(L.U2));
    if (st & 4) g2l_bytes(u_ptr<TU>(P, M.t[2], false), M.g.ni[2] * L.ld3 * us, const_cast<TU*>(L.U3));
}
template <typename TU>
__device__ __forceinline__ void fd3_issue_fwd(const Params& P, const TaskMeta& M, const double* r_src,
                                              const double* q_src, const double* p_src, const double* d_src,
                                              double* lds) {
    const Grid& g = M.g;
    const Fd3Lds<TU> L = fd3_lds<TU>(P, M, lds);
    const int n = static_cast<int>(g.ndof);
    const int64_t off = g.dof_off;
    g2l_vec(r_src + off, n, L.R);
    if (q_src) g2l_vec(q_src + off, n, L.S);
    if (p_src) g2l_vec(p_src + off, n, L.Own);
    if (d_src) g2l_vec(d_src + off, n, L.Own + n);
    g2l_vec(P.dpool + g.oDinv, n, L.Own + 2 * n);
    fd3_issue_factors<TU>(P, M, L);
}
template <typename TU>
__device__ __forceinline__ void fd3_issue_bwd(const Params& P, const TaskMeta& M, const double* rt_src,
                                              const double* rdot, double* lds) {
    const Grid& g = M.g;
    const Fd3Lds<TU> L = fd3_lds<TU>(P, M, lds);
    const int n = static_cast<int>(g.ndof);
    g2l_vec(rt_src + g.dof_off, n, L.R);
    if (rdot) g2l_vec(rdot + g.dof_off, n, L.Own);
    fd3_issue_factors<TU>(P, M, L);
}
// forward: r update (whole grid owned), then Rt = (U1 (x) U2 (x) U3)^T r / lambda
template <typename TU, typename TC>
__device__ __forceinline__ void fd3_fwd_run(const Params& P, const TaskMeta& M, const FdIO& io, double* lds) {
    const Grid& g = M.g;
    const Fd3Lds<TU> L = fd3_lds<TU>(P, M, lds);
    const int n1 = g.ni[0], n2 = g.ni[1], n3 = g.ni[2], n = n1 * n2 * n3, n12 = n1 * n2;
    const int64_t off = g.dof_off;
    // the residual update r = r_old - alpha q, written out with d += alpha p;
    // the scaled residual s r in R (the transform's input); ||r||^2
    double nrm = 0.0;
    for (int i = threadIdx.x; i < n; i += kBlock) {
        const double v = io.q ? L.R[i] - io.alpha * L.S[i] : L.R[i];
        L.R[i] = io.scale ? v * io.scale[off + i] : v;
        if (io.r_out) io.r_out[off + i] = v;
        if (io.dvec) io.dvec[off + i] = L.Own[n + i] + io.alpha * L.Own[i];
        if (io.keep) L.Own[i] = v;
        nrm += v * v;
    }
    if (io.part) {
        const double t = wg_sum(nrm, L.red);
        if (threadIdx.x == 0) *io.part = t;
    }
    __syncthreads();
    // S[i3 i2][k1] = sum_i1 R[i3 i2][i1] U1[i1][k1]
    mfma_gemm<double, TU, TC>(n2 * n3, n1, n1, L.R, n1, 1, L.U1, L.ld1, 1, L.S, n1, 1, 1, 0, 0, 0, L.red);
    // T[i3][k2][k1] = sum_i2 U2[i2][k2] S[i3][i2][k1]
    mfma_gemm<TU, double, TC>(n2, n1, n2, L.U2, 1, L.ld2, L.S, n1, 1, L.T, n1, 1, n3, 0, n12, n12);
    // R[k3][k2 k1] = sum_i3 U3[i3][k3] T[i3][k2 k1] (kept: times 1 / lambda)
    mfma_gemm<TU, double, TC>(n3, n12, n3, L.U3, 1, L.ld3, L.T, n12, 1, L.R, n12, 1, 1, 0, 0, 0, L.red,
                              io.keep ? L.Own + 2 * n : nullptr);
    if (!io.keep) {
        for (int o = threadIdx.x; o < n; o += kBlock) io.rt[off + o] = L.R[o] * L.Own[2 * n + o];
        __syncthreads();
    }
}
// One 3x3x3 convolution layer (zero padding) as an implicit GEMM on the
// matrix cores in BF16 with FP32 accumulation:
//   out[i][co] = b[co] + sum over taps t and input channels ci of
//                w[co][ci][t] in[i + off(t)][ci],
// M = points (direction 1 fastest), N = output channels, K = 27 x cip with
// the taps slowest (k = t cip + ci), so that the 8 K values a lane holds are
// 8 consecutive channels of one neighbour: one 16-byte load of the
// point-major BF16 activations in LDS, and one of the packed BF16 weights
// Wp[co][t][ci] in memory (co padded to 16, ci to cip, zero-filled).
// 16x16x32 BF16 MFMA: lane l holds A[l%16][8(l/16)+j], B[8(l/16)+j][l%16]
// and D[4(l/16)+r][l%16] (checked on the device).  Each wavefront takes
// 16-point x 16-channel tiles.  The epilogue adds the bias (FP32), applies
// the ReLU and rounds to BF16 (out[i][c] for c < coutp, pad channels 0), or
// writes FP32 values to yout (the output layer, one channel).
__device__ __forceinline__ void cnn_layer_mfma(const uint16_t* __restrict__ Wp, const float* __restrict__ bias,
                                               const uint16_t* in, int cip, uint16_t* out, int coutp, int cout,
                                               float* yout, int n1, int n2, int n3, bool relu) {
    const int n = n1 * n2 * n3;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int mt = (n + 15) >> 4, nt = (cout + 15) >> 4;
    const int K = 27 * cip, nkb = (K + 31) >> 5;
    const FDiv d1(n1), d12(n1 * n2), dcip(cip);
    for (int u = wave; u < mt * nt; u += kWaves) {  // uniform per wavefront
        const int ti = u / nt, tj = u - ti * nt;
        const int i = 16 * ti + (lane & 15), co = 16 * tj + (lane & 15);
        const bool iv = i < n;
        int i1 = 0, i2 = 0, i3 = 0;
        if (iv) {
            int rr;
            i3 = d12.div(i, &rr);
            i2 = d1.div(rr, &i1);
        }
        v4f_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int kb = 0; kb < nkb; ++kb) {
            const int k0 = 32 * kb + 8 * (lane >> 4);
            bf16x8_t av, bv;
            for (int j = 0; j < 8; ++j) {
                av[j] = static_cast<__bf16>(0.0f);
                bv[j] = static_cast<__bf16>(0.0f);
            }
            if (k0 < K) {
                int ci;
                const int t = dcip.div(k0, &ci);
                const int t3 = t / 9, t2 = (t / 3) % 3, t1 = t % 3;
                const int j1 = i1 + t1 - 1, j2 = i2 + t2 - 1, j3 = i3 + t3 - 1;
                if (iv && j1 >= 0 && j1 < n1 && j2 >= 0 && j2 < n2 && j3 >= 0 && j3 < n3)
                    av = *reinterpret_cast<const bf16x8_t*>(in + static_cast<int64_t>((j3 * n2 + j2) * n1 + j1) * cip + ci);
                bv = *reinterpret_cast<const bf16x8_t*>(Wp + static_cast<int64_t>(co * 27 + t) * cip + ci);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
        }
        const int c = 16 * tj + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int pi = 16 * ti + 4 * (lane >> 4) + r;
            if (pi >= n) continue;
            float v = c < cout ? acc[r] + bias[c] : 0.0f;
            if (relu && v < 0.0f) v = 0.0f;
            if (yout) {
                if (c == 0) yout[pi] = v;
            } else if (c < coutp) {
                reinterpret_cast<__bf16*>(out)[static_cast<int64_t>(pi) * coutp + c] = static_cast<__bf16>(v);
            }
        }
    }
    __syncthreads();
}

// Packed BF16 weights of the network (cnn_layer_mfma): per layer
// [16 ceil(cout / 16)][27][cip] with cip the input channels rounded up to 8
// (3 -> 8), zero-filled; element counts per layer.
__host__ __device__ inline int nn_pad8(int c) { return (c + 7) & ~7; }
__host__ __device__ inline int64_t nn_packed_layer(int cin, int cout) {
    return static_cast<int64_t>(16 * ((cout + 15) / 16)) * 27 * nn_pad8(cin);
}

// backward: z = (U1 (x) U2 (x) U3) Rt; part = rdot . z.  With io.learned the
// network y = N(r / ||r||, z_FD / s, log a - mean), s = ||z_FD||, corrects
// z_FD: z = z_FD + s y (additive head) or z = z_FD exp(y) (log-scale head),
// unless r . z <= 0 (then z = z_FD); part2 (if set) = z . rold.
// LEARN = false compiles the transform without the network (builds that
// never run the learned correction keep its registers free).
template <typename TU, typename TC, bool LEARN = true>
__device__ __forceinline__ void fd3_bwd_run(const Params& P, const TaskMeta& M, const FdIO& io, double* lds) {
    const Grid& g = M.g;
    const Fd3Lds<TU> L = fd3_lds<TU>(P, M, lds);
    const int n1 = g.ni[0], n2 = g.ni[1], n3 = g.ni[2], n = n1 * n2 * n3, n12 = n1 * n2;
    const int64_t off = g.dof_off;
    // T[i3][k2 k1] = sum_k3 U3[i3][k3] Rt[k3][k2 k1]
    mfma_gemm<TU, double, TC>(n3, n12, n3, L.U3, L.ld3, 1, L.R, n12, 1, L.T, n12, 1, 1, 0, 0, 0, L.red);
    // S[i3][i2][k1] = sum_k2 U2[i2][k2] T[i3][k2][k1]
    mfma_gemm<TU, double, TC>(n2, n1, n2, L.U2, L.ld2, 1, L.T, n1, 1, L.S, n1, 1, n3, 0, n12, n12);
    // Z[i3 i2][i1] = sum_k1 S[i3 i2][k1] U1[i1][k1], times the diagonal scaling
    mfma_gemm<double, TU, TC>(n2 * n3, n1, n1, L.S, n1, 1, L.U1, 1, L.ld1, L.R, n1, 1, 1, 0, 0, 0, L.red,
                              io.scale ? io.scale + off : nullptr);
    double scale = 0.0;  // s (additive head), -1 (log-scale head), 0: no learned correction
    float* Y = nullptr;
    if (LEARN && io.learned) {
        // BF16 activations in LDS after the factor region, point-major:
        // X0 [n][8] (3 feature channels, 5 zero), H1 [n][h1p], H2 [n][h2p];
        // then the FP32 output Y [n]
        const int ld[3] = {M.t[0].ldu, M.t[1].ldu, M.t[2].ldu};
        uint16_t* X0 = reinterpret_cast<uint16_t*>(reinterpret_cast<char*>(lds) + fd_layout_3d(g, ld, sizeof(TU)).total);
        const int h1 = P.nn_ch[1], h2 = P.nn_ch[2];
        const int h1p = nn_pad8(h1), h2p = nn_pad8(h2);
        uint16_t* H1 = X0 + 8 * n;
        uint16_t* H2 = H1 + static_cast<int64_t>(h1p) * n;
        Y = reinterpret_cast<float*>(H2 + static_cast<int64_t>(h2p) * n);
        double r2 = 0.0, z2 = 0.0, sa = 0.0;
        for (int i = threadIdx.x; i < n; i += kBlock) {
            r2 += L.Own[i] * L.Own[i];
            z2 += L.R[i] * L.R[i];
            sa += P.loga[off + i];
        }
        r2 = wg_sum(r2, L.red);
        z2 = wg_sum(z2, L.red);
        sa = wg_sum(sa, L.red);
        const double sr = r2 > 0.0 ? sqrt(r2) : 1.0;
        const double s = z2 > 0.0 ? sqrt(z2) : 1.0;
        const double mean = sa / n;
        __bf16* xb = reinterpret_cast<__bf16*>(X0);
        for (int i = threadIdx.x; i < n; i += kBlock) {
            xb[8 * i] = static_cast<__bf16>(static_cast<float>(L.Own[i] / sr));
            xb[8 * i + 1] = static_cast<__bf16>(static_cast<float>(L.R[i] / s));
            xb[8 * i + 2] = static_cast<__bf16>(static_cast<float>(P.loga[off + i] - mean));
            for (int c = 3; c < 8; ++c) xb[8 * i + c] = static_cast<__bf16>(0.0f);
        }
        __syncthreads();
        // biases from the FP32 parameters, weights packed in BF16
        const float* b1 = P.nn + h1 * 3 * 27;
        const float* b2 = b1 + h1 + h2 * h1 * 27;
        const float* b3 = b2 + h2 + h2 * 27;
        const uint16_t* W1 = P.nnw;
        const uint16_t* W2 = W1 + nn_packed_layer(3, h1);
        const uint16_t* W3 = W2 + nn_packed_layer(h1, h2);
        cnn_layer_mfma(W1, b1, X0, 8, H1, h1p, h1, nullptr, n1, n2, n3, true);
        cnn_layer_mfma(W2, b2, H1, h1p, H2, h2p, h2, nullptr, n1, n2, n3, true);
        cnn_layer_mfma(W3, b3, H2, h2p, nullptr, 0, 1, Y, n1, n2, n3, false);
        // acceptance: the corrected z must be a descent direction (r . z > 0)
        const bool mult = P.nn_head == 1;
        double rz = 0.0;
        for (int i = threadIdx.x; i < n; i += kBlock)
            rz += L.Own[i] * (mult ? L.R[i] * exp(static_cast<double>(Y[i])) : L.R[i] + s * Y[i]);
        rz = wg_sum(rz, L.red);
        if (rz > 0.0 && isfinite(rz)) scale = mult ? -1.0 : s;
    }
    double dot = 0.0, dot2 = 0.0, dot3 = 0.0;
    for (int o = threadIdx.x; o < n; o += kBlock) {
        const double zo = scale > 0.0 ? L.R[o] + scale * Y[o]
                                      : (scale < 0.0 ? L.R[o] * exp(static_cast<double>(Y[o])) : L.R[o]);
        io.z[off + o] = zo;
        if (io.rdot) dot += L.Own[o] * zo;
        if (io.part2) dot2 += io.rold[off + o] * zo;
        if (io.part3) dot3 += L.Own[o] * L.R[o];
    }
    if (io.part) {
        const double t = wg_sum(dot, L.red);
        if (threadIdx.x == 0) *io.part = t;
    }
    if (io.part2) {
        const double t = wg_sum(dot2, L.red);
        if (threadIdx.x == 0) *io.part2 = t;
    }
    if (io.part3) {
        const double t = wg_sum(dot3, L.red);
        if (threadIdx.x == 0) *io.part3 = t;
    }
    __syncthreads();
}

// Factor element types of the FD precisions
// (0: FP64, 1: FP32, 2: BF16 factors with FP32 accumulation).
template <int FDP> struct FdTypes;
template <> struct FdTypes<0> { using TU = double; using TC = double; };
template <> struct FdTypes<1> { using TU = float; using TC = float; };
template <> struct FdTypes<2> { using TU = uint16_t; using TC = float; };

// Copy the description of task tk into an LDS slot (all threads; ends
// synchronised): one contiguous copy of the grid's record (grid and 1D tables),
// the task's local index in the last word.
__device__ __forceinline__ void meta_fill(const Params& P, const Task& tk, TaskMeta* M) {
    __syncthreads();
    constexpr int MW = sizeof(TaskMeta) / 8;
    static_assert(offsetof(TaskMeta, grid) == 8 * (MW - 1) && offsetof(TaskMeta, local) == 8 * MW - 4,
                  "grid and local share the last word");
    const uint64_t* src = reinterpret_cast<const uint64_t*>(P.gmeta + tk.grid);
    uint64_t* dst = reinterpret_cast<uint64_t*>(M);
    for (int i = threadIdx.x; i < MW; i += kBlock) {
        uint64_t v = src[i];
        if (i == MW - 1) v = static_cast<uint32_t>(tk.grid) | (static_cast<uint64_t>(static_cast<uint32_t>(tk.local)) << 32);
        dst[i] = v;
    }
    __syncthreads();
}

// ===========================================================================
// grid-wide barrier (all workgroups co-resident: cooperative launch)
// ===========================================================================
// Grid-wide barrier of the persistent solve, two levels: the workgroups
// arrive on one of kBarGroups counters (blockIdx % kBarGroups, each on its own
// 64-byte line), the last of each group arrives on the global counter, and the
// last group advances the generation word that every workgroup polls.
// Counters only grow within a launch (k_solve_init clears them): barrier k
// takes group g from k gs to (k + 1) gs, so the last arrival is the one that
// reaches a multiple of gs.  Memory ordering: one agent-scope release fence
// before arriving, acquire-release fences where an arrival is forwarded, one
// acquire fence after the generation changes.  Against a flat counter with
// release/acquire read-modify-writes this halves the L2 write-back and
// invalidate work and the contention on one address.
__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned nwg) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned gen = __hip_atomic_load(&bar[kBarGen], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned grp = blockIdx.x % kBarGroups;
        const unsigned ng = nwg < kBarGroups ? nwg : kBarGroups;
        const unsigned gs = (nwg - grp + kBarGroups - 1) / kBarGroups;  // workgroups in this group
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned a =
            __hip_atomic_fetch_add(&bar[kBarGroup + kBarStride * grp], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((a + 1u) % gs == 0u) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            const unsigned b = __hip_atomic_fetch_add(&bar[kBarCount], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((b + 1u) % ng == 0u) {
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                __hip_atomic_store(&bar[kBarGen], gen + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        while (__hip_atomic_load(&bar[kBarGen], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen)
            __builtin_amdgcn_s_sleep(1);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// ===========================================================================
// persistent refinement + PCG over all component grids
//
// One sweep = three phases separated by grid-wide barriers:
//   1 operator   ITER: p = z + beta p, q = A p (inner precision), p.q
//                RESID: r = b - A (x + d) (FP64), ||r||^2
//   2 update     ITER: alpha, d += alpha p, r -= alpha q, FD forward of r
//                RESID: x += d, d = 0, FD forward of r
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
    int continue_cg;              // keep the search direction across residual replacements
    int learned;                  // learned correction inside flexible CG (3D)
    int learned_iters;            // ... on the first learned_iters preconditionings (0: all)
    double tol2, tol_in2;
    unsigned long long* trace;    // phase timestamps (or nullptr)
    int trace_sweeps;
    int active;                   // tasks from the per-sweep active lists (else the launch's ranges)
};

// Phase tracing (10 ns wall clock): slot 0 kernel start; per sweep s the
// barrier exits of the three phases seen by workgroup 0 (slots 1+6s..3+6s)
// and the longest busy time of any workgroup in each phase (4+6s..6+6s).
__device__ __forceinline__ void trace_busy(const SolveArgs& A, int sweep, int ph, unsigned long long t0) {
    if (A.trace && sweep < A.trace_sweeps && threadIdx.x == 0)
        atomicMax(&A.trace[1 + 6 * sweep + 3 + ph], wall_clock64() - t0);
}
__device__ __forceinline__ void trace_mark(const SolveArgs& A, int sweep, int ph) {
    if (A.trace && sweep < A.trace_sweeps && blockIdx.x == 0 && threadIdx.x == 0)
        A.trace[1 + 6 * sweep + ph] = wall_clock64();
}

__device__ __forceinline__ double* part_ptr(const Params& P, int kind, int parity) {
    return P.part + static_cast<int64_t>(kind * 2 + parity) * P.part_stride;
}
enum { PK_PQ = 0, PK_RES = 1, PK_RR = 2, PK_RZ = 3, PK_ZRO = 4, PK_RZF = 5 };
enum { ACT_SKIP = 0, ACT_RESID, ACT_ITER, ACT_DONE };

struct Decision {
    int act, status;
    double rho, rhob, rho0;
};

// Sum of count partials by one wavefront (fixed order per lane, fixed
// butterfly), result in every lane.  No workgroup barrier inside.
__device__ __forceinline__ double wave_sum_partials(const double* part, int count) {
    double v = 0.0;
    for (int i = threadIdx.x & 63; i < count; i += 64) v += part[i];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// rho: r . z of the last preconditioning (the search preconditioner: CG beta
// and alpha); rhof: r . z_FD of the plain preconditioner for the same r.  The
// stopping tests of a learned solve use rhof: the learned r . z does not
// measure the error (it can fall below the target long before r . P^-1 r
// does, which ended inner solves early and spent the refinement budget).
__device__ inline Decision decide(const SolveArgs& A, const GState& st, double rho, double rhof) {
    Decision D;
    D.status = GS_OK;
    D.rho = rho;
    D.rhob = st.rhob;
    D.rho0 = st.rho0;
    if (st.stage == STAGE_DONE) {
        D.act = ACT_SKIP;
    } else if (st.stage == STAGE_RESID) {
        D.act = ACT_RESID;
    } else if (!isfinite(rho) || rho < 0.0) {
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
    } else if ((A.learned ? rhof : rho) <= A.tol_in2 * st.rho0 || (A.learned ? rhof : rho) <= A.tol2 * st.rhob ||
               st.it >= A.maxit) {
        // inner solve done (its own tolerance, or the outer target reached by the
        // recursive residual): x += d and replace r by the FP64 residual
        D.act = ACT_RESID;
    } else {
        D.act = ACT_ITER;
    }
    return D;
}

// Per-task context, computed by wavefront 0 (whose lane 0 performed the
// agent-scope acquire of the last grid barrier) and broadcast through LDS.
struct TaskCtx {
    GState st;
    Decision D;
    double pq;    // p.Ap of the current iteration (phases 2-3)
    double rn2;   // ||b - A x||^2 of a residual sweep (phase 3)
    double zro;   // z . r_old of the last preconditioning (flexible CG, phase 1)
};
static_assert(sizeof(TaskCtx) <= kCtxBytes, "TaskCtx too large");

// Wavefront-0 registers of a task context between issue and finish.
struct CtxLoads {
    GState st;
    double vrz, vpq, vres, vzro, vrzf;
};

__device__ __forceinline__ double sum_strided(const double* p, int count) {
    const int lane = threadIdx.x & 63;
    double v = 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int i = lane + 64 * s;
        if (i < count) v += p[i];
    }
    for (int i = lane + 256; i < count; i += 64) v += p[i];  // beyond the unrolled 4 x 64
    return v;
}

// Issue the loads of a task context (wavefront 0 only): the grid state and
// the partial sums of the previous phases.
// The state and partial sums are those of the grid's solver-state group (the
// grid itself, or the patch grids of one component of a multipatch plan).
__device__ __forceinline__ void ctx_issue(const Params& P, const Grid& g, const GState* S0, int gi, int cur, int nxt,
                                          int phase, CtxLoads& c) {
    (void)gi;
    c.st = S0[g.state];
    c.vrz = sum_strided(part_ptr(P, PK_RZ, nxt) + g.gblk_off, g.gnblk);
    c.vzro = phase == 1 ? sum_strided(part_ptr(P, PK_ZRO, nxt) + g.gblk_off, g.gnblk) : 0.0;
    c.vrzf = sum_strided(part_ptr(P, PK_RZF, nxt) + g.gblk_off, g.gnblk);
    c.vpq = 0.0;
    c.vres = 0.0;
    if (phase >= 2) c.vpq = sum_strided(part_ptr(P, PK_PQ, cur) + g.gtile_off, g.gntile);
    // ||b - A x||^2 of a residual sweep: from the operator tiles, or with
    // several patches from the interface-summed residual of the FD forward
    // tasks (phase 3 only)
    if (phase == 3)
        c.vres = P.mp ? sum_strided(part_ptr(P, PK_RR, cur) + g.gblk_off, g.gnblk)
                      : sum_strided(part_ptr(P, PK_RES, cur) + g.gtile_off, g.gntile);
}

// Reduce and decide (wavefront 0 only); lane 0 writes the context to LDS.
__device__ __forceinline__ void ctx_finish(const SolveArgs& A, CtxLoads& c, int phase, TaskCtx* ctx) {
    for (int o = 32; o > 0; o >>= 1) {
        c.vrz += __shfl_xor(c.vrz, o, 64);
        c.vpq += __shfl_xor(c.vpq, o, 64);
        c.vres += __shfl_xor(c.vres, o, 64);
        c.vzro += __shfl_xor(c.vzro, o, 64);
        c.vrzf += __shfl_xor(c.vrzf, o, 64);
    }
    const Decision D = decide(A, c.st, c.st.stage == STAGE_ITER ? c.vrz : 0.0, c.st.stage == STAGE_ITER ? c.vrzf : 0.0);
    if (threadIdx.x == 0) {
        ctx->st = c.st;
        ctx->D = D;
        ctx->pq = (phase >= 2 && D.act == ACT_ITER) ? c.vpq : 0.0;
        ctx->rn2 = (phase == 3 && D.act == ACT_RESID) ? c.vres : 0.0;
        ctx->zro = c.vzro;
    }
}

// NT: threads per workgroup of the build (a template argument, so that the
// 512- and 256-thread builds of one kernel have distinct symbols)
template <int PP, int FDP, int DIM, int NT>
__global__ void __launch_bounds__(NT) k_solve(Params P, SolveArgs A) {
    static_assert(NT == kBlock, "the workgroup size is that of the translation unit's build");
    using TU = typename FdTypes<FDP>::TU;
    using TC = typename FdTypes<FDP>::TC;
    extern __shared__ double lds_all[];
    TaskCtx* ctx = reinterpret_cast<TaskCtx*>(lds_all);
    TaskMeta* meta = reinterpret_cast<TaskMeta*>(reinterpret_cast<char*>(lds_all) + kCtxBytes);
    TaskMeta* meta_op = meta;             // kMetaOp slots
    TaskMeta* meta_fd = meta + kMetaOp;   // kMetaFd slots
    TaskMeta* meta_sp = meta + kMetaSlots - 1;
    double* lds = reinterpret_cast<double*>(reinterpret_cast<char*>(lds_all) + kSolveLdsHead);  // task work arrays
    const unsigned nwg = gridDim.x;
    const int64_t N = P.ndof_total;
    const int lowp = FDP != 0;
    const bool wave0 = threadIdx.x < 64;
    if (A.trace && blockIdx.x == 0 && threadIdx.x == 0) A.trace[0] = wall_clock64();
    // Task schedule.  Static: workgroup w takes tasks w, w + nwg, ... of the
    // launch's ranges, with the descriptions of its first tasks cached in LDS
    // for the whole launch (a few tasks per workgroup).  Active lists (many
    // tasks per workgroup): the same round robin over per-sweep lists that
    // hold only the tasks of grids still iterating, rebuilt in phase 3.
    // Which workgroup runs a task changes no result (partial sums go to the
    // task's own slot).
    if (!A.active) {
        int k = 0;
        for (int t = A.op_b + blockIdx.x; t < A.op_e && k < kMetaOp; t += nwg, ++k) meta_fill(P, P.optask[t], meta_op + k);
        k = 0;
        for (int t = A.fd_b + blockIdx.x; t < A.fd_e && k < kMetaFd; t += nwg, ++k) meta_fill(P, P.fdtask[t], meta_fd + k);
    }
    auto task_meta = [&](const Task* list, int t, int k, TaskMeta* cache, int ncache) -> const TaskMeta& {
        if (!A.active && k < ncache) return cache[k];
        meta_fill(P, list[t], meta_sp);
        return *meta_sp;
    };
    // length of an active list (uniform: read through the first lane)
    auto list_len = [&](int word) {
        return static_cast<int>(__builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&P.bar[word], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
    };
    for (int sweep = 0; sweep < A.max_sweeps; ++sweep) {
        const int cur = sweep & 1, nxt = cur ^ 1;
        unsigned long long tb = A.trace ? wall_clock64() : 0ull;
        GState* S0 = P.st2 + cur * P.ngrid;
        GState* S1 = P.st2 + nxt * P.ngrid;
        double* r_new = P.r2 + cur * N;
        double* r_old = P.r2 + nxt * N;
        double* p_new = P.p2 + cur * N;
        double* p_old = P.p2 + nxt * N;
        // ---------------- phase 1: operator -------------------------------------
        const Task* ol = A.active ? P.oplist + static_cast<int64_t>(cur) * P.op_cap : P.optask + A.op_b;
        const int nop = A.active ? list_len(kBarOpLen + cur) : A.op_e - A.op_b;
        for (int t = blockIdx.x, k = 0; t < nop; t += nwg, ++k) {
            const TaskMeta& M = task_meta(ol, t, k, meta_op, kMetaOp);
            const Grid& g = M.g;
            __syncthreads();  // the previous task is done with the LDS context
            if (wave0) {
                CtxLoads c;
                ctx_issue(P, g, S0, M.grid, cur, nxt, 1, c);
                ctx_finish(A, c, 1, ctx);
            }
            __syncthreads();
            const int act = ctx->D.act;
            if (act == ACT_SKIP) {
                if (M.local == 0 && threadIdx.x == 0 && g.state == M.grid) S1[M.grid] = ctx->st;  // carry DONE forward
                continue;
            }
            OpIO io;
            if (act == ACT_ITER) {
                io.in_a = P.z;
                io.in_b = p_old;
                // beta = 0 at the start of a solve; after a residual replacement
                // either restart (0) or continue with the previous rho (continue_cg)
                const bool fresh = ctx->st.it == 0 && (!A.continue_cg || ctx->st.refine <= 1 || ctx->st.op64);
                // flexible CG (variable preconditioner): beta = z.(r - r_old) / rho_old
                const double num = A.learned && ctx->st.it > 0 ? ctx->D.rho - ctx->zro : ctx->D.rho;
                io.beta = fresh ? 0.0 : num / ctx->st.rho;
                io.out_in = p_new;
                io.out = P.q;
                io.rhs = nullptr;
                io.part = part_ptr(P, PK_PQ, cur) + g.tile_off + M.local;
                io.lowp = lowp && !ctx->st.op64;
                io.isum = P.mp;  // z of a multipatch plan is assembled patch by patch
            } else if (act == ACT_RESID) {
                // r = b - A (x + d): the pending update d is folded into x in phase 2
                io.in_a = P.x;
                io.in_b = P.d;
                io.beta = 1.0;
                io.out_in = nullptr;
                // several patches: the patch-local residual goes to q, the FD
                // forward tasks sum it across interfaces into r
                io.out = P.mp ? P.q : r_new;
                io.rhs = P.b;
                io.part = part_ptr(P, PK_RES, cur) + g.tile_off + M.local;
                io.lowp = 0;
            } else {
                continue;
            }
            if constexpr (DIM == 3) op_tile_3d<PP>(P, g, M.t[0], M.t[1], M.t[2], M.local, io, lds);
            else op_tile_2d<PP>(P, g, M.t[0], M.t[1], M.local, io, lds);
        }
        trace_busy(A, sweep, 0, tb);
        grid_barrier(P.bar, nwg);
        trace_mark(A, sweep, 0);
        if (A.trace) tb = wall_clock64();
        // ---------------- phase 2: update + FD forward ---------------------------
        const Task* fl = A.active ? P.fdlist + static_cast<int64_t>(cur) * P.fd_cap : P.fdtask + A.fd_b;
        const int nfd = A.active ? list_len(kBarFdLen + cur) : A.fd_e - A.fd_b;
        if (A.active && blockIdx.x == 0 && threadIdx.x == 0) {
            // the next sweep's lists (the previous sweep was their last reader)
            __hip_atomic_store(&P.bar[kBarOpLen + nxt], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&P.bar[kBarFdLen + nxt], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        for (int t = blockIdx.x, k = 0; t < nfd; t += nwg, ++k) {
            const TaskMeta& M = task_meta(fl, t, k, meta_fd, kMetaFd);
            const Grid& g = M.g;
            __syncthreads();
            CtxLoads c;
            if (wave0) ctx_issue(P, g, S0, M.grid, cur, nxt, 2, c);
            // operands of an iteration step, copied to LDS together with the context loads
            if constexpr (DIM == 3) fd3_issue_fwd<TU>(P, M, r_old, P.q, p_new, P.d, lds);
            else fd_issue_fwd<TU>(P, M, M.local, r_old, P.q, p_new, P.d, lds);
            if (wave0) ctx_finish(A, c, 2, ctx);
            g2l_wait_sync();
            const int act = ctx->D.act;
            FdIO io;
            io.rt = P.rt;
            io.prec = FDP;
            io.scale = P.fdscale;
            io.learned = 0;
            io.rold = nullptr;
            io.part2 = nullptr;
            io.z = nullptr;
            io.rdot = nullptr;
            io.part = part_ptr(P, PK_RR, cur) + g.blk_off + M.local;
            io.mp = DIM == 2 ? P.mp : 0;
            io.resq = 0;
            if (act == ACT_ITER) {
                const double pq = ctx->pq;
                if (!(pq > 0.0) || !isfinite(ctx->D.rho / pq)) continue;  // breakdown: committed in phase 3
                io.alpha = ctx->D.rho / pq;
                io.r_old = r_old;
                io.q = P.q;
                io.r_out = r_new;
                io.dvec = P.d;
                io.pvec = p_new;
            } else if (act == ACT_RESID) {
                io.alpha = 0.0;
                io.r_old = r_new;
                io.q = io.mp ? P.q : nullptr;
                io.resq = io.mp;
                io.r_out = io.mp ? r_new : nullptr;
                io.dvec = nullptr;
                io.pvec = nullptr;
                // x += d, d = 0 on the owned unknowns (phase 1 has read both); a
                // continued CG carries its search direction into this sweep's buffer
                if constexpr (DIM == 3) {  // one task owns the grid
                    for (int o = threadIdx.x; o < g.ndof; o += kBlock) {
                        const int64_t kk = g.dof_off + o;
                        P.x[kk] += P.d[kk];
                        P.d[kk] = 0.0;
                        if (A.continue_cg) p_new[kk] = p_old[kk];
                    }
                } else {
                    const FdBlock B(g, M.local);
                    for (int o = threadIdx.x; o < B.nown; o += kBlock) {
                        const int64_t kk = g.dof_off + B.gi(o);
                        P.x[kk] += P.d[kk];
                        P.d[kk] = 0.0;
                        if (A.continue_cg) p_new[kk] = p_old[kk];
                    }
                }
                // the residual sweep transforms r_new, not the prefetched r_old
                // (several patches: the prefetched q, summed across interfaces)
                if (!io.mp) {
                    g2l_vec(r_new + g.dof_off, g.ndof, fd_lds<TU>(M, lds).R);
                    g2l_wait_sync();
                }
            } else {
                continue;
            }
            if constexpr (DIM == 3) fd3_fwd_run<TU, TC>(P, M, io, lds);
            else fd_fwd_run<TU, TC>(P, M, M.local, io, lds);
        }
        trace_busy(A, sweep, 1, tb);
        grid_barrier(P.bar, nwg);
        trace_mark(A, sweep, 1);
        if (A.trace) tb = wall_clock64();
        // ---------------- phase 3: FD backward and commit ---------------------------
        for (int t = blockIdx.x, k = 0; t < nfd; t += nwg, ++k) {
            const TaskMeta& M = task_meta(fl, t, k, meta_fd, kMetaFd);
            const Grid& g = M.g;
            const int gi = M.grid;
            __syncthreads();
            CtxLoads c;
            if (wave0) ctx_issue(P, g, S0, gi, cur, nxt, 3, c);
            if constexpr (DIM == 3) fd3_issue_bwd<TU>(P, M, P.rt, r_new, lds);
            else fd_issue_bwd<TU>(P, M, M.local, P.rt, r_new, lds);
            if (wave0) ctx_finish(A, c, 3, ctx);
            g2l_wait_sync();
            const int act = ctx->D.act;
            if (act == ACT_SKIP) continue;
            bool run_bwd = act == ACT_RESID || (act == ACT_ITER && ctx->pq > 0.0 && isfinite(ctx->D.rho / ctx->pq));
            if (run_bwd) {
                FdIO io;
                io.rt = P.rt;
                io.z = P.z;
                io.rdot = r_new;
                io.prec = FDP;
                io.scale = P.fdscale;
                io.mp = DIM == 2 ? P.mp : 0;
                io.part = part_ptr(P, PK_RZ, cur) + g.blk_off + M.local;
                // the learned map preconditions the residuals of the CG iterations
                // (up to learned_iters of them per inner solve); the FP64 residual
                // of a residual sweep keeps the plain preconditioner, so that the
                // convergence test r . P^-1 r and the first search direction of a
                // (re)started solve are those of the plain method; z . r_old
                // (flexible CG beta) on every iteration of a learned solve
                io.learned = DIM == 3 && A.learned && P.nn != nullptr && act == ACT_ITER &&
                             (A.learned_iters == 0 || ctx->st.it + 1 < A.learned_iters);
                io.rold = r_old;
                io.part2 = DIM == 3 && A.learned && act == ACT_ITER ? part_ptr(P, PK_ZRO, cur) + g.blk_off + M.local
                                                                    : nullptr;
                io.part3 = DIM == 3 && A.learned ? part_ptr(P, PK_RZF, cur) + g.blk_off + M.local : nullptr;
                if constexpr (DIM == 3) fd3_bwd_run<TU, TC>(P, M, io, lds);
                else fd_bwd_run<TU, TC>(P, M, M.local, io, lds);
            }
            if (M.local == 0 && threadIdx.x == 0) {
                const GState& st = ctx->st;
                const Decision& D = ctx->D;
                GState ns = st;
                bool finish = false;
                if (act == ACT_ITER) {
                    ns.rhob = D.rhob;
                    ns.rho0 = D.rho0;
                    if (!run_bwd && lowp && !st.op64) {
                        // the FP32 operator lost positive definiteness: the
                        // inner solves of this grid continue with the FP64
                        // operator from a fresh FP64 residual
                        ns.op64 = 1;
                        ns.stage = STAGE_RESID;
                        ns.total_it += st.it;
                        ns.it = 0;
                    } else if (!run_bwd) {
                        ns.stage = STAGE_DONE;
                        ns.status = GS_BREAKDOWN;
                        ns.total_it += st.it;
                        finish = true;
                    } else {
                        ns.stage = STAGE_ITER;
                        ns.it = st.it + 1;
                        ns.rho = D.rho;
                    }
                } else if (act == ACT_RESID) {
                    if (st.stage == STAGE_ITER) {  // end of an inner solve
                        ns.total_it += st.it;
                        ns.prelres = D.rhob > 0.0 ? sqrt(D.rho / D.rhob) : 0.0;
                    }
                    const double rn2 = ctx->rn2;
                    const double bn2 = st.refine == 0 ? rn2 : st.bn2;
                    ns.bn2 = bn2;
                    ns.relres = bn2 > 0.0 ? sqrt(rn2 / bn2) : 0.0;
                    ns.stage = STAGE_ITER;
                    ns.it = 0;
                    ns.refine = st.refine + 1;
                } else if (act == ACT_DONE) {
                    ns.stage = STAGE_DONE;
                    ns.status = D.status;
                    ns.rhob = D.rhob;
                    ns.prelres = D.rhob > 0.0 ? sqrt(D.rho / D.rhob) : 0.0;
                    finish = true;
                }
                // the group's first grid keeps its state; every grid of a
                // group that continues puts its own tasks on the lists
                const bool lead = g.state == gi;
                if (lead) S1[gi] = ns;
                if (finish) {
                    if (lead) atomicAdd(&P.bar[kBarDone], 1u);
                } else if (A.active) {
                    // the grid keeps iterating: its tasks go on the next sweep's lists
                    const unsigned o = atomicAdd(&P.bar[kBarOpLen + nxt], static_cast<unsigned>(g.ntile));
                    Task* on = P.oplist + static_cast<int64_t>(nxt) * P.op_cap + o;
                    for (int l = 0; l < g.ntile; ++l) on[l] = Task{gi, l};
                    const unsigned f = atomicAdd(&P.bar[kBarFdLen + nxt], static_cast<unsigned>(g.nblk));
                    Task* fn = P.fdlist + static_cast<int64_t>(nxt) * P.fd_cap + f;
                    for (int l = 0; l < g.nblk; ++l) fn[l] = Task{gi, l};
                }
            }
        }
        trace_busy(A, sweep, 2, tb);
        grid_barrier(P.bar, nwg);
        trace_mark(A, sweep, 2);
        if (A.trace && blockIdx.x == 0 && threadIdx.x == 0) P.bar[kBarSweeps] = sweep + 1;
        const unsigned done = __hip_atomic_load(&P.bar[kBarDone], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (static_cast<int>(done) >= A.ndone_target) break;
    }
}

// ===========================================================================
// whole-grid solve: one workgroup runs the complete refinement + PCG of one
// grid (all its operator tiles and FD blocks in turn) and takes the next grid
// from a shared counter, in the launch's cost order (largest first).  Every
// reduction is a workgroup reduction; there is no grid-wide barrier, so a
// grid that converges early frees its workgroup at once and the grids of a
// large batch keep every CU busy.  The refinement / CG state machine, the
// operator tiles and the FD transforms are those of k_solve (decide,
// op_tile_*, fd*_run), so a grid follows the same iteration as there.
// LEARN: the build runs the learned correction (the 512-thread,
// one-workgroup-per-CU build); ROWS64: the FP64 element layers of the
// residual sweeps by rows (op_tile_3d), in the two-workgroup build.
// ===========================================================================
template <int PP, int FDP, int DIM, bool LEARN, bool ROWS64>
__device__ __forceinline__ void solve_one_grid(const Params& P, const SolveArgs& A, const TaskMeta& M,
                                               double* slots, double* lds) {
    using TU = typename FdTypes<FDP>::TU;
    using TC = typename FdTypes<FDP>::TC;
    const Grid& g = M.g;
    const int gi = M.grid;
    const int64_t N = P.ndof_total;
    GState st;
    st.rho = st.rho0 = st.rhob = st.bn2 = st.relres = st.prelres = 0.0;
    st.stage = STAGE_RESID;
    st.it = st.total_it = st.refine = 0;
    st.status = GS_RUNNING;
    st.op64 = 0;
    double rz = 0.0, zro = 0.0, rzf = 0.0;
    int pr = 0, pp = 0;  // buffer parities of r and p
    double* sl = slots;   // partial sum of one tile / block (written by thread 0)
    double* sl2 = slots + 1;
    double* sl3 = slots + 2;
    // sum of the per-tile or per-block partials, in tile order (every thread)
    auto tiles = [&](auto&& body, int n) {
        double acc = 0.0;
        for (int t = 0; t < n; ++t) {
            body(t);
            __syncthreads();
            acc += *sl;
        }
        return acc;
    };
    for (int sweep = 0; sweep < A.max_sweeps; ++sweep) {
        const Decision D = decide(A, st, st.stage == STAGE_ITER ? rz : 0.0, st.stage == STAGE_ITER ? rzf : 0.0);
        if (D.act == ACT_DONE) {
            st.stage = STAGE_DONE;
            st.status = D.status;
            st.rhob = D.rhob;
            st.prelres = D.rhob > 0.0 ? sqrt(D.rho / D.rhob) : 0.0;
            break;
        }
        double* r_cur = P.r2 + pr * N;
        double* r_oth = P.r2 + (pr ^ 1) * N;
        double* p_old = P.p2 + pp * N;
        double* p_new = P.p2 + (pp ^ 1) * N;
        FdIO fio;
        fio.rt = P.rt;
        fio.prec = FDP;
        fio.scale = P.fdscale;
        fio.learned = 0;
        fio.rold = nullptr;
        fio.part2 = nullptr;
        fio.part3 = nullptr;
        fio.z = nullptr;
        fio.rdot = nullptr;
        fio.part = sl;
        fio.keep = DIM == 3;
        if (D.act == ACT_ITER) {
            // p = z + beta p, q = A p, p.q
            const bool fresh = st.it == 0 && (!A.continue_cg || st.refine <= 1 || st.op64);
            const double num = A.learned && st.it > 0 ? D.rho - zro : D.rho;
            OpIO io;
            io.in_a = P.z;
            io.in_b = p_old;
            io.beta = fresh ? 0.0 : num / st.rho;
            io.out_in = p_new;
            io.out = P.q;
            io.rhs = nullptr;
            io.part = sl;
            io.lowp = FDP != 0 && !st.op64;
            const double pq = tiles([&](int t) {
                if constexpr (DIM == 3) op_tile_3d<PP, ROWS64>(P, g, M.t[0], M.t[1], M.t[2], t, io, lds);
                else op_tile_2d<PP>(P, g, M.t[0], M.t[1], t, io, lds);
            }, g.ntile);
            if (!(pq > 0.0) || !isfinite(D.rho / pq)) {
                st.total_it += st.it;
                if (FDP != 0 && !st.op64) {
                    // FP32 operator no longer positive definite: continue with
                    // the FP64 operator from a fresh FP64 residual
                    st.op64 = 1;
                    st.stage = STAGE_RESID;
                    st.it = 0;
                    continue;
                }
                st.stage = STAGE_DONE;
                st.status = GS_BREAKDOWN;
                break;
            }
            // alpha, d += alpha p, r -= alpha q, forward transform
            fio.alpha = D.rho / pq;
            fio.r_old = r_cur;
            fio.q = P.q;
            fio.r_out = r_oth;
            fio.dvec = P.d;
            fio.pvec = p_new;
            tiles([&](int b) {
                if constexpr (DIM == 3) {
                    fd3_issue_fwd<TU>(P, M, r_cur, P.q, p_new, P.d, lds);
                    g2l_wait_sync();
                    fd3_fwd_run<TU, TC>(P, M, fio, lds);
                } else {
                    __syncthreads();
                    fd_issue_fwd<TU>(P, M, b, r_cur, P.q, p_new, P.d, lds);
                    g2l_wait_sync();
                    fd_fwd_run<TU, TC>(P, M, b, fio, lds);
                }
            }, g.nblk);
            // backward transform -> z, r.z (and z.r_old for flexible CG)
            fio.z = P.z;
            fio.rdot = r_oth;
            fio.learned = DIM == 3 && A.learned && P.nn != nullptr &&
                          (A.learned_iters == 0 || st.it + 1 < A.learned_iters);
            fio.rold = r_cur;
            fio.part2 = DIM == 3 && A.learned ? sl2 : nullptr;
            fio.part3 = DIM == 3 && A.learned ? sl3 : nullptr;
            double z2 = 0.0, z3 = 0.0;
            const double rzn = tiles([&](int b) {
                if constexpr (DIM == 3) {
                    fd3_bwd_run<TU, TC, LEARN>(P, M, fio, lds);  // its inputs kept in LDS
                } else {
                    __syncthreads();
                    fd_issue_bwd<TU>(P, M, b, P.rt, r_oth, lds);
                    g2l_wait_sync();
                    fd_bwd_run<TU, TC>(P, M, b, fio, lds);
                }
                if (fio.part2) {
                    __syncthreads();
                    z2 += *sl2;
                    z3 += *sl3;
                }
            }, g.nblk);
            st.rhob = D.rhob;
            st.rho0 = D.rho0;
            st.stage = STAGE_ITER;
            st.it += 1;
            st.rho = D.rho;
            rz = rzn;
            zro = z2;
            rzf = fio.part3 ? z3 : rzn;
            pr ^= 1;
            pp ^= 1;
        } else {
            // FP64 residual r = b - A (x + d), then x += d, d = 0
            OpIO io;
            io.in_a = P.x;
            io.in_b = P.d;
            io.beta = 1.0;
            io.out_in = nullptr;
            io.out = r_cur;
            io.rhs = P.b;
            io.part = sl;
            io.lowp = 0;
            double rn2;
            if (DIM == 3 && st.refine == 0 && g.ntile == 1) {
                // the first residual of the solve: x = d = 0 (cleared at its
                // start), so r = b; ||r||^2 in the order of the operator tile's
                // sum (one tile: unknown o on thread o mod kBlock)
                double acc = 0.0;
                for (int o = threadIdx.x; o < g.ndof; o += kBlock) {
                    const double v = P.b[g.dof_off + o];
                    r_cur[g.dof_off + o] = v;
                    acc += v * v;
                }
                rn2 = 0.0 + wg_sum(acc, lds);
                __syncthreads();
            } else {
                rn2 = tiles([&](int t) {
                    if constexpr (DIM == 3) op_tile_3d<PP, ROWS64>(P, g, M.t[0], M.t[1], M.t[2], t, io, lds);
                    else op_tile_2d<PP>(P, g, M.t[0], M.t[1], t, io, lds);
                }, g.ntile);
            }
            for (int o = threadIdx.x; o < g.ndof; o += kBlock) {
                const int64_t k = g.dof_off + o;
                P.x[k] += P.d[k];
                P.d[k] = 0.0;
            }
            __syncthreads();
            fio.alpha = 0.0;
            fio.r_old = r_cur;
            fio.q = nullptr;
            fio.r_out = nullptr;
            fio.dvec = nullptr;
            fio.pvec = nullptr;
            tiles([&](int b) {
                if constexpr (DIM == 3) {
                    fd3_issue_fwd<TU>(P, M, r_cur, nullptr, nullptr, nullptr, lds);
                    g2l_wait_sync();
                    fd3_fwd_run<TU, TC>(P, M, fio, lds);
                } else {
                    __syncthreads();
                    fd_issue_fwd<TU>(P, M, b, r_cur, nullptr, nullptr, nullptr, lds);
                    g2l_wait_sync();
                    fd_fwd_run<TU, TC>(P, M, b, fio, lds);
                }
            }, g.nblk);
            fio.z = P.z;
            fio.rdot = r_cur;
            const double rzn = tiles([&](int b) {
                if constexpr (DIM == 3) {
                    fd3_bwd_run<TU, TC, LEARN>(P, M, fio, lds);  // its inputs kept in LDS
                } else {
                    __syncthreads();
                    fd_issue_bwd<TU>(P, M, b, P.rt, r_cur, lds);
                    g2l_wait_sync();
                    fd_bwd_run<TU, TC>(P, M, b, fio, lds);
                }
            }, g.nblk);
            if (st.stage == STAGE_ITER) {  // end of an inner solve
                st.total_it += st.it;
                st.prelres = D.rhob > 0.0 ? sqrt(D.rho / D.rhob) : 0.0;
            }
            st.bn2 = st.refine == 0 ? rn2 : st.bn2;
            st.relres = st.bn2 > 0.0 ? sqrt(rn2 / st.bn2) : 0.0;
            st.stage = STAGE_ITER;
            st.it = 0;
            st.refine += 1;
            rz = rzn;
            rzf = rzn;
        }
    }
    if (threadIdx.x == 0) {
        P.st2[gi] = st;
        P.st2[P.ngrid + gi] = st;
    }
    __syncthreads();
}

// WAVES: workgroups per CU the build is compiled for (register budget); 2
// lets two workgroups share a CU when their LDS fits (the FP64 operator
// tile then spills, so only the mixed modes use it)
template <int PP, int FDP, int DIM, int NT, int WAVES>
__global__ void __launch_bounds__(NT, WAVES) k_solve_grid(Params P, SolveArgs A) {
    static_assert(NT == kBlock, "the workgroup size is that of the translation unit's build");
    extern __shared__ double lds_all[];
    double* slots = lds_all;  // the context area: the grid handed out, two partial sums
    TaskMeta* meta = reinterpret_cast<TaskMeta*>(reinterpret_cast<char*>(lds_all) + kCtxBytes);
    double* lds = reinterpret_cast<double*>(reinterpret_cast<char*>(lds_all) + kSolveLdsHead);
    int* next = reinterpret_cast<int*>(slots + 4);
    const int ntask = A.fd_e - A.fd_b;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) *next = static_cast<int>(atomicAdd(&P.bar[kBarNext], 1u));
        __syncthreads();
        const int t = *next;
        if (t >= ntask) break;
        const Task tk = P.fdtask[A.fd_b + t];
        if (tk.local != 0) continue;  // the first block of a grid stands for the grid
        meta_fill(P, tk, meta);
        // learned solves run the 512-thread one-workgroup build only (the host
        // picks it for them); the other builds compile the transform without
        // the network
        solve_one_grid<PP, FDP, DIM, WAVES == 1 && NT == 512, WAVES == 2>(P, A, *meta, slots, lds);
    }
}

// One FD transform of block blk of a grid outside the solve (single-operation
// kernels): description in LDS slot M.
template <int FDP>
__device__ __forceinline__ void fd_apply_block(const Params& P, const TaskMeta& M, int blk, const FdIO& io,
                                               double* lds, bool fwd) {
    using TU = typename FdTypes<FDP>::TU;
    using TC = typename FdTypes<FDP>::TC;
    __syncthreads();
    if (P.dim == 3) {
        if (fwd) {
            fd3_issue_fwd<TU>(P, M, io.r_old, io.q, io.pvec, io.dvec, lds);
            g2l_wait_sync();
            fd3_fwd_run<TU, TC>(P, M, io, lds);
        } else {
            fd3_issue_bwd<TU>(P, M, io.rt, io.rdot, lds);
            g2l_wait_sync();
            fd3_bwd_run<TU, TC>(P, M, io, lds);
        }
        return;
    }
    if (fwd) {
        fd_issue_fwd<TU>(P, M, blk, io.r_old, io.q, io.pvec, io.dvec, lds);
        g2l_wait_sync();
        fd_fwd_run<TU, TC>(P, M, blk, io, lds);
    } else {
        fd_issue_bwd<TU>(P, M, blk, io.rt, io.rdot, lds);
        g2l_wait_sync();
        fd_bwd_run<TU, TC>(P, M, blk, io, lds);
    }
}

}  // namespace igasg
