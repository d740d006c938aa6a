// solve.hpp -- device code of the persistent sparse-grid solve: matrix-free
// operator tiles, fast-diagonalisation transforms, the grid-wide barrier and
// the refinement / PCG state machine (kernel template k_solve).  Included by
// the translation units that instantiate k_solve for one spline degree each
// and by kernels.hip for the single-operation kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
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
__device__ __forceinline__ void op_tile_2d(const Params& P, const Grid& g, int tile, const OpIO& io, double* lds) {
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
    // split K when there are fewer outputs than threads: short sequential
    // dot products keep the latency of a phase low
    int S = O >= kBlock ? 1 : kBlock / O;
    if (S > (K + 15) / 16) S = (K + 15) / 16;
    if (S <= 1) {
        for (int o = threadIdx.x; o < O; o += kBlock) {
            const int n = o % N, mb = o / N, m = mb % M, b = mb / M;
            const TA* a = A + b * sAb + m * sAm;
            const TB* bb = B + b * sBb + n * sBn;
            TC s = TC(0);
#pragma unroll 8
            for (int k = 0; k < K; ++k) s += ld(a, k * sAk) * ld(bb, k * sBk);
            C[b * sCb + m * sCm + n * sCn] = static_cast<double>(s);
        }
        __syncthreads();
        return;
    }
    const int kc = (K + S - 1) / S;
    const int o = threadIdx.x % O, sl = threadIdx.x / O;
    if (sl < S) {
        const int n = o % N, mb = o / N, m = mb % M, b = mb / M;
        const TA* a = A + b * sAb + m * sAm;
        const TB* bb = B + b * sBb + n * sBn;
        TC s = TC(0);
        const int k1 = min(K, (sl + 1) * kc);
#pragma unroll 8
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
};

// Owned index set of a block: unknowns whose index along g.big lies in the block.
__device__ __forceinline__ bool owned_2d(const Grid& g, int blk, int i1, int i2) {
    const int ib = g.big == 0 ? i1 : i2;
    return ib >= blk * g.blk && ib < min(g.ni[g.big], (blk + 1) * g.blk);
}

// Big-direction mode product of one FD block:
//   C[m][j] = sum_k V(m, k) U(k, c0 + j),  m < msm, j < bsa <= BS, k < K,
// V in LDS (V(m,k) = V[m*sVm + k*sVk]), U rows in global memory
// (U(k, c) = U[k*ldu + c]; ldu and the table base are multiples of 8 elements).
// Lanes cover a row segment of BS columns with 16-byte loads (CPL columns each),
// the workgroup walks the rows in strides, so each wavefront load instruction
// reads whole row segments (coalesced).  Per-thread partial sums for a chunk of
// MMC rows of V are reduced by a fixed butterfly over the lanes sharing a
// column group and a fixed-order sum over the four wavefronts (deterministic).
template <typename TU> struct VecU;
template <> struct VecU<double> {
    static constexpr int CPL = 2;
    template <typename TC> __device__ static void load(const double* p, TC* u) {
        const double2 v = *reinterpret_cast<const double2*>(p);
        u[0] = static_cast<TC>(v.x);
        u[1] = static_cast<TC>(v.y);
    }
};
template <> struct VecU<float> {
    static constexpr int CPL = 4;
    template <typename TC> __device__ static void load(const float* p, TC* u) {
        const float4 v = *reinterpret_cast<const float4*>(p);
        u[0] = v.x;
        u[1] = v.y;
        u[2] = v.z;
        u[3] = v.w;
    }
};
template <> struct VecU<uint16_t> {
    static constexpr int CPL = 8;
    template <typename TC> __device__ static void load(const uint16_t* p, TC* u) {
        const uint4 v = *reinterpret_cast<const uint4*>(p);
        const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            u[2 * i] = __uint_as_float(w[i] << 16);
            u[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
        }
    }
};

template <int BS, typename TU, typename TC>
__device__ void fd_big_t(int K, int msm, int bsa, const double* V, int sVm, int sVk, const TU* U, int64_t ldu,
                         int c0, double* red, double* C, int sCm, int sCj) {
    constexpr int CPL = VecU<TU>::CPL;
    constexpr int LPR = BS / CPL;  // lanes per row segment
    constexpr int RPW = 64 / LPR;  // rows per wavefront load
    constexpr int RPT = 4 * RPW;   // rows per workgroup pass
    constexpr int ACC = (sizeof(TC) == 8 ? 32 : 64) / CPL;
    constexpr int MMC = ACC < kBigRed / (4 * BS) ? ACC : kBigRed / (4 * BS);
    static_assert(LPR >= 1 && LPR <= 64 && MMC >= 1, "block shape");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int jc = (lane % LPR) * CPL;
    const int r0 = wave * RPW + lane / LPR;
    const bool live = jc < bsa;
    const TU* ub = U + c0 + jc;
    for (int m0 = 0; m0 < msm; m0 += MMC) {
        const int mc = min(MMC, msm - m0);
        TC acc[MMC][CPL];
#pragma unroll
        for (int m = 0; m < MMC; ++m)
#pragma unroll
            for (int j = 0; j < CPL; ++j) acc[m][j] = TC(0);
        if (live) {
#pragma unroll 4
            for (int k = r0; k < K; k += RPT) {
                TC u[CPL];
                VecU<TU>::load(ub + static_cast<int64_t>(k) * ldu, u);
                const double* vk = V + static_cast<int64_t>(m0) * sVm + static_cast<int64_t>(k) * sVk;
#pragma unroll
                for (int m = 0; m < MMC; ++m) {
                    if (m < mc) {
                        const TC v = static_cast<TC>(vk[m * sVm]);
#pragma unroll
                        for (int j = 0; j < CPL; ++j) acc[m][j] += v * u[j];
                    }
                }
            }
        }
#pragma unroll
        for (int m = 0; m < MMC; ++m) {
#pragma unroll
            for (int j = 0; j < CPL; ++j) {
                double v = static_cast<double>(acc[m][j]);
#pragma unroll
                for (int sft = LPR; sft < 64; sft <<= 1) v += __shfl_xor(v, sft, 64);
                if (lane < LPR && m < mc) red[(wave * MMC + m) * BS + jc + j] = v;
            }
        }
        __syncthreads();
        for (int o = threadIdx.x; o < mc * BS; o += kBlock) {
            const int m = o / BS, j = o % BS;
            if (j < bsa) {
                const double t = red[m * BS + j] + red[(MMC + m) * BS + j] + red[(2 * MMC + m) * BS + j] +
                                 red[(3 * MMC + m) * BS + j];
                C[(m0 + m) * sCm + j * sCj] = t;
            }
        }
        __syncthreads();
    }
}

// Dispatch on the block width BS of the grid (8, 16 or 32 columns).
template <typename TU, typename TC>
__device__ __forceinline__ void fd_big(int BS, int K, int msm, int bsa, const double* V, int sVm, int sVk,
                                       const TU* U, int64_t ldu, int c0, double* red, double* C, int sCm, int sCj) {
    if (BS <= 8) fd_big_t<8, TU, TC>(K, msm, bsa, V, sVm, sVk, U, ldu, c0, red, C, sCm, sCj);
    else if (BS <= 16) fd_big_t<16, TU, TC>(K, msm, bsa, V, sVm, sVk, U, ldu, c0, red, C, sCm, sCj);
    else fd_big_t<32, TU, TC>(K, msm, bsa, V, sVm, sVk, U, ldu, c0, red, C, sCm, sCj);
}

// Cooperative copy of an n x n U factor (row stride ldu) into LDS as dense FP64.
template <typename TU>
__device__ __forceinline__ void stage_factor(double* dst, const TU* src, int n, int ldu) {
    for (int i = threadIdx.x; i < n * n; i += kBlock) dst[i] = static_cast<double>(load_val(src, (i / n) * ldu + i % n));
}

// LDS layout of an FD task: R (n) | S (n) | red (kBigRed) | Out | Us | Ub
struct FdLds {
    double *R, *S, *red, *Out, *Us, *Ub;
};
__device__ __forceinline__ FdLds fd_lds(const Grid& g, double* lds) {
    const int n = g.ni[0] * g.ni[1];
    const int nsm = g.ni[1 - g.big];
    FdLds L;
    L.R = lds;
    L.S = lds + n;
    L.red = L.S + n;
    L.Out = L.red + kBigRed;
    L.Us = L.Out + (g.nblk > 1 ? nsm * g.blk : n);
    L.Ub = L.Us + nsm * nsm;
    return L;
}

// Forward transform of one FD block: Rt = (U1 (x) U2)^T r scaled by the
// inverse eigenvalue sums, for the block of the long direction.  The short
// direction's factor (and, for single-block grids, the long one when it fits)
// is staged in LDS first; blocked long directions stream their factor rows.
template <typename TU, typename TC>
__device__ __forceinline__ void fd_fwd_2d(const Params& P, const Grid& g, int blk, const FdIO& io, double* lds) {
    const int n1 = g.ni[0], n2 = g.ni[1], n = n1 * n2;
    const Tab1D& T1 = P.tabs[g.tab[0]];
    const Tab1D& T2 = P.tabs[g.tab[1]];
    const int ld1 = T1.ldu, ld2 = T2.ldu;
    const FdLds L = fd_lds(g, lds);
    const bool wide = g.nblk > 1, sbig = !wide && g.fdstage;
    const int64_t off = g.dof_off;
    double nrm = 0.0;
    for (int i = threadIdx.x; i < n; i += kBlock) {
        double v = io.r_old[off + i];
        if (io.q) v -= io.alpha * io.q[off + i];
        L.R[i] = v;
        const int i1 = i % n1, i2 = i / n1;
        if (owned_2d(g, blk, i1, i2)) {
            if (io.r_out) io.r_out[off + i] = v;
            if (io.dvec) io.dvec[off + i] += io.alpha * io.pvec[off + i];
            nrm += v * v;
        }
    }
    if (g.big == 0) {
        stage_factor(L.Us, u_ptr<TU>(P, T2, true), n2, ld2);
        if (sbig) stage_factor(L.Ub, u_ptr<TU>(P, T1, false), n1, ld1);
    } else {
        stage_factor(L.Us, u_ptr<TU>(P, T1, false), n1, ld1);
        if (sbig) stage_factor(L.Ub, u_ptr<TU>(P, T2, true), n2, ld2);
    }
    if (io.part) {
        double t = wg_sum(nrm, L.red);
        if (threadIdx.x == 0) *io.part = t;
    }
    __syncthreads();
    const int k0 = blk * g.blk;
    const int bs = min(g.blk, g.ni[g.big] - k0);
    const double* lam1 = P.dpool + T1.oLam;
    const double* lam2 = P.dpool + T2.oLam;
    if (g.big == 0) {
        // S[k2][i1] = sum_i2 UT2[k2][i2] R[i2][i1]
        wg_gemm<double, double, TC>(1, n2, n1, n2, L.Us, 0, n2, 1, L.R, 0, n1, 1, L.S, 0, n1, 1, L.red);
        // Rt[k2][k1] = sum_i1 S[k2][i1] U1[i1][k1], k1 in block
        if (wide)
            fd_big<TU, TC>(g.blk, n1, n2, bs, L.S, n1, 1, u_ptr<TU>(P, T1, false), ld1, k0, L.red, L.Out, bs, 1);
        else if (sbig)
            wg_gemm<double, double, TC>(1, n2, bs, n1, L.S, 0, n1, 1, L.Ub + k0, 0, n1, 1, L.Out, 0, bs, 1, L.red);
        else
            wg_gemm<double, TU, TC>(1, n2, bs, n1, L.S, 0, n1, 1, u_ptr<TU>(P, T1, false) + k0, 0, ld1, 1, L.Out,
                                    0, bs, 1, L.red);
        for (int o = threadIdx.x; o < n2 * bs; o += kBlock) {
            const int k2 = o / bs, kk = o % bs, k1 = k0 + kk;
            io.rt[off + static_cast<int64_t>(k2) * n1 + k1] = L.Out[o] / (g.fdc[0] * lam1[k1] + g.fdc[1] * lam2[k2]);
        }
    } else {
        // S[i2][k1] = sum_i1 R[i2][i1] U1[i1][k1]
        wg_gemm<double, double, TC>(1, n2, n1, n1, L.R, 0, n1, 1, L.Us, 0, n1, 1, L.S, 0, n1, 1, L.red);
        // Rt[k2][k1] = sum_i2 U2[i2][k2] S[i2][k1], k2 in block
        if (wide)
            fd_big<TU, TC>(g.blk, n2, n1, bs, L.S, 1, n1, u_ptr<TU>(P, T2, false), ld2, k0, L.red, L.Out, 1, n1);
        else if (sbig)
            wg_gemm<double, double, TC>(1, bs, n1, n2, L.Ub + static_cast<int64_t>(k0) * n2, 0, n2, 1, L.S, 0, n1,
                                        1, L.Out, 0, n1, 1, L.red);
        else
            wg_gemm<TU, double, TC>(1, bs, n1, n2, u_ptr<TU>(P, T2, true) + static_cast<int64_t>(k0) * ld2, 0, ld2,
                                    1, L.S, 0, n1, 1, L.Out, 0, n1, 1, L.red);
        for (int o = threadIdx.x; o < bs * n1; o += kBlock) {
            const int kk = o / n1, k1 = o % n1, k2 = k0 + kk;
            io.rt[off + static_cast<int64_t>(k2) * n1 + k1] = L.Out[o] / (g.fdc[0] * lam1[k1] + g.fdc[1] * lam2[k2]);
        }
    }
    __syncthreads();
}

// Backward transform of one FD block: z = (U1 (x) U2) Rt on the block.
template <typename TU, typename TC>
__device__ __forceinline__ void fd_bwd_2d(const Params& P, const Grid& g, int blk, const FdIO& io, double* lds) {
    const int n1 = g.ni[0], n2 = g.ni[1], n = n1 * n2;
    const Tab1D& T1 = P.tabs[g.tab[0]];
    const Tab1D& T2 = P.tabs[g.tab[1]];
    const int ld1 = T1.ldu, ld2 = T2.ldu;
    const FdLds L = fd_lds(g, lds);
    const bool wide = g.nblk > 1, sbig = !wide && g.fdstage;
    double* Rt = L.R;
    double* Tm = L.S;
    const int64_t off = g.dof_off;
    for (int i = threadIdx.x; i < n; i += kBlock) Rt[i] = io.rt[off + i];
    if (g.big == 0) {
        stage_factor(L.Us, u_ptr<TU>(P, T2, false), n2, ld2);
        if (sbig) stage_factor(L.Ub, u_ptr<TU>(P, T1, true), n1, ld1);
    } else {
        stage_factor(L.Us, u_ptr<TU>(P, T1, true), n1, ld1);
        if (sbig) stage_factor(L.Ub, u_ptr<TU>(P, T2, false), n2, ld2);
    }
    __syncthreads();
    const int k0 = blk * g.blk;
    const int bs = min(g.blk, g.ni[g.big] - k0);
    double dot = 0.0;
    if (g.big == 0) {
        // T[i2][k1] = sum_k2 U2[i2][k2] Rt[k2][k1]
        wg_gemm<double, double, TC>(1, n2, n1, n2, L.Us, 0, n2, 1, Rt, 0, n1, 1, Tm, 0, n1, 1, L.red);
        // Z[i2][i1] = sum_k1 T[i2][k1] UT1[k1][i1], i1 in block
        if (wide)
            fd_big<TU, TC>(g.blk, n1, n2, bs, Tm, n1, 1, u_ptr<TU>(P, T1, true), ld1, k0, L.red, L.Out, bs, 1);
        else if (sbig)
            wg_gemm<double, double, TC>(1, n2, bs, n1, Tm, 0, n1, 1, L.Ub + k0, 0, n1, 1, L.Out, 0, bs, 1, L.red);
        else
            wg_gemm<double, TU, TC>(1, n2, bs, n1, Tm, 0, n1, 1, u_ptr<TU>(P, T1, true) + k0, 0, ld1, 1, L.Out, 0,
                                    bs, 1, L.red);
        for (int o = threadIdx.x; o < n2 * bs; o += kBlock) {
            const int i2 = o / bs, i1 = k0 + o % bs;
            const int64_t gi = off + static_cast<int64_t>(i2) * n1 + i1;
            io.z[gi] = L.Out[o];
            if (io.rdot) dot += io.rdot[gi] * L.Out[o];
        }
    } else {
        // T[k2][i1] = sum_k1 Rt[k2][k1] UT1[k1][i1]
        wg_gemm<double, double, TC>(1, n2, n1, n1, Rt, 0, n1, 1, L.Us, 0, n1, 1, Tm, 0, n1, 1, L.red);
        // Z[i2][i1] = sum_k2 UT2[k2][i2] T[k2][i1], i2 in block
        if (wide)
            fd_big<TU, TC>(g.blk, n2, n1, bs, Tm, 1, n1, u_ptr<TU>(P, T2, true), ld2, k0, L.red, L.Out, 1, n1);
        else if (sbig)
            wg_gemm<double, double, TC>(1, bs, n1, n2, L.Ub + static_cast<int64_t>(k0) * n2, 0, n2, 1, Tm, 0, n1, 1,
                                        L.Out, 0, n1, 1, L.red);
        else
            wg_gemm<TU, double, TC>(1, bs, n1, n2, u_ptr<TU>(P, T2, false) + static_cast<int64_t>(k0) * ld2, 0, ld2,
                                    1, Tm, 0, n1, 1, L.Out, 0, n1, 1, L.red);
        for (int o = threadIdx.x; o < bs * n1; o += kBlock) {
            const int i2 = k0 + o / n1, i1 = o % n1;
            const int64_t gi = off + static_cast<int64_t>(i2) * n1 + i1;
            io.z[gi] = L.Out[o];
            if (io.rdot) dot += io.rdot[gi] * L.Out[o];
        }
    }
    if (io.part) {
        double t = wg_sum(dot, L.red);
        if (threadIdx.x == 0) *io.part = t;
    }
    __syncthreads();
}

// FD transforms for a factor precision fixed at compile time
// (0: FP64 factors, 1: FP32 factors, 2: BF16 factors with FP32 accumulation).
template <int FDP>
__device__ __forceinline__ void fd_fwd_p(const Params& P, const Grid& g, int blk, const FdIO& io, double* lds) {
    if constexpr (FDP == 0) fd_fwd_2d<double, double>(P, g, blk, io, lds);
    else if constexpr (FDP == 1) fd_fwd_2d<float, float>(P, g, blk, io, lds);
    else fd_fwd_2d<uint16_t, float>(P, g, blk, io, lds);
}
template <int FDP>
__device__ __forceinline__ void fd_bwd_p(const Params& P, const Grid& g, int blk, const FdIO& io, double* lds) {
    if constexpr (FDP == 0) fd_bwd_2d<double, double>(P, g, blk, io, lds);
    else if constexpr (FDP == 1) fd_bwd_2d<float, float>(P, g, blk, io, lds);
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
    unsigned long long* trace;    // phase timestamps (or nullptr)
    int trace_sweeps;
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
enum { PK_PQ = 0, PK_RES = 1, PK_RR = 2, PK_RZ = 3 };
enum { ACT_SKIP = 0, ACT_RESID, ACT_ITER, ACT_XUPD, ACT_DONE };

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

__device__ inline Decision decide(const SolveArgs& A, const GState& st, double rho) {
    Decision D;
    D.status = GS_OK;
    D.rho = rho;
    D.rhob = st.rhob;
    D.rho0 = st.rho0;
    if (st.stage == STAGE_DONE) {
        D.act = ACT_SKIP;
    } else if (st.stage == STAGE_RESID) {
        D.act = ACT_RESID;
    } else if (st.stage == STAGE_XUPD) {
        D.act = ACT_XUPD;
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
    } else if (rho <= A.tol_in2 * st.rho0 || st.it >= A.maxit) {
        D.act = ACT_XUPD;
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
};
constexpr int kCtxDoubles = 32;  // LDS slots reserved for TaskCtx
static_assert(sizeof(TaskCtx) <= kCtxDoubles * sizeof(double), "TaskCtx too large");

__device__ __forceinline__ void task_context(const Params& P, const SolveArgs& A, const Grid& g,
                                             const GState* S0, int gi, int cur, int nxt, int phase,
                                             TaskCtx* ctx) {
    __syncthreads();  // previous users of the LDS context are done
    if (threadIdx.x < 64) {
        // every load is issued before any is used: one memory round trip
        const GState st = S0[gi];
        const int lane = threadIdx.x;
        double vrz = 0.0, vpq = 0.0, vres = 0.0;
        const double* prz = part_ptr(P, PK_RZ, nxt) + g.blk_off;
        const double* ppq = part_ptr(P, PK_PQ, cur) + g.tile_off;
        const double* pres = part_ptr(P, PK_RES, cur) + g.tile_off;
        for (int i = lane; i < g.nblk; i += 64) vrz += prz[i];
        if (phase >= 2)
            for (int i = lane; i < g.ntile; i += 64) {
                vpq += ppq[i];
                vres += pres[i];
            }
        for (int o = 32; o > 0; o >>= 1) {
            vrz += __shfl_xor(vrz, o, 64);
            vpq += __shfl_xor(vpq, o, 64);
            vres += __shfl_xor(vres, o, 64);
        }
        const Decision D = decide(A, st, st.stage == STAGE_ITER ? vrz : 0.0);
        if (threadIdx.x == 0) {
            ctx->st = st;
            ctx->D = D;
            ctx->pq = (phase >= 2 && D.act == ACT_ITER) ? vpq : 0.0;
            ctx->rn2 = (phase == 3 && D.act == ACT_RESID) ? vres : 0.0;
        }
    }
    __syncthreads();
}

template <int PP, int FDP>
__global__ void __launch_bounds__(kBlock) k_solve(Params P, SolveArgs A) {
    extern __shared__ double lds_all[];
    TaskCtx* ctx = reinterpret_cast<TaskCtx*>(lds_all);
    double* lds = lds_all + kCtxDoubles;  // task work arrays
    const unsigned nwg = gridDim.x;
    const int64_t N = P.ndof_total;
    const int lowp = FDP != 0;
    if (A.trace && blockIdx.x == 0 && threadIdx.x == 0) A.trace[0] = wall_clock64();
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
        for (int t = A.op_b + blockIdx.x; t < A.op_e; t += nwg) {
            const Task tk = P.optask[t];
            const Grid& g = P.grids[tk.grid];
            task_context(P, A, g, S0, tk.grid, cur, nxt, 1, ctx);
            const int act = ctx->D.act;
            if (act == ACT_SKIP) {
                if (tk.local == 0 && threadIdx.x == 0) S1[tk.grid] = ctx->st;  // carry DONE forward
                continue;
            }
            OpIO io;
            if (act == ACT_ITER) {
                io.in_a = P.z;
                io.in_b = p_old;
                io.beta = ctx->st.it == 0 ? 0.0 : ctx->D.rho / ctx->st.rho;
                io.out_in = p_new;
                io.out = P.q;
                io.rhs = nullptr;
                io.part = part_ptr(P, PK_PQ, cur) + g.tile_off + tk.local;
                io.lowp = lowp;
            } else if (act == ACT_RESID) {
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
        trace_busy(A, sweep, 0, tb);
        grid_barrier(P.bar, nwg);
        trace_mark(A, sweep, 0);
        if (A.trace) tb = wall_clock64();
        // ---------------- phase 2: update + FD forward ---------------------------
        for (int t = A.fd_b + blockIdx.x; t < A.fd_e; t += nwg) {
            const Task tk = P.fdtask[t];
            const Grid& g = P.grids[tk.grid];
            task_context(P, A, g, S0, tk.grid, cur, nxt, 2, ctx);
            const int act = ctx->D.act;
            if (act == ACT_XUPD) {
                const int n1 = g.ni[0];
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
            io.prec = FDP;
            io.z = nullptr;
            io.rdot = nullptr;
            io.part = part_ptr(P, PK_RR, cur) + g.blk_off + tk.local;
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
                io.q = nullptr;
                io.r_out = nullptr;
                io.dvec = nullptr;
                io.pvec = nullptr;
            } else {
                continue;
            }
            fd_fwd_p<FDP>(P, g, tk.local, io, lds);
        }
        trace_busy(A, sweep, 1, tb);
        grid_barrier(P.bar, nwg);
        trace_mark(A, sweep, 1);
        if (A.trace) tb = wall_clock64();
        // ---------------- phase 3: FD backward and commit ---------------------------
        for (int t = A.fd_b + blockIdx.x; t < A.fd_e; t += nwg) {
            const Task tk = P.fdtask[t];
            const int gi = tk.grid;
            const Grid& g = P.grids[gi];
            task_context(P, A, g, S0, gi, cur, nxt, 3, ctx);
            const int act = ctx->D.act;
            if (act == ACT_SKIP) continue;
            bool run_bwd = act == ACT_RESID || (act == ACT_ITER && ctx->pq > 0.0 && isfinite(ctx->D.rho / ctx->pq));
            if (run_bwd) {
                FdIO io;
                io.rt = P.rt;
                io.z = P.z;
                io.rdot = r_new;
                io.prec = FDP;
                io.part = part_ptr(P, PK_RZ, cur) + g.blk_off + tk.local;
                fd_bwd_p<FDP>(P, g, tk.local, io, lds);
            }
            if (tk.local == 0 && threadIdx.x == 0) {
                const GState& st = ctx->st;
                const Decision& D = ctx->D;
                GState ns = st;
                bool finish = false;
                if (act == ACT_ITER) {
                    ns.rhob = D.rhob;
                    ns.rho0 = D.rho0;
                    if (!run_bwd) {
                        ns.stage = STAGE_DONE;
                        ns.status = GS_BREAKDOWN;
                        ns.total_it += st.it;
                        finish = true;
                    } else {
                        ns.stage = STAGE_ITER;
                        ns.it = st.it + 1;
                        ns.rho = D.rho;
                    }
                } else if (act == ACT_XUPD) {
                    ns.stage = STAGE_RESID;
                    ns.total_it += st.it;
                    ns.prelres = D.rhob > 0.0 ? sqrt(D.rho / D.rhob) : 0.0;
                } else if (act == ACT_RESID) {
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
                S1[gi] = ns;
                if (finish) atomicAdd(&P.bar[2], 1u);
            }
        }
        trace_busy(A, sweep, 2, tb);
        grid_barrier(P.bar, nwg);
        trace_mark(A, sweep, 2);
        if (A.trace && blockIdx.x == 0 && threadIdx.x == 0) P.bar[3] = sweep + 1;
        const unsigned done = __hip_atomic_load(&P.bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (static_cast<int>(done) >= A.ndone_target) break;
    }
}

}  // namespace igasg
