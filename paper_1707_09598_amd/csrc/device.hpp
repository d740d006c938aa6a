// device.hpp -- device helpers shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace igasg {

// de Boor's triangular scheme (values and first derivatives of the p+1
// B-splines non-zero on knot interval s), as on the host.
// Cox-de Boor values (and first derivatives) of the p+1 B-splines that are
// non-zero on knot span s, by the triangular scheme (left/right differences).
// Loops run to the compile-time bound PMAX with p <= PMAX masked at run time,
// so every array index is a constant and the arrays stay in registers.
template <int PMAX>
__device__ __forceinline__ void d_basis_funs_m(int p, const double* U, int s, double x, double* N, double* dN) {
    double left[PMAX + 2], right[PMAX + 2];
    double t[PMAX + 1][PMAX + 1];
#pragma unroll
    for (int i = 0; i <= PMAX; ++i)
#pragma unroll
        for (int j = 0; j <= PMAX; ++j) t[i][j] = 0.0;
    t[0][0] = 1.0;
#pragma unroll
    for (int j = 1; j <= PMAX; ++j) {
        if (j > p) break;
        left[j] = x - U[s + 1 - j];
        right[j] = U[s + j] - x;
        double saved = 0.0;
#pragma unroll
        for (int r = 0; r < j; ++r) {
            t[j][r] = right[r + 1] + left[j - r];
            const double tmp = t[r][j - 1] / t[j][r];
            t[r][j] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        t[j][j] = saved;
    }
    // N[r] = t[r][p]; dN from the degree p-1 functions and the knot differences
    // t[p][r] (selected by a compile-time degree so that indices stay constant)
#pragma unroll
    for (int pp = 0; pp <= PMAX; ++pp) {
        if (pp != p) continue;
#pragma unroll
        for (int r = 0; r <= pp; ++r) {
            N[r] = t[r][pp];
            if (dN) {
                double v = 0.0;
                if (pp >= 1) {
                    if (r >= 1) v += t[r - 1][pp - 1] / t[pp][r - 1];
                    if (r <= pp - 1) v -= t[r][pp - 1] / t[pp][r];
                }
                dN[r] = pp * v;
            }
        }
    }
}
__device__ __forceinline__ void d_basis_funs(int p, const double* U, int s, double x, double* N, double* dN) {
    d_basis_funs_m<kMaxPg>(p, U, s, x, N, dN);
}

__device__ __forceinline__ int d_find_interval(int p, int nk, const double* U, double x) {
    int n = nk - p - 1;
    if (x >= U[n]) {
        int s = n - 1;
        while (s > p && !(U[s] < U[s + 1])) --s;
        return s;
    }
    if (x <= U[p]) return p;
    int lo = p, hi = n;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (x < U[mid]) hi = mid;
        else lo = mid;
    }
    return lo;
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float(static_cast<unsigned>(h) << 16);
}

template <typename T>
__device__ __forceinline__ float load_f(const T* p, int64_t i);
template <>
__device__ __forceinline__ float load_f<float>(const float* p, int64_t i) { return p[i]; }
template <>
__device__ __forceinline__ float load_f<uint16_t>(const uint16_t* p, int64_t i) { return bf16_to_f32(p[i]); }

// Value of lane (lane ^ M), M = 1, 2, 4 or 8, by DPP moves: a VALU operation
// inside a row of 16 lanes, without the LDS round trip of ds_bpermute.
//   M = 1, 2: quad permutations (1,0,3,2) and (2,3,0,1);
//   M = 4: lane i reads i + 4 (row shift left) when bit 2 of i is clear and
//          i - 4 (row shift right) when it is set;
//   M = 8: row rotation by 8, i -> (i + 8) mod 16 = i ^ 8.
// Every lane of the row must be active.
template <int M>
__device__ __forceinline__ int lane_xor_i(int v) {
    static_assert(M == 1 || M == 2 || M == 4 || M == 8, "DPP lane exchange inside a row");
    if constexpr (M == 1) {
        return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);
    } else if constexpr (M == 2) {
        return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);
    } else if constexpr (M == 4) {
        const int up = __builtin_amdgcn_update_dpp(0, v, 0x104, 0xF, 0xF, false);
        const int dn = __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);
        return (threadIdx.x & 4) ? dn : up;
    } else {
        return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);
    }
}
template <int M>
__device__ __forceinline__ float lane_xor(float v) {
    return __int_as_float(lane_xor_i<M>(__float_as_int(v)));
}
template <int M>
__device__ __forceinline__ double lane_xor(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = lane_xor_i<M>(static_cast<int>(b));
    const int hi = lane_xor_i<M>(static_cast<int>(b >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Reduce-scatter over an aligned group of NG = 2, 4 or 8 lanes: c[k] is this
// lane's share of output k; the result is the group's sum of output
// j = lane % NG.  Pairs are summed first (xor 1), then pairs of pairs (xor 2,
// xor 4): ((c_0 + c_1) + (c_2 + c_3)) + ... for every output, in every lane,
// the order of a butterfly of xor steps 1, 2, 4.
template <int NG, typename T>
__device__ __forceinline__ T group_reduce_scatter(const T (&c)[NG], int j) {
    static_assert(NG == 2 || NG == 4 || NG == 8, "group of 2, 4 or 8 lanes");
    const bool b0 = j & 1;
    T h[NG / 2];
#pragma unroll
    for (int k = 0; k < NG / 2; ++k) {
        const T mine = b0 ? c[2 * k + 1] : c[2 * k];
        const T send = b0 ? c[2 * k] : c[2 * k + 1];
        h[k] = mine + lane_xor<1>(send);  // output 2k + (j & 1)
    }
    if constexpr (NG == 2) {
        return h[0];
    } else {
        const bool b1 = j & 2;
        T q[NG / 4];
#pragma unroll
        for (int k = 0; k < NG / 4; ++k) {
            const T mine = b1 ? h[2 * k + 1] : h[2 * k];
            const T send = b1 ? h[2 * k] : h[2 * k + 1];
            q[k] = mine + lane_xor<2>(send);  // output 4k + (j & 3)
        }
        if constexpr (NG == 4) {
            return q[0];
        } else {
            const bool b2 = j & 4;
            const T mine = b2 ? q[1] : q[0];
            const T send = b2 ? q[0] : q[1];
            return mine + lane_xor<4>(send);
        }
    }
}

// Deterministic workgroup sum (fixed butterfly, then fixed LDS order): xor 32
// and 16 by ds_bpermute, xor 8, 4, 2, 1 by DPP.
__device__ __forceinline__ double wg_sum(double v, double* red) {
    v += __shfl_xor(v, 32, 64);
    v += __shfl_xor(v, 16, 64);
    v += lane_xor<8>(v);
    v += lane_xor<4>(v);
    v += lane_xor<2>(v);
    v += lane_xor<1>(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += red[w];
    __syncthreads();
    return s;
}

// Sum of count partials (fixed order per lane, fixed shuffle tree); every
// thread of the workgroup gets the result.
__device__ __forceinline__ double sum_partials(const double* part, int count, double* red) {
    double v = 0.0;
    if (threadIdx.x < 64)
        for (int i = threadIdx.x; i < count; i += 64) v += part[i];
    if (threadIdx.x < 64)
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if (threadIdx.x == 0) red[0] = v;
    __syncthreads();
    double s = red[0];
    __syncthreads();
    return s;
}

// Exact quotient and remainder of i / d for 0 <= i < 2^21 and d >= 1 from a
// float reciprocal and one correction step: division by a run-time integer
// is a long dependent instruction sequence on the GPU.  The float product has
// relative error below 2^-23, so the truncated quotient is off by at most one.
struct FDiv {
    int d;
    float rcp;
    __device__ explicit FDiv(int d_) : d(d_), rcp(1.0f / static_cast<float>(d_)) {}
    __device__ __forceinline__ int div(int i, int* rem) const {
        int q = static_cast<int>(static_cast<float>(i) * rcp);
        int r = i - q * d;
        if (r < 0) {
            --q;
            r += d;
        } else if (r >= d) {
            ++q;
            r -= d;
        }
        *rem = r;
        return q;
    }
};

// x / m for the knot multiplicity m (1 for maximal regularity).
__device__ __forceinline__ int div_mult(int x, int m) { return m == 1 ? x : x / m; }

// Element range touching unknowns [a, b) of one direction whose first
// unknown is basis function lo (1 after a Dirichlet end, 0 after an interface).
__device__ __forceinline__ void d_elem_range(int a, int b, int p, int m, int E, int lo, int* elo, int* ehi) {
    const int lo_basis = a + lo, hi_basis = b - 1 + lo;
    const int e0 = (lo_basis - p <= 0) ? 0 : div_mult(lo_basis - p + m - 1, m);
    const int e1 = div_mult(hi_basis, m);
    *elo = e0 < 0 ? 0 : e0;
    *ehi = e1 > E - 1 ? E - 1 : e1;
}

}  // namespace igasg
