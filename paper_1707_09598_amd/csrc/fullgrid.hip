// fullgrid.hip -- the full tensor-product grid at level w on the whole
// device, and the sparse-grid combination as its coarse correction.
//
// A full grid at the sizes of the paper's comparison (Sec. 4.2: standard IGA
// against SG-IGA at matched accuracy) holds tens of thousands of unknowns,
// more than the LDS of one workgroup, which the persistent solve keeps its
// fast-diagonalisation vectors in.  Here the grid's vectors stay in memory
// and each step of FD-preconditioned CG is a launch over the whole device:
// the operator over its tiles (the persistent solve's tile code), the mode
// products of the preconditioner as batched FP64 matrix-core GEMMs, and
// elementwise updates with fixed-order partial sums (bitwise reproducible).
//
// The combination of Sec. 3 (eq. TD-combi-tec) as a preconditioner of the
// full problem (the outlook of Sec. 5): the component spaces are nested in the
// full space, so a residual r of the full problem restricts to each
// component (P_i^T r, P_i the tensor prolongation), the components are solved
// by the sparse-grid plan's batched solve, and y = sum_i c_i P_i u_i is
// prolonged back.  y leaves the part of the error outside the sparse-grid
// space untouched, so the preconditioner is the two-level product
// z = y + S P^-1 S (r - A y) with the full grid's fast diagonalisation as the
// second level, applied inside flexible CG (the product is not a fixed SPD
// operator: the combination coefficients have both signs and the inner
// solves stop at a tolerance).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

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
namespace {

// scalars of a whole-device solve (double slots after the partial sums)
enum : int {
    FS_ALPHA = 0,  // step length
    FS_BETA,       // direction update
    FS_RZ,         // r . z (z the search preconditioner's output)
    FS_PQ,         // p . A p
    FS_RR,         // ||r||^2
    FS_RF,         // r . P^-1 r (P the full grid's fast diagonalisation): the stopping test
    FS_ZQ,         // z . q of the previous direction (flexible CG)
    FS_BB,         // ||b||^2
    FS_RF0,        // b . P^-1 b
    FS_RP,         // r . p (flexible CG step length)
};
// partial-sum kinds
enum : int { FK_A = 0, FK_B = 1, FK_C = 2, FK_D = 3 };

constexpr int kGemmM = 64, kGemmN = 32;  // output block of one workgroup (8 MFMA tiles)

struct GemmArgs {
    int M, N, K, nb;
    const double* A;
    int sAm, sAk;
    int64_t sAb;
    const double* B;
    int sBk, sBn;
    int64_t sBb;
    double* C;
    int sCm, sCn;
    int64_t sCb;
    const double* E;  // C = alpha (A B) .* E + beta C, E with the offsets of C (or nullptr: 1)
    double alpha, beta;
};

// Batched FP64 GEMM on the matrix cores, operands in memory: workgroup
// (x, y, z) forms the 64 x 32 output block (x, y) of batch z in LDS
// (mfma_gemm: 16x16x4 FP64 MFMA, two accumulator chains per tile), then
// applies the epilogue.  Each output is written by one thread.
__global__ void __launch_bounds__(kBlock) k_fg_gemm(GemmArgs g) {
    __shared__ double tile[kGemmM * kGemmN];
    __shared__ double red[kBigRed];
    const int m0 = blockIdx.x * kGemmM, n0 = blockIdx.y * kGemmN, b = blockIdx.z;
    const int Mb = min(kGemmM, g.M - m0), Nb = min(kGemmN, g.N - n0);
    if (Mb <= 0 || Nb <= 0) return;
    mfma_gemm<double, double, double>(Mb, Nb, g.K, g.A + b * g.sAb + static_cast<int64_t>(m0) * g.sAm, g.sAm, g.sAk,
                                      g.B + b * g.sBb + static_cast<int64_t>(n0) * g.sBn, g.sBk, g.sBn, tile, kGemmN,
                                      1, 1, 0, 0, 0, red);
    for (int o = threadIdx.x; o < Mb * kGemmN; o += kBlock) {
        const int i = o / kGemmN, j = o - i * kGemmN;
        if (j >= Nb) continue;
        const int64_t at = b * g.sCb + static_cast<int64_t>(m0 + i) * g.sCm + static_cast<int64_t>(n0 + j) * g.sCn;
        double v = g.alpha * tile[i * kGemmN + j];
        if (g.E) v *= g.E[at];
        if (g.beta != 0.0) v += g.beta * g.C[at];
        g.C[at] = v;
    }
}

// q = A p over the grid's operator tiles (the persistent solve's tile code);
// out = rhs - A in when io.rhs is set.  part[t]: in . (A in) (or ||rhs - A in||^2) of tile t.
template <int PP>
__global__ void __launch_bounds__(kBlock) k_fg_op(Params P, int gi, OpIO io, double* part) {
    extern __shared__ double lds_all[];
    TaskMeta* M = reinterpret_cast<TaskMeta*>(reinterpret_cast<char*>(lds_all) + kCtxBytes);
    double* lds = reinterpret_cast<double*>(reinterpret_cast<char*>(lds_all) + kSolveLdsHead);
    meta_fill(P, Task{gi, 0}, M);
    for (int t = blockIdx.x; t < M->g.ntile; t += gridDim.x) {
        OpIO a = io;
        a.part = part ? part + t : nullptr;
        if (P.dim == 3) op_tile_3d<PP>(P, M->g, M->t[0], M->t[1], M->t[2], t, a, lds);
        else op_tile_2d<PP>(P, M->g, M->t[0], M->t[1], t, a, lds);
    }
}

// Sum of n partials in index order by one thread (n is at most a few
// thousand operator tiles, or kFgBlocks): the same sum on every run.
__device__ __forceinline__ double ordered_sum(const double* v, int n) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += v[i];
    return s;
}

// Step length: alpha = num / (p . q), num = r . z (CG) or r . p (flexible CG).
__global__ void k_fg_alpha(double* sc, const double* part, int n, int num_slot) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double pq = ordered_sum(part, n);
    sc[FS_PQ] = pq;
    sc[FS_ALPHA] = pq > 0.0 ? sc[num_slot] / pq : 0.0;
}

// x += alpha p, r -= alpha q, w = s .* r; part: ||r||^2 per block.
__global__ void __launch_bounds__(kBlock) k_fg_update(int64_t n, double* x, double* r, const double* p,
                                                       const double* q, const double* s, double* w,
                                                       const double* sc, double* part) {
    __shared__ double red[kWaves];
    const double a = sc[FS_ALPHA];
    double rr = 0.0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock) {
        x[i] += a * p[i];
        const double v = r[i] - a * q[i];
        r[i] = v;
        w[i] = s[i] * v;
        rr += v * v;
    }
    const double t = wg_sum(rr, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// w = s .* v (the scaled input of the fast diagonalisation); part: v . v per
// block (nullptr: none).
__global__ void __launch_bounds__(kBlock) k_fg_scale(int64_t n, const double* v, const double* s, double* w,
                                                      double* part) {
    __shared__ double red[kWaves];
    double vv = 0.0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock) {
        w[i] = s[i] * v[i];
        vv += v[i] * v[i];
    }
    if (part) {
        const double t = wg_sum(vv, red);
        if (threadIdx.x == 0) part[blockIdx.x] = t;
    }
}

// z = s .* Z (+ y); part_a: r . (s .* Z); part_b: z . q (flexible CG; q nullptr: none).
__global__ void __launch_bounds__(kBlock) k_fg_finish(int64_t n, const double* Z, const double* s, const double* y,
                                                       const double* r, const double* q, double* z, double* part_a,
                                                       double* part_b) {
    __shared__ double red[kWaves];
    double da = 0.0, db = 0.0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock) {
        const double zf = s[i] * Z[i];
        da += r[i] * zf;
        const double v = y ? y[i] + zf : zf;
        if (z) z[i] = v;
        if (q) db += v * q[i];
    }
    if (part_a) {
        const double t = wg_sum(da, red);
        if (threadIdx.x == 0) part_a[blockIdx.x] = t;
    }
    if (part_b) {
        const double t = wg_sum(db, red);
        if (threadIdx.x == 0) part_b[blockIdx.x] = t;
    }
}

// p = z + beta p; part: r . p per block (flexible CG step length).
__global__ void __launch_bounds__(kBlock) k_fg_dir(int64_t n, const double* z, double* p, const double* r,
                                                    const double* sc, double* part) {
    __shared__ double red[kWaves];
    const double be = sc[FS_BETA];
    double rp = 0.0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock) {
        const double v = z[i] + be * p[i];
        p[i] = v;
        rp += r[i] * v;
    }
    if (part) {
        const double t = wg_sum(rp, red);
        if (threadIdx.x == 0) part[blockIdx.x] = t;
    }
}

// Reduce the partial sums of one iteration into the scalars.  mode 0 (CG):
// rz = sum A (= r . z), rr = sum B, beta = rz / rz_old; mode 1 (flexible CG):
// rz = sum A (z . r), rf = sum C (r . P^-1 r), zq = sum D, beta = -zq / pq;
// mode 2: initial values (rr and rf also stored as ||b||^2 and b . P^-1 b);
// mode 3: beta = 0 (the first direction of a (re)start).
__global__ void k_fg_scalars(double* sc, const double* part, int mode, int nb) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (mode == 3) {
        sc[FS_BETA] = 0.0;
        return;
    }
    const double a = ordered_sum(part + FK_A * kFgBlocks, nb);
    const double rr = ordered_sum(part + FK_B * kFgBlocks, nb);
    if (mode == 0) {
        const double old = sc[FS_RZ];
        sc[FS_BETA] = old > 0.0 ? a / old : 0.0;
        sc[FS_RZ] = a;
        sc[FS_RF] = a;
        sc[FS_RR] = rr;
    } else if (mode == 1) {
        const double rf = ordered_sum(part + FK_C * kFgBlocks, nb);
        const double zq = ordered_sum(part + FK_D * kFgBlocks, nb);
        sc[FS_ZQ] = zq;
        sc[FS_BETA] = sc[FS_PQ] > 0.0 ? -zq / sc[FS_PQ] : 0.0;
        sc[FS_RZ] = a;
        sc[FS_RF] = rf;
        sc[FS_RR] = rr;
    } else {
        sc[FS_BETA] = 0.0;
        sc[FS_RZ] = a;
        sc[FS_RF] = a;
        sc[FS_RR] = rr;
        sc[FS_BB] = rr;
        sc[FS_RF0] = a;
    }
}
__global__ void k_fg_set(double* sc, int slot, const double* part, int nb) {
    if (threadIdx.x == 0 && blockIdx.x == 0) sc[slot] = ordered_sum(part, nb);
}
__global__ void __launch_bounds__(kBlock) k_fg_copy(int64_t n, const double* a, double* b) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock)
        b[i] = a[i];
}
__global__ void __launch_bounds__(kBlock) k_fg_axpy(int64_t n, double c, const double* a, double* b) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock)
        b[i] += c * a[i];
}
__global__ void __launch_bounds__(kBlock) k_fg_fill(int64_t n, double* a, double v) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock)
        a[i] = v;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct Mat {  // element [o][i] = ptr[o * so + i * si]
    const double* ptr;
    int so, si;
};

// Mode-k product of a tensor X with dims n[0..d) (direction 1 fastest):
// Y[.., o, ..] = sum_i M[o][i] X[.., i, ..] with nout outputs along k;
// Y = alpha (M x_k X) .* E + beta Y.
iga_status mode_product(hipStream_t st, int d, const int* n, int k, int nout, Mat M, const double* X, double* Y,
                        const double* E = nullptr, double alpha = 1.0, double beta = 0.0) {
    int inner = 1, outer = 1;
    for (int j = 0; j < k; ++j) inner *= n[j];
    for (int j = k + 1; j < d; ++j) outer *= n[j];
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    g.E = E;
    g.alpha = alpha;
    g.beta = beta;
    if (k == 0) {
        // Y[r][o] = sum_i X[r][i] M[o][i], r over the other directions
        g.M = outer;
        g.N = nout;
        g.K = n[0];
        g.nb = 1;
        g.A = X;
        g.sAm = n[0];
        g.sAk = 1;
        g.B = M.ptr;
        g.sBk = M.si;
        g.sBn = M.so;
        g.C = Y;
        g.sCm = nout;
        g.sCn = 1;
    } else {
        // Y[b][o][j] = sum_i M[o][i] X[b][i][j], b over the directions above k
        g.M = nout;
        g.N = inner;
        g.K = n[k];
        g.nb = outer;
        g.A = M.ptr;
        g.sAm = M.so;
        g.sAk = M.si;
        g.B = X;
        g.sBk = inner;
        g.sBn = 1;
        g.sBb = static_cast<int64_t>(n[k]) * inner;
        g.C = Y;
        g.sCm = inner;
        g.sCn = 1;
        g.sCb = static_cast<int64_t>(nout) * inner;
    }
    if (g.M <= 0 || g.N <= 0 || g.nb <= 0) return IGA_OK;
    const dim3 grid((g.M + kGemmM - 1) / kGemmM, (g.N + kGemmN - 1) / kGemmN, g.nb);
    if (grid.y > 65535u || grid.z > 65535u) {
        set_error("mode product too large for one launch (%d x %d, batch %d)", g.M, g.N, g.nb);
        return IGA_ERR_INVALID_ARG;
    }
    hipLaunchKernelGGL(k_fg_gemm, grid, dim3(kBlock), 0, st, g);
    HIP_OK(hipGetLastError());
    return IGA_OK;
}

int fg_blocks(int64_t n) {
    const int64_t b = (n + kBlock - 1) / kBlock;
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(b, kFgBlocks)));
}

// The whole-device state of a full-grid solve: device pointers into the
// plan's workspace.
struct Fg {
    iga_sg_plan_s* P;
    Params K;
    hipStream_t st;
    const Grid* g;
    int d, n[3];
    int64_t N;
    int nb;            // reduction blocks
    double *x, *r, *w, *p, *y, *q, *z, *S, *R, *s, *b;
    double* part;      // [kFgKinds][kFgBlocks]
    double* sc;        // scalars
    double* optpart;   // per-tile partials of the operator
    Mat U[3], UT[3];   // fast-diagonalisation factors: backward [i][k], forward [k][i]
    const double* dinv;
};

Fg fg_setup(iga_sg_plan_s* P) {
    Fg F;
    F.P = P;
    F.K = make_params(P, false);
    F.st = static_cast<hipStream_t>(P->stream);
    F.g = &P->grids[0];
    F.d = P->dim;
    for (int k = 0; k < 3; ++k) F.n[k] = F.g->ni[k];
    F.N = F.g->ndof;
    F.nb = fg_blocks(F.N);
    const int64_t N = P->ndof_total;
    F.x = F.K.x;
    F.r = F.K.r2;
    F.w = F.K.r2 + N;
    F.p = F.K.p2;
    F.y = F.K.p2 + N;
    F.q = F.K.q;
    F.z = F.K.z;
    F.S = F.K.d;
    F.R = F.K.rt;
    F.s = F.K.fdscale;
    F.b = F.K.b;
    char* base = reinterpret_cast<char*>(P->ws);
    F.part = reinterpret_cast<double*>(base + P->lay.fg);
    F.sc = F.part + kFgKinds * kFgBlocks;
    F.optpart = F.K.part;  // the persistent solve's partial sums, >= one per operator tile
    for (int k = 0; k < F.d; ++k) {
        const Tab1D& T = P->tabs[F.g->tab[k]];
        const double* U = F.K.dpool + T.oU;  // U[i][k] row-major, row stride ldu
        F.U[k] = Mat{U, T.ldu, 1};
        F.UT[k] = Mat{U, 1, T.ldu};
    }
    F.dinv = F.K.dpool + F.g->oDinv;
    return F;
}

template <int PP>
void launch_op(const Fg& F, const OpIO& io, double* part) {
    const size_t lds = F.P->lds_bytes;
    hipLaunchKernelGGL(k_fg_op<PP>, dim3(F.g->ntile), dim3(kBlock), lds, F.st, F.K, 0, io, part);
}
// out = A in (part: in . A in per tile), or out = rhs - A in
iga_status fg_op(const Fg& F, const double* in, double* out, const double* rhs, double* part) {
    OpIO io;
    io.in_a = in;
    io.in_b = nullptr;
    io.beta = 0.0;
    io.out_in = nullptr;
    io.out = out;
    io.rhs = rhs;
    io.part = nullptr;
    io.lowp = 0;
    io.isum = 0;
    switch (F.P->p) {
        case 1: launch_op<1>(F, io, part); break;
        case 2: launch_op<2>(F, io, part); break;
        case 3: launch_op<3>(F, io, part); break;
        default: launch_op<4>(F, io, part); break;
    }
    HIP_OK(hipGetLastError());
    return IGA_OK;
}

// Z = (U_1 (x) .. (x) U_d) diag(1/sum lambda) (..)^T W; W is overwritten.
// Buffers: W (input, then scratch), S, R (scratch); Z must differ from W, S.
iga_status fg_fd(const Fg& F, double* W, double* Z) {
    const int d = F.d;
    int dims[3] = {F.n[0], F.n[1], F.n[2]};
    iga_status s;
    if (d == 2) {
        if ((s = mode_product(F.st, 2, dims, 0, dims[0], F.UT[0], W, F.S))) return s;
        if ((s = mode_product(F.st, 2, dims, 1, dims[1], F.UT[1], F.S, F.R, F.dinv))) return s;
        if ((s = mode_product(F.st, 2, dims, 1, dims[1], F.U[1], F.R, F.S))) return s;
        if ((s = mode_product(F.st, 2, dims, 0, dims[0], F.U[0], F.S, Z))) return s;
    } else {
        if ((s = mode_product(F.st, 3, dims, 0, dims[0], F.UT[0], W, F.S))) return s;
        if ((s = mode_product(F.st, 3, dims, 1, dims[1], F.UT[1], F.S, W))) return s;
        if ((s = mode_product(F.st, 3, dims, 2, dims[2], F.UT[2], W, F.R, F.dinv))) return s;
        if ((s = mode_product(F.st, 3, dims, 2, dims[2], F.U[2], F.R, W))) return s;
        if ((s = mode_product(F.st, 3, dims, 1, dims[1], F.U[1], W, F.S))) return s;
        if ((s = mode_product(F.st, 3, dims, 0, dims[0], F.U[0], F.S, Z))) return s;
    }
    return IGA_OK;
}

struct FgHost {
    double sc[kFgScalars];
};

iga_status fg_read(const Fg& F, FgHost* h) {
    HIP_OK(hipMemcpyAsync(h->sc, F.sc, sizeof(double) * kFgScalars, hipMemcpyDeviceToHost, F.st));
    HIP_OK(hipStreamSynchronize(F.st));
    return IGA_OK;
}

// Two-level context: the sparse-grid plan and its components' prolongations.
struct TwoLevel {
    iga_sg_plan_s* G;   // sparse-grid plan (bound, assembled)
    const iga_sg_solve_opts* inner;
    int every;          // coarse correction on iterations it % every == 0 (0: first only)
    long inner_iters = 0;
    int coarse = 0;
};

Mat xfer(const Fg& F, int k, int lev, bool transpose) {
    const iga_sg_plan_s* P = F.P;
    const int nc = P->tabs[tab_index(P, 0, k, lev)].ni;
    const double* T = F.K.dpool + P->xfer_off[static_cast<size_t>(k) * (P->w + 1) + lev];
    // T[if][jc] row-major [nf][nc]
    return transpose ? Mat{T, 1, nc} : Mat{T, nc, 1};
}

// y = sum_i c_i P_i A_i^-1 P_i^T v (sparse-grid plan solve in between)
iga_status fg_coarse(const Fg& F, TwoLevel& TL, const double* v, double* y) {
    iga_sg_plan_s* G = TL.G;
    const int d = F.d;
    Params KG = make_params(G, false);
    iga_status s;
    // restriction of v to every component's right-hand side
    for (const Grid& gc : G->grids) {
        int dims[3] = {F.n[0], F.n[1], F.n[2]};
        const double* src = v;
        double* bufs[2] = {F.S, F.R};
        for (int k = 0; k < d; ++k) {
            const int nc = gc.ni[k];
            double* dst = k == d - 1 ? KG.b + gc.dof_off : bufs[k & 1];
            if (gc.lev[k] == F.P->w) {
                if (k == d - 1) {
                    hipLaunchKernelGGL(k_fg_copy, dim3(fg_blocks(gc.ndof)), dim3(kBlock), 0, F.st, gc.ndof, src, dst);
                    HIP_OK(hipGetLastError());
                }
                else continue;
            } else {
                if ((s = mode_product(F.st, d, dims, k, nc, xfer(F, k, gc.lev[k], true), src, dst))) return s;
            }
            dims[k] = nc;
            src = dst;
        }
    }
    // the components' solves
    iga_sg_report rep;
    std::memset(&rep, 0, sizeof(rep));
    iga_status ss = iga_sg_solve(G, TL.inner, &rep);
    if (ss != IGA_OK && ss != IGA_ERR_NOT_CONVERGED) return ss;
    TL.inner_iters += rep.total_iters;
    TL.coarse += 1;
    // y = sum_i c_i P_i u_i, components in plan order
    hipLaunchKernelGGL(k_fg_fill, dim3(fg_blocks(F.N)), dim3(kBlock), 0, F.st, F.N, y, 0.0);
    HIP_OK(hipGetLastError());
    for (const Grid& gc : G->grids) {
        int dims[3] = {gc.ni[0], gc.ni[1], gc.ni[2]};
        const double* src = KG.x + gc.dof_off;
        double* bufs[2] = {F.S, F.R};
        int last = -1;  // last direction that changes size
        for (int k = 0; k < d; ++k)
            if (gc.lev[k] != F.P->w) last = k;
        if (last < 0) {  // the component is the full grid itself
            hipLaunchKernelGGL(k_fg_axpy, dim3(fg_blocks(F.N)), dim3(kBlock), 0, F.st, F.N, gc.ccoef, src, y);
            HIP_OK(hipGetLastError());
        }
        for (int k = 0; k < d; ++k) {
            if (gc.lev[k] == F.P->w) continue;
            const int nf = F.n[k];
            const bool fin = k == last;
            double* dst = fin ? y : bufs[k & 1];
            if ((s = mode_product(F.st, d, dims, k, nf, xfer(F, k, gc.lev[k], false), src, dst, nullptr,
                                  fin ? gc.ccoef : 1.0, fin ? 1.0 : 0.0)))
                return s;
            dims[k] = nf;
            src = dst;
        }
    }
    return IGA_OK;
}

// The two-level product up to its last scaling: y = sum_i c_i P_i A_i^-1
// P_i^T r, then t = r - A y and the transform Z of S t, left in F.z (the
// caller forms z = y + S Z).
iga_status fg_two_level(const Fg& F, TwoLevel& TL) {
    iga_status s;
    if ((s = fg_coarse(F, TL, F.r, F.y))) return s;
    if ((s = fg_op(F, F.y, F.z, F.r, nullptr))) return s;  // t = r - A y
    hipLaunchKernelGGL(k_fg_scale, dim3(F.nb), dim3(kBlock), 0, F.st, F.N, F.z, F.s, F.w, nullptr);
    HIP_OK(hipGetLastError());
    return fg_fd(F, F.w, F.z);
}

// Full-grid solve on the whole device: CG preconditioned by the full grid's
// fast diagonalisation (TL == nullptr), or flexible CG with the two-level
// preconditioner.  The stopping test is that of the persistent solve,
// r . P^-1 r <= tol^2 b . P^-1 b with P the fast diagonalisation, on the
// recursive residual; when it passes, the FP64 residual b - A x replaces the
// recursive one and the test is repeated (at most max_refine times).
iga_status fg_solve(iga_sg_plan_s* P, const iga_sg_solve_opts* o, iga_sg_report* rep, TwoLevel* TL) {
    Fg F = fg_setup(P);
    const int nb = F.nb;
    const dim3 eg(nb), eb(kBlock);
    double* pa = F.part + FK_A * kFgBlocks;
    double* pb = F.part + FK_B * kFgBlocks;
    double* pc = F.part + FK_C * kFgBlocks;
    double* pd = F.part + FK_D * kFgBlocks;
    const double tol2 = o->tol * o->tol;
    const int max_restart = std::max(1, o->max_refine > 0 ? o->max_refine : 3);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (o->timing) {
        for (int i = 0; i < 2; ++i)
            if (!P->ev[i]) HIP_OK(hipEventCreate(reinterpret_cast<hipEvent_t*>(&P->ev[i])));
        e0 = static_cast<hipEvent_t>(P->ev[0]);
        e1 = static_cast<hipEvent_t>(P->ev[1]);
        HIP_OK(hipEventRecord(e0, F.st));
    }
    iga_status s;
    hipLaunchKernelGGL(k_fg_fill, dim3(fg_blocks(F.N)), eb, 0, F.st, F.N, F.x, 0.0);
    HIP_OK(hipGetLastError());
    int it = 0, restarts = 0, status = GS_MAXIT;
    double rf0 = 0.0, bb = 0.0, rf = 0.0, rr = 0.0;
    FgHost h;
    for (int start = 0; start <= max_restart; ++start) {
        // r = b - A x (x = 0 at the first start: r = b)
        if (start == 0) {
            hipLaunchKernelGGL(k_fg_copy, dim3(fg_blocks(F.N)), eb, 0, F.st, F.N, F.b, F.r);
            HIP_OK(hipGetLastError());
        } else {
            if ((s = fg_op(F, F.x, F.r, F.b, nullptr))) return s;
        }
        // z = P^-1 r, r . z, ||r||^2
        hipLaunchKernelGGL(k_fg_scale, eg, eb, 0, F.st, F.N, F.r, F.s, F.w, pb);
        HIP_OK(hipGetLastError());
        if ((s = fg_fd(F, F.w, F.z))) return s;
        hipLaunchKernelGGL(k_fg_finish, eg, eb, 0, F.st, F.N, F.z, F.s, nullptr, F.r, nullptr, F.z, pa, nullptr);
        HIP_OK(hipGetLastError());
        hipLaunchKernelGGL(k_fg_scalars, dim3(1), dim3(64), 0, F.st, F.sc, F.part, start == 0 ? 2 : 0, nb);
        HIP_OK(hipGetLastError());
        if ((s = fg_read(F, &h))) return s;
        if (start == 0) {
            rf0 = h.sc[FS_RF0];
            bb = h.sc[FS_BB];
        }
        rf = h.sc[FS_RF];
        rr = h.sc[FS_RR];
        if (rf0 <= 0.0 || rf <= tol2 * rf0) {
            status = GS_OK;
            break;
        }
        if (start == max_restart || it >= o->maxit) break;
        restarts = start;
        // the first search direction: the two-level output when it applies
        if (TL) {
            if ((s = fg_two_level(F, *TL))) return s;
            hipLaunchKernelGGL(k_fg_finish, eg, eb, 0, F.st, F.N, F.z, F.s, F.y, F.r, nullptr, F.z, pa, nullptr);
            HIP_OK(hipGetLastError());
            hipLaunchKernelGGL(k_fg_set, dim3(1), dim3(64), 0, F.st, F.sc, FS_RZ, pa, nb);
            HIP_OK(hipGetLastError());
        }
        hipLaunchKernelGGL(k_fg_fill, dim3(fg_blocks(F.N)), eb, 0, F.st, F.N, F.p, 0.0);
        HIP_OK(hipGetLastError());
        // beta = 0 on a (re)start: p = z
        hipLaunchKernelGGL(k_fg_scalars, dim3(1), dim3(64), 0, F.st, F.sc, F.part, 3, 0);
        HIP_OK(hipGetLastError());
        bool conv = false;
        while (it < o->maxit) {
            hipLaunchKernelGGL(k_fg_dir, eg, eb, 0, F.st, F.N, F.z, F.p, F.r, F.sc, TL ? pc : nullptr);
            HIP_OK(hipGetLastError());
            if (TL) {
                hipLaunchKernelGGL(k_fg_set, dim3(1), dim3(64), 0, F.st, F.sc, FS_RP, pc, nb);
                HIP_OK(hipGetLastError());
            }
            if ((s = fg_op(F, F.p, F.q, nullptr, F.optpart))) return s;
            hipLaunchKernelGGL(k_fg_alpha, dim3(1), dim3(64), 0, F.st, F.sc, F.optpart, F.g->ntile, TL ? FS_RP : FS_RZ);
            HIP_OK(hipGetLastError());
            hipLaunchKernelGGL(k_fg_update, eg, eb, 0, F.st, F.N, F.x, F.r, F.p, F.q, F.s, F.w, F.sc, pb);
            HIP_OK(hipGetLastError());
            ++it;
            if (!TL) {
                if ((s = fg_fd(F, F.w, F.z))) return s;
                hipLaunchKernelGGL(k_fg_finish, eg, eb, 0, F.st, F.N, F.z, F.s, nullptr, F.r, nullptr, F.z, pa,
                                   nullptr);
                HIP_OK(hipGetLastError());
                hipLaunchKernelGGL(k_fg_scalars, dim3(1), dim3(64), 0, F.st, F.sc, F.part, 0, nb);
                HIP_OK(hipGetLastError());
            } else {
                // r . P^-1 r for the stopping test
                if ((s = fg_fd(F, F.w, F.z))) return s;
                hipLaunchKernelGGL(k_fg_finish, eg, eb, 0, F.st, F.N, F.z, F.s, nullptr, F.r, nullptr, nullptr, pc,
                                   nullptr);
                HIP_OK(hipGetLastError());
                const bool coarse = TL->every > 0 && it % TL->every == 0;
                if (coarse) {
                    if ((s = fg_two_level(F, *TL))) return s;
                    hipLaunchKernelGGL(k_fg_finish, eg, eb, 0, F.st, F.N, F.z, F.s, F.y, F.r, F.q, F.z, pa, pd);
                } else {
                    // the fast diagonalisation alone: z = S (the transform of S r left in z above)
                    hipLaunchKernelGGL(k_fg_finish, eg, eb, 0, F.st, F.N, F.z, F.s, nullptr, F.r, F.q, F.z, pa, pd);
                }
                HIP_OK(hipGetLastError());
                hipLaunchKernelGGL(k_fg_scalars, dim3(1), dim3(64), 0, F.st, F.sc, F.part, 1, nb);
                HIP_OK(hipGetLastError());
            }
            if ((s = fg_read(F, &h))) return s;
            rf = h.sc[FS_RF];
            rr = h.sc[FS_RR];
            if (!(std::isfinite(rf)) || (!TL && h.sc[FS_PQ] <= 0.0)) {
                status = GS_BREAKDOWN;
                break;
            }
            if (rf <= tol2 * rf0) {
                conv = true;
                break;
            }
        }
        if (status == GS_BREAKDOWN || !conv) break;
        // converged on the recursive residual: check the FP64 residual at the next start
    }
    // ||b - A x||^2 of the final iterate
    if ((s = fg_op(F, F.x, F.r, F.b, F.optpart))) return s;
    hipLaunchKernelGGL(k_fg_set, dim3(1), dim3(64), 0, F.st, F.sc, FS_RR, F.optpart, F.g->ntile);
    HIP_OK(hipGetLastError());
    if (o->timing) HIP_OK(hipEventRecord(e1, F.st));
    if ((s = fg_read(F, &h))) return s;
    rr = h.sc[FS_RR];
    P->solved = true;
    if (rep) {
        rep->ncomp = 1;
        rep->total_iters = it;
        rep->precision = IGA_PREC_FP64;
        rep->lam_ratio = P->lam_ratio;
        rep->sweeps = TL ? static_cast<int>(TL->inner_iters) : 0;
        if (rep->iters) rep->iters[0] = it;
        if (rep->refinements) rep->refinements[0] = restarts;
        if (rep->relres) rep->relres[0] = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
        if (rep->prelres) rep->prelres[0] = rf0 > 0.0 ? std::sqrt(std::max(rf, 0.0) / rf0) : 0.0;
        if (rep->status) rep->status[0] = status;
        if (o->timing) {
            float ms = 0.0f;
            HIP_OK(hipEventElapsedTime(&ms, e0, e1));
            rep->kernel_ms[1] = ms;
        }
    }
    if (status == GS_BREAKDOWN) {
        set_error("CG breakdown in the full-grid solve");
        return IGA_ERR_BREAKDOWN;
    }
    if (status != GS_OK) {
        set_error("the full-grid solve did not reach the tolerance");
        return IGA_ERR_NOT_CONVERGED;
    }
    return IGA_OK;
}

}  // namespace

iga_status fg_solve_plain(iga_sg_plan_s* P, const iga_sg_solve_opts* o, iga_sg_report* rep) {
    return fg_solve(P, o, rep, nullptr);
}

}  // namespace igasg

namespace {

bool same_knots(const iga_sg_plan_s* A, int ta, const iga_sg_plan_s* B, int tb) {
    const Tab1D& X = A->tabs[ta];
    const Tab1D& Y = B->tabs[tb];
    if (X.nk != Y.nk || X.lo != Y.lo || X.ni != Y.ni) return false;
    for (int i = 0; i < X.nk; ++i)
        if (std::fabs(A->dpool[X.oKn + i] - B->dpool[Y.oKn + i]) > 1e-14) return false;
    return true;
}

}  // namespace

extern "C" {

iga_status iga_sg_solve_twolevel(iga_sg_plan full, iga_sg_plan sg, const iga_sg_solve_opts* outer,
                                 const iga_sg_solve_opts* inner, int coarse_every, iga_sg_report* report) {
    if (!full || !sg || !outer || !inner || coarse_every < 0) {
        set_error("invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    if (full->xfer_off.empty() || full->grids.size() != 1 || full->nsamples != 1) {
        set_error("the first plan must be a full tensor plan of one patch and one sample");
        return IGA_ERR_INVALID_ARG;
    }
    if (sg->patches.size() != 1 || sg->nsamples != 1 || sg->dim != full->dim || sg->p != full->p ||
        sg->r != full->r) {
        set_error("the sparse-grid plan must have one patch, one sample and the full plan's dimension, "
                  "degree and regularity");
        return IGA_ERR_INVALID_ARG;
    }
    for (const Grid& g : sg->grids)
        for (int k = 0; k < sg->dim; ++k) {
            if (g.lev[k] > full->w ||
                !same_knots(sg, g.tab[k], full, tab_index(full, 0, k, g.lev[k]))) {
                set_error("component levels (%d in direction %d) must be nested in the full plan's level %d "
                          "with the same knots", g.lev[k], k + 1, full->w);
                return IGA_ERR_INVALID_ARG;
            }
        }
    if (!full->assembled || !sg->assembled) {
        set_error("iga_sg_solve_twolevel before iga_sg_assemble of both plans");
        return IGA_ERR_STATE;
    }
    if (full->stream != sg->stream) {
        set_error("both plans must be bound to the same stream");
        return IGA_ERR_INVALID_ARG;
    }
    if (!(outer->tol > 0) || outer->maxit < 1) {
        set_error("invalid solve options");
        return IGA_ERR_INVALID_ARG;
    }
    if (const iga_status ws = workspace_ok(full)) return ws;
    if (const iga_status ws = workspace_ok(sg)) return ws;
    TwoLevel TL;
    TL.G = sg;
    TL.inner = inner;
    TL.every = coarse_every;
    return fg_solve(full, outer, report, &TL);
}

}  // extern "C"
