// common.hpp -- data structures shared by the host plan and the gfx950 kernels.
//
// A plan describes every component grid of the combination technique
// (eq. TD-combi-tec) as a tensor grid with per-direction 1D tables.  All
// device data lives in one caller-provided workspace; the structures below
// hold byte offsets into it, fixed at plan time.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define IGA_HD __host__ __device__
#else
#define IGA_HD
#endif

namespace igasg {

constexpr int kMaxDim = 3;
constexpr int kMaxP = 4;          // solution degree limit (register arrays)
constexpr int kMaxPg = 4;         // geometry degree limit
constexpr int kMaxPatch = 4;
// Threads per workgroup: 512 (8 wavefronts) in every kernel; the 3D
// persistent solve has a second build whose translation units define
// IGASG_THREADS 256: one 4-wavefront workgroup per CU gets the whole register
// file there (the 512-thread build holds 256 VGPRs and spills about 1 KB per
// lane).
#ifndef IGASG_THREADS
#define IGASG_THREADS 512
#endif
constexpr int kBlock = IGASG_THREADS;
constexpr int kBlockSolve3 = 256;  // threads of the 3D solve kernels
constexpr int kWaves = kBlock / 64;
constexpr int kFdStream = -2;   // Grid::fdstage of a grid solved by whole-device kernels
constexpr int kBigRed = 2048;     // doubles of LDS for cross-wavefront partial sums of FD tasks

// Grid stages of the persistent refinement/CG state machine.
enum Stage : int { STAGE_RESID = 0, STAGE_ITER = 1, STAGE_DONE = 2 };
// Per-component status codes reported to the host.
enum GridStatus : int { GS_RUNNING = -1, GS_OK = 0, GS_MAXIT = 5, GS_BREAKDOWN = 6 };

// 1D data of one (patch, direction, level): knots, Gauss tables, FD factors.
struct Tab1D {
    int nb;       // B-spline basis functions
    int ni;       // interior functions (nb - 2)
    int E;        // elements (non-empty knot intervals)
    int Q;        // quadrature points = E * nq
    int m;        // interior knot multiplicity p - r
    int pg;       // geometry degree in this direction
    int ngb;      // geometry basis functions
    int nk;       // solution knots
    int ngk;      // geometry knots
    int uniform;  // breakpoints are i / E
    int ldu;      // row stride of the U tables (multiple of 8 elements)
    int lo;       // basis index of the first unknown (1: the first function is a Dirichlet one)
    // double-pool offsets (in elements)
    int64_t oB, oD;       // [Q][p+1] basis values / derivatives at the Gauss points
    int64_t oBg, oDg;     // [Q][pg+1] geometry basis values / derivatives
    int64_t oXq, oWq;     // [Q] parametric coordinate, weight (incl. element half length)
    int64_t oBrk;         // [E+1] breakpoints
    int64_t oKn;          // [nk] solution knots
    int64_t oGkn;         // [ngk] geometry knots
    int64_t oU, oUT;      // [ni][ni] eigenvectors (U[i][k]) and transpose
    int64_t oLam;         // [ni]
    int64_t oKd, oMd;     // [ni] diagonals of the 1D stiffness and mass matrices of the pencil
    // int-pool offsets
    int64_t oGs;          // [Q] first geometry basis index at each Gauss point
    // float-pool and bf16-pool offsets
    int64_t oU32, oUT32;
    int64_t oU16, oUT16;
};

// One component grid (one patch of one combination component).
struct Grid {
    int lev[3];
    int ni[3];        // interior unknowns per direction (1 beyond dim)
    int nb[3];
    int E[3];
    int Q[3];
    int tab[3];       // Tab1D index per direction
    int patch;
    int comp;         // combination component index
    int64_t dof_off;  // offset of the interior unknowns in the vector pool
    int64_t ndof;
    int64_t qp_off;   // offset of the Gauss-point data (per component field)
    int64_t nqp;
    double ccoef;     // combination coefficient
    double fdc[3];    // per-direction scaling of the fast-diagonalisation pencil
    int64_t oDinv;    // double pool: 1 / (sum of the pencil eigenvalues), ndof values
    // fast-diagonalisation task split (2D: blocks of the longest direction)
    int big;          // direction split into blocks
    int nblk;
    int blk;          // block length
    int blk_off;      // first FD task
    int fdstage;      // 2D single-block grids: the long direction's factor is staged in LDS; blocked
                      // grids: 0 the block's slab is staged, -1 it is read from memory (long grids);
                      // kFdStream: a full tensor grid too large for the LDS of one workgroup, solved
                      // by whole-device kernels with the grid vectors in memory
    // operator tiles
    int tile[3];      // tile size in unknowns per direction
    int ntd[3];       // tiles per direction
    int ntile;
    int tile_off;     // first operator task
    int sample;       // coefficient sample (plans of several samples)
    // several patches: the grids of one component instance (one per patch,
    // consecutive) form one linear system with one solver state; its partial
    // sums span the group's operator tiles and FD blocks
    int state;        // grid index holding the group's solver state (the first of the group)
    int gtile_off, gntile, gblk_off, gnblk;
    // conforming C^0 interfaces (2D): for side s (0: xi1 = 0, 1: xi1 = 1,
    // 2: xi2 = 0, 3: xi2 = 1) in nbr_on, the unknown of the neighbouring
    // patch's grid that shares the unknown at tangential index t of that side
    // sits at dof_off + nbr_base[s] + nbr_stride[s] * t
    int nbr_on;
    int nbr_base[4], nbr_stride[4];
    int pin[4];       // unknowns fixed to their Dirichlet value (a vertex between two interfaces), or -1
    int64_t lift_off; // offset of the grid's full coefficient array of the Dirichlet lift (2D)
};

// Per-grid solver state (double-buffered by sweep parity on the device).
struct GState {
    double rho;       // r.z of the previous iteration (CG beta)
    double rho0;      // r.z at the start of the current inner solve
    double rhob;      // b.P^-1 b (reference for the outer test)
    double bn2;       // ||b||^2
    double relres;    // last FP64 relative residual ||b - A x|| / ||b||
    double prelres;   // last preconditioned relative residual sqrt(r.P^-1 r / b.P^-1 b)
    int stage;
    int it;           // iterations of the current inner solve
    int total_it;
    int refine;       // inner solves started
    int status;
    int op64;         // the inner solve uses the FP64 operator (after an inner breakdown of the
                      // FP32 operator: it lost positive definiteness on a badly graded grid)
};

struct Task {
    int grid;
    int local;
};

// A task's grid and 1D tables, copied into LDS once per solve launch so that
// the tasks of a sweep read their description without a memory round trip.
struct TaskMeta {
    Grid g;
    Tab1D t[kMaxDim];
    int grid, local;
};
static_assert(sizeof(Grid) % 8 == 0 && sizeof(Tab1D) % 8 == 0 && sizeof(TaskMeta) % 8 == 0, "8-byte words");
constexpr int kMetaOp = 2;     // cached operator tasks per workgroup
constexpr int kMetaFd = 5;     // cached fast-diagonalisation tasks per workgroup
constexpr int kMetaSlots = kMetaOp + kMetaFd + 1;  // + one slot for tasks beyond the cache
constexpr int kCtxBytes = 256;  // LDS for the per-task context
constexpr int kLdsLimit = 160 * 1024;  // LDS per workgroup on gfx950
// learned preconditioner 3 -> h1 -> h2 -> 1: the largest hidden layers, and
// the LDS bytes per unknown of its BF16 activations (3 features padded to 8
// channels, h1, h2) and FP32 output
constexpr int kNnMaxH1 = 32;
constexpr int kNnMaxH2 = 48;
constexpr int kNnLdsBytesPerDof = 2 * (8 + kNnMaxH1 + kNnMaxH2) + 4;
// packed BF16 weights of the largest network: [16 ceil(cout/16)][27][cin rounded to 8] per layer
constexpr int kNnPackedMax = 32 * 27 * 8 + 48 * 27 * kNnMaxH1 + 16 * 27 * kNnMaxH2;

// LDS layout (byte offsets) of a 2D fast-diagonalisation task:
//   R, S      two grid-sized FP64 work vectors
//   red       cross-wavefront partial sums
//   Out       block output
//   Own       three FP64 values per owned unknown (fetched operands)
//   Us, Ub    staged factor rows (short direction; long direction of a
//             single-block grid) in the factor precision, row stride ldu
//   Slab      long-direction factor rows of a blocked grid: rows x kBlock
//             threads x 16 bytes, in the order the threads consume them
struct FdLayout {
    int R, S, red, Out, Own, Us, Ub, Slab, rows, total;
};
// rows of the slab per thread for block width bs (16-byte chunks of 16/usize values)
inline IGA_HD int fd_slab_rows(int nbig, int bs, int usize) {
    const int rpt = kBlock * (16 / usize) / bs;  // rows per workgroup pass
    return (nbig + rpt - 1) / rpt;
}
inline IGA_HD FdLayout fd_layout(const Grid& g, int ldu_s, int ldu_b, int usize) {
    const int n = g.ni[0] * g.ni[1], nsm = g.ni[1 - g.big], nbig = g.ni[g.big];
    const bool wide = g.nblk > 1;
    const int bs = g.blk < nbig ? g.blk : nbig;
    FdLayout L;
    int o = 0;
    L.R = o;
    o += 8 * n;
    L.S = o;
    o += 8 * n;
    L.red = o;
    o += 8 * kBigRed;
    L.Out = o;
    o += 8 * (wide ? nsm * bs : n);
    L.Own = o;
    o += 8 * 3 * nsm * bs;
    o = (o + 15) & ~15;
    L.Us = o;
    o += nsm * ldu_s * usize;
    o = (o + 15) & ~15;
    L.Ub = o;
    if (!wide && g.fdstage) o += nbig * ldu_b * usize;
    o = (o + 15) & ~15;
    L.Slab = o;
    L.rows = wide && g.fdstage >= 0 ? fd_slab_rows(nbig, bs, usize) : 0;  // fdstage -1: slab read from memory
    o += L.rows * kBlock * 16;
    L.total = o;
    return L;
}

// LDS layout (byte offsets) of a 3D fast-diagonalisation task (one task per
// grid): three grid-sized FP64 work tensors R, S, T; red; three FP64 values
// per unknown (fetched operands); the factors U1, U2, U3 in the factor
// precision (row strides ld[k]) for the directions whose bit is set in
// g.fdstage (the others are read from global memory).  Reuses FdLayout: Us
// holds U1, Ub U2, Slab U3, Out the third work tensor.
inline IGA_HD FdLayout fd_layout_3d(const Grid& g, const int* ld, int usize) {
    const int n = g.ni[0] * g.ni[1] * g.ni[2];
    FdLayout L;
    int o = 0;
    L.R = o;
    o += 8 * n;
    L.S = o;
    o += 8 * n;
    L.Out = o;  // third work tensor T
    o += 8 * n;
    L.red = o;
    o += 8 * kBigRed;
    L.Own = o;
    o += 8 * 3 * n;
    o = (o + 15) & ~15;
    L.Us = o;
    if (g.fdstage & 1) o += g.ni[0] * ld[0] * usize;
    o = (o + 15) & ~15;
    L.Ub = o;
    if (g.fdstage & 2) o += g.ni[1] * ld[1] * usize;
    o = (o + 15) & ~15;
    L.Slab = o;
    if (g.fdstage & 4) o += g.ni[2] * ld[2] * usize;
    o = (o + 15) & ~15;
    L.rows = 0;
    L.total = o;
    return L;
}
constexpr size_t kSolveLdsHead = kCtxBytes + kMetaSlots * sizeof(TaskMeta);

// Workspace layout: byte offsets of every device array.
// Barrier block (unsigned words): generation, finished-grid count, traced
// sweeps, the next grid of the whole-grid solve, the global arrival count on its own 64-byte line, the group arrival
// counts one line apart; bytes 64..67 hold the assembly error flag.
// The lengths of the active task lists (operator and fast-diagonalisation,
// by sweep parity) follow on a line of their own.
constexpr int kBarGen = 1, kBarDone = 2, kBarSweeps = 3, kBarNext = 4, kBarCount = 32, kBarGroup = 64,
              kBarStride = 16;
constexpr int kBarGroups = 8;
constexpr int kBarOpLen = kBarGroup + kBarStride * kBarGroups;  // + parity
constexpr int kBarFdLen = kBarOpLen + 2;                        // + parity
constexpr int kBarBytes = 4 * (kBarOpLen + kBarStride);
// whole-device solves of a full tensor grid: reduction blocks and partial-sum kinds
constexpr int kFgBlocks = 256;
constexpr int kFgKinds = 4;
constexpr int kFgScalars = 32;

struct Layout {
    size_t tabs, grids, grids_lp, dpool, ipool, fpool, hpool, ctrl;
    size_t G64, G32, Fq;          // operator coefficients and load density at Gauss points
                                  // (per grid [coefficient][point]; the points in tensor
                                  // order in 2D, element-major in 3D)
    size_t b, x, d, r2, z, p2, q, rt;
    size_t st2;                   // GState[2][ngrid]
    size_t part;                  // partial sums
    size_t optask, fdtask, fdtask_lp;
    size_t loga;                  // log a at the Greville points of the unknowns
    size_t fdscale;               // diagonal scaling of the preconditioner
    size_t loc;                   // element-local load and diagonal sums [2][nloc][nelem]
    size_t lift;                  // Dirichlet lift, full coefficient arrays per grid (2D)
    size_t gmeta, gmeta_lp;       // TaskMeta per grid (FP64 / low-precision FD blocking)
    size_t oplist, fdlist;        // active task lists [2 parities][tasks]
    size_t bar;                   // barrier + counters
    size_t trace;                 // phase timestamps
    size_t fg;                    // whole-device solves: partial sums [kFgKinds][kFgBlocks], scalars
    size_t nnw;                   // packed BF16 network weights (kNnPackedMax)
    size_t total;
};

// Kernel parameter block (passed by value).
struct Params {
    const Tab1D* tabs;
    const Grid* grids;
    const double* dpool;
    const int* ipool;
    const float* fpool;
    const uint16_t* hpool;
    const double* ctrl;      // homogeneous control points [patch][...][4]
    int64_t ctrl_off[kMaxPatch];
    int gdeg[kMaxPatch][3];
    int gn[kMaxPatch][3];    // geometry basis counts
    int rational[kMaxPatch];
    int dim, p, nq, ncompG;  // ncompG: operator coefficients per Gauss point
    int ngrid, nop, nfd;
    int ngrid1;                // grids of one sample (grids are sample-major)
    int64_t nqp1, ndof1;       // Gauss points and unknowns of one sample
    int64_t nqp_total, ndof_total;
    double* G64;
    float* G32;
    double* Fq;
    double* b;
    double* x;
    double* d;
    double* r2;        // two buffers of ndof_total
    double* z;
    double* p2;        // two buffers
    double* q;
    double* rt;
    GState* st2;       // two buffers of ngrid
    double* part;      // partial sums: [6 kinds][2 parity][max(nop, nfd)]
    int64_t part_stride;
    const Task* optask;
    const Task* fdtask;
    unsigned* bar;     // [0] count, [1] generation, [2] done counter
    double gx[8], gw[8];  // Gauss-Legendre rule on [-1, 1]
    double* loga;      // log a at the Greville points of the unknowns [ndof_total]
    double* fdscale;   // s = sqrt(diag(P) / diag(A)) per unknown [ndof_total]; nullptr in a
                       // solve without scaling
    double* loc;       // element-local sums: operator diagonal [nloc][nelem], then load [nloc][nelem]
    int64_t nelem;     // elements over all grids (Gauss points / (p+1)^d)
    const TaskMeta* gmeta;  // description of every grid with its 1D tables (local = 0)
    Task* oplist;      // active operator tasks [2][op_cap] (by sweep parity)
    Task* fdlist;      // active fast-diagonalisation tasks [2][fd_cap]
    int op_cap, fd_cap;
    const double* lift;  // Dirichlet lift coefficients (full arrays per grid), nullptr without data
    double* lift_rw;     // the lift arrays (written by the assembly)
    int mp;            // several patches: interface sums and grouped solver states
    const float* nn;   // learned preconditioner parameters (or nullptr)
    const uint16_t* nnw;  // its weights packed in BF16 (workspace; filled at each learned solve)
    uint16_t* nnw_rw;
    int nn_ch[4];      // channels of its three layers (3, h1, h2, 1)
    int nn_head;       // 0: z = z_FD + s y; 1: z = z_FD exp(y)
};

}  // namespace igasg
