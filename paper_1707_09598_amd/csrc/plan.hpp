// plan.hpp -- host-side plan of the sparse-grid solver.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "iga_sg.h"
#include "common.hpp"

struct iga_sg_plan_s;

namespace igasg {

void set_error(const char* fmt, ...);

struct PatchHost {
    int degree[3];
    std::vector<double> knots[3];
    std::vector<double> ctrl;      // [..][dim]
    std::vector<double> weights;   // empty => polynomial
    int grading[3];
    double gamma[3];
};

// Host Cox-de Boor: values and first derivatives of the p+1 functions that
// are non-zero on knot interval s (knots[s] <= x < knots[s+1]).
void basis_funs(int p, const double* U, int s, double x, double* N, double* dN);
int find_interval(int p, int nk, const double* U, double x);
double grade_map(int kind, double gamma, double t);
void gauss_rule(int n, double* x, double* w);

}  // namespace igasg

struct iga_sg_plan_s {
    int dim = 0, p = 0, r = 0, w = 0, lmin = 0, nq = 0;
    std::vector<igasg::PatchHost> patches;
    std::vector<iga_interface> ifaces;
    int bc[igasg::kMaxPatch][6] = {};          // 1: Dirichlet side, 0: interface side
    int pin_corner[igasg::kMaxPatch][4] = {};  // vertex between two interfaces with a fixed value
    // components of the combination technique
    int ncomp = 0;
    int nsamples = 1;              // coefficient samples planned together
    std::vector<int> comp_levels;  // [ncomp][dim]
    std::vector<double> comp_coef;
    // tables and pools
    int Lmax = 0;
    std::vector<igasg::Tab1D> tabs;
    std::vector<double> dpool;
    std::vector<int> ipool;
    std::vector<float> fpool;
    std::vector<uint16_t> hpool;
    std::vector<double> gauss_x, gauss_w;
    // per (patch, dir, level) 1D interior matrices (dense, host only)
    std::vector<std::vector<double>> K1d, M1d;
    std::vector<igasg::Grid> grids;      // FD blocking for FP64 factors
    std::vector<igasg::Grid> grids_lp;   // same grids, FD blocking for FP32/BF16 factors
    std::vector<igasg::Task> optask, fdtask, fdtask_lp;
    std::vector<igasg::TaskMeta> gmeta, gmeta_lp;  // host copies of the per-grid task descriptions
    std::vector<double> ctrl;  // homogeneous control points, concatenated per patch
    int64_t ctrl_off[igasg::kMaxPatch] = {0, 0, 0, 0};
    int ncompG = 0;
    int rational_any = 0;
    int64_t nqp_total = 0, ndof_total = 0;
    double lam_ratio = 1.0;       // largest max/min eigenvalue ratio of the 1D tables the grids use
    int64_t nlift = 0;            // doubles of the Dirichlet lift arrays (2D: all basis functions of every grid)
    bool lifted = false;          // the last assembly had Dirichlet data
    size_t lds_bytes = 0;
    size_t lds_plain = 0;  // LDS of a solve without the learned preconditioner (3D: no activations)
    bool streamed = false;  // a full tensor grid solved by whole-device kernels (kFdStream)
    // full tensor plans (one patch): the prolongation from level l to level w in
    // direction k, interior unknowns, row-major [ni(w)][ni(l)] in the double
    // pool at xfer_off[k * (w + 1) + l] (-1 where absent)
    std::vector<int64_t> xfer_off;
    // index-set plans with keep_all: per grid the grids of levels b - z,
    // z in {0,1}^d (-1 for a negative level), [ngrid][8] in the int pool
    int64_t detail_off = -1;
    igasg::Layout lay{};
    // binding
    void* ws = nullptr;
    size_t ws_bytes = 0;
    void* stream = nullptr;
    bool bound = false, assembled = false, solved = false;
    int num_cu = 0;
    int max_wg = 0;
    void* ev[8] = {nullptr};  // timing events
    void* gexec = nullptr;    // instantiated graph of one step (iga_sg_graph_capture)
    int last_solve_coop = 1;  // the last solve launched the cooperative kernel (else the whole-grid one)
    int static_dev = -1;      // device whose static workspace the plan is bound to (iga_sg_bind_static)
    uint64_t static_gen = 0;  // that device's binding count at this plan's binding
    const float* nn = nullptr;  // learned preconditioner parameters (device, caller-owned)
    int nn_ch[4] = {0, 0, 0, 0};
    int nn_head = 0;
};

namespace igasg {
int tab_index(const iga_sg_plan_s* P, int patch, int dir, int lev);
Params make_params(iga_sg_plan_s* P, bool lowp_fd = false);
// IGA_ERR_STATE when the plan's static workspace was taken over by another plan
iga_status workspace_ok(const iga_sg_plan_s* P);
// whole-device FD-preconditioned CG of a full tensor plan's single grid
iga_status fg_solve_plain(iga_sg_plan_s* P, const iga_sg_solve_opts* o, iga_sg_report* rep);
}  // namespace igasg
