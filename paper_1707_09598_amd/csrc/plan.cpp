// plan.cpp -- host plan of the sparse-grid isogeometric solver: index set and
// combination coefficients (eq. TD-combi-tec), dyadic knot vectors (Sec. 3)
// with optional grading (Sec. 4.4), Gauss rules, 1D stiffness/mass matrices
// and their generalised eigen-decompositions (fast diagonalisation), the
// component grids, operator tiles, preconditioner blocks and the device
// workspace layout.  No GPU call is made here.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <array>
#include <functional>
#include <map>
#include <set>
#include <mutex>
#include <tuple>

#include "eigen.hpp"
#include "plan.hpp"

using namespace igasg;

namespace igasg {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
}

const char* last_error_str() { return g_err.c_str(); }

// de Boor's triangular scheme with left/right knot differences: row j of the
// table holds the degree-j functions; the strictly lower part keeps the knot
// differences needed for the derivative.
void basis_funs(int p, const double* U, int s, double x, double* N, double* dN) {
    double left[kMaxP + 2], right[kMaxP + 2];
    double t[kMaxP + 1][kMaxP + 1];
    t[0][0] = 1.0;
    for (int j = 1; j <= p; ++j) {
        left[j] = x - U[s + 1 - j];
        right[j] = U[s + j] - x;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            t[j][r] = right[r + 1] + left[j - r];
            double tmp = t[r][j - 1] / t[j][r];
            t[r][j] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        t[j][j] = saved;
    }
    for (int r = 0; r <= p; ++r) N[r] = t[r][p];
    if (!dN) return;
    for (int r = 0; r <= p; ++r) {
        double v = 0.0;
        if (r >= 1) v += t[r - 1][p - 1] / t[p][r - 1];
        if (r <= p - 1) v -= t[r][p - 1] / t[p][r];
        dN[r] = p * v;
    }
}

int find_interval(int p, int nk, const double* U, double x) {
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

double grade_map(int kind, double gamma, double t) {
    switch (kind) {
        case IGA_GRADE_RADICAL:
            return t <= 0.5 ? std::pow(2.0, gamma - 1.0) * std::pow(t, gamma)
                            : 1.0 - std::pow(2.0, gamma - 1.0) * std::pow(1.0 - t, gamma);
        case IGA_GRADE_TOWARD0:
            return std::pow(t, gamma);
        case IGA_GRADE_TOWARD1:
            return 1.0 - std::pow(1.0 - t, gamma);
        default:
            return t;
    }
}

// Gauss-Legendre nodes and weights by the Golub-Welsch method: the nodes are
// the eigenvalues of the Jacobi matrix of the Legendre recurrence, the
// weights 2 v_0^2 with v the normalised eigenvectors.
void gauss_rule(int n, double* x, double* w) {
    std::vector<double> J(static_cast<size_t>(n) * n, 0.0), I(static_cast<size_t>(n) * n, 0.0);
    for (int i = 0; i < n; ++i) I[static_cast<size_t>(i) * n + i] = 1.0;
    for (int k = 1; k < n; ++k) {
        double b = k / std::sqrt(4.0 * k * k - 1.0);
        J[static_cast<size_t>(k) * n + k - 1] = J[static_cast<size_t>(k - 1) * n + k] = b;
    }
    std::vector<double> V(static_cast<size_t>(n) * n);
    gen_eig_banded(n, 1, J.data(), I.data(), V.data(), x);
    for (int i = 0; i < n; ++i) w[i] = 2.0 * V[i] * V[i];
    if (n % 2 == 1) x[n / 2] = 0.0;
    for (int i = 0; i < n / 2; ++i) {  // exact symmetry
        double a = 0.5 * (x[n - 1 - i] - x[i]);
        x[i] = -a;
        x[n - 1 - i] = a;
        double ww = 0.5 * (w[i] + w[n - 1 - i]);
        w[i] = w[n - 1 - i] = ww;
    }
}

int tab_index(const iga_sg_plan_s* P, int patch, int dir, int lev) {
    return (patch * P->dim + dir) * (P->Lmax + 1) + lev;
}

}  // namespace igasg

namespace {

std::vector<double> make_knots(int p, int r, int lev, int gk, double gamma) {
    std::vector<double> U;
    int ne = 1 << lev;
    for (int i = 0; i <= p; ++i) U.push_back(0.0);
    for (int e = 1; e < ne; ++e) {
        double z = grade_map(gk, gamma, static_cast<double>(e) / ne);
        for (int m = 0; m < p - r; ++m) U.push_back(z);
    }
    for (int i = 0; i <= p; ++i) U.push_back(1.0);
    return U;
}

struct FDEntry {
    std::vector<double> K, M, U, lam;
    int n = 0;
    bool ok = false;  // the decomposition succeeded (or there is nothing to decompose)
};

std::mutex g_fd_mu;
std::map<std::tuple<int, int, int, int, double, int, int>, FDEntry> g_fd_cache;

// 1D stiffness/mass by Gauss quadrature on the unknowns of one direction
// (basis functions lo .. nb-1-hi: lo / hi = 1 drops the function of a
// Dirichlet end, 0 keeps the function of an interface end) and their
// eigen-pairs.
const FDEntry& fd_entry(int p, int r, int lev, int gk, double gamma, int nq, const double* gx,
                        const double* gw, int lo, int hi, bool* ok) {
    std::lock_guard<std::mutex> lk(g_fd_mu);
    auto key = std::make_tuple(p, r, lev, gk, gamma, nq, lo * 2 + hi);
    auto it = g_fd_cache.find(key);
    if (it != g_fd_cache.end()) {
        *ok = it->second.ok;
        return it->second;
    }
    FDEntry e;
    std::vector<double> U = make_knots(p, r, lev, gk, gamma);
    int nk = static_cast<int>(U.size());
    int nb = nk - p - 1, ni = nb - lo - hi;
    e.n = ni;
    e.K.assign(static_cast<size_t>(ni) * ni, 0.0);
    e.M.assign(static_cast<size_t>(ni) * ni, 0.0);
    double N[kMaxP + 1], dN[kMaxP + 1];
    for (int s = p; s < nb; ++s) {
        if (!(U[s] < U[s + 1])) continue;
        double h = U[s + 1] - U[s];
        for (int q = 0; q < nq; ++q) {
            double x = U[s] + 0.5 * h * (gx[q] + 1.0), w = 0.5 * h * gw[q];
            basis_funs(p, U.data(), s, x, N, dN);
            for (int a = 0; a <= p; ++a) {
                int ia = s - p + a - lo;
                if (ia < 0 || ia >= ni) continue;
                for (int b = 0; b <= p; ++b) {
                    int ib = s - p + b - lo;
                    if (ib < 0 || ib >= ni) continue;
                    e.K[static_cast<size_t>(ia) * ni + ib] += w * dN[a] * dN[b];
                    e.M[static_cast<size_t>(ia) * ni + ib] += w * N[a] * N[b];
                }
            }
        }
    }
    e.U.assign(static_cast<size_t>(ni) * ni, 0.0);
    e.lam.assign(ni, 0.0);
    // Graded knots make the pencil graded: its large entries sit at the fine
    // end.  The eigen-solver (Householder from the first row, QR steps chasing
    // downward) resolves the small eigenvalues of a matrix graded with its
    // large entries first (one-sided radical knots toward 1, level 10:
    // relative residual of the smallest pair 2.4 in the given order, 2e-4
    // reversed), so a pencil graded toward its last index is solved in
    // reversed order.
    const bool rev = ni > 1 && e.K[static_cast<size_t>(ni) * ni - 1] > e.K[0];
    if (rev) {
        std::vector<double> Kr(e.K.size()), Mr(e.M.size()), Ur(e.U.size());
        for (int i = 0; i < ni; ++i)
            for (int j = 0; j < ni; ++j) {
                Kr[static_cast<size_t>(ni - 1 - i) * ni + (ni - 1 - j)] = e.K[static_cast<size_t>(i) * ni + j];
                Mr[static_cast<size_t>(ni - 1 - i) * ni + (ni - 1 - j)] = e.M[static_cast<size_t>(i) * ni + j];
            }
        *ok = gen_eig_banded(ni, p, Kr.data(), Mr.data(), Ur.data(), e.lam.data());
        for (int i = 0; i < ni; ++i)
            std::memcpy(&e.U[static_cast<size_t>(i) * ni], &Ur[static_cast<size_t>(ni - 1 - i) * ni],
                        sizeof(double) * ni);
    } else {
        // no interior unknowns (degree 1 at level 0): an empty factor
        *ok = ni == 0 || gen_eig_banded(ni, p, e.K.data(), e.M.data(), e.U.data(), e.lam.data());
    }
    // failures are cached as failures, so a later plan reports them too
    e.ok = *ok;
    auto res = g_fd_cache.emplace(key, std::move(e));
    return res.first->second;
}

// Prolongation between nested spline spaces of degree p (coarse knots Uc,
// fine knots Uf, every coarse breakpoint a fine one with at least its
// multiplicity): coarse function j equals sum_i T[i][j] (fine function i).
// T is the L2 projection of the coarse basis onto the fine space, M_f T =
// M_fc, exact up to rounding because the coarse space lies in the fine one;
// both Gram matrices by nq-point Gauss rules on the fine elements (nq >= p+1
// integrates the products of degree 2p exactly), M_f by a banded Cholesky
// factorisation (half bandwidth p).  T is row-major [nb_f][nb_c].
bool prolongation_1d(int p, const std::vector<double>& Uc, const std::vector<double>& Uf, int nq, const double* gx,
                     const double* gw, std::vector<double>* Tout) {
    const int nkc = static_cast<int>(Uc.size()), nkf = static_cast<int>(Uf.size());
    const int nc = nkc - p - 1, nf = nkf - p - 1, bw = p;
    std::vector<double> Mf(static_cast<size_t>(nf) * (bw + 1), 0.0);  // Mf[i][i - j], j <= i
    std::vector<double>& T = *Tout;
    T.assign(static_cast<size_t>(nf) * nc, 0.0);
    double Nf[kMaxP + 1], Nc[kMaxP + 1];
    for (int e = p; e < nf; ++e) {
        const double a = Uf[e], b = Uf[e + 1];
        if (!(b > a)) continue;
        for (int q = 0; q < nq; ++q) {
            const double x = 0.5 * (a + b) + 0.5 * (b - a) * gx[q], wq = 0.5 * (b - a) * gw[q];
            const int sc = igasg::find_interval(p, nkc, Uc.data(), x);
            igasg::basis_funs(p, Uf.data(), e, x, Nf, nullptr);
            igasg::basis_funs(p, Uc.data(), sc, x, Nc, nullptr);
            for (int i = 0; i <= p; ++i) {
                const int fi = e - p + i;
                for (int j = 0; j <= i; ++j) Mf[static_cast<size_t>(fi) * (bw + 1) + (i - j)] += wq * Nf[i] * Nf[j];
                for (int j = 0; j <= p; ++j) T[static_cast<size_t>(fi) * nc + sc - p + j] += wq * Nf[i] * Nc[j];
            }
        }
    }
    auto m = [&](int i, int j) -> double& { return Mf[static_cast<size_t>(i) * (bw + 1) + (i - j)]; };
    for (int i = 0; i < nf; ++i) {  // M_f = L L^T, L in place of the lower band
        for (int j = std::max(0, i - bw); j <= i; ++j) {
            double v = m(i, j);
            for (int k = std::max(0, i - bw); k < j; ++k) v -= m(i, k) * m(j, k);
            if (i == j) {
                if (!(v > 0.0)) return false;
                m(i, i) = std::sqrt(v);
            } else {
                m(i, j) = v / m(j, j);
            }
        }
    }
    for (int c = 0; c < nc; ++c) {  // forward and back substitution per coarse function
        for (int i = 0; i < nf; ++i) {
            double v = T[static_cast<size_t>(i) * nc + c];
            for (int k = std::max(0, i - bw); k < i; ++k) v -= m(i, k) * T[static_cast<size_t>(k) * nc + c];
            T[static_cast<size_t>(i) * nc + c] = v / m(i, i);
        }
        for (int i = nf - 1; i >= 0; --i) {
            double v = T[static_cast<size_t>(i) * nc + c];
            for (int k = i + 1; k <= std::min(nf - 1, i + bw); ++k) v -= m(k, i) * T[static_cast<size_t>(k) * nc + c];
            T[static_cast<size_t>(i) * nc + c] = v / m(i, i);
        }
    }
    return true;
}

uint16_t to_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return static_cast<uint16_t>(u >> 16);  // inf/nan
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;  // round to nearest even
    return static_cast<uint16_t>(u >> 16);
}

double binom(int n, int k) {
    if (k < 0 || k > n) return 0.0;
    double v = 1.0;
    for (int i = 1; i <= k; ++i) v = v * (n - k + i) / i;
    return v;
}

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// Tuning knobs (tile sizes) read from the environment, with defaults.
int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    if (!v || !*v) return dflt;
    int x = std::atoi(v);
    return x > 0 ? x : dflt;
}

// Element index range touching unknowns [a, b) of one direction whose first
// unknown is basis function lo.
void elem_range(int a, int b, int p, int m, int E, int* elo, int* ehi, int lo = 1) {
    const int lo_basis = a + lo, hi_basis = b - 1 + lo;  // basis indices of the first/last owned unknown
    const int e0 = (lo_basis - p <= 0) ? 0 : (lo_basis - p + m - 1) / m;
    const int e1 = hi_basis / m;
    *elo = std::max(0, e0);
    *ehi = std::min(E - 1, e1);
}

}  // namespace

extern "C" {

const char* iga_sg_last_error(void) { return last_error_str(); }

const char* iga_sg_version(void) { return "iga-sg-mi355x 0.1 (gfx950)"; }

iga_status iga_sg_plan_create(const iga_geometry* geom, const iga_sg_disc* disc, iga_sg_plan* out) {
    if (!geom || !disc || !out) {
        set_error("null argument");
        return IGA_ERR_INVALID_ARG;
    }
    *out = nullptr;
    const int d = geom->dim;
    if (d != 2 && d != 3) {
        set_error("dim must be 2 or 3 (got %d)", d);
        return IGA_ERR_INVALID_ARG;
    }
    if (geom->npatch < 1 || geom->npatch > kMaxPatch || !geom->patches) {
        set_error("npatch must be in [1, %d]", kMaxPatch);
        return IGA_ERR_INVALID_ARG;
    }
    if (geom->npatch > 1 && d != 2) {
        set_error("several patches are supported in two dimensions");
        return IGA_ERR_INVALID_ARG;
    }
    if (geom->ninterface < 0 || (geom->ninterface > 0 && !geom->interfaces)) {
        set_error("bad interface list");
        return IGA_ERR_INVALID_ARG;
    }
    const int p = disc->p, r = disc->r;
    if (p < 1 || p > kMaxP || r < 0 || r >= p) {
        set_error("need 1 <= p <= %d and 0 <= r < p (got p=%d r=%d)", kMaxP, p, r);
        return IGA_ERR_INVALID_ARG;
    }
    if (disc->lmin < 0 || disc->w < d * disc->lmin || disc->w > 24) {
        set_error("need w >= dim*lmin, lmin >= 0, w <= 24 (got w=%d lmin=%d)", disc->w, disc->lmin);
        return IGA_ERR_INVALID_ARG;
    }
    const int nq = disc->nq > 0 ? disc->nq : p + 1;
    if (nq != p + 1) {
        set_error("the GPU path uses p+1 Gauss points per direction (got nq=%d)", nq);
        return IGA_ERR_INVALID_ARG;
    }
    auto P = new iga_sg_plan_s();
    P->dim = d;
    P->p = p;
    P->r = r;
    P->w = disc->w;
    P->lmin = disc->lmin;
    P->nq = nq;
    if (disc->nsamples < 0 || disc->nsamples > 65536) {
        set_error("nsamples must be in [0, 65536] (got %d)", disc->nsamples);
        delete P;
        return IGA_ERR_INVALID_ARG;
    }
    P->nsamples = disc->nsamples > 0 ? disc->nsamples : 1;
    P->gauss_x.resize(nq);
    P->gauss_w.resize(nq);
    gauss_rule(nq, P->gauss_x.data(), P->gauss_w.data());
    // ---- geometry ---------------------------------------------------------
    for (int pt = 0; pt < geom->npatch; ++pt) {
        const iga_patch& G = geom->patches[pt];
        PatchHost H;
        int ncp = 1;
        for (int k = 0; k < d; ++k) {
            int pg = G.degree[k], nk = G.nknots[k];
            if (pg < 1 || pg > kMaxPg || nk < 2 * (pg + 1) || !G.knots_host[k]) {
                set_error("patch %d direction %d: bad geometry degree/knots", pt, k);
                delete P;
                return IGA_ERR_GEOMETRY;
            }
            H.degree[k] = pg;
            H.knots[k].assign(G.knots_host[k], G.knots_host[k] + nk);
            for (int i = 1; i < nk; ++i)
                if (H.knots[k][i] < H.knots[k][i - 1]) {
                    set_error("patch %d direction %d: knots not non-decreasing", pt, k);
                    delete P;
                    return IGA_ERR_GEOMETRY;
                }
            for (int i = 0; i <= pg; ++i)
                if (H.knots[k][i] != 0.0 || H.knots[k][nk - 1 - i] != 1.0) {
                    set_error("patch %d direction %d: geometry knots must be open on [0,1]", pt, k);
                    delete P;
                    return IGA_ERR_GEOMETRY;
                }
            ncp *= nk - pg - 1;
            H.grading[k] = G.grading[k];
            H.gamma[k] = G.gamma[k] > 0 ? G.gamma[k] : 1.0;
            if (H.grading[k] < 0 || H.grading[k] > 3) {
                set_error("bad grading kind %d", H.grading[k]);
                delete P;
                return IGA_ERR_INVALID_ARG;
            }
        }
        if (!G.ctrl_host) {
            set_error("patch %d: missing control points", pt);
            delete P;
            return IGA_ERR_GEOMETRY;
        }
        H.ctrl.assign(G.ctrl_host, G.ctrl_host + static_cast<size_t>(ncp) * d);
        if (G.weights_host) {
            H.weights.assign(G.weights_host, G.weights_host + ncp);
            bool all_same = true;
            for (double v : H.weights) {
                if (!(v > 0)) {
                    set_error("patch %d: weights must be positive", pt);
                    delete P;
                    return IGA_ERR_GEOMETRY;
                }
                if (v != H.weights[0]) all_same = false;
            }
            if (!all_same) P->rational_any = 1;
        }
        P->patches.push_back(std::move(H));
    }
    // ---- conforming interfaces; every other side carries Dirichlet data -----
    // bc[pt][s] = 1: side s of patch pt is a Dirichlet side (its functions are
    // not unknowns), 0: an interface side (its functions are shared with the
    // neighbouring patch).  The same multi-index levels apply on every patch,
    // so the two sides of an interface run along the same direction, whose
    // knots (grading) must agree.
    for (int pt = 0; pt < kMaxPatch; ++pt)
        for (int sd = 0; sd < 6; ++sd) P->bc[pt][sd] = 1;
    for (int f = 0; f < geom->ninterface; ++f) {
        const iga_interface& I = geom->interfaces[f];
        auto fail = [&](const char* what) {
            set_error("interface %d: %s", f, what);
            delete P;
            return IGA_ERR_GEOMETRY;
        };
        if (I.patch_a < 0 || I.patch_a >= geom->npatch || I.patch_b < 0 || I.patch_b >= geom->npatch ||
            I.patch_a == I.patch_b)
            return fail("bad patch index");
        if (I.side_a < 0 || I.side_a >= 2 * d || I.side_b < 0 || I.side_b >= 2 * d) return fail("bad side");
        if (!P->bc[I.patch_a][I.side_a] || !P->bc[I.patch_b][I.side_b]) return fail("side glued twice");
        const int ta = 1 - I.side_a / 2, tb = 1 - I.side_b / 2;
        if (ta != tb) return fail("the two sides run along different parametric directions");
        const PatchHost &A = P->patches[I.patch_a], &B = P->patches[I.patch_b];
        if (A.grading[ta] != B.grading[ta] || A.gamma[ta] != B.gamma[ta])
            return fail("non-conforming: the knots along the interface differ");
        P->bc[I.patch_a][I.side_a] = 0;
        P->bc[I.patch_b][I.side_b] = 0;
        P->ifaces.push_back(I);
    }
    for (int pt = 0; pt < geom->npatch; ++pt) {
        bool dir = false;
        for (int sd = 0; sd < 2 * d; ++sd) dir = dir || P->bc[pt][sd] != 0;
        if (!dir) {
            set_error("patch %d has no Dirichlet side", pt);
            delete P;
            return IGA_ERR_GEOMETRY;
        }
    }
    // vertices between two interface sides of a patch are unknowns of its
    // tensor set; they must carry Dirichlet data (a vertex glued to a
    // Dirichlet side of some patch), their value is then fixed
    if (geom->npatch > 1) {
        const int nn = geom->npatch * 4;  // (patch, corner e0 + 2 e1)
        std::vector<int> par(nn);
        for (int i = 0; i < nn; ++i) par[i] = i;
        std::function<int(int)> find = [&](int i) { return par[i] == i ? i : (par[i] = find(par[i])); };
        for (const iga_interface& I : P->ifaces) {
            const int ka = I.side_a / 2, kb = I.side_b / 2;
            for (int et = 0; et < 2; ++et) {
                int ea[2], eb[2];
                ea[ka] = I.side_a % 2;
                ea[1 - ka] = et;
                eb[kb] = I.side_b % 2;
                eb[1 - kb] = et;
                const int u = find(I.patch_a * 4 + ea[0] + 2 * ea[1]), v = find(I.patch_b * 4 + eb[0] + 2 * eb[1]);
                if (u != v) par[std::max(u, v)] = std::min(u, v);
            }
        }
        std::vector<char> cls_dir(nn, 0);
        for (int i = 0; i < nn; ++i) {
            const int pt = i / 4, e0 = i % 2, e1 = (i / 2) % 2;
            if (P->bc[pt][e0] || P->bc[pt][2 + e1]) cls_dir[find(i)] = 1;
        }
        for (int i = 0; i < nn; ++i) {
            const int pt = i / 4, e0 = i % 2, e1 = (i / 2) % 2;
            P->pin_corner[pt][i % 4] = 0;
            if (P->bc[pt][e0] || P->bc[pt][2 + e1]) continue;
            if (!cls_dir[find(i)]) {
                set_error("patch %d: a vertex shared by several patches inside the domain is not supported", pt);
                delete P;
                return IGA_ERR_GEOMETRY;
            }
            P->pin_corner[pt][i % 4] = 1;
        }
    }
    // ---- components (eq. TD-combi-tec), lexicographic, level 1 slowest ----
    const int J = P->w - d * P->lmin;
    int lmax_set = 0;
    if (disc->nindex > 0) {
        // a caller's downward-closed index set I (absolute levels): the
        // combination of eq. (TD-combi-tec) with its outer sum over the set,
        // c_b = sum over z in {0,1}^d with b + z in I of (-1)^|z|; grids with
        // c_b = 0 are not planned
        auto fail = [&](const char* what) {
            set_error("index set: %s", what);
            delete P;
            return IGA_ERR_INVALID_ARG;
        };
        if (!disc->index_host || disc->full) return fail("null levels, or combined with full");
        std::set<std::array<int, 3>> I;
        for (int i = 0; i < disc->nindex; ++i) {
            std::array<int, 3> b{0, 0, 0};
            for (int k = 0; k < d; ++k) {
                b[k] = disc->index_host[static_cast<size_t>(i) * d + k];
                if (b[k] < 0 || b[k] > 24) return fail("levels must lie in 0..24");
                lmax_set = std::max(lmax_set, b[k]);
            }
            I.insert(b);
        }
        for (const auto& b : I)
            for (int k = 0; k < d; ++k)
                if (b[k] > 0) {
                    std::array<int, 3> c = b;
                    --c[k];
                    if (!I.count(c)) return fail("not downward closed");
                }
        for (const auto& b : I) {  // lexicographic, direction 1 slowest
            int c = 0;
            for (int z = 0; z < (1 << d); ++z) {
                std::array<int, 3> bz = b;
                int nz = 0;
                for (int k = 0; k < d; ++k)
                    if ((z >> k) & 1) {
                        ++bz[k];
                        ++nz;
                    }
                if (I.count(bz)) c += (nz & 1) ? -1 : 1;
            }
            if (c == 0 && !disc->keep_all) continue;
            for (int k = 0; k < d; ++k) P->comp_levels.push_back(b[k]);
            P->comp_coef.push_back(static_cast<double>(c));
        }
    } else if (disc->full) {
        // the full tensor-product space at level w in every direction
        // (standard IGA, the comparison of Sec. 4): one grid, coefficient 1
        for (int k = 0; k < d; ++k) P->comp_levels.push_back(P->w);
        P->comp_coef.push_back(1.0);
    } else {
        int b[3] = {0, 0, 0};
        int lim1 = d > 1 ? J : 0, lim2 = d > 2 ? J : 0;
        for (b[0] = 0; b[0] <= J; ++b[0])
            for (b[1] = 0; b[1] <= lim1; ++b[1])
                for (b[2] = 0; b[2] <= lim2; ++b[2]) {
                    int s = b[0] + b[1] + b[2];
                    if (s > J || s < J - d + 1) continue;
                    for (int k = 0; k < d; ++k) P->comp_levels.push_back(b[k] + P->lmin);
                    int j = J - s;
                    P->comp_coef.push_back(((j & 1) ? -1.0 : 1.0) * binom(d - 1, j));
                }
    }
    P->ncomp = static_cast<int>(P->comp_coef.size());
    if (disc->keep_all && disc->nindex > 0) {
        // the details' table: component of levels b - z for z in {0,1}^d
        std::map<std::array<int, 3>, int> at;
        for (int c = 0; c < P->ncomp; ++c) {
            std::array<int, 3> b{0, 0, 0};
            for (int k = 0; k < d; ++k) b[k] = P->comp_levels[c * d + k];
            at[b] = c;
        }
        P->detail_off = static_cast<int64_t>(P->ipool.size());
        for (int c = 0; c < P->ncomp; ++c)
            for (int z = 0; z < 8; ++z) {
                int idx = -1;
                if (z < (1 << d)) {
                    std::array<int, 3> b{0, 0, 0};
                    bool neg = false;
                    for (int k = 0; k < d; ++k) {
                        b[k] = P->comp_levels[c * d + k] - ((z >> k) & 1);
                        neg = neg || b[k] < 0;
                    }
                    if (!neg) idx = at.at(b);  // the set is downward closed
                }
                P->ipool.push_back(idx);
            }
    }
    P->Lmax = disc->nindex > 0 ? lmax_set : disc->full ? P->w : P->lmin + J;
    // ---- 1D tables per (patch, dir, level) ---------------------------------
    const int ntab = geom->npatch * d * (P->Lmax + 1);
    P->tabs.resize(ntab);
    P->K1d.resize(ntab);
    P->M1d.resize(ntab);
    std::map<std::tuple<int, double, int, int>, std::array<int64_t, 9>> fd_off;
    for (int pt = 0; pt < geom->npatch; ++pt)
        for (int k = 0; k < d; ++k)
            for (int lev = 0; lev <= P->Lmax; ++lev) {
                Tab1D& T = P->tabs[tab_index(P, pt, k, lev)];
                std::memset(&T, 0, sizeof(T));
                const PatchHost& H = P->patches[pt];
                std::vector<double> U = make_knots(p, r, lev, H.grading[k], H.gamma[k]);
                T.nk = static_cast<int>(U.size());
                T.nb = T.nk - p - 1;
                T.lo = P->bc[pt][2 * k];
                const int thi = P->bc[pt][2 * k + 1];
                T.ni = T.nb - T.lo - thi;
                T.E = 1 << lev;
                T.Q = T.E * nq;
                T.m = p - r;
                T.pg = H.degree[k];
                T.ngk = static_cast<int>(H.knots[k].size());
                T.ngb = T.ngk - T.pg - 1;
                T.uniform = H.grading[k] == IGA_GRADE_UNIFORM || H.gamma[k] == 1.0;
                auto& dp = P->dpool;
                T.oKn = static_cast<int64_t>(dp.size());
                dp.insert(dp.end(), U.begin(), U.end());
                T.oBrk = static_cast<int64_t>(dp.size());
                for (int e = 0; e <= T.E; ++e) dp.push_back(U[p + e * T.m]);
                T.oGkn = static_cast<int64_t>(dp.size());
                dp.insert(dp.end(), H.knots[k].begin(), H.knots[k].end());
                // Gauss tables are computed on the device at bind time
                T.oB = static_cast<int64_t>(dp.size());
                dp.resize(dp.size() + static_cast<size_t>(T.Q) * (p + 1));
                T.oD = static_cast<int64_t>(dp.size());
                dp.resize(dp.size() + static_cast<size_t>(T.Q) * (p + 1));
                T.oBg = static_cast<int64_t>(dp.size());
                dp.resize(dp.size() + static_cast<size_t>(T.Q) * (T.pg + 1));
                T.oDg = static_cast<int64_t>(dp.size());
                dp.resize(dp.size() + static_cast<size_t>(T.Q) * (T.pg + 1));
                T.oXq = static_cast<int64_t>(dp.size());
                dp.resize(dp.size() + T.Q);
                T.oWq = static_cast<int64_t>(dp.size());
                dp.resize(dp.size() + T.Q);
                T.oGs = static_cast<int64_t>(P->ipool.size());
                P->ipool.resize(P->ipool.size() + T.Q);
                // fast-diagonalisation factors (shared by equal knot families)
                bool ok = true;
                const FDEntry& F = fd_entry(p, r, lev, H.grading[k], H.gamma[k], nq, P->gauss_x.data(),
                                            P->gauss_w.data(), T.lo, thi, &ok);
                if (!ok) {
                    set_error("eigen-decomposition failed (level %d)", lev);
                    delete P;
                    return IGA_ERR_GEOMETRY;
                }
                P->K1d[tab_index(P, pt, k, lev)] = F.K;
                P->M1d[tab_index(P, pt, k, lev)] = F.M;
                auto fkey = std::make_tuple(H.grading[k], H.gamma[k], lev, T.lo * 2 + thi);
                auto fit = fd_off.find(fkey);
                if (fit == fd_off.end()) {
                    // U and U^T stored row-major with a padded row stride (a multiple of 8
                    // elements, zero-filled) so that rows start 16-byte aligned in every
                    // precision; the pools are padded to 8 elements before each table
                    std::array<int64_t, 9> o;
                    const int n = F.n, ld = (n + 7) & ~7;
                    auto Uat = [&](int i, int j, bool tr) {
                        return tr ? F.U[static_cast<size_t>(j) * n + i] : F.U[static_cast<size_t>(i) * n + j];
                    };
                    for (int t = 0; t < 2; ++t) {
                        dp.resize((dp.size() + 7) & ~static_cast<size_t>(7), 0.0);
                        o[t] = static_cast<int64_t>(dp.size());
                        for (int i = 0; i < n; ++i)
                            for (int j = 0; j < ld; ++j) dp.push_back(j < n ? Uat(i, j, t == 1) : 0.0);
                    }
                    o[2] = static_cast<int64_t>(dp.size());
                    dp.insert(dp.end(), F.lam.begin(), F.lam.end());
                    o[7] = static_cast<int64_t>(dp.size());
                    for (int i = 0; i < n; ++i) dp.push_back(F.K[static_cast<size_t>(i) * n + i]);
                    o[8] = static_cast<int64_t>(dp.size());
                    for (int i = 0; i < n; ++i) dp.push_back(F.M[static_cast<size_t>(i) * n + i]);
                    for (int t = 0; t < 2; ++t) {
                        P->fpool.resize((P->fpool.size() + 7) & ~static_cast<size_t>(7), 0.0f);
                        o[3 + t] = static_cast<int64_t>(P->fpool.size());
                        for (int i = 0; i < n; ++i)
                            for (int j = 0; j < ld; ++j)
                                P->fpool.push_back(j < n ? static_cast<float>(Uat(i, j, t == 1)) : 0.0f);
                    }
                    for (int t = 0; t < 2; ++t) {
                        P->hpool.resize((P->hpool.size() + 7) & ~static_cast<size_t>(7), 0);
                        o[5 + t] = static_cast<int64_t>(P->hpool.size());
                        for (int i = 0; i < n; ++i)
                            for (int j = 0; j < ld; ++j)
                                P->hpool.push_back(j < n ? to_bf16(static_cast<float>(Uat(i, j, t == 1))) : 0);
                    }
                    fit = fd_off.emplace(fkey, o).first;
                }
                T.ldu = (F.n + 7) & ~7;
                T.oU = fit->second[0];
                T.oUT = fit->second[1];
                T.oLam = fit->second[2];
                T.oU32 = fit->second[3];
                T.oUT32 = fit->second[4];
                T.oU16 = fit->second[5];
                T.oUT16 = fit->second[6];
                T.oKd = fit->second[7];
                T.oMd = fit->second[8];
            }
    // prolongations of a full tensor plan: level l -> level w per direction
    if (disc->full && geom->npatch == 1) {
        P->xfer_off.assign(static_cast<size_t>(d) * (P->w + 1), -1);
        for (int k = 0; k < d; ++k) {
            const PatchHost& H = P->patches[0];
            const Tab1D& Tf = P->tabs[tab_index(P, 0, k, P->w)];
            const std::vector<double> Uf = make_knots(p, r, P->w, H.grading[k], H.gamma[k]);
            for (int lev = 0; lev < P->w; ++lev) {
                const Tab1D& Tc = P->tabs[tab_index(P, 0, k, lev)];
                const std::vector<double> Uc = make_knots(p, r, lev, H.grading[k], H.gamma[k]);
                std::vector<double> T;
                if (!prolongation_1d(p, Uc, Uf, nq, P->gauss_x.data(), P->gauss_w.data(), &T)) {
                    set_error("prolongation from level %d failed", lev);
                    delete P;
                    return IGA_ERR_GEOMETRY;
                }
                const int nbc = Tc.nb;
                auto& dp = P->dpool;
                P->xfer_off[static_cast<size_t>(k) * (P->w + 1) + lev] = static_cast<int64_t>(dp.size());
                for (int i = 0; i < Tf.ni; ++i)
                    for (int j = 0; j < Tc.ni; ++j)
                        dp.push_back(T[static_cast<size_t>(Tf.lo + i) * nbc + Tc.lo + j]);
            }
        }
    }
    // homogeneous control points (w P, w) per patch
    for (int pt = 0; pt < geom->npatch; ++pt) {
        const PatchHost& H = P->patches[pt];
        P->ctrl_off[pt] = static_cast<int64_t>(P->ctrl.size());
        size_t ncp = H.ctrl.size() / d;
        for (size_t i = 0; i < ncp; ++i) {
            double wt = H.weights.empty() ? 1.0 : H.weights[i];
            for (int c = 0; c < 3; ++c) P->ctrl.push_back(c < d ? wt * H.ctrl[i * d + c] : 0.0);
            P->ctrl.push_back(wt);
        }
    }
    P->ncompG = P->rational_any ? (d == 2 ? 6 : 10) : (d == 2 ? 3 : 6);
    // ---- 2D fast-diagonalisation blocking per precision class ---------------
    // A long direction of at least wide_min unknowns is cut into blocks of 8, 16
    // or 32 columns whose factor slab (about 64 KiB) is staged in LDS.  Each
    // block is one task of the persistent solve, and a phase ends with its
    // slowest workgroup, so wide_min is raised grid length by grid length while
    // the FD tasks of a solve outnumber the workgroups of one wave and the
    // grids it makes single-block fit in LDS with both factors staged.
    int wide_min_cls[2] = {env_int("IGA_FD_WIDE", 100), env_int("IGA_FD_WIDE", 100)};
    if (d == 2 && !std::getenv("IGA_FD_WIDE")) {
        const int target = disc->fd_tasks > 0 ? disc->fd_tasks : env_int("IGA_FD_TASKS", 256);
        struct Shape { int ni0, ni1, ld0, ld1; };
        std::vector<Shape> shapes;
        for (int c = 0; c < P->ncomp; ++c)
            for (int pt = 0; pt < geom->npatch; ++pt) {
                const Tab1D& T0 = P->tabs[tab_index(P, pt, 0, P->comp_levels[c * d])];
                const Tab1D& T1 = P->tabs[tab_index(P, pt, 1, P->comp_levels[c * d + 1])];
                shapes.push_back({T0.ni, T1.ni, T0.ldu, T1.ldu});
            }
        for (int cls = 0; cls < 2; ++cls) {
            const int usize = cls == 0 ? 8 : 4;
            auto nblocks = [&](const Shape& sh, int wm) {
                const int nbig = std::max(sh.ni0, sh.ni1);
                if (nbig < wm) return 1;
                int b = 8;
                while (b < 32 && static_cast<size_t>(2 * b) * nbig * usize <= 66000) b *= 2;
                return b < nbig ? (nbig + b - 1) / b : 1;
            };
            auto fits_single = [&](const Shape& sh) {
                Grid t;
                std::memset(&t, 0, sizeof(t));
                t.ni[0] = sh.ni0;
                t.ni[1] = sh.ni1;
                t.ni[2] = 1;
                t.big = sh.ni1 > sh.ni0 ? 1 : 0;
                t.blk = t.ni[t.big];
                t.nblk = 1;
                t.fdstage = 1;
                const int ls = t.big ? sh.ld0 : sh.ld1, lb = t.big ? sh.ld1 : sh.ld0;
                return fd_layout(t, ls, lb, usize).total + kSolveLdsHead <= static_cast<size_t>(kLdsLimit);
            };
            int wm = wide_min_cls[cls];
            for (;;) {
                long ntask = 0;
                int next = 0;  // shortest long direction still cut into blocks
                for (const Shape& sh : shapes) {
                    const int nb = nblocks(sh, wm);
                    ntask += nb;
                    if (nb > 1) {
                        const int nbig = std::max(sh.ni0, sh.ni1);
                        next = next == 0 ? nbig : std::min(next, nbig);
                    }
                }
                if (ntask * P->nsamples <= target || next == 0) break;
                bool ok = true;
                for (const Shape& sh : shapes)
                    if (std::max(sh.ni0, sh.ni1) == next && !fits_single(sh)) ok = false;
                if (!ok) break;
                wm = next + 1;
            }
            wide_min_cls[cls] = wm;
        }
    }
    // ---- grids, tiles, preconditioner blocks --------------------------------
    size_t lds_max = 0, lds_op = 0, lds_fd_plain = 0;
    // the full tensor grid of one patch and one sample may exceed the LDS of a
    // workgroup: it is then solved by whole-device kernels
    const bool stream_ok = disc->full && geom->npatch == 1 && P->nsamples == 1;
    for (int c = 0; c < P->ncomp; ++c)
        for (int pt = 0; pt < geom->npatch; ++pt) {
            Grid g;
            std::memset(&g, 0, sizeof(g));
            g.comp = c;
            g.patch = pt;
            g.ccoef = P->comp_coef[c];
            g.ndof = 1;
            g.nqp = 1;
            for (int k = 0; k < 3; ++k) {
                if (k < d) {
                    int lev = P->comp_levels[c * d + k];
                    const Tab1D& T = P->tabs[tab_index(P, pt, k, lev)];
                    g.lev[k] = lev;
                    g.ni[k] = T.ni;
                    g.nb[k] = T.nb;
                    g.E[k] = T.E;
                    g.Q[k] = T.Q;
                    g.tab[k] = tab_index(P, pt, k, lev);
                } else {
                    g.ni[k] = g.nb[k] = g.E[k] = g.Q[k] = 1;
                    g.tab[k] = -1;
                }
                g.ndof *= g.ni[k];
                g.nqp *= g.Q[k];
                g.fdc[k] = 1.0;
            }
            if (g.ndof <= 0) {
                // degree 1 at level 0 with Dirichlet ends: only boundary functions
                set_error("component grid %d has no interior unknowns (degree %d at level 0): raise lmin", c, p);
                delete P;
                return IGA_ERR_INVALID_ARG;
            }
            g.dof_off = P->ndof_total;
            P->ndof_total += g.ndof;
            // inverse eigenvalue sums of the fast-diagonalisation pencil, direction 1 fastest
            {
                auto& dp = P->dpool;
                g.oDinv = static_cast<int64_t>(dp.size());
                const double* lam[3] = {nullptr, nullptr, nullptr};
                for (int k = 0; k < d; ++k) lam[k] = &dp[P->tabs[g.tab[k]].oLam];
                std::vector<double> dv(static_cast<size_t>(g.ndof));
                for (int64_t i = 0; i < g.ndof; ++i) {
                    int64_t rem = i;
                    double s = 0.0;
                    for (int k = 0; k < d; ++k) {
                        s += g.fdc[k] * lam[k][rem % g.ni[k]];
                        rem /= g.ni[k];
                    }
                    dv[static_cast<size_t>(i)] = 1.0 / s;
                }
                dp.insert(dp.end(), dv.begin(), dv.end());
            }
            g.qp_off = P->nqp_total;
            P->nqp_total += g.nqp;
            // operator tiles: minimise the elements processed (halo recompute)
            const int m = p - r;
            if (d == 2) {
                const int TT = disc->op_tile > 0 ? disc->op_tile : env_int("IGA_OP_TILE", 128);
                long best = -1;
                for (int t2 = 1; t2 <= std::min(g.ni[1], TT); ++t2) {
                    int t1 = std::min(g.ni[0], std::max(1, TT / t2));
                    int n1 = (g.ni[0] + t1 - 1) / t1, n2 = (g.ni[1] + t2 - 1) / t2;
                    int lo, hi, e1, e2;
                    elem_range(0, t1, p, m, g.E[0], &lo, &hi, P->tabs[g.tab[0]].lo);
                    e1 = hi - lo + 1 + (t1 < g.ni[0] ? 1 : 0);
                    elem_range(0, t2, p, m, g.E[1], &lo, &hi, P->tabs[g.tab[1]].lo);
                    e2 = hi - lo + 1 + (t2 < g.ni[1] ? 1 : 0);
                    long work = static_cast<long>(n1) * n2 * e1 * e2 + 64L * n1 * n2;
                    if (best < 0 || work < best) {
                        best = work;
                        g.tile[0] = t1;
                        g.tile[1] = t2;
                    }
                }
                g.tile[2] = 1;
            } else {
                // 3D: tiles of about TT unknowns whose halo and element outputs fit in LDS
                const int TT = disc->op_tile3 > 0 ? disc->op_tile3 : env_int("IGA_OP_TILE3", 256);
                const size_t pl = static_cast<size_t>(p + 1) * (p + 1) * (p + 1);
                double best = -1.0;
                g.tile[0] = g.ni[0];
                g.tile[1] = g.ni[1];
                g.tile[2] = g.ni[2];
                // the largest element range of a tile of t unknowns along direction k
                std::vector<int> maxel(3 * 65, -1);
                auto max_elems = [&](int k, int t) {
                    int& v = maxel[k * 65 + std::min(t, 64)];
                    if (t > 64 || v < 0) {
                        int lo, hi, best_k = 0;
                        for (int a = 0; a < g.ni[k]; a += t) {
                            elem_range(a, std::min(g.ni[k], a + t), p, m, g.E[k], &lo, &hi, P->tabs[g.tab[k]].lo);
                            best_k = std::max(best_k, hi - lo + 1);
                        }
                        if (t > 64) return best_k;
                        v = best_k;
                    }
                    return v;
                };
                // tiles of about TT unknowns first; where none fits (a full grid long in
                // every direction), any smaller tile
                for (int pass = 0; pass < 2 && best < 0; ++pass)
                for (int t3 = 1; t3 <= std::min(g.ni[2], 64); ++t3)
                    for (int t2 = 1; t2 <= std::min(g.ni[1], 64); ++t2)
                    for (int t1s = 1; t1s <= (pass == 0 ? 1 : std::min(g.ni[0], 64)); ++t1s) {
                        const int t1 = pass == 0 ? std::min(g.ni[0], std::max(1, TT / (t2 * t3))) : t1s;
                        const int t[3] = {t1, t2, t3};
                        // work estimate from the first tile (pass 0) or the largest one;
                        // the fit test always with the largest element range over the tiles
                        size_t nel = 1, halo = 1, ntl = 1, nelx = 1, halox = 1;
                        for (int k = 0; k < 3; ++k) {
                            int lo, hi;
                            const int nex = max_elems(k, t[k]);
                            int ne = nex;
                            if (pass == 0) {
                                elem_range(0, t[k], p, m, g.E[k], &lo, &hi, P->tabs[g.tab[k]].lo);
                                ne = hi - lo + 1 + (t[k] < g.ni[k] ? 1 : 0);
                            }
                            nel *= ne;
                            halo *= static_cast<size_t>(ne - 1) * m + p + 1;
                            nelx *= nex;
                            halox *= static_cast<size_t>(nex - 1) * m + p + 1;
                            ntl *= (g.ni[k] + t[k] - 1) / t[k];
                        }
                        // + the FP32 copy of the halo block
                        const size_t lds =
                            (std::max(halo, halox) + std::max(nel, nelx) * pl + kWaves) * sizeof(double) +
                            std::max(halo, halox) * sizeof(float);
                        if (lds + kSolveLdsHead > kLdsLimit) continue;
                        const double work = static_cast<double>(ntl) * (nel + 64.0);
                        if (best < 0 || work < best) {
                            best = work;
                            g.tile[0] = t1;
                            g.tile[1] = t2;
                            g.tile[2] = t3;
                        }
                    }
            }
            g.ntile = 1;
            for (int k = 0; k < 3; ++k) {
                g.ntd[k] = (g.ni[k] + g.tile[k] - 1) / g.tile[k];
                g.ntile *= g.ntd[k];
            }
            // LDS of one operator tile: halo unknowns (FP64 and an FP32 copy) +
            // element outputs
            if (d == 3) {
                size_t halo = 1, nel = 1;
                for (int k = 0; k < 3; ++k) {
                    int lo, hi, bestk = 0;
                    for (int t = 0; t < g.ntd[k]; ++t) {
                        int a = t * g.tile[k], b = std::min(g.ni[k], a + g.tile[k]);
                        elem_range(a, b, p, m, g.E[k], &lo, &hi, P->tabs[g.tab[k]].lo);
                        bestk = std::max(bestk, hi - lo + 1);
                    }
                    nel *= bestk;
                    halo *= static_cast<size_t>(bestk - 1) * m + p + 1;
                }
                const size_t pl = static_cast<size_t>(p + 1) * (p + 1) * (p + 1);
                lds_max = std::max(lds_max, (halo + nel * pl + kWaves) * sizeof(double) + halo * sizeof(float));
                lds_op = std::max(lds_op, (halo + nel * pl + kWaves) * sizeof(double) + halo * sizeof(float));
            }
            if (d == 2) {
                size_t halo = 1, nel = 1;
                for (int k = 0; k < d; ++k) {
                    int lo, hi, best = 0;
                    for (int t = 0; t < g.ntd[k]; ++t) {
                        int a = t * g.tile[k], b = std::min(g.ni[k], a + g.tile[k]);
                        elem_range(a, b, p, m, g.E[k], &lo, &hi, P->tabs[g.tab[k]].lo);
                        best = std::max(best, hi - lo + 1);
                    }
                    nel *= best;
                    halo *= static_cast<size_t>(best) * m + p + 1;
                }
                size_t pl = 1;
                for (int k = 0; k < d; ++k) pl *= (p + 1);
                size_t lds = (halo + nel * pl + kBlock) * sizeof(double);
                lds_max = std::max(lds_max, lds);
            }
            // fast-diagonalisation blocks (2D: split the longest direction, see the
            // blocking above); FP32/BF16 factors allow wider blocks, so each
            // precision class has its own blocking.
            Grid glp = g;
            if (d == 2) {
                for (int cls = 0; cls < 2; ++cls) {
                    Grid& gc = cls == 0 ? g : glp;
                    const int usize = cls == 0 ? 8 : 4;
                    gc.big = gc.ni[1] > gc.ni[0] ? 1 : 0;
                    const int nbig = gc.ni[gc.big];
                    int bs = nbig;
                    if (nbig >= wide_min_cls[cls]) {
                        int b = 8;
                        while (b < 32 && static_cast<size_t>(2 * b) * nbig * usize <= 66000) b *= 2;
                        if (b < nbig) bs = b;
                    }
                    gc.blk = bs;
                    gc.nblk = (nbig + bs - 1) / bs;
                    const bool wide = gc.nblk > 1;
                    const int ls = P->tabs[gc.tab[1 - gc.big]].ldu, lb = P->tabs[gc.tab[gc.big]].ldu;
                    // single-block grids stage the long factor as well when it fits
                    gc.fdstage = wide ? 0 : 1;
                    if (!wide && fd_layout(gc, ls, lb, usize).total + kSolveLdsHead > kLdsLimit) gc.fdstage = 0;
                    // long grids: the block's slab of the long factor is read from
                    // memory when it does not fit beside the grid vectors
                    if (wide && fd_layout(gc, ls, lb, usize).total + kSolveLdsHead > kLdsLimit) gc.fdstage = -1;
                    // a full tensor grid whose vectors do not fit: whole-device kernels
                    if (stream_ok && (fd_layout(gc, ls, lb, usize).total + kSolveLdsHead > kLdsLimit ||
                                      (cls == 1 && g.fdstage == kFdStream))) {
                        gc.fdstage = kFdStream;
                        P->streamed = true;
                        continue;
                    }
                    lds_max = std::max(lds_max, static_cast<size_t>(fd_layout(gc, ls, lb, usize).total));
                }
            } else {
                // 3D: one task per grid with the three factors staged in LDS
                g.big = 0;
                g.blk = g.ni[0];
                g.nblk = 1;
                const int ld[3] = {P->tabs[g.tab[0]].ldu, P->tabs[g.tab[1]].ldu, P->tabs[g.tab[2]].ldu};
                // stage the factors in LDS, smallest first, while they fit (FP64 sizes)
                int ord3[3] = {0, 1, 2};
                std::sort(ord3, ord3 + 3, [&](int a, int b) { return g.ni[a] < g.ni[b]; });
                g.fdstage = 0;
                const size_t nn_bytes = static_cast<size_t>(kNnLdsBytesPerDof) * g.ndof;
                for (int k : ord3) {
                    g.fdstage |= 1 << k;
                    if (fd_layout_3d(g, ld, 8).total + nn_bytes + kSolveLdsHead > kLdsLimit) g.fdstage &= ~(1 << k);
                }
                if (stream_ok && fd_layout_3d(g, ld, 8).total + kSolveLdsHead > kLdsLimit) {
                    g.fdstage = kFdStream;  // a full tensor grid whose vectors do not fit
                    P->streamed = true;
                }
                glp = g;
                // + the activations of the learned preconditioner
                if (g.fdstage != kFdStream) {
                    lds_max = std::max(lds_max, static_cast<size_t>(fd_layout_3d(g, ld, 8).total) +
                                                    static_cast<size_t>(kNnLdsBytesPerDof) * g.ndof);
                    lds_fd_plain = std::max(lds_fd_plain, static_cast<size_t>(fd_layout_3d(g, ld, 8).total));
                }
            }
            P->grids_lp.push_back(glp);
            P->grids.push_back(g);
        }
    // interfaces, fixed vertices, solver-state groups and the lift arrays of
    // the grids of one sample (grid c * npatch + pt is patch pt of component c)
    const int npat = geom->npatch;
    int64_t nlift = 0;
    for (size_t gi = 0; gi < P->grids.size(); ++gi) {
        Grid& g = P->grids[gi];
        const int c = g.comp, pt = g.patch;
        g.state = c * npat;
        g.nbr_on = 0;
        for (int sd = 0; sd < 4; ++sd) {
            g.nbr_base[sd] = 0;
            g.nbr_stride[sd] = 0;
            g.pin[sd] = -1;
        }
        if (d == 2) {
            g.lift_off = nlift;
            nlift += static_cast<int64_t>(g.nb[0]) * g.nb[1];
            for (int e = 0; e < 4; ++e)
                if (P->pin_corner[pt][e]) {
                    const int i0 = (e & 1) ? g.ni[0] - 1 : 0, i1 = (e & 2) ? g.ni[1] - 1 : 0;
                    g.pin[e] = i0 + g.ni[0] * i1;
                }
            for (const iga_interface& I : P->ifaces)
                for (int side = 0; side < 2; ++side) {
                    const int sa = side ? I.side_b : I.side_a, pa = side ? I.patch_b : I.patch_a;
                    const int sb = side ? I.side_a : I.side_b, pb = side ? I.patch_a : I.patch_b;
                    if (pa != pt) continue;
                    const Grid& h = P->grids[static_cast<size_t>(c) * npat + pb];
                    const int t = 1 - sa / 2, kb = sb / 2;
                    const int fixb = (sb % 2) ? h.ni[kb] - 1 : 0;
                    const int shift = P->tabs[g.tab[t]].lo - P->tabs[h.tab[t]].lo;
                    const int64_t rel = h.dof_off - g.dof_off;
                    g.nbr_on |= 1 << sa;
                    g.nbr_base[sa] = static_cast<int>(rel + (kb == 0 ? fixb + h.ni[0] * shift : h.ni[0] * fixb + shift));
                    g.nbr_stride[sa] = kb == 0 ? h.ni[0] : 1;
                    // every unknown of the side that is not fixed has its partner
                    const int fix_a = (sa % 2) ? g.ni[sa / 2] - 1 : 0;
                    for (int it = 0; it < g.ni[t]; ++it) {
                        int ia[2];
                        ia[sa / 2] = fix_a;
                        ia[t] = it;
                        const int lin = ia[0] + g.ni[0] * ia[1];
                        bool fixed = false;
                        for (int e = 0; e < 4; ++e) fixed = fixed || g.pin[e] == lin;
                        if (fixed) continue;
                        if (it + shift < 0 || it + shift >= h.ni[t]) {
                            set_error("interface of patches %d and %d: unknowns do not match", pt, pb);
                            delete P;
                            return IGA_ERR_GEOMETRY;
                        }
                    }
                }
        } else {
            g.lift_off = 0;
        }
        // the low-precision blocking's copy of the grid shares these fields
        Grid& gl = P->grids_lp[gi];
        gl.state = g.state;
        gl.nbr_on = g.nbr_on;
        for (int sd = 0; sd < 4; ++sd) {
            gl.nbr_base[sd] = g.nbr_base[sd];
            gl.nbr_stride[sd] = g.nbr_stride[sd];
            gl.pin[sd] = g.pin[sd];
        }
        gl.lift_off = g.lift_off;
    }
    P->nlift = nlift;
    for (const Grid& g : P->grids)
        for (int k = 0; k < d; ++k) {
            const Tab1D& T = P->tabs[g.tab[k]];
            double lmin = 0.0, lmax = 0.0;
            for (int i = 0; i < T.ni; ++i) {
                const double v = P->dpool[T.oLam + i];
                lmin = i == 0 ? v : std::min(lmin, v);
                lmax = i == 0 ? v : std::max(lmax, v);
            }
            if (lmin > 0.0) P->lam_ratio = std::max(P->lam_ratio, lmax / lmin);
        }
    // further samples: the same grids (tables, blocking and tiles shared) over
    // their own unknowns and Gauss points, sample-major
    {
        const size_t ng1 = P->grids.size();
        const int64_t nd1 = P->ndof_total, nq1 = P->nqp_total;
        for (int smp = 1; smp < P->nsamples; ++smp)
            for (size_t i = 0; i < ng1; ++i) {
                Grid g = P->grids[i], gl = P->grids_lp[i];
                g.sample = gl.sample = smp;
                g.dof_off += smp * nd1;
                gl.dof_off = g.dof_off;
                g.qp_off += smp * nq1;
                gl.qp_off = g.qp_off;
                g.state += smp * static_cast<int>(ng1);
                gl.state = g.state;
                g.lift_off += smp * nlift;
                gl.lift_off = g.lift_off;
                P->grids.push_back(g);
                P->grids_lp.push_back(gl);
            }
        P->ndof_total = nd1 * P->nsamples;
        P->nqp_total = nq1 * P->nsamples;
        P->nlift = nlift * P->nsamples;
    }
    if (lds_max + kSolveLdsHead > kLdsLimit) {
        set_error("a component grid needs %zu bytes of LDS (limit %d)", lds_max + kSolveLdsHead, kLdsLimit);
        delete P;
        return IGA_ERR_INVALID_ARG;
    }
    P->lds_bytes = lds_max + kSolveLdsHead;  // + task context and cached task descriptions
    // without the learned preconditioner's activations (3D): the operator
    // tiles and the FD layouts alone
    P->lds_plain = (d == 3 ? std::max(lds_op, lds_fd_plain) : lds_max) + kSolveLdsHead;
    // task lists in decreasing size of the solver-state groups (longest-
    // processing-time order; a group is one grid, or the patch grids of one
    // component), the tasks of a group contiguous so that its partial sums
    // form one range
    const int ngrp = static_cast<int>(P->grids.size()) / npat;
    std::vector<int> ord(ngrp);
    for (int i = 0; i < ngrp; ++i) ord[i] = i;
    auto gsum = [&](const std::vector<Grid>& gv, int grp, auto f) {
        double v = 0.0;
        for (int pt = 0; pt < npat; ++pt) v += f(gv[static_cast<size_t>(grp) * npat + pt]);
        return v;
    };
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
        auto nd = [](const Grid& g) { return static_cast<double>(g.ndof); };
        return gsum(P->grids, a, nd) > gsum(P->grids, b, nd);
    });
    for (int grp : ord) {
        const int off = static_cast<int>(P->optask.size());
        int cnt = 0;
        for (int pt = 0; pt < npat; ++pt) {
            const int gi = grp * npat + pt;
            Grid& g = P->grids[gi];
            g.tile_off = static_cast<int>(P->optask.size());
            P->grids_lp[gi].tile_off = g.tile_off;
            for (int t = 0; t < g.ntile; ++t) P->optask.push_back({gi, t});
            cnt += g.ntile;
        }
        for (int pt = 0; pt < npat; ++pt) {
            for (Grid* g : {&P->grids[grp * npat + pt], &P->grids_lp[grp * npat + pt]}) {
                g->gtile_off = off;
                g->gntile = cnt;
            }
        }
    }
    // FD tasks: the blocks of a group are contiguous (partial sums), groups in
    // decreasing cost of one block, so that the costliest blocks are taken
    // first by the persistent workgroups.  Cost ~ unknowns x (short length +
    // block width): the short-direction product plus the block's long product.
    for (int cls = 0; cls < 2; ++cls) {
        std::vector<Grid>& gv = cls == 0 ? P->grids : P->grids_lp;
        std::vector<Task>& tv = cls == 0 ? P->fdtask : P->fdtask_lp;
        auto cost = [&](const Grid& g) {
            const int nsm = d == 2 ? g.ni[1 - g.big] : 1;
            return static_cast<double>(g.ndof) * (nsm + std::min(g.blk, g.ni[g.big]));
        };
        std::vector<int> fo(ord);
        std::stable_sort(fo.begin(), fo.end(),
                         [&](int a, int b) { return gsum(gv, a, cost) > gsum(gv, b, cost); });
        for (int grp : fo) {
            const int off = static_cast<int>(tv.size());
            for (int pt = 0; pt < npat; ++pt) {
                Grid& g = gv[grp * npat + pt];
                g.blk_off = static_cast<int>(tv.size());
                for (int t = 0; t < g.nblk; ++t) tv.push_back({grp * npat + pt, t});
            }
            for (int pt = 0; pt < npat; ++pt) {
                gv[grp * npat + pt].gblk_off = off;
                gv[grp * npat + pt].gnblk = static_cast<int>(tv.size()) - off;
            }
        }
    }
    // ---- workspace layout ----------------------------------------------------
    Layout& L = P->lay;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + std::max<size_t>(bytes, 1));
        return o;
    };
    const size_t ng = P->grids.size(), nd = static_cast<size_t>(P->ndof_total),
                 nqp = static_cast<size_t>(P->nqp_total);
    L.tabs = take(sizeof(Tab1D) * P->tabs.size());
    L.grids = take(sizeof(Grid) * ng);
    L.grids_lp = take(sizeof(Grid) * ng);
    L.dpool = take(sizeof(double) * P->dpool.size());
    L.ipool = take(sizeof(int) * P->ipool.size());
    L.fpool = take(sizeof(float) * P->fpool.size());
    L.hpool = take(sizeof(uint16_t) * P->hpool.size());
    L.ctrl = take(sizeof(double) * P->ctrl.size());
    L.G64 = take(sizeof(double) * nqp * P->ncompG);
    L.G32 = take(sizeof(float) * nqp * P->ncompG);
    L.Fq = take(sizeof(double) * nqp);
    L.b = take(sizeof(double) * nd);
    L.x = take(sizeof(double) * nd);
    L.d = take(sizeof(double) * nd);
    L.r2 = take(sizeof(double) * nd * 2);
    L.z = take(sizeof(double) * nd);
    L.p2 = take(sizeof(double) * nd * 2);
    L.q = take(sizeof(double) * nd);
    L.rt = take(sizeof(double) * nd);
    L.st2 = take(sizeof(GState) * ng * 2);
    size_t pst = std::max(P->optask.size(), std::max(P->fdtask.size(), P->fdtask_lp.size()));
    L.part = take(sizeof(double) * pst * 12);  // [6 kinds][2 parities][tasks]
    L.loga = take(sizeof(double) * nd);
    L.fdscale = take(sizeof(double) * nd);
    // two sums per local basis function of each element; an element has as
    // many local functions as Gauss points, (p+1)^d
    L.loc = take(sizeof(double) * 2 * nqp);
    L.lift = take(sizeof(double) * static_cast<size_t>(P->nlift));
    L.gmeta = take(sizeof(TaskMeta) * ng);
    L.gmeta_lp = take(sizeof(TaskMeta) * ng);
    L.oplist = take(sizeof(Task) * 2 * P->optask.size());
    L.fdlist = take(sizeof(Task) * 2 * std::max(P->fdtask.size(), P->fdtask_lp.size()));
    L.optask = take(sizeof(Task) * P->optask.size());
    L.fdtask = take(sizeof(Task) * P->fdtask.size());
    L.fdtask_lp = take(sizeof(Task) * P->fdtask_lp.size());
    L.bar = take(kBarBytes);
    L.trace = take(sizeof(unsigned long long) * (1 + 6 * 4096));
    L.fg = take(sizeof(double) * (kFgKinds * kFgBlocks + kFgScalars));
    L.nnw = take(sizeof(uint16_t) * kNnPackedMax);
    L.total = off;
    *out = P;
    return IGA_OK;
}

iga_status iga_sg_workspace_bytes(iga_sg_plan plan, size_t* bytes) {
    if (!plan || !bytes) {
        set_error("null argument");
        return IGA_ERR_INVALID_ARG;
    }
    *bytes = plan->lay.total;
    return IGA_OK;
}

iga_status iga_sg_plan_stats(iga_sg_plan plan, int* op_tasks, int* fd_tasks_fp64, int* fd_tasks_lowp,
                             size_t* lds_bytes, size_t* lds_plain_bytes) {
    if (!plan) {
        set_error("null plan");
        return IGA_ERR_INVALID_ARG;
    }
    if (op_tasks) *op_tasks = static_cast<int>(plan->optask.size());
    if (fd_tasks_fp64) *fd_tasks_fp64 = static_cast<int>(plan->fdtask.size());
    if (fd_tasks_lowp) *fd_tasks_lowp = static_cast<int>(plan->fdtask_lp.size());
    if (lds_bytes) *lds_bytes = plan->lds_bytes;
    if (lds_plain_bytes) *lds_plain_bytes = plan->lds_plain;
    return IGA_OK;
}

iga_status iga_sg_components(iga_sg_plan plan, int* n, int* levels_host, int64_t* ndof_host,
                             double* coef_host) {
    if (!plan) {
        set_error("null plan");
        return IGA_ERR_INVALID_ARG;
    }
    if (n) *n = plan->ncomp;
    for (int c = 0; c < plan->ncomp; ++c) {
        if (levels_host)
            for (int k = 0; k < plan->dim; ++k) levels_host[c * plan->dim + k] = plan->comp_levels[c * plan->dim + k];
        if (coef_host) coef_host[c] = plan->comp_coef[c];
        if (ndof_host) {
            int64_t s = 0;
            for (const Grid& g : plan->grids)
                if (g.comp == c && g.sample == 0) s += g.ndof;  // unknowns of one sample
            ndof_host[c] = s;
        }
    }
    return IGA_OK;
}

iga_status iga_sg_fd_factor(iga_sg_plan plan, int dir, int lev, int* n, double* U_host, double* lam_host) {
    if (!plan || dir < 0 || dir >= plan->dim || lev < 0 || lev > plan->Lmax) {
        set_error("bad plan/direction/level");
        return IGA_ERR_INVALID_ARG;
    }
    const Tab1D& T = plan->tabs[tab_index(plan, 0, dir, lev)];
    if (n) *n = T.ni;
    if (U_host)
        for (int i = 0; i < T.ni; ++i)
            std::memcpy(U_host + static_cast<size_t>(i) * T.ni, &plan->dpool[T.oU + static_cast<int64_t>(i) * T.ldu],
                        T.ni * sizeof(double));
    if (lam_host) std::memcpy(lam_host, &plan->dpool[T.oLam], T.ni * sizeof(double));
    return IGA_OK;
}

iga_status iga_sg_prolongation(iga_sg_plan plan, int dir, int lev, int* nf, int* nc, double* T_host) {
    if (!plan || !nf || !nc || dir < 0 || dir >= plan->dim || lev < 0 || lev >= plan->w || plan->xfer_off.empty()) {
        set_error("iga_sg_prolongation: a full tensor plan of one patch, 0 <= dir < dim, 0 <= lev < w");
        return IGA_ERR_INVALID_ARG;
    }
    const Tab1D& Tf = plan->tabs[tab_index(plan, 0, dir, plan->w)];
    const Tab1D& Tc = plan->tabs[tab_index(plan, 0, dir, lev)];
    *nf = Tf.ni;
    *nc = Tc.ni;
    if (T_host) {
        const int64_t o = plan->xfer_off[static_cast<size_t>(dir) * (plan->w + 1) + lev];
        std::memcpy(T_host, plan->dpool.data() + o, sizeof(double) * static_cast<size_t>(Tf.ni) * Tc.ni);
    }
    return IGA_OK;
}

iga_status iga_sg_matrices_1d(iga_sg_plan plan, int dir, int lev, int* n, double* K_host, double* M_host) {
    if (!plan || dir < 0 || dir >= plan->dim || lev < 0 || lev > plan->Lmax) {
        set_error("bad plan/direction/level");
        return IGA_ERR_INVALID_ARG;
    }
    int ti = tab_index(plan, 0, dir, lev);
    const Tab1D& T = plan->tabs[ti];
    if (n) *n = T.ni;
    size_t nn = static_cast<size_t>(T.ni) * T.ni;
    if (K_host) std::memcpy(K_host, plan->K1d[ti].data(), nn * sizeof(double));
    if (M_host) std::memcpy(M_host, plan->M1d[ti].data(), nn * sizeof(double));
    return IGA_OK;
}

}  // extern "C"
