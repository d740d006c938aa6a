// eigen.cpp -- host FP64 generalised symmetric-definite eigen-solver for the
// 1D factors of the fast-diagonalisation preconditioner:
//
//     K U = M U diag(lam),   U^T M U = I,
//
// with K (stiffness) and M (mass) symmetric banded.  Method (Golub & Van Loan,
// "Matrix Computations", Sec. 8.3 and 8.7): Cholesky M = L L^T, the standard
// problem C = L^-1 K L^-T, Householder reduction of C to tridiagonal form,
// the symmetric QR algorithm (implicit steps with the Wilkinson shift,
// Alg. 8.3.2, deflation as in Alg. 8.3.3), back-transformation U = L^-T Q Z.
// The O(n^3) stages (rotation replay, reflector application, triangular
// back-substitution) are split over column chunks on host threads.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>
#include <vector>

#include "eigen.hpp"

namespace igasg {

namespace {

int num_threads(int n) {
    unsigned hc = std::thread::hardware_concurrency();
    int t = hc ? static_cast<int>(hc) : 4;
    t = std::min(t, 16);
    if (n < 256) t = 1;
    return std::max(t, 1);
}

// Run f(c0, c1) over column chunks [0, ncol) on nt threads.
template <class F>
void parallel_cols(int ncol, int nt, F&& f) {
    if (nt <= 1) {
        f(0, ncol);
        return;
    }
    std::vector<std::thread> th;
    int chunk = (ncol + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
        int c0 = t * chunk, c1 = std::min(ncol, c0 + chunk);
        if (c0 >= c1) break;
        th.emplace_back([=, &f] { f(c0, c1); });
    }
    for (auto& x : th) x.join();
}

struct Rot {
    int i;
    double c, s;
};

}  // namespace

bool gen_eig_banded(int n, int bw, const double* K, const double* M, double* U, double* lam) {
    if (n <= 0) return false;
    const int nt = num_threads(n);
    // --- Cholesky M = L L^T (banded, L stored dense row-major lower) -------
    std::vector<double> L(static_cast<size_t>(n) * n, 0.0);
    for (int i = 0; i < n; ++i) {
        int j0 = std::max(0, i - bw);
        for (int j = j0; j <= i; ++j) {
            double s = M[static_cast<size_t>(i) * n + j];
            for (int k = std::max(j0, j - bw); k < j; ++k)
                s -= L[static_cast<size_t>(i) * n + k] * L[static_cast<size_t>(j) * n + k];
            if (j < i) {
                L[static_cast<size_t>(i) * n + j] = s / L[static_cast<size_t>(j) * n + j];
            } else {
                if (!(s > 0.0)) return false;
                L[static_cast<size_t>(i) * n + i] = std::sqrt(s);
            }
        }
    }
    // --- C = L^-1 K L^-T by two banded forward substitutions on rows --------
    auto lower_solve_rows = [&](std::vector<double>& X) {
        // X <- L^-1 X, row operations, columns split over threads
        parallel_cols(n, nt, [&](int c0, int c1) {
            for (int i = 0; i < n; ++i) {
                double* xi = &X[static_cast<size_t>(i) * n];
                for (int j = std::max(0, i - bw); j < i; ++j) {
                    double l = L[static_cast<size_t>(i) * n + j];
                    const double* xj = &X[static_cast<size_t>(j) * n];
                    for (int c = c0; c < c1; ++c) xi[c] -= l * xj[c];
                }
                double inv = 1.0 / L[static_cast<size_t>(i) * n + i];
                for (int c = c0; c < c1; ++c) xi[c] *= inv;
            }
        });
    };
    std::vector<double> A(K, K + static_cast<size_t>(n) * n);
    lower_solve_rows(A);                       // A = L^-1 K
    std::vector<double> At(static_cast<size_t>(n) * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) At[static_cast<size_t>(j) * n + i] = A[static_cast<size_t>(i) * n + j];
    lower_solve_rows(At);                      // At = L^-1 K^T L^-T = C
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) {
            double s = 0.5 * (At[static_cast<size_t>(i) * n + j] + At[static_cast<size_t>(j) * n + i]);
            At[static_cast<size_t>(i) * n + j] = At[static_cast<size_t>(j) * n + i] = s;
        }
    A.swap(At);
    At.clear();
    At.shrink_to_fit();

    // --- Householder tridiagonalisation, reflectors kept ---------------------
    std::vector<double> dg(n), e(n, 0.0);
    std::vector<std::vector<double>> refl(std::max(0, n - 2));
    std::vector<double> rbeta(std::max(0, n - 2), 0.0);
    std::vector<double> pv(n), wv(n);
    for (int k = 0; k + 2 < n; ++k) {
        int m = n - k - 1;
        std::vector<double>& v = refl[k];
        v.resize(m);
        double nrm = 0.0;
        for (int r = 0; r < m; ++r) {
            v[r] = A[static_cast<size_t>(k + 1 + r) * n + k];
            nrm += v[r] * v[r];
        }
        nrm = std::sqrt(nrm);
        if (nrm == 0.0) {
            e[k] = 0.0;
            rbeta[k] = 0.0;
            continue;
        }
        double alpha = v[0] > 0 ? -nrm : nrm;
        v[0] -= alpha;
        double vtv = 0.0;
        for (int r = 0; r < m; ++r) vtv += v[r] * v[r];
        if (vtv == 0.0) {
            e[k] = alpha;
            rbeta[k] = 0.0;
            continue;
        }
        double beta = 2.0 / vtv;
        rbeta[k] = beta;
        // p = beta A22 v (A22 symmetric, rows contiguous)
        for (int r = 0; r < m; ++r) {
            const double* ar = &A[static_cast<size_t>(k + 1 + r) * n + (k + 1)];
            double s = 0.0;
            for (int c = 0; c < m; ++c) s += ar[c] * v[c];
            pv[r] = beta * s;
        }
        double kk = 0.0;
        for (int r = 0; r < m; ++r) kk += v[r] * pv[r];
        kk *= 0.5 * beta;
        for (int r = 0; r < m; ++r) wv[r] = pv[r] - kk * v[r];
        for (int r = 0; r < m; ++r) {
            double* ar = &A[static_cast<size_t>(k + 1 + r) * n + (k + 1)];
            double vr = v[r], wr = wv[r];
            for (int c = 0; c < m; ++c) ar[c] -= vr * wv[c] + wr * v[c];
        }
        e[k] = alpha;
    }
    for (int i = 0; i < n; ++i) dg[i] = A[static_cast<size_t>(i) * n + i];
    if (n >= 2) e[n - 2] = A[static_cast<size_t>(n - 1) * n + (n - 2)];
    e[n - 1] = 0.0;
    A.clear();
    A.shrink_to_fit();

    // --- symmetric QR on (dg, e): implicit steps with the Wilkinson shift ----
    // (Golub & Van Loan, Alg. 8.3.2 and 8.3.3).  e[i] couples rows i and i+1.
    // Each step chases the bulge of one plane rotation R_k (rows k, k+1:
    // row_k <- c row_k + s row_(k+1), row_(k+1) <- -s row_k + c row_(k+1)) down
    // the unreduced block [lo, hi]; T <- R_k T R_k^T.  The rotations are
    // recorded in order and replayed on Z^T = ... R_2 R_1.
    std::vector<Rot> rots;
    rots.reserve(static_cast<size_t>(n) * 8);
    const double eps = 2.220446049250313e-16;
    int hi = n - 1, steps = 0;
    while (hi > 0) {
        // deflate negligible couplings at the bottom, then find the trailing
        // unreduced block [lo, hi] (couplings inside it tested on the way up)
        auto small = [&](int i) { return std::fabs(e[i]) <= eps * (std::fabs(dg[i]) + std::fabs(dg[i + 1])); };
        while (hi > 0 && small(hi - 1)) e[--hi] = 0.0;
        if (hi == 0) break;
        int lo = hi - 1;
        while (lo > 0 && !small(lo - 1)) --lo;
        if (lo > 0) e[lo - 1] = 0.0;
        if (++steps > 60 * n) return false;
        // Wilkinson shift: the eigenvalue of the trailing 2x2 block nearer dg[hi]
        const double dd = 0.5 * (dg[hi - 1] - dg[hi]);
        const double bb = e[hi - 1];
        const double mu = dg[hi] - bb * bb / (dd + (dd >= 0.0 ? 1.0 : -1.0) * std::hypot(dd, bb));
        double x = dg[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            const double r = std::hypot(x, z);
            const double c = r > 0.0 ? x / r : 1.0, sn = r > 0.0 ? z / r : 0.0;
            if (k > lo) e[k - 1] = r;  // the bulge below e[k-1] is rotated away
            const double p = dg[k], q = dg[k + 1], ek = e[k];
            dg[k] = c * c * p + 2.0 * c * sn * ek + sn * sn * q;
            dg[k + 1] = sn * sn * p - 2.0 * c * sn * ek + c * c * q;
            e[k] = c * sn * (q - p) + (c * c - sn * sn) * ek;
            rots.push_back({k, c, sn});
            if (k + 1 < hi) {
                x = e[k];
                z = sn * e[k + 1];  // new bulge at (k+2, k)
                e[k + 1] *= c;
            }
        }
    }
    // Z^T rows = columns of Z; start from identity and replay rotations
    std::vector<double> ZT(static_cast<size_t>(n) * n, 0.0);
    for (int i = 0; i < n; ++i) ZT[static_cast<size_t>(i) * n + i] = 1.0;
    parallel_cols(n, nt, [&](int c0, int c1) {
        for (const Rot& R : rots) {
            double* zi = &ZT[static_cast<size_t>(R.i) * n];
            double* zj = &ZT[static_cast<size_t>(R.i + 1) * n];
            for (int c = c0; c < c1; ++c) {
                const double u = zi[c], v = zj[c];
                zi[c] = R.c * u + R.s * v;
                zj[c] = R.c * v - R.s * u;
            }
        }
    });
    rots.clear();
    rots.shrink_to_fit();
    // Z (row-major, Z[r][k] = component r of eigenvector k)
    std::vector<double> Z(static_cast<size_t>(n) * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Z[static_cast<size_t>(j) * n + i] = ZT[static_cast<size_t>(i) * n + j];
    ZT.clear();
    ZT.shrink_to_fit();
    // apply reflectors: Z <- H_0 H_1 ... H_{n-3} Z
    parallel_cols(n, nt, [&](int c0, int c1) {
        std::vector<double> s(c1 - c0);
        for (int k = n - 3; k >= 0; --k) {
            if (rbeta[k] == 0.0) continue;
            const std::vector<double>& v = refl[k];
            int m = n - k - 1;
            std::fill(s.begin(), s.end(), 0.0);
            for (int r = 0; r < m; ++r) {
                const double* zr = &Z[static_cast<size_t>(k + 1 + r) * n];
                double vr = v[r];
                for (int c = c0; c < c1; ++c) s[c - c0] += vr * zr[c];
            }
            for (int r = 0; r < m; ++r) {
                double* zr = &Z[static_cast<size_t>(k + 1 + r) * n];
                double f = rbeta[k] * v[r];
                for (int c = c0; c < c1; ++c) zr[c] -= f * s[c - c0];
            }
        }
    });
    // U = L^-T Z (banded back substitution on rows)
    parallel_cols(n, nt, [&](int c0, int c1) {
        for (int i = n - 1; i >= 0; --i) {
            double* zi = &Z[static_cast<size_t>(i) * n];
            for (int j = i + 1; j <= std::min(n - 1, i + bw); ++j) {
                double l = L[static_cast<size_t>(j) * n + i];
                const double* zj = &Z[static_cast<size_t>(j) * n];
                for (int c = c0; c < c1; ++c) zi[c] -= l * zj[c];
            }
            double inv = 1.0 / L[static_cast<size_t>(i) * n + i];
            for (int c = c0; c < c1; ++c) zi[c] *= inv;
        }
    });
    // ascending eigenvalues
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return dg[a] < dg[b]; });
    for (int k = 0; k < n; ++k) lam[k] = dg[ord[k]];
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) U[static_cast<size_t>(i) * n + k] = Z[static_cast<size_t>(i) * n + ord[k]];
    return true;
}

}  // namespace igasg
