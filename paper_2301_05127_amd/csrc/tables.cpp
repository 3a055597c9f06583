// Host FP64 tables of one axis: PMBC rows (paper Sec. 3.2, eq. PMBC and
// PMBC_coeffcients), row kinds, and the LU factors of the derivative systems.
//
// Rows of b = A^{-1} of the global natural-end collocation system (Sec. 3.1,
// eq. spline_cofficient_eq) are obtained from its reduction: the natural rows give
// v~_0 = v_0 and v~_N = v_N, the ghosts are v~_{-1} = 2 v~_0 - v~_1 and
// v~_{N+1} = 2 v~_N - v~_{N-1}, and the interior coefficients solve the symmetric
// Toeplitz system tridiag(1,4,1) v~ = 6 v - (boundary terms).  Row i of its inverse
// is one Thomas solve with the unit vector e_i.  The periodic line uses the
// circulant collocation system, whose inverse column has the closed form
// g_k = alpha (r^k + r^{N-k}), r = sqrt(3) - 2, from the two decaying homogeneous
// solutions of the three-term recurrence.
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "loss_internal.h"

namespace loss {
namespace {

// Solve tridiag(1,4,1) x = e_i of size n (unknowns 0..n-1), Thomas in FP64.
void toeplitz_unit_solve(int n, int i, std::vector<double> &x)
{
    std::vector<double> cpr(n), d(n, 0.0);
    x.assign(n, 0.0);
    d[i] = 1.0;
    double den = 4.0;
    cpr[0] = 1.0 / den;
    d[0] = d[0] / den;
    for (int k = 1; k < n; ++k) {
        den = 4.0 - cpr[k - 1];
        cpr[k] = 1.0 / den;
        d[k] = (d[k] - d[k - 1]) / den;
    }
    x[n - 1] = d[n - 1];
    for (int k = n - 2; k >= 0; --k) x[k] = d[k] - cpr[k] * x[k + 1];
}

// Row i (-1 <= i <= N+1) of b = A^{-1}, natural ends: out[k] = b_{i,k}, k = 0..N.
void natural_inverse_row(int N, int i, std::vector<double> &out)
{
    out.assign(N + 1, 0.0);
    if (i == 0) { out[0] = 1.0; return; }
    if (i == N) { out[N] = 1.0; return; }
    if (i == -1 || i == N + 1) {
        // ghost rows from the natural end rows
        int inner = (i == -1) ? 1 : N - 1, end = (i == -1) ? 0 : N;
        natural_inverse_row(N, inner, out);
        for (double &v : out) v = -v;
        out[end] += 2.0;
        return;
    }
    // interior: v~_i = sum_m G_{i,m} (6 v_m - [m=1] v_0 - [m=N-1] v_N), G = T^{-1},
    // T = tridiag(1,4,1) on nodes 1..N-1 (index m-1)
    std::vector<double> g;
    toeplitz_unit_solve(N - 1, i - 1, g);   // row i of G (G is symmetric)
    for (int m = 1; m <= N - 1; ++m) out[m] = 6.0 * g[m - 1];
    out[0] = -g[0];
    out[N] -= g[N - 2];
}

// First column of the circulant inverse (N distinct nodes).
void periodic_inverse_col(int N, std::vector<double> &g)
{
    const double r = std::sqrt(3.0) - 2.0;
    g.assign(N, 0.0);
    const double rN = std::pow(r, N), rN1 = std::pow(r, N - 1);
    const double alpha = 6.0 / (4.0 + 2.0 * r + 2.0 * rN1 + 4.0 * rN);
    for (int k = 0; k < N; ++k) g[k] = alpha * (std::pow(r, k) + std::pow(r, N - k));
}

// Rows of composition a chunk boundary needs in one sweep direction.  Forward
// elimination: y_r = rhs_r - f_r y_{r-1} on rows lo..hi-1 (the carry into row lo
// is exact).  The carry into row q depends on the one W rows earlier through the
// product f_{q-W} ... f_{q-1}; the window stops growing once it reaches row lo or
// that product is below tol.
int forward_reach(const std::vector<double> &f, int lo, int hi, double tol)
{
    int R = 0;
    for (int q = lo + 1; q < hi; ++q) {
        double prod = 1.0;
        int W = 0;
        while (q - W > lo && std::fabs(prod) > tol) { prod *= f[q - 1 - W]; ++W; }
        R = std::max(R, W);
    }
    return R;
}

// Back substitution: w_r = (y_r - g_r w_{r+1}) / d_r on rows lo..hi-1 (the carry
// into row hi-1 is the exact closing-row value).
int backward_reach(const std::vector<double> &g, int lo, int hi, double tol)
{
    int R = 0;
    for (int r = lo; r + 1 < hi; ++r) {
        double prod = 1.0;
        int W = 0;
        while (r + W + 1 < hi && std::fabs(prod) > tol) { prod *= g[r + 1 + W]; ++W; }
        R = std::max(R, W);
    }
    return R;
}

}  // namespace

std::string build_axis(AxisHost &ax, int N, double h, int M, int halo, int end_mode)
{
    if (N < 2) return "an axis needs at least 2 intervals";
    if (M < 1) return "patch length must be >= 1";
    if (halo < 1 || halo > kMaxHalo) return "halo must be in 1..64";
    if (!(h > 0.0)) return "spacing must be positive";
    if (end_mode == 2 && 2 * halo + 1 > N) return "periodic axis needs 2*halo+1 <= n";
    if (end_mode < 0 || end_mode > 2) return "unknown end mode";
    ax = AxisHost();
    ax.N = N; ax.M = M; ax.halo = halo; ax.end_mode = end_mode; ax.h = h;
    ax.p = (N + M - 1) / M;
    const int n = N + 1, ntap = 2 * halo + 1;
    ax.kind.assign(n, ROW_INTERIOR);
    for (int J = M; J < N; J += M) ax.kind[J] = ROW_JUNCTION;
    if (end_mode == 0) {
        ax.kind[0] = ROW_NATURAL_L;
        ax.kind[N] = ROW_NATURAL_R;
    } else {
        ax.kind[0] = ax.kind[N] = ROW_JUNCTION;
    }
    // ---- PMBC rows ------------------------------------------------------
    ax.slot.assign(n, -1);
    std::vector<double> rp, rm, g;
    if (end_mode == 2) periodic_inverse_col(N, g);
    for (int J = 0; J <= N; ++J) {
        if (ax.kind[J] != ROW_JUNCTION) continue;
        int s = (int)ax.junction_node.size();
        ax.slot[J] = s;
        ax.junction_node.push_back(J);
        ax.tap_idx.resize((size_t)(s + 1) * ntap, -1);
        ax.tap_c.resize((size_t)(s + 1) * ntap, 0.0);
        if (end_mode == 2) {
            for (int t = 0; t < ntap; ++t) {
                int k = ((J - halo + t) % N + N) % N;
                int ip = ((J + 1 - k) % N + N) % N, im = ((J - 1 - k) % N + N) % N;
                ax.tap_idx[(size_t)s * ntap + t] = k;
                ax.tap_c[(size_t)s * ntap + t] = (g[ip] - g[im]) / (2.0 * h);
            }
        } else {
            natural_inverse_row(N, J + 1, rp);
            natural_inverse_row(N, J - 1, rm);
            for (int t = 0; t < ntap; ++t) {
                int k = J - halo + t;
                if (k < 0 || k > N) continue;
                ax.tap_idx[(size_t)s * ntap + t] = k;
                ax.tap_c[(size_t)s * ntap + t] = (rp[k] - rm[k]) / (2.0 * h);
            }
        }
    }
    // ---- rows of T and G ---------------------------------------------------
    ax.sub.assign(n, 0.0); ax.diag.assign(n, 0.0); ax.sup.assign(n, 0.0);
    ax.cm.assign(n, 0.0); ax.c0.assign(n, 0.0); ax.cp.assign(n, 0.0);
    const double s3 = 3.0 / h;
    for (int i = 0; i <= N; ++i) {
        switch (ax.kind[i]) {
        case ROW_INTERIOR:
            ax.sub[i] = 1.0; ax.diag[i] = 4.0; ax.sup[i] = 1.0;
            ax.cm[i] = -s3; ax.cp[i] = s3;
            break;
        case ROW_JUNCTION:
            ax.diag[i] = 1.0;
            break;
        case ROW_NATURAL_L:
            ax.diag[i] = 2.0; ax.sup[i] = 1.0;
            ax.c0[i] = -s3; ax.cp[i] = s3;
            break;
        case ROW_NATURAL_R:
            ax.sub[i] = 1.0; ax.diag[i] = 2.0;
            ax.cm[i] = -s3; ax.c0[i] = s3;
            break;
        }
    }
    // ---- LU of T, no pivoting ---------------------------------------------
    ax.m.assign(n, 0.0); ax.invd.assign(n, 0.0);
    double dprev = 0.0;
    for (int i = 0; i <= N; ++i) {
        double mi = (i == 0) ? 0.0 : ax.sub[i] / dprev;
        double di = ax.diag[i] - (i == 0 ? 0.0 : mi * ax.sup[i - 1]);
        ax.m[i] = mi;
        ax.invd[i] = 1.0 / di;
        dprev = di;
    }
    // ---- LU of T^T ---------------------------------------------------------
    ax.mT.assign(n, 0.0); ax.invdT.assign(n, 0.0); ax.supT.assign(n, 0.0); ax.subT.assign(n, 0.0);
    dprev = 0.0;
    for (int i = 0; i <= N; ++i) {
        double subT = (i == 0) ? 0.0 : ax.sup[i - 1];
        double supT = (i == N) ? 0.0 : ax.sub[i + 1];
        double mi = (i == 0) ? 0.0 : subT / dprev;
        double di = ax.diag[i] - (i == 0 ? 0.0 : mi * ax.supT[i - 1]);
        ax.subT[i] = subT;
        ax.supT[i] = supT;
        ax.mT[i] = mi;
        ax.invdT[i] = 1.0 / di;
        dprev = di;
    }
    // ---- transposed PMBC gather ---------------------------------------------
    // (a halo wider than the patches reaches a node from several junction rows: the
    // table is as wide as the most rows reaching one node)
    std::vector<int> cnt(n, 0);
    for (size_t s = 0; s < ax.junction_node.size(); ++s)
        for (int t = 0; t < ntap; ++t) {
            const int k = ax.tap_idx[s * ntap + t];
            if (k >= 0 && ax.tap_c[s * ntap + t] != 0.0) ++cnt[k];
        }
    ax.gmax = std::max(1, *std::max_element(cnt.begin(), cnt.end()));
    ax.g_node.assign((size_t)n * ax.gmax, -1);
    ax.g_c.assign((size_t)n * ax.gmax, 0.0);
    std::fill(cnt.begin(), cnt.end(), 0);
    for (size_t s = 0; s < ax.junction_node.size(); ++s) {
        for (int t = 0; t < ntap; ++t) {
            int k = ax.tap_idx[s * ntap + t];
            if (k < 0) continue;
            double c = ax.tap_c[s * ntap + t];
            if (c == 0.0) continue;
            ax.g_node[(size_t)k * ax.gmax + cnt[k]] = ax.junction_node[s];
            ax.g_c[(size_t)k * ax.gmax + cnt[k]] = c;
            ++cnt[k];
        }
    }
    // ---- second-derivative system, patch by patch ---------------------------
    // first row: Hermite [2,1] at a junction, identity (s'' = 0) at a natural end;
    // interior rows [1,4,1]; closing row: Hermite [1,2] or identity.
    ax.m2.assign(n, 0.0); ax.invd2.assign(n, 0.0); ax.sup2.assign(n, 0.0);
    ax.m2c.assign(n, 0.0); ax.invd2c.assign(n, 0.0);
    for (int l = 0; l < ax.p; ++l) {
        int s = l * M, e = std::min(s + M, N);
        bool nat_l = ax.kind[s] == ROW_NATURAL_L, nat_r = ax.kind[e] == ROW_NATURAL_R;
        double d = nat_l ? 1.0 : 2.0;
        double supprev = nat_l ? 0.0 : 1.0;
        ax.m2[s] = 0.0; ax.invd2[s] = 1.0 / d; ax.sup2[s] = supprev;
        for (int i = s + 1; i < e; ++i) {
            double mi = 1.0 / d;
            d = 4.0 - mi * supprev;
            ax.m2[i] = mi; ax.invd2[i] = 1.0 / d; ax.sup2[i] = 1.0;
            supprev = 1.0;
        }
        if (nat_r) {
            ax.m2c[e] = 0.0; ax.invd2c[e] = 1.0;
        } else {
            double mi = 1.0 / d;
            ax.m2c[e] = mi;
            ax.invd2c[e] = 1.0 / (2.0 - mi * supprev);
        }
    }
    // ---- carry reach over the three systems, both sweeps ---------------------
    std::vector<double> g1(n), gT(n), g2(n);
    for (int i = 0; i < n; ++i) {
        g1[i] = ax.sup[i] * ax.invd[i];
        gT[i] = ax.supT[i] * ax.invdT[i];
        g2[i] = ax.sup2[i] * ax.invd2[i];
    }
    ax.reach = 1;
    for (int l = 0; l < ax.p; ++l) {
        int s = l * M, e = std::min(s + M, N);
        for (const std::vector<double> *f : {&ax.m, &ax.mT, &ax.m2})
            ax.reach = std::max(ax.reach, forward_reach(*f, s, e, kReachTol));
        for (const std::vector<double> *g : {&g1, &gT, &g2})
            ax.reach = std::max(ax.reach, backward_reach(*g, s, e, kReachTol));
    }
    return std::string();
}

}  // namespace loss
