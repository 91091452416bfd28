// pcg_shift.cpp -- a-posteriori shift selection (Section 3.2 and Section 5.1).
//
// Host code.  The local rounding errors of shifted pipelined CG enter the
// gaps of r, s, w and z through the 4x4 recurrence pi_{i+1} = P_i pi_i + eps_i
// whose matrix depends only on the iteration's alpha_i, beta_i and the shift.
// The amplification of an error made at iteration j by iteration i is the
// spectral norm of P_i P_{i-1} ... P_j, and psi_i = its maximum over
// 1 <= j <= i.  Given the alpha / beta history a solve recorded (pcg_options
// .history), psi_i is evaluated on a grid of shifts and the shift to use for
// later solves of the same operator is picked from it.
//
// The spectral norm of a 4x4 product Q is sqrt(lambda_max(Q^T Q)), with the
// eigenvalues of the symmetric 4x4 matrix found by cyclic Jacobi rotations;
// Q is rescaled by its largest entry first so that long products cannot
// overflow Q^T Q.
#include <cmath>
#include <cstring>
#include <vector>

#include "pcg.h"

namespace pcg {
pcg_status invalid(const char *why);  // records the message for pcg_last_error
}
using pcg::invalid;

namespace {

struct M4 {
    double a[4][4];
};

M4 identity()
{
    M4 m{};
    for (int k = 0; k < 4; ++k) m.a[k][k] = 1.0;
    return m;
}

M4 mul(const M4 &x, const M4 &y)
{
    M4 r{};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += x.a[i][k] * y.a[k][j];
            r.a[i][j] = s;
        }
    return r;
}

// P_i(sigma_{i-1}, sigma_i) acting on [f_i, g_{i-1}, h_i, j_{i-1}]: the gap
// recurrences f_{i+1} = f_i - alpha g_i, g_i = h_i + beta g_{i-1},
// h_{i+1} = h_i - alpha j_i - alpha sigma_i g_i and
// j_i = beta j_{i-1} - (sigma_i - sigma_{i-1}) g_i with g_i substituted
// (Section 4.2; a constant shift gives P_i(sigma) of Section 3.2).
M4 prop(double alpha, double beta, double sig_prev, double sig)
{
    const double d = sig - sig_prev;
    M4 m{};
    m.a[0][0] = 1.0;
    m.a[0][1] = -alpha * beta;
    m.a[0][2] = -alpha;
    m.a[1][1] = beta;
    m.a[1][2] = 1.0;
    m.a[2][1] = -alpha * beta * sig_prev;
    m.a[2][2] = 1.0 - alpha * sig_prev;
    m.a[2][3] = -alpha * beta;
    m.a[3][1] = -beta * d;
    m.a[3][2] = -d;
    m.a[3][3] = beta;
    return m;
}

// Largest eigenvalue of a symmetric 4x4 matrix (cyclic Jacobi rotations).
double sym_max_eig(double s[4][4])
{
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int p = 0; p < 4; ++p) {
            diag += s[p][p] * s[p][p];
            for (int q = p + 1; q < 4; ++q) off += s[p][q] * s[p][q];
        }
        if (off <= 1e-32 * diag || off == 0.0) break;
        for (int p = 0; p < 3; ++p)
            for (int q = p + 1; q < 4; ++q) {
                if (s[p][q] == 0.0) continue;
                // rotation zeroing s[p][q]
                const double theta = (s[q][q] - s[p][p]) / (2.0 * s[p][q]);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < 4; ++k) {  // columns p, q
                    const double kp = s[k][p], kq = s[k][q];
                    s[k][p] = c * kp - sn * kq;
                    s[k][q] = sn * kp + c * kq;
                }
                for (int k = 0; k < 4; ++k) {  // rows p, q
                    const double pk = s[p][k], qk = s[q][k];
                    s[p][k] = c * pk - sn * qk;
                    s[q][k] = sn * pk + c * qk;
                }
            }
    }
    double m = s[0][0];
    for (int k = 1; k < 4; ++k) m = std::fmax(m, s[k][k]);
    return m;
}

double spectral_norm(const M4 &q)
{
    double scale = 0.0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) scale = std::fmax(scale, std::fabs(q.a[i][j]));
    if (scale == 0.0) return 0.0;
    if (!std::isfinite(scale)) return INFINITY;
    double g[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += (q.a[k][i] / scale) * (q.a[k][j] / scale);
            g[i][j] = s;
        }
    return scale * std::sqrt(std::fmax(sym_max_eig(g), 0.0));
}

// psi_i with shifts sig(k) for k >= -1.
template <typename Sig>
double psi_of(const double *alpha, const double *beta, int i, Sig sig)
{
    M4 q = identity();
    double best = 0.0;
    for (int j = i; j >= 1; --j) {  // P_{j,i} = P_{j+1,i} P_j
        q = mul(q, prop(alpha[j], beta[j], sig(j - 1), sig(j)));
        best = std::fmax(best, spectral_norm(q));
    }
    return best;
}

pcg_status check_history(const double *alpha, const double *beta, int32_t i)
{
    if (!alpha || !beta) return invalid("alpha and beta must be non-null");
    if (i < 1) return invalid("psi_i needs i >= 1");
    for (int k = 1; k <= i; ++k)
        if (!std::isfinite(alpha[k]) || !std::isfinite(beta[k]))
            return invalid("alpha_k and beta_k must be finite for 1 <= k <= i");
    return PCG_OK;
}

}  // namespace

extern "C" pcg_status pcg_psi(const double *alpha, const double *beta, int32_t i, double sigma, double *psi)
{
    pcg_status st = check_history(alpha, beta, i);
    if (st) return st;
    if (!psi) return invalid("psi is null");
    if (!std::isfinite(sigma)) return invalid("sigma must be finite");
    *psi = psi_of(alpha, beta, i, [&](int) { return sigma; });
    return PCG_OK;
}

extern "C" pcg_status pcg_psi_variable(const double *alpha, const double *beta, int32_t i,
                                       const double *sigma_schedule, int32_t sigma_schedule_len, double *psi)
{
    pcg_status st = check_history(alpha, beta, i);
    if (st) return st;
    if (!psi) return invalid("psi is null");
    if (!sigma_schedule || sigma_schedule_len < 1) return invalid("sigma_schedule needs at least one entry");
    for (int k = 0; k < sigma_schedule_len; ++k)
        if (!std::isfinite(sigma_schedule[k])) return invalid("sigma_schedule entries must be finite");
    *psi = psi_of(alpha, beta, i, [&](int k) {
        const int idx = k + 1 < sigma_schedule_len ? k + 1 : sigma_schedule_len - 1;
        return sigma_schedule[idx];
    });
    return PCG_OK;
}

extern "C" pcg_status pcg_select_shift(const double *alpha, const double *beta, int32_t i, const double *grid,
                                       int32_t grid_len, double slack, double *psi_out, double *sigma_best)
{
    pcg_status st = check_history(alpha, beta, i);
    if (st) return st;
    if (!grid || grid_len < 1 || !sigma_best) return invalid("grid (>= 1 entry) and sigma_best must be non-null");
    if (!(slack >= 1.0) || !std::isfinite(slack)) return invalid("slack must be finite and >= 1");
    for (int k = 0; k < grid_len; ++k)
        if (!std::isfinite(grid[k])) return invalid("grid entries must be finite");
    std::vector<double> vals(grid_len);
    double lo = INFINITY;
    for (int k = 0; k < grid_len; ++k) {
        vals[k] = psi_of(alpha, beta, i, [&](int) { return grid[k]; });
        lo = std::fmin(lo, vals[k]);
    }
    // the smallest shift whose psi is within `slack` of the grid minimum
    double pick = NAN;
    for (int k = 0; k < grid_len; ++k)
        if (vals[k] <= slack * lo && (std::isnan(pick) || grid[k] < pick)) pick = grid[k];
    if (psi_out) std::memcpy(psi_out, vals.data(), vals.size() * sizeof(double));
    if (std::isnan(pick)) return invalid("psi is not finite on any grid point");
    *sigma_best = pick;
    return PCG_OK;
}
