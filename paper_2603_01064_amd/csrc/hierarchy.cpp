// Host FP64 construction of the grid hierarchy.
//
// Level 1 carries A_1 = alpha I + K^T K with the truncated Gaussian
// convolution K of the integral equation (Sec. 2.1); in 2D the operator is
// the Kronecker form alpha I (x) I + (K (x) K)^T (K (x) K) (Sec. 4.2 with the
// Tikhonov normal equations).  The paper's own form alpha I + K (2D
// alpha I (x) I + K (x) K) uses G_1 = K instead of K^T K.  Coarser levels are Galerkin products
// A_{l+1} = I_l^{l+1} A_l I_{l+1}^l (Algorithm 1), which keep the form
// alpha M_l (x) M_l + G_l (x) G_l with M_{l+1} = R1 M_l P1 and
// G_{l+1} = R1 G_l P1 for the 1D transfers R1 = P1^T / 2 (full weighting)
// and P1 (linear interpolation).  Every factor is a band matrix; its rows
// near the boundary differ from the interior, so rows are stored one by one.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "nmg_internal.h"

namespace nmg {

namespace {

// K K for the Toeplitz section K with taps k[-R..R]: radius 2R band.
Band gaussian_normal_band(int n, const std::vector<double>& taps, int R) {
    Band g;
    g.n = n;
    g.r = 2 * R;
    const int w = 2 * g.r + 1;
    g.a.assign((size_t)n * w, 0.0);
    for (int i = 0; i < n; ++i) {
        for (int j = std::max(0, i - g.r); j <= std::min(n - 1, i + g.r); ++j) {
            const int m0 = std::max({0, i - R, j - R});
            const int m1 = std::min({n - 1, i + R, j + R});
            double acc = 0.0;
            for (int m = m0; m <= m1; ++m) acc += taps[(size_t)(m - i + R)] * taps[(size_t)(j - m + R)];
            g.a[(size_t)i * w + (j - i + g.r)] = acc;
        }
    }
    return g;
}

// K itself: the radius-R Toeplitz band.
Band gaussian_band(int n, const std::vector<double>& taps, int R) {
    Band g;
    g.n = n;
    g.r = R;
    const int w = 2 * R + 1;
    g.a.assign((size_t)n * w, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = std::max(0, i - R); j <= std::min(n - 1, i + R); ++j) g.a[(size_t)i * w + (j - i + R)] = taps[(size_t)(j - i + R)];
    return g;
}

// R1 B P1 with R1 = P1^T/2: coarse (i, j) gathers fine rows 2i..2i+2 with
// weights 1/4, 1/2, 1/4 and fine columns 2j..2j+2 with weights 1/2, 1, 1/2.
Band galerkin(const Band& B) {
    static const double wr[3] = {0.25, 0.5, 0.25};
    static const double wp[3] = {0.5, 1.0, 0.5};
    Band c;
    c.n = (B.n - 1) / 2;
    c.r = (B.r + 2) / 2;
    const int w = 2 * c.r + 1;
    c.a.assign((size_t)c.n * w, 0.0);
    for (int i = 0; i < c.n; ++i) {
        for (int j = std::max(0, i - c.r); j <= std::min(c.n - 1, i + c.r); ++j) {
            double acc = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) acc += wr[a] * B.get(2 * i + a, 2 * j + b) * wp[b];
            c.a[(size_t)i * w + (j - i + c.r)] = acc;
        }
    }
    return c;
}

}  // namespace

bool split_toeplitz(const Band& B, ToeplitzSplit& out) {
    out = ToeplitzSplit{};
    const int n = B.n, r = B.r;
    if (n < 2 * r + 1) return false;
    const int mid = n / 2;
    out.r = r;
    out.t.assign((size_t)(2 * r + 1), 0.0);
    for (int d = -r; d <= r; ++d) out.t[(size_t)(d + r)] = B.get(mid, mid + d);
    int rc_top = 0, rc_bot = 0;
    for (int i = 0; i < n; ++i)
        for (int j = std::max(0, i - r); j <= std::min(n - 1, i + r); ++j) {
            const double dv = B.get(i, j) - out.t[(size_t)(j - i + r)];
            if (dv == 0.0) continue;
            if (i < mid && j < mid) rc_top = std::max(rc_top, std::max(i, j) + 1);
            else if (i >= mid && j >= mid) rc_bot = std::max(rc_bot, n - std::min(i, j));
            else return false;
        }
    const int rc = std::max(rc_top, rc_bot);
    if (rc > r) return false;
    out.rc = rc;
    out.dtl.assign((size_t)rc * rc, 0.0);
    out.dbr.assign((size_t)rc * rc, 0.0);
    for (int i = 0; i < rc; ++i)
        for (int j = 0; j < rc; ++j) {
            const double tij = std::abs(j - i) <= r ? out.t[(size_t)(j - i + r)] : 0.0;
            out.dtl[(size_t)i * rc + j] = B.get(i, j) - tij;
            const int bi = n - rc + i, bj = n - rc + j;
            out.dbr[(size_t)i * rc + j] = B.get(bi, bj) - tij;
        }
    out.ok = true;
    return true;
}

// D of the 1D regulariser -(a u')' with a(z) = 1 + 0.5 sin(2 pi z) taken at
// the cell midpoints (i + 1/2) h; the 1/h^2 factor is left out so that D has
// the O(1) scale of the identity it replaces (Sec. 4.1, anisotropic case).
Band anisotropic_band(int n) {
    Band d;
    d.n = n;
    d.r = 1;
    d.a.assign((size_t)n * 3, 0.0);
    const double h = 1.0 / (n + 1);
    auto a = [&](int k) { return 1.0 + 0.5 * std::sin(2.0 * M_PI * (k + 0.5) * h); };
    for (int i = 0; i < n; ++i) {
        if (i > 0) d.a[(size_t)i * 3 + 0] = -a(i);
        d.a[(size_t)i * 3 + 1] = a(i) + a(i + 1);
        if (i + 1 < n) d.a[(size_t)i * 3 + 2] = -a(i + 1);
    }
    return d;
}

// Cholesky of the symmetric band matrix cx X + cy Y + shift I in O(n r^2);
// true when every pivot is positive (the matrix is positive definite).
bool band_pd(const Band& X, double cx, const Band& Y, double cy, double shift) {
    const int n = X.n, r = std::max(X.r, Y.r), w = r + 1;
    std::vector<double> L((size_t)n * w, 0.0);  // L[i*w + (i - j)], j in [i - r, i]
    for (int i = 0; i < n; ++i) {
        for (int j = std::max(0, i - r); j <= i; ++j) {
            double v = cx * X.get(i, j) + cy * Y.get(i, j) + (i == j ? shift : 0.0);
            for (int m = std::max(0, i - r); m < j; ++m) v -= L[(size_t)i * w + (i - m)] * L[(size_t)j * w + (j - m)];
            if (j == i) {
                if (!(v > 0.0) || !std::isfinite(v)) return false;
                L[(size_t)i * w] = std::sqrt(v);
            } else {
                L[(size_t)i * w + (i - j)] = v / L[(size_t)j * w];
            }
        }
    }
    return true;
}

// Smallest alpha (to bisection accuracy, rounded up) at or below which the
// finest operator is not positive definite; 0 when it is for every alpha > 0.
//  1D: alpha M + G with M = I or D, by bisection on alpha.
//  2D: alpha I + G (x) G has eigenvalues alpha + g_i g_j, so the floor is
//      -g_min g_max when g_min < 0; both ends of the spectrum of G by
//      bisection on a shift.
double alpha_floor_of(const Band& M, const Band& G, int dim) {
    const int n = G.n;
    Band zero;
    zero.n = n;
    zero.r = 0;
    zero.a.assign((size_t)n, 0.0);
    if (dim == 1) {
        if (band_pd(G, 1.0, M, 0.0, 0.0)) return 0.0;
        double hi = 1e-12;
        while (!band_pd(M, hi, G, 1.0, 0.0)) {
            hi *= 2.0;
            if (hi > 1e12) return INFINITY;
        }
        double lo = 0.0;
        for (int it = 0; it < 64; ++it) {
            const double mid = 0.5 * (lo + hi);
            (band_pd(M, mid, G, 1.0, 0.0) ? hi : lo) = mid;
        }
        return hi;
    }
    if (band_pd(G, 1.0, zero, 0.0, 0.0)) return 0.0;
    double gersh = 0.0, dmin = INFINITY, dmax = -INFINITY;
    for (int i = 0; i < n; ++i) {
        double off = 0.0;
        for (int j = std::max(0, i - G.r); j <= std::min(n - 1, i + G.r); ++j)
            if (j != i) off += std::fabs(G.get(i, j));
        gersh = std::max(gersh, std::fabs(G.get(i, i)) + off);
        dmin = std::min(dmin, G.get(i, i));
        dmax = std::max(dmax, G.get(i, i));
    }
    // lambda_min: G - t I is positive definite exactly for t < lambda_min
    double ok = -gersh, bad = dmin;
    for (int it = 0; it < 64; ++it) {
        const double mid = 0.5 * (ok + bad);
        (band_pd(G, 1.0, zero, 0.0, -mid) ? ok : bad) = mid;
    }
    const double gmin = ok;  // at or below lambda_min
    // lambda_max: t I - G is positive definite exactly for t > lambda_max
    double okm = gersh, badm = dmax;
    for (int it = 0; it < 64; ++it) {
        const double mid = 0.5 * (okm + badm);
        (band_pd(G, -1.0, zero, 0.0, mid) ? okm : badm) = mid;
    }
    return -gmin * okm;  // okm at or above lambda_max
}

// Simultaneous diagonalisation of the coarsest level's factors for an exact
// solve of alpha M (x) M + G (x) G at any alpha: with M = L L^T (Cholesky) and
// L^-1 G L^-T = Q diag(lam) Q^T (cyclic Jacobi rotations), V = L^-T Q gives
// V^T M V = I and V^T G V = diag(lam), so the 2D operator becomes diagonal,
// alpha + lam_i lam_j, in the basis V (x) V.  V is row-major n x n.
bool coarse_eigenbasis(const Band& M, const Band& G, std::vector<double>& V, std::vector<double>& lam,
                       std::string& err) {
    const int n = M.n;
    std::vector<double> Lc((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double v = M.get(i, j);
            for (int k = 0; k < j; ++k) v -= Lc[(size_t)i * n + k] * Lc[(size_t)j * n + k];
            if (i == j) {
                if (!(v > 0.0)) {
                    err = "coarsest mass factor is not positive definite";
                    return false;
                }
                Lc[(size_t)i * n + i] = std::sqrt(v);
            } else {
                Lc[(size_t)i * n + j] = v / Lc[(size_t)j * n + j];
            }
        }
    // S = L^-1 G L^-T: W = L^-1 G by forward substitution on columns, S = L^-1 W^T (W^T = G L^-T)
    std::vector<double> W((size_t)n * n), S((size_t)n * n);
    for (int col = 0; col < n; ++col)
        for (int i = 0; i < n; ++i) {
            double v = G.get(i, col);
            for (int k = 0; k < i; ++k) v -= Lc[(size_t)i * n + k] * W[(size_t)k * n + col];
            W[(size_t)i * n + col] = v / Lc[(size_t)i * n + i];
        }
    for (int col = 0; col < n; ++col)
        for (int i = 0; i < n; ++i) {
            double v = W[(size_t)col * n + i];  // (W^T)[i][col]
            for (int k = 0; k < i; ++k) v -= Lc[(size_t)i * n + k] * S[(size_t)k * n + col];
            S[(size_t)i * n + col] = v / Lc[(size_t)i * n + i];
        }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) S[(size_t)i * n + j] = S[(size_t)j * n + i] = 0.5 * (S[(size_t)i * n + j] + S[(size_t)j * n + i]);
    // cyclic Jacobi: S <- J^T S J until the off-diagonal part is negligible
    std::vector<double> Q((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
    double scale = 0.0;
    for (double v : S) scale += v * v;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += 2.0 * S[(size_t)i * n + j] * S[(size_t)i * n + j];
        if (off <= 1e-30 * scale) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = S[(size_t)p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                const double theta = (S[(size_t)q * n + q] - S[(size_t)p * n + p]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < n; ++k) {  // columns p, q
                    const double skp = S[(size_t)k * n + p], skq = S[(size_t)k * n + q];
                    S[(size_t)k * n + p] = c * skp - sn * skq;
                    S[(size_t)k * n + q] = sn * skp + c * skq;
                }
                for (int k = 0; k < n; ++k) {  // rows p, q
                    const double spk = S[(size_t)p * n + k], sqk = S[(size_t)q * n + k];
                    S[(size_t)p * n + k] = c * spk - sn * sqk;
                    S[(size_t)q * n + k] = sn * spk + c * sqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double qkp = Q[(size_t)k * n + p], qkq = Q[(size_t)k * n + q];
                    Q[(size_t)k * n + p] = c * qkp - sn * qkq;
                    Q[(size_t)k * n + q] = sn * qkp + c * qkq;
                }
            }
    }
    lam.assign((size_t)n, 0.0);
    for (int i = 0; i < n; ++i) lam[(size_t)i] = S[(size_t)i * n + i];
    // V = L^-T Q by back substitution, column by column
    V.assign((size_t)n * n, 0.0);
    for (int col = 0; col < n; ++col)
        for (int i = n - 1; i >= 0; --i) {
            double v = Q[(size_t)i * n + col];
            for (int k = i + 1; k < n; ++k) v -= Lc[(size_t)k * n + i] * V[(size_t)k * n + col];
            V[(size_t)i * n + col] = v / Lc[(size_t)i * n + i];
        }
    return true;
}

bool build_host_hierarchy(int n, double s, double trunc, int levels, int dim, int form, std::vector<HostLevel>& out,
                          int* taps_radius, double* alpha_floor, std::string& err) {
    if (form != NMG_OP_NORMAL && form != NMG_OP_KERNEL && form != NMG_OP_ANISO) {
        err = "unknown operator form";
        return false;
    }
    if (form == NMG_OP_ANISO && dim != 1) {
        err = "the anisotropic regulariser is one-dimensional";
        return false;
    }
    if (n < 1) {
        err = "n must be positive";
        return false;
    }
    if (((n + 1) & n) != 0) {
        err = "n must be 2^k - 1";
        return false;
    }
    if (!(s > 0.0) || !(trunc > 0.0)) {
        err = "s and trunc must be positive";
        return false;
    }
    int nl = n;
    for (int l = 1; l < levels; ++l) {
        if (nl < 3) {
            err = "too many levels for this grid";
            return false;
        }
        nl = (nl - 1) / 2;
    }
    const double h = 1.0 / (n + 1);
    const int R = (int)std::floor(trunc * s / h + 1e-9);
    std::vector<double> taps((size_t)(2 * R + 1));
    const double norm = h / (std::sqrt(2.0 * M_PI) * s);
    for (int j = -R; j <= R; ++j) {
        const double z = j * h;
        taps[(size_t)(j + R)] = norm * std::exp(-z * z / (2.0 * s * s));
    }
    *taps_radius = R;
    out.clear();
    HostLevel l0;
    l0.n = n;
    l0.G = form == NMG_OP_NORMAL ? gaussian_normal_band(n, taps, R) : gaussian_band(n, taps, R);
    if (form == NMG_OP_ANISO) {
        l0.M = anisotropic_band(n);
    } else {
        l0.M.n = n;
        l0.M.r = 0;
        l0.M.a.assign((size_t)n, 1.0);
    }
    // K^T K is positive semi-definite, so the normal equations need only alpha > 0
    *alpha_floor = form == NMG_OP_NORMAL ? 0.0 : alpha_floor_of(l0.M, l0.G, dim);
    out.push_back(std::move(l0));
    for (int l = 1; l < levels; ++l) {
        HostLevel c;
        c.M = galerkin(out.back().M);
        c.G = galerkin(out.back().G);
        c.n = c.M.n;
        out.push_back(std::move(c));
    }
    for (auto& hl : out) {
        split_toeplitz(hl.M, hl.Ms);
        split_toeplitz(hl.G, hl.Gs);
    }
    return true;
}

}  // namespace nmg
