// Host FP64 construction of the grid hierarchy.
//
// Level 1 carries A_1 = alpha I + K^T K with the truncated Gaussian
// convolution K of the integral equation (Sec. 2.1); in 2D the operator is
// the Kronecker form alpha I (x) I + (K (x) K)^T (K (x) K) (Sec. 4.2 with the
// Tikhonov normal equations).  Coarser levels are Galerkin products
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

bool build_host_hierarchy(int n, double s, double trunc, int levels, std::vector<HostLevel>& out,
                          int* taps_radius, std::string& err) {
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
    l0.G = gaussian_normal_band(n, taps, R);
    l0.M.n = n;
    l0.M.r = 0;
    l0.M.a.assign((size_t)n, 1.0);
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
