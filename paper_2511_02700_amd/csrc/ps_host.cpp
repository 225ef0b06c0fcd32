// Host-side discretization of the price-space scheme (Sec. 3.2, Sec. 3.3,
// Sec. 4 settings).  FP64 throughout.
#include "ps_host.hpp"

#include <algorithm>
#include <cmath>

namespace lpide {

namespace {

// Lagrange basis through the four nodes p[0..3] at t.
void lagrange4(const double* p, double t, double* w) {
    for (int i = 0; i < 4; ++i) {
        double v = 1.0;
        for (int k = 0; k < 4; ++k)
            if (k != i) v *= (t - p[k]) / (p[i] - p[k]);
        w[i] = v;
    }
}

// The c > 0 with ps_fraction(c) = F.  F falls monotonically from 1 (c -> 0)
// to x_int / x_max (c -> inf), so bisection in log c brackets the root.
double c_for_fraction(double x_int, double x_max, double F) {
    double lo = std::log(1e-9 * x_max), hi = std::log(1e9 * x_max);
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (ps_fraction(std::exp(mid), x_int, x_max) > F) lo = mid; else hi = mid;
        if (hi - lo < 1e-15) break;
    }
    return std::exp(0.5 * (lo + hi));
}

// Integral over the cell [a1, b1] x [a2, b2] of max(K - (x1 + x2) / 2, 0): the
// pay-off is linear on the part of the cell below the line x1 + x2 = 2K, a
// convex polygon, so the integral is its area times the pay-off at its
// centroid (shoelace formulas, in coordinates relative to the cell corner).
double cell_integral_put_avg(double K, double a1, double b1, double a2, double b2) {
    const double w = b1 - a1, hgt = b2 - a2, cut = 2.0 * K - a1 - a2;
    const double px[4] = {0.0, w, w, 0.0}, py[4] = {0.0, 0.0, hgt, hgt};
    double qx[8], qy[8];
    int nq = 0;
    for (int i = 0; i < 4; ++i) {
        const int j = (i + 1) % 4;
        const double f0 = px[i] + py[i] - cut, f1 = px[j] + py[j] - cut;
        if (f0 <= 0.0) { qx[nq] = px[i]; qy[nq] = py[i]; ++nq; }
        if ((f0 < 0.0 && f1 > 0.0) || (f0 > 0.0 && f1 < 0.0)) {
            const double t = f0 / (f0 - f1);
            qx[nq] = px[i] + t * (px[j] - px[i]);
            qy[nq] = py[i] + t * (py[j] - py[i]);
            ++nq;
        }
    }
    double A = 0.0, mx = 0.0, my = 0.0;
    for (int i = 0; i < nq; ++i) {
        const int j = (i + 1) % nq;
        const double cr = qx[i] * qy[j] - qx[j] * qy[i];
        A += 0.5 * cr;
        mx += (qx[i] + qx[j]) * cr / 6.0;
        my += (qy[i] + qy[j]) * cr / 6.0;
    }
    if (A == 0.0) return 0.0;
    return A * (K - 0.5 * (a1 + a2)) - 0.5 * (mx + my);
}

}  // namespace

Cubic cubic_at(const std::vector<double>& nodes, double t) {
    const int n = int(nodes.size());
    int j = int(std::upper_bound(nodes.begin(), nodes.end(), t) - nodes.begin()) - 1;
    j = std::min(std::max(j, 0), n - 1);
    Cubic c;
    c.s = std::min(std::max(j - 1, 0), n - 4);
    lagrange4(&nodes[c.s], t, c.w);
    return c;
}

int largest_prime(int m) {
    int f = 1;
    for (int p = 2; m > 1; ++p)
        while (m % p == 0) { f = p; m /= p; }
    return f;
}

double ps_fraction(double c, double x_int, double x_max) {
    return 1.0 / (1.0 + (c / x_int) * std::asinh((x_max - x_int) / c));
}

bool build_ps_host(const lpide_ps_grid& g, const lpide_levy& lv, double K, PsHost& hp, std::string& err) {
    hp = PsHost();
    if (g.N_x < 8 || g.N_x > 4095) { err = "N_x must lie in [8, 4095]"; return false; }
    if (!(K > 0.0)) { err = "K must be positive"; return false; }
    const double x_int = g.x_int > 0.0 ? g.x_int : 2.5 * K;
    if (!(g.x_max > x_int)) { err = "x_max must exceed x_int (default 5K/2)"; return false; }
    if (!(g.fraction > 0.0 && g.fraction < 1.0)) { err = "fraction must lie in (0, 1)"; return false; }
    if (!(g.c >= 0.0)) { err = "c must be >= 0"; return false; }
    if (g.nz_per_nx < 1) { err = "nz_per_nx must be >= 1"; return false; }
    if (g.m1 < 1) { err = "m1 must be >= 1"; return false; }
    if (!(g.ell_cut > 0.0 && g.ell_cut < 1.0)) { err = "ell_cut must lie in (0, 1)"; return false; }
    if (!(g.zmax2_frac > 0.0 && g.zmax2_frac <= 1.0)) { err = "zmax2_frac must lie in (0, 1]"; return false; }
    if (g.gl_nodes < 2 || g.gl_nodes > 64) { err = "gl_nodes must lie in [2, 64]"; return false; }
    if (!std::isfinite(lv.r)) { err = "r must be finite"; return false; }
    const double sdet = lv.sigma_bs[0] * lv.sigma_bs[2] - lv.sigma_bs[1] * lv.sigma_bs[1];
    if (lv.sigma_bs[0] < 0.0 || lv.sigma_bs[2] < 0.0 || sdet < -1e-15) {
        err = "sigma_bs must be positive semi-definite";
        return false;
    }
    if (!make_nts(lv, hp.nts, err)) return false;

    // the grid: phi(xi) = c xi on [0, xi_int], x_int + c sinh(xi - xi_int) beyond
    hp.N_x = g.N_x;
    hp.n = g.N_x + 1;
    hp.K = K;
    hp.x_max = g.x_max;
    hp.x_int = x_int;
    hp.F = std::max(g.fraction, x_int / g.x_max);
    hp.c = g.c > 0.0 ? g.c : c_for_fraction(x_int, g.x_max, hp.F);
    const double xi_int = x_int / hp.c, xi_max = xi_int + std::asinh((g.x_max - x_int) / hp.c);
    hp.x.resize(hp.n);
    for (int m = 0; m < hp.n; ++m) {
        const double xi = xi_max * m / g.N_x;
        hp.x[m] = xi <= xi_int ? hp.c * xi : x_int + hp.c * std::sinh(xi - xi_int);
    }
    hp.x[hp.n - 1] = g.x_max;
    const int n = hp.n;

    // D: three-point first and second differences on the nonuniform grid.
    // At x = 0 both derivative terms vanish with their x factors; at x_max the
    // second derivative is dropped (v linear there) and the first difference
    // is the backward one.
    hp.D1c.assign(size_t(3) * n, 0.0);
    hp.D2c.assign(size_t(3) * n, 0.0);
    for (int m = 1; m < n - 1; ++m) {
        const double hm = hp.x[m] - hp.x[m - 1], hq = hp.x[m + 1] - hp.x[m];
        hp.D1c[3 * m + 0] = -hq / (hm * (hm + hq));
        hp.D1c[3 * m + 1] = (hq - hm) / (hm * hq);
        hp.D1c[3 * m + 2] = hm / (hq * (hm + hq));
        hp.D2c[3 * m + 0] = 2.0 / (hm * (hm + hq));
        hp.D2c[3 * m + 1] = -2.0 / (hm * hq);
        hp.D2c[3 * m + 2] = 2.0 / (hq * (hm + hq));
    }
    {
        const double hl = hp.x[n - 1] - hp.x[n - 2];
        hp.D1c[3 * (n - 1) + 0] = -1.0 / hl;
        hp.D1c[3 * (n - 1) + 1] = 1.0 / hl;
    }
    hp.A1.assign(size_t(3) * n, 0.0);
    hp.A2.assign(size_t(3) * n, 0.0);
    for (int m = 0; m < n; ++m)
        for (int t = 0; t < 3; ++t) {
            hp.A1[3 * m + t] = hp.x[m] * hp.D1c[3 * m + t];
            hp.A2[3 * m + t] = 0.5 * hp.x[m] * hp.x[m] * hp.D2c[3 * m + t];
        }

    hp.r = lv.r;
    for (int k = 0; k < 3; ++k) hp.sbs[k] = lv.sigma_bs[k];
    hp.M1 = g.m1;
    if (hp.nts.jumps) {
        // Sec. 4: N_z = 2 N_x, h_z = z_max^III / N_z, z_max^I = M1 h_z,
        // z_max^II = h_z ceil(zmax2_frac N_z - 1/2)
        hp.z_star = z_star(hp.nts, g.ell_cut);
        hp.N_z = g.nz_per_nx * g.N_x;
        hp.h_z = hp.z_star / hp.N_z;
        hp.M2 = int(std::ceil(g.zmax2_frac * hp.N_z - 0.5));
        integral_weights(hp.nts, hp.h_z, hp.N_z, hp.M1, hp.M2, g.gl_nodes, hp.omega);
        small_jump_cov(hp.nts, hp.M1 * hp.h_z, hp.S);
        drift_and_rate(hp.omega, hp.h_z, hp.N_z, lv.r, &hp.sum_omega, hp.kappa, &hp.r_omega);

        // y grids: N_y^- = ceil(-ln(x_1) / h_z) + N_y^*, N_y^+ = ceil(ln(x_max) / h_z) + N_y^*,
        // N_y^* the least shift that leaves no prime factor above 7 in #in
        const int bm = int(std::ceil(-std::log(hp.x[1]) / hp.h_z));
        const int bp = int(std::ceil(std::log(g.x_max) / hp.h_z));
        int star = 0;
        while (largest_prime(bm + bp + 2 * hp.N_z + 2 * star) > 7) ++star;
        hp.N_ystar = star;
        hp.N_ym = bm + star;
        hp.N_yp = bp + star;
        hp.n_in = hp.N_ym + hp.N_yp + 2 * hp.N_z;
        hp.n_out = hp.N_ym + hp.N_yp + 1;
        if (hp.n_out < 4) { err = "the y^out grid needs at least 4 nodes"; return false; }
        // T^in: v = 0 outside [0, x_max], so only the y^in nodes inside carry rows
        hp.tin.clear();
        for (int i = 0; i < hp.n_in; ++i) {
            const double y = std::exp((i - hp.N_z - hp.N_ym + 0.5) * hp.h_z);
            if (y > g.x_max) break;
            hp.tin.push_back(cubic_at(hp.x, y));
        }
        hp.n_nz = int(hp.tin.size());
        // T^out: cubic from y^out to x_1 .. x_max; linear extrapolation to x_0 = 0
        std::vector<double> yo(hp.n_out);
        for (int o = 0; o < hp.n_out; ++o) yo[o] = std::exp((o - hp.N_ym) * hp.h_z);
        hp.tout.assign(n, Cubic{});
        hp.tout[0].s = 0;
        hp.tout[0].w[0] = yo[1] / (yo[1] - yo[0]);
        hp.tout[0].w[1] = -yo[0] / (yo[1] - yo[0]);
        hp.tout[0].w[2] = hp.tout[0].w[3] = 0.0;
        for (int m = 1; m < n; ++m) hp.tout[m] = cubic_at(yo, hp.x[m]);
    } else {
        hp.kappa[0] = hp.kappa[1] = lv.r;
        hp.r_omega = lv.r;
    }
    for (int k = 0; k < 3; ++k) hp.a[k] = hp.sbs[k] + hp.S[k];
    return true;
}

void ps_sl_rows(const PsHost& hp, double factor, std::vector<Cubic>& rows) {
    rows.resize(hp.n);
    for (int m = 0; m < hp.n; ++m) rows[m] = cubic_at(hp.x, hp.x[m] * factor);
}

void ps_line_factors(const PsHost& hp, double aii, double rate, double c, std::vector<double>& fl,
                     std::vector<double>& bu, std::vector<double>& bc) {
    const int n = hp.n;
    std::vector<double> sub(n), dia(n), up(n);
    for (int m = 0; m < n; ++m) {
        sub[m] = -c * aii * hp.A2[3 * m + 0];
        dia[m] = 1.0 + c * rate - c * aii * hp.A2[3 * m + 1];
        up[m] = -c * aii * hp.A2[3 * m + 2];
    }
    thomas_factors(sub, dia, up, fl, bu, bc);
}

bool ps_initial(const PsHost& hp, const lpide_payoff& pay, std::vector<double>& v0, std::string& err) {
    const int n = hp.n;
    const double K = pay.K;
    if (pay.kind != LPIDE_PUT_AVG && pay.kind != LPIDE_PUT_1) {
        err = "the price-space plan takes the pay-offs LPIDE_PUT_AVG and LPIDE_PUT_1";
        return false;
    }
    // cell faces x_{m -/+ 1/2}; the outer faces mirror the inner ones about x_0 and x_max
    std::vector<double> f(n + 1);
    for (int m = 1; m < n; ++m) f[m] = 0.5 * (hp.x[m - 1] + hp.x[m]);
    f[0] = -f[1];
    f[n] = 2.0 * hp.x[n - 1] - f[n - 1];
    v0.assign(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double v;
            if (pay.kind == LPIDE_PUT_AVG) {
                v = std::max(K - 0.5 * (hp.x[i] + hp.x[j]), 0.0);
                if (pay.cell_avg && f[i] + f[j] < 2.0 * K && 2.0 * K < f[i + 1] + f[j + 1])
                    v = cell_integral_put_avg(K, f[i], f[i + 1], f[j], f[j + 1]) /
                        ((f[i + 1] - f[i]) * (f[j + 1] - f[j]));
            } else {
                v = std::max(K - hp.x[i], 0.0);
                if (pay.cell_avg && f[i] < K && K < f[i + 1]) v = 0.5 * (K - f[i]) * (K - f[i]) / (f[i + 1] - f[i]);
            }
            v0[size_t(i) * n + j] = v;
        }
    return true;
}

}  // namespace lpide
