// Host-side discretization: Levy density, z-grid sizes, quadrature weights,
// artificial diffusion, drift and kill rate (Sec. 3.1 and the Sec. 4 settings),
// the folded correlation kernel, cell-averaged pay-off (Sec. 3.2.3), line-solve
// factors and semi-Lagrangian weights (Sec. 3.3).  FP64 throughout.
#include "host_plan.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <functional>
#include <limits>
#include <thread>

namespace lpide {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

// Neumaier-compensated accumulator.
struct Sum {
    double s = 0, c = 0;
    void add(double x) {
        double t = s + x;
        if (std::fabs(s) >= std::fabs(x)) c += (s - t) + x; else c += (x - t) + s;
        s = t;
    }
    double value() const { return s + c; }
};

// log K_nu(x) for x > 0: libstdc++'s cyl_bessel_k where it does not underflow,
// else the large-argument expansion K_nu(x) ~ sqrt(pi/2x) e^-x sum_k a_k x^-k,
// a_k = a_{k-1} (4 nu^2 - (2k-1)^2) / (8k)  (accurate to rounding for x >= 500).
double log_bessel_k(double nu, double x) {
    if (x < 500.0) return std::log(std::cyl_bessel_k(nu, x));
    double mu = 4.0 * nu * nu, term = 1.0, sum = 1.0;
    for (int k = 1; k < 12; ++k) {
        term *= (mu - (2.0 * k - 1) * (2.0 * k - 1)) / (8.0 * k * x);
        sum += term;
        if (std::fabs(term) < 1e-18) break;
    }
    return -x + 0.5 * std::log(kPi / (2.0 * x)) + std::log(sum);
}

// Gauss-Legendre nodes/weights on [-1, 1] (Newton iteration on P_n).
void gauss_legendre(int m, std::vector<double>& x, std::vector<double>& w) {
    x.assign(m, 0.0);
    w.assign(m, 0.0);
    for (int i = 0; i < (m + 1) / 2; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (m + 0.5));
        double pp = 0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= m; ++k) {
                double p2 = ((2.0 * k - 1) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (m == 1) { p1 = z; p0 = 1.0; }
            pp = m * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / pp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // recompute derivative at the converged node
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= m; ++k) {
            double p2 = ((2.0 * k - 1) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        pp = m * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        x[m - 1 - i] = z;
        w[i] = w[m - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
    if (m % 2 == 1) x[m / 2] = 0.0;
}

// Run fn(b, e) over [0, count) on up to 16 host threads, handing out blocks of
// `grain` items from a shared counter (the items may differ much in cost).
void parallel_for(int64_t count, const std::function<void(int64_t, int64_t)>& fn, int64_t grain = 1) {
    unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const int64_t nblk = (count + grain - 1) / grain;
    const int64_t nt = std::min<int64_t>(hw, nblk);
    if (nt <= 1) { fn(0, count); return; }
    std::atomic<int64_t> next{0};
    auto work = [&] {
        for (;;) {
            const int64_t k = next.fetch_add(1);
            if (k >= nblk) break;
            fn(k * grain, std::min(count, (k + 1) * grain));
        }
    };
    std::vector<std::thread> th;
    for (int64_t t = 0; t < nt; ++t) th.emplace_back(work);
    for (auto& t : th) t.join();
}

double density(const Nts& p, double z1, double z2) {
    double v = log_density(p, z1, z2);
    return v == -std::numeric_limits<double>::infinity() ? 0.0 : std::exp(v);
}

// Lagrange basis through integer nodes s..s+P at x.
void lagrange(int s, int P, double x, double* w) {
    for (int i = 0; i <= P; ++i) {
        double v = 1.0;
        for (int j = 0; j <= P; ++j)
            if (j != i) v *= (x - (s + j)) / double(i - j);
        w[i] = v;
    }
}

}  // namespace

bool make_nts(const lpide_levy& lv, Nts& p, std::string& err) {
    p = Nts();
    if (!lv.no_jumps) {
        if (!(lv.alpha >= 0.0 && lv.alpha < 1.0)) { err = "alpha must lie in [0, 1)"; return false; }
        if (!(lv.delta > 0.0) || !(lv.lambda > 0.0)) { err = "delta and lambda must be positive"; return false; }
        double det = lv.rho[0] * lv.rho[2] - lv.rho[1] * lv.rho[1];
        if (!(lv.rho[0] > 0.0) || !(det > 0.0)) { err = "rho must be positive definite"; return false; }
        if (!std::isfinite(lv.eta[0]) || !std::isfinite(lv.eta[1])) { err = "eta must be finite"; return false; }
        for (int i = 0; i < 2; ++i) {
            double rii = i == 0 ? lv.rho[0] : lv.rho[2];
            if (!(lv.lambda - lv.eta[i] - 0.5 * rii > 0.0)) {
                err = "lambda - eta_i - rho_ii/2 must be positive (exponential moment)";
                return false;
            }
        }
        p.jumps = true;
        p.alpha = lv.alpha;
        p.delta = lv.delta;
        p.lambda = lv.lambda;
        p.eta[0] = lv.eta[0];
        p.eta[1] = lv.eta[1];
        for (int k = 0; k < 3; ++k) p.rho[k] = lv.rho[k];
        p.det = det;
        p.ri[0] = lv.rho[2] / det;
        p.ri[1] = -lv.rho[1] / det;
        p.ri[2] = lv.rho[0] / det;
        p.ri_eta[0] = p.ri[0] * p.eta[0] + p.ri[1] * p.eta[1];
        p.ri_eta[1] = p.ri[1] * p.eta[0] + p.ri[2] * p.eta[1];
        double en2 = p.eta[0] * p.ri_eta[0] + p.eta[1] * p.ri_eta[1];
        p.c1 = std::sqrt(en2 + 2.0 * p.lambda);
        p.nu = 1.0 + p.alpha;
        p.logpref = std::log(p.delta / kPi) + p.nu * std::log(p.c1) - 0.5 * std::log(det);
    }
    return true;
}

double log_density(const Nts& p, double z1, double z2) {
    double q2 = p.ri[0] * z1 * z1 + 2.0 * p.ri[1] * z1 * z2 + p.ri[2] * z2 * z2;
    double q = std::sqrt(q2);
    double x = p.c1 * q;
    if (!(x > 0.0)) return std::numeric_limits<double>::infinity();
    return p.logpref + log_bessel_k(p.nu, x) - p.nu * std::log(q) + p.ri_eta[0] * z1 + p.ri_eta[1] * z2;
}

// Radius of the level set along a unit direction: log l(r u) is strictly
// decreasing in r (its derivative is at most -(c1 - ||eta||_rho) ||u||_rho), so a
// bracket by doubling followed by bisection finds the unique crossing.
static double ray_radius(const Nts& p, double u1, double u2, double logcut) {
    auto f = [&](double r) { return log_density(p, r * u1, r * u2) - logcut; };
    double lo = 0.0, hi = 1e-4;
    while (f(hi) > 0.0) {
        lo = hi;
        hi *= 2.0;
        if (hi > 1e7) return hi;
    }
    // bisection: the bracket [hi/2, hi] shrinks to rounding in about 55 halvings
    for (int it = 0; it < 200 && hi - lo > 4e-16 * hi; ++it) {
        double mid = 0.5 * (lo + hi);
        if (f(mid) > 0.0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

double z_star(const Nts& p, double cut) {
    const double logcut = std::log(cut);
    auto g = [&](double phi) {
        double c = std::cos(phi), s = std::sin(phi);
        return ray_radius(p, c, s, logcut) * std::max(std::fabs(c), std::fabs(s));
    };
    const int NA = 2048;
    std::vector<double> vals(NA);
    parallel_for(NA, [&](int64_t b, int64_t e) {
        for (int64_t k = b; k < e; ++k) vals[k] = g(2.0 * kPi * k / NA);
    });
    int kb = int(std::max_element(vals.begin(), vals.end()) - vals.begin());
    double best = vals[kb];
    // golden-section maximisation on the bracket of the best ray
    double a = 2.0 * kPi * (kb - 1) / NA, b = 2.0 * kPi * (kb + 1) / NA;
    const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
    double x1 = b - gr * (b - a), x2 = a + gr * (b - a), f1 = g(x1), f2 = g(x2);
    for (int it = 0; it < 80 && b - a > 1e-13; ++it) {
        if (f1 < f2) { a = x1; x1 = x2; f1 = f2; x2 = a + gr * (b - a); f2 = g(x2); }
        else { b = x2; x2 = x1; f2 = f1; x1 = b - gr * (b - a); f1 = g(x1); }
    }
    return std::max(best, std::max(f1, f2));
}

// Artificial diffusion S = int over [-M1 h, M1 h]^2 of z z^T l(z) dz (Sec. 3.1):
// polar coordinates per octant, Gauss-Legendre in the angle, tanh-sinh in the
// radius (the radial integrand r^3 l(r u) ~ r^(1 - 2 alpha) at the origin).
void small_jump_cov(const Nts& p, double half, double S[3]) {
    std::vector<double> gx, gw;
    gauss_legendre(48, gx, gw);
    // tanh-sinh nodes on [0, 1]: x = 1/(1 + e^{-pi sinh t}), dx = pi cosh t e^{-pi sinh t}/(1+e^{-pi sinh t})^2
    const double hts = 1.0 / 32.0;
    std::vector<double> tx, tw;
    for (int k = -160; k <= 160; ++k) {
        double t = k * hts, s = kPi * std::sinh(t);
        double e = std::exp(-s);
        double x = 1.0 / (1.0 + e);
        double w = hts * kPi * std::cosh(t) * e / ((1.0 + e) * (1.0 + e));
        if (!(x > 1e-60) || !(w > 0.0) || !std::isfinite(w)) continue;
        tx.push_back(x);
        tw.push_back(w);
    }
    // one radial integral per (octant, angle node), in parallel; summed in order
    const int na = int(gx.size());
    std::vector<double> Iv(size_t(8) * na), U1(Iv.size()), U2(Iv.size());
    parallel_for(8 * na, [&](int64_t b, int64_t e) {
        for (int64_t q = b; q < e; ++q) {
            const int oct = int(q / na), i = int(q % na);
            double a = oct * kPi / 4.0, bb = (oct + 1) * kPi / 4.0;
            double phi = 0.5 * (bb - a) * gx[i] + 0.5 * (a + bb);
            double wphi = 0.5 * (bb - a) * gw[i];
            double u1 = std::cos(phi), u2 = std::sin(phi);
            double R = half / std::max(std::fabs(u1), std::fabs(u2));
            Sum rad;
            for (size_t k = 0; k < tx.size(); ++k) {
                double r = R * tx[k];
                double ld = log_density(p, r * u1, r * u2);
                if (ld == -std::numeric_limits<double>::infinity()) continue;
                rad.add(tw[k] * R * std::exp(3.0 * std::log(r) + ld));
            }
            Iv[q] = rad.value() * wphi;
            U1[q] = u1;
            U2[q] = u2;
        }
    }, 8);
    Sum s11, s12, s22;
    for (size_t q = 0; q < Iv.size(); ++q) {
        s11.add(U1[q] * U1[q] * Iv[q]);
        s12.add(U1[q] * U2[q] * Iv[q]);
        s22.add(U2[q] * U2[q] * Iv[q]);
    }
    S[0] = s11.value();
    S[1] = s12.value();
    S[2] = s22.value();
}

void integral_weights(const Nts& p, double h, int N_z, int M1, int M2, int ng, std::vector<double>& omega) {
    const int N = N_z, W2 = 2 * N;
    omega.assign(size_t(W2) * W2, 0.0);
    std::vector<double> gx, gw;
    gauss_legendre(ng, gx, gw);
    parallel_for(W2, [&](int64_t b, int64_t e) {
        for (int64_t a = b; a < e; ++a) {
            int l1 = int(a) - N;
            double c1 = (l1 + 0.5) * h;
            for (int bb = 0; bb < W2; ++bb) {
                int l2 = bb - N;
                double c2 = (l2 + 0.5) * h;
                double cn = std::max(std::fabs(l1 + 0.5), std::fabs(l2 + 0.5));
                double w;
                if (cn <= M1) {
                    w = 0.0;                                  // R_I
                } else if (cn <= M2) {                        // R_II: ||z_l||^-2 int_cell ||z||^2 l
                    Sum acc;
                    for (int i = 0; i < ng; ++i) {
                        double z1 = c1 + 0.5 * h * gx[i];
                        for (int j = 0; j < ng; ++j) {
                            double z2 = c2 + 0.5 * h * gx[j];
                            acc.add(gw[i] * gw[j] * (z1 * z1 + z2 * z2) * density(p, z1, z2));
                        }
                    }
                    w = acc.value() * 0.25 * h * h / (c1 * c1 + c2 * c2);
                } else {                                      // R_III: midpoint
                    w = density(p, c1, c2) * h * h;
                }
                omega[size_t(a) * W2 + bb] = w;
            }
        }
    });
}

void drift_and_rate(const std::vector<double>& omega, double h, int N_z, double r, double* sum_omega,
                    double kappa[2], double* r_omega) {
    const int N = N_z, W2 = 2 * N;
    Sum so, k1, k2;
    for (int a = 0; a < W2; ++a) {
        double e1 = std::expm1((a - N + 0.5) * h);
        for (int bb = 0; bb < W2; ++bb) {
            double w = omega[size_t(a) * W2 + bb];
            double e2 = std::expm1((bb - N + 0.5) * h);
            so.add(w);
            k1.add(w * e1);
            k2.add(w * e2);
        }
    }
    *sum_omega = so.value();
    kappa[0] = r - k1.value();
    kappa[1] = r - k2.value();
    *r_omega = r + *sum_omega;
}

bool build_host_plan(const lpide_grid& g, const lpide_levy& lv, HostPlan& hp, std::string& err) {
    hp = HostPlan();
    if (g.n < 8 || g.n > 4096) { err = "n must lie in [8, 4096]"; return false; }
    double w0 = g.y_hi[0] - g.y_lo[0], w1 = g.y_hi[1] - g.y_lo[1];
    if (!(w0 > 0.0) || !(w1 > 0.0) || std::fabs(w0 - w1) > 1e-12 * std::max(1.0, w0)) {
        err = "both axes need the same positive width y_hi - y_lo";
        return false;
    }
    if ((g.sl_order != 1 && g.sl_order != 3) || (g.in_order != 1 && g.in_order != 3)) {
        err = "sl_order and in_order must be 1 or 3";
        return false;
    }
    if (g.m1 < 1) { err = "m1 must be >= 1"; return false; }
    if (!(g.ell_cut > 0.0 && g.ell_cut < 1.0)) { err = "ell_cut must lie in (0, 1)"; return false; }
    if (!(g.zmax2_frac > 0.0 && g.zmax2_frac <= 1.0)) { err = "zmax2_frac must lie in (0, 1]"; return false; }
    if (g.gl_nodes < 2 || g.gl_nodes > 64) { err = "gl_nodes must lie in [2, 64]"; return false; }
    if (!std::isfinite(lv.r)) { err = "r must be finite"; return false; }
    double sdet = lv.sigma_bs[0] * lv.sigma_bs[2] - lv.sigma_bs[1] * lv.sigma_bs[1];
    if (lv.sigma_bs[0] < 0.0 || lv.sigma_bs[2] < 0.0 || sdet < -1e-15) {
        err = "sigma_bs must be positive semi-definite";
        return false;
    }
    if (!make_nts(lv, hp.nts, err)) return false;

    hp.n = g.n;
    hp.y_lo[0] = g.y_lo[0];
    hp.y_lo[1] = g.y_lo[1];
    hp.h = w0 / (g.n - 1);
    hp.sl_order = g.sl_order;
    hp.in_order = g.in_order;
    hp.r = lv.r;
    for (int k = 0; k < 3; ++k) hp.sbs[k] = lv.sigma_bs[k];
    hp.M1 = g.m1;
    const double h = hp.h;

    if (hp.nts.jumps) {
        hp.z_star = z_star(hp.nts, g.ell_cut);
        hp.N_z = g.nz_fixed > 0 ? g.nz_fixed : int(std::ceil(hp.z_star / h));
        hp.M2 = int(std::ceil(g.zmax2_frac * hp.N_z - 0.5));
        if (hp.N_z < 1) hp.N_z = 1;
        integral_weights(hp.nts, h, hp.N_z, hp.M1, hp.M2, g.gl_nodes, hp.omega);
        small_jump_cov(hp.nts, hp.M1 * h, hp.S);
        drift_and_rate(hp.omega, h, hp.N_z, lv.r, &hp.sum_omega, hp.kappa, &hp.r_omega);
    } else {
        hp.kappa[0] = hp.kappa[1] = lv.r;
        hp.r_omega = lv.r;
    }
    for (int k = 0; k < 3; ++k) hp.a[k] = hp.sbs[k] + hp.S[k];

    // folded kernel K_d = sum_{l + j = d} omega_l s_j1 s_j2, s = T^in taps at +h/2
    if (hp.nts.jumps) {
        const int P = hp.in_order;
        const int jlo = -(P - 1) / 2, jhi = (P + 1) / 2;
        double s[4];
        lagrange(jlo, P, 0.5, s);   // nodes jlo..jhi evaluated at +1/2
        const int N = hp.N_z, W2 = 2 * N;
        hp.dlo = -N + jlo;
        hp.dhi = N - 1 + jhi;
        const int KW = hp.dhi - hp.dlo + 1;
        hp.kern.assign(size_t(KW) * KW, 0.0);
        std::vector<double> tmp(size_t(KW) * W2, 0.0);   // axis-1 convolution first
        for (int a = 0; a < W2; ++a)
            for (int j = 0; j <= P; ++j) {
                int d1 = a - N + jlo + j - hp.dlo;
                for (int bb = 0; bb < W2; ++bb) tmp[size_t(d1) * W2 + bb] += s[j] * hp.omega[size_t(a) * W2 + bb];
            }
        for (int d1 = 0; d1 < KW; ++d1)
            for (int bb = 0; bb < W2; ++bb)
                for (int j = 0; j <= P; ++j) {
                    int d2 = bb - N + jlo + j - hp.dlo;
                    hp.kern[size_t(d1) * KW + d2] += s[j] * tmp[size_t(d1) * W2 + bb];
                }
        hp.L_need = hp.n + std::max(-hp.dlo, hp.dhi);
        hp.L = fft_size_at_least(hp.L_need);
        if (hp.L == 0) { err = "FFT side above 4096: n + N_z + 1 must not exceed 4096"; return false; }
    }
    return true;
}

bool fft_size_supported(int L) {
    for (int v : kFftSizes)
        if (v == L) return true;
    return false;
}

int fft_size_at_least(int need) {
    for (int v : kFftAutoSizes)
        if (v >= need) return v;
    return 0;
}

// ---------------------------------------------------------------------------
// Pay-off and cell averaging (Sec. 3.2.3, Sec. 4)
// ---------------------------------------------------------------------------
namespace {

// g with pay-off = K max(g, 0) in the variables y_i = ln(S_i/K).
double payoff_g(int kind, double y1, double y2) {
    switch (kind) {
        case LPIDE_PUT_AVG: return 1.0 - 0.5 * (std::exp(y1) + std::exp(y2));
        case LPIDE_CALL_AVG: return 0.5 * (std::exp(y1) + std::exp(y2)) - 1.0;
        case LPIDE_PUT_1: return 1.0 - std::exp(y1);
        case LPIDE_CALL_1: return std::exp(y1) - 1.0;
        case LPIDE_SPREAD: return std::exp(y1) - std::exp(y2) - 1.0;
        default: return std::exp(y1) - std::exp(y2);   // exchange
    }
}

// int_{a2}^{b2} max(g(y1, y2), 0) dy2 in closed form.
double inner_closed(int kind, double y1, double a2, double b2) {
    double e1 = std::exp(y1);
    switch (kind) {
        case LPIDE_PUT_AVG: {           // positive for e^{y2} < 2 - e^{y1}
            double c = 1.0 - 0.5 * e1;
            if (!(c > 0.0)) return 0.0;
            double u = std::min(b2, std::log(2.0 * c));
            if (!(u > a2)) return 0.0;
            return c * (u - a2) - 0.5 * (std::exp(u) - std::exp(a2));
        }
        case LPIDE_CALL_AVG: {          // positive for e^{y2} > 2 - e^{y1}
            double c = 1.0 - 0.5 * e1;
            double u = c > 0.0 ? std::max(a2, std::log(2.0 * c)) : a2;
            if (!(b2 > u)) return 0.0;
            return 0.5 * (std::exp(b2) - std::exp(u)) - c * (b2 - u);
        }
        case LPIDE_PUT_1: return std::max(1.0 - e1, 0.0) * (b2 - a2);
        case LPIDE_CALL_1: return std::max(e1 - 1.0, 0.0) * (b2 - a2);
        case LPIDE_SPREAD: {            // positive for e^{y2} < e^{y1} - 1
            const double c = e1 - 1.0;
            if (!(c > 0.0)) return 0.0;
            const double u = std::min(b2, std::log(c));
            if (!(u > a2)) return 0.0;
            return c * (u - a2) - (std::exp(u) - std::exp(a2));
        }
        default: {                      // exchange: positive for y2 < y1
            double u = std::min(b2, y1);
            if (!(u > a2)) return 0.0;
            return e1 * (u - a2) - (std::exp(u) - std::exp(a2));
        }
    }
}

// y1 values where the kink curve {g = 0} crosses y2 = t.
void kink_crossings(int kind, double t, std::vector<double>& out) {
    switch (kind) {
        case LPIDE_PUT_AVG:
        case LPIDE_CALL_AVG: {
            double v = 2.0 - std::exp(t);
            if (v > 0.0) out.push_back(std::log(v));
            break;
        }
        case LPIDE_PUT_1:
        case LPIDE_CALL_1: out.push_back(0.0); break;
        case LPIDE_SPREAD: out.push_back(std::log1p(std::exp(t))); break;
        default: out.push_back(t); break;
    }
}

}  // namespace

bool initial_values(const HostPlan& hp, const lpide_payoff& pay, std::vector<double>& v0, std::string& err) {
    if (pay.kind < LPIDE_PUT_AVG || pay.kind > LPIDE_SPREAD) { err = "unknown pay-off kind"; return false; }
    if (!(pay.K > 0.0) || !(pay.T > 0.0)) { err = "K and T must be positive"; return false; }
    const int n = hp.n;
    const double h = hp.h, hh = 0.5 * h;
    v0.assign(size_t(n) * n, 0.0);
    std::vector<double> gx, gw;
    gauss_legendre(24, gx, gw);
    parallel_for(n, [&](int64_t b, int64_t e) {
        std::vector<double> bps;
        for (int64_t j1 = b; j1 < e; ++j1) {
            double y1 = hp.y_lo[0] + j1 * h;
            for (int j2 = 0; j2 < n; ++j2) {
                double y2 = hp.y_lo[1] + j2 * h;
                double val = std::max(payoff_g(pay.kind, y1, y2), 0.0);
                if (pay.cell_avg) {
                    double gmin = 1e300, gmax = -1e300;
                    for (int s1 = -1; s1 <= 1; s1 += 2)
                        for (int s2 = -1; s2 <= 1; s2 += 2) {
                            double gv = payoff_g(pay.kind, y1 + s1 * hh, y2 + s2 * hh);
                            gmin = std::min(gmin, gv);
                            gmax = std::max(gmax, gv);
                        }
                    if (gmin <= 0.0 && gmax >= 0.0) {
                        double a1 = y1 - hh, b1 = y1 + hh, a2 = y2 - hh, b2 = y2 + hh;
                        bps.clear();
                        bps.push_back(a1);
                        kink_crossings(pay.kind, a2, bps);
                        kink_crossings(pay.kind, b2, bps);
                        bps.push_back(b1);
                        std::sort(bps.begin(), bps.end());
                        Sum acc;
                        for (size_t k = 0; k + 1 < bps.size(); ++k) {
                            double s = std::max(a1, bps[k]), t = std::min(b1, bps[k + 1]);
                            if (!(t > s)) continue;
                            for (size_t q = 0; q < gx.size(); ++q) {
                                double yy = 0.5 * (t - s) * gx[q] + 0.5 * (s + t);
                                acc.add(0.5 * (t - s) * gw[q] * inner_closed(pay.kind, yy, a2, b2));
                            }
                        }
                        val = acc.value() / (h * h);
                    }
                }
                v0[size_t(j1) * n + j2] = pay.K * val;
            }
        }
    });
    return true;
}

// Thomas factors of the tridiagonal matrix with rows (sub[j], dia[j], up[j]),
// each followed by kLinePad zeros.
void thomas_factors(const std::vector<double>& sub, const std::vector<double>& dia, const std::vector<double>& up,
                    std::vector<double>& fl, std::vector<double>& bu, std::vector<double>& bc) {
    const int n = int(dia.size());
    fl.assign(n, 0.0);
    bu.assign(n, 0.0);
    bc.assign(n, 0.0);
    std::vector<double> d(n);
    for (int j = 0; j < n; ++j) {
        if (j == 0) {
            d[j] = dia[j];
        } else {
            double l = sub[j] / d[j - 1];
            fl[j] = -l;
            d[j] = dia[j] - l * up[j - 1];
        }
    }
    for (int j = 0; j < n; ++j) {
        bu[j] = 1.0 / d[j];
        bc[j] = -up[j] / d[j];
    }
    fl.resize(n + kLinePad, 0.0);
    bu.resize(n + kLinePad, 0.0);
    bc.resize(n + kLinePad, 0.0);
}

namespace {

// Rows of T = I - c A with A = 1/2 aii [(v+ - 2v + v-)/h^2 - (v+ - v-)/(2h)] - r_omega/2 v
// on interior rows and A = -r_omega/2 v on the two boundary rows.
void line_rows_of(int n, double h, double aii, double r_omega, double c, std::vector<double>& sub,
                  std::vector<double>& dia, std::vector<double>& up) {
    const double lo_in = -c * 0.5 * aii * (1.0 / (h * h) + 0.5 / h);
    const double up_in = -c * 0.5 * aii * (1.0 / (h * h) - 0.5 / h);
    const double di_in = 1.0 + c * (aii / (h * h) + 0.5 * r_omega);
    const double di_bd = 1.0 + c * 0.5 * r_omega;
    sub.assign(n, 0.0);
    dia.assign(n, 0.0);
    up.assign(n, 0.0);
    for (int j = 0; j < n; ++j) {
        const bool in = j > 0 && j < n - 1;
        sub[j] = in ? lo_in : 0.0;
        dia[j] = in ? di_in : di_bd;
        up[j] = in ? up_in : 0.0;
    }
}

}  // namespace

void line_factors(int n, double h, double aii, double r_omega, double c,
                  std::vector<double>& fl, std::vector<double>& bu, std::vector<double>& bc) {
    std::vector<double> sub, dia, up;
    line_rows_of(n, h, aii, r_omega, c, sub, dia, up);
    thomas_factors(sub, dia, up, fl, bu, bc);
}

void line_factors_T(int n, double h, double aii, double r_omega, double c,
                    std::vector<double>& fl, std::vector<double>& bu, std::vector<double>& bc) {
    std::vector<double> sub, dia, up;
    line_rows_of(n, h, aii, r_omega, c, sub, dia, up);
    // transpose: row j of T^T has sub = up[j-1], super = sub[j+1]
    std::vector<double> ts(n, 0.0), tu(n, 0.0);
    for (int j = 0; j < n; ++j) {
        ts[j] = j > 0 ? up[j - 1] : 0.0;
        tu[j] = j < n - 1 ? sub[j + 1] : 0.0;
    }
    thomas_factors(ts, dia, tu, fl, bu, bc);
}

void sl_dweights(int n, double shift, int P, std::vector<double>& dw) {
    dw.assign(size_t(n) * (P + 1), 0.0);
    for (int j = 0; j < n; ++j) {
        const double xi = j + shift;
        int s = int(std::floor(xi)) - (P - 1) / 2;
        s = std::min(std::max(s, 0), n - 1 - P);
        // d/dx of the Lagrange basis through s..s+P: sum over the dropped factor
        for (int i = 0; i <= P; ++i) {
            double acc = 0.0;
            for (int k = 0; k <= P; ++k) {
                if (k == i) continue;
                double v = 1.0 / double(i - k);
                for (int q = 0; q <= P; ++q)
                    if (q != i && q != k) v *= (xi - (s + q)) / double(i - q);
                acc += v;
            }
            dw[size_t(j) * (P + 1) + i] = acc;
        }
    }
}

int sl_transpose(int n, int P, const std::vector<int32_t>& start, const std::vector<double>& w,
                 std::vector<int32_t>& idx, std::vector<double>& wt) {
    std::vector<std::vector<std::pair<int, double>>> rows(n);
    for (int j = 0; j < n; ++j)
        for (int t = 0; t <= P; ++t) rows[start[j] + t].push_back({j, w[size_t(j) * (P + 1) + t]});
    int width = 1;
    for (auto& r : rows) width = std::max<int>(width, int(r.size()));
    idx.assign(size_t(n) * width, 0);
    wt.assign(size_t(n) * width, 0.0);
    for (int m = 0; m < n; ++m)
        for (size_t q = 0; q < rows[m].size(); ++q) {
            idx[size_t(m) * width + q] = rows[m][q].first;
            wt[size_t(m) * width + q] = rows[m][q].second;
        }
    return width;
}

// Stencil starts and Lagrange weights of the departure points j + shift:
// start[j] = clamp(floor(j + shift) - (P - 1) / 2, 0, n - 1 - P).
void sl_weights(int n, double shift, int P, std::vector<int32_t>& start, std::vector<double>& w) {
    start.assign(n, 0);
    w.assign(size_t(n) * (P + 1), 0.0);
    for (int j = 0; j < n; ++j) {
        double xi = j + shift;
        int s = int(std::floor(xi)) - (P - 1) / 2;
        s = std::min(std::max(s, 0), n - 1 - P);
        start[j] = s;
        lagrange(s, P, xi, &w[size_t(j) * (P + 1)]);
    }
}

std::vector<std::pair<double, double>> step_list(double theta, double T, int N_t, bool damping) {
    std::vector<std::pair<double, double>> s;
    double dt = T / N_t;
    if (damping) {
        for (int k = 0; k < 4; ++k) s.emplace_back(1.0, 0.25 * dt);
        for (int k = 1; k < N_t; ++k) s.emplace_back(theta, dt);
    } else {
        for (int k = 0; k < N_t; ++k) s.emplace_back(theta, dt);
    }
    return s;
}

}  // namespace lpide
