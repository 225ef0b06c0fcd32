// CPU check of the library's host discretization (paper_2511_02700_amd/csrc/
// host_plan.cpp) built with AddressSanitizer and UBSan: the NTS density and its
// level set, the weights on the z-cells, the artificial diffusion, the folded
// correlation kernel, the cell-averaged initial grid for every pay-off, the
// line factors and their transposes, and the semi-Lagrangian weights with their
// transposed tables.  Arguments: alpha delta lambda eta1 eta2 rho11 rho12 rho22
// r n y_lo y_hi.  Prints the derived quantities as "key value" lines (the
// Python test compares them with the oracle's) and "OK" at the end.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "host_plan.hpp"

using namespace lpide;

int main(int argc, char** argv) {
    if (argc != 13) {
        std::fprintf(stderr, "usage: alpha delta lambda eta1 eta2 rho11 rho12 rho22 r n y_lo y_hi\n");
        return 2;
    }
    lpide_levy lv;
    std::memset(&lv, 0, sizeof lv);
    lv.alpha = std::atof(argv[1]);
    lv.delta = std::atof(argv[2]);
    lv.lambda = std::atof(argv[3]);
    lv.eta[0] = std::atof(argv[4]);
    lv.eta[1] = std::atof(argv[5]);
    lv.rho[0] = std::atof(argv[6]);
    lv.rho[1] = std::atof(argv[7]);
    lv.rho[2] = std::atof(argv[8]);
    lv.r = std::atof(argv[9]);
    lpide_grid g;
    std::memset(&g, 0, sizeof g);
    g.n = std::atoi(argv[10]);
    g.y_lo[0] = g.y_lo[1] = std::atof(argv[11]);
    g.y_hi[0] = g.y_hi[1] = std::atof(argv[12]);
    g.sl_order = 3;
    g.in_order = 3;
    g.m1 = 2;
    g.ell_cut = 1e-14;
    g.zmax2_frac = std::sqrt(0.1);
    g.gl_nodes = 8;
    HostPlan hp;
    std::string err;
    if (!build_host_plan(g, lv, hp, err)) {
        std::fprintf(stderr, "build_host_plan: %s\n", err.c_str());
        return 1;
    }
    std::printf("N_z %d\nM2 %d\nL_need %d\nz_star %.17g\nsum_omega %.17g\nr_omega %.17g\n", hp.N_z, hp.M2,
                hp.L_need, hp.z_star, hp.sum_omega, hp.r_omega);
    std::printf("kappa1 %.17g\nkappa2 %.17g\nS11 %.17g\nS12 %.17g\nS22 %.17g\n", hp.kappa[0], hp.kappa[1], hp.S[0],
                hp.S[1], hp.S[2]);
    double ksum = 0.0;
    for (double v : hp.kern) ksum += v;
    std::printf("kernel_sum %.17g\n", ksum);
    const int n = hp.n;
    for (int kind = LPIDE_PUT_AVG; kind <= LPIDE_SPREAD; ++kind) {
        lpide_payoff pay;
        std::memset(&pay, 0, sizeof pay);
        pay.kind = kind;
        pay.K = 100.0;
        pay.T = 1.0;
        pay.cell_avg = 1;
        std::vector<double> v0;
        if (!initial_values(hp, pay, v0, err)) {
            std::fprintf(stderr, "initial_values(%d): %s\n", kind, err.c_str());
            return 1;
        }
        double s = 0.0;
        for (double v : v0) s += v;
        std::printf("v0_sum_%d %.17g\n", kind, s);
    }
    for (int ax = 0; ax < 2; ++ax) {
        std::vector<double> fl, bu, bc, flt, but, bct;
        line_factors(n, hp.h, hp.a[2 * ax], hp.r_omega, 0.5 / 64, fl, bu, bc);
        line_factors_T(n, hp.h, hp.a[2 * ax], hp.r_omega, 0.5 / 64, flt, but, bct);
        std::vector<int32_t> st, idx;
        std::vector<double> w, wt, dw;
        const double shift = hp.kappa[ax] * (1.0 / 64) / hp.h;
        sl_weights(n, shift, 3, st, w);
        sl_dweights(n, shift, 3, dw);
        const int width = sl_transpose(n, 3, st, w, idx, wt);
        double wsum = 0.0;
        for (double v : wt) wsum += v;
        std::printf("sl_transpose_width_%d %d\nsl_transpose_sum_%d %.17g\n", ax, width, ax, wsum);
    }
    std::printf("OK\n");
    return 0;
}
