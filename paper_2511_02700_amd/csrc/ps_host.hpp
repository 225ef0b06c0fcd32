// Host-side discretization of the paper's own price-space scheme (Sec. 3.2,
// Sec. 3.3 and the Sec. 4 settings): the graded grid x in each price axis, the
// nonuniform difference operator D, the log-uniform y grids of the summation
// operator with the interpolations T^in and T^out, the semi-Lagrangian
// weights and the cell-averaged pay-off.  FP64, once per plan, on the CPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "host_plan.hpp"
#include "lpide.h"

namespace lpide {

// Cubic Lagrange interpolation from ascending nodes to one target: the stencil
// of the four nearest nodes in index order (start s = clamp(j - 1, 0, n - 4)
// with nodes[j] <= t < nodes[j + 1]), so targets beyond either end are
// extrapolated by the end polynomial.
struct Cubic {
    int32_t s;
    double w[4];
};
Cubic cubic_at(const std::vector<double>& nodes, double t);

struct PsHost {
    // grid (Sec. 4: x_m = phi(xi_max m / N_x), uniform on [0, x_int], sinh-graded beyond)
    int N_x = 0, n = 0;
    double K = 0, x_max = 0, x_int = 0, c = 0, F = 0;
    std::vector<double> x;
    // model and integral part (Sec. 3.1 with h_z = z_max^III / N_z)
    double r = 0, sbs[3] = {0, 0, 0};
    Nts nts;
    int N_z = 0, M1 = 2, M2 = 0;
    double z_star = 0, h_z = 0, sum_omega = 0, kappa[2] = {0, 0}, r_omega = 0, S[3] = {0, 0, 0}, a[3] = {0, 0, 0};
    std::vector<double> omega;          // (2 N_z)^2, omega[(l1 + N_z) * 2 N_z + (l2 + N_z)]
    // y grids (Sec. 3.2.2, Sec. 4): y^out_o = e^{(o - N_y^-) h_z}, o < n_out;
    // y^in_i = e^{(i - N_z - N_y^- + 1/2) h_z}, i < n_in; the first n_nz of them lie in [0, x_max]
    int N_ym = 0, N_yp = 0, N_ystar = 0, n_in = 0, n_out = 0, n_nz = 0;
    std::vector<Cubic> tin;             // n_nz rows of T^in (per axis; both axes alike)
    std::vector<Cubic> tout;            // n rows of T^out; row 0 is the linear extrapolation to x = 0
    // D (Sec. 3.2.1) per node m: A1[3m + t] = x_m d1_{m, m-1+t}, A2[3m + t] = x_m^2 d2_{m, m-1+t} / 2,
    // and the difference coefficients themselves, D1c[3m + t] = d1_{m, m-1+t}, D2c[3m + t] = d2_{m, m-1+t}
    std::vector<double> A1, A2, D1c, D2c;
};

// Limit fraction F of the grid points in [0, x_int] for the constant c (Sec. 4).
double ps_fraction(double c, double x_int, double x_max);

// The grid, the integral discretization, the y grids and every table above.
bool build_ps_host(const lpide_ps_grid& g, const lpide_levy& lv, double K, PsHost& hp, std::string& err);

// Semi-Lagrangian rows of one axis: the departure points x_m e^{kappa_i dt} (Sec. 3.3).
void ps_sl_rows(const PsHost& hp, double factor, std::vector<Cubic>& rows);

// Thomas factors of T_i = I - c (a_ii x^2 D2 / 2 - rate) along one axis (the
// preconditioner of the fixed-point iteration; the plan puts the whole kill
// rate r_omega into T_1 and none into T_2, so that on smooth grids T_1 T_2
// damps like the paper's I - c (D - r_omega)).
void ps_line_factors(const PsHost& hp, double aii, double rate, double c, std::vector<double>& fl,
                     std::vector<double>& bu, std::vector<double>& bc);

// Pay-off at the nodes, cell averaged on the cells [x_{m-1/2}, x_{m+1/2}]^2 that
// meet its kink (Sec. 3.2.3); row-major n x n.  Kinds LPIDE_PUT_AVG and LPIDE_PUT_1.
bool ps_initial(const PsHost& hp, const lpide_payoff& pay, std::vector<double>& v0, std::string& err);

// Largest prime factor of m >= 1.
int largest_prime(int m);

}  // namespace lpide
