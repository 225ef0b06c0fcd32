// Host-side discretization of the two-asset exponential-Levy PIDE
// (Moda, in 't Hout, Vanmaele, Benth, arXiv 2511.02700) on a uniform
// log-moneyness grid.  Everything here runs once per plan, in FP64, on the CPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "lpide.h"

namespace lpide {

// NTS Levy measure with derived constants (Sec. 4: the Bessel-K_{1+alpha} density).
struct Nts {
    bool   jumps = false;
    double alpha = 0, delta = 0, lambda = 0, eta[2] = {0, 0}, rho[3] = {0, 0, 0};
    double det = 0;          // det rho
    double ri[3] = {0, 0, 0};// rho^{-1} (11, 12, 22)
    double ri_eta[2] = {0, 0};
    double c1 = 0;           // sqrt(||eta||_rho^2 + 2 lambda)
    double nu = 1;           // 1 + alpha
    double logpref = 0;      // log(delta/pi * sqrt(c1^(2 nu) / det))
};

// Everything a plan needs that is computed on the host.
struct HostPlan {
    // grid
    int    n = 0;
    double y_lo[2] = {0, 0}, h = 0;
    int    sl_order = 3, in_order = 3;
    // model
    double r = 0, sbs[3] = {0, 0, 0};
    Nts    nts;
    // integral discretization (Sec. 3.1)
    int    N_z = 0, M1 = 2, M2 = 0;
    double z_star = 0, sum_omega = 0, kappa[2] = {0, 0}, r_omega = 0, S[3] = {0, 0, 0}, a[3] = {0, 0, 0};
    std::vector<double> omega;   // (2 N_z)^2, omega[(l1+N_z)*2N_z + (l2+N_z)]
    // folded correlation kernel K = omega (*) (s x s) on offsets [dlo, dhi]^2
    int    dlo = 0, dhi = -1, L = 0;
    int    L_need = 0;           // n + max(-dlo, dhi): the least transform side without wrap-around
    std::vector<double> kern;    // (dhi-dlo+1)^2, row-major in d1
};

// Validates the model; fills the derived constants.  Returns false with a message.
bool make_nts(const lpide_levy& lv, Nts& out, std::string& err);

// log l(z) (Sec. 4); -inf where the density underflows every representation.
double log_density(const Nts& p, double z1, double z2);

// z_max^III before rounding: largest |z|_inf on {l = cut} (Sec. 4 settings).
double z_star(const Nts& p, double cut);

// Weights omega_l of the z-cells l in [-N_z, N_z)^2 of width h (Sec. 3.1): zero on
// R_I (|l + 1/2|_inf <= M1), the ||z||^2-weighted cell integral over ||z_l||^2 on
// R_II (<= M2, ng x ng Gauss-Legendre), the midpoint rule on R_III.
void integral_weights(const Nts& p, double h, int N_z, int M1, int M2, int ng, std::vector<double>& omega);

// Artificial diffusion S = integral over [-half, half]^2 of z z^T l(z) dz (Sec. 3.1).
void small_jump_cov(const Nts& p, double half, double S[3]);

// sum omega, kappa_omega^(i) = r - sum omega_l (e^{z_l^(i)} - 1) and r_omega = r + sum omega (Sec. 3.1).
void drift_and_rate(const std::vector<double>& omega, double h, int N_z, double r, double* sum_omega,
                    double kappa[2], double* r_omega);

// Zeros after the n factors of each array: the chunked device solves read their
// factors up to kLinePad - 1 elements past the end of a chunk without testing
// the index (at least the chunk capacity of the device solves).
constexpr int kLinePad = 32;

// Thomas factors of the tridiagonal matrix with rows (sub[j], dia[j], up[j]):
// forward multipliers fl, backward scales bu and couplings bc, each of length
// n + kLinePad (the last kLinePad zero).
void thomas_factors(const std::vector<double>& sub, const std::vector<double>& dia, const std::vector<double>& up,
                    std::vector<double>& fl, std::vector<double>& bu, std::vector<double>& bc);

// Builds the discretization (grid + integral part + folded kernel); no device work.
bool build_host_plan(const lpide_grid& g, const lpide_levy& lv, HostPlan& hp, std::string& err);

// Transform sides of the workgroup FFT: powers of two and 3 * 2^m (largest
// prime factor at most 3; Sec. 4 asks for transform sizes with small prime
// factors), ascending.
constexpr int kFftSizes[] = {64, 128, 256, 512, 768, 1024, 1536, 2048, 3072, 4096};
bool fft_size_supported(int L);
// Sides the automatic choice takes: all but 768, which allows E = 4 only and
// measured 3% slower than 1024 for whole solves at n = 512 (1536 and 3072 beat
// 2048 and 4096 by 8% and 10% at n = 1024 and 2048).
constexpr int kFftAutoSizes[] = {64, 128, 256, 512, 1024, 1536, 2048, 3072, 4096};
// The smallest automatic side >= need, or 0 when need exceeds the largest.
int fft_size_at_least(int need);

// Cell-averaged initial grid (Sec. 3.2.3), row-major n x n.
bool initial_values(const HostPlan& hp, const lpide_payoff& pay, std::vector<double>& v0, std::string& err);

// Factors of T_i = I - c (1/2 a_ii [interior](d2 - d1) - 1/2 r_omega), c = dt theta, as
// forward multipliers fl, backward scales bu and couplings bc (length n each).
void line_factors(int n, double h, double aii, double r_omega, double c,
                  std::vector<double>& fl, std::vector<double>& bu, std::vector<double>& bc);

// Factors of T_i^T (the transposed line operator, for the adjoint march).
void line_factors_T(int n, double h, double aii, double r_omega, double c,
                    std::vector<double>& fl, std::vector<double>& bu, std::vector<double>& bc);

// Derivatives of the semi-Lagrangian weights with respect to the departure
// position xi = j + shift, with the stencil start held fixed.
void sl_dweights(int n, double shift, int P, std::vector<double>& dw);

// Transpose of the interpolation matrix given by (start, w): for each m the
// source rows j and weights, padded to a common width (returned):
// idx[m*width + q], wt[m*width + q] (zero weights in the padding).
int sl_transpose(int n, int P, const std::vector<int32_t>& start, const std::vector<double>& w,
                 std::vector<int32_t>& idx, std::vector<double>& wt);

// Semi-Lagrangian interpolation weights along one axis: departure index j + shift,
// order P, clamped stencil start; start[j] and w[j*(P+1) + t].
void sl_weights(int n, double shift, int P, std::vector<int32_t>& start, std::vector<double>& w);

// The (theta, dt) step list with optional damping (Sec. 3.3).
std::vector<std::pair<double, double>> step_list(double theta, double T, int N_t, bool damping);

}  // namespace lpide
