// Device kernels of the time march (gfx950).  FP64 grids are row-major n x n,
// V[i * n + j], i the axis-1 index (slow), j the axis-2 index (fast).
//
// The FFT correlation (B v)_m = sum_d K_d v_{m+d} (Sec. 3.2.2 with the
// half-cell interpolation folded into K) is three passes over an
// intermediate X stored transposed, X[k2 * ldx + i1] (column k2 of the
// row-transformed grid is contiguous):
//   rows_fwd : pairs of real rows -> one complex length-L FFT -> split into
//              the two half spectra k2 = 0..L/2 (zero padding n -> L);
//   cols     : per column k2: forward FFT over i1 (zero padded), multiply by
//              the stored spectrum conj(K^)/L^2, inverse FFT, keep n rows;
//   rows_inv : per pair of rows: Hermitian completion of the two half
//              spectra into one complex sequence, inverse FFT, real part ->
//              row a, imaginary part -> row b, keep n columns, then a fused
//              epilogue (plain store, or the affine stencil form below).
#pragma once

#include <hip/hip_runtime.h>

#include "fft.hpp"

namespace lpide {

// Coefficients of the log-grid diffusion operator D (Sec. 3.2.1):
// D u = 1/2 a11 [i interior](d11 - d1) u + a12 d~1 d~2 u + 1/2 a22 [j interior](d22 - d2) u.
struct StencilArgs {
    int    n;
    double h, a11, a12, a22;
};

// Bijective block -> work-item remap that gives each of the 8 XCDs (which
// receive blocks round-robin) a contiguous range of work items.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int x = b & 7, i = b >> 3, q = nb >> 3, rem = nb & 7;
    return x * q + (x < rem ? x : rem) + i;
}

// D applied to U at (i, j).  Second differences only on interior indices of
// their own axis (the log form of the boundary rule "v linear in x"); the
// mixed term uses d~ = central inside, forward at 0, backward at n-1.
__device__ __forceinline__ double apply_D(const double* __restrict__ U, const StencilArgs& s, int i, int j,
                                          double u) {
    const int n = s.n;
    const double ih2 = 1.0 / (s.h * s.h), i2h = 0.5 / s.h;
    double d = 0.0;
    if (i > 0 && i < n - 1) {
        const double um = U[(size_t)(i - 1) * n + j], up = U[(size_t)(i + 1) * n + j];
        d += 0.5 * s.a11 * ((up - 2.0 * u + um) * ih2 - (up - um) * i2h);
    }
    if (j > 0 && j < n - 1) {
        const double um = U[(size_t)i * n + j - 1], up = U[(size_t)i * n + j + 1];
        d += 0.5 * s.a22 * ((up - 2.0 * u + um) * ih2 - (up - um) * i2h);
    }
    if (s.a12 != 0.0) {
        int i0, i1, j0, j1;
        double gi, gj;
        if (i == 0) { i0 = 0; i1 = 1; gi = 1.0 / s.h; }
        else if (i == n - 1) { i0 = n - 2; i1 = n - 1; gi = 1.0 / s.h; }
        else { i0 = i - 1; i1 = i + 1; gi = i2h; }
        if (j == 0) { j0 = 0; j1 = 1; gj = 1.0 / s.h; }
        else if (j == n - 1) { j0 = n - 2; j1 = n - 1; gj = 1.0 / s.h; }
        else { j0 = j - 1; j1 = j + 1; gj = i2h; }
        const double u00 = U[(size_t)i0 * n + j0], u01 = U[(size_t)i0 * n + j1];
        const double u10 = U[(size_t)i1 * n + j0], u11 = U[(size_t)i1 * n + j1];
        d += s.a12 * gi * gj * ((u11 - u10) - (u01 - u00));
    }
    return d;
}

// apply_D with all eight neighbours read at indices clamped into the grid
// (the mixed term's nodes are those neighbours): every read valid and none
// conditional, so that a node's reads are in flight together; the interior
// tests select the arithmetic only (a zero a12 adds a zero mixed term).  For
// row kernels with one element per thread and loop pass; kernels that unroll
// many elements keep apply_D, whose branches throttle the reads in flight.
__device__ __forceinline__ double apply_D_ahead(const double* __restrict__ U, const StencilArgs& s, int i, int j,
                                                double u) {
    const int n = s.n;
    const double ih2 = 1.0 / (s.h * s.h), i2h = 0.5 / s.h;
    const bool iin = i > 0 && i < n - 1, jin = j > 0 && j < n - 1;
    const int im = i > 0 ? i - 1 : 0, ip = i < n - 1 ? i + 1 : n - 1;
    const int jm = j > 0 ? j - 1 : 0, jp = j < n - 1 ? j + 1 : n - 1;
    const double* rm = U + (size_t)im * n;
    const double* rp = U + (size_t)ip * n;
    const double u1m = rm[j], u1p = rp[j];
    const double u2m = U[(size_t)i * n + jm], u2p = U[(size_t)i * n + jp];
    const double u00 = rm[jm], u01 = rm[jp], u10 = rp[jm], u11 = rp[jp];
    double d = 0.0;
    if (iin) d += 0.5 * s.a11 * ((u1p - 2.0 * u + u1m) * ih2 - (u1p - u1m) * i2h);
    if (jin) d += 0.5 * s.a22 * ((u2p - 2.0 * u + u2m) * ih2 - (u2p - u2m) * i2h);
    const double gi = iin ? i2h : 1.0 / s.h, gj = jin ? i2h : 1.0 / s.h;
    d += s.a12 * gi * gj * ((u11 - u10) - (u01 - u00));
    return d;
}

// The three unit-coefficient parts of D at (i, j): D u = a11 d11 + a12 d12 + a22 d22
// (the derivative of D u with respect to each coefficient).
__device__ __forceinline__ void apply_D_parts(const double* __restrict__ U, int n, double h, int i, int j, double u,
                                              double& d11, double& d12, double& d22) {
    const double ih2 = 1.0 / (h * h), i2h = 0.5 / h;
    d11 = d12 = d22 = 0.0;
    if (i > 0 && i < n - 1) {
        const double um = U[(size_t)(i - 1) * n + j], up = U[(size_t)(i + 1) * n + j];
        d11 = 0.5 * ((up - 2.0 * u + um) * ih2 - (up - um) * i2h);
    }
    if (j > 0 && j < n - 1) {
        const double um = U[(size_t)i * n + j - 1], up = U[(size_t)i * n + j + 1];
        d22 = 0.5 * ((up - 2.0 * u + um) * ih2 - (up - um) * i2h);
    }
    int i0, i1, j0, j1;
    double gi, gj;
    if (i == 0) { i0 = 0; i1 = 1; gi = 1.0 / h; }
    else if (i == n - 1) { i0 = n - 2; i1 = n - 1; gi = 1.0 / h; }
    else { i0 = i - 1; i1 = i + 1; gi = i2h; }
    if (j == 0) { j0 = 0; j1 = 1; gj = 1.0 / h; }
    else if (j == n - 1) { j0 = n - 2; j1 = n - 1; gj = 1.0 / h; }
    else { j0 = j - 1; j1 = j + 1; gj = i2h; }
    const double u00 = U[(size_t)i0 * n + j0], u01 = U[(size_t)i0 * n + j1];
    const double u10 = U[(size_t)i1 * n + j0], u11 = U[(size_t)i1 * n + j1];
    d12 = gi * gj * ((u11 - u10) - (u01 - u00));
}

// Column p of the one-dimensional first-difference matrix G used by the mixed
// term (rows: central inside, forward at 0, backward at n-1): the (at most two)
// rows r with G[r][p] != 0 and those entries.
__device__ __forceinline__ int diff_T(int n, double h, int p, int* r, double* c) {
    int m = 0;
    const double i2h = 0.5 / h, ih = 1.0 / h;
    if (p - 1 >= 1 && p - 1 <= n - 2) { r[m] = p - 1; c[m] = i2h; ++m; }    // G[p-1][p]
    if (p + 1 >= 1 && p + 1 <= n - 2) { r[m] = p + 1; c[m] = -i2h; ++m; }   // G[p+1][p]
    if (p == 0) { r[m] = 0; c[m] = -ih; ++m; }                               // row 0: (v1 - v0)/h
    if (p == 1) { r[m] = 0; c[m] = ih; ++m; }
    if (p == n - 2) { r[m] = n - 1; c[m] = -ih; ++m; }                       // row n-1: (v_{n-1} - v_{n-2})/h
    if (p == n - 1) { r[m] = n - 1; c[m] = ih; ++m; }
    return m;
}

// D^T applied to U at (i, j): the transposed log-grid stencil, boundary rows
// included (the adjoint of apply_D).
__device__ __forceinline__ double apply_DT(const double* __restrict__ U, const StencilArgs& s, int i, int j,
                                           double u) {
    const int n = s.n;
    const double ih2 = 1.0 / (s.h * s.h), i2h = 0.5 / s.h;
    // Away from the edges (every neighbour an interior node) the transposed
    // stencil is the forward one with the first differences negated: the
    // second differences and the product of two central differences are
    // symmetric, a central difference is antisymmetric.
    if (i >= 2 && i <= n - 3 && j >= 2 && j <= n - 3) {
        const double u1m = U[(size_t)(i - 1) * n + j], u1p = U[(size_t)(i + 1) * n + j];
        const double u2m = U[(size_t)i * n + j - 1], u2p = U[(size_t)i * n + j + 1];
        double d = 0.5 * s.a11 * ((u1p - 2.0 * u + u1m) * ih2 + (u1p - u1m) * i2h) +
                   0.5 * s.a22 * ((u2p - 2.0 * u + u2m) * ih2 + (u2p - u2m) * i2h);
        if (s.a12 != 0.0) {
            const double* rm = U + (size_t)(i - 1) * n;
            const double* rp = U + (size_t)(i + 1) * n;
            d += s.a12 * i2h * i2h * ((rp[j + 1] - rp[j - 1]) - (rm[j + 1] - rm[j - 1]));
        }
        return d;
    }
    // second-difference parts: row r (interior) holds 1/2 [(v_{r+1} - 2 v_r + v_{r-1})/h^2 - (v_{r+1} - v_{r-1})/(2h)]
    const double cu = 0.5 * (ih2 - i2h);   // coefficient of v_{r+1} in row r
    const double cl = 0.5 * (ih2 + i2h);   // coefficient of v_{r-1} in row r
    double d = 0.0;
    {
        double t = 0.0;
        if (i > 0 && i < n - 1) t -= ih2 * u;
        if (i - 1 >= 1 && i - 1 <= n - 2) t += cu * U[(size_t)(i - 1) * n + j];
        if (i + 1 >= 1 && i + 1 <= n - 2) t += cl * U[(size_t)(i + 1) * n + j];
        d += s.a11 * t;
    }
    {
        double t = 0.0;
        if (j > 0 && j < n - 1) t -= ih2 * u;
        if (j - 1 >= 1 && j - 1 <= n - 2) t += cu * U[(size_t)i * n + j - 1];
        if (j + 1 >= 1 && j + 1 <= n - 2) t += cl * U[(size_t)i * n + j + 1];
        d += s.a22 * t;
    }
    if (s.a12 != 0.0) {
        int ri[4], rj[4];
        double ci[4], cj[4];
        const int mi = diff_T(n, s.h, i, ri, ci), mj = diff_T(n, s.h, j, rj, cj);
        double t = 0.0;
        for (int a = 0; a < mi; ++a)
            for (int b = 0; b < mj; ++b) t += ci[a] * cj[b] * U[(size_t)ri[a] * n + rj[b]];
        d += s.a12 * t;
    }
    return d;
}

}  // namespace lpide
