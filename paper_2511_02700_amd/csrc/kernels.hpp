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

}  // namespace lpide
