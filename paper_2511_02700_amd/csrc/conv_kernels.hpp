// Stand-alone FFT correlation kernels (FP64, conv_e(L) elements per thread) for the
// plan-time spectrum, the stand-alone correlation lpide_apply_B and the
// adjoint's kernel-gradient transforms, and a plain copy kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "fft.hpp"
#include "kernels.hpp"

namespace lpide {
namespace detail {

// Forward real FFT of pairs of rows (2p, 2p+1) of Y (n_rows x n_cols used,
// zero padded to L) into the transposed half spectra X[k2 * ldx + row].
template <int L>
__global__ __launch_bounds__(L / conv_e(L)) void k_rows_fwd(const double* __restrict__ Y, int ldy, int n_rows,
                                                   int n_cols, double2* __restrict__ X, int ldx,
                                                   const double2* __restrict__ tw) {
    constexpr int KE = conv_e(L), T = L / KE;
    __shared__ double2 lds[lds_slots(L)];
    __shared__ double2 tw4[tw_slots<L, KE>()];
    load_twiddles<L, KE>(tw, tw4);
    const int np = (n_rows + 1) >> 1;
    const int p = xcd_remap(blockIdx.x, np);
    const int ra = 2 * p, rb = 2 * p + 1;
    const bool hasb = rb < n_rows;
    const double* ya = Y + (size_t)ra * ldy;
    const double* yb = Y + (size_t)(hasb ? rb : ra) * ldy;
    const int tid = threadIdx.x;
    double2 reg[KE];
#pragma unroll
    for (int e = 0; e < KE; ++e) {
        const int idx = tid + e * T;
        double a = 0.0, b = 0.0;
        if (idx < n_cols) {
            a = ya[idx];
            b = hasb ? yb[idx] : 0.0;
        }
        reg[e] = make_double2(a, b);
    }
    fft_block<L, KE, false>(reg, lds, tw4);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < KE; ++e) lds[tid + e * T] = reg[e];
    __syncthreads();
    // Z = FFT(a + i b): A_k = (Z_k + conj Z_{L-k}) / 2, B_k = (Z_k - conj Z_{L-k}) / (2i)
    for (int k = tid; k <= L / 2; k += T) {
        const double2 z = lds[k], w = lds[k == 0 ? 0 : L - k];
        const double2 A = make_double2(0.5 * (z.x + w.x), 0.5 * (z.y - w.y));
        const double2 B = make_double2(0.5 * (z.y + w.y), -0.5 * (z.x - w.x));
        double2* xk = X + (size_t)k * ldx;
        xk[ra] = A;
        if (hasb) xk[rb] = B;
    }
}

// Column pass.  MODE 0: X[col] <- first n_out of IFFT(FFT(X[col], zero padded
// from n_in) * spec[col]).  MODE 1 (plan time): spec_out[col] = conj(FFT(X[col])) * scale.
// MODE 2: X[col] <- first n_out of IFFT(X[col], zero padded from n_in).
template <int L, int MODE>
__global__ __launch_bounds__(L / conv_e(L)) void k_cols(double2* __restrict__ X, int ldx, int n_in, int n_out,
                                               const double2* __restrict__ spec,
                                               double2* __restrict__ spec_out, double scale,
                                               const double2* __restrict__ tw) {
    constexpr int KE = conv_e(L), T = L / KE;
    __shared__ double2 lds[lds_slots(L)];
    __shared__ double2 tw4[tw_slots<L, KE>()];
    load_twiddles<L, KE>(tw, tw4);
    const int col = blockIdx.x;
    const int tid = threadIdx.x;
    double2* xc = X + (size_t)col * ldx;
    double2 reg[KE];
#pragma unroll
    for (int e = 0; e < KE; ++e) {
        const int idx = tid + e * T;
        reg[e] = idx < n_in ? xc[idx] : make_double2(0.0, 0.0);
    }
    if constexpr (MODE != 2) fft_block<L, KE, false>(reg, lds, tw4);
    if constexpr (MODE == 2) {
        fft_block<L, KE, true>(reg, lds, tw4);
#pragma unroll
        for (int e = 0; e < KE; ++e) {
            const int idx = tid + e * T;
            if (idx < n_out) xc[idx] = reg[e];
        }
        return;
    } else if constexpr (MODE == 1) {
        double2* so = spec_out + (size_t)col * L;
#pragma unroll
        for (int e = 0; e < KE; ++e) so[tid + e * T] = make_double2(reg[e].x * scale, -reg[e].y * scale);
        return;
    } else {
        const double2* sc = spec + (size_t)col * L;
#pragma unroll
        for (int e = 0; e < KE; ++e) reg[e] = cmul(reg[e], sc[tid + e * T]);
        fft_block<L, KE, true>(reg, lds, tw4);
#pragma unroll
        for (int e = 0; e < KE; ++e) {
            const int idx = tid + e * T;
            if (idx < n_out) xc[idx] = reg[e];
        }
    }
}

// Inverse real FFT of row pairs from the transposed half spectra; keeps the
// first n columns: row a <- real part, row b <- imaginary part.
template <int L>
__global__ __launch_bounds__(L / conv_e(L)) void k_rows_inv(const double2* __restrict__ X, int ldx, int n,
                                                   double* __restrict__ out, const double2* __restrict__ tw) {
    constexpr int KE = conv_e(L), T = L / KE;
    __shared__ double2 lds[lds_slots(L)];
    __shared__ double2 tw4[tw_slots<L, KE>()];
    load_twiddles<L, KE>(tw, tw4);
    const int np = (n + 1) >> 1;
    const int p = xcd_remap(blockIdx.x, np);
    const int ra = 2 * p, rb = 2 * p + 1;
    const bool hasb = rb < n;
    const int tid = threadIdx.x;
    double2 reg[KE];
#pragma unroll
    for (int e = 0; e < KE; ++e) {
        const int idx = tid + e * T;
        const bool lo = idx <= L / 2;
        const int k = lo ? idx : L - idx;
        const double2* xk = X + (size_t)k * ldx;
        const bool real_bin = k == 0 || k == L / 2;    // imaginary parts dropped at DC and Nyquist
        const double2 ta = xk[ra];
        const double2 tb = hasb ? xk[rb] : make_double2(0.0, 0.0);
        const double2 ha = make_double2(ta.x, real_bin ? 0.0 : ta.y);
        const double2 hb = make_double2(tb.x, real_bin ? 0.0 : tb.y);
        // Z_k = A_k + i B_k, with A_{L-k} = conj A_k, B_{L-k} = conj B_k
        reg[e] = lo ? make_double2(ha.x - hb.y, ha.y + hb.x) : make_double2(ha.x + hb.y, hb.x - ha.y);
    }
    fft_block<L, KE, true>(reg, lds, tw4);
#pragma unroll
    for (int e = 0; e < KE; ++e) {
        const int j = tid + e * T;
        if (j >= n) continue;
        out[(size_t)ra * n + j] = reg[e].x;
        if (hasb) out[(size_t)rb * n + j] = reg[e].y;
    }
}


static __global__ void k_copy(const double* __restrict__ a, double* __restrict__ b, size_t cnt) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) b[i] = a[i];
}

}  // namespace detail
}  // namespace lpide
