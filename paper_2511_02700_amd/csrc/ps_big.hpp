// Two-level transforms of the price-space correlation for sides L = R M
// beyond one workgroup's LDS (M = 4096; R = 3, 4, 6: L = 12288, 16384, 24576;
// the paper's grids need up to #in = 16807, Sec. 4).
//
// With w_N = exp(-2 pi i / N), a length-L transform splits by decimation in
// frequency into R transforms of length M,
//   Z_{R q + r} = FFT_M(y^(r))_q,   y^(r)_m = w_L^{m r} sum_s z_{m + s M} w_R^{s r},
// and its inverse by decimation in time back into them,
//   z_{m + s M} = sum_r w_R^{-s r} w_L^{-m r} IFFT_M(Z_{R . + r})_m.
// One workgroup of 512 threads handles one length-L sequence and runs its R
// length-M transforms one after the other through LDS; the inverse sums the
// R contributions in registers, for the SO segments of length M that hold
// kept outputs (SO = ceil(n_out / M) <= R).  The spectrum of the weights is stored per
// column in the order (r, q): entry r M + q of column k2 holds frequency
// R q + r, so that the column pass multiplies each length-M transform by a
// contiguous slice.  The row r2c split needs Z_k and Z_{L-k}: for k = R q + r
// the partner lies in sub-sequence R - r at index M - 1 - q (sub-sequence 0
// at (M - q) mod M for r = 0), so the row kernel transforms the
// sub-sequences in those pairs, one held in registers and its partner in LDS,
// and each thread writes both members of its pairs (k, L - k).
#pragma once

#include <hip/hip_runtime.h>

#include "ps_kernels.hpp"

namespace lpide {
namespace ps {

constexpr int BIG_T = 512;   // threads of every two-level kernel
// Inner transform length of a two-level side: 4096 (8 elements per thread).
// Inner transforms of 8192 would halve the sub-transforms, but with 16
// elements per thread the column pass and row inverse spill their
// accumulators (700-1000 bytes per lane at 512 threads).
constexpr int big_m(int) { return 4096; }

__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// Rows forward of a length-L real transform, two rows per workgroup (as one
// complex sequence), the half spectra into X[k * ldx + row], k = 0..L/2.
// MODE 0: the rows of v^in = T^in U (U: n x ldu; n_nz rows and columns);
// MODE 1: rows of a dense real array G (nrows x ncols, row stride ldu).
template <int M, int R, int MODE>
__global__ __launch_bounds__(BIG_T) void ps_big_rows_fwd(const double* __restrict__ U, int ldu, int nrows, int ncols,
                                                         double2* __restrict__ X, int ldx,
                                                         const int* __restrict__ tin_s,
                                                         const double* __restrict__ tin_w,
                                                         const double2* __restrict__ twL,
                                                         const double2* __restrict__ twM, const PsCtl* ctl, int k,
                                                         double tol) {
    if (ps_halted(ctl, k, tol)) return;
    constexpr int E = M / BIG_T, T = BIG_T, L = R * M;
    __shared__ double2 lds[lds_slots(M)];
    __shared__ double2 tw4[tw_slots<M, E>()];
    load_twiddles<M, E>(twM, tw4);
    const int np = (nrows + 1) >> 1;
    const int p = xcd_remap(blockIdx.x, np);
    const int ra = 2 * p, rb = 2 * p + 1;
    const bool hasb = rb < nrows;
    const int tid = threadIdx.x;
    const double *ua, *ub;
    double wa[4] = {1.0, 0.0, 0.0, 0.0}, wb[4] = {0.0, 0.0, 0.0, 0.0};
    if constexpr (MODE == 0) {
        ua = U + (size_t)tin_s[ra] * ldu;
        ub = U + (size_t)tin_s[hasb ? rb : ra] * ldu;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            wa[t] = tin_w[4 * ra + t];
            wb[t] = hasb ? tin_w[4 * rb + t] : 0.0;
        }
    } else {
        ua = U + (size_t)ra * ldu;
        ub = U + (size_t)(hasb ? rb : ra) * ldu;
        wb[0] = hasb ? 1.0 : 0.0;
    }
    // y^(r) and y^(r2) for this thread's m from one pass over the inputs (the
    // two sub-sequences of a pair read the same z), then the transform of y^(r)
    auto gather2 = [&](int r, int r2, double2 (&y1)[E], double2 (&y2)[E]) {
#pragma unroll
        for (int e = 0; e < E; ++e) y1[e] = y2[e] = make_double2(0.0, 0.0);
#pragma unroll 1
        for (int s = 0; s < R; ++s) {
            const double2 w1 = twL[((s * r) % R) * M], w2 = twL[((s * r2) % R) * M];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int j = tid + e * T + s * M;
                if (j < ncols) {
                    double a = 0.0, b = 0.0;
                    if constexpr (MODE == 0) {
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            a += wa[t] * ua[(size_t)t * ldu + j];
                            b += wb[t] * ub[(size_t)t * ldu + j];
                        }
                    } else {
                        a = ua[j];
                        b = wb[0] * ub[j];
                    }
                    y1[e].x += a * w1.x - b * w1.y;
                    y1[e].y += a * w1.y + b * w1.x;
                    y2[e].x += a * w2.x - b * w2.y;
                    y2[e].y += a * w2.y + b * w2.x;
                }
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            y1[e] = cmul(y1[e], twL[(tid + e * T) * r]);
            y2[e] = cmul(y2[e], twL[(tid + e * T) * r2]);
        }
    };
    auto fft = [&](double2 (&reg)[E]) {
        __syncthreads();                                  // LDS free for the transform
        fft_block<M, E, false>(reg, lds, tw4);
    };
    // A_k, B_k of the two rows from Z_k = z and Z_{L-k} = w
    auto put = [&](int kk, double2 z, double2 w) {
        double2* xk = X + (size_t)kk * ldx;
        xk[ra] = make_double2(0.5 * (z.x + w.x), 0.5 * (z.y - w.y));
        if (hasb) xk[rb] = make_double2(0.5 * (z.y + w.y), -0.5 * (z.x - w.x));
    };
#pragma unroll 1
    for (int r = 0; r <= R / 2; ++r) {
        const int r2 = (R - r) % R;                       // the partner sub-sequence
        double2 yr[E], yp[E];
        gather2(r, r2, yr, yp);                           // (yp = yr when the pair is r itself)
        fft(yr);
        if (r2 != r) fft(yp);
        __syncthreads();
        if (r2 != r) {
#pragma unroll
            for (int e = 0; e < E; ++e) lds[tid + e * T] = yp[e];
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) lds[tid + e * T] = yr[e];
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int q = tid + e * T;
            const int kk = R * q + r;
            if (r2 == r) {
                // the partner of R q + r lies in the same sub-sequence
                const double2 w = lds[r == 0 ? ((M - q) & (M - 1)) : M - 1 - q];
                if (kk <= L / 2) put(kk, yr[e], w);
            } else {
                const double2 w = lds[M - 1 - q];             // Y^(r2)_{M-1-q} = Z_{L-k}
                if (kk <= L / 2) put(kk, yr[e], w);
                const int k2 = R * (M - 1 - q) + r2;          // and Z_{L-k2} = Y^(r)_q
                if (k2 <= L / 2) put(k2, w, yr[e]);
            }
        }
    }
}

// Column k2 (length L over the first n_in rows, zero padded).  MODE 0: forward
// transform, product with the stored spectrum, inverse, the first n_out entries
// back into X.  MODE 1 (plan time): spec_out column = conj(forward) * scale in
// the (r, q) order.
template <int M, int R, int SO, int MODE>
__global__ __launch_bounds__(BIG_T) void ps_big_cols(double2* __restrict__ X, int ldx, int n_in, int n_out,
                                                             const double2* __restrict__ spec,
                                                             double2* __restrict__ spec_out, double scale,
                                                             const double2* __restrict__ twL,
                                                             const double2* __restrict__ twM, const PsCtl* ctl, int k,
                                                             double tol) {
    if (ps_halted(ctl, k, tol)) return;
    constexpr int E = M / BIG_T, T = BIG_T, L = R * M;
    __shared__ double2 lds[lds_slots(M)];
    __shared__ double2 tw4[tw_slots<M, E>()];
    load_twiddles<M, E>(twM, tw4);
    const int col = blockIdx.x;
    const int tid = threadIdx.x;
    double2* xc = X + (size_t)col * ldx;
    double2 acc[MODE == 0 ? SO : 1][E];
    if constexpr (MODE == 0) {
#pragma unroll
        for (int s = 0; s < SO; ++s)
#pragma unroll
            for (int e = 0; e < E; ++e) acc[s][e] = make_double2(0.0, 0.0);
    }
#pragma unroll 1
    for (int r = 0; r < R; ++r) {
        double2 reg[E];
#pragma unroll
        for (int e = 0; e < E; ++e) reg[e] = make_double2(0.0, 0.0);
#pragma unroll 1
        for (int s = 0; s < R; ++s) {
            const double2 w = twL[((s * r) % R) * M];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int j = tid + e * T + s * M;
                if (j < n_in) {
                    const double2 v = cmul(xc[j], w);
                    reg[e].x += v.x;
                    reg[e].y += v.y;
                }
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) reg[e] = cmul(reg[e], twL[(tid + e * T) * r]);
        __syncthreads();
        fft_block<M, E, false>(reg, lds, tw4);
        if constexpr (MODE == 1) {
            double2* so = spec_out + (size_t)col * L + (size_t)r * M;
#pragma unroll
            for (int e = 0; e < E; ++e) so[tid + e * T] = make_double2(reg[e].x * scale, -reg[e].y * scale);
        } else {
            const double2* sc = spec + (size_t)col * L + (size_t)r * M;
#pragma unroll
            for (int e = 0; e < E; ++e) reg[e] = cmul(reg[e], sc[tid + e * T]);
            __syncthreads();
            fft_block<M, E, true>(reg, lds, tw4);
#pragma unroll
            for (int e = 0; e < E; ++e) reg[e] = cmul(reg[e], cconj(twL[(tid + e * T) * r]));
#pragma unroll
            for (int s = 0; s < SO; ++s) {
                const double2 w = cconj(twL[((s * r) % R) * M]);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const double2 v = cmul(reg[e], w);
                    acc[s][e].x += v.x;
                    acc[s][e].y += v.y;
                }
            }
        }
    }
    if constexpr (MODE == 0) {
        __syncthreads();                                  // every read of the column is done
#pragma unroll
        for (int s = 0; s < SO; ++s)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int j = tid + e * T + s * M;
                if (j < n_out) xc[j] = acc[s][e];
            }
    }
}

// y^out rows (2p, 2p+1): the inverse length-L transform of A + i B (Hermitian
// completion of the half spectra), then the axis-2 T^out gather through LDS
// windows of the inverse row: Z[row][m] = sum_t T^out_{m, s_m + t} row[s_m + t].
template <int M, int R, int SO>
__global__ __launch_bounds__(BIG_T) void ps_big_rows_inv(const double2* __restrict__ X, double* __restrict__ Z,
                                                                 PsOps o, const double2* __restrict__ twL,
                                                                 const double2* __restrict__ twM, const PsCtl* ctl,
                                                                 int k, double tol) {
    if (ps_halted(ctl, k, tol)) return;
    constexpr int E = M / BIG_T, T = BIG_T, L = R * M;
    constexpr int WIN = lds_slots(M);
    __shared__ double2 lds[lds_slots(M)];
    __shared__ double2 tw4[tw_slots<M, E>()];
    load_twiddles<M, E>(twM, tw4);
    const int m_out = o.n_out, np = (m_out + 1) >> 1;
    const int p = xcd_remap(blockIdx.x, np);
    const int ra = 2 * p, rb = 2 * p + 1;
    const bool hasb = rb < m_out;
    const int tid = threadIdx.x;
    double2 acc[SO][E];
#pragma unroll
    for (int s = 0; s < SO; ++s)
#pragma unroll
        for (int e = 0; e < E; ++e) acc[s][e] = make_double2(0.0, 0.0);
#pragma unroll 1
    for (int r = 0; r < R; ++r) {
        double2 reg[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int kk = R * (tid + e * T) + r;
            const bool lo = kk <= L / 2;
            const int kc = lo ? kk : L - kk;
            const double2* xk = X + (size_t)kc * o.ldx;
            const bool real_bin = kc == 0 || kc == L / 2;    // imaginary parts dropped at DC and Nyquist
            const double2 ta = xk[ra];
            const double2 tb = hasb ? xk[rb] : make_double2(0.0, 0.0);
            const double2 ha = make_double2(ta.x, real_bin ? 0.0 : ta.y);
            const double2 hb = make_double2(tb.x, real_bin ? 0.0 : tb.y);
            // Z_k = A_k + i B_k, with A_{L-k} = conj A_k, B_{L-k} = conj B_k
            reg[e] = lo ? make_double2(ha.x - hb.y, ha.y + hb.x) : make_double2(ha.x + hb.y, hb.x - ha.y);
        }
        __syncthreads();
        fft_block<M, E, true>(reg, lds, tw4);
#pragma unroll
        for (int e = 0; e < E; ++e) reg[e] = cmul(reg[e], cconj(twL[(tid + e * T) * r]));
#pragma unroll
        for (int s = 0; s < SO; ++s) {
            const double2 w = cconj(twL[((s * r) % R) * M]);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double2 v = cmul(reg[e], w);
                acc[s][e].x += v.x;
                acc[s][e].y += v.y;
            }
        }
    }
    // windows [wlo, whi) of the inverse row, overlapping by 3; node m is done in
    // the window with wlo <= s_m <= whi - 4 (exactly one: the next starts at whi - 3)
    const int n = o.n;
    for (int wlo = 0;;) {
        const int whi = min(m_out, wlo + WIN);
        __syncthreads();
#pragma unroll
        for (int s = 0; s < SO; ++s)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int j = tid + e * T + s * M;
                if (j >= wlo && j < whi) lds[j - wlo] = acc[s][e];
            }
        __syncthreads();
        for (int q = tid; q < n; q += T) {
            const int sq = o.tout_s[q];
            if (sq < wlo || sq > whi - 4) continue;
            const double* w = o.tout_w + 4 * q;
            const double2* v = lds + (sq - wlo);
            Z[(size_t)ra * n + q] = w[0] * v[0].x + w[1] * v[1].x + w[2] * v[2].x + w[3] * v[3].x;
            if (hasb) Z[(size_t)rb * n + q] = w[0] * v[0].y + w[1] * v[1].y + w[2] * v[2].y + w[3] * v[3].y;
        }
        if (whi >= m_out) break;
        wlo = whi - 3;
    }
}

}  // namespace ps
}  // namespace lpide
