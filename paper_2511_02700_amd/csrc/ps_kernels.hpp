// Device kernels of the price-space march (Sec. 3.2, Sec. 3.3, Sec. 4
// settings; gfx950).  Grids are row-major n x n, V[i * n + j] at (x_i, x_j).
//
// B_omega v = T^out I~ C T^in v is four passes:
//   tin2     : U = v (T^in)^T, the axis-2 interpolation to the y^in nodes
//              inside [0, x_max] (n x n_nz; the rows of T^in beyond x_max are
//              zero, so those nodes are the zero padding of the transform);
//   rows_fwd : per pair of y^in rows, the axis-1 interpolation (four rows of
//              U), one complex length-L FFT, the two half spectra stored
//              transposed, X[k2 * ldx + i];
//   cols     : per column k2: FFT over i, times the stored spectrum
//              conj(FFT(omega placed at j mod L)) / L^2, inverse FFT, the
//              first n_out entries kept (the rows I~ keeps);
//   rows_inv : per pair of y^out rows: inverse FFT and the axis-2 T^out
//              gather from LDS, Z = (C T^in v on y^out x y^out) (T^out)^T,
//              n_out x n.
// The axis-1 T^out gather, B v = T^out Z, is taken inside the kernel that
// uses it (the residual, the explicit part, the stand-alone product).
//
// One fixed-point iteration of a step (c = dt theta) is
//   tin2, rows_fwd, cols, rows_inv on Y (B Y),
//   resid_rows: R = W - (I - c (D + B - r_omega)) Y on each grid row, then
//               the axis-2 solve Q = T_2^{-1} R,
//   line_cols : the axis-1 solve delta = T_1^{-1} Q, Y += delta and the
//               stopping-rule maximum max |delta| / max(1, |Y|),
// with T_1 = I - c (a_11 x_1^2 D2_1 / 2 - r_omega), T_2 = I - c a_22 x_2^2 D2_2 / 2
// tridiagonal.  Its fixed point solves the step equation
// (I - c (D + B - r_omega)) Y = W exactly.
// Every kernel of iteration k returns at once when iteration k - 1 met the
// tolerance or the control block's failure flag is set.
#pragma once

#include <hip/hip_runtime.h>

#include "fft.hpp"
#include "kernels.hpp"
#include "linesolve.hpp"

namespace lpide {
namespace ps {

constexpr int PS_MAXK = 128;   // iterations per step the control block can record

// FFT elements per thread of the price-space transforms: 16 above 4096 (one
// workgroup of 384 or 512 threads, 104 or 148 KB of LDS at 6144 and 8192).
constexpr int ps_e(int L) { return L > 4096 ? 16 : conv_e(L); }

// Control block of a price-space march.
struct PsCtl {
    unsigned long long err[PS_MAXK + 2];   // err[k]: stopping-rule value of iteration k (FP64 bits); 0 = unset
    unsigned long long last;               // stopping-rule value of the last converged step
    int fail;                              // 1: the enqueued iterations of a step did not meet tol; 2: NaN
    int pad;
};

// Spatial operator tables (device pointers) and the coefficients of D.
struct PsOps {
    int n, n_nz, n_out, ldx;
    const int* tin_s;        // n_nz rows of T^in: stencil start and 4 weights
    const double* tin_w;
    const int* tout_s;       // n rows of T^out (from the n_out nodes of y^out)
    const double* tout_w;
    const double* A1;        // per node m: x_m d1 (3 coefficients at m-1, m, m+1)
    const double* A2;        // per node m: x_m^2 d2 / 2
    double a11, a12, a22, r_omega;
};

// One step kind: c = dt theta and the Thomas factors of T_1 and T_2.
struct PsStepK {
    double c;
    const double *fl1, *bu1, *bc1, *fl2, *bu2, *bc2;
};

__device__ __forceinline__ double ps_bits(unsigned long long b) { return __longlong_as_double((long long)b); }

__device__ __forceinline__ bool ps_halted(const PsCtl* c, int k, double tol) {
    if (c == nullptr) return false;
    if (c->fail) return true;
    return k > 1 && ps_bits(c->err[k - 1]) < tol;
}

// D Y at (i, j): a11 x_i^2 d2_i / 2 + a22 x_j^2 d2_j / 2 + a12 (x_i d1_i)(x_j d1_j).
// Indices outside the grid carry zero coefficients (clamped reads).
__device__ __forceinline__ double ps_DY(const double* __restrict__ Y, const PsOps& o, int i, int j) {
    const int n = o.n;
    const int im = i > 0 ? i - 1 : 0, ip = i < n - 1 ? i + 1 : n - 1;
    const int jm = j > 0 ? j - 1 : 0, jp = j < n - 1 ? j + 1 : n - 1;
    const double* a1i = o.A1 + 3 * i;
    const double* a2i = o.A2 + 3 * i;
    const double* a1j = o.A1 + 3 * j;
    const double* a2j = o.A2 + 3 * j;
    const double* r0 = Y + (size_t)im * n;
    const double* r1 = Y + (size_t)i * n;
    const double* r2 = Y + (size_t)ip * n;
    const double yc = r1[j];
    double d = o.a11 * (a2i[0] * r0[j] + a2i[1] * yc + a2i[2] * r2[j]) +
               o.a22 * (a2j[0] * r1[jm] + a2j[1] * yc + a2j[2] * r1[jp]);
    if (o.a12 != 0.0) {
        const double g0 = a1j[0] * r0[jm] + a1j[1] * r0[j] + a1j[2] * r0[jp];
        const double g1 = a1j[0] * r1[jm] + a1j[1] * yc + a1j[2] * r1[jp];
        const double g2 = a1j[0] * r2[jm] + a1j[1] * r2[j] + a1j[2] * r2[jp];
        d += o.a12 * (a1i[0] * g0 + a1i[1] * g1 + a1i[2] * g2);
    }
    return d;
}

// (B Y)(i, j) = sum_t T^out_{i, s_i + t} Z[s_i + t][j].
__device__ __forceinline__ double ps_BY(const double* __restrict__ Z, const PsOps& o, int i, int j) {
    const int s = o.tout_s[i];
    const double* w = o.tout_w + 4 * i;
    const double* z = Z + (size_t)s * o.n + j;
    return w[0] * z[0] + w[1] * z[o.n] + w[2] * z[2 * o.n] + w[3] * z[3 * o.n];
}

// U[row][q] = sum_t T^in_{q, s_q + t} Y[row][s_q + t]; grid (ceil(n_nz / 256), n).
static __global__ __launch_bounds__(256) void ps_tin2(const double* __restrict__ Y, double* __restrict__ U, PsOps o,
                                                      const PsCtl* ctl, int k, double tol) {
    if (ps_halted(ctl, k, tol)) return;
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= o.n_nz) return;
    const int row = blockIdx.y;
    const int s = o.tin_s[q];
    const double* w = o.tin_w + 4 * q;
    const double* y = Y + (size_t)row * o.n + s;
    U[(size_t)row * o.n_nz + q] = w[0] * y[0] + w[1] * y[1] + w[2] * y[2] + w[3] * y[3];
}

// Rows (2p, 2p+1) of v^in = T^in U (four rows of U each, zero beyond n_nz
// columns), one complex FFT, the half spectra into X[k2 * ldx + row].
template <int L>
__global__ __launch_bounds__(L / ps_e(L)) void ps_rows_fwd(const double* __restrict__ U, double2* __restrict__ X,
                                                             PsOps o, const double2* __restrict__ tw,
                                                             const PsCtl* ctl, int k, double tol) {
    if (ps_halted(ctl, k, tol)) return;
    constexpr int KE = ps_e(L), T = L / KE;
    __shared__ double2 lds[lds_slots(L)];
    __shared__ double2 tw4[tw_slots<L, KE>()];
    load_twiddles<L, KE>(tw, tw4);
    const int m = o.n_nz, np = (m + 1) >> 1;
    const int p = xcd_remap(blockIdx.x, np);
    const int ra = 2 * p, rb = 2 * p + 1;
    const bool hasb = rb < m;
    const int sa = o.tin_s[ra], sb = o.tin_s[hasb ? rb : ra];
    double wa[4], wb[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        wa[t] = o.tin_w[4 * ra + t];
        wb[t] = hasb ? o.tin_w[4 * rb + t] : 0.0;
    }
    const double* ua = U + (size_t)sa * m;
    const double* ub = U + (size_t)sb * m;
    const int tid = threadIdx.x;
    double2 reg[KE];
#pragma unroll
    for (int e = 0; e < KE; ++e) {
        const int idx = tid + e * T;
        double a = 0.0, b = 0.0;
        if (idx < m) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                a += wa[t] * ua[(size_t)t * m + idx];
                b += wb[t] * ub[(size_t)t * m + idx];
            }
        }
        reg[e] = make_double2(a, b);
    }
    fft_block<L, KE, false>(reg, lds, tw4);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < KE; ++e) lds[tid + e * T] = reg[e];
    __syncthreads();
    // Z = FFT(a + i b): A_k = (Z_k + conj Z_{L-k}) / 2, B_k = (Z_k - conj Z_{L-k}) / (2i).
    // Item idx is frequency idx / 2 of row ra + idx mod 2: the two rows of a
    // frequency are adjacent in X, so a lane pair stores them as one 32-byte piece.
    constexpr int NI = (L + 2 + T - 1) / T;
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int idx = tid + it * T;
        const int kk = idx >> 1, r = idx & 1;
        if (kk > L / 2 || (r == 1 && !hasb)) continue;
        const double2 z = lds[kk], w = lds[kk == 0 ? 0 : L - kk];
        X[(size_t)kk * o.ldx + ra + r] = r == 0 ? make_double2(0.5 * (z.x + w.x), 0.5 * (z.y - w.y))
                                                : make_double2(0.5 * (z.y + w.y), -0.5 * (z.x - w.x));
    }
}

// Column k2: FFT over the n_nz rows (zero padded to L), times the spectrum,
// inverse FFT, the first n_out entries back into X.  L/2 blocks for the L/2 + 1
// columns: block 0 filters the two real columns 0 and L/2 as one complex column
// (mul_real_pair; the row inverse reads only their real parts).
template <int L>
__global__ __launch_bounds__(L / ps_e(L)) void ps_cols(double2* __restrict__ X, const double2* __restrict__ spec,
                                                         PsOps o, const double2* __restrict__ tw, const PsCtl* ctl,
                                                         int k, double tol) {
    if (ps_halted(ctl, k, tol)) return;
    constexpr int KE = ps_e(L), T = L / KE;
    __shared__ double2 lds[lds_slots(L)];
    __shared__ double2 tw4[tw_slots<L, KE>()];
    load_twiddles<L, KE>(tw, tw4);
    const int col = blockIdx.x;
    const int tid = threadIdx.x;
    const bool pair = col == 0;
    double2* xc = X + (size_t)col * o.ldx;
    double2* xn = X + (size_t)(L / 2) * o.ldx;
    double2 reg[KE];
#pragma unroll
    for (int e = 0; e < KE; ++e) {
        const int idx = tid + e * T;
        if (idx < o.n_nz) reg[e] = pair ? make_double2(xc[idx].x, xn[idx].x) : xc[idx];
        else reg[e] = make_double2(0.0, 0.0);
    }
    fft_block<L, KE, false>(reg, lds, tw4);
    const double2* sc = spec + (size_t)col * L;
    if (pair) {
        mul_real_pair<L, KE, false>(reg, lds, sc, spec + (size_t)(L / 2) * L);
    } else {
#pragma unroll
        for (int e = 0; e < KE; ++e) reg[e] = cmul(reg[e], sc[tid + e * T]);
    }
    fft_block<L, KE, true>(reg, lds, tw4);
#pragma unroll
    for (int e = 0; e < KE; ++e) {
        const int idx = tid + e * T;
        if (idx >= o.n_out) continue;
        if (pair) {
            xc[idx] = make_double2(reg[e].x, 0.0);
            xn[idx] = make_double2(reg[e].y, 0.0);
        } else {
            xc[idx] = reg[e];
        }
    }
}

// y^out rows (2p, 2p+1): Hermitian completion of the two half spectra, inverse
// FFT, the n_out kept columns staged in LDS, then the axis-2 T^out gather:
// Z[row][m] = sum_t T^out_{m, s_m + t} row[s_m + t], m < n.
template <int L>
__global__ __launch_bounds__(L / ps_e(L)) void ps_rows_inv(const double2* __restrict__ X, double* __restrict__ Z,
                                                             PsOps o, const double2* __restrict__ tw,
                                                             const PsCtl* ctl, int k, double tol) {
    if (ps_halted(ctl, k, tol)) return;
    constexpr int KE = ps_e(L), T = L / KE;
    __shared__ double2 lds[lds_slots(L)];
    __shared__ double2 tw4[tw_slots<L, KE>()];
    load_twiddles<L, KE>(tw, tw4);
    const int m = o.n_out, np = (m + 1) >> 1;
    const int p = xcd_remap(blockIdx.x, np);
    const int ra = 2 * p, rb = 2 * p + 1;
    const bool hasb = rb < m;
    const int tid = threadIdx.x;
    // Z_k = A_k + i B_k for k <= L/2 and Z_{L-k} = conj A_k + i conj B_k (imaginary
    // parts dropped at DC and Nyquist).  Item idx is frequency idx / 2 of row
    // ra + idx mod 2: a lane pair reads the 32 contiguous bytes of one frequency
    // once, swaps its values, the even lane forms Z_k and the odd one Z_{L-k},
    // and LDS takes them to the canonical layout.
    constexpr int NI = (L + 2 + T - 1) / T;
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int idx = tid + it * T;
        const int kk = idx >> 1, r = idx & 1;
        const bool in = kk <= L / 2;
        const double2 v = (in && (r == 0 || hasb)) ? X[(size_t)kk * o.ldx + ra + r] : make_double2(0.0, 0.0);
        // every lane of the wave takes part in the swap (pairs never straddle the range end)
        const double2 u = make_double2(__shfl_xor(v.x, 1), __shfl_xor(v.y, 1));
        const bool real_bin = kk == 0 || kk == L / 2;
        const double2 ta = r == 0 ? v : u, tb = r == 0 ? u : v;
        const double2 ha = make_double2(ta.x, real_bin ? 0.0 : ta.y);
        const double2 hb = make_double2(tb.x, real_bin ? 0.0 : tb.y);
        if (in && r == 0) lds[lds_slot(kk)] = make_double2(ha.x - hb.y, ha.y + hb.x);
        if (in && r == 1 && kk > 0 && kk < L / 2) lds[lds_slot(L - kk)] = make_double2(ha.x + hb.y, hb.x - ha.y);
    }
    __syncthreads();
    double2 reg[KE];
#pragma unroll
    for (int e = 0; e < KE; ++e) reg[e] = lds[lds_slot(tid + e * T)];
    fft_block<L, KE, true>(reg, lds, tw4);
    __syncthreads();
    double* rows = reinterpret_cast<double*>(lds);       // row a at [0, L), row b at [L, 2L)
#pragma unroll
    for (int e = 0; e < KE; ++e) {
        const int j = tid + e * T;
        if (j < m) {
            rows[j] = reg[e].x;
            rows[L + j] = reg[e].y;
        }
    }
    __syncthreads();
    const int n = o.n;
    for (int q = tid; q < n; q += T) {
        const int s = o.tout_s[q];
        const double* w = o.tout_w + 4 * q;
        Z[(size_t)ra * n + q] = w[0] * rows[s] + w[1] * rows[s + 1] + w[2] * rows[s + 2] + w[3] * rows[s + 3];
        if (hasb)
            Z[(size_t)rb * n + q] =
                w[0] * rows[L + s] + w[1] * rows[L + s + 1] + w[2] * rows[L + s + 2] + w[3] * rows[L + s + 3];
    }
}

// Residual of the step equation on grid rows and the axis-2 solve:
// Q = T_2^{-1} (W - Y + c (D Y + B Y - r_omega Y)).  256 threads: 256 / P rows
// per block, P chunks per row (P a power of two, n <= MM P).  Z = nullptr:
// no jumps (B = 0).
template <int MM>
__global__ __launch_bounds__(256) void ps_resid_rows(const double* __restrict__ Y,
                                                            const double* __restrict__ W,
                                                            const double* __restrict__ Z, double* __restrict__ Q,
                                                            PsOps o, PsStepK sk, int P, const PsCtl* ctl, int k,
                                                            double tol) {
    if (ps_halted(ctl, k, tol)) return;
    __shared__ double2 wtot[256];
    const int n = o.n, lpb = 256 / P;
    const int g = threadIdx.x / P, t = threadIdx.x % P;
    const int i = blockIdx.x * lpb + g;
    const int mlen = (n + P - 1) / P;
    const int s = t * mlen;
    const int cnt = i < n ? max(0, min(mlen, n - s)) : 0;
    double x[MM];
#pragma unroll
    for (int q = 0; q < MM; ++q) {
        x[q] = 0.0;
        if (q < cnt) {
            const int j = s + q;
            const size_t o_ = (size_t)i * n + j;
            const double y = Y[o_];
            const double by = Z ? ps_BY(Z, o, i, j) : 0.0;
            x[q] = W[o_] - y + sk.c * (ps_DY(Y, o, i, j) + by - o.r_omega * y);
        }
    }
    chunk_solve<MM>(x, s, cnt, g, t, P, 1, sk.fl2, sk.bu2, sk.bc2, wtot);
#pragma unroll
    for (int q = 0; q < MM; ++q)
        if (q < cnt) Q[(size_t)i * n + s + q] = x[q];
}

// Axis-1 solve of 4 adjacent columns (P chunks each, 4 P threads, P >= 16),
// the update Y += delta (store_delta: delta back into Q instead, for Anderson
// mixing) and the block maximum of |delta| / max(1, |Y + delta|) into err[k]
// (non-negative doubles order like their bit patterns; NaN above inf).
// MM: chunk capacity (at least ceil(n / P)).
template <int MM>
__global__ __launch_bounds__(1024) void ps_line_cols(double* __restrict__ Q, double* __restrict__ Y, PsOps o,
                                                     PsStepK sk, int P, PsCtl* ctl, int k, double tol,
                                                     int store_delta) {
    if (ps_halted(ctl, k, tol)) return;
    __shared__ double2 wtot[256];
    __shared__ double wmax[16];
    const int n = o.n;
    const int c = threadIdx.x & 3, t = threadIdx.x >> 2;
    const int col = blockIdx.x * 4 + c;
    const int mlen = (n + P - 1) / P;
    const int s = t * mlen;
    const int cnt = col < n ? max(0, min(mlen, n - s)) : 0;
    double x[MM];
#pragma unroll
    for (int q = 0; q < MM; ++q) x[q] = q < cnt ? Q[(size_t)(s + q) * n + col] : 0.0;
    chunk_solve<MM>(x, s, cnt, c, t, P, 4, sk.fl1, sk.bu1, sk.bc1, wtot);
    double emax = 0.0;
#pragma unroll
    for (int q = 0; q < MM; ++q) {
        if (q < cnt) {
            const size_t o_ = (size_t)(s + q) * n + col;
            const double y = Y[o_] + x[q];
            if (store_delta) Q[o_] = x[q];        // each thread rewrites the elements it read
            else Y[o_] = y;
            const double ev = fabs(x[q]) / fmax(1.0, fabs(y));
            emax = (ev > emax || ev != ev) ? ev : emax;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double v = __shfl_xor(emax, off, 64);
        emax = (v > emax || v != v) ? v : emax;
    }
    const int nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = emax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = wmax[0];
        for (int w = 1; w < nw; ++w) b = (wmax[w] > b || wmax[w] != wmax[w]) ? wmax[w] : b;
        atomicMax(&ctl->err[k], (unsigned long long)__double_as_longlong(b));
    }
}

// Anderson mixing of the fixed-point iteration.  The paper iterates
// Y_k = Y_{k-1} + delta_k with delta_k = T_1^{-1} T_2^{-1} r(Y_{k-1}) (Sec.
// 3.3); mixing of depth m keeps that fixed point and stopping rule and takes
//   Y_k = Y_{k-1} + delta_k - sum_i gamma_i (dY_i + dF_i),
// gamma = argmin |delta_k - sum_i gamma_i dF_i|_2 over the last m difference
// pairs dF = delta_j - delta_{j-1}, dY = Y_{j-1} - Y_{j-2} of the step's
// iterations (a plain step at k = 1, when err_k already meets tol, and when
// the small system is singular).  gamma solves the normal equations.
constexpr int PS_AA_MAX = 6;          // largest depth
constexpr int PS_AA_T = 256;          // threads of the grid-wide kernels
constexpr int PS_AA_EPT = 4;          // elements per thread

struct PsAA {
    double G[PS_AA_MAX][PS_AA_MAX];   // Gram matrix of the dF columns, by ring slot
    double gamma[PS_AA_MAX];          // coefficients of this iteration, by ring slot (0: unused)
    int mk;                           // columns held (0..m)
    int head;                         // ring slot of the newest column
    int use;                          // gamma valid for this iteration
    int stalls;                       // stalls in this step (two: plain steps to its end)
};

struct PsAABufs {
    const double* F;                  // delta_k (written by the line solves)
    double* Fp;                       // delta_{k-1}
    double* Yp;                       // Y_{k-2}
    double* dF;                       // m ring columns of N
    double* dY;
    double* part;                     // per-block partial sums, nblk x 2m
    PsAA* st;
    int m, nblk;
};

// Part 1, after the line solves of iteration k (Y = Y_{k-1}): the new pair
// into the ring slot after head, each block's partial sums of dF_new . dF_i
// (value i) and dF_i . delta_k (value m + i) over every slot (the new pair in
// its slot), and delta_k, Y_{k-1} kept as the previous ones (k = 1: only
// these).
static __global__ __launch_bounds__(PS_AA_T) void ps_aa_dots(const double* __restrict__ Y, PsAABufs b, size_t N,
                                                           const PsCtl* ctl, int k, double tol) {
    if (ps_halted(ctl, k, tol) || ps_bits(ctl->err[k]) < tol || (k > 1 && b.st->stalls >= 2)) return;
    const int m = b.m, slot = (b.st->head + 1) % m;
    double acc[2 * PS_AA_MAX];
#pragma unroll
    for (int i = 0; i < 2 * PS_AA_MAX; ++i) acc[i] = 0.0;
#pragma unroll
    for (int e = 0; e < PS_AA_EPT; ++e) {
        const size_t idx = ((size_t)blockIdx.x * PS_AA_EPT + e) * PS_AA_T + threadIdx.x;
        if (idx >= N) break;
        const double f = b.F[idx], y = Y[idx];
        if (k > 1) {
            const double dfn = f - b.Fp[idx];
            b.dF[slot * N + idx] = dfn;
            b.dY[slot * N + idx] = y - b.Yp[idx];
#pragma unroll
            for (int i = 0; i < PS_AA_MAX; ++i) {
                if (i >= m) break;
                const double v = i == slot ? dfn : b.dF[i * N + idx];
                acc[i] += dfn * v;
                acc[PS_AA_MAX + i] += v * f;
            }
        }
        b.Fp[idx] = f;
        b.Yp[idx] = y;
    }
    if (k == 1) return;
    // block sums in a fixed order (wave shuffles, then the waves in order)
    __shared__ double red[2 * PS_AA_MAX][PS_AA_T / 64];
#pragma unroll
    for (int i = 0; i < 2 * PS_AA_MAX; ++i) {
        double v = acc[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((threadIdx.x & 63) == 0) red[i][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 2 * m) {
        const int i = threadIdx.x < m ? threadIdx.x : PS_AA_MAX + threadIdx.x - m;
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < PS_AA_T / 64; ++w) v += red[i][w];
        b.part[(size_t)blockIdx.x * 2 * m + threadIdx.x] = v;
    }
}

// Part 2, one block of PS_AA_T threads: the partial sums added in a fixed
// order, the Gram matrix's new row and column, gamma from the normal equations
// (Cholesky, diagonal shifted by 1e-10 of its largest entry).  Safeguards: a
// stopping value that did not decrease since the last iteration (a stall), or
// a non-positive pivot, drops the history and makes this a plain step; after
// the second stall of a step its remaining iterations are plain (near the
// rounding floor the largest increments are rounding noise, which no fit
// removes, and the paper's iteration settles them).  k = 1 starts the step.
static __global__ __launch_bounds__(PS_AA_T) void ps_aa_solve(PsAABufs b, const PsCtl* ctl, int k, double tol) {
    if (ps_halted(ctl, k, tol)) return;
    PsAA& s = *b.st;
    const int m = b.m, nv = 2 * m;
    const double ek = ps_bits(ctl->err[k]);
    const bool stalled = k > 1 && !(ek < ps_bits(ctl->err[k - 1]));
    if (k == 1 || ek < tol || stalled || s.stalls >= 2) {
        if (threadIdx.x == 0) {
            if (k == 1) {
                s.head = m - 1;
                s.stalls = 0;
            }
            if (k == 1 || stalled) s.mk = 0;
            if (stalled) ++s.stalls;
            s.use = 0;
        }
        return;
    }
    __shared__ double red[PS_AA_T];
    __shared__ double d[2 * PS_AA_MAX];
    for (int j = 0; j < nv; ++j) {
        double v = 0.0;
        for (int q = threadIdx.x; q < b.nblk; q += PS_AA_T) v += b.part[(size_t)q * nv + j];
        red[threadIdx.x] = v;
        __syncthreads();
        for (int w = PS_AA_T / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) d[j] = red[0];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const int slot = (s.head + 1) % m;
    for (int i = 0; i < m; ++i) s.G[slot][i] = s.G[i][slot] = d[i];
    s.head = slot;
    s.mk = s.mk < m ? s.mk + 1 : m;
    const int mk = s.mk;
    int c[PS_AA_MAX];
    double A[PS_AA_MAX][PS_AA_MAX], r[PS_AA_MAX], gmax = 0.0;
    for (int q = 0; q < mk; ++q) {
        c[q] = (slot - q + m) % m;            // newest first
        gmax = fmax(gmax, s.G[c[q]][c[q]]);
    }
    for (int q = 0; q < mk; ++q) {
        for (int t = 0; t < mk; ++t) A[q][t] = s.G[c[q]][c[t]];
        A[q][q] += 1e-10 * gmax;
        r[q] = d[m + c[q]];
    }
    bool ok = gmax > 0.0 && gmax == gmax;
    for (int j = 0; j < mk && ok; ++j) {      // A = R^T R, R upper triangular in A
        double sum = A[j][j];
        for (int q = 0; q < j; ++q) sum -= A[q][j] * A[q][j];
        if (!(sum > 0.0)) {
            ok = false;
            break;
        }
        A[j][j] = sqrt(sum);
        for (int t = j + 1; t < mk; ++t) {
            double v = A[j][t];
            for (int q = 0; q < j; ++q) v -= A[q][j] * A[q][t];
            A[j][t] = v / A[j][j];
        }
    }
    for (int i = 0; i < PS_AA_MAX; ++i) s.gamma[i] = 0.0;
    if (!ok) {
        s.mk = 0;
        s.use = 0;
        return;
    }
    double z[PS_AA_MAX];
    for (int j = 0; j < mk; ++j) {            // R^T z = r
        double v = r[j];
        for (int q = 0; q < j; ++q) v -= A[q][j] * z[q];
        z[j] = v / A[j][j];
    }
    for (int j = mk - 1; j >= 0; --j) {       // R g = z
        double v = z[j];
        for (int t = j + 1; t < mk; ++t) v -= A[j][t] * s.gamma[c[t]];
        s.gamma[c[j]] = v / A[j][j];
    }
    s.use = 1;
}

// Part 3: Y_k = Y_{k-1} + delta_k - sum_i gamma_i (dY_i + dF_i) (plain step
// without valid gamma).
static __global__ __launch_bounds__(PS_AA_T) void ps_aa_update(double* __restrict__ Y, PsAABufs b, size_t N,
                                                             const PsCtl* ctl, int k, double tol) {
    if (ps_halted(ctl, k, tol)) return;
    const PsAA& s = *b.st;
    const bool mix = s.use && k > 1 && !(ps_bits(ctl->err[k]) < tol);
#pragma unroll
    for (int e = 0; e < PS_AA_EPT; ++e) {
        const size_t idx = ((size_t)blockIdx.x * PS_AA_EPT + e) * PS_AA_T + threadIdx.x;
        if (idx >= N) break;
        double y = Y[idx] + b.F[idx];
        if (mix) {
#pragma unroll
            for (int i = 0; i < PS_AA_MAX; ++i) {
                if (i >= b.m) break;
                const double g = s.gamma[i];
                if (g != 0.0) y -= g * (b.dY[i * N + idx] + b.dF[i * N + idx]);
            }
        }
        Y[idx] = y;
    }
}

// Explicit part E = V + d (D V + B V - r_omega V), d = dt (1 - theta).
static __global__ __launch_bounds__(256) void ps_expl(const double* __restrict__ V, const double* __restrict__ Z,
                                                      double* __restrict__ E, PsOps o, double d,
                                                      const PsCtl* ctl) {
    if (ctl && ctl->fail) return;
    const int n = o.n;
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)n * n) return;
    const int i = int(idx / n), j = int(idx % n);
    const double v = V[idx];
    const double bv = Z ? ps_BY(Z, o, i, j) : 0.0;
    E[idx] = v + d * (ps_DY(V, o, i, j) + bv - o.r_omega * v);
}

// Semi-Lagrangian step and start value of a step.
struct PsSL {
    const int *s1, *s2;             // per node: stencil starts of the departure points, axis 1 / axis 2
    const double *w1, *w2;          // and their 4 weights
    const double* src;              // E~ = src + rho (src - wp) (wp = nullptr: E~ = src)
    const double* wp;
    double rho;
    double* W;                      // W = (T^SL_1 (x) T^SL_2) E~
    const double* H[4];             // Y^0 = sum_q coef_q H_q
    double coef[4];
    int nh;
    double* Y;
};

static __global__ __launch_bounds__(256) void ps_sl(PsOps o, PsSL a, const PsCtl* ctl) {
    if (ctl->fail) return;
    const int n = o.n;
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)n * n) return;
    const int i = int(idx / n), j = int(idx % n);
    const int s1 = a.s1[i], s2 = a.s2[j];
    const double* w1 = a.w1 + 4 * i;
    const double* w2 = a.w2 + 4 * j;
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const size_t rowo = (size_t)(s1 + t) * n + s2;
        double r = 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            double e = a.src[rowo + u];
            if (a.wp) e += a.rho * (e - a.wp[rowo + u]);
            r += w2[u] * e;
        }
        acc += w1[t] * r;
    }
    a.W[idx] = acc;
    double y = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (q < a.nh) y += a.coef[q] * a.H[q][idx];
    a.Y[idx] = y;
}

// End of step s after kmax iterations: the first k with err_k < tol becomes
// the step's count and err is cleared for the next step; without one the
// failure flag is set (2 if an increment was not finite) and err is kept, so
// that the host can add iterations.  One thread.
static __global__ void ps_step_end(PsCtl* ctl, int* counts, int s, int kmax, double tol) {
    if (ctl->fail) return;
    int kc = 0;
    bool nan = false;
    for (int k = 1; k <= kmax; ++k) {
        const double e = ps_bits(ctl->err[k]);
        if (e != e) nan = true;
        if (kc == 0 && e < tol) kc = k;
    }
    if (kc == 0) {
        ctl->fail = nan ? 2 : 1;
        counts[s] = 0;
        return;
    }
    counts[s] = kc;
    ctl->last = ctl->err[kc];
    for (int k = 0; k < PS_MAXK + 2; ++k) ctl->err[k] = 0ull;
}

static __global__ void ps_ctl_reset(PsCtl* ctl, int clear_err) {
    ctl->fail = 0;
    if (clear_err) {
        for (int k = 0; k < PS_MAXK + 2; ++k) ctl->err[k] = 0ull;
        ctl->last = 0ull;
    }
}

// Stand-alone product: bv = T^out Z (axis 1).
static __global__ __launch_bounds__(256) void ps_tout1(const double* __restrict__ Z, double* __restrict__ bv,
                                                       PsOps o) {
    const int n = o.n;
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)n * n) return;
    bv[idx] = ps_BY(Z, o, int(idx / n), int(idx % n));
}

static __global__ __launch_bounds__(256) void ps_fill(double* __restrict__ a, size_t cnt, double v) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < cnt) a[i] = v;
}

// Delta and Gamma surfaces by the difference schemes of D (Sec. 3.2.1):
// out = [delta1, delta2, gamma11, gamma12, gamma22], each n x n; D1c, D2c hold
// the three coefficients per node (zero where the scheme drops a term).
static __global__ __launch_bounds__(256) void ps_greeks(const double* __restrict__ V, double* __restrict__ out,
                                                        int n, const double* __restrict__ D1c,
                                                        const double* __restrict__ D2c) {
    const size_t N = (size_t)n * n;
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= N) return;
    const int i = int(idx / n), j = int(idx % n);
    const int ii[3] = {i > 0 ? i - 1 : 0, i, i < n - 1 ? i + 1 : n - 1};
    const int jj[3] = {j > 0 ? j - 1 : 0, j, j < n - 1 ? j + 1 : n - 1};
    const double* a1 = D1c + 3 * i;
    const double* b1 = D2c + 3 * i;
    const double* a2 = D1c + 3 * j;
    const double* b2 = D2c + 3 * j;
    double d1 = 0.0, d2 = 0.0, g11 = 0.0, g12 = 0.0, g22 = 0.0;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const double vi = V[(size_t)ii[t] * n + j], vj = V[(size_t)i * n + jj[t]];
        d1 += a1[t] * vi;
        g11 += b1[t] * vi;
        d2 += a2[t] * vj;
        g22 += b2[t] * vj;
        double r = 0.0;
#pragma unroll
        for (int u = 0; u < 3; ++u) r += a2[u] * V[(size_t)ii[t] * n + jj[u]];
        g12 += a1[t] * r;
    }
    out[idx] = d1;
    out[N + idx] = d2;
    out[2 * N + idx] = g11;
    out[3 * N + idx] = g12;
    out[4 * N + idx] = g22;
}

// Prices at spot pairs: tensor-product cubic Lagrange on the four nearest
// nodes of each axis (stencil start clamp(j - 1, 0, n - 4), x_j <= S < x_{j+1}).
__device__ __forceinline__ int ps_stencil(const double* __restrict__ x, int n, double t, double* w) {
    int lo = 0, hi = n;                          // first index with x > t
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (x[mid] <= t) lo = mid + 1; else hi = mid;
    }
    int j = lo - 1;
    j = j < 0 ? 0 : (j > n - 1 ? n - 1 : j);
    int s = j - 1;
    s = s < 0 ? 0 : (s > n - 4 ? n - 4 : s);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        double v = 1.0;
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if (b != a) v *= (t - x[s + b]) / (x[s + a] - x[s + b]);
        w[a] = v;
    }
    return s;
}

static __global__ void ps_price(const double* __restrict__ V, const double* __restrict__ x, int n, int npts,
                                const double* __restrict__ spots, double* __restrict__ price) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npts) return;
    double w1[4], w2[4];
    const int s1 = ps_stencil(x, n, spots[2 * q], w1);
    const int s2 = ps_stencil(x, n, spots[2 * q + 1], w2);
    double acc = 0.0;
    for (int a = 0; a < 4; ++a) {
        double r = 0.0;
        for (int b = 0; b < 4; ++b) r += w2[b] * V[(size_t)(s1 + a) * n + s2 + b];
        acc += w1[a] * r;
    }
    price[q] = acc;
}

}  // namespace ps
}  // namespace lpide
