// Exact tridiagonal line solves with constant factors, parallel over chunks.
//
// T x = r with T = L U (Thomas factors precomputed on the host) is
//   forward:  y_i = r_i + fl_i y_{i-1}           (fl_0 = 0)
//   backward: x_i = bu_i y_i + bc_i x_{i+1}      (bc_{n-1} = 0).
// A line is cut into P chunks of at most m consecutive elements, one chunk per
// thread, held in registers.  Each chunk runs its recurrence from a zero carry
// and summarises itself as the affine map carry_out = G carry_in + B; an
// exclusive scan of these maps over the chunks (wave shuffles, then one LDS
// round between waves) gives every chunk its true carry-in, and a fix-up adds
// carry_in times the running product of the multipliers.  The result equals
// the sequential recurrence up to rounding.
#pragma once

#include <hip/hip_runtime.h>

namespace lpide {

constexpr int LINE_MM = 32;   // max chunk length held in registers

// Exclusive scan of affine maps y_out = G y_in + B over the chunks t = 0..P-1 of
// a line (in reverse chunk order if REV).  Chunk t of line g is held by the
// lane that sits dl lanes after the holder of chunk t-1 inside a wave; runs of
// CW consecutive chunks, CW the largest power of two dividing P that is at most
// 64/dl, sit inside one wave (a line's first chunk sits at a lane that is a
// multiple of CW dl).  The scan runs inside each run with lane shuffles
// (log2 CW rounds), then the runs of a line combine their totals through LDS
// (wtot: lines x P/CW double2).  All threads of the block must call it.  Returns the carry-in
// (M_{t-1} o ... o M_0)(0) (reverse order if REV).
template <bool REV>
__device__ __forceinline__ double scan_affine(double G, double B, int g, int t, int P, int dl, double2* wtot) {
    const int CW = min(P & -P, 64 / dl);
    const int NW = P / CW;
    const int pos = t % CW;
    const int tl = REV ? CW - 1 - pos : pos;           // position in scan order inside the wave run
    for (int d = 1; d < CW; d <<= 1) {
        const double pg = REV ? __shfl_down(G, d * dl) : __shfl_up(G, d * dl);
        const double pb = REV ? __shfl_down(B, d * dl) : __shfl_up(B, d * dl);
        if (tl >= d) {
            B = G * pb + B;                              // (later o earlier)
            G = G * pg;
        }
    }
    // exclusive inside the run: inclusive value of the previous chunk in scan order
    double eg = REV ? __shfl_down(G, dl) : __shfl_up(G, dl);
    double eb = REV ? __shfl_down(B, dl) : __shfl_up(B, dl);
    if (tl == 0) { eg = 1.0; eb = 0.0; }
    const int wr = REV ? NW - 1 - t / CW : t / CW;      // run index in scan order
    if (tl == CW - 1) wtot[g * NW + wr] = make_double2(G, B);
    __syncthreads();
    double ypre = 0.0;
    for (int q = 0; q < wr; ++q) {
        const double2 m = wtot[g * NW + q];
        ypre = m.x * ypre + m.y;
    }
    __syncthreads();
    return eg * ypre + eb;
}

// Solve the chunk x[0..m) (factor indices i0..i0+m-1) of a line; x holds the
// right-hand side on entry and the solution on exit.  Every thread of the block
// must call it (m may be 0); (g, t, P, dl) place the chunk for scan_affine.
__device__ __forceinline__ void chunk_solve(double (&x)[LINE_MM], int i0, int m, int g, int t, int P, int dl,
                                            const double* __restrict__ fl, const double* __restrict__ bu,
                                            const double* __restrict__ bc, double2* wtot) {
    double y = 0.0, G = 1.0;
#pragma unroll
    for (int k = 0; k < LINE_MM; ++k) {
        if (k < m) {
            const double f = fl[i0 + k];
            y = x[k] + f * y;
            G *= f;
            x[k] = y;
        }
    }
    const double yin = scan_affine<false>(G, y, g, t, P, dl, wtot);
    double gp = 1.0;
#pragma unroll
    for (int k = 0; k < LINE_MM; ++k) {
        if (k < m) {
            gp *= fl[i0 + k];
            x[k] += gp * yin;
        }
    }
    double xh = 0.0, H = 1.0;
#pragma unroll
    for (int k = LINE_MM - 1; k >= 0; --k) {
        if (k < m) {
            const double c = bc[i0 + k];
            xh = bu[i0 + k] * x[k] + c * xh;
            H *= c;
            x[k] = xh;
        }
    }
    const double xin = scan_affine<true>(H, xh, g, t, P, dl, wtot);
    double hp = 1.0;
#pragma unroll
    for (int k = LINE_MM - 1; k >= 0; --k) {
        if (k < m) {
            hp *= bc[i0 + k];
            x[k] += hp * xin;
        }
    }
}

}  // namespace lpide
