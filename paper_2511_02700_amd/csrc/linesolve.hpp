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

constexpr int LINE_W = 8;     // factor reads kept in flight ahead of a recurrence

// Factor reads through the global address space: global (not flat) loads,
// whose waits count memory operations only and retire in order, so that a
// wait for one factor does not drain the reads issued after it.
using gdouble = __attribute__((address_space(1))) const double;

// Solve the chunk x[0..m) (factor indices i0..i0+m-1, m <= MM) of a line; x
// holds the right-hand side on entry and the solution on exit (x[m..MM) is
// left undefined).  Every thread of the block must call it (m may be 0); (g, t, P,
// dl) place the chunk for scan_affine.  The factor arrays are global memory
// and readable MM - 1 elements past the line's end (their zero tail of
// kLinePad >= LINE_MM elements).
//
// The recurrences depend element to element, their factors do not: every
// sweep reads its factors LINE_W elements ahead into a ring of registers (the
// scheduling fences keep the reads there instead of all at the top), so the
// recurrence waits for memory about once per sweep instead of once per
// element.  The sweeps run over all LINE_MM slots without branches; past the
// chunk's end the factors are replaced by ones that make a step the identity
// (fl = 1 and r = 0 forward, bu = 0 and bc = 1 backward), so the chunk's
// affine summary is that of its m elements.
template <int MM = LINE_MM>
__device__ __forceinline__ void chunk_solve(double (&x)[MM], int i0, int m, int g, int t, int P, int dl,
                                            const double* __restrict__ fl, const double* __restrict__ bu,
                                            const double* __restrict__ bc, double2* wtot) {
    // reads ahead at most the capacity: every factor read of the chunk then
    // lies in [i0, i0 + MM) (the backward sweeps start MM - 1 past i0)
    constexpr int W = LINE_W < MM ? LINE_W : MM;
    const int b = m > 0 ? i0 : 0;                     // chunks past the line's end read from its start
    const gdouble* F = (const gdouble*)(fl + b);
    const gdouble* U = (const gdouble*)(bu + b);
    const gdouble* C = (const gdouble*)(bc + b);
    double w[W], v[W];
    // forward sweep y_k = r_k + fl_k y_{k-1} from a zero carry
#pragma unroll
    for (int k = 0; k < W; ++k) w[k] = F[k];
    double y = 0.0, G = 1.0;
#pragma unroll
    for (int k = 0; k < MM; ++k) {
        const double f = k < m ? w[k % W] : 1.0, r = k < m ? x[k] : 0.0;
        if (k + W < MM) w[k % W] = F[k + W];
        y = r + f * y;
        G *= f;
        x[k] = y;
        __builtin_amdgcn_sched_barrier(0);
    }
    const double yin = scan_affine<false>(G, y, g, t, P, dl, wtot);
    // the fix-ups read the factors again (cache hits): an opaque copy of the
    // offset keeps the compiler from merging these reads with the sweep's and
    // holding all MM factors in registers across the scan
    int b2 = b;
    asm volatile("" : "+v"(b2));
    F = (const gdouble*)(fl + b2);
#pragma unroll
    for (int k = 0; k < W; ++k) w[k] = F[k];
    double gp = 1.0;
#pragma unroll
    for (int k = 0; k < MM; ++k) {
        const double f = k < m ? w[k % W] : 1.0;
        if (k + W < MM) w[k % W] = F[k + W];
        gp *= f;
        x[k] += gp * yin;
        __builtin_amdgcn_sched_barrier(0);
    }
    // backward sweep x_k = bu_k y_k + bc_k x_{k+1} from a zero carry (q counts down from the last slot)
#pragma unroll
    for (int q = 0; q < W; ++q) {
        w[q] = U[MM - 1 - q];
        v[q] = C[MM - 1 - q];
    }
    double xh = 0.0, H = 1.0;
#pragma unroll
    for (int q = 0; q < MM; ++q) {
        const int k = MM - 1 - q;
        const double u = k < m ? w[q % W] : 0.0, c = k < m ? v[q % W] : 1.0;
        if (q + W < MM) {
            w[q % W] = U[k - W];
            v[q % W] = C[k - W];
        }
        xh = u * x[k] + c * xh;
        H *= c;
        x[k] = xh;
        __builtin_amdgcn_sched_barrier(0);
    }
    const double xin = scan_affine<true>(H, xh, g, t, P, dl, wtot);
    int b3 = b;
    asm volatile("" : "+v"(b3));
    C = (const gdouble*)(bc + b3);
#pragma unroll
    for (int q = 0; q < W; ++q) v[q] = C[MM - 1 - q];
    double hp = 1.0;
#pragma unroll
    for (int q = 0; q < MM; ++q) {
        const int k = MM - 1 - q;
        const double c = k < m ? v[q % W] : 1.0;
        if (q + W < MM) v[q % W] = C[k - W];
        hp *= c;
        x[k] += hp * xin;
        __builtin_amdgcn_sched_barrier(0);
    }
}

}  // namespace lpide
