// Exact tridiagonal line solves with constant factors, parallel over chunks.
//
// T x = r with T = L U (Thomas factors precomputed on the host) is
//   forward:  y_i = r_i + fl_i y_{i-1}           (fl_0 = 0)
//   backward: x_i = bu_i y_i + bc_i x_{i+1}      (bc_{n-1} = 0).
// A line is cut into P chunks of at most m consecutive elements, one chunk per
// thread, held in registers.  Each chunk runs its recurrence from a zero carry
// and summarises itself as the affine map carry_out = G carry_in + B; an
// exclusive scan of these maps over the chunks gives every chunk its true
// carry-in, and a fix-up adds carry_in times the running product of the
// multipliers.  The result equals the sequential recurrence up to rounding.
#pragma once

#include <hip/hip_runtime.h>

namespace lpide {

constexpr int LINE_MM = 32;   // max chunk length held in registers

// Exclusive scan of affine maps over t = 0..P-1 for groups of P threads (group g
// uses slots [g*P, g*P + P) of buf; buf holds 2 * nslots double2).  All threads
// of the block must call it.  Returns (M_{t-1} o ... o M_0)(0).
__device__ __forceinline__ double scan_affine(double G, double B, int g, int t, int P, int nslots,
                                              double2* buf) {
    double2* cur = buf;
    double2* nxt = buf + nslots;
    const int s = g * P + t;
    cur[s] = make_double2(G, B);
    __syncthreads();
    for (int d = 1; d < P; d <<= 1) {
        double2 me = cur[s];
        if (t >= d) {
            const double2 pr = cur[s - d];
            me = make_double2(me.x * pr.x, me.x * pr.y + me.y);
        }
        nxt[s] = me;
        __syncthreads();
        double2* tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    const double carry = t > 0 ? cur[s - 1].y : 0.0;
    __syncthreads();
    return carry;
}

// Solve the chunk x[0..m) (factor indices i0..i0+m-1) of a line; x holds the
// right-hand side on entry and the solution on exit.  Every thread of the block
// must call it (m may be 0).
__device__ __forceinline__ void chunk_solve(double (&x)[LINE_MM], int i0, int m, int g, int t, int P, int nslots,
                                            const double* __restrict__ fl, const double* __restrict__ bu,
                                            const double* __restrict__ bc, double2* buf) {
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
    const double yin = scan_affine(G, y, g, t, P, nslots, buf);
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
    const double xin = scan_affine(H, xh, g, P - 1 - t, P, nslots, buf);
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
