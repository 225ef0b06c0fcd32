// Workgroup-level Stockham FFT for CDNA4 (gfx950), FP64 and FP32 complex.
//
// One workgroup transforms one length-L sequence (L a power of two, 128..8192)
// with T = L/8 threads.  Each thread keeps E = 8 elements in registers in the
// canonical layout reg[e] = element (tid + e*T); the radix-R stages (radix 8,
// plus one radix-2 or radix-4 stage when log2 L is not a multiple of 3)
// exchange data through one LDS buffer of L complex values.  Input and output
// of the whole transform are in the canonical layout, so a load or store of
// element (tid + e*T) by thread tid is coalesced, and the output registers of a
// forward transform are the input registers of an inverse transform, which
// lets a pointwise spectrum multiply sit between the two without touching LDS.
//
// The stage (Stockham autosort, Ns = product of the radices already applied):
//   butterfly j, k = j mod Ns: v_r = x[j + r L/R] * W_{Ns R}^{r k},
//   R-point DFT of v, y[(j - k) R + k + r Ns] = v_r.
// Twiddles W_N^m = exp(-+2 pi i m / N) come from the table exp(-2 pi i q / L)
// (q = m L / N), kept in LDS as its first quarter (the other three quarters
// follow by multiplying with -i), conjugated for the inverse transform.
#pragma once

#include <hip/hip_runtime.h>

namespace lpide {

template <typename R2>
struct CplxOps;

template <>
struct CplxOps<double2> {
    using real = double;
    static __device__ __forceinline__ double2 make(double x, double y) { return make_double2(x, y); }
};
template <>
struct CplxOps<float2> {
    using real = float;
    static __device__ __forceinline__ float2 make(float x, float y) { return make_float2(x, y); }
};

template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { return CplxOps<C>::make(a.x + b.x, a.y + b.y); }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { return CplxOps<C>::make(a.x - b.x, a.y - b.y); }
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
    return CplxOps<C>::make(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename C>
__device__ __forceinline__ C cmulc(C a, C b) {
    return CplxOps<C>::make(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C>
__device__ __forceinline__ C mul_mi(C a) {
    return INV ? CplxOps<C>::make(-a.y, a.x) : CplxOps<C>::make(a.y, -a.x);
}

template <bool INV, typename C>
__device__ __forceinline__ void dft2(C* v) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <bool INV, typename C>
__device__ __forceinline__ void dft4(C& v0, C& v1, C& v2, C& v3) {
    C t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), t3 = mul_mi<INV>(csub(v1, v3));
    v0 = cadd(t0, t2);
    v2 = csub(t0, t2);
    v1 = cadd(t1, t3);
    v3 = csub(t1, t3);
}

template <bool INV, typename C>
__device__ __forceinline__ void dft4(C* v) { dft4<INV>(v[0], v[1], v[2], v[3]); }

template <bool INV, typename C>
__device__ __forceinline__ void dft8(C* v) {
    using Rl = typename CplxOps<C>::real;
    const Rl s = Rl(0.70710678118654752440084436210484904);
    C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<INV>(e0, e1, e2, e3);
    dft4<INV>(o0, o1, o2, o3);
    // o_k *= W_8^k ; forward W_8 = (1 - i)/sqrt2, inverse its conjugate
    C w1 = INV ? CplxOps<C>::make(s * (o1.x - o1.y), s * (o1.x + o1.y))
               : CplxOps<C>::make(s * (o1.x + o1.y), s * (o1.y - o1.x));
    C w2 = mul_mi<INV>(o2);
    C w3 = INV ? CplxOps<C>::make(-s * (o3.x + o3.y), s * (o3.x - o3.y))
               : CplxOps<C>::make(s * (o3.y - o3.x), -s * (o3.x + o3.y));
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, w1);
    v[5] = csub(e1, w1);
    v[2] = cadd(e2, w2);
    v[6] = csub(e2, w2);
    v[3] = cadd(e3, w3);
    v[7] = csub(e3, w3);
}

template <int R, bool INV, typename C>
__device__ __forceinline__ void dft(C* v) {
    if constexpr (R == 2) dft2<INV>(v);
    else if constexpr (R == 4) dft4<INV>(v);
    else dft8<INV>(v);
}

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }

// Twiddle exp(-+2 pi i q / L), q in [0, L), from a quarter table
// tw4[r] = exp(-2 pi i r / L), r in [0, L/4) (held in LDS): exp(-2 pi i q / L) =
// (-i)^quadrant * tw4[q mod L/4]; conjugated for the inverse transform.
template <int L, bool INV, typename C>
__device__ __forceinline__ C twiddle(const C* tw4, int q) {
    using Rl = typename CplxOps<C>::real;
    constexpr int Q = L / 4;
    const C w = tw4[q & (Q - 1)];
    const int quad = q / Q;
    // quadrant 0: w; 1: w (-i) = (y, -x); 2: -w; 3: w (+i) = (-y, x)  (branch-free selects)
    const bool odd = (quad & 1) != 0;
    const Rl a = odd ? w.y : w.x;
    const Rl b = odd ? w.x : w.y;
    const Rl re = quad >= 2 ? -a : a;
    Rl im = (quad == 1 || quad == 2) ? -b : b;
    if (INV) im = -im;
    return CplxOps<C>::make(re, im);
}

// Cooperative load of the quarter twiddle table (first L/4 entries of the full
// table tw) into LDS; visible to the FFT stages after the next barrier.
template <int L, typename C>
__device__ __forceinline__ void load_twiddles(const C* __restrict__ tw, C* tw4) {
    for (int q = threadIdx.x; q < L / 4; q += L / 8) tw4[q] = tw[q];
}

// One Stockham stage.  Preconditions: if !FIRST, the previous stage's LDS writes
// are complete and visible (barrier).  Postcondition: if !LAST, this stage's
// LDS writes are complete and visible; if LAST, the result is in reg.
template <int L, int R, bool INV, bool FIRST, bool LAST, typename C>
__device__ __forceinline__ void fft_stage(C (&reg)[8], C* lds, int Ns, const C* tw4) {
    constexpr int T = L / 8;
    constexpr int NB = 8 / R;          // butterflies per thread
    const int tid = threadIdx.x;
    if constexpr (!FIRST) {
#pragma unroll
        for (int e = 0; e < 8; ++e) reg[e] = lds[tid + e * T];
    }
    if constexpr (!LAST) __syncthreads();
    const int step = L / (Ns * R);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = tid + b * T;
        const int k = j & (Ns - 1);
        C v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = reg[b + r * NB];
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) v[r] = cmul(v[r], twiddle<L, INV>(tw4, r * k * step));
        }
        dft<R, INV>(v);
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) reg[b + r * NB] = v[r];
        } else {
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[base + r * Ns] = v[r];
        }
    }
    if constexpr (!LAST) __syncthreads();
}

template <int L, bool INV, int S, int NST, typename C>
__device__ __forceinline__ void fft_stages(C (&reg)[8], C* lds, int Ns, const C* tw4) {
    constexpr int REM = ilog2c(L) % 3;
    constexpr int R = (S == 0 && REM == 1) ? 2 : (S == 0 && REM == 2) ? 4 : 8;
    fft_stage<L, R, INV, S == 0, S == NST - 1>(reg, lds, Ns, tw4);
    if constexpr (S + 1 < NST) fft_stages<L, INV, S + 1, NST>(reg, lds, Ns * R, tw4);
}

// Unnormalised length-L transform of the workgroup's sequence held in the
// canonical register layout; INV selects exp(+2 pi i jk / L).  tw4 is the
// quarter twiddle table in LDS, written (load_twiddles) before the call; the
// first stage needs no twiddles and its barrier publishes the table.  After
// return, other threads may still read LDS: barrier before reusing it.
template <int L, bool INV, typename C>
__device__ __forceinline__ void fft_block(C (&reg)[8], C* lds, const C* tw4) {
    constexpr int LOG = ilog2c(L);
    constexpr int NST = LOG / 3 + (LOG % 3 ? 1 : 0);
    static_assert((1 << LOG) == L && L >= 64, "L must be a power of two >= 64");
    fft_stages<L, INV, 0, NST>(reg, lds, 1, tw4);
}

}  // namespace lpide
