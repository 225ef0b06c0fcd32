// Workgroup-level Stockham FFT for CDNA4 (gfx950), FP64 and FP32 complex data
// (twiddles always formed in FP64; see twmul).
//
// One workgroup transforms one length-L sequence (L a power of two, 128..8192)
// with T = L/8 threads.  Each thread keeps E = 8 elements in registers in the
// canonical layout reg[e] = element (tid + e*T); the radix-R stages (radix 8,
// plus one radix-2 or radix-4 stage when log2 L is not a multiple of 3)
// exchange data through one LDS buffer of L complex values (plus padding).  Input and output
// of the whole transform are in the canonical layout, so a load or store of
// element (tid + e*T) by thread tid is coalesced, and the output registers of a
// forward transform are the input registers of an inverse transform, which
// lets a pointwise spectrum multiply sit between the two without touching LDS.
//
// The stage (Stockham autosort, Ns = product of the radices already applied):
//   butterfly j, k = j mod Ns: v_r = x[j + r L/R] * W_{Ns R}^{r k},
//   R-point DFT of v, y[(j - k) R + k + r Ns] = v_r.
// Twiddles W_N^m = exp(-+2 pi i m / N): per stage only W_N^k is stored in LDS
// (see TwTab), its powers are formed in registers; conjugated for the inverse.
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

// LDS slot of exchange element a: one pad slot per 16 elements.  Spreads the
// radix-8 stage writes (stride 8 elements in the first stage) over distinct
// banks while keeping the contiguous stage reads conflict free.  The exchange
// buffer needs lds_slots(L) elements.
__device__ __forceinline__ int lds_slot(int a) { return a + (a >> 4); }
constexpr int lds_slots(int L) { return L + L / 16; }

// v * w for a twiddle w computed in FP64.  FP64 data: a complex product.  FP32
// data: compensated product v (w_hi + w_lo) with w_hi = fl32(w) and
// w_lo = fl32(w - w_hi), so the twiddle enters with FP64 accuracy and only the
// FP32 arithmetic rounds.
__device__ __forceinline__ double2 twmul(double2 v, double2 w) { return cmul(v, w); }
__device__ __forceinline__ float2 twmul(float2 v, double2 w) {
    const float hx = (float)w.x, hy = (float)w.y;
    const float lx = (float)(w.x - (double)hx), ly = (float)(w.y - (double)hy);
    const float2 a = cmul(v, make_float2(hx, hy));
    const float2 b = cmul(v, make_float2(lx, ly));
    return make_float2(a.x + b.x, a.y + b.y);
}

// Stage twiddle tables.  Stage s >= 1 is always radix 8 with Ns = R0 8^(s-1)
// (R0 the radix of stage 0); its butterfly k needs W^r = exp(-+2 pi i r k / (8 Ns)),
// r = 1..7.  Only the base W = exp(-2 pi i k / (8 Ns)), k in [0, Ns), is stored
// (stage tables concatenated, k contiguous, so a wave reads consecutive
// entries without bank conflicts); the powers W^2..W^7 are formed in registers
// with at most three complex products each.
template <int L>
struct TwTab {
    static constexpr int LOG = ilog2c(L);
    static constexpr int R0 = (LOG % 3 == 1) ? 2 : (LOG % 3 == 2) ? 4 : 8;
    static constexpr int NST = LOG / 3 + (LOG % 3 ? 1 : 0);
    // Ns of stage s and the offset of its table (sum of Ns over stages 1..s-1);
    // closed forms, so runtime uses compile to shifts (no recursion on the device)
    static constexpr __host__ __device__ int ns(int s) { return s == 0 ? 1 : R0 << (3 * (s - 1)); }
    static constexpr __host__ __device__ int off(int s) { return s <= 1 ? 0 : R0 * ((1 << (3 * (s - 1))) - 1) / 7; }
    static constexpr int size = off(NST);           // entries over stages 1..NST-1
};
template <int L>
constexpr int tw_slots() { return TwTab<L>::size; }

// Build the stage tables in LDS from the full table tw[q] = exp(-2 pi i q / L);
// visible to the FFT stages after the next barrier (stage 0 needs none).
template <int L>
__device__ __forceinline__ void load_twiddles(const double2* __restrict__ tw, double2* tab) {
    using TT = TwTab<L>;
    for (int i = threadIdx.x; i < TT::size; i += L / 8) {
        int s = 1;
#pragma unroll
        for (int q = 2; q < TT::NST; ++q)
            if (i >= TT::off(q)) s = q;
        const int k = i - TT::off(s);
        tab[i] = tw[k * (L / (TT::ns(s) * 8))];
    }
}

// One Stockham stage.  Preconditions: if !FIRST, the previous stage's LDS writes
// are complete and visible (barrier).  Postcondition: if !LAST, this stage's
// LDS writes are complete and visible; if LAST, the result is in reg.
template <int L, int R, bool INV, bool FIRST, bool LAST, typename C>
__device__ __forceinline__ void fft_stage(C (&reg)[8], C* lds, int Ns, int toff, const double2* tab) {
    constexpr int T = L / 8;
    constexpr int NB = 8 / R;          // butterflies per thread
    const int tid = threadIdx.x;
    if constexpr (!FIRST) {
#pragma unroll
        for (int e = 0; e < 8; ++e) reg[e] = lds[lds_slot(tid + e * T)];
    }
    if constexpr (!LAST) __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = tid + b * T;
        const int k = j & (Ns - 1);
        C v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = reg[b + r * NB];
        if constexpr (!FIRST) {
            static_assert(R == 8, "stages after the first are radix 8");
            const double2 t = tab[toff + k];
            const double2 w1 = make_double2(t.x, INV ? -t.y : t.y);
            const double2 w2 = cmul(w1, w1), w3 = cmul(w2, w1), w4 = cmul(w2, w2);
            v[1] = twmul(v[1], w1);
            v[2] = twmul(v[2], w2);
            v[3] = twmul(v[3], w3);
            v[4] = twmul(v[4], w4);
            v[5] = twmul(v[5], cmul(w4, w1));
            v[6] = twmul(v[6], cmul(w4, w2));
            v[7] = twmul(v[7], cmul(w4, w3));
        }
        dft<R, INV>(v);
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) reg[b + r * NB] = v[r];
        } else {
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[lds_slot(base + r * Ns)] = v[r];
        }
    }
    if constexpr (!LAST) __syncthreads();
}

template <int L, bool INV, int S, int NST, typename C>
__device__ __forceinline__ void fft_stages(C (&reg)[8], C* lds, const double2* tab) {
    using TT = TwTab<L>;
    constexpr int R = S == 0 ? TT::R0 : 8;
    fft_stage<L, R, INV, S == 0, S == NST - 1>(reg, lds, TT::ns(S), S == 0 ? 0 : TT::off(S), tab);
    if constexpr (S + 1 < NST) fft_stages<L, INV, S + 1, NST>(reg, lds, tab);
}

// Unnormalised length-L transform of the workgroup's sequence held in the
// canonical register layout; INV selects exp(+2 pi i jk / L).  tab holds the
// stage twiddle tables in LDS, written (load_twiddles) before the call; the
// first stage needs no twiddles and its barrier publishes them.  After
// return, other threads may still read LDS: barrier before reusing it.
template <int L, bool INV, typename C>
__device__ __forceinline__ void fft_block(C (&reg)[8], C* lds, const double2* tab) {
    constexpr int LOG = ilog2c(L);
    constexpr int NST = LOG / 3 + (LOG % 3 ? 1 : 0);
    static_assert((1 << LOG) == L && L >= 64, "L must be a power of two >= 64");
    fft_stages<L, INV, 0, NST>(reg, lds, tab);
}

}  // namespace lpide
