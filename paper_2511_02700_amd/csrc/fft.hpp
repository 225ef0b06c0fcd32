// Workgroup-level Stockham FFT for CDNA4 (gfx950), FP64 and FP32 complex data
// (twiddles always formed in FP64; see twmul).
//
// One workgroup transforms one length-L sequence, L = 2^m (64..8192) or
// L = 2^m 3^a 5^b 7^c (transform sizes whose largest prime factor is at most
// 7, Sec. 4), with T = L/E threads, E in {4, 8, 16} elements per thread held
// in registers in the canonical layout reg[e] = element (tid + e*T).  The
// power-of-two part is done by radix-E stages plus one smaller first stage
// when its log2 is not a multiple of log2 E; the odd factors are radix-3, 5
// and 7 stages that follow the first stage.  Stages exchange data through one LDS buffer of L
// complex values (plus padding).  Input and output of the whole transform are
// in the canonical layout, so a load or store of element (tid + e*T) by thread
// tid is coalesced, and the output registers of a forward transform are the
// input registers of an inverse transform, which lets a pointwise spectrum
// multiply sit between the two without touching LDS.
//
// The stage (Stockham autosort, Ns = product of the radices already applied):
//   butterfly j, k = j mod Ns: v_r = x[j + r L/R] * W_{Ns R}^{r k},
//   R-point DFT of v, y[(j - k) R + k + r Ns] = v_r.
// Twiddles W_N^m = exp(-+2 pi i m / N): per stage only W_N^k is stored in LDS
// (see TwTab), its powers are formed in registers; conjugated for the inverse.
// The power-of-two stages hold E/R butterflies per thread in registers; the
// odd stages (L/p butterflies, not a multiple of T) read their operands from
// LDS and write back to LDS, so they are never the first stage; when no
// power-of-two stage follows them, the result is read from LDS into the
// canonical registers.
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

// 16-point DFT as 4 x 4: DFT4 over the stride-4 subsequences, twiddles
// W16^{q k}, DFT4 across, output index k + 4 m.
template <bool INV, typename C>
__device__ __forceinline__ void dft16(C* v) {
    using Rl = typename CplxOps<C>::real;
    const Rl c1 = Rl(0.92387953251128675612818318939678829), s1 = Rl(0.38268343236508977172845998403039887);
    const Rl h = Rl(0.70710678118654752440084436210484904);
    C a[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        a[q][0] = v[q];
        a[q][1] = v[q + 4];
        a[q][2] = v[q + 8];
        a[q][3] = v[q + 12];
        dft4<INV>(a[q][0], a[q][1], a[q][2], a[q][3]);   // a[q][k] = sum_m v[q + 4m] W4^{mk}
    }
    // W16^{q k} for q, k in 0..3 (forward sign; conjugated for the inverse)
    auto tw = [&](C x, int e) -> C {
        // e = q k in 0..9: W16^e = cos(2 pi e/16) -/+ i sin(2 pi e/16)
        Rl cr, si;
        switch (e) {
            case 0: return x;
            case 1: cr = c1; si = s1; break;
            case 2: cr = h; si = h; break;
            case 3: cr = s1; si = c1; break;
            case 4: return mul_mi<INV>(x);
            case 6: cr = -h; si = h; break;
            case 9: cr = -c1; si = -s1; break;
            default: cr = 0; si = 0; break;
        }
        const C w = INV ? CplxOps<C>::make(cr, si) : CplxOps<C>::make(cr, -si);
        return cmul(x, w);
    };
#pragma unroll
    for (int q = 1; q < 4; ++q)
#pragma unroll
        for (int k = 1; k < 4; ++k) a[q][k] = tw(a[q][k], q * k);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        C b0 = a[0][k], b1 = a[1][k], b2 = a[2][k], b3 = a[3][k];
        dft4<INV>(b0, b1, b2, b3);                        // across q: output k + 4 m
        v[k] = b0;
        v[k + 4] = b1;
        v[k + 8] = b2;
        v[k + 12] = b3;
    }
}

// 3-point DFT: y0 = v0 + t, y1,2 = v0 - t/2 -+ i sin(2 pi/3) (v1 - v2) (forward;
// signs of the i terms swap for the inverse), t = v1 + v2.
template <bool INV, typename C>
__device__ __forceinline__ void dft3(C* v) {
    using Rl = typename CplxOps<C>::real;
    const Rl s3 = Rl(0.86602540378443864676372317075293618);
    const C t = cadd(v[1], v[2]);
    const C d = mul_mi<INV>(csub(v[1], v[2]));
    const C m = CplxOps<C>::make(v[0].x - Rl(0.5) * t.x, v[0].y - Rl(0.5) * t.y);
    v[0] = cadd(v[0], t);
    v[1] = CplxOps<C>::make(m.x + s3 * d.x, m.y + s3 * d.y);
    v[2] = CplxOps<C>::make(m.x - s3 * d.x, m.y - s3 * d.y);
}

// P-point DFT for odd P (5, 7) in the symmetric form: with A_j = v_j + v_{P-j},
// B_j = v_j - v_{P-j} (j = 1..(P-1)/2), y_0 = v_0 + sum A_j and, for k = 1..(P-1)/2,
//   y_k = v_0 + sum_j A_j cos(2 pi jk/P) - i sum_j B_j sin(2 pi jk/P),
//   y_{P-k} = v_0 + sum_j A_j cos(2 pi jk/P) + i sum_j B_j sin(2 pi jk/P)
// (forward; the i terms change sign for the inverse).
template <int P>
struct OddRoots;
template <>
struct OddRoots<5> {
    static constexpr double c[3] = {1.0, 0.30901699437494745, -0.8090169943749473};   // cos(2 pi m/5)
    static constexpr double s[3] = {0.0, 0.9510565162951535, 0.5877852522924732};     // sin(2 pi m/5)
};
template <>
struct OddRoots<7> {
    static constexpr double c[4] = {1.0, 0.6234898018587336, -0.22252093395631434, -0.900968867902419};
    static constexpr double s[4] = {0.0, 0.7818314824680298, 0.9749279121818236, 0.43388373911755823};
};

template <int P, bool INV, typename C>
__device__ __forceinline__ void dft_odd(C* v) {
    using Rl = typename CplxOps<C>::real;
    constexpr int H = (P - 1) / 2;
    C A[H + 1], B[H + 1];
#pragma unroll
    for (int j = 1; j <= H; ++j) {
        A[j] = cadd(v[j], v[P - j]);
        B[j] = csub(v[j], v[P - j]);
    }
    C y[P];
    y[0] = v[0];
#pragma unroll
    for (int j = 1; j <= H; ++j) y[0] = cadd(y[0], A[j]);
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        C a = v[0], b = CplxOps<C>::make(Rl(0), Rl(0));
#pragma unroll
        for (int j = 1; j <= H; ++j) {
            // cos and sin of 2 pi (jk mod P)/P from the half table (sin odd about P/2)
            const int m = (j * k) % P;
            const Rl cm = Rl(OddRoots<P>::c[m <= H ? m : P - m]);
            const Rl sm = m <= H ? Rl(OddRoots<P>::s[m]) : -Rl(OddRoots<P>::s[P - m]);
            a = CplxOps<C>::make(a.x + cm * A[j].x, a.y + cm * A[j].y);
            b = CplxOps<C>::make(b.x + sm * B[j].x, b.y + sm * B[j].y);
        }
        const C d = mul_mi<INV>(b);
        y[k] = cadd(a, d);
        y[P - k] = csub(a, d);
    }
#pragma unroll
    for (int k = 0; k < P; ++k) v[k] = y[k];
}

template <int R, bool INV, typename C>
__device__ __forceinline__ void dft(C* v) {
    if constexpr (R == 2) dft2<INV>(v);
    else if constexpr (R == 4) dft4<INV>(v);
    else if constexpr (R == 8) dft8<INV>(v);
    else dft16<INV>(v);
}

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }

// LDS slot of exchange element a: one pad slot per 16 elements.  Spreads the
// strided stage writes (stride R elements for radix R) over distinct banks
// while keeping the contiguous stage reads conflict free.  The exchange buffer
// needs lds_slots(L) elements.
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

// Odd factor of a transform size: 1 for powers of two, 3 for 3 * 2^m, and so on.
constexpr int fft_odd(int L) { return (L % 2 == 0) ? fft_odd(L / 2) : L; }
// Whether an odd factor has no prime factor above 7.
constexpr bool seven_smooth_odd(int o) {
    return o == 1 ? true : (o % 3 == 0 ? seven_smooth_odd(o / 3)
                                       : (o % 5 == 0 ? seven_smooth_odd(o / 5)
                                                     : (o % 7 == 0 ? seven_smooth_odd(o / 7) : false)));
}

// Whether the kernels run a size-L transform with E elements per thread: the
// workgroup is a power of two (L a power of two), or whole waves (L = 3 * 2^m:
// the block-level reductions and line scans work on whole waves), and a
// radix-3 stage has a power-of-two stage before and after it.
//
// Other odd factors (5, 7, 9, 15, ...; the price-space plan's sides only):
// the power-of-two part holds at least E (a full first stage), and at most
// 1024 threads.
constexpr bool fft_ok(int L, int E) {
    return (E == 4 || E == 8 || (E == 16 && L >= 256)) &&
           (fft_odd(L) == 1 || (fft_odd(L) == 3 && (L / E) % 64 == 0 && L / 3 > E) ||
            (fft_odd(L) != 3 && seven_smooth_odd(fft_odd(L)) && L / fft_odd(L) >= E && L / E <= 1024));
}

// Elements per thread of the stand-alone transform kernels (8 where allowed).
constexpr int conv_e(int L) { return fft_ok(L, 8) ? 8 : 4; }

// Multiplicity of the prime p in m.
constexpr int pcount(int m, int p) { return m % p == 0 ? 1 + pcount(m / p, p) : 0; }

// Stage twiddle tables.  Stage 0 (radix R0, no twiddles); stages 1..NODD are
// the odd factors (radix 3, then 5, then 7; for L = 3 * 2^m the single stage 1
// is radix 3); the others are radix E.  Stage s >= 1 with radix R and
// Ns = R_0 ... R_{s-1} needs, for butterfly k, W^r = exp(-+2 pi i r k / (R Ns)),
// r = 1..R-1.  Only the base W = exp(-2 pi i k / (R Ns)), k in [0, Ns), is
// stored (stage tables concatenated, k contiguous, so a wave reads consecutive
// entries without bank conflicts); the powers are formed in registers with a
// product tree of depth log2 R.  All members are evaluated at compile time:
// callers pass constant stage indices.
template <int L, int E>
struct TwTab {
    static constexpr int ODD = fft_odd(L);
    static constexpr int LOG = ilog2c(L / ODD);     // log2 of the power-of-two part
    static constexpr int LE = ilog2c(E);
    static constexpr int R0 = (LOG % LE) ? (1 << (LOG % LE)) : E;
    static constexpr int NP2 = LOG / LE + (LOG % LE ? 1 : 0);   // power-of-two stages
    static constexpr int N3 = pcount(ODD, 3), N5 = pcount(ODD, 5), N7 = pcount(ODD, 7);
    static constexpr int NODD = N3 + N5 + N7;                    // odd stages 1..NODD
    static constexpr int NST = NP2 + NODD;
    static constexpr int S3 = ODD == 3 ? 1 : -1;                 // the radix-3 stage of L = 3 * 2^m
    static constexpr __host__ __device__ int radix(int s) {
        return s == 0 ? R0 : (s <= N3 ? 3 : (s <= N3 + N5 ? 5 : (s <= NODD ? 7 : E)));
    }
    static constexpr __host__ __device__ int ns(int s) {
        int v = 1;
        for (int q = 0; q < s; ++q) v *= radix(q);
        return v;
    }
    static constexpr __host__ __device__ int off(int s) {
        int v = 0;
        for (int q = 1; q < s; ++q) v += ns(q);
        return v;
    }
    static constexpr int size = off(NST);           // entries over stages 1..NST-1
};
template <int L, int E>
constexpr int tw_slots() { return TwTab<L, E>::size > 0 ? TwTab<L, E>::size : 1; }

// Build the stage tables in LDS from the full table tw[q] = exp(-2 pi i q / L);
// visible to the FFT stages after the next barrier (stage 0 needs none).
template <int L, int E>
__device__ __forceinline__ void load_twiddles(const double2* __restrict__ tw, double2* tab) {
    using TT = TwTab<L, E>;
    for (int i = threadIdx.x; i < TT::size; i += L / E) {
#pragma unroll
        for (int q = 1; q < TT::NST; ++q) {
            if (i >= TT::off(q) && i < TT::off(q + 1))
                tab[i] = tw[(i - TT::off(q)) * (L / (TT::ns(q) * TT::radix(q)))];
        }
    }
}

// W^1..W^{R-1} from W^1 = w1 by a product tree (in FP64).
template <int R>
__device__ __forceinline__ void twiddle_powers(double2 w1, double2 (&w)[R]) {
    w[1] = w1;
    if constexpr (R > 2) w[2] = cmul(w1, w1);
    if constexpr (R > 3) w[3] = cmul(w[2], w1);
    if constexpr (R > 4) {
        w[4] = cmul(w[2], w[2]);
        w[5] = cmul(w[4], w1);
        w[6] = cmul(w[4], w[2]);
        w[7] = cmul(w[4], w[3]);
    }
    if constexpr (R > 8) {
        w[8] = cmul(w[4], w[4]);
#pragma unroll
        for (int r = 9; r < R; ++r) w[r] = cmul(w[8], w[r - 8]);
    }
}

// One power-of-two Stockham stage (radix R, NS = product of the earlier
// radices).  Preconditions: if !FIRST, the previous stage's LDS writes are
// complete and visible (barrier).  Postcondition: if !LAST, this stage's LDS
// writes are complete and visible; if LAST, the result is in reg.
template <int L, int E, int R, int NS, bool INV, bool FIRST, bool LAST, typename C>
__device__ __forceinline__ void fft_stage(C (&reg)[E], C* lds, int toff, const double2* tab) {
    constexpr int T = L / E;
    constexpr int NB = E / R;          // butterflies per thread
    const int tid = threadIdx.x;
    if constexpr (!FIRST) {
#pragma unroll
        for (int e = 0; e < E; ++e) reg[e] = lds[lds_slot(tid + e * T)];
    }
    if constexpr (!LAST) __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = tid + b * T;
        const int k = j % NS;
        C v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = reg[b + r * NB];
        if constexpr (!FIRST) {
            static_assert(R == E, "power-of-two stages after the first are radix E");
            const double2 t = tab[toff + k];
            double2 w[R];
            twiddle_powers<R>(make_double2(t.x, INV ? -t.y : t.y), w);
#pragma unroll
            for (int r = 1; r < R; ++r) v[r] = twmul(v[r], w[r]);
        }
        dft<R, INV>(v);
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) reg[b + r * NB] = v[r];
        } else {
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[lds_slot(base + r * NS)] = v[r];
        }
    }
    if constexpr (!LAST) __syncthreads();
}

// The radix-3 stage, LDS to LDS (same pre- and postcondition as a middle
// stage): L/3 butterflies, thread tid takes j = tid, tid + T, ...
template <int L, int E, int NS, bool INV, typename C>
__device__ __forceinline__ void fft_stage3(C* lds, int toff, const double2* tab) {
    constexpr int T = L / E;
    constexpr int NBF = L / 3;
    constexpr int MB = (NBF + T - 1) / T;
    const int tid = threadIdx.x;
    C v[MB][3];
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        const int j = tid + b * T;
        if (j < NBF) {
#pragma unroll
            for (int r = 0; r < 3; ++r) v[b][r] = lds[lds_slot(j + r * NBF)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        const int j = tid + b * T;
        if (j < NBF) {
            const int k = j % NS;
            const double2 t = tab[toff + k];
            const double2 w1 = make_double2(t.x, INV ? -t.y : t.y);
            v[b][1] = twmul(v[b][1], w1);
            v[b][2] = twmul(v[b][2], cmul(w1, w1));
            dft3<INV>(v[b]);
            const int base = (j - k) * 3 + k;
#pragma unroll
            for (int r = 0; r < 3; ++r) lds[lds_slot(base + r * NS)] = v[b][r];
        }
    }
    __syncthreads();
}

// A radix-5 or radix-7 stage, LDS to LDS like the radix-3 stage: L/P
// butterflies, thread tid takes j = tid, tid + T, ...; twiddle powers by
// repeated products of the base W^k (in FP64).
template <int L, int E, int P, int NS, bool INV, typename C>
__device__ __forceinline__ void fft_stage_odd(C* lds, int toff, const double2* tab) {
    constexpr int T = L / E;
    constexpr int NBF = L / P;
    constexpr int MB = (NBF + T - 1) / T;
    const int tid = threadIdx.x;
    C v[MB][P];
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        const int j = tid + b * T;
        if (j < NBF) {
#pragma unroll
            for (int r = 0; r < P; ++r) v[b][r] = lds[lds_slot(j + r * NBF)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        const int j = tid + b * T;
        if (j < NBF) {
            const int k = j % NS;
            const double2 t = tab[toff + k];
            const double2 w1 = make_double2(t.x, INV ? -t.y : t.y);
            double2 w = w1;
#pragma unroll
            for (int r = 1; r < P; ++r) {
                v[b][r] = twmul(v[b][r], w);
                w = cmul(w, w1);
            }
            dft_odd<P, INV>(v[b]);
            const int base = (j - k) * P + k;
#pragma unroll
            for (int r = 0; r < P; ++r) lds[lds_slot(base + r * NS)] = v[b][r];
        }
    }
    __syncthreads();
}

template <int L, int E, bool INV, int S, int NST, typename C>
__device__ __forceinline__ void fft_stages(C (&reg)[E], C* lds, const double2* tab) {
    using TT = TwTab<L, E>;
    constexpr int R = TT::radix(S), NS = TT::ns(S), OFF = TT::off(S);
    constexpr bool ODDSTAGE = S >= 1 && S <= TT::NODD;
    if constexpr (ODDSTAGE && R == 3) fft_stage3<L, E, NS, INV>(lds, OFF, tab);
    else if constexpr (ODDSTAGE) fft_stage_odd<L, E, R, NS, INV>(lds, OFF, tab);
    else fft_stage<L, E, R, NS, INV, S == 0, S == NST - 1>(reg, lds, OFF, tab);
    if constexpr (S + 1 < NST) {
        fft_stages<L, E, INV, S + 1, NST>(reg, lds, tab);
    } else if constexpr (ODDSTAGE) {
        // the last stage was an odd one: the result into the canonical registers
        constexpr int T = L / E;
#pragma unroll
        for (int e = 0; e < E; ++e) reg[e] = lds[lds_slot(threadIdx.x + e * T)];
    }
}

// Unnormalised length-L transform of the workgroup's sequence held in the
// canonical register layout; INV selects exp(+2 pi i jk / L).  tab holds the
// stage twiddle tables in LDS, written (load_twiddles) before the call; the
// first stage needs no twiddles and its barrier publishes them.  After
// return, other threads may still read LDS: barrier before reusing it.
template <int L, int E, bool INV, typename C>
__device__ __forceinline__ void fft_block(C (&reg)[E], C* lds, const double2* tab) {
    using TT = TwTab<L, E>;
    static_assert((1 << TT::LOG) * TT::ODD == L && L >= 64 && fft_ok(L, E), "unsupported transform size");
    static_assert(TT::ODD != 3 || TT::NP2 >= 2, "the radix-3 stage of 3 * 2^m sits between two power-of-two stages");
    static_assert(TT::NP2 >= 1, "a power-of-two first stage");
    fft_stages<L, E, INV, 0, TT::NST>(reg, lds, tab);
}

// Two real columns a, b filtered by one transform pair: reg holds Z = FFT(a + i b)
// in canonical order (a fft_block result).  The transforms of the real parts
// follow from Hermitian symmetry, with W = Z_{L-m}:
//   A_m = (Z_m + conj W) / 2,   B_m = (Z_m - conj W) / (2 i),
// and reg becomes A sa + i B sb (CONJ: A conj(sa) + i B conj(sb)), both products
// Hermitian, so the inverse transform returns p + i q with p, q the real
// filtered columns.  sa, sb: the two spectrum columns (length L).  Goes through
// LDS once (the partner W sits in another thread); all threads of the block call it.
// The spectrum reads are not hoisted ahead of each other (one block of a launch
// runs this; its registers must not raise the kernel's count).
template <int L, int E, bool CONJ, typename C>
__device__ __forceinline__ void mul_real_pair(C (&reg)[E], C* lds, const C* __restrict__ sa,
                                              const C* __restrict__ sb) {
    using Rl = typename CplxOps<C>::real;
    constexpr int T = L / E;
    const int tid = threadIdx.x;
    __syncthreads();                      // the transform's last LDS reads are done
#pragma unroll
    for (int e = 0; e < E; ++e) lds[lds_slot(tid + e * T)] = reg[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int m = tid + e * T;
        const C z = reg[e], w = lds[lds_slot(m == 0 ? 0 : L - m)];
        const C A = CplxOps<C>::make(Rl(0.5) * (z.x + w.x), Rl(0.5) * (z.y - w.y));
        const C B = CplxOps<C>::make(Rl(0.5) * (z.y + w.y), Rl(-0.5) * (z.x - w.x));
        const C P = CONJ ? cmulc(A, sa[m]) : cmul(A, sa[m]);
        const C Q = CONJ ? cmulc(B, sb[m]) : cmul(B, sb[m]);
        reg[e] = CplxOps<C>::make(P.x - Q.y, P.y + Q.x);
        __builtin_amdgcn_sched_barrier(0);
    }
}

}  // namespace lpide
