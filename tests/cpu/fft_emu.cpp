// CPU check of the workgroup FFT of paper_2511_02700_amd/csrc/fft.hpp (the
// unchanged header, compiled for the host against tests/cpu/emu): every
// transform side up to 4096 and elements-per-thread choice the library
// instantiates, and sides with odd factors 5, 7 and 9, FP64
// and FP32 data, forward and inverse, one OS thread per GPU thread with a
// barrier for __syncthreads, the LDS exchange buffer and the twiddle tables in
// exactly sized heap arrays (so AddressSanitizer reports any access outside
// them).  Each transform is compared with the DFT evaluated in long double (at
// every output up to L = 2048, at 512 spread outputs above).
// Prints one line per case and "ALL OK" at the end; exits non-zero on a
// mismatch.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <random>
#include <thread>
#include <vector>

#include "fft.hpp"

using namespace lpide;

template <typename C>
struct Real;
template <>
struct Real<double2> { using T = double; };
template <>
struct Real<float2> { using T = float; };

// one workgroup: T threads transform x (length L, canonical layout in and out)
template <int L, int E, bool INV, typename C>
void run_block(const std::vector<double2>& tw_full, std::vector<C>& x) {
    constexpr int T = L / E;
    auto lds = std::make_unique<C[]>(lds_slots(L));
    auto tab = std::make_unique<double2[]>(tw_slots<L, E>());
    std::barrier<> bar(T);
    emu_block_barrier = &bar;
    std::vector<std::thread> th;
    th.reserve(T);
    for (int t = 0; t < T; ++t) {
        th.emplace_back([&, t] {
            threadIdx.x = unsigned(t);
            load_twiddles<L, E>(tw_full.data(), tab.get());
            C reg[E];
            for (int e = 0; e < E; ++e) reg[e] = x[t + e * T];
            bar.arrive_and_wait();       // every thread has read x before anyone writes it
            fft_block<L, E, INV>(reg, lds.get(), tab.get());
            for (int e = 0; e < E; ++e) x[t + e * T] = reg[e];
        });
    }
    for (auto& h : th) h.join();
    emu_block_barrier = nullptr;
}

template <int L, int E, typename C>
bool check(std::mt19937_64& rng, double tol) {
    using R = typename Real<C>::T;
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<double2> tw(L);
    for (int q = 0; q < L; ++q) {
        const long double a = -2.0L * pi * q / L;
        tw[q] = make_double2(double(cosl(a)), double(sinl(a)));
    }
    std::vector<long double> cs(L), sn(L);       // exp(-2 pi i q / L) in long double
    for (int q = 0; q < L; ++q) {
        cs[q] = cosl(2.0L * pi * q / L);
        sn[q] = -sinl(2.0L * pi * q / L);
    }
    std::normal_distribution<double> nd;
    bool ok = true;
    for (int inv = 0; inv < 2; ++inv) {
        std::vector<C> x(L);
        for (auto& v : x) v = C{R(nd(rng)), R(nd(rng))};
        const std::vector<C> x0 = x;
        if (inv) run_block<L, E, true>(tw, x);
        else run_block<L, E, false>(tw, x);
        long double err = 0.0L, scale = 0.0L;
        // every output up to 2048; above, 512 outputs spread over the whole range
        // (a wrong stage corrupts far more outputs than that misses)
        const int nk = L > 2048 ? 512 : L;
        for (int t = 0; t < nk; ++t) {
            const int k = L > 2048 ? int((unsigned long long)t * 2654435761ull % (unsigned long long)L) : t;
            long double re = 0.0L, im = 0.0L;
            for (int j = 0; j < L; ++j) {
                const int q = int((long long)j * k % L);
                const long double c = cs[q], s = inv ? -sn[q] : sn[q];
                re += x0[j].x * c - x0[j].y * s;
                im += x0[j].x * s + x0[j].y * c;
            }
            err = std::max(err, fabsl(re - x[k].x) + fabsl(im - x[k].y));
            scale = std::max(scale, fabsl(re) + fabsl(im));
        }
        const double rel = double(err / scale);
        const bool good = rel < tol;
        std::printf("L=%4d E=%2d %s %s max rel err %.3e %s\n", L, E, sizeof(R) == 8 ? "fp64" : "fp32",
                    inv ? "inverse" : "forward", rel, good ? "ok" : "FAIL");
        ok = ok && good;
    }
    return ok;
}

// Two real columns a, b filtered as one complex column (mul_real_pair between a
// forward and an inverse transform) against p = IDFT(DFT(a) sa) and
// q = IDFT(DFT(b) sb) in long double, for Hermitian spectra sa, sb (the
// transforms of real sequences); CONJ multiplies by their conjugates.
template <int L, int E, bool CONJ, typename C>
bool check_real_pair(std::mt19937_64& rng, double tol) {
    using R = typename Real<C>::T;
    constexpr int T = L / E;
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<double2> tw(L);
    std::vector<long double> cs(L), sn(L);
    for (int q = 0; q < L; ++q) {
        const long double ang = -2.0L * pi * q / L;
        tw[q] = make_double2(double(cosl(ang)), double(sinl(ang)));
        cs[q] = cosl(ang);
        sn[q] = sinl(ang);
    }
    // DFT (sign -1) or inverse (sign +1, unnormalised) of a complex sequence in long double
    auto dft = [&](const std::vector<long double>& re, const std::vector<long double>& im, int sign,
                   std::vector<long double>& ore, std::vector<long double>& oim) {
        ore.assign(L, 0.0L);
        oim.assign(L, 0.0L);
        for (int k = 0; k < L; ++k)
            for (int j = 0; j < L; ++j) {
                const int q = int((long long)j * k % L);
                const long double c = cs[q], s = sign < 0 ? sn[q] : -sn[q];
                ore[k] += re[j] * c - im[j] * s;
                oim[k] += re[j] * s + im[j] * c;
            }
    };
    std::normal_distribution<double> nd;
    std::vector<long double> a(L), b(L), ga(L), gb(L), zero(L, 0.0L);
    for (int j = 0; j < L; ++j) {
        a[j] = R(nd(rng));
        b[j] = R(nd(rng));
        ga[j] = nd(rng);
        gb[j] = nd(rng);
    }
    std::vector<long double> Ar, Ai, Br, Bi, Sar, Sai, Sbr, Sbi;
    dft(a, zero, -1, Ar, Ai);
    dft(b, zero, -1, Br, Bi);
    dft(ga, zero, -1, Sar, Sai);
    dft(gb, zero, -1, Sbr, Sbi);
    std::vector<C> sa(L), sb(L), x(L);
    std::vector<long double> Pr(L), Pi(L), Qr(L), Qi(L);
    for (int m = 0; m < L; ++m) {
        sa[m] = C{R(Sar[m]), R(Sai[m])};
        sb[m] = C{R(Sbr[m]), R(Sbi[m])};
        const long double sai = CONJ ? -(long double)sa[m].y : (long double)sa[m].y;
        const long double sbi = CONJ ? -(long double)sb[m].y : (long double)sb[m].y;
        Pr[m] = Ar[m] * sa[m].x - Ai[m] * sai;
        Pi[m] = Ar[m] * sai + Ai[m] * sa[m].x;
        Qr[m] = Br[m] * sb[m].x - Bi[m] * sbi;
        Qi[m] = Br[m] * sbi + Bi[m] * sb[m].x;
        x[m] = C{R(a[m]), R(b[m])};
    }
    std::vector<long double> pr, pi_, qr, qi;
    dft(Pr, Pi, +1, pr, pi_);
    dft(Qr, Qi, +1, qr, qi);
    auto lds = std::make_unique<C[]>(lds_slots(L));
    auto tab = std::make_unique<double2[]>(tw_slots<L, E>());
    std::barrier<> bar(T);
    emu_block_barrier = &bar;
    std::vector<std::thread> th;
    th.reserve(T);
    for (int t = 0; t < T; ++t) {
        th.emplace_back([&, t] {
            threadIdx.x = unsigned(t);
            load_twiddles<L, E>(tw.data(), tab.get());
            C reg[E];
            for (int e = 0; e < E; ++e) reg[e] = x[t + e * T];
            bar.arrive_and_wait();
            fft_block<L, E, false>(reg, lds.get(), tab.get());
            mul_real_pair<L, E, CONJ>(reg, lds.get(), sa.data(), sb.data());
            fft_block<L, E, true>(reg, lds.get(), tab.get());
            bar.arrive_and_wait();       // every thread has finished before x is overwritten
            for (int e = 0; e < E; ++e) x[t + e * T] = reg[e];
        });
    }
    for (auto& h : th) h.join();
    emu_block_barrier = nullptr;
    long double err = 0.0L, scale = 0.0L;
    for (int j = 0; j < L; ++j) {
        err = std::max(err, fabsl(pr[j] - x[j].x) + fabsl(qr[j] - x[j].y));
        scale = std::max(scale, fabsl(pr[j]) + fabsl(qr[j]));
    }
    const double rel = double(err / scale);
    const bool good = rel < tol;
    std::printf("L=%4d E=%2d %s real pair%s max rel err %.3e %s\n", L, E, sizeof(R) == 8 ? "fp64" : "fp32",
                CONJ ? " (conj)" : "", rel, good ? "ok" : "FAIL");
    return good;
}

template <int L, typename C>
bool sizes(std::mt19937_64& rng, double tol) {
    bool ok = true;
    if constexpr (fft_ok(L, 4)) ok = check<L, 4, C>(rng, tol) && ok;
    if constexpr (fft_ok(L, 8)) ok = check<L, 8, C>(rng, tol) && ok;
    if constexpr (fft_ok(L, 16)) ok = check<L, 16, C>(rng, tol) && ok;
    return ok;
}

// The cases are split into FFT_EMU_PARTS programs (compiled separately, in
// parallel; part FFT_EMU_PART instantiates only its own cases): case I belongs
// to part I mod FFT_EMU_PARTS.
#ifndef FFT_EMU_PARTS
#define FFT_EMU_PARTS 1
#endif
#ifndef FFT_EMU_PART
#define FFT_EMU_PART 0
#endif
template <int I>
constexpr bool mine() { return I % FFT_EMU_PARTS == FFT_EMU_PART; }

template <typename C>
bool all_sizes(std::mt19937_64& rng, double tol) {
    bool ok = true;
    if constexpr (mine<0>()) ok = sizes<64, C>(rng, tol) && ok;
    if constexpr (mine<1>()) ok = sizes<128, C>(rng, tol) && ok;
    if constexpr (mine<2>()) ok = sizes<256, C>(rng, tol) && ok;
    if constexpr (mine<3>()) ok = sizes<512, C>(rng, tol) && ok;
    if constexpr (mine<4>()) ok = sizes<768, C>(rng, tol) && ok;
    if constexpr (mine<5>()) ok = sizes<1024, C>(rng, tol) && ok;
    if constexpr (mine<6>()) ok = sizes<1536, C>(rng, tol) && ok;
    if constexpr (mine<7>()) ok = sizes<2048, C>(rng, tol) && ok;
    if constexpr (mine<8>()) ok = sizes<3072, C>(rng, tol) && ok;
    if constexpr (mine<9>()) ok = sizes<4096, C>(rng, tol) && ok;
    // sides with odd factors 5, 7 and 9 (radix-5, radix-7 and two radix-3
    // stages): every E in FP64, the two smallest in FP32 as well (the stages
    // are the same code for both), the largest with the 16 elements per thread
    // the price-space plan uses there
    if constexpr (mine<10>()) ok = sizes<640, C>(rng, tol) && ok;
    if constexpr (mine<11>()) ok = sizes<896, C>(rng, tol) && ok;
    if constexpr (sizeof(typename Real<C>::T) == 8) {
        if constexpr (mine<12>()) ok = sizes<1152, C>(rng, tol) && ok;
        if constexpr (mine<13>()) ok = sizes<1280, C>(rng, tol) && ok;
        if constexpr (mine<14>()) ok = sizes<1792, C>(rng, tol) && ok;
        if constexpr (mine<15>()) ok = sizes<2304, C>(rng, tol) && ok;
        if constexpr (mine<16>()) ok = sizes<2560, C>(rng, tol) && ok;
        if constexpr (mine<17>()) ok = sizes<3584, C>(rng, tol) && ok;
        if constexpr (mine<18>()) ok = check<4608, 16, C>(rng, tol) && ok;
        if constexpr (mine<19>()) ok = check<5120, 16, C>(rng, tol) && ok;
        if constexpr (mine<20>()) ok = check<7168, 16, C>(rng, tol) && ok;
    }
    // DC and Nyquist columns filtered together (the column passes' block 0)
    if constexpr (mine<21>()) {
        ok = check_real_pair<3072, 4, false, C>(rng, tol) && ok;
        ok = check_real_pair<3072, 4, true, C>(rng, tol) && ok;
    }
    if constexpr (mine<22>()) {
        ok = check_real_pair<1024, 16, false, C>(rng, tol) && ok;
        ok = check_real_pair<640, 4, false, C>(rng, tol) && ok;
    }
    return ok;
}

int main() {
    std::mt19937_64 rng(20251102);
    bool ok = all_sizes<double2>(rng, 1e-14);
    ok = all_sizes<float2>(rng, 2e-6) && ok;
    std::printf(ok ? "ALL OK\n" : "MISMATCH\n");
    return ok ? 0 : 1;
}
