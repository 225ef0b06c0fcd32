// Structures of the price-space plan shared by ps.hip (the plan, its march
// and the C ABI) and ps_L.hip (the correlation launches for one transform
// side each).
#pragma once

#include <hip/hip_runtime.h>

#include "ps_kernels.hpp"

namespace lpide {
namespace ps {

// What the four correlation passes of B_omega need.
struct PsConv {
    hipStream_t stream = nullptr;
    PsOps o{};
    double* U = nullptr;            // n x n_nz
    double2* X = nullptr;           // (L/2 + 1) x ldx
    double* Z = nullptr;            // n_out x n
    const double2* spec = nullptr;  // (L/2 + 1) x L
    const double2* tw = nullptr;    // L twiddles exp(-2 pi i q / L)
    const PsCtl* ctl = nullptr;     // nullptr: no early exit
    double tol = 0.0;
};

template <int L>
struct PsL {
    // Z = (C T^in Y restricted to y^out) (T^out)^T for iteration k (k = 0: always runs).
    static void bapply(const PsConv& c, const double* Y, int k);
    // spec = conj(FFT2(G)) / L^2 of the L x L real grid G (Xfull: (L/2 + 1) x L scratch).
    static void spectrum(hipStream_t s, const double* G, double2* Xfull, double2* spec, const double2* tw);
};
extern template struct PsL<64>;
extern template struct PsL<128>;
extern template struct PsL<256>;
extern template struct PsL<512>;
extern template struct PsL<768>;
extern template struct PsL<1024>;
extern template struct PsL<1536>;
extern template struct PsL<2048>;
extern template struct PsL<3072>;
extern template struct PsL<4096>;
extern template struct PsL<6144>;
extern template struct PsL<8192>;

}  // namespace ps
}  // namespace lpide
