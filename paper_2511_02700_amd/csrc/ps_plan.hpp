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
    const double2* twM = nullptr;   // sides above 8192: the twiddles of the inner transforms (length 4096 or 8192)
    const PsCtl* ctl = nullptr;     // nullptr: no early exit
    double tol = 0.0;
};

template <int L>
struct PsL {
    // Z = (C T^in Y restricted to y^out) (T^out)^T for iteration k (k = 0: always runs).
    static void bapply(const PsConv& c, const double* Y, int k);
    // spec = conj(FFT2(G)) / L^2 of the L x L real grid G that holds the W2 x W2
    // weights W (row-major) in its corner [0, W2)^2 and zeros elsewhere (Xf:
    // (L/2 + 1) x W2 scratch).  Natural order up to 8192; in the (r, q) order of
    // the two-level transforms above.
    static void spectrum(hipStream_t s, const double* W, int W2, double2* Xf, double2* spec, const double2* tw,
                         const double2* twM);
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
extern template struct PsL<640>;
extern template struct PsL<896>;
extern template struct PsL<1152>;
extern template struct PsL<1280>;
extern template struct PsL<1792>;
extern template struct PsL<2304>;
extern template struct PsL<2560>;
extern template struct PsL<3584>;
extern template struct PsL<4608>;
extern template struct PsL<5120>;
extern template struct PsL<7168>;
extern template struct PsL<12288>;
extern template struct PsL<16384>;
extern template struct PsL<24576>;

}  // namespace ps
}  // namespace lpide
