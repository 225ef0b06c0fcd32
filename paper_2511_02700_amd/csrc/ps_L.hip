// Correlation launches of the price-space plan for one transform side L
// (compiled once per side with -DLPIDE_L=L).
#include "conv_kernels.hpp"
#include "ps_big.hpp"
#include "ps_plan.hpp"

#ifndef LPIDE_L
#error "compile with -DLPIDE_L=<transform size>"
#endif

namespace lpide {
namespace ps {

// Column pass and row inverse of the two-level sides with SO = so output
// segments (so <= R), chosen at run time among the instantiations 1..R.
template <int M, int R, int SO>
void big_inverse(const PsConv& c, int so, int k) {
    if constexpr (SO < R) {
        if (so > SO) return big_inverse<M, R, SO + 1>(c, so, k);
    }
    const PsOps& o = c.o;
    constexpr int L = R * M;
    hipLaunchKernelGGL((ps_big_cols<M, R, SO, 0>), dim3(L / 2 + 1), dim3(BIG_T), 0, c.stream, c.X, o.ldx, o.n_nz,
                       o.n_out, c.spec, (double2*)nullptr, 0.0, c.tw, c.twM, c.ctl, k, c.tol);
    hipLaunchKernelGGL((ps_big_rows_inv<M, R, SO>), dim3((o.n_out + 1) / 2), dim3(BIG_T), 0, c.stream,
                       (const double2*)c.X, c.Z, o, c.tw, c.twM, c.ctl, k, c.tol);
}

template <int L>
void PsL<L>::bapply(const PsConv& c, const double* Y, int k) {
    const PsOps& o = c.o;
    hipLaunchKernelGGL(ps_tin2, dim3((o.n_nz + 255) / 256, o.n), dim3(256), 0, c.stream, Y, c.U, o, c.ctl, k, c.tol);
    if constexpr (L > 8192) {
        constexpr int M = big_m(L), R = L / M;
        hipLaunchKernelGGL((ps_big_rows_fwd<M, R, 0>), dim3((o.n_nz + 1) / 2), dim3(BIG_T), 0, c.stream,
                           (const double*)c.U, o.n_nz, o.n_nz, o.n_nz, c.X, o.ldx, o.tin_s, o.tin_w, c.tw, c.twM, c.ctl,
                           k, c.tol);
        // the segments of length M that hold kept outputs (compile-time register count)
        const int so = (o.n_out + M - 1) / M;
        big_inverse<M, R, 1>(c, so, k);
    } else {
        constexpr int T = L / ps_e(L);
        hipLaunchKernelGGL((ps_rows_fwd<L>), dim3((o.n_nz + 1) / 2), dim3(T), 0, c.stream, (const double*)c.U, c.X, o,
                           c.tw, c.ctl, k, c.tol);
        hipLaunchKernelGGL((ps_cols<L>), dim3(L / 2), dim3(T), 0, c.stream, c.X, c.spec, o, c.tw, c.ctl, k, c.tol);
        hipLaunchKernelGGL((ps_rows_inv<L>), dim3((o.n_out + 1) / 2), dim3(T), 0, c.stream, (const double2*)c.X, c.Z, o,
                           c.tw, c.ctl, k, c.tol);
    }
}

template <int L>
void PsL<L>::spectrum(hipStream_t s, const double* W, int W2, double2* Xf, double2* spec, const double2* tw,
                      const double2* twM) {
    using namespace lpide::detail;
    const double scale = 1.0 / (double(L) * double(L));
    if constexpr (L > 8192) {
        constexpr int M = big_m(L), R = L / M;
        hipLaunchKernelGGL((ps_big_rows_fwd<M, R, 1>), dim3((W2 + 1) / 2), dim3(BIG_T), 0, s, W, W2, W2, W2, Xf, W2,
                           (const int*)nullptr, (const double*)nullptr, tw, twM, (const PsCtl*)nullptr, 0, 0.0);
        hipLaunchKernelGGL((ps_big_cols<M, R, 1, 1>), dim3(L / 2 + 1), dim3(BIG_T), 0, s, Xf, W2, W2, 0,
                           (const double2*)nullptr, spec, scale, tw, twM, (const PsCtl*)nullptr, 0, 0.0);
    } else {
        hipLaunchKernelGGL((k_rows_fwd<L>), dim3((W2 + 1) / 2), dim3(L / conv_e(L)), 0, s, W, W2, W2, W2, Xf, W2, tw);
        hipLaunchKernelGGL((k_cols<L, 1>), dim3(L / 2 + 1), dim3(L / conv_e(L)), 0, s, Xf, W2, W2, L,
                           (const double2*)nullptr, spec, scale, tw);
    }
}

template struct PsL<LPIDE_L>;

}  // namespace ps
}  // namespace lpide
