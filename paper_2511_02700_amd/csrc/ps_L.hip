// Correlation launches of the price-space plan for one transform side L
// (compiled once per side with -DLPIDE_L=L).
#include "conv_kernels.hpp"
#include "ps_plan.hpp"

#ifndef LPIDE_L
#error "compile with -DLPIDE_L=<transform size>"
#endif

namespace lpide {
namespace ps {

template <int L>
void PsL<L>::bapply(const PsConv& c, const double* Y, int k) {
    constexpr int T = L / ps_e(L);
    const PsOps& o = c.o;
    hipLaunchKernelGGL(ps_tin2, dim3((o.n_nz + 255) / 256, o.n), dim3(256), 0, c.stream, Y, c.U, o, c.ctl, k, c.tol);
    hipLaunchKernelGGL((ps_rows_fwd<L>), dim3((o.n_nz + 1) / 2), dim3(T), 0, c.stream, (const double*)c.U, c.X, o, c.tw,
                       c.ctl, k, c.tol);
    hipLaunchKernelGGL((ps_cols<L>), dim3(L / 2 + 1), dim3(T), 0, c.stream, c.X, c.spec, o, c.tw, c.ctl, k, c.tol);
    hipLaunchKernelGGL((ps_rows_inv<L>), dim3((o.n_out + 1) / 2), dim3(T), 0, c.stream, (const double2*)c.X, c.Z, o,
                       c.tw, c.ctl, k, c.tol);
}

template <int L>
void PsL<L>::spectrum(hipStream_t s, const double* G, double2* Xfull, double2* spec, const double2* tw) {
    using namespace lpide::detail;
    const double scale = 1.0 / (double(L) * double(L));
    hipLaunchKernelGGL((k_rows_fwd<L>), dim3(L / 2), dim3(L / conv_e(L)), 0, s, G, L, L, L, Xfull, L, tw);
    hipLaunchKernelGGL((k_cols<L, 1>), dim3(L / 2 + 1), dim3(L / conv_e(L)), 0, s, Xfull, L, L, L,
                       (const double2*)nullptr, spec, scale, tw);
}

template struct PsL<LPIDE_L>;

}  // namespace ps
}  // namespace lpide
