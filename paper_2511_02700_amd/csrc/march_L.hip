// Launch sequences for one transform size L (compiled once per size with
// -DLPIDE_L=L): the device-controlled march (one step slot or one iteration
// for a group of plans, every kernel class with its radix schedule), the
// stand-alone correlation and plan-time spectrum, and one reverse step of the
// adjoint march.
#include "conv_kernels.hpp"
#include "plan.hpp"

#ifndef LPIDE_L
#error "compile with -DLPIDE_L=<transform size>"
#endif

namespace lpide {
namespace detail {
namespace {

// ---- stand-alone correlation (apply_B) and plan-time spectrum ----
// X: the transposed intermediate, (L/2 + 1) x n complex (the plan's own, or a
// caller-independent scratch buffer of at least that size).
template <int L>
void launch_conv(Plan* p, const double* Y, double* out, double2* X) {
    const int n = p->hp.n, np = (n + 1) / 2;
    hipLaunchKernelGGL((k_rows_fwd<L>), dim3(np), dim3(L / conv_e(L)), 0, p->stream, Y, n, n, n, X, n, p->tw);
    hipLaunchKernelGGL((k_cols<L, 0>), dim3(L / 2 + 1), dim3(L / conv_e(L)), 0, p->stream, X, n, n, n, p->spec,
                       (double2*)nullptr, 0.0, p->tw);
    hipLaunchKernelGGL((k_rows_inv<L>), dim3(np), dim3(L / conv_e(L)), 0, p->stream, X, n, n, out, p->tw);
}

template <int L>
void launch_spectrum(Plan* p, const double* G, double2* Xfull) {
    const double scale = 1.0 / (double(L) * double(L));
    hipLaunchKernelGGL((k_rows_fwd<L>), dim3(L / 2), dim3(L / conv_e(L)), 0, p->stream, G, L, L, L, Xfull, L, p->tw);
    hipLaunchKernelGGL((k_cols<L, 1>), dim3(L / 2 + 1), dim3(L / conv_e(L)), 0, p->stream, Xfull, L, L, L,
                       (const double2*)nullptr, p->spec, scale, p->tw);
}

template <int L>
void launch_rows_fwd(Plan* p, const double* Y, hipStream_t s) {
    const int n = p->hp.n;
    hipLaunchKernelGGL((k_rows_fwd<L>), dim3((n + 1) / 2), dim3(L / conv_e(L)), 0, s, Y, n, n, n, p->X, n, p->tw);
}

// The axis-1 line-solve kernel for the launch's columns per block; bounds of
// 256 threads where the block fits (no register cap of 128), and the smallest
// chunk capacity of 8, 16 and LINE_MM that holds every chunk (the chunks of the
// largest plan hold ceil(n / P_cols) <= ceil(xcols cpb / P_cols) rows; the
// sweeps run over all capacity slots).
template <int CPB, int MAXT, typename Go>
void with_line_cols_mm(const Launch& c, Go&& go) {
    const int ch = (c.xcols * c.cpb + c.P_cols - 1) / c.P_cols;
    if (ch <= 8) go(ks_line_cols<CPB, MAXT, 8>);
    else if (ch <= 16) go(ks_line_cols<CPB, MAXT, 16>);
    else go(ks_line_cols<CPB, MAXT, LINE_MM>);
}

template <typename Go>
void with_line_cols(const Launch& c, Go&& go) {
    const bool small = c.cpb * c.P_cols <= 256;
    if (c.cpb == 2) {
        if (small) with_line_cols_mm<2, 256>(c, go);
        else with_line_cols_mm<2, 1024>(c, go);
    } else {
        if (small) with_line_cols_mm<4, 256>(c, go);
        else with_line_cols_mm<4, 1024>(c, go);
    }
}

// The line-row kernel with E elements per thread and the smallest chunk
// capacity (E, 3E/2 or 2E) that holds the longest chunk of the launch's plans.
template <int L, int E, bool FFT, bool MIXED, typename Go>
void with_line_rows(const Launch& c, Go&& go) {
    constexpr int PR = L / E / 2;
    const int m = (c.xaff + PR - 1) / PR;
    if (m <= E) go(ks_line_rows<L, E, FFT, MIXED, E>);
    else if (m <= 3 * E / 2) go(ks_line_rows<L, E, FFT, MIXED, 3 * E / 2>);
    else go(ks_line_rows<L, E, FFT, MIXED, 2 * E>);
}

template <int L, bool FFT, bool MIXED>
void launch_iteration(const Launch& c, int k) {
    using C = typename std::conditional<MIXED, float2, double2>::type;
    if (c.timer) c.timer->tag_k = k;
    // steady FP64 slots: iteration 1 is rows_lin alone (the column pass and the
    // row c2r kernel would exit)
    const bool lean1 = FFT && !MIXED && c.lean && k == 1;
    if (FFT && !lean1) {
        {
            KTime t(c.timer, LPIDE_K_COLS);
            with_E<L>(c.E_cols, [&](auto e) {
                constexpr int E = decltype(e)::value;
                t.launch((ks_cols<L, E, C>), dim3(L / 2, c.np), dim3(L / E), 0, c.stream, c.A, k);
            });
        }
        {
            KTime t(c.timer, LPIDE_K_ROWS_INV);
            with_E<L>(c.E_rinv, [&](auto e) {
                constexpr int E = decltype(e)::value;
                t.launch((ks_rows_inv<L, E, MIXED ? 2 : 1>), dim3(c.xrows, c.np), dim3(L / E), 0, c.stream, c.A,
                         k);
            });
        }
    }
    if (FFT && !MIXED && k == 1) {        // B Y^0 by linearity (the two above exit then)
        KTime t(c.timer, LPIDE_K_ROWS_LIN);
        t.launch(ks_rows_lin, dim3(c.xaff, c.np), dim3(256), 0, c.stream, c.A);
    }
    if (!FFT) {
        KTime t(c.timer, LPIDE_K_ROWS_INV);
        t.launch((ks_affine_noB<false>), dim3(c.xaff, c.np), dim3(256), 0, c.stream, c.A, k);
    }
    {
        KTime t(c.timer, LPIDE_K_LINE_COLS);
        with_line_cols(c, [&](auto kern) {
            t.launch(kern, dim3(c.xcols, c.np), dim3(c.cpb * c.P_cols), sizeof(double2) * c.cpb * c.P_cols, c.stream,
                     c.A, k);
        });
    }
    KTime t(c.timer, LPIDE_K_LINE_ROWS);
    with_E<L>(c.E_lrows, [&](auto e) {
        constexpr int E = decltype(e)::value;
        with_line_rows<L, E, FFT, MIXED>(c, [&](auto kern) {
            t.launch(kern, dim3(c.xrows, c.np), dim3(L / E), 0, c.stream, c.A, k);
        });
    });
}

// One entry of every plan's step list.  The FP64 correlation of V^{n-1} runs
// when the explicit part needs it (theta < 1) and, in the mixed form, in every
// step (B V^{n-1} anchors the FP32 increments); the kernels decide on the
// device, so the launch sequence is the same for every step, except in slots
// the host knows to be steady (Launch::lean: both FP64 shortcuts apply to every
// plan), where the kernels that would exit are left out.  In the FP64 form the
// row transform of V^{n-1} is left in X by the previous step's last iteration;
// the mixed form recomputes it (its iterations transform increments).
template <int L, bool FFT, bool MIXED>
void launch_step(const Launch& c, int kmax) {
    if (c.timer) c.timer->tag_k = 0;
    const dim3 gr(c.xrows, c.np), gc(L / 2, c.np);
    const bool lean = FFT && !MIXED && c.lean;
    if (FFT && !lean) {
        if (MIXED) {
            KTime t(c.timer, LPIDE_K_ROWS_FWD);
            with_E<L>(c.E_rinv, [&](auto e) {
                constexpr int E = decltype(e)::value;
                t.launch((ks_rows_fwd<L, E>), gr, dim3(L / E), 0, c.stream, c.A);
            });
        }
        {
            KTime t(c.timer, LPIDE_K_EXPL_COLS);
            with_E<L>(c.E_cols, [&](auto e) {
                constexpr int E = decltype(e)::value;
                t.launch((ks_cols<L, E, double2>), gc, dim3(L / E), 0, c.stream, c.A, 0);
            });
        }
        {
            KTime t(c.timer, LPIDE_K_EXPL_ROWS);
            with_E<L>(c.E_rinv, [&](auto e) {
                constexpr int E = decltype(e)::value;
                t.launch((ks_rows_inv<L, E, 0>), gr, dim3(L / E), 0, c.stream, c.A, 0);
            });
        }
        if (MIXED) {                      // steps between anchors without the identity (the three above exit)
            KTime t(c.timer, LPIDE_K_CARRY);
            t.launch(ks_carry, dim3(c.xaff, c.np), dim3(256), 0, c.stream, c.A);
        }
        {                                 // explicit part from the previous step's equation (the two above exit)
            KTime t(c.timer, LPIDE_K_EXPL_ID);
            t.launch(ks_expl_identity, dim3(c.xaff, c.np), dim3(256), 0, c.stream, c.A);
        }
    } else if (lean) {                    // steady: the explicit part from the previous step's equation
        KTime t(c.timer, LPIDE_K_EXPL_ID);
        t.launch(ks_expl_identity, dim3(c.xaff, c.np), dim3(256), 0, c.stream, c.A);
    } else {
        KTime t(c.timer, LPIDE_K_EXPL_ROWS);
        t.launch((ks_affine_noB<true>), dim3(c.xaff, c.np), dim3(256), 0, c.stream, c.A, 0);
    }
    if (!lean) {
        KTime t(c.timer, LPIDE_K_SL);
        with_E<L>(c.E_sl, [&](auto e) {
            constexpr int E = decltype(e)::value;
            if (c.sl_order == 1)
                t.launch((ks_sl<L, E, 1, FFT, MIXED>), gr, dim3(L / E), 0, c.stream, c.A);
            else
                t.launch((ks_sl<L, E, 3, FFT, MIXED>), gr, dim3(L / E), 0, c.stream, c.A);
        });
    }
    if (FFT && !MIXED) {                  // steps with B Y^0 by linearity (ks_sl exits in them)
        KTime t(c.timer, LPIDE_K_SL_LIN);
        const size_t shm = sizeof(double) * c.xaff;   // the combined source rows of the largest plan
        if (c.sl_order == 1) t.launch(ks_sl_lin<1>, dim3(c.xaff, c.np), dim3(256), shm, c.stream, c.A);
        else t.launch(ks_sl_lin<3>, dim3(c.xaff, c.np), dim3(256), shm, c.stream, c.A);
    }
    if (c.record) hipLaunchKernelGGL(ks_store_E, dim3(c.store_blocks, c.np), dim3(256), 0, c.stream, c.A);
    for (int k = 1; k <= kmax; ++k) launch_iteration<L, FFT, MIXED>(c, k);
    if (c.timer) c.timer->tag_k = 0;
    {
        KTime t(c.timer, LPIDE_K_STEP_END);
        t.launch(ks_step_end, dim3(1, c.np), dim3(64), 0, c.stream, c.A, kmax);
    }
    if (c.record) hipLaunchKernelGGL(ks_store_V, dim3(c.store_blocks, c.np), dim3(256), 0, c.stream, c.A);
}

template <int L>
void launch_slots_L(const Launch& c, int first_tag, int nslots, int kmax) {
    for (int s = 0; s < nslots; ++s) {
        if (c.timer) c.timer->tag_step = first_tag + s;
        if (!c.jumps) launch_step<L, false, false>(c, kmax);
        else if (c.mixed) launch_step<L, true, true>(c, kmax);
        else launch_step<L, true, false>(c, kmax);
    }
}

template <int L>
void launch_iteration_L(const Launch& c, int k) {
    if (!c.jumps) launch_iteration<L, false, false>(c, k);
    else if (c.mixed) launch_iteration<L, true, true>(c, k);
    else launch_iteration<L, true, false>(c, k);
}

template <int L>
void launch_adj_iteration(const Launch& c, int k) {
    with_E<L>(c.E_cols, [&](auto e) {
        constexpr int E = decltype(e)::value;
        hipLaunchKernelGGL((ks_cols<L, E, double2, true>), dim3(L / 2, 1), dim3(L / E), 0, c.stream, c.A, k);
    });
    with_E<L>(c.E_rinv, [&](auto e) {
        constexpr int E = decltype(e)::value;
        hipLaunchKernelGGL((ks_rows_inv<L, E, 3>), dim3(c.xrows, 1), dim3(L / E), 0, c.stream, c.A, k);
    });
    with_line_cols(c, [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(c.xcols, 1), dim3(c.cpb * c.P_cols), sizeof(double2) * c.cpb * c.P_cols,
                           c.stream, c.A, k);
    });
    with_E<L>(c.E_lrows, [&](auto e) {
        constexpr int E = decltype(e)::value;
        with_line_rows<L, E, true, false>(c, [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(c.xrows, 1), dim3(L / E), 0, c.stream, c.A, k);
        });
    });
}

// One reverse step s: Ybar (in adj->ybar) -> cotangent of V^s (in adj->ybar),
// gradient terms accumulated.  Y = V^{s+1}, V = V^s, E = E_s.
template <int L>
int adj_step(Plan* p, const Launch& c, int s, int* kpred, const double* Y, const double* V, const double* E) {
    Adjoint* a = p->adj;
    const int n = p->hp.n;
    const size_t N = (size_t)n * n;
    const StepDesc& sd = p->sets[p->step_set[s]];
    const dim3 gr(c.xrows, 1);
    hipLaunchKernelGGL(ks_adj_begin, dim3(1), dim3(64), 0, c.stream, c.A, s);
    const double cth = sd.dt * sd.theta;
    // the correction lam - Ybar = dt theta A^T lam of the previous reverse
    // steps, rescaled to this step's dt theta and extrapolated over the run of
    // previous steps of the same kind (up to four: kept, linear, quadratic,
    // cubic, as the forward march extrapolates its start values)
    static constexpr double kExtrap[4][4] = {{1, 0, 0, 0}, {2, -1, 0, 0}, {3, -3, 1, 0}, {4, -6, 4, -1}};
    int run = 0;
    if (a->have_corr >= 1 && a->corr_c[0] > 0.0) {
        run = 1;
        while (run < a->have_corr && a->corr_c[run] == a->corr_c[0]) ++run;
    }
    const double* cp[4] = {nullptr, nullptr, nullptr, nullptr};
    double cw[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = 0; q < run; ++q) {
        cp[q] = a->corr[q];
        cw[q] = kExtrap[run - 1][q] * (cth / a->corr_c[0]);
    }
    with_E<L>(c.E_rinv, [&](auto e) {
        constexpr int E = decltype(e)::value;
        hipLaunchKernelGGL((ks_adj_start<L, E>), gr, dim3(L / E), 0, c.stream, c.A, cp[0], cw[0], cp[1], cw[1], cp[2],
                           cw[2], cp[3], cw[3]);
    });
    int k = *kpred;
    for (int q = 1; q <= k; ++q) launch_adj_iteration<L>(c, q);
    hipLaunchKernelGGL(ks_adj_end, dim3(1), dim3(64), 0, c.stream, c.A, k);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(a->ctl_h, a->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c.stream));
    HIP_TRY(hipStreamSynchronize(c.stream));
    while (a->ctl_h->fail) {
        const double ek = err_of(*a->ctl_h, k);
        if (!std::isfinite(ek)) return fail(LPIDE_E_NAN, "non-finite adjoint increment in step " + std::to_string(s));
        if (k >= p->opts.max_iter) {
            char buf[160];
            snprintf(buf, sizeof buf, "adjoint fixed point not converged in step %d after %d iterations (increment %.3e)",
                     s, k, ek);
            return fail(LPIDE_E_NOCONV, buf);
        }
        ++k;
        hipLaunchKernelGGL(ks_clear_fail, dim3(1), dim3(64), 0, c.stream, c.A, 0);
        launch_adj_iteration<L>(c, k);
        hipLaunchKernelGGL(ks_adj_end, dim3(1), dim3(64), 0, c.stream, c.A, k);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(a->ctl_h, a->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c.stream));
        HIP_TRY(hipStreamSynchronize(c.stream));
    }
    int used = k;
    for (int q = 1; q <= k; ++q)
        if (err_of(*a->ctl_h, q) < p->opts.tol) { used = q; break; }
    // the last iteration left the row transform of the converged lam in X:
    // kept for the spectral gradient term (the transposed SL overwrites X)
    const size_t xbytes = sizeof(double2) * (size_t)(L / 2 + 1) * n;
    if (p->jumps) HIP_TRY(hipMemcpyAsync(a->XA, p->X, xbytes, hipMemcpyDeviceToDevice, c.stream));
    a->counts_h[s] = used;
    *kpred = std::max(1, std::min(p->opts.max_iter, used));
    const int sb = int(std::min<size_t>(1024, (N + 255) / 256));
    {
        double* oldest = a->corr[3];
        for (int q = 3; q > 0; --q) {
            a->corr[q] = a->corr[q - 1];
            a->corr_c[q] = a->corr_c[q - 1];
        }
        a->corr[0] = oldest;
    }
    hipLaunchKernelGGL(ks_adj_corr, dim3(sb), dim3(256), 0, c.stream, c.A, a->corr[0]);
    a->have_corr = std::min(4, a->have_corr + 1);
    a->corr_c[0] = cth;
    // mu = (T^SL)^T lam (its row transform also into XC for the spectral
    // gradient term when theta < 1), then the cotangent of V^s
    const double c1 = sd.dt * sd.theta, c2 = sd.dt * (1.0 - sd.theta);
    double2* x2 = (p->jumps && c2 != 0.0) ? a->XC : nullptr;
    const bool narrow = sd.wt1 <= 8 && sd.wt2 <= 8;
    with_E<L>(c.E_sl, [&](auto e) {
        constexpr int E = decltype(e)::value;
        if (narrow) hipLaunchKernelGGL((ks_adj_sl<L, E, 8>), gr, dim3(L / E), 0, c.stream, c.A, x2);
        else hipLaunchKernelGGL((ks_adj_sl<L, E, 0>), gr, dim3(L / E), 0, c.stream, c.A, x2);
    });
    if (sd.theta < 1.0) {
        with_E<L>(c.E_cols, [&](auto e) {
            constexpr int E = decltype(e)::value;
            hipLaunchKernelGGL((ks_cols<L, E, double2, true>), dim3(L / 2, 1), dim3(L / E), 0, c.stream, c.A, 0);
        });
        with_E<L>(c.E_rinv, [&](auto e) {
            constexpr int E = decltype(e)::value;
            hipLaunchKernelGGL((ks_rows_inv<L, E, 4>), gr, dim3(L / E), 0, c.stream, c.A, 0);
        });
    }
    // gradient terms (they read lam and mu; the new cotangent is written last)
    if (p->hp.sl_order == 1)
        hipLaunchKernelGGL(ks_adj_accum<1>, dim3(n, 1), dim3(256), 0, c.stream, c.A, Y, V, E, a->acc);
    else
        hipLaunchKernelGGL(ks_adj_accum<3>, dim3(n, 1), dim3(256), 0, c.stream, c.A, Y, V, E, a->acc);
    if (p->jumps) {
        const int np = (n + 1) / 2;
        // the row transform of Y = V^{s+1} is the V transform of reverse step s + 1 when it had one;
        // those of lam (XA) and mu (XC) are in place already
        if (a->xb_is_v) std::swap(a->XB, a->XD);
        else hipLaunchKernelGGL((k_rows_fwd<L>), dim3(np), dim3(L / conv_e(L)), 0, c.stream, Y, n, n, n, a->XB, n, p->tw);
        a->xb_is_v = false;
        if (c2 != 0.0) {
            hipLaunchKernelGGL((k_rows_fwd<L>), dim3(np), dim3(L / conv_e(L)), 0, c.stream, V, n, n, n, a->XD, n, p->tw);
            a->xb_is_v = true;
        }
        hipLaunchKernelGGL((ks_adj_spec<L>), dim3(L / 2 + 1), dim3(L / conv_e(L)), 0, c.stream, a->XA, a->XB, a->XC, a->XD, n,
                           c1, c2, a->S, p->tw);
    }
    if (sd.theta >= 1.0)
        hipLaunchKernelGGL(k_copy, dim3((N + 255) / 256), dim3(256), 0, c.stream, a->mu, a->ybar, N);
    HIP_TRY(hipGetLastError());
    return LPIDE_OK;
}

// Inverse 2D transform of the spectral accumulator (column inverse FFTs in
// place, then the row c2r): G[d1 mod L][d2 mod L] = L^2 x (kernel gradient).
template <int L>
void launch_adj_kernel_grad(Plan* p, hipStream_t s) {
    Adjoint* a = p->adj;
    hipLaunchKernelGGL((k_cols<L, 2>), dim3(L / 2 + 1), dim3(L / conv_e(L)), 0, s, a->S, L, L, L, (const double2*)nullptr,
                       (double2*)nullptr, 0.0, p->tw);
    hipLaunchKernelGGL((k_rows_inv<L>), dim3(L / 2), dim3(L / conv_e(L)), 0, s, (const double2*)a->S, L, L, a->G, p->tw);
}

}  // namespace

template <int L>
void PerL<L>::slots(const Launch& c, int first_tag, int nslots, int kmax) { launch_slots_L<L>(c, first_tag, nslots, kmax); }
template <int L>
void PerL<L>::iteration(const Launch& c, int k) { launch_iteration_L<L>(c, k); }
template <int L>
void PerL<L>::conv(Plan* p, const double* Y, double* out, double2* X) { launch_conv<L>(p, Y, out, X); }
template <int L>
void PerL<L>::spectrum(Plan* p, const double* G, double2* Xfull) { launch_spectrum<L>(p, G, Xfull); }
template <int L>
void PerL<L>::rows_fwd(Plan* p, const double* Y, hipStream_t s) { launch_rows_fwd<L>(p, Y, s); }
template <int L>
int PerL<L>::adj_step(Plan* p, const Launch& c, int s, int* kpred, const double* Y, const double* V, const double* E) {
    return ::lpide::detail::adj_step<L>(p, c, s, kpred, Y, V, E);
}
template <int L>
void PerL<L>::adj_kernel_grad(Plan* p, hipStream_t s) { launch_adj_kernel_grad<L>(p, s); }

template struct PerL<LPIDE_L>;

}  // namespace detail
}  // namespace lpide
