/*
 * lpide.h -- C ABI of the MI355X solver for two-asset exponential-Levy option
 * PIDEs (method of Moda, in 't Hout, Vanmaele and Benth, arXiv 2511.02700).
 *
 * The solver prices a European two-asset option u(S, T) by time-marching the
 * pricing PIDE u_t = A u - r u (Sec. 2.2, the initial value problem) with the
 * paper's discretization, written in log-moneyness y_i = ln(S_i / K) on a
 * uniform n x n grid:
 *   - the integral term is replaced by the artificial diffusion over R_I and
 *     the weighted sum B over the z-cells of R_II and R_III (Sec. 3.1), and B is
 *     applied as a zero-padded 2D FFT correlation (Sec. 3.2.2);
 *   - the diffusion term is the Kronecker-sum finite-difference matrix D
 *     (Sec. 3.2.1) and the pay-off is cell averaged near its kink (Sec. 3.2.3);
 *   - time stepping is the semi-Lagrangian theta-method with four damped
 *     quarter steps first and a fixed-point iteration on B in every step,
 *     started from an extrapolated value (Sec. 3.3, Algorithm 1).
 *
 * Conventions for every entry point:
 *   - All functions return an int status: LPIDE_OK (0) or a negative LPIDE_E_*
 *     code.  Nothing throws across the ABI.  lpide_last_error() returns a
 *     thread-local, NUL-terminated description of the last failure on the
 *     calling thread (valid until that thread's next failing call).
 *   - Grids are row-major n x n FP64 arrays V[j1 * n + j2] with
 *     y_1 = y_lo[0] + j1 h (slow index) and y_2 = y_lo[1] + j2 h (fast index).
 *   - Pointers documented as "device" must be device-accessible memory of the
 *     plan's HIP device (e.g. torch CUDA tensors' data_ptr()); "host" pointers
 *     are ordinary CPU memory.  The caller owns every input and output buffer.
 *   - A plan owns all of its device workspace.  Its work is queued on the
 *     stream given in lpide_opts.stream; a plan is not re-entrant (calls on one
 *     plan must not overlap), different plans are independent.
 */
#ifndef LPIDE_H
#define LPIDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LPIDE_OK        0
#define LPIDE_E_PARAM  -1   /* invalid argument (parameter out of range, NULL pointer, size) */
#define LPIDE_E_NOCONV -2   /* fixed-point iteration did not meet tol within max_iter in some step */
#define LPIDE_E_NAN    -3   /* a NaN or Inf appeared in the fixed-point increments */
#define LPIDE_E_HIP    -4   /* a HIP runtime call failed (no device, launch failure, ...) */
#define LPIDE_E_OOM    -5   /* device or host allocation failed */

/* pay-off kinds, all with strike K: payoff(S) = max(g(S), 0) */
#define LPIDE_PUT_AVG   0   /* K - (S1 + S2)/2   (put-on-the-average, Sec. 4) */
#define LPIDE_CALL_AVG  1   /* (S1 + S2)/2 - K */
#define LPIDE_PUT_1     2   /* K - S1 */
#define LPIDE_CALL_1    3   /* S1 - K */
#define LPIDE_EXCHANGE  4   /* S1 - S2  (K only sets the log-moneyness origin) */
#define LPIDE_SPREAD    5   /* S1 - S2 - K  (spread call, among the extensions of Sec. 5) */

/* Arithmetic of the FFT correlation.  In the mixed form the fixed-point
 * iterations apply B in FP32 to increments only (Y^0 - V^{n-1}, then
 * Y^k - Y^{k-1}) and accumulate B Y^k in FP64, with twiddles entering in FP64
 * accuracy (split into two FP32 parts).  B V^{n-1} is carried in FP64 from one
 * step to the next (the previous step's accumulated B Y) and computed afresh by
 * the FP64 correlation every lpide_opts.mixed_anchor steps.  The FP32 error is
 * relative to the increments, so prices stay within about 1e-8 relative of the
 * FP64 form.  Without jumps the precision has no effect. */
#define LPIDE_FP64       0  /* everything in FP64 */
#define LPIDE_FP32_CONV  1  /* iteration correlations in FP32 on increments, all else FP64 */

/* Spatial grid and integral-discretization settings (Sec. 3.1, Sec. 4 settings). */
typedef struct {
    int32_t n;            /* nodes per axis, both ends included; 8 <= n <= 4096, and the
                             FFT side (lpide_opts.fft_size; at least n + N_z + 1) must not
                             exceed 4096 */
    double  y_lo[2];      /* lower ends of the log-moneyness axes y_i = ln(S_i/K) */
    double  y_hi[2];      /* upper ends; y_hi[i] - y_lo[i] must be equal on both axes,
                             so that one mesh width h = (y_hi - y_lo)/(n - 1) serves
                             both axes and the z-grid (h_z = h) */
    int32_t sl_order;     /* Lagrange order of the semi-Lagrangian interpolation T^SL:
                             1 (bilinear) or 3 (bicubic, the paper's choice) */
    int32_t in_order;     /* Lagrange order of the half-cell interpolation T^in from the
                             grid to the y^in grid, 1 or 3 (paper: 3) */
    int32_t m1;           /* z_max^I = m1 h (paper: 2) */
    double  ell_cut;      /* z_max^III level: largest |z|_inf with l(z) = ell_cut
                             (1e-14 reproduces the paper's printed values) */
    double  zmax2_frac;   /* z_max^II = h ceil(zmax2_frac N_z - 1/2) (paper: sqrt(0.1)) */
    int32_t gl_nodes;     /* Gauss-Legendre nodes per axis for the R_II cell integrals */
    int32_t nz_fixed;     /* 0: N_z = ceil(z_max^III / h) (Sec. 4); > 0: N_z fixed to this value
                             (frozen structure: plans that differ only in the model parameters
                             then share N_z, M2, the kernel window and the FFT side) */
} lpide_grid;

/* Model (Sec. 2.1, Sec. 4): r, the 2D NTS Levy measure and an optional
 * independent Brownian covariance sigma sigma^T. */
typedef struct {
    double  r;            /* risk-free rate */
    double  alpha;        /* NTS index, 0 <= alpha < 1 (0: VG, 1/2: NIG) */
    double  delta;        /* NTS delta > 0 */
    double  lambda;       /* NTS lambda > 0 */
    double  eta[2];       /* NTS drift of the subordinated Brownian motion */
    double  rho[3];       /* NTS covariance rho11, rho12, rho22 (positive definite) */
    double  sigma_bs[3];  /* Brownian covariance (sigma sigma^T)_11, _12, _22; the paper
                             takes 0; must be positive semi-definite */
    int32_t no_jumps;     /* 1: zero Levy measure (Black-Scholes); NTS fields ignored */
} lpide_levy;

typedef struct {
    int32_t kind;         /* LPIDE_PUT_AVG ... */
    double  K;            /* strike > 0; also the log-moneyness origin y = ln(S/K) */
    double  T;            /* maturity > 0 */
    int32_t cell_avg;     /* 1: cell averaging of the pay-off near its kink (Sec. 3.2.3) */
} lpide_payoff;

typedef struct {
    double  tol;          /* fixed-point stopping tolerance on
                             max|Y^k - Y^{k-1}| / max(1, |Y^k|)  (Sec. 3.3) */
    int32_t max_iter;     /* fixed-point iterations allowed per time step */
    int32_t precision;    /* LPIDE_FP64 or LPIDE_FP32_CONV */
    int32_t damping;      /* 1: first step replaced by 4 steps of dt/4 with theta = 1 */
    int32_t device;       /* HIP device ordinal */
    void*   stream;       /* hipStream_t for all of the plan's work (NULL: null stream) */
    int32_t fft_radix;    /* elements per thread of every FFT kernel of the march, i.e. the radix
                             of their power-of-two stages: 4, 8 or 16 (16 needs a transform of
                             >= 256; at L = 3 * 2^m, L / fft_radix must be a multiple of 64);
                             0: a default per kernel class and transform size */
    int32_t fft_size;     /* side L of the zero-padded correlation transform: 0 picks the
                             smallest of 64, 128, 256, 512, 1024, 1536, 2048, 3072, 4096 that
                             is >= n + max(-d_lo, d_hi) (the support of the folded kernel);
                             otherwise one of the supported sizes 64, 128, 256, 512, 768, 1024,
                             1536, 2048, 3072, 4096 that is at least that bound (LPIDE_E_PARAM
                             if not).  Ignored without jumps. */
    int32_t mixed_anchor; /* mixed form: B V^{n-1} is computed afresh by the FP64 correlation
                             every mixed_anchor steps (the first step of a march always); in
                             the steps between it is carried from the previous step's FP64
                             sum B Y.  0: 8.  1: every step. */
    int32_t all_correlations; /* FP64 form with jumps.  0: two products of Algorithm 1 are
                             taken without the correlation.  (a) The explicit part of a
                             step, E = V + dt (1 - theta) A V, from the implicit equation of
                             the step before it, (I - c A) V = W with c = dt theta of that
                             step: E = V + dt (1 - theta) (V - W) / c.  (b) B Y^0 of the first
                             iteration from the products B V stored for the grids of the
                             start-value combination Y^0 = sum coef V (each is B applied to
                             the last iterate of its step).  Both are exact at the fixed
                             point of the theta-scheme (Sec. 3.3): (a) carries the stopping
                             rule's residual, (b) only moves the start of the iteration.
                             The first steps of a march, whose grids did not come from it,
                             and steps after theta = 0 use the correlation.  1: every
                             product by the correlation, as Algorithm 1 reads. */
    int32_t accel;        /* price-space plan only (the log plan requires 0): acceleration of
                             the fixed-point iteration of Sec. 3.3.  0: the paper's iteration
                             Y^k = Y^{k-1} + delta^k.  1..6: Anderson mixing of that depth,
                             Y^k = Y^{k-1} + delta^k - sum_i gamma_i (dY_i + dF_i) with gamma
                             the least-squares fit of delta^k by the step's last differences
                             of increments dF (dY: of iterates); same fixed point and stopping
                             rule, fewer iterations where the iteration contracts slowly.
                             -1: depth 4 when the predicted contraction h_t theta sum_omega /
                             (1 + h_t theta sum_omega) of the main steps exceeds 0.3, else 0. */
} lpide_opts;

/* Plan-time quantities and run statistics. */
typedef struct {
    int32_t n, N_z, M1, M2, L;        /* grid size, z-grid half size, region bounds, FFT side */
    int32_t N_t, n_steps;             /* time steps, entries of the step list (N_t + 3 damped) */
    double  h, z_star;                /* mesh width, z_max^III before rounding to the z-grid */
    double  sum_omega;                /* sum of the weights */
    double  kappa[2], r_omega;        /* modified drift coefficients and kill rate (Sec. 3.1) */
    double  S[3];                     /* artificial diffusion over R_I (11, 12, 22) */
    double  a[3];                     /* sigma_omega sigma_omega^T = sigma sigma^T + S */
    int64_t total_iters;              /* fixed-point iterations summed over the last solve */
    int32_t max_step_iters;           /* largest per-step count in the last solve */
    int32_t last_step_iters;
    double  last_increment;           /* last stopping-rule value of the last solve */
    int64_t device_bytes;             /* device memory held by the plan */
    int32_t radix[4];                 /* FFT elements per thread (radix schedule) of the march's
                                         column pass, row c2r kernels, line-row kernel, SL kernel */
} lpide_info;

/* Default settings: the paper's scheme settings (Sec. 4) on an n x n grid over
 * [y_lo, y_hi]^2: sl_order = in_order = 3, m1 = 2, ell_cut = 1e-14,
 * zmax2_frac = sqrt(0.1), gl_nodes = 8, nz_fixed = 0. */
void lpide_grid_default(lpide_grid* g, int32_t n, double y_lo, double y_hi);

/* Defaults: tol = 1e-12, max_iter = 100, FP64, damping on, device 0, NULL stream. */
void lpide_opts_default(lpide_opts* o);

/* Fill an lpide_levy from the subordinated-Brownian-motion parameters: Brownian
 * volatilities sigma1, sigma2 > 0 and correlation corr in (-1, 1) (rho), drifts
 * theta1, theta2 (eta), subordinator variance kappa > 0 with unit mean, index
 * alpha in [0, 1).  From Table 4: lambda = (1 - alpha)/kappa and
 * delta = lambda^(1-alpha)/Gamma(1-alpha).  sigma_bs is set to 0.
 * Returns LPIDE_E_PARAM for out-of-range input. */
int lpide_levy_from_std(double sigma1, double sigma2, double corr, double theta1, double theta2,
                        double kappa, double alpha, double r, lpide_levy* out);

/* Build a plan: host-side discretization (z-grid sizes, weights, artificial
 * diffusion, drift and kill rate, cell-averaged pay-off, line-solve factors,
 * semi-Lagrangian weights) and, on the device, the kernel spectrum of the FFT
 * correlation and all workspace.  theta in [0, 1]; M = N_t >= 1 time steps of
 * size T / M (Sec. 3.3).  Validation errors (LPIDE_E_PARAM): n out of range,
 * unequal axis widths, orders not in {1, 3}, alpha outside [0,1), delta,
 * lambda, K, T <= 0, rho not positive definite, sigma_bs not positive
 * semi-definite, lambda - eta_i - rho_ii/2 <= 0 (no exponential moment),
 * theta outside [0, 1], tol <= 0, max_iter < 1.  *out is set only on success. */
int lpide_plan_create(const lpide_grid* grid, const lpide_levy* levy, const lpide_payoff* payoff,
                      double theta, int32_t M, const lpide_opts* opts, void** out);

/* Release a plan and its device memory.  NULL is accepted. */
int lpide_plan_destroy(void* plan);

/* Copy the plan's quantities and the last solve's statistics to *info (host). */
int lpide_plan_info(void* plan, lpide_info* info);

/* Full march (Algorithm 1): V^0 -> V^{N_t}.  v_out: device, n*n FP64.  Returns
 * LPIDE_E_NOCONV if some step needs more than max_iter iterations, LPIDE_E_NAN
 * if an increment is not finite.  Synchronises the plan's stream before it
 * returns (the per-iteration stopping rule is read back on the host). */
int lpide_solve(void* plan, double* v_out);

/* The first `steps` entries of the step list only (0 <= steps <= n_steps): the
 * state after them, for step-by-step comparisons.  v_out: device, n*n. */
int lpide_solve_steps(void* plan, int32_t steps, double* v_out);

/* Entries [s0, s1) of the step list starting from the state v_in (the state
 * after the first s0 entries; device, n*n, not modified), result in v_out
 * (device, n*n; may equal v_in).  The extrapolated start values (Sec. 3.3)
 * restart from v_in alone, so the result equals an uninterrupted march to the
 * fixed-point tolerance, not bit for bit.  0 <= s0 <= s1 <= n_steps. */
int lpide_solve_range(void* plan, int32_t s0, int32_t s1, const double* v_in, double* v_out);

/* Cell-averaged initial grid V^0 (Sec. 3.2.3).  v_out: device, n*n. */
int lpide_initial(void* plan, double* v_out);

/* One application of the summation operator (B v)_m = sum_l omega_l v^in_{m+l}
 * (Sec. 3.2.2) by the FFT correlation.  v, bv: device, n*n, must not alias. */
int lpide_apply_B(void* plan, const double* v, double* bv);

/* Allocation-free variant of lpide_apply_B, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same correlation and the same kernels, with the
 * transposed intermediate in a library-owned static device array of
 * LPIDE_NOALLOC_SCRATCH_BYTES per GPU (held until the process ends) instead of
 * the plan's workspace.  The call itself allocates and frees nothing; the
 * array's device address is taken when the first plan on a device is created.
 * v, bv: device, n*n FP64, must not alias.  Needs n * (L/2 + 1) * 16 bytes of
 * scratch (L = the plan's transform side): larger plans are refused with
 * LPIDE_E_PARAM before anything is enqueued.  Every call on one GPU uses the
 * same array (its contents are fully rewritten by each call; nothing needs to
 * start at zero), so calls that overlap on one GPU -- on different streams or
 * from different threads -- race; serialise them.  A plan without a Levy
 * measure gets bv = 0 from a fill kernel (no memset node). */
#define LPIDE_NOALLOC_SCRATCH_BYTES (64u << 20)
int lpide_apply_B_noalloc(void* plan, const double* v, double* bv);

/* Prices (and deltas) at npts spot pairs by tensor-product cubic Lagrange
 * interpolation of the grid v in y (Sec. 4): spots[2k], spots[2k+1] = (S1, S2);
 * price[k]; delta[2k + i] = dP/dS_i (delta may be NULL).  All device pointers;
 * with npts = 0 nothing is read or written and spots, price may be NULL. */
int lpide_price(void* plan, const double* v, int32_t npts, const double* spots,
                double* price, double* delta);

/* Delta and Gamma surfaces of a grid solution at the nodes (Sec. 4 plots them
 * over the spot plane).  With S_i = K e^{y_i}:
 *   delta_i = V_{y_i} / S_i,  gamma_ii = (V_{y_i y_i} - V_{y_i}) / S_i^2,
 *   gamma_12 = V_{y_1 y_2} / (S_1 S_2),
 * the y-derivatives by second-order differences: central inside, one-sided
 * (-3, 4, -1)/2h and (2, -5, 4, -1)/h^2 on the edges; V_{y_1 y_2} is the first
 * difference along axis 1 of the first difference along axis 2.
 * v: device, n*n FP64 (the layout lpide_solve writes); out: device, 5*n*n FP64,
 * caller-owned, must not alias v: delta1, delta2, gamma11, gamma12, gamma22, each
 * n*n row-major.  Enqueued on the plan's stream (no synchronisation). */
int lpide_greeks(void* plan, const double* v, double* out);

/* Host-only discretization (no device is touched): fills info (n, N_z, M1, M2,
 * L, h, z_star, sum_omega, kappa, r_omega, S, a) and, if omega is not NULL and
 * omega_len >= (2 N_z)^2, the weights omega[(l1 + N_z) * 2 N_z + (l2 + N_z)].
 * payoff may be NULL; if v0 is not NULL (host, n*n) it receives V^0. */
int lpide_discretize_host(const lpide_grid* grid, const lpide_levy* levy, const lpide_payoff* payoff,
                          lpide_info* info, double* omega, int64_t omega_len, double* v0);

/* Kernel classes for lpide_timing / lpide_kernel_stats.  Classes 0-3 run once
 * per fixed-point iteration, 4-8 once per time step. */
#define LPIDE_K_COLS       0   /* column pass of B Y: FFT, spectrum multiply, inverse FFT
                                  (FP32 in the mixed form) */
#define LPIDE_K_ROWS_INV   1   /* row inverse FFTs + fused residual stencil */
#define LPIDE_K_LINE_COLS  2   /* line solves along axis 1 */
#define LPIDE_K_LINE_ROWS  3   /* line solves along axis 2 + update + stopping rule + row FFT
                                  of Y (of the increment in the mixed form) */
#define LPIDE_K_SL         4   /* semi-Lagrangian gather + extrapolated start + row FFT of Y^0 */
#define LPIDE_K_STEP_END   5   /* end-of-step control (convergence verdict, history rotation) */
#define LPIDE_K_EXPL_COLS  6   /* FP64 column pass of B V^{n-1} (theta < 1: first step of a march or
                                  all_correlations; mixed form: anchor steps) */
#define LPIDE_K_EXPL_ROWS  7   /* row inverse FFTs + explicit part (E, and B V^{n-1} at mixed anchors) */
#define LPIDE_K_ROWS_FWD   8   /* FP64 row FFTs of V^{n-1} (mixed form, anchor steps) */
#define LPIDE_K_CARRY      9   /* mixed form between anchors: B V^{n-1} carried, explicit part */
#define LPIDE_K_EXPL_ID   10   /* FP64: explicit part from the previous step's implicit equation */
#define LPIDE_K_ROWS_LIN  11   /* FP64 iteration 1 with B Y^0 by linearity: residual from the stored
                                  products (the column pass and the row c2r kernel exit) */
#define LPIDE_K_SL_LIN    12   /* FP64 steps with B Y^0 by linearity: SL gather and start value without
                                  the row transform (the SL kernel exits) */
#define LPIDE_KCLASSES    13

/* Kernel timing.  With bit c of class_mask set, every launch of kernel class c
 * in single-plan marches carries a start and a stop HIP event bound to the
 * dispatch itself (hipExtLaunchKernel), so the elapsed time is the kernel's
 * own duration; the times are summed per class.  Each call resets the
 * counters (after folding in pending events).  class_mask = 0 disables timing
 * (the default). */
int lpide_timing(void* plan, uint32_t class_mask);

/* Per-class launch counts and summed durations in milliseconds since the last
 * lpide_timing call (host arrays of LPIDE_KCLASSES entries).  Synchronises the
 * plan's stream. */
int lpide_kernel_stats(void* plan, int64_t* launches, double* ms);

/* ---- Adjoint (reverse-mode) form ----
 * The cotangent of the whole march (Algorithm 1 as a function of the model):
 * for J with dJ/dV^{N_t} = v_bar, each step n (V^{n-1} -> Y = V^n, the exact
 * fixed point of (I - dt theta A) Y = T^SL (I + dt (1 - theta) A) V^{n-1},
 * A = D + B - r_omega, Sec. 3.3) is reversed as
 *   lam = (I - dt theta A)^{-T} Ybar      (transposed preconditioned iteration:
 *                                          B^T by the conjugate spectrum, D^T,
 *                                          transposed line solves; stopping rule
 *                                          and tol as the forward),
 *   mu = (T^SL)^T lam,  Vbar^{n-1} = (I + dt (1 - theta) A)^T mu,
 * and the step's terms of dJ/d(a11, a12, a22, r_omega, kappa_omega, K) are
 * accumulated (K: the folded kernel, by a spectral cross-correlation of lam
 * with Y and of mu with V^{n-1}).  States come from checkpoints every
 * checkpoint_every steps; each segment is recomputed with recording before it
 * is reversed.  A checkpoint_every of at least the step count (lpide_info
 * n_steps) keeps every state and explicit part of the forward march instead,
 * (2 n_steps + 1) n^2 FP64 (8.5 GB at n = 1024, 512 time steps), and the
 * reverse march runs without recompute.  The structure (N_z, M2, L, stencil
 * starts) is held fixed. */
typedef struct {
    int64_t adj_iters;                /* adjoint fixed-point iterations, summed over the steps */
    int32_t max_step_iters;
    double  forward_ms;               /* checkpointed forward (0 when the last solve recorded them) */
    double  recompute_ms, reverse_ms, gather_ms, jacobian_ms;
} lpide_adjoint_info;

/* Keep checkpoints in later lpide_solve calls (every `every` steps; 0: off;
 * at least the step count: every state and explicit part), so that an
 * lpide_adjoint with the same stride skips its forward pass. */
int lpide_plan_set_checkpoints(void* plan, int32_t every);

/* v_bar: device n*n.  native (host, may be NULL): 6 + (2 N_z)^2 values,
 * dJ/d(a11, a12, a22, r_omega, kappa_omega1, kappa_omega2) then dJ/d omega_l at
 * index 6 + (l1 + N_z) * 2 N_z + (l2 + N_z).  grad (host[8], may be NULL):
 * dJ/d(sigma1, sigma2, corr, theta1, theta2, kappa, alpha, r), the
 * subordination parameters std_params (host[8], same order) the plan's model
 * was made from by lpide_levy_from_std (checked); the host quantities are
 * differentiated by central differences in the seven Levy parameters (step
 * 1e-4 max(|x|, 0.1), structure fixed) and exactly in r (it enters only
 * kappa_omega and r_omega, with unit slope); the Jacobian is cached per plan
 * and point.  Needs a plan with jumps.  The reverse march is FP64; on a
 * mixed-form plan the forward states it differentiates at (recomputed from
 * the checkpoints, with B V anchored at each checkpoint) carry the mixed
 * form's error.  Synchronises. */
int lpide_adjoint(void* plan, const double* v_bar, int32_t checkpoint_every, const double* std_params,
                  double* grad, double* native, lpide_adjoint_info* info);

/* Transpose of lpide_price: v_bar[node] = sum_k price_bar[k] w_k(node), the
 * cotangent of the grid for price cotangents price_bar (device arrays: spots
 * npts x 2, price_bar npts, v_bar n*n, overwritten; with npts = 0 v_bar is
 * zeroed and spots, price_bar may be NULL). */
int lpide_price_adjoint(void* plan, int32_t npts, const double* spots, const double* price_bar, double* v_bar);

/* ---- Batched form ----
 * Many independent plans (different grids, Levy parameters, pay-offs, step
 * counts) marched together.  Plans with the same row-kernel size (lpide_info.L,
 * or the power of two >= n without jumps), jump switch, precision and SL order
 * form a group: every march kernel is launched once for the whole group
 * (one grid, the plan in the second grid dimension), each plan converging and
 * stopping on its own.  Each group runs on a stream of its own, and the host
 * interleaves the groups.  With use_graph, a group's step slots (one step of
 * every plan each) are captured once in a hipGraph and replayed. */
typedef struct {
    int32_t use_graph;   /* 1: replay captured hipGraphs of the step slots (default) */
    int32_t slots;       /* step slots enqueued between host checks, 1..256 (default 32) */
    void*   stream;      /* hipStream_t of the caller: the batch's work starts after the work
                            queued on it before lpide_batch_solve, and later work on it waits for
                            the batch (NULL: the null stream) */
} lpide_batch_opts;

typedef struct {
    int32_t n_plans, L, mixed;        /* plans of the group, row-kernel size, mixed form */
    int32_t P_cols, slots, use_graph; /* launch configuration (set by lpide_batch_tune) */
    int32_t radix[4];                 /* radix schedule, as lpide_info.radix */
    double  trial_ms;                 /* wall time of the tuning trial kept (0 before tuning) */
} lpide_group_info;

void lpide_batch_opts_default(lpide_batch_opts* o);

/* Create a batch over count plans (host array of handles from
 * lpide_plan_create, all on one device).  The plans stay owned by the caller,
 * must outlive the batch and must not be used concurrently with it. */
int lpide_batch_create(int32_t count, void* const* plans, const lpide_batch_opts* opts, void** out);
int lpide_batch_destroy(void* batch);

/* Short forms of the plan calls: lpide_plan = lpide_plan_create,
 * lpide_destroy = lpide_plan_destroy (same arguments, ownership and errors). */
int lpide_plan(const lpide_grid* grid, const lpide_levy* levy, const lpide_payoff* payoff, double theta, int32_t M,
               const lpide_opts* opts, void** out);
int lpide_destroy(void* plan);

/* Plans and their batch in one call: plan i from grids[i], levys[i],
 * payoffs[i] (host arrays of count) with M[i] time steps, theta and opts shared
 * (opts may be NULL; its stream becomes the batch's caller stream), then a
 * batch over them with default batch options.  The batch owns these plans:
 * lpide_batch_destroy destroys them too.  On error nothing is left allocated
 * and the status of the first failing plan (or of the batch) is returned. */
int lpide_plan_batch(int32_t count, const lpide_grid* grids, const lpide_levy* levys, const lpide_payoff* payoffs,
                     double theta, const int32_t* M, const lpide_opts* opts, void** batch);

/* Same as lpide_batch_solve. */
int lpide_solve_batch(void* batch, double* const* v_out);

/* March every plan over its whole step list (Algorithm 1 per plan).  v_out:
 * host array of count device pointers, plan i's n_i * n_i FP64 result.
 * Returns when the results are queued on the caller's stream.  Errors as
 * lpide_solve, for the first plan that fails. */
int lpide_batch_solve(void* batch, double* const* v_out);

/* As lpide_batch_solve over the first min(steps, n_steps_i) entries of each
 * step list; v_out may be NULL (results not copied: timing and tuning). */
int lpide_batch_solve_steps(void* batch, int32_t steps, double* const* v_out);

/* Autotuner: for each group, march every plan once to step-list entry
 * min(8, n_steps) (past the damped block and the first main steps), then time
 * the march of the next trial_steps entries from there -- steady steps, as in
 * the bulk of a march -- under candidate launch configurations and keep the
 * fastest, in three passes: the FFT radix schedule (4, 8 or 16 elements per
 * thread, per kernel class, one class at a time from the default), the axis-1
 * line-solve chunking P_cols in {P/2, P, 2P} around the default P, then
 * hipGraph replay on/off with 32 step slots per host check, and with 16 when
 * trial_steps >= 32; each candidate runs twice with the second timed.
 * Allocates one n*n start state per plan for its duration.  Synchronises the
 * device work of the batch. */
int lpide_batch_tune(void* batch, int32_t trial_steps);

/* Groups of the batch: *n_groups, and up to cap entries of groups (may be NULL). */
int lpide_batch_info(void* batch, int32_t* n_groups, lpide_group_info* groups, int32_t cap);

/* Thread-local description of the last error on the calling thread. */
const char* lpide_last_error(void);

/* ---------------------------------------------------------------------------
 * The paper's own price-space discretization (Sec. 3.2, Sec. 3.3 and the
 * Sec. 4 settings), a second plan type beside the log-moneyness plan above.
 *
 * The grid is x_m = phi(xi_max m / N_x), m = 0..N_x, in each price axis:
 * uniform on [0, x_int], sinh-graded on [x_int, x_max] (Sec. 4), the same on
 * both axes.  Grids are row-major (N_x+1) x (N_x+1) FP64 arrays
 * V[m1 * (N_x+1) + m2] at (x_{m1}, x_{m2}).
 *   - D: three-point differences on the nonuniform grid with the x_i and x_i^2
 *     factors (Sec. 3.2.1); no derivative terms at x_i = 0, no second
 *     derivative and a backward first difference at x_max.
 *   - B_omega = T^out I~ C T^in (Sec. 3.2.2): cubic Lagrange interpolation
 *     T^in from the x grid to the log-uniform grid y^in (v = 0 outside
 *     [0, x_max]^2), the correlation C with the weights omega on
 *     #in x #in points by a zero-padded 2D FFT, the kept #out x #out outputs
 *     on y^out, and cubic Lagrange interpolation T^out back to the x grid
 *     (linear extrapolation to the x_i = 0 rows).  h_z = z_max^III / N_z with
 *     N_z = nz_per_nx N_x, N_y^-, N_y^+ and the least N_y^* that makes #in
 *     7-smooth as in Sec. 4.
 *   - Time stepping: the semi-Lagrangian theta-method of Sec. 3.3 with the
 *     departure points x e^{kappa_omega^(i) dt} (cubic Lagrange, stencils of
 *     the four nearest nodes, extrapolating beyond x_max), four damped
 *     quarter steps, extrapolated start values and the fixed-point
 *     iteration on B of Algorithm 1.  The implicit systems are solved by the
 *     same preconditioned iteration as the log-moneyness plan (tridiagonal
 *     line solves in each axis, residual of the full step equation), whose
 *     fixed point is the step equation's solution.
 * Pay-offs: LPIDE_PUT_AVG and LPIDE_PUT_1, cell averaged on the cells
 * [x_{m-1/2}, x_{m+1/2}]^2 that meet the kink when cell_avg = 1.  Options
 * used: tol, max_iter, damping, device, stream, fft_size (0: the smallest
 * supported transform side >= #in among 64, 128, 256, 512, 640, 896, 1024,
 * 1152, 1280, 1536, 1792, 2048, 2304, 2560, 3072, 3584, 4096, 4608, 5120,
 * 6144, 7168, 8192, 12288, 16384, 24576 (largest prime factor at most 7, as
 * Sec. 4 asks); otherwise one of these or 768, at least #in; sides above 8192
 * run as (3, 4, 6) transforms of length 4096 per sequence) and
 * all_correlations (0: the explicit part of a step after one
 * with theta > 0 from that step's implicit equation, as the log plan does;
 * 1: by the correlation).  precision must be LPIDE_FP64. */
typedef struct {
    int32_t N_x;          /* grid intervals per axis, 8 <= N_x <= 4095 */
    double  x_max;        /* upper end of both price axes */
    double  x_int;        /* end of the uniform part; 0: 5K/2 (Sec. 4) */
    double  fraction;     /* F target: c makes the limit fraction of nodes in [0, x_int]
                             max(fraction, x_int / x_max) (paper: 0.65) */
    double  c;            /* > 0: the constant of the map phi as given (Sec. 4 prints one
                             per parameter set); 0: the root of the relation for F */
    int32_t nz_per_nx;    /* N_z = nz_per_nx N_x (paper: 2) */
    int32_t m1;           /* z_max^I = m1 h_z (paper: 2) */
    double  ell_cut;      /* z_max^III level (1e-14 reproduces the printed values) */
    double  zmax2_frac;   /* z_max^II = h_z ceil(zmax2_frac N_z - 1/2) (paper: sqrt(0.1)) */
    int32_t gl_nodes;     /* Gauss-Legendre nodes per axis for the R_II cell integrals */
} lpide_ps_grid;

typedef struct {
    int32_t N_x, n;                   /* intervals, nodes per axis (N_x + 1) */
    int32_t N_z, M1, M2;              /* z-grid half size and region bounds */
    int32_t N_ym, N_yp, N_ystar;      /* N_y^-, N_y^+, N_y^* (Sec. 4) */
    int32_t n_in, n_out;              /* #in and #out per axis */
    int32_t n_nz;                     /* y^in nodes inside [0, x_max] (rows of T^in that are not zero) */
    int32_t L;                        /* side of the zero-padded correlation transform (>= #in) */
    int32_t N_t, n_steps;             /* time steps, entries of the step list */
    double  c, x_int, F;              /* grid constant, end of the uniform part, fraction target */
    double  h_z, z_star, sum_omega;
    double  kappa[2], r_omega, S[3], a[3];
    int64_t total_iters;              /* fixed-point iterations of the last march */
    int32_t max_step_iters;
    double  last_increment;           /* last stopping-rule value of the last march */
    int64_t device_bytes;
    int32_t accel_depth;              /* Anderson depth in use (0: the paper's iteration) */
} lpide_ps_info;

/* The paper's settings on N_x intervals over [0, x_max]: x_int = 5K/2,
 * fraction 0.65, c from the relation for F, N_z = 2 N_x, m1 = 2,
 * ell_cut = 1e-14, zmax2_frac = sqrt(0.1), gl_nodes = 8. */
void lpide_ps_grid_default(lpide_ps_grid* g, int32_t N_x, double x_max);

/* Host-only discretization of the price-space plan (no device is touched):
 * fills info (sizes of the grids, c, h_z, z_star, sum_omega, kappa, r_omega,
 * S, a; L is the automatic transform side, 0 without jumps) and, where not
 * NULL, x (host, N_x + 1 nodes), v0 (host, (N_x+1)^2 pay-off grid) and omega
 * (host, (2 N_z)^2 weights, only if omega_len is at least that).  Errors as
 * lpide_ps_plan_create's validation. */
int lpide_ps_discretize_host(const lpide_ps_grid* grid, const lpide_levy* levy, const lpide_payoff* payoff,
                             lpide_ps_info* info, double* x, double* v0, double* omega, int64_t omega_len);

/* Build a price-space plan: the grid, the integral discretization with
 * h_z = z_max^III / N_z, the y grids and interpolation tables, the
 * difference operator, the cell-averaged pay-off, the semi-Lagrangian tables
 * and line factors of every step kind, and on the device the spectrum of the
 * weights and all workspace.  N_t >= 1 steps of T / N_t (the paper takes
 * N_t = round(N_x / 2)).  Errors: LPIDE_E_PARAM for invalid settings (as
 * lpide_plan_create, plus x_max <= x_int, a pay-off other than the two above,
 * precision other than FP64, #in above the transform side or 24576),
 * LPIDE_E_OOM, LPIDE_E_HIP.  *out is set only on success. */
int lpide_ps_plan_create(const lpide_ps_grid* grid, const lpide_levy* levy, const lpide_payoff* payoff,
                         double theta, int32_t N_t, const lpide_opts* opts, void** out);

/* Release a price-space plan and its device memory.  NULL is accepted. */
int lpide_ps_plan_destroy(void* plan);

/* Plan quantities and last-march statistics (host). */
int lpide_ps_plan_info(void* plan, lpide_ps_info* info);

/* The grid nodes x_0 .. x_{N_x} (host array of N_x + 1). */
int lpide_ps_nodes(void* plan, double* x);

/* The cell-averaged pay-off V^0.  v_out: device, (N_x+1)^2. */
int lpide_ps_initial(void* plan, double* v_out);

/* One application of B_omega = T^out I~ C T^in.  v, bv: device, (N_x+1)^2,
 * must not alias.  Enqueued on the plan's stream. */
int lpide_ps_apply_B(void* plan, const double* v, double* bv);

/* The first `steps` entries of the step list (0 <= steps <= n_steps; the
 * whole march with steps = n_steps).  v_out: device, (N_x+1)^2.  Errors as
 * lpide_solve (LPIDE_E_NOCONV, LPIDE_E_NAN).  Synchronises the plan's
 * stream (the stopping rule is read back between batches of steps). */
int lpide_ps_solve_steps(void* plan, int32_t steps, double* v_out);

/* Delta and Gamma surfaces of a price-space grid at the nodes by the
 * difference schemes of D (Sec. 3.2.1; the paper plots them in Sec. 4):
 * delta_i = D1 along axis i, gamma_ii = D2 along axis i, gamma_12 = D1 along
 * both axes, with the coefficients of Sec. 3.2.1 (central three-point on the
 * nonuniform grid; zero on the x_i = 0 rows; at x_max the backward first
 * difference and no second derivative).  v: device, (N_x+1)^2; out: device,
 * 5 (N_x+1)^2 FP64, caller-owned, must not alias v: delta1, delta2, gamma11,
 * gamma12, gamma22.  Enqueued on the plan's stream. */
int lpide_ps_greeks(void* plan, const double* v, double* out);

/* Prices at npts spot pairs by tensor-product cubic Lagrange interpolation in
 * x (stencils of the four nearest nodes): spots[2k], spots[2k+1] = (S1, S2),
 * price[k].  Device pointers; npts = 0 reads and writes nothing. */
int lpide_ps_price(void* plan, const double* v, int32_t npts, const double* spots, double* price);

#ifdef __cplusplus
}
#endif
#endif /* LPIDE_H */
