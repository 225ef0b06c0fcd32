// Device-controlled time steps (Sec. 3.3, Algorithm 1) for gfx950.
//
// The host enqueues whole time steps without waiting: every step is
//   [explicit part: cols + rows_inv(explicit)]        (theta < 1 only)
//   sl        W = T^SL E, Y^0, and the row FFT of Y^0
//   kmax x {  cols          column pass of B Y (spectrum multiply)
//             rows_inv      R = W + dt theta ((D - r_omega) Y + B Y) - Y
//             line_cols     R <- T_1^{-1} R                 (axis 1)
//             line_rows     delta = T_2^{-1} R; Y += delta; err_k; row FFT of Y }
//   step_end  first k with err_k < tol; rotate the history; set up the next step
// Iteration k's kernels return at once when err_{k-1} < tol (the step has
// converged) or when a step failed to converge within its kmax iterations
// (then everything after it is a no-op until the host has added iterations).
// All buffers are addressed through a control block updated only by step_end,
// so the same launch sequence serves every step, whatever its kind (the
// explicit-part kernels return at once in theta = 1 steps of the FP64 form).
//
// Every kernel serves a group of independent plans with the same transform
// size: blockIdx.y selects the plan (its MarchArgs in device memory), and each
// plan has its own control block, so plans advance, converge and stop
// independently inside one launch.
//
// Mixed form (FP32 correlation, FP64 everything else): each step first applies
// B to V^{n-1} in FP64 (BV, and the explicit part), then the iteration
// correlations run in FP32 on increments only: B Y^0 = BV + B32(Y^0 - V^{n-1})
// and B Y^k = B Y^{k-1} + B32(delta^k), accumulated in FP64.  FP32 rounding is
// thus relative to the increments, which shrink geometrically, and does not
// accumulate across steps.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "fft.hpp"
#include "kernels.hpp"
#include "linesolve.hpp"

namespace lpide {

constexpr int KSLOTS = 136;          // err[.][0] (sentinel) + up to 128 iterations per step
constexpr int NX = 8;                 // stopping-rule partial maxima per iteration (one per XCD)
constexpr int MAX_ITER_CAP = 128;
constexpr int POOL = 6;               // grid buffers: history (4) + start state + iterate

struct Ctl {
    int step;                         // completed entries of the step list
    int fail;                         // current step not converged within its launched iterations
    int fail_step;
    int hold;                         // set by the host while another plan of the group is being completed
    int cur;                          // pool index of the state the current step starts from
    int y;                            // pool index of the iterate
    int hc;                           // history length (main steps)
    int nsrc;                         // terms of the starting-value combination
    int hist[4];                      // pool indices, newest first
    int bvalid;                       // bit b: bpool[b] holds B applied to pool[b] (this march)
    int src[4];
    double coef[4];                   // Y^0 = sum_q coef[q] pool[src[q]]; past nsrc,
                                      // src[q] = src[0] and coef[q] = 0 (so a loop
                                      // over all four terms gives the same sums)
    // stopping-rule value after iteration k: the maximum over x of err[x][k]
    // (bit patterns of non-negative doubles).  The row blocks of the line-solve
    // kernel reduce into the partial of their XCD, so the atomics of one launch
    // go to eight cache lines instead of one (they are serialised per line).
    unsigned long long err[NX][KSLOTS];
};

struct StepDesc {
    double theta, dt;
    const double *fl1, *bu1, *bc1;    // axis-1 line factors of I - dt theta A_1
    const double *fl2, *bu2, *bc2;    // axis-2 line factors
    const int *s1, *s2;               // semi-Lagrangian stencil starts per axis
    const double *w1, *w2;            // semi-Lagrangian weights per axis
    // adjoint march only (null otherwise): transposed SL matrices per axis
    // (source rows and weights, padded to widths wt1, wt2) and the weight
    // derivatives with respect to the drift coefficient kappa_omega^(i)
    const int *t1i, *t2i;
    const double *t1w, *t2w;
    int wt1, wt2;
    const double *w1d, *w2d;
};

struct MarchArgs {
    Ctl* ctl;
    double* pool[POOL];
    const StepDesc* sets;
    const int* step_set;
    int n, n_sub, damping, P_cols;
    double* W;
    double* R;
    double2* X;
    const double2* spec;
    const double2* tw;
    int* counts;
    double* incs;
    double tol, r_omega;
    StencilArgs st;
    int mixed;                        // FP32 iteration correlations on increments
    float2* X32;                      // FP32 intermediate (mixed form)
    const float2* spec32;             // FP32 spectrum (mixed form)
    double* BV;                       // B V^{n-1}, FP64 (mixed form)
    double* BY;                       // B Y^k accumulated in FP64 (mixed form)
    int nsteps;                       // step-list entries to march (the plan stops after them)
    int step0;                        // step-list index of the state in pool[0] at the start
    double* seg;                      // recorded states: V^s to seg[(s - seg_base) / seg_every] (or null)
    double* segE;                     // recorded explicit parts E_s = M_E V^s to segE[s - seg_base] (theta < 1)
    int seg_base, seg_every;
    int anchor_every;                 // mixed form: B V^{n-1} afresh in FP64 every this many steps
    const double* cn_rho;             // per step: rho of the explicit part from the previous step's
                                      // implicit equation (0: by the correlation); null: never
    double* bpool[POOL];              // B applied to the pool grids (FP64 form; bpool[0] null: off)
};

template <typename C> __device__ __forceinline__ C* xbuf(const MarchArgs& a);
template <> __device__ __forceinline__ double2* xbuf<double2>(const MarchArgs& a) { return a.X; }
template <> __device__ __forceinline__ float2* xbuf<float2>(const MarchArgs& a) { return a.X32; }
template <typename C> __device__ __forceinline__ const C* specbuf(const MarchArgs& a);
template <> __device__ __forceinline__ const double2* specbuf<double2>(const MarchArgs& a) { return a.spec; }
template <> __device__ __forceinline__ const float2* specbuf<float2>(const MarchArgs& a) { return a.spec32; }

__device__ __forceinline__ double bits_to_d(unsigned long long b) { return __longlong_as_double((long long)b); }

// Stopping-rule value after iteration k (maximum of the partials).
__device__ __forceinline__ double err_max(const Ctl* c, int k) {
    unsigned long long m = c->err[0][k];
#pragma unroll
    for (int x = 1; x < NX; ++x) m = c->err[x][k] > m ? c->err[x][k] : m;
    return bits_to_d(m);
}

// Reset the stopping-rule partials (err[.][0] = +inf sentinel); by all threads of a block.
__device__ __forceinline__ void err_reset(Ctl* c) {
    for (int q = threadIdx.x; q < NX * KSLOTS; q += blockDim.x)
        c->err[q / KSLOTS][q % KSLOTS] = (q % KSLOTS) == 0 ? 0x7FF0000000000000ull : 0ull;
}

// The same for slots 0..kmax only: a step that ran iterations 1..kmax wrote
// no other slot, and every other slot is still zero from an earlier reset.
__device__ __forceinline__ void err_reset_upto(Ctl* c, int kmax) {
    const int w = kmax + 1;
    for (int q = threadIdx.x; q < NX * w; q += blockDim.x)
        c->err[q / w][q % w] = (q % w) == 0 ? 0x7FF0000000000000ull : 0ull;
}

// Uniform early-exit test of iteration k (k = 0: parts that run once per step).
__device__ __forceinline__ bool halted(const MarchArgs& a, int k) {
    const Ctl* c = a.ctl;
    if (c->fail || c->hold || c->step >= a.nsteps) return true;
    return k > 0 && err_max(c, k - 1) < a.tol;
}

// The explicit part (and the FP64 correlation of V^{n-1}) is needed when
// theta < 1, and in every step of the mixed form.
__device__ __forceinline__ bool needs_explicit(const MarchArgs& a);

__device__ __forceinline__ const StepDesc& cur_set(const MarchArgs& a) { return a.sets[a.step_set[a.ctl->step]]; }

__device__ __forceinline__ bool needs_explicit(const MarchArgs& a) { return a.mixed || cur_set(a).theta < 1.0; }

// Mixed form: the steps whose B V^{n-1} is computed afresh by the FP64
// correlation (every anchor_every-th step of the march, its first step
// included).  In the others B V^{n-1} is carried from the previous step: its
// last accumulated B Y, still in BY when the step's first iteration adds to it.
__device__ __forceinline__ bool is_anchor(const MarchArgs& a) {
    return (a.ctl->step - a.step0) % a.anchor_every == 0;
}

// Explicit part of a step from the implicit equation of the step before it.
// That step solved (I - c A) V^{n-1} = W (c = dt theta of that step, W still
// in a.W), so A V^{n-1} = (V^{n-1} - W) / c and
//   E = V^{n-1} + dt (1 - theta) A V^{n-1} = V^{n-1} + rho (V^{n-1} - W),
// rho = dt (1 - theta) / c: the same explicit part without applying B, exact
// at the fixed point (the converged iterate leaves the stopping-rule residual).
// Used from the second step of a march on, when the previous step had
// theta > 0 (cn_rho > 0, set by the host; null with every product by the
// correlation and in the adjoint march); in the mixed form outside its anchor
// steps, whose FP64 correlation forms the explicit part.
__device__ __forceinline__ bool explicit_by_identity(const MarchArgs& a) {
    return a.cn_rho && a.ctl->step > a.step0 && a.cn_rho[a.ctl->step] > 0.0;
}

// B Y^0 of the first iteration by linearity: Y^0 = sum_q coef_q V^{src_q}, so
// B Y^0 = sum_q coef_q B V^{src_q}, with B V^{src_q} stored by the row kernel of
// the step that produced V^{src_q} (B applied to its last iterate before the
// final update, so B V^{src_q} is off by B of an increment below the stopping
// tolerance; the first iteration only sets where the iteration starts, its
// fixed point is unchanged).  Needs every source grid from this march.
__device__ __forceinline__ bool start_by_linearity(const MarchArgs& a) {
    if (!a.bpool[0]) return false;
    const Ctl* c = a.ctl;
    bool ok = true;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (q < c->nsrc) ok = ok && ((c->bvalid >> c->src[q]) & 1);
    return ok;
}

// Whether the step runs the FP64 correlation of V^{n-1}: for the explicit part
// (theta < 1, unless it comes from the previous step's equation), or to anchor
// B V^{n-1} in the mixed form.
__device__ __forceinline__ bool needs_explicit_fft(const MarchArgs& a) {
    return a.mixed ? is_anchor(a) : (cur_set(a).theta < 1.0 && !explicit_by_identity(a));
}

// The plan of this block.
__device__ __forceinline__ const MarchArgs& plan_args(const MarchArgs* __restrict__ A) { return A[blockIdx.y]; }

// Column pass of the correlation on the intermediate X (transposed half
// spectra), FP64 (C = double2) or FP32 (C = float2); L/2 blocks for the
// L/2 + 1 columns.  Columns 0 (DC) and L/2 (Nyquist) hold real values (the row
// transforms of real rows; the row c2r kernels read only their real parts), so
// block 0 filters both as one complex column (mul_real_pair): a launch of
// L/2 + 1 blocks would end with one block running alone after the last full
// set of resident blocks had finished.
// CONJ (adjoint march): multiply by the conjugate spectrum, which applies B^T
// (the correlation with the reflected kernel).
template <int L, int E, typename C, bool CONJ = false>
__global__ __launch_bounds__(L / E) void ks_cols(const MarchArgs* __restrict__ A, int k) {
    const MarchArgs& a = plan_args(A);
    if (halted(a, k) || (k == 0 && !needs_explicit_fft(a)) || (k == 1 && start_by_linearity(a))) return;
    constexpr int T = L / E;
    __shared__ C lds[lds_slots(L)];
    __shared__ double2 tw4[tw_slots<L, E>()];
    load_twiddles<L, E>(a.tw, tw4);
    const int n = a.n, col = blockIdx.x, tid = threadIdx.x;
    C reg[E];
    if (col == 0) {
        C* x0 = xbuf<C>(a);
        C* xh = x0 + (size_t)(L / 2) * n;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = tid + e * T;
            reg[e] = idx < n ? CplxOps<C>::make(x0[idx].x, xh[idx].x) : CplxOps<C>::make(0, 0);
        }
        fft_block<L, E, false>(reg, lds, tw4);
        mul_real_pair<L, E, CONJ>(reg, lds, specbuf<C>(a), specbuf<C>(a) + (size_t)(L / 2) * L);
        fft_block<L, E, true>(reg, lds, tw4);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = tid + e * T;
            if (idx < n) {
                x0[idx] = CplxOps<C>::make(reg[e].x, 0);
                xh[idx] = CplxOps<C>::make(reg[e].y, 0);
            }
        }
        return;
    }
    C* xc = xbuf<C>(a) + (size_t)col * n;
    const C* sc = specbuf<C>(a) + (size_t)col * L;
    C sp[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int idx = tid + e * T;
        reg[e] = idx < n ? xc[idx] : CplxOps<C>::make(0, 0);
        sp[e] = sc[idx];                  // spectrum fetched up front, used after the forward FFT
    }
    fft_block<L, E, false>(reg, lds, tw4);
#pragma unroll
    for (int e = 0; e < E; ++e) reg[e] = CONJ ? cmulc(reg[e], sp[e]) : cmul(reg[e], sp[e]);
    fft_block<L, E, true>(reg, lds, tw4);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int idx = tid + e * T;
        if (idx < n) xc[idx] = reg[e];
    }
}

// Forward FFT of the row pair (ra, ra+1) of the FP64 grid U at the step start
// (mixed form: the FP64 correlation of V^{n-1}).
template <int L, int E>
__global__ __launch_bounds__(L / E) void ks_rows_fwd(const MarchArgs* __restrict__ A);

// The packed spectrum of the row pair (ra, ra+1) from the transposed half
// spectra, into the canonical registers: z[k] = X_a[k] + i X_b[k] for k <= L/2
// and z[L-k] = conj(X_a[k]) + i conj(X_b[k]) (imaginary parts dropped at DC and
// Nyquist).  Item idx is frequency (idx >> 1) of row ra + (idx & 1), so a lane
// pair reads the 32 contiguous bytes of one frequency once; the pair swaps its
// values, the even lane forms z[k], the odd one z[L-k], and both go through LDS
// to the canonical layout.
template <int L, int E, typename C>
__device__ __forceinline__ void rows_inv_gather(C (&reg)[E], C* lds, const C* __restrict__ X, int n, int ra,
                                                bool hasb) {
    constexpr int T = L / E, NI = (L + 2 + T - 1) / T;
    const int tid = threadIdx.x;
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int idx = tid + it * T;
        const int kk = idx >> 1, r = idx & 1;
        const bool in = kk <= L / 2;
        const C v = (in && (r == 0 || hasb)) ? X[(size_t)kk * n + ra + r] : CplxOps<C>::make(0, 0);
        // every lane of the wave takes part in the swap (pairs never straddle the range end)
        const C u = CplxOps<C>::make(__shfl_xor(v.x, 1), __shfl_xor(v.y, 1));
        const bool real_bin = kk == 0 || kk == L / 2;
        const C ta = r == 0 ? v : u, tb = r == 0 ? u : v;
        const C ha = CplxOps<C>::make(ta.x, real_bin ? 0 : ta.y);
        const C hb = CplxOps<C>::make(tb.x, real_bin ? 0 : tb.y);
        if (in && r == 0) lds[lds_slot(kk)] = CplxOps<C>::make(ha.x - hb.y, ha.y + hb.x);
        if (in && r == 1 && kk > 0 && kk < L / 2)
            lds[lds_slot(L - kk)] = CplxOps<C>::make(ha.x + hb.y, hb.x - ha.y);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) reg[e] = lds[lds_slot(tid + e * T)];
}

// Row inverse FFT of the pairs (2p, 2p+1) with a fused epilogue.
// MODE 0 (once per step, FP64): E = V + dt(1-theta)((D - r_omega) V + B V) into R
//         (theta < 1), and B V into BV (mixed form);
// MODE 1 (FP64 iteration):  R = W + dt theta((D - r_omega) Y + B Y) - Y;
// MODE 2 (mixed iteration): B Y = (k == 1 in an anchor step ? BV : B Y) + B32(increment)
//         into BY, then R as in MODE 1 with that B Y (k == 1 elsewhere: BY still holds
//         the previous step's last B Y, the carried B V^{n-1}).
// Adjoint march (B^T from a CONJ column pass, D^T the transposed stencil):
// MODE 3 (iteration): R = Ybar + dt theta ((D^T - r_omega) lam + B^T lam) - lam,
//         with Ybar in W and lam the iterate;
// MODE 4 (once per step, theta < 1): W = mu + dt (1 - theta)((D^T - r_omega) mu + B^T mu),
//         mu in pool[cur]: the cotangent of V^{n-1}.
template <int L, int E, int MODE>
__global__ __launch_bounds__(L / E) void ks_rows_inv(const MarchArgs* __restrict__ A, int k) {
    const MarchArgs& a = plan_args(A);
    if (halted(a, k) || ((MODE == 0 || MODE == 4) && !needs_explicit_fft(a)) ||
        (MODE == 1 && k == 1 && start_by_linearity(a)))   // ks_rows_lin runs instead
        return;
    using C = typename std::conditional<MODE == 2, float2, double2>::type;
    constexpr int T = L / E;
    const int n = a.n, np = (n + 1) >> 1;
    const int p = xcd_remap(blockIdx.x, gridDim.x);
    if (p >= np) return;
    __shared__ C lds[lds_slots(L)];
    __shared__ double2 tw4[tw_slots<L, E>()];
    load_twiddles<L, E>(a.tw, tw4);
    const int ra = 2 * p, rb = 2 * p + 1;
    const bool hasb = rb < n;
    const int tid = threadIdx.x;
    const C* X = xbuf<C>(a);
    C reg[E];
    rows_inv_gather<L, E>(reg, lds, X, n, ra, hasb);
    fft_block<L, E, true>(reg, lds, tw4);
    // FP64 iterations store B Y of the iterate for the start of later steps
    double* Bout = nullptr;
    if constexpr (MODE == 1) {
        if (a.bpool[0]) Bout = a.bpool[a.ctl->y];
    }
    const StepDesc& sd = cur_set(a);
    constexpr bool EXPL = MODE == 0 || MODE == 4;
    const double* U = EXPL ? a.pool[a.ctl->cur] : a.pool[a.ctl->y];
    const double* P0 = EXPL ? U : a.W;
    double* out = MODE == 4 ? a.W : a.R;
    const double c = EXPL ? sd.dt * (1.0 - sd.theta) : sd.dt * sd.theta;
    const double c0 = EXPL ? 0.0 : -1.0;
    const bool want_r = MODE != 0 || sd.theta < 1.0;
    const double* base = (MODE == 2 && k == 1 && is_anchor(a)) ? a.BV : a.BY;
    // the arguments the loop needs, read once: the stores below go through
    // plain pointers, after which every field of a would be read again
    const StencilArgs st = a.st;
    const double r_omega = a.r_omega;
    double* const BY = a.BY;
    double* const BV = a.mixed ? a.BV : nullptr;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = tid + e * T;
        if (j >= n) continue;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            if (r == 1 && !hasb) break;
            const int i = ra + r;
            const size_t o = (size_t)i * n + j;
            double bu = r == 0 ? (double)reg[e].x : (double)reg[e].y;
            if constexpr (MODE == 1) {
                if (Bout) Bout[o] = bu;
            }
            if constexpr (MODE == 2) {
                bu += base[o];
                BY[o] = bu;
            }
            if constexpr (MODE == 0) {
                if (BV) BV[o] = bu;
            }
            if (want_r) {
                const double u = U[o];
                const double d = MODE >= 3 ? apply_DT(U, st, i, j, u) : apply_D(U, st, i, j, u);
                out[o] = P0[o] + c * (d + bu - r_omega * u) + c0 * u;
            }
        }
    }
}

// The same affine forms without the correlation (zero Levy measure); one
// block per grid row.
template <bool EXPLICIT>
__global__ __launch_bounds__(256) void ks_affine_noB(const MarchArgs* __restrict__ A, int k) {
    const MarchArgs& a = plan_args(A);
    if (halted(a, k) || (EXPLICIT && !needs_explicit(a))) return;
    const int n = a.n;
    const int i = xcd_remap(blockIdx.x, gridDim.x);   // neighbouring rows on one XCD (stencil reads share L2)
    if (i >= n) return;
    const StepDesc& sd = cur_set(a);
    const double* U = EXPLICIT ? a.pool[a.ctl->cur] : a.pool[a.ctl->y];
    const double* P0 = EXPLICIT ? U : a.W;
    const double c = EXPLICIT ? sd.dt * (1.0 - sd.theta) : sd.dt * sd.theta;
    const double c0 = EXPLICIT ? 0.0 : -1.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const size_t o = (size_t)i * n + j;
        const double u = U[o];
        const double d = apply_D(U, a.st, i, j, u);
        a.R[o] = P0[o] + c * (d - a.r_omega * u) + c0 * u;
    }
}

// Mixed form, steps between anchors whose explicit part does not come from the
// previous step's equation (explicit_by_identity): B V^{n-1} is carried from
// the previous step, whose last iteration left B Y in BY (FP64 sums of FP32
// correlations of the increments; it misses B applied to the final increment,
// which is below the stopping tolerance), and the explicit part
// E = V + dt (1 - theta)((D - r_omega) V + B V) (theta < 1) is formed without
// a correlation.  One block per grid row.
static __global__ __launch_bounds__(256) void ks_carry(const MarchArgs* __restrict__ A) {
    const MarchArgs& a = plan_args(A);
    if (halted(a, 0) || !a.mixed || is_anchor(a) || explicit_by_identity(a) || cur_set(a).theta >= 1.0) return;
    const int n = a.n;
    const int i = xcd_remap(blockIdx.x, gridDim.x);   // neighbouring rows on one XCD (stencil reads share L2)
    if (i >= n) return;
    const StepDesc& sd = cur_set(a);
    const double* U = a.pool[a.ctl->cur];
    const double c = sd.dt * (1.0 - sd.theta);
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const size_t o = (size_t)i * n + j;
        const double u = U[o];
        a.R[o] = u + c * (apply_D(U, a.st, i, j, u) + a.BY[o] - a.r_omega * u);
    }
}

// Explicit part from the previous step's implicit equation (explicit_by_identity):
// R = V + rho (V - W); one block per grid row.  Mixed form: not in anchor steps.
static __global__ __launch_bounds__(256) void ks_expl_identity(const MarchArgs* __restrict__ A) {
    const MarchArgs& a = plan_args(A);
    if (halted(a, 0) || !explicit_by_identity(a) || (a.mixed && is_anchor(a))) return;
    const int n = a.n;
    const int i = blockIdx.x;
    if (i >= n) return;
    const double rho = a.cn_rho[a.ctl->step];
    const double* V = a.pool[a.ctl->cur] + (size_t)i * n;
    const double* W = a.W + (size_t)i * n;
    double* R = a.R + (size_t)i * n;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double v = V[j];
        R[j] = v + rho * (v - W[j]);
    }
}

// FP64 iteration 1 when B Y^0 comes by linearity (start_by_linearity):
// B Y^0 = sum_q coef_q B V^{src_q} from the stored products, the residual
// R = W + dt theta((D - r_omega) Y^0 + B Y^0) - Y^0, and B Y^0 stored for the
// iterate; one block per grid row (the row c2r kernel exits in these steps).
// The element loop has no branch and the arguments are read once before it (the
// stores go through plain pointers, after which they would be read again), so
// that an element's reads are in flight together.  One loop serves every count
// of stored products: the terms past the count repeat the first product at
// weight zero (Ctl: reads of lines the thread has just fetched, and the same
// sums, since adding a signed zero changes no value).  A dispatch to one loop
// per count cost 10 us per launch at 2048^2 (90 against 80).
template <int UN = 4>
__device__ __forceinline__ void rows_lin_row(const MarchArgs& a, int i, double cth) {
    constexpr int NS = 4;
    const Ctl* c = a.ctl;
    const int n = a.n;
    const double* __restrict__ Hb[NS];
    double cf[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        Hb[q] = a.bpool[c->src[q]];
        cf[q] = c->coef[q];
    }
    const double* __restrict__ U = a.pool[c->y];
    const double* __restrict__ W = a.W;
    double* __restrict__ R = a.R;
    double* __restrict__ Bout = a.bpool[c->y];
    const double r_omega = a.r_omega;
    const StencilArgs st = a.st;
    // UN elements per thread and pass, the products and W of all of them read
    // first (their reads in flight together: 90 -> 80 -> 71 us per launch at
    // 2048^2 with one loop per count, one loop, one loop of UN = 4)
    for (int j0 = threadIdx.x; j0 < n; j0 += UN * blockDim.x) {
        double bu[UN], w[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const int j = j0 + u * blockDim.x;
            const size_t o = (size_t)i * n + (j < n ? j : j0);   // past the row end: a repeated read, not used
            bu[u] = 0.0;
#pragma unroll
            for (int q = 0; q < NS; ++q) bu[u] += cf[q] * Hb[q][o];
            w[u] = W[o];
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const int j = j0 + u * blockDim.x;
            if (j >= n) break;
            const size_t o = (size_t)i * n + j;
            const double y = U[o];
            const double d = apply_D_ahead(U, st, i, j, y);
            R[o] = w[u] + cth * (d + bu[u] - r_omega * y) - y;
            Bout[o] = bu[u];
        }
    }
}

static __global__ __launch_bounds__(256) void ks_rows_lin(const MarchArgs* __restrict__ A) {
    const MarchArgs& a = plan_args(A);
    if (halted(a, 1) || !start_by_linearity(a)) return;
    const int n = a.n;
    const int i = xcd_remap(blockIdx.x, gridDim.x);   // neighbouring rows on one XCD (stencil reads share L2)
    if (i >= n) return;
    const StepDesc& sd = cur_set(a);
    rows_lin_row(a, i, sd.dt * sd.theta);
}

// The row of ks_sl_lin with NS history grids in the start value.  The gather
// is taken in its separable order: the row weights combine the P + 1 source
// rows into ec (LDS, n values: four coalesced reads per element instead of
// (P + 1)^2 stencil reads), then each node takes its P + 1 column taps from ec.
// Two elements per thread and pass, their history reads issued together; no
// branch in the element loop and the step's tables read once before it.
template <int P, int NS>
__device__ __forceinline__ void sl_lin_row(const MarchArgs& a, int i, double* __restrict__ ec) {
    const Ctl* c = a.ctl;
    const int n = a.n;
    const StepDesc& sd = cur_set(a);
    // the grids read (E, history) and written (W, Y) are distinct pool, R and W buffers
    const double* __restrict__ Ex = sd.theta < 1.0 ? a.R : a.pool[c->cur];
    double* __restrict__ Y = a.pool[c->y];
    double* __restrict__ Wo = a.W;
    const double* __restrict__ H[NS];
    double cf[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        H[q] = a.pool[c->src[q]];
        cf[q] = c->coef[q];
    }
    const int a0 = sd.s1[i];
    double w1[P + 1];
#pragma unroll
    for (int q = 0; q <= P; ++q) w1[q] = sd.w1[i * (P + 1) + q];
    const double* __restrict__ er0 = Ex + (size_t)a0 * n;
    const int T = blockDim.x;
    for (int k = threadIdx.x; k < n; k += T) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q <= P; ++q) v += w1[q] * er0[(size_t)q * n + k];
        ec[k] = v;
    }
    __syncthreads();
    const int* __restrict__ s2 = sd.s2;
    const double* __restrict__ wt2 = sd.w2;
    constexpr int UN = 2;
    for (int j0 = threadIdx.x; j0 < n; j0 += UN * T) {
        double hv[UN][NS];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const int j = j0 + u * T;
            const size_t o = (size_t)i * n + (j < n ? j : j0);   // past the row end: a repeated read, not used
#pragma unroll
            for (int q = 0; q < NS; ++q) hv[u][q] = H[q][o];
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const int j = j0 + u * T;
            if (j >= n) break;
            const int b0 = s2[j];
            double acc = 0.0;
#pragma unroll
            for (int b = 0; b <= P; ++b) acc += wt2[j * (P + 1) + b] * ec[b0 + b];
            const size_t o = (size_t)i * n + j;
            double y = cf[0] * hv[u][0];
#pragma unroll
            for (int q = 1; q < NS; ++q) y += cf[q] * hv[u][q];
            Wo[o] = acc;
            Y[o] = y;
        }
    }
}

// SL gather W = T^SL E and start value Y^0 of an FP64 step whose B Y^0 comes by
// linearity (no row transform of Y^0): one block per grid row, streaming; at
// least 8 waves per SIMD (64 registers), so that the reads hoisted out of the
// branch-free loop do not cost occupancy.  Dynamic LDS: n doubles (the largest
// n of the launch's plans).
template <int P>
__global__ __launch_bounds__(256, 8) void ks_sl_lin(const MarchArgs* __restrict__ A) {
    extern __shared__ double sl_ec[];
    const MarchArgs& a = plan_args(A);
    if (halted(a, 0) || a.mixed || !start_by_linearity(a)) return;
    const int n = a.n;
    const int i = xcd_remap(blockIdx.x, gridDim.x);   // neighbouring rows share E rows in L2
    if (i >= n) return;
    switch (a.ctl->nsrc) {                           // uniform: one loop per count of history grids (1..4)
        case 1: sl_lin_row<P, 1>(a, i, sl_ec); break;
        case 2: sl_lin_row<P, 2>(a, i, sl_ec); break;
        case 3: sl_lin_row<P, 3>(a, i, sl_ec); break;
        default: sl_lin_row<P, 4>(a, i, sl_ec); break;
    }
}

// Forward FFT of the row pair held in reg (canonical layout) into the
// transposed half spectra X[k2 * n + row].
// X2, if not null, receives a second copy.
template <int L, int E, typename C>
__device__ __forceinline__ void rows_fwd_store(C (&reg)[E], C* lds, const double2* tw4, C* __restrict__ X, int n,
                                               int ra, bool hasb, C* __restrict__ X2 = nullptr) {
    constexpr int T = L / E;
    using Rl = typename CplxOps<C>::real;
    const int tid = threadIdx.x;
    __syncthreads();
    fft_block<L, E, false>(reg, lds, tw4);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) lds[tid + e * T] = reg[e];
    __syncthreads();
    // item idx = frequency (idx >> 1) of row ra + (idx & 1): the two rows of a
    // frequency are adjacent in X, so a lane pair stores them as one 32-byte piece
    constexpr int NI = (L + 2 + T - 1) / T;
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int idx = tid + it * T;
        const int kk = idx >> 1, r = idx & 1;
        if (kk > L / 2 || (r == 1 && !hasb)) continue;
        const C z = lds[kk], w = lds[kk == 0 ? 0 : L - kk];
        const C v = r == 0 ? CplxOps<C>::make(Rl(0.5) * (z.x + w.x), Rl(0.5) * (z.y - w.y))
                           : CplxOps<C>::make(Rl(0.5) * (z.y + w.y), Rl(-0.5) * (z.x - w.x));
        const size_t o = (size_t)kk * n + ra + r;
        X[o] = v;
        if (X2) X2[o] = v;
    }
}

template <int L, int E>
__global__ __launch_bounds__(L / E) void ks_rows_fwd(const MarchArgs* __restrict__ A) {
    const MarchArgs& a = plan_args(A);
    if (halted(a, 0) || !a.mixed || !is_anchor(a)) return;
    constexpr int T = L / E;
    const int n = a.n, np = (n + 1) >> 1;
    const int p = xcd_remap(blockIdx.x, gridDim.x);
    if (p >= np) return;
    __shared__ double2 lds[lds_slots(L)];
    __shared__ double2 tw4[tw_slots<L, E>()];
    load_twiddles<L, E>(a.tw, tw4);
    const int ra = 2 * p, rb = 2 * p + 1;
    const bool hasb = rb < n;
    const double* U = a.pool[a.ctl->cur];
    double2 reg[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = threadIdx.x + e * T;
        reg[e] = j < n ? make_double2(U[(size_t)ra * n + j], hasb ? U[(size_t)rb * n + j] : 0.0)
                       : make_double2(0.0, 0.0);
    }
    rows_fwd_store<L, E>(reg, lds, tw4, a.X, n, ra, hasb);
}

// Semi-Lagrangian gather W = (T_1 (x) T_2) E (order P), starting value Y^0 into
// the iterate buffer, and (FFT) the row transform of Y^0 (FP64) or, in the
// mixed form, of Y^0 - V^{n-1} (FP32); one row pair per block.
template <int L, int E, int P, bool FFT, bool MIXED>
__global__ __launch_bounds__(L / E) void ks_sl(const MarchArgs* __restrict__ A) {
    const MarchArgs& a = plan_args(A);
    // FP64 steps whose B Y^0 comes by linearity need no row transform of Y^0:
    // ks_sl_lin does their gather and start value
    if (halted(a, 0) || (FFT && !MIXED && start_by_linearity(a))) return;
    constexpr int T = L / E;
    using C = typename std::conditional<MIXED, float2, double2>::type;
    const int n = a.n, np = (n + 1) >> 1;
    const int p = xcd_remap(blockIdx.x, gridDim.x);
    if (p >= np) return;
    __shared__ C lds[FFT ? lds_slots(L) : 1];
    __shared__ double2 tw4[FFT ? tw_slots<L, E>() : 1];
    if constexpr (FFT) load_twiddles<L, E>(a.tw, tw4);
    const int ra = 2 * p, rb = 2 * p + 1;
    const bool hasb = rb < n;
    const int tid = threadIdx.x;
    const Ctl* c = a.ctl;
    const StepDesc& sd = cur_set(a);
    const double* Ex = sd.theta < 1.0 ? a.R : a.pool[c->cur];   // explicit part E_s
    double* Y = a.pool[c->y];
    const int nsrc = c->nsrc;
    const double* H[4];
    double cf[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        H[q] = a.pool[c->src[q]];
        cf[q] = c->coef[q];
    }
    const double* V = a.pool[c->cur];
    // Two phases: the gathers and the history reads of every element first,
    // then the writes (the compiler cannot tell that W and Y alias none of the
    // read grids, so reads after writes would wait for each element in turn).
    double wv[E][2], yv[E][2], yf[E][2];   // W, Y^0, and the row-transform input
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = tid + e * T;
        wv[e][0] = wv[e][1] = yv[e][0] = yv[e][1] = yf[e][0] = yf[e][1] = 0.0;
        if (j < n) {
            const int b0 = sd.s2[j];
            double w2[P + 1];
#pragma unroll
            for (int b = 0; b <= P; ++b) w2[b] = sd.w2[j * (P + 1) + b];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int i = ra + r;
                if (r == 1 && !hasb) break;
                const int a0 = sd.s1[i];
                double acc = 0.0;
#pragma unroll
                for (int aa = 0; aa <= P; ++aa) {
                    const double* er = Ex + (size_t)(a0 + aa) * n + b0;
                    double s = 0.0;
#pragma unroll
                    for (int b = 0; b <= P; ++b) s += w2[b] * er[b];
                    acc += sd.w1[i * (P + 1) + aa] * s;
                }
                const size_t o = (size_t)i * n + j;
                wv[e][r] = acc;
                // unrolled with a predicate, so the history reads are all in flight together
                double y = 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (q < nsrc) y += cf[q] * H[q][o];
                yv[e][r] = y;
                yf[e][r] = MIXED ? y - V[o] : y;      // the mixed form transforms Y^0 - V^{n-1}
            }
        }
    }
    C reg[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = tid + e * T;
        double y0[2] = {0.0, 0.0};
        if (j < n) {
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                if (r == 1 && !hasb) break;
                const size_t o = (size_t)(ra + r) * n + j;
                a.W[o] = wv[e][r];
                Y[o] = yv[e][r];
                y0[r] = yf[e][r];
            }
        }
        reg[e] = CplxOps<C>::make(y0[0], y0[1]);
    }
    if constexpr (FFT) rows_fwd_store<L, E>(reg, lds, tw4, xbuf<C>(a), n, ra, hasb);
}

// Axis-1 line solves R <- T_1^{-1} R: CPB adjacent columns x P chunks per block
// (thread = column + CPB * chunk); launched with CPB * P <= MAXT threads.
// MM: chunk capacity (at least ceil(n / P_cols)).
template <int CPB, int MAXT, int MM>
__global__ __launch_bounds__(MAXT) void ks_line_cols(const MarchArgs* __restrict__ A, int k) {
    const MarchArgs& a = plan_args(A);
    if (halted(a, k)) return;
    extern __shared__ double2 sbuf[];
    const int n = a.n, P = a.P_cols;
    const int c = threadIdx.x % CPB, t = threadIdx.x / CPB;
    const int g = xcd_remap(blockIdx.x, gridDim.x);
    if (CPB * g >= n) return;
    const int col = g * CPB + c;
    const int m = (n + P - 1) / P;
    const int s = t * m;
    const int cnt = col < n ? max(0, min(m, n - s)) : 0;
    const StepDesc& sd = cur_set(a);
    double x[MM];
#pragma unroll
    for (int q = 0; q < MM; ++q) x[q] = q < cnt ? a.R[(size_t)(s + q) * n + col] : 0.0;
    chunk_solve<MM>(x, s, cnt, c, t, P, CPB, sd.fl1, sd.bu1, sd.bc1, sbuf);
#pragma unroll
    for (int q = 0; q < MM; ++q)
        if (q < cnt) a.R[(size_t)(s + q) * n + col] = x[q];
}

// Axis-2 line solves of a row pair, the update Y += delta, the stopping-rule
// maximum err_k = max |delta| / max(1, |Y|), and (FFT) the row transform of the
// updated Y (FP64) or, in the mixed form, of delta (FP32) for the next iteration.
// MM: the chunk capacity, at least the longest chunk ceil(n / PR) of the
// launch's plans (at most 2E, since n <= L = 2 E PR); the line-solve sweeps run
// over all MM slots, so the host takes the smallest of E, 3E/2 and 2E that
// holds the chunks (24 instead of 32 at n = 2048, L = 3072: 65 -> 55 us alone).
template <int L, int E, bool FFT, bool MIXED, int MM = 2 * E>
__global__ __launch_bounds__(L / E) void ks_line_rows(const MarchArgs* __restrict__ A, int k) {
    static_assert(MM <= 2 * E && MM % 2 == 0, "chunk capacity: even, at most 2E");
    const MarchArgs& a = plan_args(A);
    if (halted(a, k)) return;
    constexpr int T = L / E, PR = T / 2;
    using C = typename std::conditional<MIXED, float2, double2>::type;
    const int n = a.n, np = (n + 1) >> 1;
    const int p = xcd_remap(blockIdx.x, gridDim.x);
    if (p >= np) return;
    // union: row buffer 2 (n + PR + 1) doubles (n <= L) | scan totals | FFT exchange buffer
    __shared__ double2 lds[L + (PR > L / 16 ? PR : L / 16) + 2];
    __shared__ double2 tw4[FFT ? tw_slots<L, E>() : 1];
    if constexpr (FFT) load_twiddles<L, E>(a.tw, tw4);
    double* rows = reinterpret_cast<double*>(lds);
    const int ra = 2 * p, rb = 2 * p + 1;
    const bool hasb = rb < n;
    const int tid = threadIdx.x;
    const int m = (n + PR - 1) / PR;
    const int stride = n + PR + 1;
    const StepDesc& sd = cur_set(a);
    double* Y = a.pool[a.ctl->y];
    // each thread reads its chunk of the residual row straight from memory: the
    // chunks of consecutive lanes are adjacent, so the reads stay coalesced
    const int r = tid / PR, ch = tid % PR;
    const int s = ch * m;
    const int cnt = (r == 1 && !hasb) ? 0 : max(0, min(m, n - s));
    double x[MM];
    {
        const double* Rr = a.R + (size_t)(r == 0 ? ra : rb) * n + s;
        if (((n | m) & 1) == 0) {
            // 16-byte loads: the chunk starts at an even element of a row of
            // even length, so every pair is aligned (half the load
            // instructions and addresses of element-wise reads)
            const double2* R2 = reinterpret_cast<const double2*>(Rr);
#pragma unroll
            for (int q = 0; q < MM / 2; ++q) {
                const double2 v = 2 * q < cnt ? R2[q] : make_double2(0.0, 0.0);
                x[2 * q] = v.x;
                x[2 * q + 1] = v.y;
            }
        } else {
#pragma unroll
            for (int q = 0; q < MM; ++q) x[q] = q < cnt ? Rr[q] : 0.0;
        }
    }
    chunk_solve<MM>(x, s, cnt, r, ch, PR, 1, sd.fl2, sd.bu2, sd.bc2, lds);
#pragma unroll
    for (int q = 0; q < MM; ++q)
        if (q < cnt) rows[r * stride + s + q + ch] = x[q];
    __syncthreads();
    // the iterate, every element read before any write of the update (reads
    // after those writes would wait element by element: the compiler cannot
    // separate them).  Read here rather than at the start, it is not held in
    // registers across the line solve: 162 registers instead of 221 at
    // L = 3072, E = 16 (55.7 -> 53.1 us alone).
    double yoa[E], yob[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = tid + e * T;
        yoa[e] = j < n ? Y[(size_t)ra * n + j] : 0.0;
        yob[e] = (j < n && hasb) ? Y[(size_t)rb * n + j] : 0.0;
    }
    double emax = 0.0;
    C reg[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = tid + e * T;
        double ya = 0.0, yb = 0.0, da = 0.0, db = 0.0;
        if (j < n) {
            da = rows[j + j / m];
            const size_t oa = (size_t)ra * n + j;
            ya = yoa[e] + da;
            Y[oa] = ya;
            double ev = fabs(da) / fmax(1.0, fabs(ya));
            emax = (ev > emax || ev != ev) ? ev : emax;
            if (hasb) {
                db = rows[stride + j + j / m];
                const size_t ob = (size_t)rb * n + j;
                yb = yob[e] + db;
                Y[ob] = yb;
                ev = fabs(db) / fmax(1.0, fabs(yb));
                emax = (ev > emax || ev != ev) ? ev : emax;
            }
        }
        reg[e] = MIXED ? CplxOps<C>::make(da, db) : CplxOps<C>::make(ya, yb);
    }
    // block maximum: a wave reduction over the active lanes (T may be below
    // 64), the wave maxima through LDS, then one atomic per block
    // (non-negative doubles order like their bit patterns; NaN sorts above
    // +inf).  Same-address atomics serialise in the L2, so one per block
    // instead of one per wave shortens the tail of the kernel.
    constexpr int WL = T < 64 ? T : 64, NWV = (T + 63) / 64;
#pragma unroll
    for (int off = WL / 2; off > 0; off >>= 1) {
        const double o = __shfl_xor(emax, off, WL);
        emax = (o > emax || o != o) ? o : emax;
    }
    __shared__ double wmax[NWV];
    if ((tid & 63) == 0) wmax[tid >> 6] = emax;
    __syncthreads();
    if (tid == 0) {                       // issued before the row transform, which hides its latency
        double b = wmax[0];
#pragma unroll
        for (int w = 1; w < NWV; ++w) b = (wmax[w] > b || wmax[w] != wmax[w]) ? wmax[w] : b;
        atomicMax(&a.ctl->err[(blockIdx.x + blockIdx.y * gridDim.x) & (NX - 1)][k],
                  (unsigned long long)__double_as_longlong(b));
    }
    if constexpr (FFT) rows_fwd_store<L, E>(reg, reinterpret_cast<C*>(lds), tw4, xbuf<C>(a), n, ra, hasb);
}

// End of a step: convergence verdict, history rotation, next starting value.
// One block per plan.
static __global__ void ks_step_end(const MarchArgs* __restrict__ A, int kmax) {
    const MarchArgs& a = plan_args(A);
    Ctl* c = a.ctl;
    if (c->hold || c->step >= a.nsteps) return;
    __shared__ int ok;
    __shared__ double ek[KSLOTS];
    for (int q = threadIdx.x; q <= kmax; q += blockDim.x) ek[q] = err_max(c, q);
    __syncthreads();
    if (threadIdx.x == 0) {
        ok = 0;
        if (!c->fail) {
            const int s = c->step;
            int kk = 0;
            for (int q = 1; q <= kmax; ++q)
                if (ek[q] < a.tol) { kk = q; break; }
            if (kk == 0) {
                c->fail = 1;
                c->fail_step = s;
            } else {
                ok = 1;
                a.counts[s] = kk;
                a.incs[s] = ek[kk];
                const bool inner_sub = a.damping && s < a.n_sub - 1;
                if (inner_sub) {
                    c->cur = c->y;                        // next damped sub-step starts here
                } else {
                    for (int q = 3; q > 0; --q) c->hist[q] = c->hist[q - 1];
                    c->hist[0] = c->y;
                    c->hc = c->hc < 4 ? c->hc + 1 : 4;
                    c->cur = c->y;
                }
                c->bvalid |= 1 << c->cur;                 // its B Y was stored by the row kernel
                int fr = -1;
                for (int b = 0; b < POOL && fr < 0; ++b) {
                    bool used = b == c->cur;
                    for (int q = 0; q < c->hc; ++q) used = used || b == c->hist[q];
                    if (!used) fr = b;
                }
                c->y = fr;
                c->bvalid &= ~(1 << fr);                  // the free grid takes the next iterate
                const int s2 = s + 1;
                c->step = s2;
                for (int q = 0; q < 4; ++q) { c->src[q] = c->hist[q]; c->coef[q] = 0.0; }
                if (a.damping && s2 < a.n_sub) {
                    c->nsrc = 1;
                    c->src[0] = c->cur;
                    c->coef[0] = 1.0;
                } else {
                    c->nsrc = c->hc;
                    if (c->hc == 1) { c->coef[0] = 1.0; }
                    else if (c->hc == 2) { c->coef[0] = 2.0; c->coef[1] = -1.0; }
                    else if (c->hc == 3) { c->coef[0] = 3.0; c->coef[1] = -3.0; c->coef[2] = 1.0; }
                    else { c->coef[0] = 4.0; c->coef[1] = -6.0; c->coef[2] = 4.0; c->coef[3] = -1.0; }
                }
                for (int q = c->nsrc; q < 4; ++q) c->src[q] = c->src[0];   // weight 0 (above)
            }
        }
    }
    __syncthreads();
    if (ok) err_reset_upto(c, kmax);
}

// Recording for the adjoint march.  After sl (once per step): E_s, held in R
// when theta < 1, to segE.  After step_end: the current state to seg when its
// step index is on the recording stride (idempotent: a slot whose step did not
// advance writes the same state again).
static __global__ void ks_store_E(const MarchArgs* __restrict__ A) {
    const MarchArgs& a = plan_args(A);
    if (halted(a, 0) || !a.segE || cur_set(a).theta >= 1.0) return;
    const size_t N = (size_t)a.n * a.n;
    double* dst = a.segE + (size_t)(a.ctl->step - a.seg_base) * N;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = a.R[i];
}

static __global__ void ks_store_V(const MarchArgs* __restrict__ A) {
    const MarchArgs& a = plan_args(A);
    const Ctl* c = a.ctl;
    if (!a.seg || c->hold) return;
    const int rel = c->step - a.seg_base;
    if (rel < 0 || rel % a.seg_every != 0) return;
    const size_t N = (size_t)a.n * a.n;
    const double* src = a.pool[c->cur];
    double* dst = a.seg + (size_t)(rel / a.seg_every) * N;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// ---- adjoint march (reverse time steps) ----
// Per reverse step s (forward V^s -> V^{s+1} = Y): lam solves
// (I - dt theta A)^T lam = Ybar by the transposed preconditioned iteration
// (the forward iteration kernels with B^T, D^T and the transposed line factors),
// mu = (T^SL)^T lam, and the cotangent of V^s is (I + dt (1 - theta) A)^T mu.
// Buffers of the adjoint MarchArgs: pool[1] = lam, pool[0] = mu, W = Ybar.

// Control block for reverse step s: iterate in pool[1], no failure, stopping values reset.
static __global__ void ks_adj_begin(const MarchArgs* __restrict__ A, int s) {
    Ctl* c = A[0].ctl;
    err_reset(c);
    if (threadIdx.x == 0) {
        c->step = s;
        c->fail = 0;
        c->fail_step = -1;
        c->hold = 0;
        c->cur = 0;
        c->y = 1;
    }
}

// Starting value lam^0 = Ybar + w1 c1 + w2 c2 + w3 c3 + w4 c4 and its row
// transform, where c1..c4 = lam - Ybar of the previous reverse steps, newest
// first (lam - Ybar = dt theta A^T lam), weighted by the host: the correction
// extrapolated over the previous steps of the same kind and rescaled to this
// step's dt theta; unused c are null.
template <int L, int E>
__global__ __launch_bounds__(L / E) void ks_adj_start(const MarchArgs* __restrict__ A,
                                                     const double* __restrict__ c1, double w1,
                                                     const double* __restrict__ c2, double w2,
                                                     const double* __restrict__ c3, double w3,
                                                     const double* __restrict__ c4, double w4) {
    const MarchArgs& a = plan_args(A);
    if (halted(a, 0)) return;
    constexpr int T = L / E;
    const int n = a.n, np = (n + 1) >> 1;
    const int p = xcd_remap(blockIdx.x, gridDim.x);
    if (p >= np) return;
    __shared__ double2 lds[lds_slots(L)];
    __shared__ double2 tw4[tw_slots<L, E>()];
    load_twiddles<L, E>(a.tw, tw4);
    const int ra = 2 * p, rb = 2 * p + 1;
    const bool hasb = rb < n;
    double* lam = a.pool[a.ctl->y];
    double2 reg[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = threadIdx.x + e * T;
        double va = 0.0, vb = 0.0;
        if (j < n) {
            const size_t oa = (size_t)ra * n + j, ob = (size_t)rb * n + j;
            va = a.W[oa] + (c1 ? w1 * c1[oa] : 0.0) + (c2 ? w2 * c2[oa] : 0.0) + (c3 ? w3 * c3[oa] : 0.0) +
                 (c4 ? w4 * c4[oa] : 0.0);
            lam[oa] = va;
            if (hasb) {
                vb = a.W[ob] + (c1 ? w1 * c1[ob] : 0.0) + (c2 ? w2 * c2[ob] : 0.0) + (c3 ? w3 * c3[ob] : 0.0) +
                     (c4 ? w4 * c4[ob] : 0.0);
                lam[ob] = vb;
            }
        }
        reg[e] = make_double2(va, vb);
    }
    rows_fwd_store<L, E>(reg, lds, tw4, a.X, n, ra, hasb);
}

// corr = lam - Ybar after the adjoint fixed point converged (start of the next
// reverse step).
static __global__ void ks_adj_corr(const MarchArgs* __restrict__ A, double* __restrict__ corr) {
    const MarchArgs& a = plan_args(A);
    if (halted(a, 0)) return;
    const size_t N = (size_t)a.n * a.n;
    const double* lam = a.pool[a.ctl->y];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x)
        corr[i] = lam[i] - a.W[i];
}

// Verdict of the adjoint fixed point of the current reverse step: iteration
// count (first k with err_k < tol) or the failure flag.
static __global__ void ks_adj_end(const MarchArgs* __restrict__ A, int kmax) {
    const MarchArgs& a = A[0];
    Ctl* c = a.ctl;
    if (c->fail) return;
    __shared__ double ek[KSLOTS];
    for (int q = threadIdx.x; q <= kmax; q += blockDim.x) ek[q] = err_max(c, q);
    __syncthreads();
    if (threadIdx.x != 0) return;
    int kk = 0;
    for (int q = 1; q <= kmax; ++q)
        if (ek[q] < a.tol) { kk = q; break; }
    if (kk == 0) {
        c->fail = 1;
        c->fail_step = c->step;
    } else {
        a.counts[c->step] = kk;
        a.incs[c->step] = ek[kk];
    }
}

// mu = (T_1^T (x) T_2^T) lam (the transposed semi-Lagrangian gather) into
// pool[0]; when theta < 1 also its row transform for B^T mu, into X and, if
// X2 is not null, into X2 as well (the spectral gradient term reads it).
// WM > 0: the transposed tables are at most WM wide (the host checks), so
// each thread holds its columns' sources and weights in registers and the
// loops have fixed bounds; WM = 0: any width.
template <int L, int E, int WM>
__global__ __launch_bounds__(L / E) void ks_adj_sl(const MarchArgs* __restrict__ A, double2* __restrict__ X2) {
    const MarchArgs& a = plan_args(A);
    if (halted(a, 0)) return;
    constexpr int T = L / E;
    const int n = a.n, np = (n + 1) >> 1;
    const int p = xcd_remap(blockIdx.x, gridDim.x);
    if (p >= np) return;
    __shared__ double2 lds[lds_slots(L)];
    __shared__ double2 tw4[tw_slots<L, E>()];
    const StepDesc& sd = cur_set(a);
    const bool fft = sd.theta < 1.0;
    if (fft) load_twiddles<L, E>(a.tw, tw4);
    const int ra = 2 * p, rb = 2 * p + 1;
    const bool hasb = rb < n;
    const double* __restrict__ lam = a.pool[a.ctl->y];
    double* __restrict__ mu = a.pool[a.ctl->cur];
    const int W1 = sd.wt1, W2 = sd.wt2;
    double outv[E][2];
    if constexpr (WM > 0) {
        // the sources of rows ra and rb (block-uniform)
        int ia[WM], ib[WM];
        double wa[WM], wb[WM];
#pragma unroll
        for (int q = 0; q < WM; ++q) {
            const bool in = q < W1;
            ia[q] = in ? sd.t1i[(size_t)ra * W1 + q] : ra;
            wa[q] = in ? sd.t1w[(size_t)ra * W1 + q] : 0.0;
            ib[q] = (in && hasb) ? sd.t1i[(size_t)rb * W1 + q] : ra;
            wb[q] = (in && hasb) ? sd.t1w[(size_t)rb * W1 + q] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = threadIdx.x + e * T;
            double sa = 0.0, sb = 0.0;
            if (j < n) {
                int jc[WM];
                double wc[WM];
#pragma unroll
                for (int q = 0; q < WM; ++q) {
                    const bool in = q < W2;
                    jc[q] = in ? sd.t2i[(size_t)j * W2 + q] : j;
                    wc[q] = in ? sd.t2w[(size_t)j * W2 + q] : 0.0;
                }
#pragma unroll
                for (int q1 = 0; q1 < WM; ++q1) {
                    if (q1 >= W1) break;
                    const double* la = lam + (size_t)ia[q1] * n;
                    const double* lb = lam + (size_t)ib[q1] * n;
                    double ta = 0.0, tb = 0.0;
#pragma unroll
                    for (int q2 = 0; q2 < WM; ++q2) {
                        if (q2 < W2) {
                            ta += wc[q2] * la[jc[q2]];
                            tb += wc[q2] * lb[jc[q2]];
                        }
                    }
                    sa += wa[q1] * ta;
                    sb += wb[q1] * tb;
                }
            }
            outv[e][0] = sa;
            outv[e][1] = hasb ? sb : 0.0;
        }
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = threadIdx.x + e * T;
            outv[e][0] = outv[e][1] = 0.0;
            if (j < n) {
                for (int r = 0; r < 2; ++r) {
                    const int i = ra + r;
                    if (r == 1 && !hasb) break;
                    double acc = 0.0;
                    for (int q1 = 0; q1 < W1; ++q1) {
                        const double w = sd.t1w[(size_t)i * W1 + q1];
                        const double* lr = lam + (size_t)sd.t1i[(size_t)i * W1 + q1] * n;
                        double s2 = 0.0;
                        for (int q2 = 0; q2 < W2; ++q2)
                            s2 += sd.t2w[(size_t)j * W2 + q2] * lr[sd.t2i[(size_t)j * W2 + q2]];
                        acc += w * s2;
                    }
                    outv[e][r] = acc;
                }
            }
        }
    }
    // the writes after every read (mu is not read here, but the compiler
    // cannot tell)
    double2 reg[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = threadIdx.x + e * T;
        if (j < n) {
            mu[(size_t)ra * n + j] = outv[e][0];
            if (hasb) mu[(size_t)rb * n + j] = outv[e][1];
        }
        reg[e] = make_double2(outv[e][0], outv[e][1]);
    }
    if (fft) rows_fwd_store<L, E>(reg, lds, tw4, a.X, n, ra, hasb, X2);
}

// Per-step gradient terms of the reverse step (one block per row pair,
// deterministic per-block accumulators acc[block * 8 + q]):
//   q = 0, 1, 2: dt theta lam . D_c Y + dt (1 - theta) mu . D_c V    (c = 11, 12, 22)
//   q = 3:       -(dt theta lam . Y + dt (1 - theta) mu . V)         (r_omega)
//   q = 4, 5:    lam . ((dT_1 (x) T_2) E), lam . ((T_1 (x) dT_2) E)   (kappa_omega^(1,2))
// with Y = V^{s+1}, V = V^s and E = E_s (V^s when theta = 1).
template <int P>
__global__ __launch_bounds__(256) void ks_adj_accum(const MarchArgs* __restrict__ A, const double* __restrict__ Yg,
                                                    const double* __restrict__ Vg, const double* __restrict__ Eg,
                                                    double* __restrict__ acc) {
    const MarchArgs& a = plan_args(A);
    if (halted(a, 0)) return;
    const int n = a.n;
    const int i = xcd_remap(blockIdx.x, gridDim.x);   // neighbouring rows on one XCD (stencil reads share L2)
    if (i >= n) return;
    const StepDesc& sd = cur_set(a);
    const double* lam = a.pool[a.ctl->y];
    const double* mu = a.pool[a.ctl->cur];
    const double ci = sd.dt * sd.theta, ce = sd.dt * (1.0 - sd.theta);
    double t[6] = {0, 0, 0, 0, 0, 0};
    const int a0 = sd.s1[i];
    double w1[P + 1], w1d[P + 1];
#pragma unroll
    for (int q = 0; q <= P; ++q) {
        w1[q] = sd.w1[i * (P + 1) + q];
        w1d[q] = sd.w1d[i * (P + 1) + q];
    }
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const size_t o = (size_t)i * n + j;
        const double l = lam[o], m = mu[o], y = Yg[o], v = Vg[o];
        double y11, y12, y22, v11 = 0.0, v12 = 0.0, v22 = 0.0;
        apply_D_parts(Yg, n, a.st.h, i, j, y, y11, y12, y22);
        if (ce != 0.0) apply_D_parts(Vg, n, a.st.h, i, j, v, v11, v12, v22);
        t[0] += ci * l * y11 + ce * m * v11;
        t[1] += ci * l * y12 + ce * m * v12;
        t[2] += ci * l * y22 + ce * m * v22;
        t[3] -= ci * l * y + ce * m * v;
        const int b0 = sd.s2[j];
        double w2[P + 1], w2d[P + 1];
#pragma unroll
        for (int b = 0; b <= P; ++b) {
            w2[b] = sd.w2[j * (P + 1) + b];
            w2d[b] = sd.w2d[j * (P + 1) + b];
        }
        double g1 = 0.0, g2 = 0.0;
#pragma unroll
        for (int aa = 0; aa <= P; ++aa) {
            const double* er = Eg + (size_t)(a0 + aa) * n + b0;
            double s0 = 0.0, sdd = 0.0;
#pragma unroll
            for (int b = 0; b <= P; ++b) {
                s0 += w2[b] * er[b];
                sdd += w2d[b] * er[b];
            }
            g1 += w1d[aa] * s0;
            g2 += w1[aa] * sdd;
        }
        t[4] += l * g1;
        t[5] += l * g2;
    }
    __shared__ double red[6][256];
    for (int q = 0; q < 6; ++q) red[q][threadIdx.x] = t[q];
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 6; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 6; ++q) acc[(size_t)i * 8 + q] += red[q][0];
}

// Spectral accumulation of the kernel gradient: per column k2 of the row
// transforms (transposed half spectra, n rows each), the column FFTs and
// S[k2][k1] += c1 conj(FFT XA) FFT XB (+ c2 conj(FFT XC) FFT XD when c2 != 0).
// After the march, the inverse 2D transform of S / L^2 is sum_m lam_m Y_{m+d}
// summed over the steps with their weights: the gradient of the loss with
// respect to the folded kernel K_d.
template <int L, int E = conv_e(L)>
__global__ __launch_bounds__(L / E) void ks_adj_spec(const double2* __restrict__ XA, const double2* __restrict__ XB,
                                                     const double2* __restrict__ XC, const double2* __restrict__ XD,
                                                     int n, double c1, double c2, double2* __restrict__ S,
                                                     const double2* __restrict__ tw) {
    constexpr int T = L / E;
    __shared__ double2 lds[lds_slots(L)];
    __shared__ double2 tw4[tw_slots<L, E>()];
    load_twiddles<L, E>(tw, tw4);
    const int col = blockIdx.x, tid = threadIdx.x;
    double2 acc[E];
    double2* sc = S + (size_t)col * L;
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = sc[tid + e * T];
    for (int pass = 0; pass < 2; ++pass) {
        const double cf = pass == 0 ? c1 : c2;
        if (cf == 0.0) continue;
        const double2* xa = (pass == 0 ? XA : XC) + (size_t)col * n;
        const double2* xb = (pass == 0 ? XB : XD) + (size_t)col * n;
        double2 ra[E], rb[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = tid + e * T;
            ra[e] = idx < n ? xa[idx] : make_double2(0.0, 0.0);
            rb[e] = idx < n ? xb[idx] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        fft_block<L, E, false>(ra, lds, tw4);
        __syncthreads();
        fft_block<L, E, false>(rb, lds, tw4);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const double2 pr = cmulc(rb[e], ra[e]);    // conj(A) B
            acc[e] = make_double2(acc[e].x + cf * pr.x, acc[e].y + cf * pr.y);
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) sc[tid + e * T] = acc[e];
}

// Control block at the start of a march: the state of step-list entry step0
// in pool[0], the iterate in pool[1], no history before it.  One block per plan.
static __global__ void ks_init(const MarchArgs* __restrict__ A) {
    const MarchArgs& a = plan_args(A);
    Ctl* c = a.ctl;
    err_reset(c);
    if (threadIdx.x == 0) {
        c->step = a.step0;
        c->fail = 0;
        c->fail_step = -1;
        c->hold = 0;
        c->cur = 0;
        c->y = 1;
        c->hc = 1;
        c->nsrc = 1;
        c->bvalid = 0;
        for (int q = 0; q < 4; ++q) { c->hist[q] = 0; c->src[q] = 0; c->coef[q] = 0.0; }
        c->coef[0] = 1.0;
    }
}

static __global__ void ks_clear_fail(const MarchArgs* __restrict__ A, int plan) {
    if (threadIdx.x == 0) A[plan].ctl->fail = 0;
}

// hold = 1 on every plan of the group except `keep` (keep < 0: release all).
static __global__ void ks_hold(const MarchArgs* __restrict__ A, int np, int keep) {
    for (int q = threadIdx.x; q < np; q += blockDim.x) A[q].ctl->hold = (keep >= 0 && q != keep) ? 1 : 0;
}

}  // namespace lpide
