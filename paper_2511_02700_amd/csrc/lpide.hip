// MI355X (gfx950) time march of the two-asset exponential-Levy PIDE scheme
// (arXiv 2511.02700, Sec. 3, Algorithm 1) behind the C ABI of include/lpide.h.
//
// Per time step (theta, dt) of the step list (Sec. 3.3, four damped quarter
// steps first):
//   E = V + dt (1 - theta)((D - r_omega) V + B V)       rows_fwd/cols/rows_inv, affine epilogue
//   W = T^SL E,  Y^0 = extrapolation of V^{n-1..n-4}   sl_extrap
//   repeat: R = W + dt theta ((D - r_omega) Y + B Y) - Y  (FFT passes + affine epilogue)
//           delta = T_2^{-1} T_1^{-1} R                  line_rows, line_cols (+ update)
//           Y += delta, err = max|delta| / max(1, |Y|)   (fused into line_cols)
//   until err < tol (Sec. 3.3 stopping rule).
// The preconditioned iteration has the same fixed point as the paper's
// iteration (I - dt theta (D - r_omega)) Y^k = dt theta B Y^{k-1} + W, namely the
// solution of the theta-scheme equation, with T_i = I - dt theta A_i the
// one-dimensional factors of D - r_omega without its mixed term.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "conv_kernels.hpp"
#include "plan.hpp"

namespace lpide {
namespace detail {

static thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

double bits_d(unsigned long long b) {
    double d;
    std::memcpy(&d, &b, sizeof d);
    return d;
}

// Stopping-rule value after iteration k from a host copy of a control block.
double err_of(const Ctl& c, int k) {
    unsigned long long m = c.err[0][k];
    for (int x = 1; x < NX; ++x) m = std::max(m, c.err[x][k]);
    return bits_d(m);
}

// Device address of `scratch` per HIP device (null until set up on it).
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double2* g_scratch[kMaxDevices] = {};

// Take the address of this device's copy of `scratch` (the device must be
// current); once per device.
int scratch_setup(int dev);

// The address taken for device dev, or null.
double2* scratch_ptr(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch[dev];
}

hipEvent_t next_event(Plan* p) {
    if (p->ev_used == p->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        p->ev_pool.push_back(e);
    }
    return p->ev_pool[p->ev_used++];
}

KTime::KTime(Plan* pl, int c) : p(pl), cls(c), on(pl && ((pl->time_mask >> c) & 1u)) {}

bool KTime::events(hipEvent_t* a, hipEvent_t* b) {
    const size_t idx = p->ev_used;
    *a = next_event(p);
    *b = next_event(p);
    if (!*a || !*b) return false;
    p->ev_recs.push_back({cls, idx, p->tag_step, p->tag_k});
    return true;
}

}  // namespace detail
}  // namespace lpide

using namespace lpide;
using namespace lpide::detail;

// the chunked line solves read up to LINE_MM - 1 factors past a line (its zero tail)
static_assert(LINE_MM <= kLinePad, "factor arrays need a tail of at least the chunk capacity");

// First-difference weights at index i of a line of n >= 3 nodes (spacing h):
// central inside, second-order one-sided on the two ends; nodes p[0..2].
__device__ __forceinline__ void d1_weights(int i, int n, double h, int* p, double* w) {
    const double c = 0.5 / h;
    if (i == 0) { p[0] = 0; p[1] = 1; p[2] = 2; w[0] = -3.0 * c; w[1] = 4.0 * c; w[2] = -c; }
    else if (i == n - 1) { p[0] = n - 1; p[1] = n - 2; p[2] = n - 3; w[0] = 3.0 * c; w[1] = -4.0 * c; w[2] = c; }
    else { p[0] = i - 1; p[1] = i; p[2] = i + 1; w[0] = -c; w[1] = 0.0; w[2] = c; }
}

// Second-difference weights at index i of a line of n >= 4 nodes: (1, -2, 1)/h^2
// inside, (2, -5, 4, -1)/h^2 on the two ends; nodes p[0..3] (w[3] = 0 inside).
__device__ __forceinline__ void d2_weights(int i, int n, double h, int* p, double* w) {
    const double c = 1.0 / (h * h);
    if (i == 0) { p[0] = 0; p[1] = 1; p[2] = 2; p[3] = 3; w[0] = 2.0 * c; w[1] = -5.0 * c; w[2] = 4.0 * c; w[3] = -c; }
    else if (i == n - 1) {
        p[0] = n - 1; p[1] = n - 2; p[2] = n - 3; p[3] = n - 4;
        w[0] = 2.0 * c; w[1] = -5.0 * c; w[2] = 4.0 * c; w[3] = -c;
    } else { p[0] = i - 1; p[1] = i; p[2] = i + 1; p[3] = i; w[0] = c; w[1] = -2.0 * c; w[2] = c; w[3] = 0.0; }
}

// Delta and Gamma surfaces at the nodes: one thread per node (i, j), j fast.
// out[q * n^2 + i * n + j], q = delta1, delta2, gamma11, gamma12, gamma22.
__global__ void k_greeks(const double* __restrict__ V, int n, double y0, double y1, double h, double K,
                         double* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= n) return;
    int pi[4], pj[4];
    double wi[4], wj[4];
    auto at = [&](int a, int b) { return V[(size_t)a * n + b]; };
    d1_weights(i, n, h, pi, wi);
    d1_weights(j, n, h, pj, wj);
    double v1 = 0.0, v2 = 0.0, v12 = 0.0;
    for (int q = 0; q < 3; ++q) {
        v1 += wi[q] * at(pi[q], j);
        v2 += wj[q] * at(i, pj[q]);
        double t = 0.0;
        for (int r = 0; r < 3; ++r) t += wj[r] * at(pi[q], pj[r]);
        v12 += wi[q] * t;
    }
    d2_weights(i, n, h, pi, wi);
    d2_weights(j, n, h, pj, wj);
    double v11 = 0.0, v22 = 0.0;
    for (int q = 0; q < 4; ++q) {
        v11 += wi[q] * at(pi[q], j);
        v22 += wj[q] * at(i, pj[q]);
    }
    const double S1 = K * exp(y0 + h * i), S2 = K * exp(y1 + h * j);
    const size_t o = (size_t)i * n + j, N = (size_t)n * n;
    out[o] = v1 / S1;
    out[N + o] = v2 / S2;
    out[2 * N + o] = (v11 - v1) / (S1 * S1);
    out[3 * N + o] = v12 / (S1 * S2);
    out[4 * N + o] = (v22 - v2) / (S2 * S2);
}

// Prices and deltas at spot pairs: tensor cubic Lagrange in y with the clamped
// stencil start clamp(floor(xi) - 1, 0, n - 4).
__global__ void k_price(const double* __restrict__ V, int n, double y0, double y1, double h, double K,
                        int npts, const double* __restrict__ spots, double* __restrict__ price,
                        double* __restrict__ delta) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= npts) return;
    const double S1 = spots[2 * k], S2 = spots[2 * k + 1];
    const double x1 = (log(S1 / K) - y0) / h, x2 = (log(S2 / K) - y1) / h;
    const int a = min(max((int)floor(x1) - 1, 0), n - 4);
    const int b = min(max((int)floor(x2) - 1, 0), n - 4);
    double w1[4], w2[4], d1[4], d2[4];
    for (int q = 0; q < 2; ++q) {
        const double x = q == 0 ? x1 : x2;
        const int s = q == 0 ? a : b;
        double* w = q == 0 ? w1 : w2;
        double* d = q == 0 ? d1 : d2;
        for (int i = 0; i < 4; ++i) {
            double v = 1.0, dv = 0.0;
            for (int j2 = 0; j2 < 4; ++j2) {
                if (j2 == i) continue;
                const double f = 1.0 / double(i - j2);
                dv = dv * (x - (s + j2)) * f + v * f;
                v *= (x - (s + j2)) * f;
            }
            w[i] = v;
            d[i] = dv / h;
        }
    }
    double p = 0.0, p1 = 0.0, p2 = 0.0;
    for (int i = 0; i < 4; ++i)
        for (int j2 = 0; j2 < 4; ++j2) {
            const double v = V[(size_t)(a + i) * n + b + j2];
            p += w1[i] * w2[j2] * v;
            p1 += d1[i] * w2[j2] * v;
            p2 += w1[i] * d2[j2] * v;
        }
    price[k] = p;
    if (delta) {
        delta[2 * k] = p1 / S1;
        delta[2 * k + 1] = p2 / S2;
    }
}

// Transpose of the price interpolation: vbar[node] = sum over spot pairs whose
// 4 x 4 stencil holds the node of price_bar[k] times its weight (one thread
// per node, so the sum order is fixed).
__global__ void k_price_adjoint(int n, double y0, double y1, double h, double K, int npts,
                                const double* __restrict__ spots, const double* __restrict__ price_bar,
                                double* __restrict__ vbar) {
    const size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= (size_t)n * n) return;
    const int i = int(o / n), j = int(o % n);
    double acc = 0.0;
    for (int k = 0; k < npts; ++k) {
        const double x1 = (log(spots[2 * k] / K) - y0) / h, x2 = (log(spots[2 * k + 1] / K) - y1) / h;
        const int a = min(max((int)floor(x1) - 1, 0), n - 4);
        const int b = min(max((int)floor(x2) - 1, 0), n - 4);
        if (i < a || i > a + 3 || j < b || j > b + 3) continue;
        double wi = 1.0, wj = 1.0;
        for (int q = 0; q < 4; ++q) {
            if (q != i - a) wi *= (x1 - (a + q)) / double((i - a) - q);
            if (q != j - b) wj *= (x2 - (b + q)) / double((j - b) - q);
        }
        acc += price_bar[k] * wi * wj;
    }
    vbar[o] = acc;
}

// Round the FP64 spectrum to FP32 (mixed form).
__global__ void k_to_f32(const double2* __restrict__ a, float2* __restrict__ b, size_t cnt) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

// Zero fill of n values (a plain kernel, so that callers under graph capture
// record no memset node).
__global__ void k_zero(double* __restrict__ out, size_t cnt) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) out[i] = 0.0;
}

// Scratch of the allocation-free correlation (lpide_apply_B_noalloc): the
// transposed intermediate of the three FFT passes, LPIDE_NOALLOC_SCRATCH_BYTES
// per GPU, held by each device the library runs on until the process ends.
// In host code this name is only a handle: its device address (one per GPU)
// comes from hipGetSymbolAddress, taken once per device at plan creation with
// that device current, and only that address is passed to kernels.
static __device__ __align__(256) double2 scratch[LPIDE_NOALLOC_SCRATCH_BYTES / sizeof(double2)];



namespace lpide {
namespace detail {

int scratch_setup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return fail(LPIDE_E_PARAM, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev]) return LPIDE_OK;
    void* addr = nullptr;
    hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !addr)
        return fail(LPIDE_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = static_cast<double2*>(addr);
    return LPIDE_OK;
}

namespace {

std::vector<char> linearity_steps(const Plan* p, int step0, int nend);

// Fold recorded event pairs into the per-class totals (synchronises the stream).
// Launches of iterations after a step had converged, per-step kernels that
// had nothing to do (explicit part of a theta = 1 step, the variant of the
// explicit part a step did not use) and the slots enqueued behind a step that
// needed more iterations than predicted are left out, so the totals describe
// working launches only.
int harvest_times(Plan* p) {
    if (p->ev_recs.empty()) return LPIDE_OK;
    HIP_TRY(hipStreamSynchronize(p->stream));
    const std::vector<char> lin = linearity_steps(p, p->march_step0, p->n_steps);
    for (auto& r : p->ev_recs) {
        if (r.cls < 0) continue;            // launched in a slot behind a step that needed more iterations (no-op)
        const bool known = r.step >= 0 && r.step < (int)p->counts_h.size();
        if (r.k > 0 && known && r.k > p->counts_h[r.step]) continue;
        if ((r.cls == LPIDE_K_EXPL_COLS || r.cls == LPIDE_K_EXPL_ROWS) && known && !p->mixed &&
            p->sets[p->step_set[r.step]].theta >= 1.0)
            continue;
        if (p->mixed && known) {            // the mixed form: the anchor kernels, the identity or the carry
            const bool anchor = (r.step - p->march_step0) % p->anchor_every == 0;
            const bool ident = !p->opts.all_correlations && r.step > p->march_step0 && p->cn_rho[r.step] > 0.0;
            const bool theta1 = p->sets[p->step_set[r.step]].theta >= 1.0;
            const bool anchor_cls =
                r.cls == LPIDE_K_EXPL_COLS || r.cls == LPIDE_K_EXPL_ROWS || r.cls == LPIDE_K_ROWS_FWD;
            if ((anchor_cls && !anchor) || (r.cls == LPIDE_K_CARRY && (anchor || ident || theta1)) ||
                (r.cls == LPIDE_K_EXPL_ID && (anchor || !ident)))
                continue;
        }
        if (known && r.k == 1) {            // iteration 1: B Y^0 by linearity or by the correlation
            if (lin[r.step] && (r.cls == LPIDE_K_COLS || r.cls == LPIDE_K_ROWS_INV)) continue;
            if (!lin[r.step] && r.cls == LPIDE_K_ROWS_LIN) continue;
        }
        if (known && r.k == 0) {            // the SL kernel with the row transform, or without
            if (lin[r.step] && r.cls == LPIDE_K_SL && !p->mixed && p->jumps) continue;
            if (!lin[r.step] && r.cls == LPIDE_K_SL_LIN) continue;
        }
        if (!p->mixed && known) {           // FP64: the explicit correlation or the identity kernel
            const bool ident = !p->opts.all_correlations && r.step > p->march_step0 && p->cn_rho[r.step] > 0.0;
            if (((r.cls == LPIDE_K_EXPL_COLS || r.cls == LPIDE_K_EXPL_ROWS) && ident) ||
                (r.cls == LPIDE_K_EXPL_ID && !ident))
                continue;
        }
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p->ev_pool[r.idx], p->ev_pool[r.idx + 1]));
        p->k_launch[r.cls] += 1;
        p->k_ms[r.cls] += ms;
    }
    p->ev_recs.clear();
    p->ev_used = 0;
    return LPIDE_OK;
}

template <typename Tp>
int dalloc_into(std::vector<void*>& allocs, int64_t* bytes, Tp** out, size_t count) {
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, std::max<size_t>(1, count) * sizeof(Tp));
    if (e != hipSuccess) return fail(LPIDE_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    allocs.push_back(d);
    if (bytes) *bytes += int64_t(count * sizeof(Tp));
    *out = static_cast<Tp*>(d);
    return LPIDE_OK;
}

template <typename Tp>
int dalloc(Plan* p, Tp** out, size_t count) { return dalloc_into(p->allocs, &p->bytes, out, count); }

template <typename Tp>
int upload_into(std::vector<void*>& allocs, Tp** out, const std::vector<Tp>& v) {
    int rc = dalloc_into(allocs, nullptr, out, v.size());
    if (rc) return rc;
    HIP_TRY(hipMemcpy(*out, v.data(), v.size() * sizeof(Tp), hipMemcpyHostToDevice));
    return LPIDE_OK;
}

template <typename Tp>
int upload(Plan* p, Tp** out, const std::vector<Tp>& v) {
    int rc = dalloc(p, out, v.size());
    if (rc) return rc;
    HIP_TRY(hipMemcpy(*out, v.data(), v.size() * sizeof(Tp), hipMemcpyHostToDevice));
    return LPIDE_OK;
}

StencilArgs stencil_of(const Plan* p) {
    StencilArgs s;
    s.n = p->hp.n;
    s.h = p->hp.h;
    s.a11 = p->hp.a[0];
    s.a12 = p->hp.a[1];
    s.a22 = p->hp.a[2];
    return s;
}

// The plan's march arguments (control pointers are filled in by its group).
MarchArgs march_args(const Plan* p) {
    MarchArgs a{};
    for (int b = 0; b < POOL; ++b) a.pool[b] = p->pool[b];
    a.sets = p->sets_d;
    a.step_set = p->step_set_d;
    a.n = p->hp.n;
    a.n_sub = p->opts.damping ? 4 : 1;
    a.damping = p->opts.damping ? 1 : 0;
    a.P_cols = p->P_cols;
    a.W = p->Wb;
    a.R = p->Rb;
    a.X = p->X;
    a.spec = p->spec;
    a.tw = p->tw;
    a.tol = p->opts.tol;
    a.r_omega = p->hp.r_omega;
    a.st = stencil_of(p);
    a.mixed = p->mixed ? 1 : 0;
    a.X32 = p->X32;
    a.spec32 = p->spec32;
    a.BV = p->BV;
    a.BY = p->BY;
    a.nsteps = p->n_steps;
    a.step0 = 0;
    a.anchor_every = p->anchor_every;
    a.cn_rho = p->opts.all_correlations ? nullptr : p->cn_rho_d;
    for (int b = 0; b < POOL; ++b) a.bpool[b] = p->bpool[b];
    return a;
}

// Steps of a march over [step0, nend) whose first iteration takes B Y^0 by
// linearity: the host's replay of the pool bookkeeping of ks_init and
// ks_step_end (which grids hold a stored B, which form the start value).
std::vector<char> linearity_steps(const Plan* p, int step0, int nend) {
    std::vector<char> out(p->n_steps, 0);
    if (!p->bpool[0]) return out;
    const bool damping = p->opts.damping != 0;
    const int n_sub = damping ? 4 : 1;
    int cur = 0, y = 1, hc = 1, nsrc = 1, hist[4] = {0, 0, 0, 0}, src[4] = {0, 0, 0, 0};
    unsigned valid = 0;
    for (int s = step0; s < nend && s < p->n_steps; ++s) {
        bool ok = true;
        for (int q = 0; q < nsrc; ++q) ok = ok && ((valid >> src[q]) & 1u);
        out[s] = ok ? 1 : 0;
        if (damping && s < n_sub - 1) {
            cur = y;
        } else {
            for (int q = 3; q > 0; --q) hist[q] = hist[q - 1];
            hist[0] = y;
            hc = hc < 4 ? hc + 1 : 4;
            cur = y;
        }
        valid |= 1u << cur;
        int fr = -1;
        for (int b = 0; b < POOL && fr < 0; ++b) {
            bool used = b == cur;
            for (int q = 0; q < hc; ++q) used = used || b == hist[q];
            if (!used) fr = b;
        }
        y = fr;
        valid &= ~(1u << fr);
        for (int q = 0; q < 4; ++q) src[q] = hist[q];
        if (damping && s + 1 < n_sub) {
            nsrc = 1;
            src[0] = cur;
        } else {
            nsrc = hc;
        }
    }
    return out;
}

// Default radix schedule.  From measurements on MI355X (each kernel alone):
// the column pass gains from radix 16 at L >= 1024; the row c2r, line-row and
// SL kernels from radix 4 up to L = 1024 and radix 8 above.
// Preferred E per kernel class, from single-kernel timings at n = 512 (L = 768,
// 1024) and n = 2048 (L = 3072, 4096); lowered to the next supported value
// where the size does not allow it (L = 3 * 2^m needs whole waves: L / E a
// multiple of 64).
static int supported_e(int L, int E) {
    while (E > 4 && !e_supported(L, E)) E /= 2;
    return E;
}

Schedule default_schedule(int L) {
    Schedule s;
    if (fft_odd(L) == 3) {
        // the radix-3 stage favours many threads per transform in the row
        // passes; the column pass takes E = 8 at 1536 and 4 at 3072; the axis-2
        // line-row kernel E = 4 at 1536 (4% faster than 8 on a 1024^2 solve) and
        // E = 16 at 3072 (fewest registers per chunk of the FFT's operands)
        s.cols = L == 1536 ? 8 : 4;
        s.rinv = 4;
        s.lrows = supported_e(L, L >= 3072 ? 16 : 4);
        s.sl = 4;
        return s;
    }
    s.cols = supported_e(L, L >= 1024 ? 16 : 8);
    s.rinv = supported_e(L, L <= 1024 ? 4 : 8);
    s.lrows = supported_e(L, L <= 1024 ? 4 : 8);
    s.sl = supported_e(L, L <= 1024 ? 4 : 8);
    return s;
}

Schedule uniform_schedule(int E) { return Schedule{E, E, E, E}; }

bool schedule_ok(int L, const Schedule& s) {
    return e_supported(L, s.cols) && e_supported(L, s.rinv) && e_supported(L, s.lrows) && e_supported(L, s.sl);
}

void apply_schedule(Launch& c, const Schedule& s) {
    c.E_cols = s.cols;
    c.E_rinv = s.rinv;
    c.E_lrows = s.lrows;
    c.E_sl = s.sl;
}

#define LPIDE_SWITCH_L(Lv, CALL)                                                         \
    switch (Lv) {                                                                       \
        case 64: CALL(64); break;                                                       \
        case 128: CALL(128); break;                                                     \
        case 256: CALL(256); break;                                                     \
        case 512: CALL(512); break;                                                     \
        case 768: CALL(768); break;                                                     \
        case 1024: CALL(1024); break;                                                   \
        case 1536: CALL(1536); break;                                                   \
        case 2048: CALL(2048); break;                                                   \
        case 3072: CALL(3072); break;                                                   \
        case 4096: CALL(4096); break;                                                   \
        default: return fail(LPIDE_E_PARAM, "unsupported transform size");              \
    }

int issue_slots(const Launch& c, int first_tag, int nslots, int kmax) {
#define CALL_SLOTS(Lc) PerL<Lc>::slots(c, first_tag, nslots, kmax)
    LPIDE_SWITCH_L(c.L, CALL_SLOTS)
#undef CALL_SLOTS
    HIP_TRY(hipGetLastError());
    return LPIDE_OK;
}

int issue_iteration(const Launch& c, int k) {
#define CALL_IT(Lc) PerL<Lc>::iteration(c, k)
    LPIDE_SWITCH_L(c.L, CALL_IT)
#undef CALL_IT
    HIP_TRY(hipGetLastError());
    return LPIDE_OK;
}

int dispatch_conv(Plan* p, const double* Y, double* out, double2* X) {
#define CALL_CONV(Lc) PerL<Lc>::conv(p, Y, out, X)
    LPIDE_SWITCH_L(p->L, CALL_CONV)
#undef CALL_CONV
    HIP_TRY(hipGetLastError());
    return LPIDE_OK;
}

int dispatch_spectrum(Plan* p, const double* G, double2* Xfull) {
#define CALL_SPEC(Lc) PerL<Lc>::spectrum(p, G, Xfull)
    LPIDE_SWITCH_L(p->L, CALL_SPEC)
#undef CALL_SPEC
    HIP_TRY(hipGetLastError());
    return LPIDE_OK;
}

int dispatch_rows_fwd(Plan* p, const double* Y, hipStream_t s) {
#define CALL_RF(Lc) PerL<Lc>::rows_fwd(p, Y, s)
    LPIDE_SWITCH_L(p->L, CALL_RF)
#undef CALL_RF
    HIP_TRY(hipGetLastError());
    return LPIDE_OK;
}

// ---- groups ----
void destroy_group(Group* g) {
    if (!g) return;
    if (g->lc.stream) (void)hipStreamSynchronize(g->lc.stream);
    for (auto& x : g->graphs) (void)hipGraphExecDestroy(x.exec);
    for (void* a : g->allocs) (void)hipFree(a);
    if (g->ctl_h) (void)hipHostFree(g->ctl_h);
    delete g;
}

// Launch shape of the axis-1 line solves: 4 columns per block, chunks of about
// 8 rows (4 rows up to n = 512, where the grid gives few blocks and shorter
// chunks shorten each thread's recurrence: 2% of a 512^2 solve), P_cols a
// power of two in [16, 128] (above 128 chunks per column the scan across waves
// costs more than longer chunks; measured at n = 2048, where 64, 128 and 256
// chunks per column take 82, 72 and 110 ms per solve with the factor reads
// kept ahead).
int default_P_cols(int n) {
    const int m = n <= 512 ? 4 : 8;
    int P = 16;
    while (P < 128 && (n + P - 1) / P > m) P *= 2;
    return P;
}

bool P_cols_valid(int n, int P) { return P >= 16 && P <= 256 && (n + P - 1) / P <= LINE_MM; }

// A group over plans that share Lr, the jump switch, the precision and the SL
// order; the kernels run on `stream`.
int make_group(const std::vector<Plan*>& plans, hipStream_t stream, Group** out) {
    Group* g = new Group();
    g->plans = plans;
    const int np = int(plans.size());
    Launch& c = g->lc;
    c.stream = stream;
    c.np = np;
    c.L = plans[0]->Lr;
    c.jumps = plans[0]->jumps;
    c.mixed = plans[0]->mixed;
    c.sl_order = plans[0]->hp.sl_order;
    apply_schedule(c, plans[0]->sched);
    int nmax = 0;
    for (Plan* p : plans) {
        nmax = std::max(nmax, p->hp.n);
        g->maxsteps = std::max(g->maxsteps, p->n_steps);
    }
    c.xrows = (nmax + 1) / 2;
    c.cpb = line_cols_cpb(nmax, np);
    c.xcols = (nmax + c.cpb - 1) / c.cpb;
    c.xaff = nmax;
    c.P_cols = default_P_cols(nmax);
    int rc = LPIDE_OK;
    if ((rc = dalloc_into(g->allocs, nullptr, &g->A, np)) || (rc = dalloc_into(g->allocs, nullptr, &g->ctl, np)) ||
        (rc = dalloc_into(g->allocs, nullptr, &g->counts, (size_t)np * g->maxsteps)) ||
        (rc = dalloc_into(g->allocs, nullptr, &g->incs, (size_t)np * g->maxsteps))) {
        destroy_group(g);
        return rc;
    }
    if (hipHostMalloc((void**)&g->ctl_h, sizeof(Ctl) * np, hipHostMallocDefault) != hipSuccess) {
        destroy_group(g);
        return fail(LPIDE_E_OOM, "hipHostMalloc failed");
    }
    std::memset(g->ctl_h, 0, sizeof(Ctl) * np);
    g->counts_h.assign((size_t)np * g->maxsteps, 0);
    g->incs_h.assign((size_t)np * g->maxsteps, 0.0);
    g->args_h.resize(np);
    for (int i = 0; i < np; ++i) {
        MarchArgs a = march_args(plans[i]);
        a.ctl = g->ctl + i;
        a.counts = g->counts + (size_t)i * g->maxsteps;
        a.incs = g->incs + (size_t)i * g->maxsteps;
        a.P_cols = c.P_cols;
        g->args_h[i] = a;
    }
    *out = g;
    return LPIDE_OK;
}

void drop_graphs(Group* g) {
    for (auto& x : g->graphs) (void)hipGraphExecDestroy(x.exec);
    g->graphs.clear();
}

// Set the axis-1 line-solve chunking of every plan of the group.
int set_P_cols(Group* g, int P) {
    for (Plan* p : g->plans)
        if (!P_cols_valid(p->hp.n, P)) return fail(LPIDE_E_PARAM, "P_cols not valid for the grid size");
    g->lc.P_cols = P;
    for (auto& a : g->args_h) a.P_cols = P;
    drop_graphs(g);
    return LPIDE_OK;
}

// Set the radix schedule (elements per thread) of the group's FFT kernels.
int set_schedule(Group* g, const Schedule& s) {
    if (!schedule_ok(g->lc.L, s)) return fail(LPIDE_E_PARAM, "radix schedule not available for this size");
    apply_schedule(g->lc, s);
    drop_graphs(g);
    return LPIDE_OK;
}

// Enqueue nslots step slots with kmax iterations each: replay of a captured
// graph when the group uses graphs (and no timing is on), else direct launches.
int enqueue_slots(Group* g, int first_tag, int nslots, int kmax) {
    if (!g->use_graph || g->lc.timer) return issue_slots(g->lc, first_tag, nslots, kmax);
    hipGraphExec_t exec = nullptr;
    for (auto& x : g->graphs)
        if (x.kmax == kmax && x.nslots == nslots && x.record == g->lc.record && x.lean == g->lc.lean) exec = x.exec;
    if (!exec) {
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(g->lc.stream, hipStreamCaptureModeThreadLocal));
        int rc = issue_slots(g->lc, first_tag, nslots, kmax);
        hipError_t e = hipStreamEndCapture(g->lc.stream, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return fail(LPIDE_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(LPIDE_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        g->graphs.push_back({kmax, nslots, g->lc.record, g->lc.lean, exec});
    }
    HIP_TRY(hipGraphLaunch(exec, g->lc.stream));
    return LPIDE_OK;
}

// Read every plan's control block and per-step statistics.
int read_back(Group* g) {
    const int np = g->lc.np;
    hipStream_t s = g->lc.stream;
    HIP_TRY(hipMemcpyAsync(g->ctl_h, g->ctl, sizeof(Ctl) * np, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(g->counts_h.data(), g->counts, sizeof(int) * g->counts_h.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(g->incs_h.data(), g->incs, sizeof(double) * g->incs_h.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return LPIDE_OK;
}

// Complete the current step of plan i, whose predicted iterations did not
// reach tol: the other plans are held while iterations are added one at a
// time (each followed by the step verdict).  Returns the iterations used.
int complete_step(Group* g, int i, int kused, int* k_out) {
    const Launch& c = g->lc;
    Plan* p = g->plans[i];
    hipLaunchKernelGGL(ks_hold, dim3(1), dim3(256), 0, c.stream, c.A, c.np, i);
    int k = kused;
    const int sf = g->ctl_h[i].fail_step;
    int rc = LPIDE_OK;
    for (;;) {
        const double ek = err_of(g->ctl_h[i], k);
        if (!std::isfinite(ek)) {
            rc = fail(LPIDE_E_NAN, "non-finite fixed-point increment in step " + std::to_string(sf));
            break;
        }
        if (k >= p->opts.max_iter) {
            char buf[160];
            snprintf(buf, sizeof buf, "fixed point not converged in step %d after %d iterations (increment %.3e)", sf,
                     k, ek);
            rc = fail(LPIDE_E_NOCONV, buf);
            break;
        }
        ++k;
        hipLaunchKernelGGL(ks_clear_fail, dim3(1), dim3(64), 0, c.stream, c.A, i);
        if (c.timer) c.timer->tag_step = sf;
        if ((rc = issue_iteration(c, k))) break;
        hipLaunchKernelGGL(ks_step_end, dim3(1, c.np), dim3(64), 0, c.stream, c.A, k);
        if (c.record) hipLaunchKernelGGL(ks_store_V, dim3(c.store_blocks, c.np), dim3(256), 0, c.stream, c.A);
        if ((rc = read_back(g))) break;
        if (!g->ctl_h[i].fail) break;
    }
    hipLaunchKernelGGL(ks_hold, dim3(1), dim3(256), 0, c.stream, c.A, c.np, -1);
    if (rc == LPIDE_OK) HIP_TRY(hipGetLastError());
    *k_out = k;
    return rc;
}

// March plan i of the group over step-list entries [step0, nsteps[i]) from
// the state v_in[i] (V^0 when v_in is null), all plans together; the results
// go to v_out[i].  Steps are enqueued in slots without waiting; each slot
// launches kmax iterations (a running prediction), of which those after
// convergence exit at once.  A plan whose step needs more is completed by
// extra iterations while the others are held (the slots behind it were no-ops
// for it, and are enqueued again).  The march is split in phases so that a
// batch can interleave its groups: begin, then enqueue/check until done, end.
struct MarchState {
    std::vector<int> nsteps, at;
    int step0 = 0, kpred = 8, maxit = 1;
    bool done = false;
};

int march_begin(Group* g, MarchState& st, const int* nsteps, int step0, const double* const* v_in) {
    const int np = g->lc.np;
    hipStream_t s = g->lc.stream;
    st.nsteps.assign(nsteps, nsteps + np);
    st.at.assign(np, step0);
    st.step0 = step0;
    st.done = false;
    for (Plan* p : g->plans) {
        p->march_step0 = step0;
        // steps where both FP64 shortcuts apply (the device takes the same
        // decisions: explicit_by_identity, start_by_linearity)
        p->steady.assign(p->n_steps, 0);
        if (p->bpool[0] && p->cn_rho_d && !p->mixed && !p->opts.all_correlations) {
            const std::vector<char> lin = linearity_steps(p, step0, p->n_steps);
            for (int q = step0 + 1; q < p->n_steps; ++q) p->steady[q] = (lin[q] && p->cn_rho[q] > 0.0) ? 1 : 0;
        }
    }
    for (int i = 0; i < np; ++i) {
        Plan* p = g->plans[i];
        const int n = p->hp.n;
        const size_t N = (size_t)n * n;
        if (nsteps[i] < step0 || nsteps[i] > p->n_steps) return fail(LPIDE_E_PARAM, "steps out of range");
        g->args_h[i].nsteps = nsteps[i];
        g->args_h[i].step0 = step0;
        const double* src = v_in ? v_in[i] : p->V0;
        hipLaunchKernelGGL(k_copy, dim3((N + 255) / 256), dim3(256), 0, s, src, p->pool[0], N);
        if (p->jumps && !p->mixed) {     // the first explicit part reads the row FFT of the start state
            int rc = dispatch_rows_fwd(p, p->pool[0], s);
            if (rc) return rc;
        }
    }
    HIP_TRY(hipMemcpyAsync(g->A, g->args_h.data(), sizeof(MarchArgs) * np, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(ks_init, dim3(1, np), dim3(64), 0, s, g->A);
    HIP_TRY(hipGetLastError());
    g->lc.A = g->A;
    st.maxit = 1;
    for (Plan* p : g->plans) st.maxit = std::max(st.maxit, p->opts.max_iter);
    st.kpred = std::min(8, st.maxit);
    return LPIDE_OK;
}

int march_enqueue(Group* g, MarchState& st) {
    int remaining = 0;
    for (int i = 0; i < g->lc.np; ++i) remaining = std::max(remaining, st.nsteps[i] - st.at[i]);
    if (remaining == 0) {
        st.done = true;
        return LPIDE_OK;
    }
    if (g->lc.timer) g->lc.timer->ev_mark = g->lc.timer->ev_recs.size();
    int ns = std::min(g->slots, remaining);
    // lean slots when every plan's steps in them are steady.  A window whose
    // first steps are not steady (the start of a march, or of a recompute
    // segment) ends where the steady run of every plan begins, so that the
    // rest goes out lean in the next windows.
    auto steady_from = [&](int k) {          // every plan steady on [at + k, at + ns)
        for (int i = 0; i < g->lc.np; ++i) {
            const Plan* p = g->plans[i];
            for (int q = st.at[i] + k; q < st.at[i] + ns && q < st.nsteps[i]; ++q)
                if (q >= (int)p->steady.size() || !p->steady[q]) return false;
        }
        return true;
    };
    bool lean = g->lc.jumps && !g->lc.mixed && steady_from(0);
    if (g->lc.jumps && !g->lc.mixed && !lean) {
        for (int k = 1; k < ns; ++k)
            if (steady_from(k)) {
                ns = k;
                break;
            }
    }
    g->lc.lean = lean;
    return enqueue_slots(g, st.at[0], ns, st.kpred);
}

int march_check(Group* g, MarchState& st) {
    if (st.done) return LPIDE_OK;
    const int np = g->lc.np;
    int rc = read_back(g);
    if (rc) return rc;
    int knext = 0;
    for (int i = 0; i < np; ++i) {
        if (g->ctl_h[i].fail) {
            Plan* tp = g->lc.timer;
            if (tp && tp == g->plans[i]) {  // the slots behind the failed step ran as no-ops; enqueued again later
                for (size_t q = tp->ev_mark; q < tp->ev_recs.size(); ++q)
                    if (tp->ev_recs[q].step > g->ctl_h[i].fail_step) tp->ev_recs[q].cls = -1;
            }
            int k = 0;
            if ((rc = complete_step(g, i, st.kpred, &k))) return rc;
            knext = std::max(knext, k);
        }
    }
    bool all = true;
    for (int i = 0; i < np; ++i) {
        const int reached = g->ctl_h[i].step;
        for (int q = st.at[i]; q < reached; ++q) knext = std::max(knext, g->counts_h[(size_t)i * g->maxsteps + q]);
        st.at[i] = reached;
        all = all && reached >= st.nsteps[i];
    }
    if (knext > 0) st.kpred = std::min(st.maxit, knext);
    st.done = all;
    return LPIDE_OK;
}

int march_end(Group* g, MarchState& st, double* const* v_out) {
    hipStream_t s = g->lc.stream;
    for (int i = 0; i < g->lc.np; ++i) {
        Plan* p = g->plans[i];
        const size_t N = (size_t)p->hp.n * p->hp.n;
        const int n1 = st.nsteps[i];
        p->counts_h.assign(p->n_steps, 0);
        p->total_iters = 0;
        p->max_step_iters = 0;
        p->last_step_iters = 0;
        p->last_inc = 0;
        for (int q = st.step0; q < n1; ++q) {
            const int cnt = g->counts_h[(size_t)i * g->maxsteps + q];
            p->counts_h[q] = cnt;
            p->total_iters += cnt;
            p->max_step_iters = std::max(p->max_step_iters, cnt);
        }
        if (n1 > st.step0) {
            p->last_step_iters = g->counts_h[(size_t)i * g->maxsteps + n1 - 1];
            p->last_inc = g->incs_h[(size_t)i * g->maxsteps + n1 - 1];
        }
        const int last = n1 > st.step0 ? g->ctl_h[i].cur : 0;   // the start state sits in pool[0]
        if (v_out && v_out[i])
            hipLaunchKernelGGL(k_copy, dim3((N + 255) / 256), dim3(256), 0, s, p->pool[last], v_out[i], N);
    }
    HIP_TRY(hipGetLastError());
    return LPIDE_OK;
}

// kpred0 > 0: the first prediction of iterations per step (else 8).
int march_group(Group* g, const int* nsteps, int step0, const double* const* v_in, double* const* v_out,
                int kpred0 = 0) {
    MarchState st;
    int rc = march_begin(g, st, nsteps, step0, v_in);
    if (!rc && kpred0 > 0) st.kpred = std::min(kpred0, st.maxit);
    while (!rc && !st.done) {
        rc = march_enqueue(g, st);
        if (!rc) rc = march_check(g, st);
    }
    if (!rc) rc = march_end(g, st, v_out);
    if (!rc) HIP_TRY(hipStreamSynchronize(g->lc.stream));
    return rc;
}

// March of one plan alone (its solo group on the plan's stream).
int march(Plan* p, int count, double* v_out) {
    Group* g = p->solo;
    g->lc.timer = p->time_mask ? p : nullptr;
    return march_group(g, &count, 0, nullptr, &v_out);
}

void destroy_adjoint(Adjoint* a) {
    if (!a) return;
    for (void* x : a->allocs) (void)hipFree(x);
    if (a->ctl_h) (void)hipHostFree(a->ctl_h);
    delete a;
}

// Allocate the adjoint buffers and the transposed step sets (once per plan and
// checkpoint stride).
int adj_prepare(Plan* p, int C) {
    if (p->adj && p->adj->C == C) return LPIDE_OK;
    destroy_adjoint(p->adj);
    p->adj = nullptr;
    p->ckpt_valid = false;
    Adjoint* a = new Adjoint();
    p->adj = a;
    const int n = p->hp.n, L = p->L, hc = L / 2 + 1, P = p->hp.sl_order;
    const size_t N = (size_t)n * n;
    a->C = C;
    a->n_ckpt = p->n_steps / C + 1;
    // a stride of at least the step count keeps every state and explicit part
    // of the march (one segment, recorded by the forward march itself)
    const size_t Cs = (size_t)std::min(C, p->n_steps);
    auto& al = a->allocs;
    int rc = LPIDE_OK;
    if ((rc = dalloc_into(al, nullptr, &a->ckpt, N * a->n_ckpt)) || (rc = dalloc_into(al, nullptr, &a->seg, N * (Cs + 1))) ||
        (rc = dalloc_into(al, nullptr, &a->segE, N * std::max<size_t>(1, Cs))) || (rc = dalloc_into(al, nullptr, &a->lam, N)) ||
        (rc = dalloc_into(al, nullptr, &a->mu, N)) || (rc = dalloc_into(al, nullptr, &a->ybar, N)) ||
        (rc = dalloc_into(al, nullptr, &a->dummy, N)) || (rc = dalloc_into(al, nullptr, &a->acc, (size_t)n * 8)) ||
        (rc = dalloc_into(al, nullptr, &a->corr[0], N)) || (rc = dalloc_into(al, nullptr, &a->corr[1], N)) ||
            (rc = dalloc_into(al, nullptr, &a->corr[2], N)) || (rc = dalloc_into(al, nullptr, &a->corr[3], N)) ||
        (rc = dalloc_into(al, nullptr, &a->ctl, 1)) || (rc = dalloc_into(al, nullptr, &a->counts, p->n_steps)) ||
        (rc = dalloc_into(al, nullptr, &a->incs, p->n_steps)) || (rc = dalloc_into(al, nullptr, &a->A, 1)))
        return rc;
    if (p->jumps) {
        if ((rc = dalloc_into(al, nullptr, &a->XA, (size_t)hc * n)) ||
            (rc = dalloc_into(al, nullptr, &a->XB, (size_t)hc * n)) ||
            (rc = dalloc_into(al, nullptr, &a->XC, (size_t)hc * n)) ||
            (rc = dalloc_into(al, nullptr, &a->XD, (size_t)hc * n)) ||
            (rc = dalloc_into(al, nullptr, &a->S, (size_t)hc * L)) ||
            (rc = dalloc_into(al, nullptr, &a->G, (size_t)L * L)))
            return rc;
    }
    if (hipHostMalloc((void**)&a->ctl_h, sizeof(Ctl), hipHostMallocDefault) != hipSuccess)
        return fail(LPIDE_E_OOM, "hipHostMalloc failed");
    a->counts_h.assign(p->n_steps, 0);
    // transposed step sets
    for (const StepDesc& fs : p->sets) {
        StepDesc sd = fs;
        const double c = sd.dt * sd.theta;
        std::vector<double> fl, bu, bc;
        double *f1, *u1, *c1, *f2, *u2, *c2;
        line_factors_T(n, p->hp.h, p->hp.a[0], p->hp.r_omega, c, fl, bu, bc);
        if ((rc = upload_into(al, &f1, fl)) || (rc = upload_into(al, &u1, bu)) || (rc = upload_into(al, &c1, bc))) return rc;
        line_factors_T(n, p->hp.h, p->hp.a[2], p->hp.r_omega, c, fl, bu, bc);
        if ((rc = upload_into(al, &f2, fl)) || (rc = upload_into(al, &u2, bu)) || (rc = upload_into(al, &c2, bc))) return rc;
        sd.fl1 = f1; sd.bu1 = u1; sd.bc1 = c1;
        sd.fl2 = f2; sd.bu2 = u2; sd.bc2 = c2;
        for (int ax = 0; ax < 2; ++ax) {
            const double shift = p->hp.kappa[ax] * sd.dt / p->hp.h;
            std::vector<int32_t> st, ti;
            std::vector<double> w, dw, tw;
            sl_weights(n, shift, P, st, w);
            sl_dweights(n, shift, P, dw);
            for (double& x : dw) x *= sd.dt / p->hp.h;        // d/d kappa_omega = (dt / h) d/d xi
            const int width = sl_transpose(n, P, st, w, ti, tw);
            int* tid = nullptr;
            double *twd = nullptr, *dwd = nullptr;
            if ((rc = upload_into(al, &tid, ti)) || (rc = upload_into(al, &twd, tw)) || (rc = upload_into(al, &dwd, dw)))
                return rc;
            if (ax == 0) { sd.t1i = tid; sd.t1w = twd; sd.wt1 = width; sd.w1d = dwd; }
            else { sd.t2i = tid; sd.t2w = twd; sd.wt2 = width; sd.w2d = dwd; }
        }
        a->sets.push_back(sd);
    }
    if ((rc = upload_into(al, &a->sets_d, a->sets))) return rc;
    MarchArgs m = march_args(p);
    m.pool[0] = a->mu;
    m.pool[1] = a->lam;
    for (int b = 2; b < POOL; ++b) m.pool[b] = a->dummy;
    m.sets = a->sets_d;
    m.W = a->ybar;
    m.ctl = a->ctl;
    m.counts = a->counts;
    m.incs = a->incs;
    m.mixed = 0;
    m.cn_rho = nullptr;                // the reverse march forms its explicit parts by the correlation
    for (int b = 0; b < POOL; ++b) m.bpool[b] = nullptr;
    m.nsteps = p->n_steps;
    m.seg = nullptr;
    m.segE = nullptr;
    a->args = m;
    HIP_TRY(hipMemcpy(a->A, &a->args, sizeof(MarchArgs), hipMemcpyHostToDevice));
    return LPIDE_OK;
}

// Forward march with recording: states every `every` steps from seg_base to
// `seg`, and (every == 1) the explicit parts to segE.
int march_recorded(Plan* p, int step0, int nsteps, const double* v_in, double* seg, double* segE, int every,
                   double* v_out, int kpred0 = 0) {
    Group* g = p->solo;
    MarchArgs& m = g->args_h[0];
    m.seg = seg;
    m.segE = segE;
    m.seg_base = step0;
    m.seg_every = every;
    g->lc.record = true;
    g->lc.timer = nullptr;
    const size_t N = (size_t)p->hp.n * p->hp.n;
    g->lc.store_blocks = int(std::min<size_t>(1024, (N + 255) / 256));
    double* outs[1] = {v_out};
    const double* ins[1] = {v_in};
    int rc = march_group(g, &nsteps, step0, v_in ? ins : nullptr, outs, kpred0);
    m.seg = nullptr;
    m.segE = nullptr;
    g->lc.record = false;
    return rc;
}

int dispatch_adj_step(Plan* p, const Launch& c, int s, int* kpred, const double* Y, const double* V,
                      const double* E) {
#define CALL_ADJ(Lc) return PerL<Lc>::adj_step(p, c, s, kpred, Y, V, E)
    LPIDE_SWITCH_L(p->Lr, CALL_ADJ)
#undef CALL_ADJ
    return LPIDE_OK;
}

int dispatch_adj_kernel_grad(Plan* p, hipStream_t s) {
#define CALL_KG(Lc) PerL<Lc>::adj_kernel_grad(p, s)
    LPIDE_SWITCH_L(p->L, CALL_KG)
#undef CALL_KG
    HIP_TRY(hipGetLastError());
    return LPIDE_OK;
}

// Host model quantities that the march depends on continuously, at the
// subordination parameters x (sigma1, sigma2, corr, theta1, theta2, kappa,
// alpha, r), structure frozen at the plan's N_z: a11, a12, a22, r_omega,
// kappa_omega^(1,2), then omega.
int model_quantities(const Plan* p, const double* x, std::vector<double>& out) {
    lpide_levy lv;
    int rc = lpide_levy_from_std(x[0], x[1], x[2], x[3], x[4], x[5], x[6], x[7], &lv);
    if (rc) return rc;
    lpide_grid g;
    lpide_grid_default(&g, p->hp.n, 0.0, 1.0);
    g.y_lo[0] = p->hp.y_lo[0];
    g.y_lo[1] = p->hp.y_lo[1];
    g.y_hi[0] = p->hp.y_lo[0] + p->hp.h * (p->hp.n - 1);
    g.y_hi[1] = p->hp.y_lo[1] + p->hp.h * (p->hp.n - 1);
    g.sl_order = p->hp.sl_order;
    g.in_order = p->hp.in_order;
    g.m1 = p->hp.M1;
    g.ell_cut = p->grid.ell_cut;
    g.zmax2_frac = p->grid.zmax2_frac;
    g.gl_nodes = p->grid.gl_nodes;
    g.nz_fixed = p->hp.N_z;
    HostPlan hp;
    std::string err;
    if (!build_host_plan(g, lv, hp, err)) return fail(LPIDE_E_PARAM, "model quantities: " + err);
    if (hp.M2 != p->hp.M2 || hp.L_need > p->L) return fail(LPIDE_E_PARAM, "structure changed under the perturbation");
    out.assign(6 + hp.omega.size(), 0.0);
    out[0] = hp.a[0];
    out[1] = hp.a[1];
    out[2] = hp.a[2];
    out[3] = hp.r_omega;
    out[4] = hp.kappa[0];
    out[5] = hp.kappa[1];
    std::copy(hp.omega.begin(), hp.omega.end(), out.begin() + 6);
    return LPIDE_OK;
}

// Central differences of model_quantities with steps 1e-4 max(|x_q|, 0.1)
// for the seven Levy parameters; r enters only as kappa_omega = r - ... and
// r_omega = r + sum omega, so its column is exact (0, 0, 0, 1, 1, 1, 0...).
int model_jacobian(Plan* p, const double* x) {
    Adjoint* a = p->adj;
    if (a->jac_valid && std::equal(x, x + 8, a->jac_std)) return LPIDE_OK;
    std::vector<double> fp, fm;
    size_t m = 0;
    for (int q = 0; q < 7; ++q) {
        double xp[8], xm[8];
        std::copy(x, x + 8, xp);
        std::copy(x, x + 8, xm);
        const double hq = 1e-4 * std::max(std::fabs(x[q]), 0.1);
        xp[q] += hq;
        xm[q] -= hq;
        int rc = model_quantities(p, xp, fp);
        if (!rc) rc = model_quantities(p, xm, fm);
        if (rc) return rc;
        if (q == 0) {
            m = fp.size();
            a->jac.assign(8 * m, 0.0);
        }
        for (size_t i = 0; i < m; ++i) a->jac[q * m + i] = (fp[i] - fm[i]) / (2.0 * hq);
    }
    a->jac[7 * m + 3] = 1.0;
    a->jac[7 * m + 4] = 1.0;
    a->jac[7 * m + 5] = 1.0;
    std::copy(x, x + 8, a->jac_std);
    a->jac_valid = true;
    return LPIDE_OK;
}

// The full adjoint: checkpointed forward (unless the last solve recorded the
// same checkpoints), then per segment from the last: recompute with
// recording, reverse steps.  native[0..5] = dJ/d(a11, a12, a22, r_omega,
// kappa1, kappa2), native[6..] = dJ/d omega.
// The forward march with the adjoint's records: checkpoints every C steps, or,
// when C is at least the step count, every state and explicit part (the
// reverse march then needs no recompute).  Needs adj_prepare(p, C).
int record_forward(Plan* p, int C, double* v_out) {
    Adjoint* a = p->adj;
    const size_t N = (size_t)p->hp.n * p->hp.n;
    if (C >= p->n_steps) {
        hipLaunchKernelGGL(k_copy, dim3((N + 255) / 256), dim3(256), 0, p->stream, p->V0, a->seg, N);
        return march_recorded(p, 0, p->n_steps, nullptr, a->seg, a->segE, 1, v_out);
    }
    hipLaunchKernelGGL(k_copy, dim3((N + 255) / 256), dim3(256), 0, p->stream, p->V0, a->ckpt, N);
    return march_recorded(p, 0, p->n_steps, nullptr, a->ckpt, nullptr, C, v_out);
}

int adjoint(Plan* p, const double* v_bar, int C, std::vector<double>& native, lpide_adjoint_info* info) {
    int rc = adj_prepare(p, C);
    if (rc) return rc;
    Adjoint* a = p->adj;
    const int n = p->hp.n, Ns = p->n_steps;
    const size_t N = (size_t)n * n;
    hipStream_t s = p->stream;
    auto now = [] { return std::chrono::steady_clock::now(); };
    auto ms = [](std::chrono::steady_clock::time_point t0, std::chrono::steady_clock::time_point t1) {
        return std::chrono::duration<double, std::milli>(t1 - t0).count();
    };
    double t_fwd = 0.0;
    const bool keep_all = C >= Ns;     // every state kept by the forward march: no recompute
    if (!(p->ckpt_valid && p->ckpt_every == C)) {
        auto t0 = now();
        if ((rc = record_forward(p, C, nullptr))) return rc;
        t_fwd = ms(t0, now());
    }
    HIP_TRY(hipMemcpyAsync(a->ybar, v_bar, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemsetAsync(a->acc, 0, sizeof(double) * N / n * 8, s));
    if (p->jumps) HIP_TRY(hipMemsetAsync(a->S, 0, sizeof(double2) * (size_t)(p->L / 2 + 1) * p->L, s));
    Launch c;
    c.stream = s;
    c.A = a->A;
    c.np = 1;
    c.L = p->Lr;
    c.xrows = (n + 1) / 2;
    c.cpb = line_cols_cpb(n, 1);
    c.xcols = (n + c.cpb - 1) / c.cpb;
    c.xaff = n;
    c.P_cols = p->solo->lc.P_cols;
    c.sl_order = p->hp.sl_order;
    c.jumps = p->jumps;
    c.E_cols = p->solo->lc.E_cols;
    c.E_rinv = p->solo->lc.E_rinv;
    c.E_lrows = p->solo->lc.E_lrows;
    c.E_sl = p->solo->lc.E_sl;
    a->args.P_cols = c.P_cols;
    HIP_TRY(hipMemcpyAsync(a->A, &a->args, sizeof(MarchArgs), hipMemcpyHostToDevice, s));
    double t_rec = 0.0, t_rev = 0.0;
    int kpred = std::min(8, p->opts.max_iter);
    // iteration counts of the forward march: each segment's recompute starts
    // from their maximum over the segment instead of the default prediction
    const std::vector<int> fwd_counts = p->counts_h;
    int64_t iters = 0;
    int maxit = 0;
    a->have_corr = 0;
    a->xb_is_v = false;
    for (int q = (Ns - 1) / C; q >= 0; --q) {
        const int s0 = q * C, s1 = std::min(Ns, s0 + C);
        auto ta = now();
        if (!keep_all) {
            HIP_TRY(hipMemcpyAsync(a->seg, a->ckpt + (size_t)q * N, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
            int k0 = 0;
            for (int st = s0; st < s1 && st < (int)fwd_counts.size(); ++st) k0 = std::max(k0, fwd_counts[st]);
            if ((rc = march_recorded(p, s0, s1, a->ckpt + (size_t)q * N, a->seg, a->segE, 1, nullptr, k0))) return rc;
        }
        HIP_TRY(hipStreamSynchronize(s));
        auto tb = now();
        for (int st = s1 - 1; st >= s0; --st) {
            const double* Y = a->seg + (size_t)(st + 1 - s0) * N;
            const double* V = a->seg + (size_t)(st - s0) * N;
            const double* E = p->sets[p->step_set[st]].theta < 1.0 ? a->segE + (size_t)(st - s0) * N : V;
            if ((rc = dispatch_adj_step(p, c, st, &kpred, Y, V, E))) return rc;
            iters += a->counts_h[st];
            maxit = std::max(maxit, a->counts_h[st]);
        }
        HIP_TRY(hipStreamSynchronize(s));
        t_rec += ms(ta, tb);
        t_rev += ms(tb, now());
    }
    // gradient terms to the host
    auto tc = now();
    std::vector<double> acc(N / n * 8);
    HIP_TRY(hipMemcpy(acc.data(), a->acc, sizeof(double) * acc.size(), hipMemcpyDeviceToHost));
    const int Nz = p->hp.N_z, W2 = 2 * Nz;
    native.assign(6 + (p->jumps ? (size_t)W2 * W2 : 0), 0.0);
    for (int q = 0; q < 6; ++q) {
        double t = 0.0;
        for (int i = 0; i < n; ++i) t += acc[(size_t)i * 8 + q];
        native[q] = t;
    }
    if (p->jumps) {
        if ((rc = dispatch_adj_kernel_grad(p, s))) return rc;
        const int L = p->L;
        std::vector<double> G((size_t)L * L);
        HIP_TRY(hipMemcpyAsync(G.data(), a->G, sizeof(double) * G.size(), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const double inv = 1.0 / (double(L) * double(L));
        auto gk = [&](int d1, int d2) {
            return G[(size_t)(((d1 % L) + L) % L) * L + (((d2 % L) + L) % L)] * inv;
        };
        // dJ/d omega_l = sum_j s_j1 s_j2 dJ/dK_{l + jlo + j}  (K = omega folded with the half-cell taps)
        const int Pin = p->hp.in_order, jlo = -(Pin - 1) / 2;
        double sw[4];
        for (int i = 0; i <= Pin; ++i) {
            double v = 1.0;
            for (int j = 0; j <= Pin; ++j)
                if (j != i) v *= (0.5 - (jlo + j)) / double(i - j);
            sw[i] = v;
        }
        auto rows = [&](int r0, int r1) {
            for (int l1 = r0 - Nz; l1 < r1 - Nz; ++l1)
                for (int l2 = -Nz; l2 < Nz; ++l2) {
                    double t = 0.0;
                    for (int j1 = 0; j1 <= Pin; ++j1)
                        for (int j2 = 0; j2 <= Pin; ++j2) t += sw[j1] * sw[j2] * gk(l1 + jlo + j1, l2 + jlo + j2);
                    native[6 + (size_t)(l1 + Nz) * W2 + (l2 + Nz)] = t;
                }
        };
        const int nth = int(std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
        std::vector<std::thread> th;
        for (int t = 0; t < nth; ++t) {
            const int r0 = int((int64_t)W2 * t / nth), r1 = int((int64_t)W2 * (t + 1) / nth);
            if (r0 < r1) th.emplace_back(rows, r0, r1);
        }
        for (auto& x : th) x.join();
    }
    if (info) {
        info->adj_iters = iters;
        info->max_step_iters = maxit;
        info->forward_ms = t_fwd;
        info->recompute_ms = t_rec;
        info->reverse_ms = t_rev;
        info->gather_ms = ms(tc, now());
    }
    return LPIDE_OK;
}

void destroy(Plan* p) {
    if (!p) return;
    (void)hipStreamSynchronize(p->stream);
    destroy_group(p->solo);
    destroy_adjoint(p->adj);
    for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
    for (void* a : p->allocs) (void)hipFree(a);
    delete p;
}

// ---- batches ----
struct Batch {
    std::vector<Plan*> plans;
    std::vector<Group*> groups;
    std::vector<std::vector<int>> members;     // plan indices of each group
    std::vector<hipStream_t> streams;          // one per group
    std::vector<hipEvent_t> events;            // one per group + 1
    hipStream_t caller = nullptr;
    bool tuned = false;
    bool owns_plans = false;                   // made by lpide_plan_batch
};

void destroy_batch(Batch* b) {
    if (!b) return;
    for (Group* g : b->groups) destroy_group(g);
    for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
    for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
    if (b->owns_plans)
        for (Plan* p : b->plans) destroy(p);
    delete b;
}

// March every plan of the batch over its whole step list (or its first
// steps_cap entries); groups run on their own streams, joined to the caller's
// stream before and after.  The host interleaves the groups: it enqueues a
// round of slots for every group, then checks each group (waiting only on
// that group's stream), so the device overlaps the groups.
int batch_march(Batch* b, double* const* v_out, int steps_cap) {
    const int ng = int(b->groups.size());
    HIP_TRY(hipEventRecord(b->events[ng], b->caller));
    for (int q = 0; q < ng; ++q) HIP_TRY(hipStreamWaitEvent(b->streams[q], b->events[ng], 0));
    std::vector<MarchState> st(ng);
    for (int q = 0; q < ng; ++q) {
        std::vector<int> ns;
        for (int i : b->members[q])
            ns.push_back(steps_cap >= 0 ? std::min(steps_cap, b->plans[i]->n_steps) : b->plans[i]->n_steps);
        int rc = march_begin(b->groups[q], st[q], ns.data(), 0, nullptr);
        if (rc) return rc;
    }
    for (;;) {
        bool all = true;
        for (int q = 0; q < ng; ++q) {
            if (st[q].done) continue;
            int rc = march_enqueue(b->groups[q], st[q]);
            if (rc) return rc;
        }
        for (int q = 0; q < ng; ++q) {
            int rc = march_check(b->groups[q], st[q]);
            if (rc) return rc;
            all = all && st[q].done;
        }
        if (all) break;
    }
    for (int q = 0; q < ng; ++q) {
        std::vector<double*> outs;
        for (int i : b->members[q]) outs.push_back(v_out ? v_out[i] : nullptr);
        int rc = march_end(b->groups[q], st[q], outs.data());
        if (rc) return rc;
        HIP_TRY(hipEventRecord(b->events[q], b->streams[q]));
    }
    for (int q = 0; q < ng; ++q) HIP_TRY(hipStreamWaitEvent(b->caller, b->events[q], 0));
    return LPIDE_OK;
}

}  // namespace
}  // namespace detail
}  // namespace lpide

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void lpide_grid_default(lpide_grid* g, int32_t n, double y_lo, double y_hi) {
    if (!g) return;
    std::memset(g, 0, sizeof *g);
    g->n = n;
    g->y_lo[0] = g->y_lo[1] = y_lo;
    g->y_hi[0] = g->y_hi[1] = y_hi;
    g->sl_order = 3;
    g->in_order = 3;
    g->m1 = 2;
    g->ell_cut = 1e-14;
    g->zmax2_frac = std::sqrt(0.1);
    g->gl_nodes = 8;
}

void lpide_opts_default(lpide_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->tol = 1e-12;
    o->max_iter = 100;
    o->precision = LPIDE_FP64;
    o->damping = 1;
    o->device = 0;
    o->stream = nullptr;
}

int lpide_levy_from_std(double sigma1, double sigma2, double corr, double theta1, double theta2, double kappa,
                        double alpha, double r, lpide_levy* out) {
    if (!out) return fail(LPIDE_E_PARAM, "out is NULL");
    if (!(sigma1 > 0) || !(sigma2 > 0) || !(corr > -1 && corr < 1) || !(kappa > 0) || !(alpha >= 0 && alpha < 1) ||
        !std::isfinite(theta1) || !std::isfinite(theta2) || !std::isfinite(r))
        return fail(LPIDE_E_PARAM, "parameters out of range");
    std::memset(out, 0, sizeof *out);
    out->r = r;
    out->alpha = alpha;
    out->lambda = (1.0 - alpha) / kappa;
    out->delta = std::pow(out->lambda, 1.0 - alpha) / std::tgamma(1.0 - alpha);
    out->eta[0] = theta1;
    out->eta[1] = theta2;
    out->rho[0] = sigma1 * sigma1;
    out->rho[1] = corr * sigma1 * sigma2;
    out->rho[2] = sigma2 * sigma2;
    return LPIDE_OK;
}

int lpide_discretize_host(const lpide_grid* grid, const lpide_levy* levy, const lpide_payoff* payoff,
                          lpide_info* info, double* omega, int64_t omega_len, double* v0) {
    if (!grid || !levy || !info) return fail(LPIDE_E_PARAM, "NULL argument");
    HostPlan hp;
    std::string err;
    if (!build_host_plan(*grid, *levy, hp, err)) return fail(LPIDE_E_PARAM, err);
    std::memset(info, 0, sizeof *info);
    info->n = hp.n;
    info->N_z = hp.N_z;
    info->M1 = hp.M1;
    info->M2 = hp.M2;
    info->L = hp.L;
    info->h = hp.h;
    info->z_star = hp.z_star;
    info->sum_omega = hp.sum_omega;
    info->kappa[0] = hp.kappa[0];
    info->kappa[1] = hp.kappa[1];
    info->r_omega = hp.r_omega;
    for (int k = 0; k < 3; ++k) {
        info->S[k] = hp.S[k];
        info->a[k] = hp.a[k];
    }
    if (omega && omega_len >= (int64_t)hp.omega.size())
        std::memcpy(omega, hp.omega.data(), hp.omega.size() * sizeof(double));
    if (v0) {
        if (!payoff) return fail(LPIDE_E_PARAM, "payoff is NULL but v0 requested");
        std::vector<double> v;
        if (!initial_values(hp, *payoff, v, err)) return fail(LPIDE_E_PARAM, err);
        std::memcpy(v0, v.data(), v.size() * sizeof(double));
    }
    return LPIDE_OK;
}

int lpide_plan_create(const lpide_grid* grid, const lpide_levy* levy, const lpide_payoff* payoff, double theta,
                      int32_t M, const lpide_opts* opts, void** out) {
    if (!grid || !levy || !payoff || !out) return fail(LPIDE_E_PARAM, "NULL argument");
    lpide_opts o;
    if (opts) o = *opts; else lpide_opts_default(&o);
    if (!(theta >= 0.0 && theta <= 1.0)) return fail(LPIDE_E_PARAM, "theta must lie in [0, 1]");
    if (M < 1) return fail(LPIDE_E_PARAM, "M (time steps) must be >= 1");
    if (!(o.tol > 0.0) || o.max_iter < 1) return fail(LPIDE_E_PARAM, "tol must be > 0 and max_iter >= 1");
    if (o.precision != LPIDE_FP64 && o.precision != LPIDE_FP32_CONV)
        return fail(LPIDE_E_PARAM, "precision must be LPIDE_FP64 or LPIDE_FP32_CONV");
    if (o.max_iter > MAX_ITER_CAP) return fail(LPIDE_E_PARAM, "max_iter must not exceed 128");
    if (o.fft_radix != 0 && o.fft_radix != 4 && o.fft_radix != 8 && o.fft_radix != 16)
        return fail(LPIDE_E_PARAM, "fft_radix must be 0, 4, 8 or 16");
    if (o.mixed_anchor < 0) return fail(LPIDE_E_PARAM, "mixed_anchor must be >= 0");
    if (o.all_correlations != 0 && o.all_correlations != 1) return fail(LPIDE_E_PARAM, "all_correlations must be 0 or 1");
    if (o.accel != 0) return fail(LPIDE_E_PARAM, "accel applies to the price-space plan only (0 here)");
    Plan* p = new Plan();
    std::string err;
    if (!build_host_plan(*grid, *levy, p->hp, err)) { delete p; return fail(LPIDE_E_PARAM, err); }
    std::vector<double> v0;
    if (!initial_values(p->hp, *payoff, v0, err)) { delete p; return fail(LPIDE_E_PARAM, err); }
    p->opts = o;
    p->grid = *grid;
    p->pay = *payoff;
    p->theta = theta;
    p->N_t = M;
    p->stream = static_cast<hipStream_t>(o.stream);
    p->jumps = p->hp.nts.jumps;
    p->mixed = p->jumps && o.precision == LPIDE_FP32_CONV;
    p->anchor_every = o.mixed_anchor > 0 ? o.mixed_anchor : 8;
    if (p->jumps && o.fft_size != 0) {
        if (!fft_size_supported(o.fft_size) || o.fft_size < p->hp.L_need) {
            const std::string msg = "fft_size " + std::to_string(o.fft_size) +
                                    " is not a supported transform side of at least " + std::to_string(p->hp.L_need);
            delete p;
            return fail(LPIDE_E_PARAM, msg);
        }
        p->hp.L = o.fft_size;
    }
    p->L = p->hp.L;
    int rc = LPIDE_OK;
    auto bail = [&](int code) { destroy(p); return code; };
    {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) { destroy(p); return fail(LPIDE_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e)); }
        e = hipSetDevice(o.device);
        if (e != hipSuccess) { destroy(p); return fail(LPIDE_E_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e)); }
    }
    // this device's copy of the allocation-free entry point's scratch
    if ((rc = scratch_setup(o.device))) return bail(rc);
    const int n = p->hp.n;
    const size_t N = (size_t)n * n;
    if ((rc = upload(p, &p->V0, v0))) return bail(rc);
    for (int b = 0; b < POOL; ++b)
        if ((rc = dalloc(p, &p->pool[b], N))) return bail(rc);
    if ((rc = dalloc(p, &p->Wb, N))) return bail(rc);
    if ((rc = dalloc(p, &p->Rb, N))) return bail(rc);
    if (p->jumps && !p->mixed && !o.all_correlations)    // B of the pool grids, for B Y^0 by linearity
        for (int b = 0; b < POOL; ++b)
            if ((rc = dalloc(p, &p->bpool[b], N))) return bail(rc);
    // axis-1 line solves: 4 columns per block, chunks of about 8 rows
    p->P_cols = default_P_cols(n);
    if (!P_cols_valid(n, p->P_cols)) return bail(fail(LPIDE_E_PARAM, "n too large for the line solves"));
    // transform side of the row-pair kernels (without jumps: the power of two >= n)
    p->Lr = p->L;
    if (!p->jumps) {
        p->Lr = 64;
        while (p->Lr < n) p->Lr *= 2;
    }
    if (p->Lr > 4096) return bail(fail(LPIDE_E_PARAM, "n too large"));
    // step list and its distinct (theta, dt) sets
    {
        auto steps = step_list(theta, payoff->T, M, o.damping != 0);
        p->n_steps = int(steps.size());
        for (auto& st : steps) {
            int id = -1;
            for (size_t q = 0; q < p->sets.size(); ++q)
                if (p->sets[q].theta == st.first && p->sets[q].dt == st.second) id = int(q);
            if (id < 0) {
                StepDesc sd{};
                sd.theta = st.first;
                sd.dt = st.second;
                const double c = sd.dt * sd.theta;
                std::vector<double> fl, bu, bc;
                double *f1, *u1, *c1, *f2, *u2, *c2, *w1, *w2;
                int *s1, *s2;
                line_factors(n, p->hp.h, p->hp.a[0], p->hp.r_omega, c, fl, bu, bc);
                if ((rc = upload(p, &f1, fl)) || (rc = upload(p, &u1, bu)) || (rc = upload(p, &c1, bc))) return bail(rc);
                line_factors(n, p->hp.h, p->hp.a[2], p->hp.r_omega, c, fl, bu, bc);
                if ((rc = upload(p, &f2, fl)) || (rc = upload(p, &u2, bu)) || (rc = upload(p, &c2, bc))) return bail(rc);
                std::vector<int32_t> st1, st2;
                std::vector<double> ww1, ww2;
                sl_weights(n, p->hp.kappa[0] * sd.dt / p->hp.h, p->hp.sl_order, st1, ww1);
                sl_weights(n, p->hp.kappa[1] * sd.dt / p->hp.h, p->hp.sl_order, st2, ww2);
                if ((rc = upload(p, &s1, st1)) || (rc = upload(p, &s2, st2)) || (rc = upload(p, &w1, ww1)) ||
                    (rc = upload(p, &w2, ww2)))
                    return bail(rc);
                sd.fl1 = f1; sd.bu1 = u1; sd.bc1 = c1;
                sd.fl2 = f2; sd.bu2 = u2; sd.bc2 = c2;
                sd.s1 = s1; sd.s2 = s2; sd.w1 = w1; sd.w2 = w2;
                p->sets.push_back(sd);
                id = int(p->sets.size()) - 1;
            }
            p->step_set.push_back(id);
        }
        if ((rc = upload(p, &p->sets_d, p->sets)) || (rc = upload(p, &p->step_set_d, p->step_set))) return bail(rc);
        p->counts_h.assign(p->n_steps, 0);
        // rho of the explicit part from the previous step's implicit equation:
        // dt (1 - theta) / (dt theta of the step before); 0 where the correlation is needed
        p->cn_rho.assign(p->n_steps, 0.0);
        for (int q = 1; q < p->n_steps; ++q) {
            const StepDesc& cu = p->sets[p->step_set[q]];
            const StepDesc& pr = p->sets[p->step_set[q - 1]];
            if (cu.theta < 1.0 && pr.theta > 0.0) p->cn_rho[q] = cu.dt * (1.0 - cu.theta) / (pr.dt * pr.theta);
        }
        if ((rc = upload(p, &p->cn_rho_d, p->cn_rho))) return bail(rc);
    }
    // kernel spectrum conj(FFT(K placed at d mod L)) / L^2
    if (p->jumps) {
        const int L = p->L;
        std::vector<double2> tw(L);
        for (int q = 0; q < L; ++q) {
            // exp(-2 pi i q / L), evaluated in long double
            const long double ang = -2.0L * 3.14159265358979323846264338327950288L * q / L;
            tw[q] = make_double2((double)cosl(ang), (double)sinl(ang));
        }
        if ((rc = upload(p, &p->tw, tw))) return bail(rc);
        if ((rc = dalloc(p, &p->spec, (size_t)(L / 2 + 1) * L))) return bail(rc);
        if ((rc = dalloc(p, &p->X, (size_t)(L / 2 + 1) * n))) return bail(rc);
        std::vector<double> G((size_t)L * L, 0.0);
        const int KW = p->hp.dhi - p->hp.dlo + 1;
        for (int a = 0; a < KW; ++a) {
            const int d1 = a + p->hp.dlo, r1 = ((d1 % L) + L) % L;
            for (int b = 0; b < KW; ++b) {
                const int d2 = b + p->hp.dlo, r2 = ((d2 % L) + L) % L;
                G[(size_t)r1 * L + r2] = p->hp.kern[(size_t)a * KW + b];
            }
        }
        double* Gd = nullptr;
        double2* Xf = nullptr;
        if (hipMalloc(&Gd, G.size() * sizeof(double)) != hipSuccess) return bail(fail(LPIDE_E_OOM, "hipMalloc G"));
        if (hipMalloc(&Xf, (size_t)(L / 2 + 1) * L * sizeof(double2)) != hipSuccess) {
            (void)hipFree(Gd);
            return bail(fail(LPIDE_E_OOM, "hipMalloc Xf"));
        }
        hipError_t e = hipMemcpy(Gd, G.data(), G.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) rc = dispatch_spectrum(p, Gd, Xf);
        if (e == hipSuccess && rc == LPIDE_OK) e = hipStreamSynchronize(p->stream);
        (void)hipFree(Gd);
        (void)hipFree(Xf);
        if (e != hipSuccess) return bail(fail(LPIDE_E_HIP, std::string("spectrum: ") + hipGetErrorString(e)));
        if (rc) return bail(rc);
        if (p->mixed) {
            const size_t ns = (size_t)(L / 2 + 1) * L;
            if ((rc = dalloc(p, &p->spec32, ns)) || (rc = dalloc(p, &p->X32, (size_t)(L / 2 + 1) * n)) ||
                (rc = dalloc(p, &p->BV, N)) || (rc = dalloc(p, &p->BY, N)))
                return bail(rc);
            hipLaunchKernelGGL(k_to_f32, dim3((ns + 255) / 256), dim3(256), 0, p->stream, p->spec, p->spec32, ns);
            e = hipGetLastError();
            if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
            if (e != hipSuccess) return bail(fail(LPIDE_E_HIP, std::string("spectrum32: ") + hipGetErrorString(e)));
        }
    }
    p->sched = o.fft_radix ? uniform_schedule(o.fft_radix) : default_schedule(p->Lr);
    if (!schedule_ok(p->Lr, p->sched))
        return bail(fail(LPIDE_E_PARAM, "fft_radix " + std::to_string(o.fft_radix) + " is not supported at transform side " +
                                            std::to_string(p->Lr)));
    if ((rc = make_group(std::vector<Plan*>{p}, p->stream, &p->solo))) return bail(rc);
    *out = p;
    return LPIDE_OK;
}

int lpide_plan_destroy(void* plan) {
    destroy(static_cast<Plan*>(plan));
    return LPIDE_OK;
}

int lpide_plan_info(void* plan, lpide_info* info) {
    if (!plan || !info) return fail(LPIDE_E_PARAM, "NULL argument");
    const Plan* p = static_cast<const Plan*>(plan);
    std::memset(info, 0, sizeof *info);
    info->n = p->hp.n;
    info->N_z = p->hp.N_z;
    info->M1 = p->hp.M1;
    info->M2 = p->hp.M2;
    info->L = p->L;
    info->N_t = p->N_t;
    info->n_steps = int32_t(p->n_steps);
    info->h = p->hp.h;
    info->z_star = p->hp.z_star;
    info->sum_omega = p->hp.sum_omega;
    info->kappa[0] = p->hp.kappa[0];
    info->kappa[1] = p->hp.kappa[1];
    info->r_omega = p->hp.r_omega;
    for (int k = 0; k < 3; ++k) {
        info->S[k] = p->hp.S[k];
        info->a[k] = p->hp.a[k];
    }
    info->total_iters = p->total_iters;
    info->max_step_iters = p->max_step_iters;
    info->last_step_iters = p->last_step_iters;
    info->last_increment = p->last_inc;
    info->device_bytes = p->bytes;
    info->radix[0] = p->solo->lc.E_cols;
    info->radix[1] = p->solo->lc.E_rinv;
    info->radix[2] = p->solo->lc.E_lrows;
    info->radix[3] = p->solo->lc.E_sl;
    return LPIDE_OK;
}

int lpide_solve(void* plan, double* v_out) {
    if (!plan || !v_out) return fail(LPIDE_E_PARAM, "NULL argument");
    Plan* p = static_cast<Plan*>(plan);
    p->ckpt_valid = false;
    if (p->ckpt_every > 0) {
        int rc = adj_prepare(p, p->ckpt_every);
        if (rc) return rc;
        rc = record_forward(p, p->ckpt_every, v_out);
        p->ckpt_valid = rc == LPIDE_OK;
        return rc;
    }
    return march(p, p->n_steps, v_out);
}

int lpide_plan_set_checkpoints(void* plan, int32_t every) {
    if (!plan || every < 0) return fail(LPIDE_E_PARAM, "NULL plan or every < 0");
    Plan* p = static_cast<Plan*>(plan);
    if (every > 0 && !p->jumps) return fail(LPIDE_E_PARAM, "the adjoint march needs a Levy measure");
    p->ckpt_every = every;
    p->ckpt_valid = false;
    return LPIDE_OK;
}

int lpide_adjoint(void* plan, const double* v_bar, int32_t checkpoint_every, const double* std_params, double* grad,
                  double* native, lpide_adjoint_info* info) {
    if (!plan || !v_bar) return fail(LPIDE_E_PARAM, "NULL argument");
    Plan* p = static_cast<Plan*>(plan);
    if (!p->jumps) return fail(LPIDE_E_PARAM, "the adjoint march needs a Levy measure");
    if (checkpoint_every < 1) return fail(LPIDE_E_PARAM, "checkpoint_every must be >= 1");
    if (grad && !std_params) return fail(LPIDE_E_PARAM, "grad needs std_params");
    if (info) std::memset(info, 0, sizeof *info);
    std::vector<double> nat;
    int rc = adjoint(p, v_bar, checkpoint_every, nat, info);
    if (rc) return rc;
    if (native) std::copy(nat.begin(), nat.end(), native);
    if (grad) {
        // the std point must be the one the plan's model came from
        lpide_levy lv;
        if ((rc = lpide_levy_from_std(std_params[0], std_params[1], std_params[2], std_params[3], std_params[4],
                                      std_params[5], std_params[6], std_params[7], &lv)))
            return rc;
        const Nts& q = p->hp.nts;
        auto close = [](double x, double y) { return std::fabs(x - y) <= 1e-12 * std::max(1.0, std::fabs(y)); };
        if (!close(lv.alpha, q.alpha) || !close(lv.delta, q.delta) || !close(lv.lambda, q.lambda) ||
            !close(lv.eta[0], q.eta[0]) || !close(lv.eta[1], q.eta[1]) || !close(lv.rho[0], q.rho[0]) ||
            !close(lv.rho[1], q.rho[1]) || !close(lv.rho[2], q.rho[2]) || !close(lv.r, p->hp.r))
            return fail(LPIDE_E_PARAM, "std_params do not map to the plan's model");
        const auto t0 = std::chrono::steady_clock::now();
        if ((rc = model_jacobian(p, std_params))) return rc;
        const size_t m = nat.size();
        for (int k = 0; k < 8; ++k) {
            double t = 0.0;
            const double* jr = p->adj->jac.data() + (size_t)k * m;
            for (size_t i = 0; i < m; ++i) t += nat[i] * jr[i];
            grad[k] = t;
        }
        if (info)
            info->jacobian_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return LPIDE_OK;
}

int lpide_price_adjoint(void* plan, int32_t npts, const double* spots, const double* price_bar, double* v_bar) {
    if (!plan || !v_bar || npts < 0 || (npts > 0 && (!spots || !price_bar)))
        return fail(LPIDE_E_PARAM, "NULL argument or npts < 0");
    Plan* p = static_cast<Plan*>(plan);
    const int n = p->hp.n;
    const size_t N = (size_t)n * n;
    hipLaunchKernelGGL(k_price_adjoint, dim3((N + 255) / 256), dim3(256), 0, p->stream, n, p->hp.y_lo[0],
                       p->hp.y_lo[1], p->hp.h, p->pay.K, npts, spots, price_bar, v_bar);
    HIP_TRY(hipGetLastError());
    return LPIDE_OK;
}

int lpide_solve_range(void* plan, int32_t s0, int32_t s1, const double* v_in, double* v_out) {
    if (!plan || !v_in || !v_out) return fail(LPIDE_E_PARAM, "NULL argument");
    Plan* p = static_cast<Plan*>(plan);
    if (s0 < 0 || s1 < s0 || s1 > p->n_steps) return fail(LPIDE_E_PARAM, "step range out of bounds");
    Group* g = p->solo;
    g->lc.timer = p->time_mask ? p : nullptr;
    const double* ins[1] = {v_in};
    double* outs[1] = {v_out};
    int n1 = s1;
    return march_group(g, &n1, s0, ins, outs);
}

int lpide_solve_steps(void* plan, int32_t steps, double* v_out) {
    if (!plan || !v_out) return fail(LPIDE_E_PARAM, "NULL argument");
    Plan* p = static_cast<Plan*>(plan);
    if (steps < 0 || steps > p->n_steps) return fail(LPIDE_E_PARAM, "steps out of range");
    return march(p, steps, v_out);
}

int lpide_initial(void* plan, double* v_out) {
    if (!plan || !v_out) return fail(LPIDE_E_PARAM, "NULL argument");
    Plan* p = static_cast<Plan*>(plan);
    const size_t N = (size_t)p->hp.n * p->hp.n;
    hipLaunchKernelGGL(k_copy, dim3((N + 255) / 256), dim3(256), 0, p->stream, p->V0, v_out, N);
    HIP_TRY(hipGetLastError());
    return LPIDE_OK;
}

int lpide_apply_B(void* plan, const double* v, double* bv) {
    if (!plan || !v || !bv) return fail(LPIDE_E_PARAM, "NULL argument");
    if (v == bv) return fail(LPIDE_E_PARAM, "v and bv must not alias");
    Plan* p = static_cast<Plan*>(plan);
    if (!p->jumps) {
        HIP_TRY(hipMemsetAsync(bv, 0, sizeof(double) * (size_t)p->hp.n * p->hp.n, p->stream));
        return LPIDE_OK;
    }
    return dispatch_conv(p, v, bv, p->X);
}

int lpide_apply_B_noalloc(void* plan, const double* v, double* bv) {
    if (!plan || !v || !bv) return fail(LPIDE_E_PARAM, "NULL argument");
    if (v == bv) return fail(LPIDE_E_PARAM, "v and bv must not alias");
    Plan* p = static_cast<Plan*>(plan);
    const size_t N = (size_t)p->hp.n * p->hp.n;
    if (!p->jumps) {
        hipLaunchKernelGGL(k_zero, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, p->stream, bv, N);
        HIP_TRY(hipGetLastError());
        return LPIDE_OK;
    }
    const size_t need = (size_t)p->hp.n * (size_t)(p->L / 2 + 1) * sizeof(double2);
    if (need > (size_t)LPIDE_NOALLOC_SCRATCH_BYTES) {
        char buf[200];
        snprintf(buf, sizeof buf, "apply_B_noalloc: n = %d with transform side %d needs %zu bytes of scratch, above "
                 "the limit of %zu", p->hp.n, p->L, need, (size_t)LPIDE_NOALLOC_SCRATCH_BYTES);
        return fail(LPIDE_E_PARAM, buf);
    }
    double2* X = scratch_ptr(p->opts.device);
    if (!X) return fail(LPIDE_E_HIP, "apply_B_noalloc: scratch not set up on the plan's device");
    return dispatch_conv(p, v, bv, X);
}

int lpide_price(void* plan, const double* v, int32_t npts, const double* spots, double* price, double* delta) {
    if (!plan || !v) return fail(LPIDE_E_PARAM, "NULL argument");
    if (npts < 0) return fail(LPIDE_E_PARAM, "npts < 0");
    if (npts == 0) return LPIDE_OK;       // nothing is read or written
    if (!spots || !price) return fail(LPIDE_E_PARAM, "NULL argument");
    Plan* p = static_cast<Plan*>(plan);
    hipLaunchKernelGGL(k_price, dim3((npts + 127) / 128), dim3(128), 0, p->stream, v, p->hp.n, p->hp.y_lo[0],
                       p->hp.y_lo[1], p->hp.h, p->pay.K, npts, spots, price, delta);
    HIP_TRY(hipGetLastError());
    return LPIDE_OK;
}

int lpide_greeks(void* plan, const double* v, double* out) {
    if (!plan || !v || !out) return fail(LPIDE_E_PARAM, "NULL argument");
    Plan* p = static_cast<Plan*>(plan);
    const int n = p->hp.n;
    if (n < 4) return fail(LPIDE_E_PARAM, "the Greeks need n >= 4");
    const size_t N = (size_t)n * n;
    if (out < v + N && v < out + 5 * N) return fail(LPIDE_E_PARAM, "out must not alias v");
    hipLaunchKernelGGL(k_greeks, dim3((n + 127) / 128, n), dim3(128), 0, p->stream, v, n, p->hp.y_lo[0],
                       p->hp.y_lo[1], p->hp.h, p->pay.K, out);
    HIP_TRY(hipGetLastError());
    return LPIDE_OK;
}

int lpide_timing(void* plan, uint32_t class_mask) {
    if (!plan) return fail(LPIDE_E_PARAM, "NULL argument");
    Plan* p = static_cast<Plan*>(plan);
    int rc = harvest_times(p);
    if (rc) return rc;
    p->time_mask = class_mask & ((1u << LPIDE_KCLASSES) - 1u);
    for (int c = 0; c < LPIDE_KCLASSES; ++c) {
        p->k_launch[c] = 0;
        p->k_ms[c] = 0.0;
    }
    return LPIDE_OK;
}

int lpide_kernel_stats(void* plan, int64_t* launches, double* ms) {
    if (!plan || !launches || !ms) return fail(LPIDE_E_PARAM, "NULL argument");
    Plan* p = static_cast<Plan*>(plan);
    int rc = harvest_times(p);
    if (rc) return rc;
    for (int c = 0; c < LPIDE_KCLASSES; ++c) {
        launches[c] = p->k_launch[c];
        ms[c] = p->k_ms[c];
    }
    return LPIDE_OK;
}

void lpide_batch_opts_default(lpide_batch_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->use_graph = 1;
    o->slots = 32;
    o->stream = nullptr;
}

int lpide_batch_create(int32_t count, void* const* plans, const lpide_batch_opts* opts, void** out) {
    if (!plans || !out || count < 1) return fail(LPIDE_E_PARAM, "count must be >= 1 and plans, out not NULL");
    lpide_batch_opts o;
    if (opts) o = *opts; else lpide_batch_opts_default(&o);
    if (o.slots < 1 || o.slots > 256) return fail(LPIDE_E_PARAM, "slots must lie in [1, 256]");
    Batch* b = new Batch();
    b->caller = static_cast<hipStream_t>(o.stream);
    for (int i = 0; i < count; ++i) {
        if (!plans[i]) { destroy_batch(b); return fail(LPIDE_E_PARAM, "NULL plan in the batch"); }
        b->plans.push_back(static_cast<Plan*>(plans[i]));
    }
    // groups: plans with the same row-kernel size, jump switch, precision and SL order
    for (int i = 0; i < count; ++i) {
        Plan* p = b->plans[i];
        int q = -1;
        for (size_t g = 0; g < b->members.size(); ++g) {
            Plan* r = b->plans[b->members[g][0]];
            if (r->Lr == p->Lr && r->jumps == p->jumps && r->mixed == p->mixed && r->hp.sl_order == p->hp.sl_order)
                q = int(g);
        }
        if (q < 0) {
            b->members.push_back({});
            q = int(b->members.size()) - 1;
        }
        b->members[q].push_back(i);
    }
    for (auto& m : b->members) {
        hipStream_t s = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) { destroy_batch(b); return fail(LPIDE_E_HIP, std::string("hipStreamCreate: ") + hipGetErrorString(e)); }
        b->streams.push_back(s);
        std::vector<Plan*> ps;
        for (int i : m) ps.push_back(b->plans[i]);
        Group* g = nullptr;
        int rc = make_group(ps, s, &g);
        if (rc) { destroy_batch(b); return rc; }
        g->use_graph = o.use_graph != 0;
        g->slots = o.slots;
        b->groups.push_back(g);
    }
    for (size_t q = 0; q <= b->groups.size(); ++q) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            destroy_batch(b);
            return fail(LPIDE_E_HIP, "hipEventCreate failed");
        }
        b->events.push_back(e);
    }
    *out = b;
    return LPIDE_OK;
}

int lpide_plan(const lpide_grid* grid, const lpide_levy* levy, const lpide_payoff* payoff, double theta, int32_t M,
               const lpide_opts* opts, void** out) {
    return lpide_plan_create(grid, levy, payoff, theta, M, opts, out);
}

int lpide_destroy(void* plan) { return lpide_plan_destroy(plan); }

int lpide_plan_batch(int32_t count, const lpide_grid* grids, const lpide_levy* levys, const lpide_payoff* payoffs,
                     double theta, const int32_t* M, const lpide_opts* opts, void** out) {
    if (!grids || !levys || !payoffs || !M || !out || count < 1)
        return fail(LPIDE_E_PARAM, "count must be >= 1 and the arrays and out not NULL");
    std::vector<void*> plans;
    int rc = LPIDE_OK;
    for (int i = 0; i < count && rc == LPIDE_OK; ++i) {
        void* h = nullptr;
        rc = lpide_plan_create(&grids[i], &levys[i], &payoffs[i], theta, M[i], opts, &h);
        if (rc == LPIDE_OK) plans.push_back(h);
    }
    void* b = nullptr;
    if (rc == LPIDE_OK) {
        lpide_batch_opts bo;
        lpide_batch_opts_default(&bo);
        bo.stream = opts ? opts->stream : nullptr;
        rc = lpide_batch_create(count, plans.data(), &bo, &b);
    }
    if (rc != LPIDE_OK) {
        for (void* h : plans) destroy(static_cast<Plan*>(h));
        return rc;
    }
    static_cast<Batch*>(b)->owns_plans = true;
    *out = b;
    return LPIDE_OK;
}

int lpide_solve_batch(void* batch, double* const* v_out) { return lpide_batch_solve(batch, v_out); }

int lpide_batch_destroy(void* batch) {
    destroy_batch(static_cast<Batch*>(batch));
    return LPIDE_OK;
}

int lpide_batch_solve(void* batch, double* const* v_out) {
    if (!batch || !v_out) return fail(LPIDE_E_PARAM, "NULL argument");
    Batch* b = static_cast<Batch*>(batch);
    for (size_t i = 0; i < b->plans.size(); ++i)
        if (!v_out[i]) return fail(LPIDE_E_PARAM, "NULL output pointer in v_out");
    return batch_march(b, v_out, -1);
}

int lpide_batch_solve_steps(void* batch, int32_t steps, double* const* v_out) {
    if (!batch || steps < 0) return fail(LPIDE_E_PARAM, "NULL batch or steps < 0");
    return batch_march(static_cast<Batch*>(batch), v_out, steps);
}

// Autotuning: per group, time the march of the first trial_steps entries
// under candidate launch configurations and keep the fastest, in three passes:
// the radix schedule of the FFT kernels (4, 8 or 16 elements per thread), then
// the axis-1 line-solve chunking P_cols (P/2, P, 2P around the default), then
// hipGraph replay on/off with 16 or 32 step slots per host check.  Each
// candidate runs twice; the second run is timed, so graph capture and
// first-launch costs are not counted.
int lpide_batch_tune(void* batch, int32_t trial_steps) {
    if (!batch || trial_steps < 1) return fail(LPIDE_E_PARAM, "NULL batch or trial_steps < 1");
    Batch* b = static_cast<Batch*>(batch);
    // Candidates are timed on a window of trial_steps entries that starts
    // after the damped block and the first main steps (entry S0, from states
    // marched there once), so the window is made of the steady steps that
    // dominate a real march (explicit part from the previous step's equation,
    // B Y^0 by linearity, slots without the exiting kernels).
    constexpr int S0 = 8;
    for (size_t q = 0; q < b->groups.size(); ++q) {
        Group* g = b->groups[q];
        std::vector<int> ns, ns0;
        int nmax = 0;
        int s0 = S0;
        for (Plan* p : g->plans) s0 = std::min(s0, p->n_steps);
        std::vector<double*> start;
        struct Free {
            std::vector<double*>& v;
            ~Free() { for (double* x : v) (void)hipFree(x); }
        } free_start{start};
        for (Plan* p : g->plans) {
            ns0.push_back(s0);
            ns.push_back(std::min<int>(s0 + trial_steps, p->n_steps));
            nmax = std::max(nmax, p->hp.n);
            double* d = nullptr;
            HIP_TRY(hipMalloc(&d, sizeof(double) * (size_t)p->hp.n * p->hp.n));
            start.push_back(d);
        }
        {
            int rc = march_group(g, ns0.data(), 0, nullptr, start.data());
            if (rc) return rc;
        }
        auto trial = [&](double* out) -> int {
            double ms = 0.0;
            for (int rep = 0; rep < 2; ++rep) {
                HIP_TRY(hipStreamSynchronize(g->lc.stream));
                const auto t0 = std::chrono::steady_clock::now();
                int rc = march_group(g, ns.data(), s0, start.data(), nullptr);
                if (rc) return rc;
                ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            }
            *out = ms;
            return LPIDE_OK;
        };
        double best = 1e300, ms = 0.0;
        int rc = LPIDE_OK;
        // pass 1: radix schedule, one kernel class at a time from the default
        Schedule bs = g->lc.E_cols ? Schedule{g->lc.E_cols, g->lc.E_rinv, g->lc.E_lrows, g->lc.E_sl}
                                   : default_schedule(g->lc.L);
        g->use_graph = true;
        g->slots = 32;
        if ((rc = set_schedule(g, bs)) || (rc = trial(&best))) return rc;
        for (int cls = 0; cls < 4; ++cls)
            for (int E : {4, 8, 16}) {
                Schedule t = bs;
                int* f = cls == 0 ? &t.cols : cls == 1 ? &t.rinv : cls == 2 ? &t.lrows : &t.sl;
                if (*f == E || !e_supported(g->lc.L, E)) continue;
                *f = E;
                if ((rc = set_schedule(g, t)) || (rc = trial(&ms))) return rc;
                if (ms < best) { best = ms; bs = t; }
            }
        if ((rc = set_schedule(g, bs))) return rc;
        // pass 2: line-solve chunking
        const int P0 = default_P_cols(nmax);
        int bP = g->lc.P_cols;
        best = 1e300;
        for (int P : {P0 / 2, P0, 2 * P0}) {
            bool ok = 4 * P <= 1024;
            for (Plan* p : g->plans) ok = ok && P_cols_valid(p->hp.n, P);
            if (!ok) continue;
            if ((rc = set_P_cols(g, P)) || (rc = trial(&ms))) return rc;
            if (ms < best) { best = ms; bP = P; }
        }
        if ((rc = set_P_cols(g, bP))) return rc;
        // pass 3: graph replay and slots (a slot count is compared only when
        // the window spans at least two of its batches of slots)
        int bG = 1, bS = 32;
        best = 1e300;
        for (int G : {0, 1})
            for (int S : {16, 32}) {
                if (trial_steps < 2 * S && S != 32) continue;
                g->use_graph = G != 0;
                g->slots = S;
                if ((rc = trial(&ms))) return rc;
                if (ms < best) { best = ms; bG = G; bS = S; }
            }
        g->use_graph = bG != 0;
        g->slots = bS;
        g->tuned_ms = best;
    }
    b->tuned = true;
    return LPIDE_OK;
}

int lpide_batch_info(void* batch, int32_t* n_groups, lpide_group_info* groups, int32_t cap) {
    if (!batch || !n_groups) return fail(LPIDE_E_PARAM, "NULL argument");
    Batch* b = static_cast<Batch*>(batch);
    *n_groups = int32_t(b->groups.size());
    for (int q = 0; q < (int)b->groups.size() && groups && q < cap; ++q) {
        const Group* g = b->groups[q];
        lpide_group_info& gi = groups[q];
        std::memset(&gi, 0, sizeof gi);
        gi.n_plans = g->lc.np;
        gi.L = g->lc.L;
        gi.mixed = g->lc.mixed ? 1 : 0;
        gi.P_cols = g->lc.P_cols;
        gi.slots = g->slots;
        gi.use_graph = g->use_graph ? 1 : 0;
        gi.radix[0] = g->lc.E_cols;
        gi.radix[1] = g->lc.E_rinv;
        gi.radix[2] = g->lc.E_lrows;
        gi.radix[3] = g->lc.E_sl;
        gi.trial_ms = g->tuned_ms;
    }
    return LPIDE_OK;
}

const char* lpide_last_error(void) { return g_err.c_str(); }

}  // extern "C"
