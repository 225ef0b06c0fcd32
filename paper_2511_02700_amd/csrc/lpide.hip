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
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "host_plan.hpp"
#include "kernels.hpp"
#include "lpide.h"

using namespace lpide;

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(e_ == hipErrorOutOfMemory ? LPIDE_E_OOM : LPIDE_E_HIP,            \
                        std::string(#call) + ": " + hipGetErrorString(e_));               \
    } while (0)

// ---------------------------------------------------------------------------
// FFT correlation kernels
// ---------------------------------------------------------------------------
// Forward real FFT of pairs of rows (2p, 2p+1) of Y (n_rows x n_cols used,
// zero padded to L) into the transposed half spectra X[k2 * ldx + row].
template <int L>
__global__ __launch_bounds__(L / 8) void k_rows_fwd(const double* __restrict__ Y, int ldy, int n_rows,
                                                   int n_cols, double2* __restrict__ X, int ldx,
                                                   const double2* __restrict__ tw) {
    constexpr int T = L / 8;
    __shared__ double2 lds[L];
    const int np = (n_rows + 1) >> 1;
    const int p = xcd_remap(blockIdx.x, np);
    const int ra = 2 * p, rb = 2 * p + 1;
    const bool hasb = rb < n_rows;
    const double* ya = Y + (size_t)ra * ldy;
    const double* yb = Y + (size_t)(hasb ? rb : ra) * ldy;
    const int tid = threadIdx.x;
    double2 reg[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int idx = tid + e * T;
        double a = 0.0, b = 0.0;
        if (idx < n_cols) {
            a = ya[idx];
            b = hasb ? yb[idx] : 0.0;
        }
        reg[e] = make_double2(a, b);
    }
    fft_block<L, false>(reg, lds, tw);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 8; ++e) lds[tid + e * T] = reg[e];
    __syncthreads();
    // Z = FFT(a + i b): A_k = (Z_k + conj Z_{L-k}) / 2, B_k = (Z_k - conj Z_{L-k}) / (2i)
    for (int k = tid; k <= L / 2; k += T) {
        const double2 z = lds[k], w = lds[(L - k) & (L - 1)];
        const double2 A = make_double2(0.5 * (z.x + w.x), 0.5 * (z.y - w.y));
        const double2 B = make_double2(0.5 * (z.y + w.y), -0.5 * (z.x - w.x));
        double2* xk = X + (size_t)k * ldx;
        xk[ra] = A;
        if (hasb) xk[rb] = B;
    }
}

// Column pass.  MODE 0: X[col] <- first n_out of IFFT(FFT(X[col], zero padded
// from n_in) * spec[col]).  MODE 1 (plan time): spec_out[col] = conj(FFT(X[col])) * scale.
template <int L, int MODE>
__global__ __launch_bounds__(L / 8) void k_cols(double2* __restrict__ X, int ldx, int n_in, int n_out,
                                               const double2* __restrict__ spec,
                                               double2* __restrict__ spec_out, double scale,
                                               const double2* __restrict__ tw) {
    constexpr int T = L / 8;
    __shared__ double2 lds[L];
    const int col = blockIdx.x;
    const int tid = threadIdx.x;
    double2* xc = X + (size_t)col * ldx;
    double2 reg[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int idx = tid + e * T;
        reg[e] = idx < n_in ? xc[idx] : make_double2(0.0, 0.0);
    }
    fft_block<L, false>(reg, lds, tw);
    if constexpr (MODE == 1) {
        double2* so = spec_out + (size_t)col * L;
#pragma unroll
        for (int e = 0; e < 8; ++e) so[tid + e * T] = make_double2(reg[e].x * scale, -reg[e].y * scale);
        return;
    } else {
        const double2* sc = spec + (size_t)col * L;
#pragma unroll
        for (int e = 0; e < 8; ++e) reg[e] = cmul(reg[e], sc[tid + e * T]);
        fft_block<L, true>(reg, lds, tw);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int idx = tid + e * T;
            if (idx < n_out) xc[idx] = reg[e];
        }
    }
}

// Inverse real FFT of row pairs from the transposed half spectra; keeps the
// first n columns.  EPI 0: out = result.  EPI 1: affine stencil epilogue.
template <int L, int EPI>
__global__ __launch_bounds__(L / 8) void k_rows_inv(const double2* __restrict__ X, int ldx, int n,
                                                   double* __restrict__ out, AffineArgs aa,
                                                   const double2* __restrict__ tw) {
    constexpr int T = L / 8;
    __shared__ double2 lds[L];
    const int np = (n + 1) >> 1;
    const int p = xcd_remap(blockIdx.x, np);
    const int ra = 2 * p, rb = 2 * p + 1;
    const bool hasb = rb < n;
    const int tid = threadIdx.x;
    double2 reg[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int idx = tid + e * T;
        const bool lo = idx <= L / 2;
        const int k = lo ? idx : L - idx;
        const double2* xk = X + (size_t)k * ldx;
        double2 ha = xk[ra];
        double2 hb = hasb ? xk[rb] : make_double2(0.0, 0.0);
        if (k == 0 || k == L / 2) { ha.y = 0.0; hb.y = 0.0; }
        // Z_k = A_k + i B_k, with A_{L-k} = conj A_k, B_{L-k} = conj B_k
        reg[e] = lo ? make_double2(ha.x - hb.y, ha.y + hb.x) : make_double2(ha.x + hb.y, hb.x - ha.y);
    }
    fft_block<L, true>(reg, lds, tw);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int j = tid + e * T;
        if (j >= n) continue;
        if constexpr (EPI == 0) {
            out[(size_t)ra * n + j] = reg[e].x;
            if (hasb) out[(size_t)rb * n + j] = reg[e].y;
        } else {
            {
                const size_t o = (size_t)ra * n + j;
                const double u = aa.U[o];
                const double d = apply_D(aa.U, aa.st, ra, j, u);
                aa.out[o] = aa.P0[o] + aa.c * (d + reg[e].x - aa.r_omega * u) + aa.c0 * u;
            }
            if (hasb) {
                const size_t o = (size_t)rb * n + j;
                const double u = aa.U[o];
                const double d = apply_D(aa.U, aa.st, rb, j, u);
                aa.out[o] = aa.P0[o] + aa.c * (d + reg[e].y - aa.r_omega * u) + aa.c0 * u;
            }
        }
    }
}

// Affine stencil form without the correlation (zero Levy measure).
__global__ void k_affine_noB(AffineArgs aa) {
    const int n = aa.st.n;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= n) return;
    const size_t o = (size_t)i * n + j;
    const double u = aa.U[o];
    const double d = apply_D(aa.U, aa.st, i, j, u);
    aa.out[o] = aa.P0[o] + aa.c * (d - aa.r_omega * u) + aa.c0 * u;
}

// ---------------------------------------------------------------------------
// Line solves T x = r with constant factors (forward multipliers fl, backward
// scales bu and couplings bc):  y_i = r_i + fl_i y_{i-1};  x_i = bu_i y_i + bc_i x_{i+1}.
// Each line is cut into P chunks of m consecutive elements, one per thread.
// A chunk solves its recurrence locally from a zero carry, the carries between
// chunks follow from a scan of the chunks' affine maps y_out = G y_in + B, and
// a fix-up adds the carried-in value times the running product of the
// multipliers.  Exact up to rounding (no truncation of the coupling).
// ---------------------------------------------------------------------------
constexpr int LINE_MM = 32;   // max chunk length held in registers

// Exclusive scan of affine maps over t = 0..P-1 within groups of P threads
// (group g uses slots [g*P, g*P+P) of buf, 2 * groups * P entries).  Returns the
// carried-in value y_in(t) = (M_{t-1} o ... o M_0)(0).
__device__ __forceinline__ double scan_affine(double G, double B, int g, int t, int P, double2* buf) {
    double2* cur = buf;
    double2* nxt = buf + blockDim.x;
    const int s = g * P + t;
    cur[s] = make_double2(G, B);
    __syncthreads();
    for (int d = 1; d < P; d <<= 1) {
        double2 me = cur[s];
        if (t >= d) {
            const double2 pr = cur[s - d];
            me = make_double2(me.x * pr.x, me.x * pr.y + me.y);
        }
        nxt[s] = me;
        __syncthreads();
        double2* tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    const double carry = t > 0 ? cur[s - 1].y : 0.0;
    __syncthreads();
    return carry;
}

// Solve one chunk (elements idx(k), k < m, of a line whose factor index is
// i0 + k) given its carries.  x[] holds r on entry and the solution on exit.
__device__ __forceinline__ void chunk_solve(double (&x)[LINE_MM], int i0, int m, int g, int t, int P,
                                            const double* __restrict__ fl, const double* __restrict__ bu,
                                            const double* __restrict__ bc, double2* buf) {
    // forward: local pass from a zero carry
    double y = 0.0, G = 1.0;
#pragma unroll
    for (int k = 0; k < LINE_MM; ++k) {
        if (k < m) {
            const double f = fl[i0 + k];
            y = x[k] + f * y;
            G *= f;
            x[k] = y;
        }
    }
    const double yin = scan_affine(G, y, g, t, P, buf);
    double gp = 1.0;
#pragma unroll
    for (int k = 0; k < LINE_MM; ++k) {
        if (k < m) {
            gp *= fl[i0 + k];
            x[k] += gp * yin;
        }
    }
    // backward: local pass from a zero carry, scanned in reverse chunk order
    double xh = 0.0, H = 1.0;
#pragma unroll
    for (int k = LINE_MM - 1; k >= 0; --k) {
        if (k < m) {
            const double c = bc[i0 + k];
            xh = bu[i0 + k] * x[k] + c * xh;
            H *= c;
            x[k] = xh;
        }
    }
    const double xin = scan_affine(H, xh, g, P - 1 - t, P, buf);
    double hp = 1.0;
#pragma unroll
    for (int k = LINE_MM - 1; k >= 0; --k) {
        if (k < m) {
            hp *= bc[i0 + k];
            x[k] += hp * xin;
        }
    }
}

// Axis 2 (rows, contiguous): one row per block of 256 threads, staged through
// LDS with one padding slot per chunk so the chunk reads avoid bank conflicts.
__global__ __launch_bounds__(256) void k_line_rows(double* __restrict__ U, int n, const double* __restrict__ fl,
                                                  const double* __restrict__ bu,
                                                  const double* __restrict__ bc) {
    extern __shared__ double smem[];
    const int P = blockDim.x;
    const int m = (n + P - 1) / P;
    double* row = smem;                                   // n + P slots
    double2* buf = reinterpret_cast<double2*>(smem + ((n + P + 1) & ~1));   // 2P entries
    const int r = xcd_remap(blockIdx.x, gridDim.x);
    double* u = U + (size_t)r * n;
    const int tid = threadIdx.x;
    for (int i = tid; i < n; i += P) row[i + i / m] = u[i];
    __syncthreads();
    const int s = tid * m;
    const int cnt = max(0, min(m, n - s));
    double x[LINE_MM];
#pragma unroll
    for (int k = 0; k < LINE_MM; ++k) x[k] = k < cnt ? row[s + k + tid] : 0.0;
    chunk_solve(x, s, cnt, 0, tid, P, fl, bu, bc, buf);
#pragma unroll
    for (int k = 0; k < LINE_MM; ++k)
        if (k < cnt) row[s + k + tid] = x[k];
    __syncthreads();
    for (int i = tid; i < n; i += P) u[i] = row[i + i / m];
}

// Axis 1 (columns, stride n): a block covers 16 adjacent columns x P chunks
// (thread = column + 16 * chunk, so a wave reads 4 rows x 128 contiguous bytes).
// UPDATE: Y += x and the stopping-rule maximum max |x| / max(1, |Y_new|).
template <bool UPDATE>
__global__ __launch_bounds__(1024) void k_line_cols(double* __restrict__ U, int n, int P,
                                                   const double* __restrict__ fl,
                                                   const double* __restrict__ bu,
                                                   const double* __restrict__ bc, double* __restrict__ Y,
                                                   unsigned long long* __restrict__ err) {
    extern __shared__ double2 sbuf[];
    const int c = threadIdx.x & 15, t = threadIdx.x >> 4;
    const int col = blockIdx.x * 16 + c;
    const bool valid = col < n;
    const int m = (n + P - 1) / P;
    const int s = t * m;
    const int cnt = valid ? max(0, min(m, n - s)) : 0;
    double x[LINE_MM];
#pragma unroll
    for (int k = 0; k < LINE_MM; ++k) x[k] = k < cnt ? U[(size_t)(s + k) * n + col] : 0.0;
    chunk_solve(x, s, cnt, c, t, P, fl, bu, bc, sbuf);
    // chunk_solve groups threads by g = c with slots g*P + t: consistent for all threads
    if constexpr (!UPDATE) {
#pragma unroll
        for (int k = 0; k < LINE_MM; ++k)
            if (k < cnt) U[(size_t)(s + k) * n + col] = x[k];
    } else {
        double emax = 0.0;
#pragma unroll
        for (int k = 0; k < LINE_MM; ++k) {
            if (k < cnt) {
                const size_t o = (size_t)(s + k) * n + col;
                const double yn = Y[o] + x[k];
                Y[o] = yn;
                const double e = fabs(x[k]) / fmax(1.0, fabs(yn));
                emax = (e > emax || e != e) ? e : emax;
            }
        }
        // wave reduction, then one atomic per wave (bit patterns of non-negative
        // doubles order like the values; NaN sorts above +inf)
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(emax, off);
            emax = (o > emax || o != o) ? o : emax;
        }
        if ((threadIdx.x & 63) == 0) atomicMax(err, (unsigned long long)__double_as_longlong(emax));
    }
}

// ---------------------------------------------------------------------------
// Semi-Lagrangian gather W = (T_1 (x) T_2) E with per-node stencil starts and
// weights, fused with the extrapolated start Y0 = sum_k c_k H_k.
// ---------------------------------------------------------------------------
template <int P>
__global__ void k_sl_extrap(const double* __restrict__ E, double* __restrict__ W, int n,
                            const int* __restrict__ s1, const double* __restrict__ w1,
                            const int* __restrict__ s2, const double* __restrict__ w2,
                            const double* __restrict__ H0, const double* __restrict__ H1,
                            const double* __restrict__ H2, const double* __restrict__ H3, double c0,
                            double c1, double c2, double c3, double* __restrict__ Y0) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= n) return;
    const int a0 = s1[i], b0 = s2[j];
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        const double* er = E + (size_t)(a0 + a) * n + b0;
        double ra = 0.0;
#pragma unroll
        for (int b = 0; b <= P; ++b) ra += w2[j * (P + 1) + b] * er[b];
        acc += w1[i * (P + 1) + a] * ra;
    }
    const size_t o = (size_t)i * n + j;
    W[o] = acc;
    double y = c0 * H0[o];
    if (H1) y += c1 * H1[o];
    if (H2) y += c2 * H2[o];
    if (H3) y += c3 * H3[o];
    Y0[o] = y;
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

__global__ void k_copy(const double* __restrict__ a, double* __restrict__ b, size_t cnt) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) b[i] = a[i];
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
namespace {

struct StepSet {
    double theta = 0, dt = 0;
    double *fl1 = nullptr, *bu1 = nullptr, *bc1 = nullptr, *fl2 = nullptr, *bu2 = nullptr, *bc2 = nullptr;
    int *s1 = nullptr, *s2 = nullptr;
    double *w1 = nullptr, *w2 = nullptr;
};

struct Plan {
    HostPlan hp;
    lpide_opts opts{};
    lpide_payoff pay{};
    double theta = 0.5;
    int N_t = 1;
    hipStream_t stream = nullptr;
    int L = 0;
    bool jumps = false;
    std::vector<void*> allocs;
    int64_t bytes = 0;
    double2* tw = nullptr;
    double2* spec = nullptr;
    double2* X = nullptr;
    double* V0 = nullptr;
    double* pool[6] = {};
    double* Wb = nullptr;
    double* Rb = nullptr;
    unsigned long long* err_d = nullptr;
    double* err_h = nullptr;
    std::vector<StepSet> sets;
    std::vector<int> step_set;
    std::vector<std::pair<double, double>> steps;
    int P_cols = 16;
    // kernel timing (HIP events on the plan's stream around each timed launch)
    uint32_t time_mask = 0;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, size_t>> ev_recs;   // (kernel class, index of the start event)
    size_t ev_used = 0;
    int64_t k_launch[LPIDE_KCLASSES] = {};
    double k_ms[LPIDE_KCLASSES] = {};
    // statistics of the last solve
    int64_t total_iters = 0;
    int max_step_iters = 0, last_step_iters = 0;
    double last_inc = 0;
};

// Event pair around one launch of kernel class cls (no-op unless timed).
struct KTime {
    Plan* p;
    int cls;
    bool on;
    KTime(Plan* pl, int c);
    ~KTime();
};

hipEvent_t next_event(Plan* p) {
    if (p->ev_used == p->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        p->ev_pool.push_back(e);
    }
    return p->ev_pool[p->ev_used++];
}

KTime::KTime(Plan* pl, int c) : p(pl), cls(c), on((pl->time_mask >> c) & 1u) {
    if (!on) return;
    const size_t idx = p->ev_used;
    hipEvent_t a = next_event(p), b = next_event(p);
    if (!a || !b) { on = false; return; }
    (void)hipEventRecord(a, p->stream);
    p->ev_recs.emplace_back(cls, idx);
}
KTime::~KTime() {
    if (on) (void)hipEventRecord(p->ev_pool[p->ev_recs.back().second + 1], p->stream);
}

// Fold recorded event pairs into the per-class totals (synchronises the stream).
int harvest_times(Plan* p) {
    if (p->ev_recs.empty()) return LPIDE_OK;
    HIP_TRY(hipStreamSynchronize(p->stream));
    for (auto& r : p->ev_recs) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p->ev_pool[r.second], p->ev_pool[r.second + 1]));
        p->k_launch[r.first] += 1;
        p->k_ms[r.first] += ms;
    }
    p->ev_recs.clear();
    p->ev_used = 0;
    return LPIDE_OK;
}

template <typename Tp>
int dalloc(Plan* p, Tp** out, size_t count) {
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, count * sizeof(Tp));
    if (e != hipSuccess) return fail(LPIDE_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    p->allocs.push_back(d);
    p->bytes += int64_t(count * sizeof(Tp));
    *out = static_cast<Tp*>(d);
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

template <int L>
void launch_conv(Plan* p, const double* Y, int epi, const AffineArgs& aa, double* out) {
    const int n = p->hp.n, np = (n + 1) / 2;
    {
        KTime t(p, LPIDE_K_ROWS_FWD);
        hipLaunchKernelGGL((k_rows_fwd<L>), dim3(np), dim3(L / 8), 0, p->stream, Y, n, n, n, p->X, n, p->tw);
    }
    {
        KTime t(p, LPIDE_K_COLS);
        hipLaunchKernelGGL((k_cols<L, 0>), dim3(L / 2 + 1), dim3(L / 8), 0, p->stream, p->X, n, n, n, p->spec,
                           (double2*)nullptr, 0.0, p->tw);
    }
    KTime t(p, LPIDE_K_ROWS_INV);
    if (epi == 0)
        hipLaunchKernelGGL((k_rows_inv<L, 0>), dim3(np), dim3(L / 8), 0, p->stream, p->X, n, n, out, aa, p->tw);
    else
        hipLaunchKernelGGL((k_rows_inv<L, 1>), dim3(np), dim3(L / 8), 0, p->stream, p->X, n, n, out, aa, p->tw);
}

template <int L>
void launch_spectrum(Plan* p, const double* G, double2* Xfull) {
    const double scale = 1.0 / (double(L) * double(L));
    hipLaunchKernelGGL((k_rows_fwd<L>), dim3(L / 2), dim3(L / 8), 0, p->stream, G, L, L, L, Xfull, L, p->tw);
    hipLaunchKernelGGL((k_cols<L, 1>), dim3(L / 2 + 1), dim3(L / 8), 0, p->stream, Xfull, L, L, L,
                       (const double2*)nullptr, p->spec, scale, p->tw);
}

int dispatch_conv(Plan* p, const double* Y, int epi, const AffineArgs& aa, double* out) {
    switch (p->L) {
        case 64: launch_conv<64>(p, Y, epi, aa, out); break;
        case 128: launch_conv<128>(p, Y, epi, aa, out); break;
        case 256: launch_conv<256>(p, Y, epi, aa, out); break;
        case 512: launch_conv<512>(p, Y, epi, aa, out); break;
        case 1024: launch_conv<1024>(p, Y, epi, aa, out); break;
        case 2048: launch_conv<2048>(p, Y, epi, aa, out); break;
        case 4096: launch_conv<4096>(p, Y, epi, aa, out); break;
        case 8192: launch_conv<8192>(p, Y, epi, aa, out); break;
        default: return fail(LPIDE_E_PARAM, "unsupported FFT side");
    }
    HIP_TRY(hipGetLastError());
    return LPIDE_OK;
}

int dispatch_spectrum(Plan* p, const double* G, double2* Xfull) {
    switch (p->L) {
        case 64: launch_spectrum<64>(p, G, Xfull); break;
        case 128: launch_spectrum<128>(p, G, Xfull); break;
        case 256: launch_spectrum<256>(p, G, Xfull); break;
        case 512: launch_spectrum<512>(p, G, Xfull); break;
        case 1024: launch_spectrum<1024>(p, G, Xfull); break;
        case 2048: launch_spectrum<2048>(p, G, Xfull); break;
        case 4096: launch_spectrum<4096>(p, G, Xfull); break;
        case 8192: launch_spectrum<8192>(p, G, Xfull); break;
        default: return fail(LPIDE_E_PARAM, "unsupported FFT side");
    }
    HIP_TRY(hipGetLastError());
    return LPIDE_OK;
}

// P (chunks per column) so that a chunk holds at most LINE_MM elements.
// At least 4 chunks, so a block has at least one full wave of 64 lanes.
int cols_chunks(int n) {
    int P = 4;
    while ((n + P - 1) / P > LINE_MM) P *= 2;
    return P;
}

// (B Y) with the chosen epilogue; for a zero Levy measure only the stencil form.
int apply_affine(Plan* p, const double* P0, const double* U, double* out, double c, double c0) {
    AffineArgs aa;
    aa.P0 = P0;
    aa.U = U;
    aa.out = out;
    aa.c = c;
    aa.c0 = c0;
    aa.r_omega = p->hp.r_omega;
    aa.st = stencil_of(p);
    if (p->jumps) return dispatch_conv(p, U, 1, aa, out);
    const int n = p->hp.n;
    KTime t(p, LPIDE_K_ROWS_INV);
    hipLaunchKernelGGL(k_affine_noB, dim3((n + 255) / 256, n), dim3(256), 0, p->stream, aa);
    HIP_TRY(hipGetLastError());
    return LPIDE_OK;
}

int line_solves(Plan* p, const StepSet& s, double* R, double* Y) {
    const int n = p->hp.n;
    const size_t rows_lds = sizeof(double) * (size_t)(((n + 256 + 1) & ~1)) + sizeof(double2) * 512;
    {
        KTime t(p, LPIDE_K_LINE_ROWS);
        hipLaunchKernelGGL(k_line_rows, dim3(n), dim3(256), rows_lds, p->stream, R, n, s.fl2, s.bu2, s.bc2);
    }
    const int P = p->P_cols;
    KTime t(p, LPIDE_K_LINE_COLS);
    hipLaunchKernelGGL((k_line_cols<true>), dim3((n + 15) / 16), dim3(16 * P), sizeof(double2) * 2 * 16 * P,
                       p->stream, R, n, P, s.fl1, s.bu1, s.bc1, Y, p->err_d);
    HIP_TRY(hipGetLastError());
    return LPIDE_OK;
}

int sl_extrap(Plan* p, const StepSet& s, const double* E, double* W, const double* const H[4], const double c[4],
              double* Y0) {
    const int n = p->hp.n;
    dim3 grid((n + 127) / 128, n);
    KTime t(p, LPIDE_K_SL);
    if (p->hp.sl_order == 1)
        hipLaunchKernelGGL((k_sl_extrap<1>), grid, dim3(128), 0, p->stream, E, W, n, s.s1, s.w1, s.s2, s.w2, H[0],
                           H[1], H[2], H[3], c[0], c[1], c[2], c[3], Y0);
    else
        hipLaunchKernelGGL((k_sl_extrap<3>), grid, dim3(128), 0, p->stream, E, W, n, s.s1, s.w1, s.s2, s.w2, H[0],
                           H[1], H[2], H[3], c[0], c[1], c[2], c[3], Y0);
    HIP_TRY(hipGetLastError());
    return LPIDE_OK;
}

void destroy(Plan* p) {
    if (!p) return;
    (void)hipStreamSynchronize(p->stream);
    for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
    for (void* a : p->allocs) (void)hipFree(a);
    if (p->err_h) (void)hipHostFree(p->err_h);
    delete p;
}

// March the first `count` entries of the step list from V^0; result in v_out.
int march(Plan* p, int count, double* v_out) {
    const int n = p->hp.n;
    const size_t N = (size_t)n * n;
    p->total_iters = 0;
    p->max_step_iters = 0;
    p->last_step_iters = 0;
    p->last_inc = 0;
    // buffer roles: hist[0..hc) newest first; vsub = state inside the damped block
    int hist[4], hc = 0, vsub = -1;
    auto in_use = [&](int b) {
        for (int k = 0; k < hc; ++k)
            if (hist[k] == b) return true;
        return b == vsub;
    };
    auto grab = [&]() {
        for (int b = 0; b < 6; ++b)
            if (!in_use(b)) return b;
        return -1;
    };
    hipLaunchKernelGGL(k_copy, dim3((N + 255) / 256), dim3(256), 0, p->stream, p->V0, p->pool[0], N);
    hist[0] = 0;
    hc = 1;
    const int n_sub = p->opts.damping ? 4 : 1;
    for (int s = 0; s < count; ++s) {
        const StepSet& ss = p->sets[p->step_set[s]];
        const double th = ss.theta, dt = ss.dt;
        const bool damped = p->opts.damping && s < n_sub;
        const int start = (damped && vsub >= 0) ? vsub : hist[0];
        const double* Vs = p->pool[start];
        // explicit part into Rb (skipped for theta = 1)
        const double* E = Vs;
        if (th < 1.0) {
            int rc = apply_affine(p, Vs, Vs, p->Rb, dt * (1.0 - th), 0.0);
            if (rc) return rc;
            E = p->Rb;
        }
        // starting value
        const int yb = grab();
        if (yb < 0) return fail(LPIDE_E_PARAM, "internal: no free grid buffer");
        double* Y = p->pool[yb];
        const double* H[4] = {Vs, nullptr, nullptr, nullptr};
        double c[4] = {1.0, 0.0, 0.0, 0.0};
        if (!damped) {
            for (int k = 0; k < hc; ++k) H[k] = p->pool[hist[k]];
            if (hc == 2) { c[0] = 2; c[1] = -1; }
            else if (hc == 3) { c[0] = 3; c[1] = -3; c[2] = 1; }
            else if (hc >= 4) { c[0] = 4; c[1] = -6; c[2] = 4; c[3] = -1; }
        }
        int rc = sl_extrap(p, ss, E, p->Wb, H, c, Y);
        if (rc) return rc;
        // fixed-point iteration
        int k = 0;
        double errv = 0;
        for (;;) {
            ++k;
            hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, p->stream, p->err_d);
            rc = apply_affine(p, p->Wb, Y, p->Rb, dt * th, -1.0);
            if (rc) return rc;
            rc = line_solves(p, ss, p->Rb, Y);
            if (rc) return rc;
            HIP_TRY(hipMemcpyAsync(p->err_h, p->err_d, sizeof(double), hipMemcpyDeviceToHost, p->stream));
            HIP_TRY(hipStreamSynchronize(p->stream));
            errv = *p->err_h;
            if (!std::isfinite(errv)) {
                return fail(LPIDE_E_NAN, "non-finite fixed-point increment in step " + std::to_string(s));
            }
            if (errv < p->opts.tol) break;
            if (k >= p->opts.max_iter) {
                char buf[160];
                snprintf(buf, sizeof buf, "fixed point not converged in step %d after %d iterations (increment %.3e)",
                         s, k, errv);
                return fail(LPIDE_E_NOCONV, buf);
            }
        }
        p->total_iters += k;
        p->max_step_iters = std::max(p->max_step_iters, k);
        p->last_step_iters = k;
        p->last_inc = errv;
        // bookkeeping of the history (main steps) and the damped sub-step state
        if (damped && s < n_sub - 1) {
            vsub = yb;
        } else {
            vsub = -1;
            for (int q = std::min(hc, 3); q > 0; --q) hist[q] = hist[q - 1];
            hist[0] = yb;
            hc = std::min(hc + 1, 4);
        }
    }
    const int last = (vsub >= 0) ? vsub : hist[0];
    hipLaunchKernelGGL(k_copy, dim3((N + 255) / 256), dim3(256), 0, p->stream, p->pool[last], v_out, N);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(p->stream));
    return LPIDE_OK;
}

}  // namespace

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
    if (o.precision != LPIDE_FP64) return fail(LPIDE_E_PARAM, "precision mode not available");
    Plan* p = new Plan();
    std::string err;
    if (!build_host_plan(*grid, *levy, p->hp, err)) { delete p; return fail(LPIDE_E_PARAM, err); }
    std::vector<double> v0;
    if (!initial_values(p->hp, *payoff, v0, err)) { delete p; return fail(LPIDE_E_PARAM, err); }
    p->opts = o;
    p->pay = *payoff;
    p->theta = theta;
    p->N_t = M;
    p->stream = static_cast<hipStream_t>(o.stream);
    p->jumps = p->hp.nts.jumps;
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
    const int n = p->hp.n;
    const size_t N = (size_t)n * n;
    if ((rc = upload(p, &p->V0, v0))) return bail(rc);
    for (int b = 0; b < 6; ++b)
        if ((rc = dalloc(p, &p->pool[b], N))) return bail(rc);
    if ((rc = dalloc(p, &p->Wb, N))) return bail(rc);
    if ((rc = dalloc(p, &p->Rb, N))) return bail(rc);
    if ((rc = dalloc(p, &p->err_d, 1))) return bail(rc);
    if (hipHostMalloc((void**)&p->err_h, sizeof(double), hipHostMallocDefault) != hipSuccess)
        return bail(fail(LPIDE_E_OOM, "hipHostMalloc failed"));
    p->P_cols = cols_chunks(n);
    if (16 * p->P_cols > 1024) return bail(fail(LPIDE_E_PARAM, "n too large for the column line solve"));
    // step list and its distinct (theta, dt) sets
    p->steps = step_list(theta, payoff->T, M, o.damping != 0);
    for (auto& st : p->steps) {
        int id = -1;
        for (size_t q = 0; q < p->sets.size(); ++q)
            if (p->sets[q].theta == st.first && p->sets[q].dt == st.second) id = int(q);
        if (id < 0) {
            StepSet ss;
            ss.theta = st.first;
            ss.dt = st.second;
            const double c = ss.dt * ss.theta;
            std::vector<double> fl, bu, bc;
            line_factors(n, p->hp.h, p->hp.a[0], p->hp.r_omega, c, fl, bu, bc);
            if ((rc = upload(p, &ss.fl1, fl)) || (rc = upload(p, &ss.bu1, bu)) || (rc = upload(p, &ss.bc1, bc)))
                return bail(rc);
            line_factors(n, p->hp.h, p->hp.a[2], p->hp.r_omega, c, fl, bu, bc);
            if ((rc = upload(p, &ss.fl2, fl)) || (rc = upload(p, &ss.bu2, bu)) || (rc = upload(p, &ss.bc2, bc)))
                return bail(rc);
            std::vector<int32_t> st1, st2;
            std::vector<double> w1, w2;
            sl_weights(n, p->hp.kappa[0] * ss.dt / p->hp.h, p->hp.sl_order, st1, w1);
            sl_weights(n, p->hp.kappa[1] * ss.dt / p->hp.h, p->hp.sl_order, st2, w2);
            if ((rc = upload(p, &ss.s1, st1)) || (rc = upload(p, &ss.s2, st2)) || (rc = upload(p, &ss.w1, w1)) ||
                (rc = upload(p, &ss.w2, w2)))
                return bail(rc);
            p->sets.push_back(ss);
            id = int(p->sets.size()) - 1;
        }
        p->step_set.push_back(id);
    }
    // kernel spectrum conj(FFT(K placed at d mod L)) / L^2
    if (p->jumps) {
        const int L = p->L;
        std::vector<double2> tw(L);
        for (int q = 0; q < L; ++q) {
            // exp(-2 pi i q / L) with the angle reduced to the first octant for accuracy
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
    }
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
    info->n_steps = int32_t(p->steps.size());
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
    return LPIDE_OK;
}

int lpide_solve(void* plan, double* v_out) {
    if (!plan || !v_out) return fail(LPIDE_E_PARAM, "NULL argument");
    Plan* p = static_cast<Plan*>(plan);
    return march(p, int(p->steps.size()), v_out);
}

int lpide_solve_steps(void* plan, int32_t steps, double* v_out) {
    if (!plan || !v_out) return fail(LPIDE_E_PARAM, "NULL argument");
    Plan* p = static_cast<Plan*>(plan);
    if (steps < 0 || steps > int(p->steps.size())) return fail(LPIDE_E_PARAM, "steps out of range");
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
    AffineArgs aa{};
    return dispatch_conv(p, v, 0, aa, bv);
}

int lpide_price(void* plan, const double* v, int32_t npts, const double* spots, double* price, double* delta) {
    if (!plan || !v || !spots || !price) return fail(LPIDE_E_PARAM, "NULL argument");
    if (npts < 0) return fail(LPIDE_E_PARAM, "npts < 0");
    Plan* p = static_cast<Plan*>(plan);
    if (npts == 0) return LPIDE_OK;
    hipLaunchKernelGGL(k_price, dim3((npts + 127) / 128), dim3(128), 0, p->stream, v, p->hp.n, p->hp.y_lo[0],
                       p->hp.y_lo[1], p->hp.h, p->pay.K, npts, spots, price, delta);
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

const char* lpide_last_error(void) { return g_err.c_str(); }

}  // extern "C"
