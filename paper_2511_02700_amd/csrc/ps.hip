// The price-space plan (Sec. 3.2, Sec. 3.3, Sec. 4 settings): creation, the
// march and its C ABI.
//
// The host enqueues the steps of a march in batches of 16 without waiting:
// each step is the explicit part (from the previous step's implicit equation,
// or by the correlation), the semi-Lagrangian gather with the extrapolated
// start value, a predicted number of fixed-point iterations and an
// end-of-step kernel.  The iteration kernels read the stopping rule of the
// iteration before them on the device and return at once after convergence,
// so the host reads the control block only once per batch.  A step that has
// not converged after its predicted iterations sets the failure flag, which
// turns the rest of the batch into no-ops; the host then adds iterations to
// that step one at a time and resumes the batch after it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "lpide.h"
#include "ps_host.hpp"
#include "ps_big.hpp"
#include "ps_plan.hpp"

static_assert(lpide::LINE_MM <= lpide::kLinePad, "factor arrays need a tail of at least the chunk capacity");

namespace lpide {
namespace detail {
int fail(int code, const std::string& msg);
}
namespace ps {
namespace {

using detail::fail;

constexpr int POOLN = 6;        // 4 history grids, the current grid, the iterate

// Transform sides of the price-space correlation: powers of two up to 8192,
// sides 2^m p with odd factor p = 3, 5, 7 or 9 (largest prime factor at most
// 7, Sec. 4) that one workgroup's LDS holds, and the two-level sides 12288,
// 16384 and 24576 = (3, 4, 6) x 4096.
constexpr int kPsSides[] = {64,   128,  256,  512,  640,  768,  896,  1024, 1152,  1280,  1536,  1792, 2048,
                            2304, 2560, 3072, 3584, 4096, 4608, 5120, 6144, 7168, 8192, 12288, 16384, 24576};
constexpr int kPsAutoSides[] = {64,   128,  256,  512,  640,  896,  1024, 1152, 1280,  1536,  1792,  2048, 2304,
                                2560, 3072, 3584, 4096, 4608, 5120, 6144, 7168, 8192, 12288, 16384, 24576};

bool ps_side_supported(int L) {
    for (int v : kPsSides)
        if (v == L) return true;
    return false;
}

int ps_side_at_least(int need) {
    for (int v : kPsAutoSides)
        if (v >= need) return v;
    return 0;
}
constexpr int BATCH = 16;       // steps enqueued between host checks

struct Kind {
    double theta = 0.0, dt = 0.0;
    PsStepK sk{};
    int *s1 = nullptr, *s2 = nullptr;
    double *w1 = nullptr, *w2 = nullptr;
};

struct PsPlan {
    PsHost hp;
    lpide_opts opts{};
    lpide_payoff pay{};
    double theta = 0.5;
    int N_t = 1;
    hipStream_t stream = nullptr;
    int L = 0;
    bool jumps = false;
    std::vector<void*> allocs;
    int64_t bytes = 0;
    PsOps ops{};
    PsConv conv{};
    double* x_d = nullptr;
    double* D1c = nullptr;          // difference coefficients (Greeks)
    double* D2c = nullptr;
    double* V0 = nullptr;
    double* pool[POOLN] = {};
    double* Wb[2] = {};
    double* E = nullptr;
    double* Q = nullptr;
    std::vector<Kind> kinds;
    std::vector<std::pair<double, double>> steps;
    std::vector<int> step_kind;
    PsCtl* ctl = nullptr;
    PsCtl* ctl_h = nullptr;         // pinned mirror
    int* counts_d = nullptr;
    std::vector<int> counts_h;
    int P_rows = 16, P_cols = 16;
    int64_t total_iters = 0;
    int max_step_iters = 0;
    double last_inc = 0.0;
    int aa_m = 0;                   // Anderson depth (0: the paper's iteration)
    PsAABufs aab{};
};

#define PS_TRY(call)                                                                                      \
    do {                                                                                                  \
        hipError_t e_ = (call);                                                                           \
        if (e_ != hipSuccess)                                                                             \
            return fail(e_ == hipErrorOutOfMemory ? LPIDE_E_OOM : LPIDE_E_HIP,                            \
                        std::string(#call) + ": " + hipGetErrorString(e_));                               \
    } while (0)

template <typename T>
int dalloc(PsPlan* p, T** out, size_t count) {
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, std::max<size_t>(1, count) * sizeof(T));
    if (e != hipSuccess) return fail(LPIDE_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    p->allocs.push_back(d);
    p->bytes += int64_t(count * sizeof(T));
    *out = static_cast<T*>(d);
    return LPIDE_OK;
}

template <typename T>
int upload(PsPlan* p, T** out, const std::vector<T>& v) {
    int rc = dalloc(p, out, v.size());
    if (rc) return rc;
    PS_TRY(hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return LPIDE_OK;
}

int upload_rows(PsPlan* p, const std::vector<Cubic>& rows, int** s, double** w) {
    std::vector<int> sv(rows.size());
    std::vector<double> wv(4 * rows.size());
    for (size_t i = 0; i < rows.size(); ++i) {
        sv[i] = rows[i].s;
        for (int t = 0; t < 4; ++t) wv[4 * i + t] = rows[i].w[t];
    }
    int rc = upload(p, s, sv);
    return rc ? rc : upload(p, w, wv);
}

void destroy(PsPlan* p) {
    if (!p) return;
    for (void* a : p->allocs) (void)hipFree(a);
    if (p->ctl_h) (void)hipHostFree(p->ctl_h);
    delete p;
}

// Correlation launches for the plan's transform side.
void bapply(PsPlan* p, const PsConv& c, const double* Y, int k) {
    switch (p->L) {
#define PS_CASE(Lc) \
    case Lc: PsL<Lc>::bapply(c, Y, k); break;
        PS_CASE(64) PS_CASE(128) PS_CASE(256) PS_CASE(512) PS_CASE(640) PS_CASE(768) PS_CASE(896)
        PS_CASE(1024) PS_CASE(1152) PS_CASE(1280) PS_CASE(1536) PS_CASE(1792) PS_CASE(2048) PS_CASE(2304)
        PS_CASE(2560) PS_CASE(3072) PS_CASE(3584) PS_CASE(4096) PS_CASE(4608) PS_CASE(5120) PS_CASE(6144)
        PS_CASE(7168) PS_CASE(8192) PS_CASE(12288) PS_CASE(16384) PS_CASE(24576)
#undef PS_CASE
        default: break;
    }
}

void spectrum(PsPlan* p, const double* W, int W2, double2* Xf) {
    switch (p->L) {
#define PS_CASE(Lc) \
    case Lc: PsL<Lc>::spectrum(p->stream, W, W2, Xf, const_cast<double2*>(p->conv.spec), p->conv.tw, p->conv.twM); break;
        PS_CASE(64) PS_CASE(128) PS_CASE(256) PS_CASE(512) PS_CASE(640) PS_CASE(768) PS_CASE(896)
        PS_CASE(1024) PS_CASE(1152) PS_CASE(1280) PS_CASE(1536) PS_CASE(1792) PS_CASE(2048) PS_CASE(2304)
        PS_CASE(2560) PS_CASE(3072) PS_CASE(3584) PS_CASE(4096) PS_CASE(4608) PS_CASE(5120) PS_CASE(6144)
        PS_CASE(7168) PS_CASE(8192) PS_CASE(12288) PS_CASE(16384) PS_CASE(24576)
#undef PS_CASE
        default: break;
    }
}

// Chunks per line of the line solves: a power of two with chunks of at most
// `target` elements (at most LINE_MM), between lo and 256.
int chunks_for(int n, int target, int lo) {
    int P = lo;
    while (P < 256 && (n + P - 1) / P > target) P <<= 1;
    return P;
}

int make_kinds(PsPlan* p) {
    const PsHost& hp = p->hp;
    p->steps = step_list(p->theta, p->pay.T, p->N_t, p->opts.damping != 0);
    p->step_kind.assign(p->steps.size(), 0);
    for (size_t q = 0; q < p->steps.size(); ++q) {
        int found = -1;
        for (size_t k = 0; k < p->kinds.size(); ++k)
            if (p->kinds[k].theta == p->steps[q].first && p->kinds[k].dt == p->steps[q].second) found = int(k);
        if (found < 0) {
            Kind kd;
            kd.theta = p->steps[q].first;
            kd.dt = p->steps[q].second;
            kd.sk.c = kd.dt * kd.theta;
            std::vector<double> fl, bu, bc;
            int rc;
            double* f[6];
            ps_line_factors(hp, hp.a[0], hp.r_omega, kd.sk.c, fl, bu, bc);
            if ((rc = upload(p, &f[0], fl)) || (rc = upload(p, &f[1], bu)) || (rc = upload(p, &f[2], bc))) return rc;
            ps_line_factors(hp, hp.a[2], 0.0, kd.sk.c, fl, bu, bc);
            if ((rc = upload(p, &f[3], fl)) || (rc = upload(p, &f[4], bu)) || (rc = upload(p, &f[5], bc))) return rc;
            kd.sk.fl1 = f[0]; kd.sk.bu1 = f[1]; kd.sk.bc1 = f[2];
            kd.sk.fl2 = f[3]; kd.sk.bu2 = f[4]; kd.sk.bc2 = f[5];
            std::vector<Cubic> rows;
            ps_sl_rows(hp, std::exp(hp.kappa[0] * kd.dt), rows);
            if ((rc = upload_rows(p, rows, &kd.s1, &kd.w1))) return rc;
            ps_sl_rows(hp, std::exp(hp.kappa[1] * kd.dt), rows);
            if ((rc = upload_rows(p, rows, &kd.s2, &kd.w2))) return rc;
            p->kinds.push_back(kd);
            found = int(p->kinds.size()) - 1;
        }
        p->step_kind[q] = found;
    }
    return LPIDE_OK;
}

int create(const lpide_ps_grid* g, const lpide_levy* lv, const lpide_payoff* pay, double theta, int32_t N_t,
           const lpide_opts* opts, void** out) {
    if (!g || !lv || !pay || !out) return fail(LPIDE_E_PARAM, "NULL argument");
    lpide_opts o;
    if (opts) o = *opts; else lpide_opts_default(&o);
    if (!(theta >= 0.0 && theta <= 1.0)) return fail(LPIDE_E_PARAM, "theta must lie in [0, 1]");
    if (N_t < 1) return fail(LPIDE_E_PARAM, "N_t must be >= 1");
    if (!(o.tol > 0.0)) return fail(LPIDE_E_PARAM, "tol must be positive");
    if (o.max_iter < 1 || o.max_iter > PS_MAXK)
        return fail(LPIDE_E_PARAM, "max_iter must lie in [1, " + std::to_string(PS_MAXK) + "]");
    if (o.precision != LPIDE_FP64) return fail(LPIDE_E_PARAM, "the price-space plan computes in FP64 only");
    if (o.accel < -1 || o.accel > PS_AA_MAX)
        return fail(LPIDE_E_PARAM, "accel must lie in [-1, " + std::to_string(PS_AA_MAX) + "]");
    if (!(pay->K > 0.0) || !(pay->T > 0.0)) return fail(LPIDE_E_PARAM, "K and T must be positive");
    PsPlan* p = new PsPlan;
    std::string err;
    if (!build_ps_host(*g, *lv, pay->K, p->hp, err)) { delete p; return fail(LPIDE_E_PARAM, err); }
    std::vector<double> v0;
    if (!ps_initial(p->hp, *pay, v0, err)) { delete p; return fail(LPIDE_E_PARAM, err); }
    p->opts = o;
    p->pay = *pay;
    p->theta = theta;
    p->N_t = N_t;
    p->stream = static_cast<hipStream_t>(o.stream);
    p->jumps = p->hp.nts.jumps;
    const PsHost& hp = p->hp;
    if (p->jumps) {
        if (o.fft_size != 0) {
            if (!ps_side_supported(o.fft_size) || o.fft_size < hp.n_in) {
                const std::string msg = "fft_size " + std::to_string(o.fft_size) +
                                        " is not a supported transform side of at least #in = " +
                                        std::to_string(hp.n_in);
                delete p;
                return fail(LPIDE_E_PARAM, msg);
            }
            p->L = o.fft_size;
        } else {
            p->L = ps_side_at_least(hp.n_in);
            if (p->L == 0) {
                const std::string msg = "#in = " + std::to_string(hp.n_in) + " exceeds the largest transform side 24576";
                delete p;
                return fail(LPIDE_E_PARAM, msg);
            }
        }
    }
    {
        hipError_t e = hipSetDevice(o.device);
        if (e != hipSuccess) { delete p; return fail(LPIDE_E_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e)); }
    }
    int rc = LPIDE_OK;
    auto bail = [&](int code) { destroy(p); return code; };
    const int n = hp.n;
    const size_t N = size_t(n) * n;
    double *A1 = nullptr, *A2 = nullptr;
    if ((rc = upload(p, &p->x_d, hp.x)) || (rc = upload(p, &p->V0, v0)) || (rc = upload(p, &A1, hp.A1)) ||
        (rc = upload(p, &A2, hp.A2)) || (rc = upload(p, &p->D1c, hp.D1c)) || (rc = upload(p, &p->D2c, hp.D2c)))
        return bail(rc);
    for (int b = 0; b < POOLN; ++b)
        if ((rc = dalloc(p, &p->pool[b], N))) return bail(rc);
    if ((rc = dalloc(p, &p->Wb[0], N)) || (rc = dalloc(p, &p->Wb[1], N)) || (rc = dalloc(p, &p->E, N)) ||
        (rc = dalloc(p, &p->Q, N)) || (rc = dalloc(p, &p->ctl, 1)) || (rc = dalloc(p, &p->counts_d, p->N_t + 8)))
        return bail(rc);
    {
        hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&p->ctl_h), sizeof(PsCtl), hipHostMallocDefault);
        if (e != hipSuccess) { p->ctl_h = nullptr; return bail(fail(LPIDE_E_OOM, "hipHostMalloc ctl")); }
    }
    // Anderson mixing: the chosen depth, or depth 4 where the paper's iteration
    // is predicted to contract slowly (factor c sum_omega / (1 + c sum_omega),
    // c = h_t theta of the main steps)
    p->aa_m = o.accel;
    if (o.accel < 0) {
        const double c = pay->T / N_t * theta, cs = c * hp.sum_omega;
        p->aa_m = p->jumps && cs / (1.0 + cs) > 0.3 ? 4 : 0;
    }
    if (p->aa_m > 0) {
        PsAABufs& b = p->aab;
        b.m = p->aa_m;
        b.nblk = int((N + PS_AA_T * PS_AA_EPT - 1) / (PS_AA_T * PS_AA_EPT));
        double *Fp, *Yp, *dF, *dY, *part;
        PsAA* st;
        if ((rc = dalloc(p, &Fp, N)) || (rc = dalloc(p, &Yp, N)) || (rc = dalloc(p, &dF, size_t(b.m) * N)) ||
            (rc = dalloc(p, &dY, size_t(b.m) * N)) || (rc = dalloc(p, &part, size_t(b.nblk) * 2 * b.m)) ||
            (rc = dalloc(p, &st, 1)))
            return bail(rc);
        hipError_t e = hipMemset(dF, 0, size_t(b.m) * N * sizeof(double));
        if (e == hipSuccess) e = hipMemset(dY, 0, size_t(b.m) * N * sizeof(double));
        if (e == hipSuccess) e = hipMemset(st, 0, sizeof(PsAA));
        if (e != hipSuccess) return bail(fail(LPIDE_E_HIP, std::string("hipMemset: ") + hipGetErrorString(e)));
        b.F = p->Q;
        b.Fp = Fp;
        b.Yp = Yp;
        b.dF = dF;
        b.dY = dY;
        b.part = part;
        b.st = st;
    }
    PsOps& op = p->ops;
    op.n = n;
    op.A1 = A1;
    op.A2 = A2;
    op.a11 = hp.a[0];
    op.a12 = hp.a[1];
    op.a22 = hp.a[2];
    op.r_omega = hp.r_omega;
    if (p->jumps) {
        op.n_nz = hp.n_nz;
        op.n_out = hp.n_out;
        op.ldx = std::max(hp.n_nz, hp.n_out);
        int* s = nullptr;
        double* w = nullptr;
        if ((rc = upload_rows(p, hp.tin, &s, &w))) return bail(rc);
        op.tin_s = s;
        op.tin_w = w;
        if ((rc = upload_rows(p, hp.tout, &s, &w))) return bail(rc);
        op.tout_s = s;
        op.tout_w = w;
        const int L = p->L;
        auto twiddles = [](int N) {
            std::vector<double2> t(N);
            for (int q = 0; q < N; ++q) {
                // exp(-2 pi i q / N), evaluated in long double
                const long double ang = -2.0L * 3.14159265358979323846264338327950288L * q / N;
                t[q] = make_double2((double)cosl(ang), (double)sinl(ang));
            }
            return t;
        };
        double2 *twd = nullptr, *twM = nullptr, *spec = nullptr, *X = nullptr;
        double *U = nullptr, *Z = nullptr;
        if ((rc = upload(p, &twd, twiddles(L)))) return bail(rc);
        if (L > 8192 && (rc = upload(p, &twM, twiddles(big_m(L))))) return bail(rc);
        if ((rc = dalloc(p, &spec, size_t(L / 2 + 1) * L)) || (rc = dalloc(p, &X, size_t(L / 2 + 1) * op.ldx)) ||
            (rc = dalloc(p, &U, size_t(n) * hp.n_nz)) || (rc = dalloc(p, &Z, size_t(hp.n_out) * n)))
            return bail(rc);
        PsConv& c = p->conv;
        c.stream = p->stream;
        c.o = op;
        c.U = U;
        c.X = X;
        c.Z = Z;
        c.spec = spec;
        c.tw = twd;
        c.twM = twM;
        c.ctl = p->ctl;
        c.tol = o.tol;
        // the weights omega_{j1 - N_z, j2 - N_z} at offset (j1, j2) mod L: the
        // correlation out[o] = sum_j omega_j v^in[o + j] (Sec. 3.2.2)
        const int W2 = 2 * hp.N_z;
        double* Wd = nullptr;
        double2* Xf = nullptr;
        if (hipMalloc(&Wd, hp.omega.size() * sizeof(double)) != hipSuccess) return bail(fail(LPIDE_E_OOM, "hipMalloc W"));
        if (hipMalloc(&Xf, size_t(L / 2 + 1) * W2 * sizeof(double2)) != hipSuccess) {
            (void)hipFree(Wd);
            return bail(fail(LPIDE_E_OOM, "hipMalloc Xf"));
        }
        hipError_t e = hipMemcpy(Wd, hp.omega.data(), hp.omega.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            spectrum(p, Wd, W2, Xf);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        (void)hipFree(Wd);
        (void)hipFree(Xf);
        if (e != hipSuccess) return bail(fail(LPIDE_E_HIP, std::string("spectrum: ") + hipGetErrorString(e)));
    }
    p->conv.o = op;
    if ((rc = make_kinds(p))) return bail(rc);
    if (int(p->steps.size()) > p->N_t + 8) return bail(fail(LPIDE_E_PARAM, "step list longer than expected"));
    // chunks of at most 4 elements per line-solve thread: at N_x = 400 the row
    // solves then run 201 workgroups instead of 51 (march 9% faster than with 16)
    p->P_rows = chunks_for(n, 4, 8);
    p->P_cols = chunks_for(n, 4, 16);
    if ((n + p->P_rows - 1) / p->P_rows > LINE_MM || (n + p->P_cols - 1) / p->P_cols > LINE_MM)
        return bail(fail(LPIDE_E_PARAM, "N_x too large for the line solves"));
    hipLaunchKernelGGL(ps_ctl_reset, dim3(1), dim3(1), 0, p->stream, p->ctl, 1);
    {
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) return bail(fail(LPIDE_E_HIP, std::string("plan set-up: ") + hipGetErrorString(e)));
    }
    *out = p;
    return LPIDE_OK;
}

// Host bookkeeping of a march: pool slots of the current grid and of the
// extrapolation history (oldest first), the SL output of the step before.
struct MState {
    int cur = 0;
    int hist[4] = {0, 0, 0, 0};
    int nh = 0;
    int wprev = -1;
    double cprev = 0.0;        // dt theta of the step before (0: none)
    int y = -1, w = -1;        // iterate slot and SL buffer of the step just enqueued
};

int free_slot(const MState& m) {
    for (int b = 0; b < POOLN; ++b) {
        bool used = b == m.cur;
        for (int q = 0; q < m.nh; ++q) used = used || m.hist[q] == b;
        if (!used) return b;
    }
    return -1;
}

void iteration(PsPlan* p, const Kind& kd, double* Y, const double* W, int k) {
    const int n = p->hp.n;
    const double tol = p->opts.tol;
    if (p->jumps) bapply(p, p->conv, Y, k);
    const int lpb = 256 / p->P_rows;
    // the smallest chunk capacity of 4, 8 and LINE_MM that holds every chunk (the
    // plan's chunks hold at most 4 up to n = 1024; the sweeps run over all slots)
    const int chr = (n + p->P_rows - 1) / p->P_rows, chc = (n + p->P_cols - 1) / p->P_cols;
    auto rows = chr <= 4 ? ps_resid_rows<4> : chr <= 8 ? ps_resid_rows<8> : ps_resid_rows<LINE_MM>;
    auto cols = chc <= 4 ? ps_line_cols<4> : chc <= 8 ? ps_line_cols<8> : ps_line_cols<LINE_MM>;
    hipLaunchKernelGGL(rows, dim3((n + lpb - 1) / lpb), dim3(256), 0, p->stream, (const double*)Y, W,
                       p->jumps ? (const double*)p->conv.Z : (const double*)nullptr, p->Q, p->ops, kd.sk, p->P_rows,
                       (const PsCtl*)p->ctl, k, tol);
    const bool aa = p->aa_m > 0;
    hipLaunchKernelGGL(cols, dim3((n + 3) / 4), dim3(4 * p->P_cols), 0, p->stream, p->Q, Y, p->ops, kd.sk,
                       p->P_cols, p->ctl, k, tol, aa ? 1 : 0);
    if (aa) {
        const size_t N = size_t(n) * n;
        const PsAABufs& b = p->aab;
        hipLaunchKernelGGL(ps_aa_dots, dim3(b.nblk), dim3(PS_AA_T), 0, p->stream, (const double*)Y, b, N,
                           (const PsCtl*)p->ctl, k, tol);
        hipLaunchKernelGGL(ps_aa_solve, dim3(1), dim3(PS_AA_T), 0, p->stream, b, (const PsCtl*)p->ctl, k, tol);
        hipLaunchKernelGGL(ps_aa_update, dim3(b.nblk), dim3(PS_AA_T), 0, p->stream, Y, b, N, (const PsCtl*)p->ctl,
                           k, tol);
    }
}

// Enqueue step s with kmax iterations; advances m.
void enqueue_step(PsPlan* p, int s, int kmax, MState& m) {
    const double th = p->steps[s].first, dt = p->steps[s].second;
    const Kind& kd = p->kinds[p->step_kind[s]];
    const int n = p->hp.n;
    const size_t N = size_t(n) * n;
    const dim3 eb((unsigned)((N + 255) / 256));
    double* V = p->pool[m.cur];
    PsSL a{};
    a.s1 = kd.s1;
    a.s2 = kd.s2;
    a.w1 = kd.w1;
    a.w2 = kd.w2;
    a.src = V;
    a.wp = nullptr;
    a.rho = 0.0;
    if (th < 1.0) {
        if (!p->opts.all_correlations && m.wprev >= 0 && m.cprev > 0.0) {
            // (I - c A) V = W of the step before: E = V + dt (1 - theta) (V - W) / c
            a.wp = p->Wb[m.wprev];
            a.rho = dt * (1.0 - th) / m.cprev;
        } else {
            if (p->jumps) bapply(p, p->conv, V, 0);
            hipLaunchKernelGGL(ps_expl, eb, dim3(256), 0, p->stream, (const double*)V,
                               p->jumps ? (const double*)p->conv.Z : (const double*)nullptr, p->E, p->ops,
                               dt * (1.0 - th), (const PsCtl*)p->ctl);
            a.src = p->E;
        }
    }
    const int wcur = m.wprev == 0 ? 1 : 0;
    const int y = free_slot(m);
    a.W = p->Wb[wcur];
    a.Y = p->pool[y];
    const bool damped = p->opts.damping && s < 4;
    if (damped) {
        a.H[0] = V;
        a.coef[0] = 1.0;
        a.nh = 1;
    } else {
        // extrapolated start from V^{n-1}, V^{n-2}, ... (Sec. 3.3), newest first
        static const double cf[4][4] = {{1, 0, 0, 0}, {2, -1, 0, 0}, {3, -3, 1, 0}, {4, -6, 4, -1}};
        a.nh = m.nh;
        for (int q = 0; q < m.nh; ++q) {
            a.H[q] = p->pool[m.hist[m.nh - 1 - q]];
            a.coef[q] = cf[m.nh - 1][q];
        }
    }
    hipLaunchKernelGGL(ps_sl, eb, dim3(256), 0, p->stream, p->ops, a, (const PsCtl*)p->ctl);
    for (int k = 1; k <= kmax; ++k) iteration(p, kd, a.Y, a.W, k);
    hipLaunchKernelGGL(ps_step_end, dim3(1), dim3(1), 0, p->stream, p->ctl, p->counts_d, s, kmax, p->opts.tol);
    m.y = y;
    m.w = wcur;
    m.cur = y;
    if (!p->opts.damping || s >= 3) {
        if (m.nh == 4) {
            for (int q = 0; q < 3; ++q) m.hist[q] = m.hist[q + 1];
            m.nh = 3;
        }
        m.hist[m.nh++] = y;
    }
    m.wprev = wcur;
    m.cprev = dt * th;
}

int march(PsPlan* p, int nsteps, double* v_out) {
    PS_TRY(hipSetDevice(p->opts.device));
    const int n = p->hp.n;
    const size_t N = size_t(n) * n;
    hipLaunchKernelGGL(ps_ctl_reset, dim3(1), dim3(1), 0, p->stream, p->ctl, 1);
    PS_TRY(hipMemcpyAsync(p->pool[0], p->V0, N * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
    MState m;
    m.cur = 0;
    m.hist[0] = 0;
    m.nh = 1;
    const int maxk = p->opts.max_iter;
    std::vector<int> kpred(p->kinds.size(), std::min(6, maxk));
    p->counts_h.assign(nsteps, 0);
    p->total_iters = 0;
    p->max_step_iters = 0;
    std::vector<int> cb(BATCH);
    int s = 0;
    while (s < nsteps) {
        const int e = std::min(nsteps, s + BATCH);
        std::vector<MState> st(e - s + 1);
        std::vector<int> kused(e - s);
        st[0] = m;
        for (int q = s; q < e; ++q) {
            kused[q - s] = kpred[p->step_kind[q]];
            enqueue_step(p, q, kused[q - s], m);
            st[q - s + 1] = m;
        }
        PS_TRY(hipGetLastError());
        PS_TRY(hipMemcpyAsync(p->ctl_h, p->ctl, sizeof(PsCtl), hipMemcpyDeviceToHost, p->stream));
        PS_TRY(hipMemcpyAsync(cb.data(), p->counts_d + s, (e - s) * sizeof(int), hipMemcpyDeviceToHost, p->stream));
        PS_TRY(hipStreamSynchronize(p->stream));
        int f = e;
        if (p->ctl_h->fail) {
            f = s;
            while (f < e && cb[f - s] > 0) ++f;
        }
        std::vector<int> kmax_seen(p->kinds.size(), 0);
        for (int q = s; q < f; ++q) {
            p->counts_h[q] = cb[q - s];
            kmax_seen[p->step_kind[q]] = std::max(kmax_seen[p->step_kind[q]], cb[q - s]);
        }
        if (f < e) {
            if (p->ctl_h->fail == 2) return fail(LPIDE_E_NAN, "a fixed-point increment is not finite in step " + std::to_string(f));
            // step f needs more iterations than predicted: add them one at a time
            const Kind& kd = p->kinds[p->step_kind[f]];
            const MState& after = st[f - s + 1];
            int k = kused[f - s];
            for (;;) {
                if (k >= maxk)
                    return fail(LPIDE_E_NOCONV, "fixed-point iteration did not meet tol within max_iter in step " +
                                                    std::to_string(f));
                ++k;
                hipLaunchKernelGGL(ps_ctl_reset, dim3(1), dim3(1), 0, p->stream, p->ctl, 0);
                iteration(p, kd, p->pool[after.y], p->Wb[after.w], k);
                hipLaunchKernelGGL(ps_step_end, dim3(1), dim3(1), 0, p->stream, p->ctl, p->counts_d, f, k, p->opts.tol);
                PS_TRY(hipGetLastError());
                PS_TRY(hipMemcpyAsync(p->ctl_h, p->ctl, sizeof(PsCtl), hipMemcpyDeviceToHost, p->stream));
                PS_TRY(hipStreamSynchronize(p->stream));
                if (p->ctl_h->fail == 2)
                    return fail(LPIDE_E_NAN, "a fixed-point increment is not finite in step " + std::to_string(f));
                if (!p->ctl_h->fail) break;
            }
            int cf = 0;
            PS_TRY(hipMemcpy(&cf, p->counts_d + f, sizeof(int), hipMemcpyDeviceToHost));
            p->counts_h[f] = cf;
            kmax_seen[p->step_kind[f]] = std::max(kmax_seen[p->step_kind[f]], cf);
            m = after;
            s = f + 1;
        } else {
            s = e;
        }
        for (size_t k = 0; k < kpred.size(); ++k)
            if (kmax_seen[k] > 0) kpred[k] = std::min(maxk, kmax_seen[k]);
    }
    {
        const unsigned long long b = p->ctl_h->last;
        std::memcpy(&p->last_inc, &b, sizeof b);
    }
    for (int q = 0; q < nsteps; ++q) {
        p->total_iters += p->counts_h[q];
        p->max_step_iters = std::max(p->max_step_iters, p->counts_h[q]);
    }
    PS_TRY(hipMemcpyAsync(v_out, p->pool[m.cur], N * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
    PS_TRY(hipStreamSynchronize(p->stream));
    return LPIDE_OK;
}

PsPlan* as_plan(void* plan) { return static_cast<PsPlan*>(plan); }

}  // namespace
}  // namespace ps
}  // namespace lpide

using lpide::detail::fail;
using lpide::ps::PsPlan;

extern "C" {

void lpide_ps_grid_default(lpide_ps_grid* g, int32_t N_x, double x_max) {
    if (!g) return;
    std::memset(g, 0, sizeof *g);
    g->N_x = N_x;
    g->x_max = x_max;
    g->x_int = 0.0;
    g->fraction = 0.65;
    g->c = 0.0;
    g->nz_per_nx = 2;
    g->m1 = 2;
    g->ell_cut = 1e-14;
    g->zmax2_frac = std::sqrt(0.1);
    g->gl_nodes = 8;
}

int lpide_ps_discretize_host(const lpide_ps_grid* grid, const lpide_levy* levy, const lpide_payoff* payoff,
                             lpide_ps_info* info, double* x, double* v0, double* omega, int64_t omega_len) {
    if (!grid || !levy || !payoff || !info) return fail(LPIDE_E_PARAM, "NULL argument");
    if (!(payoff->K > 0.0)) return fail(LPIDE_E_PARAM, "K must be positive");
    lpide::PsHost hp;
    std::string err;
    if (!lpide::build_ps_host(*grid, *levy, payoff->K, hp, err)) return fail(LPIDE_E_PARAM, err);
    std::vector<double> v;
    if (v0 && !lpide::ps_initial(hp, *payoff, v, err)) return fail(LPIDE_E_PARAM, err);
    std::memset(info, 0, sizeof *info);
    info->N_x = hp.N_x;
    info->n = hp.n;
    info->N_z = hp.N_z;
    info->M1 = hp.M1;
    info->M2 = hp.M2;
    info->N_ym = hp.N_ym;
    info->N_yp = hp.N_yp;
    info->N_ystar = hp.N_ystar;
    info->n_in = hp.n_in;
    info->n_out = hp.n_out;
    info->n_nz = hp.n_nz;
    info->L = hp.nts.jumps ? lpide::ps::ps_side_at_least(hp.n_in) : 0;
    info->c = hp.c;
    info->x_int = hp.x_int;
    info->F = hp.F;
    info->h_z = hp.h_z;
    info->z_star = hp.z_star;
    info->sum_omega = hp.sum_omega;
    info->kappa[0] = hp.kappa[0];
    info->kappa[1] = hp.kappa[1];
    info->r_omega = hp.r_omega;
    for (int k = 0; k < 3; ++k) {
        info->S[k] = hp.S[k];
        info->a[k] = hp.a[k];
    }
    if (x) std::memcpy(x, hp.x.data(), hp.x.size() * sizeof(double));
    if (v0) std::memcpy(v0, v.data(), v.size() * sizeof(double));
    if (omega && omega_len >= int64_t(hp.omega.size()))
        std::memcpy(omega, hp.omega.data(), hp.omega.size() * sizeof(double));
    return LPIDE_OK;
}

int lpide_ps_plan_create(const lpide_ps_grid* grid, const lpide_levy* levy, const lpide_payoff* payoff,
                         double theta, int32_t N_t, const lpide_opts* opts, void** out) {
    return lpide::ps::create(grid, levy, payoff, theta, N_t, opts, out);
}

int lpide_ps_plan_destroy(void* plan) {
    if (!plan) return LPIDE_OK;
    PsPlan* p = lpide::ps::as_plan(plan);
    (void)hipSetDevice(p->opts.device);
    (void)hipStreamSynchronize(p->stream);
    lpide::ps::destroy(p);
    return LPIDE_OK;
}

int lpide_ps_plan_info(void* plan, lpide_ps_info* info) {
    if (!plan || !info) return fail(LPIDE_E_PARAM, "NULL argument");
    const PsPlan* p = lpide::ps::as_plan(plan);
    const lpide::PsHost& hp = p->hp;
    std::memset(info, 0, sizeof *info);
    info->N_x = hp.N_x;
    info->n = hp.n;
    info->N_z = hp.N_z;
    info->M1 = hp.M1;
    info->M2 = hp.M2;
    info->N_ym = hp.N_ym;
    info->N_yp = hp.N_yp;
    info->N_ystar = hp.N_ystar;
    info->n_in = hp.n_in;
    info->n_out = hp.n_out;
    info->n_nz = hp.n_nz;
    info->L = p->L;
    info->N_t = p->N_t;
    info->n_steps = int32_t(p->steps.size());
    info->c = hp.c;
    info->x_int = hp.x_int;
    info->F = hp.F;
    info->h_z = hp.h_z;
    info->z_star = hp.z_star;
    info->sum_omega = hp.sum_omega;
    info->kappa[0] = hp.kappa[0];
    info->kappa[1] = hp.kappa[1];
    info->r_omega = hp.r_omega;
    for (int k = 0; k < 3; ++k) {
        info->S[k] = hp.S[k];
        info->a[k] = hp.a[k];
    }
    info->total_iters = p->total_iters;
    info->max_step_iters = p->max_step_iters;
    info->last_increment = p->last_inc;
    info->device_bytes = p->bytes;
    info->accel_depth = p->aa_m;
    return LPIDE_OK;
}

int lpide_ps_nodes(void* plan, double* x) {
    if (!plan || !x) return fail(LPIDE_E_PARAM, "NULL argument");
    const PsPlan* p = lpide::ps::as_plan(plan);
    std::memcpy(x, p->hp.x.data(), p->hp.x.size() * sizeof(double));
    return LPIDE_OK;
}

int lpide_ps_initial(void* plan, double* v_out) {
    if (!plan || !v_out) return fail(LPIDE_E_PARAM, "NULL argument");
    PsPlan* p = lpide::ps::as_plan(plan);
    const size_t N = size_t(p->hp.n) * p->hp.n;
    hipError_t e = hipSetDevice(p->opts.device);
    if (e == hipSuccess) e = hipMemcpyAsync(v_out, p->V0, N * sizeof(double), hipMemcpyDeviceToDevice, p->stream);
    if (e != hipSuccess) return fail(LPIDE_E_HIP, std::string("lpide_ps_initial: ") + hipGetErrorString(e));
    return LPIDE_OK;
}

int lpide_ps_apply_B(void* plan, const double* v, double* bv) {
    if (!plan || !v || !bv) return fail(LPIDE_E_PARAM, "NULL argument");
    if (static_cast<const void*>(v) == static_cast<const void*>(bv)) return fail(LPIDE_E_PARAM, "v and bv must not alias");
    PsPlan* p = lpide::ps::as_plan(plan);
    const size_t N = size_t(p->hp.n) * p->hp.n;
    hipError_t e = hipSetDevice(p->opts.device);
    if (e != hipSuccess) return fail(LPIDE_E_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    const dim3 eb((unsigned)((N + 255) / 256));
    if (!p->jumps) {
        hipLaunchKernelGGL(lpide::ps::ps_fill, eb, dim3(256), 0, p->stream, bv, N, 0.0);
    } else {
        lpide::ps::PsConv c = p->conv;
        c.ctl = nullptr;
        lpide::ps::bapply(p, c, v, 0);
        hipLaunchKernelGGL(lpide::ps::ps_tout1, eb, dim3(256), 0, p->stream, (const double*)c.Z, bv, p->ops);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return fail(LPIDE_E_HIP, std::string("lpide_ps_apply_B: ") + hipGetErrorString(e));
    return LPIDE_OK;
}

int lpide_ps_solve_steps(void* plan, int32_t steps, double* v_out) {
    if (!plan || !v_out) return fail(LPIDE_E_PARAM, "NULL argument");
    PsPlan* p = lpide::ps::as_plan(plan);
    if (steps < 0 || steps > int32_t(p->steps.size()))
        return fail(LPIDE_E_PARAM, "steps must lie in [0, " + std::to_string(p->steps.size()) + "]");
    return lpide::ps::march(p, steps, v_out);
}

int lpide_ps_greeks(void* plan, const double* v, double* out) {
    if (!plan || !v || !out) return fail(LPIDE_E_PARAM, "NULL argument");
    PsPlan* p = lpide::ps::as_plan(plan);
    const size_t N = size_t(p->hp.n) * p->hp.n;
    if (static_cast<const void*>(v) == static_cast<const void*>(out)) return fail(LPIDE_E_PARAM, "v and out must not alias");
    hipError_t e = hipSetDevice(p->opts.device);
    if (e != hipSuccess) return fail(LPIDE_E_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    hipLaunchKernelGGL(lpide::ps::ps_greeks, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, p->stream, v, out, p->hp.n,
                       (const double*)p->D1c, (const double*)p->D2c);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(LPIDE_E_HIP, std::string("lpide_ps_greeks: ") + hipGetErrorString(e));
    return LPIDE_OK;
}

int lpide_ps_price(void* plan, const double* v, int32_t npts, const double* spots, double* price) {
    if (!plan) return fail(LPIDE_E_PARAM, "NULL plan");
    if (npts < 0) return fail(LPIDE_E_PARAM, "npts must be >= 0");
    if (npts == 0) return LPIDE_OK;
    if (!v || !spots || !price) return fail(LPIDE_E_PARAM, "NULL argument");
    PsPlan* p = lpide::ps::as_plan(plan);
    hipError_t e = hipSetDevice(p->opts.device);
    if (e != hipSuccess) return fail(LPIDE_E_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    hipLaunchKernelGGL(lpide::ps::ps_price, dim3((npts + 63) / 64), dim3(64), 0, p->stream, v,
                       (const double*)p->x_d, p->hp.n, npts, spots, price);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(LPIDE_E_HIP, std::string("lpide_ps_price: ") + hipGetErrorString(e));
    return LPIDE_OK;
}

}  // extern "C"
