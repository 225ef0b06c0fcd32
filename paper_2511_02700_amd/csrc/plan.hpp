// Internal structures of the solver library, shared by its translation units
// (lpide.hip: plans, groups, batches, the adjoint driver and the C ABI;
// march_L.hip: the launch sequences for one transform size each).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <string>
#include <type_traits>
#include <vector>

#include "host_plan.hpp"
#include "kernels.hpp"
#include "lpide.h"
#include "step_kernels.hpp"

namespace lpide {
namespace detail {

// Records msg as the calling thread's last error; returns code.
int fail(int code, const std::string& msg);

#define HIP_TRY(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ::lpide::detail::fail(e_ == hipErrorOutOfMemory ? LPIDE_E_OOM : LPIDE_E_HIP, \
                                         std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct Plan;

// Radix schedule (FFT elements per thread) of each kernel class of the march:
// column pass, row c2r kernels (+ explicit part, row FFT of V), line rows, SL.
struct Schedule { int cols, rinv, lrows, sl; };

// Launch shape of a group of plans that share the transform size: the march
// kernels run one grid for all of them (blockIdx.y = plan).
struct Launch {
    hipStream_t stream = nullptr;
    const MarchArgs* A = nullptr;   // device array, np entries
    int np = 0;
    int L = 0;                      // Lr of the plans (transform side of the row kernels)
    int xrows = 0;                  // max row pairs
    int cpb = 4;                    // columns per block of the axis-1 line solves (2 or 4)
    int xcols = 0;                  // max column groups of the axis-1 line solves
    int xaff = 0;                   // max rows (affine kernels without jumps)
    int P_cols = 16;
    int sl_order = 3;
    // FFT elements per thread (radix schedule: 4, 8 or 16) of each kernel class:
    // column pass, row c2r (+ explicit part, row FFT of V), line rows, SL
    int E_cols = 8, E_rinv = 8, E_lrows = 8, E_sl = 8;
    bool jumps = false, mixed = false;
    Plan* timer = nullptr;          // records kernel timing (single-plan marches only)
    bool record = false;            // launch the state-recording kernels (adjoint checkpoints)
    bool lean = false;              // every plan's steps in these slots are steady (FP64 shortcuts of
                                    // both kinds apply): the kernels that would exit are not launched
    int store_blocks = 1;           // grid of the recording copies
};

// Control state of a march over a group: one control block and per-step
// statistics per plan, with pinned host mirrors.
struct Group {
    std::vector<Plan*> plans;
    Launch lc;
    std::vector<MarchArgs> args_h;
    MarchArgs* A = nullptr;
    Ctl* ctl = nullptr;
    Ctl* ctl_h = nullptr;
    int* counts = nullptr;          // np x maxsteps
    double* incs = nullptr;
    std::vector<int> counts_h;
    std::vector<double> incs_h;
    int maxsteps = 0;
    bool use_graph = false;
    int slots = 32;                 // step slots enqueued between host checks
    struct G { int kmax, nslots; bool record, lean; hipGraphExec_t exec; };   // record: with the adjoint's store kernels
    std::vector<G> graphs;
    std::vector<void*> allocs;
    double tuned_ms = 0.0;
};

struct Adjoint;

struct Plan {
    HostPlan hp;
    lpide_grid grid{};
    lpide_opts opts{};
    lpide_payoff pay{};
    double theta = 0.5;
    int N_t = 1;
    hipStream_t stream = nullptr;
    int L = 0;        // FFT side (0 without jumps)
    int Lr = 0;       // transform side of the row-pair kernels (L, or a power of two >= n without jumps)
    bool jumps = false;
    bool mixed = false;            // FP32 iteration correlations (needs jumps)
    std::vector<void*> allocs;
    int64_t bytes = 0;
    double2* tw = nullptr;
    double2* spec = nullptr;
    double2* X = nullptr;
    float2* X32 = nullptr;
    float2* spec32 = nullptr;
    double* BV = nullptr;
    double* BY = nullptr;
    double* bpool[POOL] = {};      // B applied to the pool grids (FP64 form, B Y^0 by linearity)
    double* V0 = nullptr;
    double* pool[POOL] = {};
    double* Wb = nullptr;
    double* Rb = nullptr;
    StepDesc* sets_d = nullptr;
    int* step_set_d = nullptr;
    std::vector<StepDesc> sets;
    std::vector<int> step_set;
    int n_steps = 0;
    int P_cols = 16;
    Schedule sched{8, 8, 8, 8};    // radix schedule of the march kernels
    Group* solo = nullptr;         // this plan alone, on its own stream
    // adjoint march (allocated on the first lpide_adjoint call)
    struct Adjoint* adj = nullptr;
    std::vector<double> cn_rho;    // per step: rho of the explicit part from the previous step's equation (0: none)
    double* cn_rho_d = nullptr;
    int anchor_every = 8;          // mixed form: FP64 B V^{n-1} afresh every this many steps
    int march_step0 = 0;           // first step of the last march (anchors count from it)
    std::vector<char> steady;      // per step of the current march: both FP64 shortcuts apply
    int ckpt_every = 0;            // lpide_solve records checkpoints every this many steps (0: none)
    bool ckpt_valid = false;       // checkpoints of the last full solve are in adj->ckpt
    std::vector<int> counts_h;     // per-step iteration counts of the last march
    // kernel timing (HIP events on the plan's stream around each timed launch)
    uint32_t time_mask = 0;
    std::vector<hipEvent_t> ev_pool;
    struct EvRec { int cls; size_t idx; int step, k; };
    std::vector<EvRec> ev_recs;   // timed launches: class, start event, step and iteration (k = 0: once per step)
    int tag_step = -1, tag_k = 0; // step/iteration of the launches being enqueued
    size_t ev_used = 0;
    size_t ev_mark = 0;           // first record of the slots enqueued last
    int64_t k_launch[LPIDE_KCLASSES] = {};
    double k_ms[LPIDE_KCLASSES] = {};
    // statistics of the last solve
    int64_t total_iters = 0;
    int max_step_iters = 0, last_step_iters = 0;
    double last_inc = 0;
};

// Timing of one launch of kernel class cls.  A timed launch goes through
// hipExtLaunchKernelGGL with a start and a stop event, which then carry the
// dispatch's own begin and end timestamps (no marker packets between the
// kernels of the march, so the timed sequence runs as the untimed one).
struct KTime {
    Plan* p;
    int cls;
    bool on;
    KTime(Plan* pl, int c);
    bool events(hipEvent_t* a, hipEvent_t* b);   // a fresh pair, registered for harvest_times

    template <typename... P, typename... Args>
    void launch(void (*kernel)(P...), const dim3& g, const dim3& b, uint32_t shm, hipStream_t s, Args... args) {
        hipEvent_t e0, e1;
        if (on && events(&e0, &e1))
            hipExtLaunchKernelGGL(kernel, g, b, shm, s, e0, e1, 0u, static_cast<P>(args)...);
        else
            hipLaunchKernelGGL(kernel, g, b, shm, s, static_cast<P>(args)...);
    }
};

// State of the adjoint march (allocated on the first lpide_adjoint call).
struct Adjoint {
    int C = 0;                      // checkpoint stride
    int n_ckpt = 0;
    std::vector<void*> allocs;
    double* ckpt = nullptr;         // n_ckpt states V^{qC}
    double* seg = nullptr;          // C + 1 states of the segment being reversed
    double* segE = nullptr;         // C explicit parts of that segment
    double *lam = nullptr, *mu = nullptr, *ybar = nullptr, *dummy = nullptr;
    double* corr[4] = {};            // lam - Ybar of the last reverse steps, newest first
    double corr_c[4] = {};           // dt theta of those steps
    int have_corr = 0;               // how many of corr[] are set
    bool xb_is_v = false;            // XD holds the row transform of V^{s+1} from the previous reverse step
    double2 *XA = nullptr, *XB = nullptr, *XC = nullptr, *XD = nullptr;
    double2* S = nullptr;           // (L/2+1) x L spectral accumulator
    double* G = nullptr;            // L x L inverse transform of S
    double* acc = nullptr;          // n x 8 per-row accumulators
    StepDesc* sets_d = nullptr;
    std::vector<StepDesc> sets;
    MarchArgs* A = nullptr;
    MarchArgs args{};
    Ctl* ctl = nullptr;
    Ctl* ctl_h = nullptr;
    int* counts = nullptr;
    double* incs = nullptr;
    std::vector<int> counts_h;
    // host Jacobian of (a11, a12, a22, r_omega, kappa1, kappa2, omega) with respect to the
    // 8 subordination parameters, cached for the std point it was taken at
    double jac_std[8] = {};
    bool jac_valid = false;
    std::vector<double> jac;        // 8 x (6 + (2 N_z)^2)
};

// Radix schedules instantiated per transform size: the E for which the
// workgroup FFT runs at L (fft_ok: E = 4 and 8 for powers of two, E = 16 from
// L = 256 on; at L = 3 * 2^m only E with L / E a multiple of 64).
constexpr bool e_supported(int L, int E) { return fft_ok(L, E); }

// Call f(std::integral_constant<int, E>) for the runtime E of a kernel class
// (E must be supported at L; E = 4 always is).
template <int L, typename F>
void with_E(int E, F&& f) {
    if constexpr (fft_ok(L, 16)) {
        if (E == 16) return f(std::integral_constant<int, 16>{});
    }
    if constexpr (fft_ok(L, 8)) {
        if (E == 8) return f(std::integral_constant<int, 8>{});
    }
    f(std::integral_constant<int, 4>{});
}

// Columns per block of the axis-1 line solves: 4 adjacent columns share cache
// lines, but when the groups of 4 would leave CUs idle (fewer blocks than
// CUs over the whole group of plans) blocks take 2.
inline int line_cols_cpb(int nmax, int np) { return ((nmax + 3) / 4) * np < 256 ? 2 : 4; }

double bits_d(unsigned long long b);

// Stopping-rule value after iteration k from a host copy of a control block.
double err_of(const Ctl& c, int k);

// Work that depends on the transform size L, instantiated in one translation
// unit per size (march_L.hip compiled with -DLPIDE_L=L).
template <int L>
struct PerL {
    static void slots(const Launch& c, int first_tag, int nslots, int kmax);
    static void iteration(const Launch& c, int k);
    static void conv(Plan* p, const double* Y, double* out, double2* X);
    static void spectrum(Plan* p, const double* G, double2* Xfull);
    static void rows_fwd(Plan* p, const double* Y, hipStream_t s);
    static int adj_step(Plan* p, const Launch& c, int s, int* kpred, const double* Y, const double* V,
                        const double* E);
    static void adj_kernel_grad(Plan* p, hipStream_t s);
};
extern template struct PerL<64>;
extern template struct PerL<128>;
extern template struct PerL<256>;
extern template struct PerL<512>;
extern template struct PerL<768>;
extern template struct PerL<1024>;
extern template struct PerL<1536>;
extern template struct PerL<2048>;
extern template struct PerL<3072>;
extern template struct PerL<4096>;

}  // namespace detail
}  // namespace lpide
