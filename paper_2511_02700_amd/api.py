"""Python front end of the MI355X solver: builds the C structs, passes torch
tensors' device pointers to the C ABI and returns torch tensors.  PyTorch is
used for device memory and streams only; all arithmetic of the time march runs
in the HIP kernels of liblpide.so."""

import ctypes as C
import math

from . import _lib
from ._lib import Grid, Info, Levy, Opts, Payoff, PsGrid, PsInfo, check, lib


def _torch():
    import torch
    return torch


def levy_from_std(sigma1, sigma2, corr, theta1, theta2, kappa, alpha, r):
    """NTS parameters from the subordinated-Brownian-motion form (unit-mean
    subordinator with variance kappa); see lpide_levy_from_std."""
    lv = Levy()
    check(lib().lpide_levy_from_std(sigma1, sigma2, corr, theta1, theta2, kappa, alpha, r, C.byref(lv)))
    return lv


def levy_nts(alpha, delta, lam, eta, rho, r, sigma_bs=(0.0, 0.0, 0.0)):
    """NTS parameters as in the paper (alpha, delta, lambda, eta, rho = (rho11, rho12, rho22))."""
    lv = Levy()
    lv.r, lv.alpha, lv.delta, lv.lambda_ = r, alpha, delta, lam
    lv.eta[:] = list(eta)
    lv.rho[:] = list(rho)
    lv.sigma_bs[:] = list(sigma_bs)
    return lv


def levy_black_scholes(r, sigma_bs):
    """Zero Levy measure with Brownian covariance sigma_bs = (s11, s12, s22)."""
    lv = Levy()
    lv.r = r
    lv.sigma_bs[:] = list(sigma_bs)
    lv.no_jumps = 1
    return lv


def make_grid(n, y_lo, y_hi, sl_order=3, in_order=3, **kw):
    g = Grid()
    lib().lpide_grid_default(C.byref(g), n, y_lo, y_hi)
    g.sl_order, g.in_order = sl_order, in_order
    for k, v in kw.items():
        if k in ("y_lo", "y_hi"):
            getattr(g, k)[:] = list(v)
        else:
            setattr(g, k, v)
    return g


def make_payoff(kind="put_avg", K=100.0, T=1.0, cell_avg=True):
    return Payoff(_lib.PAYOFF[kind], K, T, 1 if cell_avg else 0)


def discretize_host(grid, levy, payoff=None, want_omega=False, want_v0=False):
    """Host-side plan quantities (no device needed): info dict, weights, V^0."""
    import numpy as np
    info = Info()
    check(lib().lpide_discretize_host(C.byref(grid), C.byref(levy), None, C.byref(info), None, 0, None))
    om = None
    v0 = None
    if want_omega and info.N_z > 0:
        om = np.zeros((2 * info.N_z, 2 * info.N_z))
    if want_v0:
        v0 = np.zeros((grid.n, grid.n))
    check(lib().lpide_discretize_host(
        C.byref(grid), C.byref(levy), C.byref(payoff) if payoff is not None else None, C.byref(info),
        om.ctypes.data_as(C.c_void_p) if om is not None else None, om.size if om is not None else 0,
        v0.ctypes.data_as(C.c_void_p) if v0 is not None else None))
    return info.to_dict(), om, v0


class Plan:
    """A planned solve on one HIP device (see lpide_plan_create)."""

    def __init__(self, grid, levy, payoff, theta=0.5, M=32, tol=1e-12, max_iter=100, precision="fp64",
                 damping=True, device=0, stream=None, fft_radix=0, fft_size=0, mixed_anchor=0,
                 all_correlations=False):
        torch = _torch()
        o = Opts()
        lib().lpide_opts_default(C.byref(o))
        o.tol, o.max_iter, o.precision, o.damping, o.device = tol, max_iter, _lib.PRECISION[precision], \
            1 if damping else 0, device
        o.fft_radix = fft_radix
        o.fft_size = fft_size
        o.mixed_anchor = mixed_anchor
        o.all_correlations = 1 if all_correlations else 0
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        o.stream = C.c_void_p(stream.cuda_stream)
        self.grid, self.levy, self.payoff = grid, levy, payoff
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().lpide_plan_create(C.byref(grid), C.byref(levy), C.byref(payoff), theta, M, C.byref(o),
                                          C.byref(h)))
        self._h = h
        self.n = grid.n

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().lpide_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        i = Info()
        check(lib().lpide_plan_info(self._h, C.byref(i)))
        return i.to_dict()

    def set_timing(self, classes=()):
        """Enable HIP-event timing for the named kernel classes (resets counters)."""
        mask = 0
        for c in classes:
            mask |= 1 << _lib.KCLASSES.index(c)
        check(lib().lpide_timing(self._h, mask))

    def kernel_stats(self):
        """{class: (launches, total ms)} since the last set_timing."""
        n = len(_lib.KCLASSES)
        la = (C.c_int64 * n)()
        ms = (C.c_double * n)()
        check(lib().lpide_kernel_stats(self._h, la, ms))
        return {c: (la[i], ms[i]) for i, c in enumerate(_lib.KCLASSES)}

    def _grid_tensor(self, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty((self.n, self.n), dtype=torch.float64, device=self.device)
        assert out.dtype == torch.float64 and out.is_contiguous() and out.numel() == self.n * self.n
        return out

    def solve(self, out=None):
        out = self._grid_tensor(out)
        check(lib().lpide_solve(self._h, C.c_void_p(out.data_ptr())))
        return out

    def solve_steps(self, steps, out=None):
        out = self._grid_tensor(out)
        check(lib().lpide_solve_steps(self._h, int(steps), C.c_void_p(out.data_ptr())))
        return out

    def solve_range(self, s0, s1, v_in, out=None):
        """Step-list entries [s0, s1) from the state v_in (see lpide_solve_range)."""
        torch = _torch()
        v_in = v_in.to(self.device, torch.float64).contiguous()
        out = self._grid_tensor(out)
        check(lib().lpide_solve_range(self._h, int(s0), int(s1), C.c_void_p(v_in.data_ptr()),
                                      C.c_void_p(out.data_ptr())))
        return out

    def initial(self, out=None):
        out = self._grid_tensor(out)
        check(lib().lpide_initial(self._h, C.c_void_p(out.data_ptr())))
        return out

    def apply_B(self, v, out=None):
        torch = _torch()
        v = v.to(self.device, torch.float64).contiguous()
        out = self._grid_tensor(out)
        check(lib().lpide_apply_B(self._h, C.c_void_p(v.data_ptr()), C.c_void_p(out.data_ptr())))
        return out

    def apply_B_noalloc(self, v, out):
        """B v into the caller's tensor out, with no device allocation by the
        library (lpide_apply_B_noalloc): v and out must already be contiguous
        float64 tensors on the plan's device."""
        torch = _torch()
        assert v.dtype == torch.float64 and v.is_contiguous() and v.device == self.device
        out = self._grid_tensor(out)
        check(lib().lpide_apply_B_noalloc(self._h, C.c_void_p(v.data_ptr()), C.c_void_p(out.data_ptr())))
        return out

    def set_checkpoints(self, every):
        """Let later solve() calls keep the checkpoints an adjoint with the same
        stride needs (0: off)."""
        check(lib().lpide_plan_set_checkpoints(self._h, int(every)))

    def adjoint(self, v_bar, checkpoint_every=32, std_params=None):
        """Reverse-mode gradient of J with dJ/dV^{N_t} = v_bar (lpide_adjoint).
        Returns (grad, native, info): grad = dJ/d(sigma1, sigma2, corr, theta1,
        theta2, kappa, alpha, r) (None unless std_params, the point the plan's
        model was built from, is given); native = numpy array of
        dJ/d(a11, a12, a22, r_omega, kappa_omega1, kappa_omega2) followed by
        dJ/d omega (2 N_z x 2 N_z, row-major)."""
        import numpy as np
        torch = _torch()
        v_bar = v_bar.to(self.device, torch.float64).contiguous()
        nz = self.info()["N_z"]
        native = np.zeros(6 + (2 * nz) ** 2)
        grad = np.zeros(8) if std_params is not None else None
        sp = (C.c_double * 8)(*[float(x) for x in std_params]) if std_params is not None else None
        ai = _lib.AdjInfo()
        check(lib().lpide_adjoint(self._h, C.c_void_p(v_bar.data_ptr()), int(checkpoint_every), sp,
                                  grad.ctypes.data_as(C.POINTER(C.c_double)) if grad is not None else None,
                                  native.ctypes.data_as(C.POINTER(C.c_double)), C.byref(ai)))
        return grad, native, ai.to_dict()

    def price_adjoint(self, spots, price_bar):
        """Cotangent of the grid for price cotangents (the transpose of price)."""
        torch = _torch()
        sp = torch.as_tensor(spots, dtype=torch.float64).reshape(-1, 2).to(self.device).contiguous()
        pb = torch.as_tensor(price_bar, dtype=torch.float64).reshape(-1).to(self.device).contiguous()
        out = self._grid_tensor()
        check(lib().lpide_price_adjoint(self._h, sp.shape[0], C.c_void_p(sp.data_ptr()), C.c_void_p(pb.data_ptr()),
                                        C.c_void_p(out.data_ptr())))
        return out

    def price(self, v, spots, with_delta=False):
        torch = _torch()
        sp = torch.as_tensor(spots, dtype=torch.float64).reshape(-1, 2).to(self.device).contiguous()
        k = sp.shape[0]
        pr = torch.empty(k, dtype=torch.float64, device=self.device)
        dl = torch.empty((k, 2), dtype=torch.float64, device=self.device) if with_delta else None
        check(lib().lpide_price(self._h, C.c_void_p(v.data_ptr()), k, C.c_void_p(sp.data_ptr()),
                                C.c_void_p(pr.data_ptr()), C.c_void_p(dl.data_ptr()) if dl is not None else None))
        return (pr, dl) if with_delta else pr

    def greeks(self, v):
        """Delta and Gamma surfaces at the nodes (lpide_greeks): a (5, n, n)
        float64 tensor delta1, delta2, gamma11, gamma12, gamma22."""
        torch = _torch()
        n = v.shape[0]
        out = torch.empty((5, n, n), dtype=torch.float64, device=self.device)
        check(lib().lpide_greeks(self._h, C.c_void_p(v.contiguous().data_ptr()), C.c_void_p(out.data_ptr())))
        return out


class Batch:
    """Many plans marched together (see lpide_batch_create).  The plans must
    stay alive while the batch is used; results are torch float64 tensors."""

    def __init__(self, plans, use_graph=True, slots=32, stream=None):
        torch = _torch()
        if not plans:
            raise ValueError("empty batch")
        self.plans = list(plans)
        self.device = self.plans[0].device
        o = _lib.BatchOpts()
        lib().lpide_batch_opts_default(C.byref(o))
        o.use_graph, o.slots = (1 if use_graph else 0), slots
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        o.stream = C.c_void_p(stream.cuda_stream)
        hs = (C.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().lpide_batch_create(len(self.plans), hs, C.byref(o), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().lpide_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _outs(self, outs):
        if outs is None:
            outs = [p._grid_tensor() for p in self.plans]
        for p, o in zip(self.plans, outs):
            p._grid_tensor(o)
        return outs, (C.c_void_p * len(outs))(*[o.data_ptr() for o in outs])

    def solve(self, outs=None):
        outs, ptrs = self._outs(outs)
        check(lib().lpide_batch_solve(self._h, ptrs))
        return outs

    def solve_steps(self, steps, outs=None):
        outs, ptrs = self._outs(outs)
        check(lib().lpide_batch_solve_steps(self._h, int(steps), ptrs))
        return outs

    def tune(self, trial_steps=12):
        check(lib().lpide_batch_tune(self._h, int(trial_steps)))
        return self.groups()

    def groups(self):
        n = C.c_int32()
        check(lib().lpide_batch_info(self._h, C.byref(n), None, 0))
        arr = (_lib.GroupInfo * max(1, n.value))()
        check(lib().lpide_batch_info(self._h, C.byref(n), arr, n.value))
        return [arr[i].to_dict() for i in range(n.value)]


def std_params_of(w):
    """(sigma1, sigma2, corr, theta1, theta2, kappa, alpha, r) of a workload."""
    m = w["model"]
    return (m["sigma1"], m["sigma2"], m["corr"], m["theta1"], m["theta2"], m["kappa"], m["alpha"], w["r"])


def plan_from_workload(w, device=0, **over):
    """A Plan for a workload dict of ``workloads.WORKLOADS`` (pure data)."""
    m = w["model"]
    lv = levy_from_std(m["sigma1"], m["sigma2"], m["corr"], m["theta1"], m["theta2"], m["kappa"], m["alpha"], w["r"])
    g = make_grid(w["n"], w["y_lo"], w["y_hi"], sl_order=over.pop("sl_order", 3), in_order=over.pop("in_order", 3),
                  nz_fixed=over.pop("nz_fixed", 0))
    pay = make_payoff(w.get("payoff", "put_avg"), w["K"], w["T"])
    return Plan(g, lv, pay, theta=w["theta"], M=w["N_t"], tol=over.pop("tol", w["tol"]), device=device, **over)


def solve(grid, levy, payoff, theta=0.5, M=32, **opts):
    """One-shot solve: plan, march every step, return V^{N_t} as an n x n
    float64 tensor on the plan's device (lpide_plan, lpide_solve,
    lpide_destroy).  opts are the Plan keywords (tol, precision, ...)."""
    plan = Plan(grid, levy, payoff, theta=theta, M=M, **opts)
    try:
        v = plan.solve()
        plan.stream.synchronize()
        return v
    finally:
        plan.close()


def make_ps_grid(N_x, x_max, **kw):
    """Price-space grid settings (lpide_ps_grid); the paper's defaults unless
    overridden (x_int, fraction, c, nz_per_nx, m1, ell_cut, zmax2_frac, gl_nodes)."""
    g = PsGrid()
    lib().lpide_ps_grid_default(C.byref(g), int(N_x), float(x_max))
    for k, v in kw.items():
        setattr(g, k, v)
    return g


def ps_discretize_host(grid, levy, payoff, want_v0=False, want_omega=False):
    """Host-side quantities of the price-space plan (no device needed):
    (info dict, x nodes, V^0 or None, omega or None)."""
    import numpy as np
    info = PsInfo()
    x = np.zeros(grid.N_x + 1)
    check(lib().lpide_ps_discretize_host(C.byref(grid), C.byref(levy), C.byref(payoff), C.byref(info),
                                         x.ctypes.data_as(C.c_void_p), None, None, 0))
    v0 = np.zeros((grid.N_x + 1, grid.N_x + 1)) if want_v0 else None
    om = np.zeros((2 * info.N_z, 2 * info.N_z)) if want_omega and info.N_z > 0 else None
    if v0 is not None or om is not None:
        check(lib().lpide_ps_discretize_host(
            C.byref(grid), C.byref(levy), C.byref(payoff), C.byref(info), None,
            v0.ctypes.data_as(C.c_void_p) if v0 is not None else None,
            om.ctypes.data_as(C.c_void_p) if om is not None else None, om.size if om is not None else 0))
    return info.to_dict(), x, v0, om


class PsPlan:
    """A price-space plan on one HIP device (see lpide_ps_plan_create)."""

    def __init__(self, grid, levy, payoff, theta=0.5, N_t=None, tol=1e-10, max_iter=128, damping=True, device=0,
                 stream=None, fft_size=0, all_correlations=False, accel=-1):
        """accel: 0 the paper's fixed-point iteration, 1..6 Anderson mixing of that depth,
        -1 (default) depth 4 where the iteration is predicted to contract slowly.
        tol: the stopping value's rounding floor grows with the grid on the NIG sets and lies
        near 1e-10 on the paper's own grids (N_x = 400, 800); use 1e-9 there (the paper: 1e-7)."""
        torch = _torch()
        o = Opts()
        lib().lpide_opts_default(C.byref(o))
        o.tol, o.max_iter, o.damping, o.device = tol, max_iter, 1 if damping else 0, device
        o.fft_size = fft_size
        o.all_correlations = 1 if all_correlations else 0
        o.accel = int(accel)
        if N_t is None:
            N_t = max(1, int(round(0.5 * grid.N_x)))     # Sec. 4: N_t = round(N_x / 2)
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        o.stream = C.c_void_p(stream.cuda_stream)
        self.grid, self.levy, self.payoff = grid, levy, payoff
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().lpide_ps_plan_create(C.byref(grid), C.byref(levy), C.byref(payoff), theta, int(N_t),
                                             C.byref(o), C.byref(h)))
        self._h = h
        self.n = grid.N_x + 1

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().lpide_ps_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        i = PsInfo()
        check(lib().lpide_ps_plan_info(self._h, C.byref(i)))
        return i.to_dict()

    def nodes(self):
        import numpy as np
        x = np.zeros(self.n)
        check(lib().lpide_ps_nodes(self._h, x.ctypes.data_as(C.c_void_p)))
        return x

    def _grid_tensor(self, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty((self.n, self.n), dtype=torch.float64, device=self.device)
        assert out.dtype == torch.float64 and out.is_contiguous() and out.numel() == self.n * self.n
        return out

    def initial(self, out=None):
        out = self._grid_tensor(out)
        check(lib().lpide_ps_initial(self._h, C.c_void_p(out.data_ptr())))
        return out

    def apply_B(self, v, out=None):
        torch = _torch()
        v = v.to(self.device, torch.float64).contiguous()
        out = self._grid_tensor(out)
        check(lib().lpide_ps_apply_B(self._h, C.c_void_p(v.data_ptr()), C.c_void_p(out.data_ptr())))
        return out

    def solve_steps(self, steps, out=None):
        out = self._grid_tensor(out)
        check(lib().lpide_ps_solve_steps(self._h, int(steps), C.c_void_p(out.data_ptr())))
        return out

    def solve(self, out=None):
        return self.solve_steps(self.info()["n_steps"], out)

    def greeks(self, v):
        """Delta and Gamma surfaces (5, n, n): delta1, delta2, gamma11, gamma12, gamma22."""
        torch = _torch()
        v = v.to(self.device, torch.float64).contiguous()
        out = torch.empty((5, self.n, self.n), dtype=torch.float64, device=self.device)
        check(lib().lpide_ps_greeks(self._h, C.c_void_p(v.data_ptr()), C.c_void_p(out.data_ptr())))
        return out

    def price(self, v, spots):
        torch = _torch()
        sp = torch.as_tensor(spots, dtype=torch.float64).reshape(-1, 2).to(self.device).contiguous()
        out = torch.empty(sp.shape[0], dtype=torch.float64, device=self.device)
        check(lib().lpide_ps_price(self._h, C.c_void_p(v.data_ptr()), int(sp.shape[0]), C.c_void_p(sp.data_ptr()),
                                   C.c_void_p(out.data_ptr())))
        return out


class PricesFn:
    """Prices at spot pairs as a differentiable function of the subordination
    parameters and the spots: ``PricesFn.apply(params, spots, grid_args,
    payoff_args)`` with params = tensor (sigma1, sigma2, corr, theta1, theta2,
    kappa, alpha, r) (float64), spots = tensor (k, 2); grid_args = dict(n, y_lo,
    y_hi, N_t, theta, tol, sl_order, checkpoint_every), payoff_args =
    dict(kind, K, T).  The backward pass is the library's adjoint march
    (lpide_price_adjoint, lpide_adjoint) for the parameters and the deltas for
    the spots; the structure (N_z, L) is fixed at the point of the forward."""

    @staticmethod
    def apply(params, spots, grid_args, payoff_args):
        return _prices_function().apply(params, spots, grid_args, payoff_args)


_PF = None


def _prices_function():
    global _PF
    if _PF is not None:
        return _PF
    torch = _torch()

    class _Prices(torch.autograd.Function):
        @staticmethod
        def forward(ctx, params, spots, grid_args, payoff_args):
            x = [float(v) for v in params.detach().cpu().reshape(-1)]
            ga = dict(grid_args)
            lv = levy_from_std(*x)
            g = make_grid(ga["n"], ga["y_lo"], ga["y_hi"], sl_order=ga.get("sl_order", 3),
                          nz_fixed=ga.get("nz_fixed", 0))
            pay = make_payoff(payoff_args.get("kind", "put_avg"), payoff_args["K"], payoff_args["T"])
            plan = Plan(g, lv, pay, theta=ga.get("theta", 0.5), M=ga["N_t"], tol=ga.get("tol", 1e-12))
            C_every = ga.get("checkpoint_every", 32)
            plan.set_checkpoints(C_every)
            V = plan.solve()
            sp = spots.detach().to(plan.device, torch.float64).reshape(-1, 2).contiguous()
            pr, dl = plan.price(V, sp, with_delta=True)
            ctx.plan, ctx.x, ctx.sp, ctx.dl, ctx.C = plan, x, sp, dl, C_every
            ctx.params_device, ctx.spots_device = params.device, spots.device
            return pr.to(params.device)

        @staticmethod
        def backward(ctx, gout):
            plan = ctx.plan
            g = gout.detach().to(plan.device, torch.float64).reshape(-1).contiguous()
            vbar = plan.price_adjoint(ctx.sp, g)
            grad, _, _ = plan.adjoint(vbar, ctx.C, std_params=ctx.x)
            # each gradient lives where its input does
            gp = torch.as_tensor(grad, dtype=torch.float64).to(ctx.params_device)
            gs = (g[:, None] * ctx.dl).to(ctx.spots_device)
            return gp, gs, None, None

    _PF = _Prices
    return _PF
