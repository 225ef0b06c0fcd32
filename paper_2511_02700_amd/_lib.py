"""ctypes binding of liblpide.so (include/lpide.h).  Argument marshalling only:
every step of the time march runs in the library's HIP kernels."""

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LPIDE_LIB") or os.path.join(HERE, "liblpide.so")

LPIDE_OK = 0
ERRORS = {-1: "LPIDE_E_PARAM", -2: "LPIDE_E_NOCONV", -3: "LPIDE_E_NAN", -4: "LPIDE_E_HIP", -5: "LPIDE_E_OOM"}
PAYOFF = {"put_avg": 0, "call_avg": 1, "put_1": 2, "call_1": 3, "exchange": 4, "spread": 5}
PRECISION = {"fp64": 0, "fp32conv": 1}
KCLASSES = ["cols", "rows_inv", "line_cols", "line_rows", "sl", "step_end", "expl_cols", "expl_rows", "rows_fwd",
            "carry", "expl_id", "rows_lin", "sl_lin"]


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32), ("y_lo", C.c_double * 2), ("y_hi", C.c_double * 2),
                ("sl_order", C.c_int32), ("in_order", C.c_int32), ("m1", C.c_int32),
                ("ell_cut", C.c_double), ("zmax2_frac", C.c_double), ("gl_nodes", C.c_int32),
                ("nz_fixed", C.c_int32)]


class Levy(C.Structure):
    _fields_ = [("r", C.c_double), ("alpha", C.c_double), ("delta", C.c_double), ("lambda_", C.c_double),
                ("eta", C.c_double * 2), ("rho", C.c_double * 3), ("sigma_bs", C.c_double * 3),
                ("no_jumps", C.c_int32)]


class Payoff(C.Structure):
    _fields_ = [("kind", C.c_int32), ("K", C.c_double), ("T", C.c_double), ("cell_avg", C.c_int32)]


class Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("precision", C.c_int32),
                ("damping", C.c_int32), ("device", C.c_int32), ("stream", C.c_void_p), ("fft_radix", C.c_int32),
                ("fft_size", C.c_int32), ("mixed_anchor", C.c_int32),
                ("all_correlations", C.c_int32), ("accel", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("n", C.c_int32), ("N_z", C.c_int32), ("M1", C.c_int32), ("M2", C.c_int32), ("L", C.c_int32),
                ("N_t", C.c_int32), ("n_steps", C.c_int32),
                ("h", C.c_double), ("z_star", C.c_double), ("sum_omega", C.c_double),
                ("kappa", C.c_double * 2), ("r_omega", C.c_double), ("S", C.c_double * 3), ("a", C.c_double * 3),
                ("total_iters", C.c_int64), ("max_step_iters", C.c_int32), ("last_step_iters", C.c_int32),
                ("last_increment", C.c_double), ("device_bytes", C.c_int64), ("radix", C.c_int32 * 4)]

    def to_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


class AdjInfo(C.Structure):
    _fields_ = [("adj_iters", C.c_int64), ("max_step_iters", C.c_int32), ("forward_ms", C.c_double),
                ("recompute_ms", C.c_double), ("reverse_ms", C.c_double), ("gather_ms", C.c_double),
                ("jacobian_ms", C.c_double)]

    def to_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class BatchOpts(C.Structure):
    _fields_ = [("use_graph", C.c_int32), ("slots", C.c_int32), ("stream", C.c_void_p)]


class GroupInfo(C.Structure):
    _fields_ = [("n_plans", C.c_int32), ("L", C.c_int32), ("mixed", C.c_int32), ("P_cols", C.c_int32),
                ("slots", C.c_int32), ("use_graph", C.c_int32), ("radix", C.c_int32 * 4),
                ("trial_ms", C.c_double)]

    def to_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


class PsGrid(C.Structure):
    _fields_ = [("N_x", C.c_int32), ("x_max", C.c_double), ("x_int", C.c_double), ("fraction", C.c_double),
                ("c", C.c_double), ("nz_per_nx", C.c_int32), ("m1", C.c_int32), ("ell_cut", C.c_double),
                ("zmax2_frac", C.c_double), ("gl_nodes", C.c_int32)]


class PsInfo(C.Structure):
    _fields_ = [("N_x", C.c_int32), ("n", C.c_int32), ("N_z", C.c_int32), ("M1", C.c_int32), ("M2", C.c_int32),
                ("N_ym", C.c_int32), ("N_yp", C.c_int32), ("N_ystar", C.c_int32), ("n_in", C.c_int32),
                ("n_out", C.c_int32), ("n_nz", C.c_int32), ("L", C.c_int32), ("N_t", C.c_int32),
                ("n_steps", C.c_int32), ("c", C.c_double), ("x_int", C.c_double), ("F", C.c_double),
                ("h_z", C.c_double), ("z_star", C.c_double), ("sum_omega", C.c_double),
                ("kappa", C.c_double * 2), ("r_omega", C.c_double), ("S", C.c_double * 3), ("a", C.c_double * 3),
                ("total_iters", C.c_int64), ("max_step_iters", C.c_int32), ("last_increment", C.c_double),
                ("device_bytes", C.c_int64), ("accel_depth", C.c_int32)]

    def to_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


# exported symbol -> (restype, argtypes)
SIGNATURES = {
    "lpide_grid_default": (None, [C.POINTER(Grid), C.c_int32, C.c_double, C.c_double]),
    "lpide_opts_default": (None, [C.POINTER(Opts)]),
    "lpide_levy_from_std": (C.c_int, [C.c_double] * 8 + [C.POINTER(Levy)]),
    "lpide_plan_create": (C.c_int, [C.POINTER(Grid), C.POINTER(Levy), C.POINTER(Payoff), C.c_double, C.c_int32,
                                    C.POINTER(Opts), C.POINTER(C.c_void_p)]),
    "lpide_plan_destroy": (C.c_int, [C.c_void_p]),
    "lpide_plan": (C.c_int, [C.POINTER(Grid), C.POINTER(Levy), C.POINTER(Payoff), C.c_double, C.c_int32,
                             C.POINTER(Opts), C.POINTER(C.c_void_p)]),
    "lpide_destroy": (C.c_int, [C.c_void_p]),
    "lpide_plan_batch": (C.c_int, [C.c_int32, C.POINTER(Grid), C.POINTER(Levy), C.POINTER(Payoff), C.c_double,
                                   C.POINTER(C.c_int32), C.POINTER(Opts), C.POINTER(C.c_void_p)]),
    "lpide_solve_batch": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "lpide_plan_info": (C.c_int, [C.c_void_p, C.POINTER(Info)]),
    "lpide_solve": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lpide_solve_steps": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "lpide_solve_range": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    "lpide_initial": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lpide_apply_B": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lpide_apply_B_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lpide_price": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lpide_greeks": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lpide_discretize_host": (C.c_int, [C.POINTER(Grid), C.POINTER(Levy), C.POINTER(Payoff), C.POINTER(Info),
                                        C.c_void_p, C.c_int64, C.c_void_p]),
    "lpide_timing": (C.c_int, [C.c_void_p, C.c_uint32]),
    "lpide_kernel_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "lpide_plan_set_checkpoints": (C.c_int, [C.c_void_p, C.c_int32]),
    "lpide_adjoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                C.POINTER(C.c_double), C.POINTER(AdjInfo)]),
    "lpide_price_adjoint": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lpide_batch_opts_default": (None, [C.POINTER(BatchOpts)]),
    "lpide_batch_create": (C.c_int, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(BatchOpts),
                                     C.POINTER(C.c_void_p)]),
    "lpide_batch_destroy": (C.c_int, [C.c_void_p]),
    "lpide_batch_solve": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "lpide_batch_solve_steps": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)]),
    "lpide_batch_tune": (C.c_int, [C.c_void_p, C.c_int32]),
    "lpide_batch_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(GroupInfo), C.c_int32]),
    "lpide_last_error": (C.c_char_p, []),
    "lpide_ps_grid_default": (None, [C.POINTER(PsGrid), C.c_int32, C.c_double]),
    "lpide_ps_discretize_host": (C.c_int, [C.POINTER(PsGrid), C.POINTER(Levy), C.POINTER(Payoff), C.POINTER(PsInfo),
                                           C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "lpide_ps_plan_create": (C.c_int, [C.POINTER(PsGrid), C.POINTER(Levy), C.POINTER(Payoff), C.c_double,
                                       C.c_int32, C.POINTER(Opts), C.POINTER(C.c_void_p)]),
    "lpide_ps_plan_destroy": (C.c_int, [C.c_void_p]),
    "lpide_ps_plan_info": (C.c_int, [C.c_void_p, C.POINTER(PsInfo)]),
    "lpide_ps_nodes": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lpide_ps_initial": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lpide_ps_apply_B": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lpide_ps_solve_steps": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "lpide_ps_price": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "lpide_ps_greeks": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
}

_lib = None


class LpideError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "error"), code, msg))
        self.code = code


def lib():
    """The loaded library.  Raises if it has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblpide.so is not built; run `python -m paper_2511_02700_amd.build` "
                              "(or __graft_entry__.build())")
        # torch ships its own HIP runtime under the same soname as the one the
        # library links; whichever is loaded first serves the process.  Loading
        # torch first keeps its kernels and ours on torch's runtime (the other
        # order makes torch's own launches fail with "invalid device function").
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != LPIDE_OK:
        raise LpideError(rc, lib().lpide_last_error().decode(errors="replace"))
    return rc
