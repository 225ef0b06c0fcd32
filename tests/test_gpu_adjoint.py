"""GPU tests of the adjoint march (lpide_adjoint through the C ABI).

* The native gradient (dJ/d(a11, a12, a22, r_omega, kappa_omega), dJ/d omega)
  against the oracle's dense discrete adjoint on small grids, within 1e-8
  relative to each quantity's scale (both are FP64; the GPU solves every fixed
  point to 1e-12).
* The gradient with respect to the eight subordination parameters against
  central finite differences of the GPU forward march (step 1e-5 max(|x|, 0.1),
  structure fixed), within 1e-5 per component, each relative to its own size
  (floored at 1e-2 of the largest component), on a small grid and on the
  1024 x 1024, 512-step workload with checkpoints every 32 steps.
* The spot deltas of the 1024 x 1024 march against central differences of the
  prices at bumped spots (relative step 1e-5), within 1e-5.
* The autograd wrapper: its parameter gradient equals the adjoint's and its
  spot gradient equals the deltas times the cotangent, with CPU and with GPU
  inputs (each gradient on its input's device).
"""

import sys
import time

import numpy as np
import pytest

import workloads
from oracle import adjoint as oadj
from oracle import integral, levy, scheme

pytestmark = pytest.mark.gpu


def _note(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lp():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_2511_02700_amd as m
    m.lib()
    return m


def _oracle_problem(w):
    m = w["model"]
    p = levy.nts_from_std(m["sigma1"], m["sigma2"], m["corr"], m["theta1"], m["theta2"], m["kappa"], m["alpha"])
    n = w["n"]
    h = (w["y_hi"] - w["y_lo"]) / (n - 1)
    d = integral.discretize(p, h, w["r"])
    return scheme.Problem(n, (w["y_lo"], w["y_lo"]), h, d, payoff=w["payoff"], K=w["K"], T=w["T"], N_t=w["N_t"],
                          theta=w["theta"])


@pytest.mark.parametrize("alpha,corr,C", [(0.5, 0.3, 32), (0.3, -0.4, 2), (0.5, 0.3, 8)])
def test_native_adjoint_matches_oracle(lp, alpha, corr, C):
    import torch
    w = workloads.workload("nig64", n=18, N_t=5, y_lo=-2.0, y_hi=2.0, alpha=alpha, corr=corr)
    _note("adjoint native vs oracle alpha=%g corr=%g C=%d" % (alpha, corr, C))
    prob = _oracle_problem(w)
    vbar = np.random.default_rng(5).standard_normal((w["n"], w["n"]))
    ref = oadj.adjoint(prob, vbar)
    plan = lp.plan_from_workload(w)
    _, native, info = plan.adjoint(torch.from_numpy(vbar).cuda(), checkpoint_every=C)
    Nz = prob.disc["N_z"]
    assert plan.info()["N_z"] == Nz
    g6 = native[:6]
    scale6 = np.maximum(np.abs(ref["native"]), 1e-3 * np.max(np.abs(ref["native"])))
    e6 = np.max(np.abs(g6 - ref["native"]) / scale6)
    gw = native[6:].reshape(2 * Nz, 2 * Nz)
    ew = np.max(np.abs(gw - ref["omega"])) / np.max(np.abs(ref["omega"]))
    _note("native rel err %.2e, omega rel err %.2e, adjoint iterations %d" % (e6, ew, info["adj_iters"]))
    assert e6 < 1e-8 and ew < 1e-8


def _fd_grad(lp, w, spots, wts, x0, nz, h_rel=1e-5):
    """Central differences of J = sum_k wts_k P_k with the structure fixed at N_z = nz."""
    out = np.zeros(8)
    for q in range(8):
        hq = h_rel * max(abs(x0[q]), 0.1)
        J = []
        for sgn in (1.0, -1.0):
            x = list(x0)
            x[q] += sgn * hq
            wq = workloads.workload("nig64", **{k: v for k, v in w.items() if k != "model"})
            wq["model"] = dict(w["model"], sigma1=x[0], sigma2=x[1], corr=x[2], theta1=x[3], theta2=x[4], kappa=x[5],
                               alpha=x[6])
            wq["r"] = x[7]
            plan = lp.plan_from_workload(wq, nz_fixed=nz)
            V = plan.solve()
            J.append(float(np.sum(wts * plan.price(V, spots).cpu().numpy())))
            del plan, V
        out[q] = (J[0] - J[1]) / (2 * hq)
    return out


def _adjoint_grad(lp, w, spots, wts, C=32):
    import torch
    plan = lp.plan_from_workload(w)
    plan.solve()                                  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    V = plan.solve()
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    plan.set_checkpoints(C)                       # the forward keeps the adjoint's checkpoints
    V = plan.solve()
    vbar = plan.price_adjoint(spots, wts)
    t0 = time.perf_counter()
    grad, native, info = plan.adjoint(vbar, checkpoint_every=C, std_params=lp.std_params_of(w))
    t_adj = time.perf_counter() - t0
    return plan, grad, info, t_fwd, t_adj


def test_grad_vs_finite_differences_small(lp):
    w = workloads.workload("nig64", n=40, N_t=8, y_lo=-2.5, y_hi=2.5)
    spots = workloads.spot_pairs(16, seed=4, lo=90.0, hi=110.0)
    wts = np.random.default_rng(4).standard_normal(16)
    _note("adjoint grad vs FD, 40x40")
    plan, grad, info, _, _ = _adjoint_grad(lp, w, spots, wts, C=4)
    fd = _fd_grad(lp, w, spots, wts, lp.std_params_of(w), plan.info()["N_z"])
    err = _per_component_err(grad, fd)
    _note("grad %s\nfd   %s\nrel err %s" % (np.array2string(grad, precision=8), np.array2string(fd, precision=8),
                                            np.array2string(err, precision=2)))
    assert np.all(err < 1e-5)


def _per_component_err(grad, fd):
    """|g - fd| relative to each component's own size, floored at 1e-2 of the
    largest, so that a small component is held to its own scale."""
    return np.abs(grad - fd) / np.maximum(np.abs(fd), 1e-2 * np.max(np.abs(fd)))


@pytest.mark.parametrize("device", ["cpu", "cuda"])
def test_autograd_prices(lp, device):
    import torch
    w = workloads.workload("nig64", n=40, N_t=8, y_lo=-2.5, y_hi=2.5)
    _note("autograd wrapper, inputs on %s" % device)
    spots = torch.tensor(workloads.spot_pairs(8, seed=6, lo=90.0, hi=110.0), dtype=torch.float64, device=device,
                         requires_grad=True)
    params = torch.tensor(lp.std_params_of(w), dtype=torch.float64, device=device, requires_grad=True)
    ga = dict(n=w["n"], y_lo=w["y_lo"], y_hi=w["y_hi"], N_t=w["N_t"], theta=w["theta"], tol=w["tol"],
              checkpoint_every=4)
    pa = dict(kind=w["payoff"], K=w["K"], T=w["T"])
    pr = lp.PricesFn.apply(params, spots, ga, pa)
    g = torch.linspace(0.5, 1.5, 8, dtype=torch.float64)
    (pr.cpu() * g).sum().backward()
    assert params.grad.device == params.device and spots.grad.device == spots.device
    sp = spots.detach().cpu().numpy()
    plan, grad, _, _, _ = _adjoint_grad(lp, w, sp, g.numpy(), C=4)
    assert np.max(np.abs(params.grad.cpu().numpy() - grad)) < 1e-9 * np.max(np.abs(grad))
    _, dl = plan.price(plan.solve(), sp, with_delta=True)
    assert np.max(np.abs(spots.grad.cpu().numpy() - g.numpy()[:, None] * dl.cpu().numpy())) < 1e-12


def test_adjoint_1024_vs_finite_differences(lp):
    """The adjoint workload: 1024 x 1024 on [-4, 4]^2, 512 steps, alpha = 0.4,
    checkpoints every 32 steps; J = sum of 64 seeded spot-pair prices with
    seeded weights."""
    w = workloads.workload("nts1024")
    spots = workloads.spot_pairs(64, seed=4)
    wts = np.random.default_rng(4).standard_normal(64)
    _note("adjoint 1024^2, 512 steps")
    plan, grad, info, t_fwd, t_adj = _adjoint_grad(lp, w, spots, wts, C=32)
    dev = info["forward_ms"] + info["recompute_ms"] + info["reverse_ms"] + info["gather_ms"]
    _note("forward %.1f ms; adjoint %.1f ms wall (march part %.1f ms = %.2f x forward: recompute %.1f, reverse %.1f, "
          "gather %.1f; host Jacobian %.1f ms); adjoint iterations %d, forward iterations %d" % (
              1e3 * t_fwd, 1e3 * t_adj, dev, dev / (1e3 * t_fwd), info["recompute_ms"], info["reverse_ms"],
              info["gather_ms"], info["jacobian_ms"], info["adj_iters"], plan.info()["total_iters"]))
    assert info["forward_ms"] == 0.0              # the solve's checkpoints were reused
    fd = _fd_grad(lp, w, spots, wts, lp.std_params_of(w), plan.info()["N_z"])
    err = _per_component_err(grad, fd)
    _note("grad %s\nfd   %s\nrel err %s" % (np.array2string(grad, precision=8), np.array2string(fd, precision=8),
                                            np.array2string(err, precision=2)))
    assert np.all(err < 1e-5)


def test_spot_deltas_1024_vs_finite_differences(lp):
    """Spot deltas of the 1024 x 1024 march (lpide_price) against central
    differences of lpide_price at spots bumped by 1e-5 S_i, same grid."""
    w = workloads.workload("nts1024")
    spots = workloads.spot_pairs(64, seed=4)
    _note("spot deltas vs FD, 1024^2")
    plan = lp.plan_from_workload(w)
    V = plan.solve()
    _, dl = plan.price(V, spots, with_delta=True)
    dl = dl.cpu().numpy()
    for i in (0, 1):
        hs = 1e-5 * spots[:, i]
        up, dn = spots.copy(), spots.copy()
        up[:, i] += hs
        dn[:, i] -= hs
        fd = (plan.price(V, up).cpu().numpy() - plan.price(V, dn).cpu().numpy()) / (2 * hs)
        err = float(np.max(np.abs(fd - dl[:, i])))
        _note("axis %d: max |delta - FD| %.2e (deltas %.3f .. %.3f)" % (i, err, dl[:, i].min(), dl[:, i].max()))
        assert err < 1e-5


def test_keep_every_state_equals_checkpoints(lp):
    """A checkpoint stride of at least the step count keeps every state and
    explicit part of the forward march and reverses it without recompute; the
    native gradient equals the one from checkpoints every 4 steps (both from
    the recording solve and from the adjoint's own forward pass)."""
    import torch
    w = workloads.workload("nig64", n=24, N_t=12, y_lo=-2.0, y_hi=2.0)
    _note("adjoint keep-all vs checkpoints")
    vbar = torch.from_numpy(np.random.default_rng(9).standard_normal((w["n"], w["n"]))).cuda()
    res = {}
    for C in (4, 1000):
        plan = lp.plan_from_workload(w)
        _, n_own, info_own = plan.adjoint(vbar, checkpoint_every=C)      # its own forward pass
        plan.set_checkpoints(C)
        plan.solve()
        _, n_rec, info_rec = plan.adjoint(vbar, checkpoint_every=C)      # the solve's records
        assert info_rec["forward_ms"] == 0.0
        if C == 1000:
            assert info_rec["recompute_ms"] < info_own["reverse_ms"]
        res[C] = (np.asarray(n_own), np.asarray(n_rec))
    scale = np.max(np.abs(res[4][0]))
    for a in res[1000] + res[4][1:]:
        assert np.max(np.abs(a - res[4][0])) / scale < 1e-11
