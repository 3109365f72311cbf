"""The learned surrogate on the GPU: BF16 forward/backward kernels against
the FP64 reference network, the Adam step, the input and target builders
against the oracle, the residual gate (forced fallback, accepted exact
predictions) and training on patches produced by the FP64 path.

Tolerances of the network kernels: BF16 weights, activations and output
gradients (unit roundoff 2^-9 relative per rounding, several roundings per
layer) against a float64 reference: relative L2 2e-2 per tensor.
"""

import numpy as np
import pytest

import inputs
from oracle import cnn as ocnn
from oracle.discretization import total_mobility
from tests.gpu_util import oracle_basis_padded, rel, run_oracle, say

pytestmark = pytest.mark.gpu

TOL_NET = 2e-2


def _torch():
    import torch
    return torch


def _net_inputs(B, seed):
    torch = _torch()
    rng = np.random.default_rng(seed)
    x = np.zeros((B, 256, 8), dtype=np.float32)
    x[:, :, 0] = rng.normal(0.0, 0.8, size=(B, 256))
    for ch, cells in ((1, np.arange(16) * 16), (2, np.arange(16) * 16 + 15), (3, np.arange(16)),
                      (4, 240 + np.arange(16))):
        x[:, cells, ch] = 1.0
    xt = torch.from_numpy(x).to(torch.bfloat16).cuda()
    return xt, xt.float().cpu().numpy().astype(np.float64)


def _net(max_batch=64, seed=3):
    from paper_2104_04653_amd import SurrogateNet
    return SurrogateNet(max_batch, seed=seed)


def _layers(v):
    """Split a parameter vector into (name, slice) pieces per layer."""
    out = []
    for i, (wo, cout, kp, cin, bo, _) in enumerate(ocnn.layout()[0]):
        out.append(("W%d" % (i + 1), slice(wo, wo + cout * kp)))
        out.append(("b%d" % (i + 1), slice(bo, bo + cout)))
    return out


def test_parameter_layout_and_initialisation():
    say("case: cnn parameter layout")
    net = _net()
    assert net.n_params == ocnn.n_params()
    p = net.params()
    wo, cout, kp, cin, bo, _ = ocnn.layout()[0][0]
    W1 = p[wo:wo + cout * kp].reshape(cout, kp)
    assert np.all(W1[:, 72:] == 0.0)                               # padded tap
    assert np.all(W1[:, :72].reshape(cout, 9, 8)[:, :, 5:] == 0.0)  # padded channels
    for _, sl in _layers(p)[1::2]:
        assert np.all(p[sl] == 0.0)                                # zero biases
    std = p[_layers(p)[2][1]].std()
    assert 0.5 * np.sqrt(2 / 288) < std < 2.0 * np.sqrt(2 / 288)  # He-normal scale
    q = ocnn.he_params(4).astype(np.float32)
    net.set_params(q)
    np.testing.assert_array_equal(net.params(), q)
    net.close()


def test_forward_matches_fp64_reference():
    say("case: cnn forward vs fp64 reference")
    torch = _torch()
    net = _net()
    p = ocnn.he_params(11).astype(np.float32)
    net.set_params(p)
    xt, x = _net_inputs(12, 5)
    y = net.forward(xt).cpu().numpy()
    ref = ocnn.forward(p.astype(np.float64), x)
    e = rel(y, ref)
    say("  forward rel L2 %.2e" % e)
    assert e < TOL_NET
    assert torch.isfinite(torch.from_numpy(y)).all()
    net.close()


def test_loss_and_gradients_match_fp64_reference():
    say("case: cnn loss/gradients vs fp64 reference")
    torch = _torch()
    net = _net()
    p = ocnn.he_params(12).astype(np.float32)
    net.set_params(p)
    xt, x = _net_inputs(16, 6)
    t = np.random.default_rng(7).normal(0.0, 0.5, size=(16, 256, 16)).astype(np.float32)
    L, g = net.loss_grad(xt, torch.from_numpy(t).cuda())
    Lr, gr = ocnn.loss_grad(p.astype(np.float64), x, t.astype(np.float64))
    say("  loss gpu %.6e  ref %.6e" % (L, Lr))
    assert abs(L - Lr) <= TOL_NET * Lr
    for name, sl in _layers(g):
        e = rel(g[sl], gr[sl])
        say("  grad %-3s rel L2 %.2e" % (name, e))
        assert e < TOL_NET, name
    # padded entries receive no gradient
    wo, cout, kp, cin, bo, _ = ocnn.layout()[0][0]
    W1 = g[wo:wo + cout * kp].reshape(cout, kp)
    assert np.all(W1[:, 72:] == 0.0)
    # the same batch gives the same gradient bit for bit (fixed-order reductions)
    L2, g2 = net.loss_grad(xt, torch.from_numpy(t).cuda())
    assert L2 == L and np.array_equal(g2, g)
    net.close()


def test_adam_step_and_training_reduce_the_loss():
    say("case: adam step + short training on a fixed batch")
    torch = _torch()
    net = _net()
    xt, _ = _net_inputs(32, 8)
    t = torch.from_numpy(np.random.default_rng(9).normal(0.0, 0.3, size=(32, 256, 16))
                         .astype(np.float32)).cuda()
    p0 = net.params()
    L0, g = net.loss_grad(xt, t)
    lr = 1e-3
    net.train_step(xt, t, lr)
    p1 = net.params()
    # first Adam step: m_hat = g, v_hat = g^2
    expect = p0 - lr * g / (np.abs(g).astype(np.float64) + 1e-8)
    live = np.abs(g) > 1e-6
    np.testing.assert_allclose(p1[live], expect[live], rtol=1e-5, atol=1e-7)
    assert np.array_equal(p1[~live & (g == 0)], p0[~live & (g == 0)])
    losses = [net.train_step(xt, t, lr) for _ in range(60)]
    say("  loss %.4e -> %.4e" % (L0, losses[-1]))
    assert losses[-1] < 0.5 * L0
    net.close()


def _prob_and_lam(seed=2, **over):
    prob = inputs.make_problem("gauss64", seed=seed, **over)
    s = inputs.synthetic_saturation(prob, 3, 10)
    return prob, s, total_mobility(s, prob.mu_w, prob.mu_o)


def test_inputs_and_targets_match_oracle():
    say("case: surrogate inputs/targets vs oracle (gauss64)")
    from paper_2104_04653_amd import MRCMSolver
    prob, s, lam = _prob_and_lam()
    with MRCMSolver(prob, precision="fp64") as sol:
        sol.update_mobility(s)
        sol.solve()
        xin = sol.surrogate_inputs().float().cpu().numpy()
        tgt = sol.surrogate_targets().cpu().numpy()
    ref = run_oracle(prob, lam=lam)
    Xo = oracle_basis_padded(prob, ref)               # [sd][cell][17]
    kap = prob.perm * lam
    SX, SY = prob.nx // 16, prob.ny // 16
    li, lj = np.meshgrid(np.arange(16), np.arange(16))
    for sd in range(SX * SY):
        I, J = sd % SX, sd // SX
        cells = ((J * 16 + lj) * prob.nx + I * 16 + li).ravel()
        lk = np.log(kap[cells])
        z = (lk - lk.mean()) / 4.0
        assert np.all(np.abs(xin[sd, :, 0] - z) <= 2.0 ** -8 * 1.001 * np.abs(z) + 1e-30)
        has = [I > 0, I < SX - 1, J > 0, J < SY - 1]
        masks = [li.ravel() == 0, li.ravel() == 15, lj.ravel() == 0, lj.ravel() == 15]
        for side in range(4):
            np.testing.assert_array_equal(xin[sd, :, 1 + side], (masks[side] & has[side]) * 1.0)
        assert np.all(xin[sd, :, 5:] == 0.0)
        kg = np.exp(lk.mean())
        for q in range(16):
            side, k = divmod(q, 4)
            H = 16 * (prob.hy if side < 2 else prob.hx)
            scale = 1.0 if k < 2 else kg / (prob.alpha * H)
            want = Xo[sd][:, 1 + q] * scale
            assert np.allclose(tgt[sd, :, q], want, rtol=2e-7, atol=1e-7 * np.abs(want).max() + 1e-30)


def _particular_subdomains(prob):
    """Subdomains with source or non-zero physical boundary data."""
    SX, SY = prob.nx // 16, prob.ny // 16
    out = set()
    src = None if prob.source is None else prob.source.reshape(prob.ny, prob.nx)
    for sd in range(SX * SY):
        I, J = sd % SX, sd // SX
        if src is not None and np.any(src[J * 16:(J + 1) * 16, I * 16:(I + 1) * 16] != 0):
            out.add(sd)
        for side, touch in enumerate([I == 0, I == SX - 1, J == 0, J == SY - 1]):
            v = prob.bc_value[side]
            if touch and prob.bc_kind[side] == 1 and v is not None and np.any(np.asarray(v) != 0):
                out.add(sd)
    return out


def _run(prob, s, precision, net=None, pred=None, tol=None):
    from paper_2104_04653_amd import MRCMSolver
    with MRCMSolver(prob, precision=precision) as sol:
        sol.update_mobility(s)
        if tol is not None:
            sol.set_gate_tolerance(tol)
        if pred is not None:
            sol.solve_with_predictions(pred)
        else:
            if net is not None:
                sol.set_surrogate(net)
            sol.solve()
        p, ux, uy, imb = sol.fine_flux()
        out = {"p": p, "f": np.r_[ux, uy], "stats": sol.stats(), "imb": imb,
               "coef": sol.interface_solution()}
        if precision == "fp64":
            out["targets"] = sol.surrogate_targets()
    return out


def test_gate_rejects_random_network_and_equals_fp64():
    say("case: gate with an untrained network (all subdomains fall back)")
    prob, s, _ = _prob_and_lam()
    net = _net(seed=21)
    a = _run(prob, s, "surrogate", net=net)
    b = _run(prob, s, "fp64")
    st = a["stats"]
    say("  fallbacks %d of %d, ms_surrogate %.3f" % (st["fallbacks"], st["n_sub"], st["ms_surrogate"]))
    assert st["fallbacks"] == st["n_sub"]
    for k in ("p", "f", "coef"):
        assert np.array_equal(a[k], b[k]), k
    net.close()


def test_gate_accepts_exact_predictions():
    """FP32 copies of the FP64 basis functions (the network's output form)
    pass the default 1e-6 gate once the gate's FP64 relaxation sweeps have
    removed their rounding noise; only subdomains with particular data fall
    back.  The result carries the accepted residual (about 1e-7), and the
    cell balance holds to it, not to FP64 rounding."""
    say("case: gate with exact FP32 predictions (gauss64)")
    torch = _torch()
    prob, s, lam = _prob_and_lam()
    b = _run(prob, s, "fp64")
    pred = b["targets"]
    part = _particular_subdomains(prob)
    for tol in (1e-6, 1e-4):
        a = _run(prob, s, "surrogate", pred=pred, tol=tol)
        st = a["stats"]
        ep, ef = rel(a["p"], b["p"]), rel(a["f"], b["f"])
        say("  tol %.0e: fallbacks %d (particular data: %d) of %d; vs FP64: p %.2e flux %.2e "
            "imbalance %.2e" % (tol, st["fallbacks"], len(part), st["n_sub"], ep, ef, a["imb"]))
        assert st["fallbacks"] == len(part)
        assert ep < 1e-6 and ef < 1e-6
        # an accepted subdomain's local mass balance holds only up to its
        # residual; the stitch spreads that defect over the subdomain's cells
        assert a["imb"] < 1e-6
    # predictions with a smooth relative error of 1e-3 (the kind of error a
    # network makes, which relaxation does not remove) fail everywhere
    n, cells = pred.shape[0], pred.shape[1]
    ramp = torch.linspace(-1.0, 1.0, cells, device=pred.device, dtype=pred.dtype)[None, :, None]
    off = (pred * (1.0 + 1e-3 * ramp)).contiguous()
    d = _run(prob, s, "surrogate", pred=off, tol=1e-4)
    say("  smooth 1e-3 error at tol 1e-4: fallbacks %d of %d" % (d["stats"]["fallbacks"], n))
    assert d["stats"]["fallbacks"] == d["stats"]["n_sub"]
    assert np.array_equal(d["p"], b["p"])


def test_training_on_method_patches_and_gain():
    """Train on patches the FP64 path produces (log-normal and channelized
    fields), check that the loss falls on held-out patches, then report
    what the trained network gains on a 256 x 256 two-phase step: ms and
    error against the FP64 path, and the fallback rate (sign included)."""
    say("case: training on FP64 patches + gain report")
    from paper_2104_04653_amd import surrogate
    cases = []
    for seed in range(4):
        prob = inputs.make_problem("gauss1024", seed=100 + seed, nx=256, ny=256, lx=0.25, ly=0.25)
        cases.append((prob, inputs.synthetic_saturation(prob, seed, 4)))
    prob = inputs.make_problem("channel256_q5", seed=7)
    cases.append((prob, inputs.synthetic_saturation(prob, 2, 4)))
    x, y = surrogate.method_patches(cases)
    say("  %d patches" % x.shape[0])
    n_hold = 256
    xtr, ytr, xho, yho = x[n_hold:], y[n_hold:], x[:n_hold], y[:n_hold]
    net = _net(max_batch=256, seed=5)
    e0 = surrogate.evaluate(net, xho, yho)
    losses = surrogate.train(net, xtr, ytr, steps=400, batch=128, lr=2e-3, lr_final=2e-4)
    e1 = surrogate.evaluate(net, xho, yho)
    say("  held-out mse %.4e -> %.4e (train batch loss %.4e -> %.4e)"
        % (e0, e1, losses[0], losses[-1]))
    assert e1 < 0.5 * e0
    # gain on an unseen field, at the 1e-6 gate and at looser gates
    tprob = inputs.make_problem("gauss1024", seed=999, nx=256, ny=256, lx=0.25, ly=0.25)
    ts = inputs.synthetic_saturation(tprob, 1, 4)
    ref = _run(tprob, ts, "fp64")
    t0 = ref["stats"]["ms_local"] + ref["stats"]["ms_interface"]
    prev = None
    for tol in (1e-6, 1e-3, 1e-1):
        sur = _run(tprob, ts, "surrogate", net=net, tol=tol)
        st1 = sur["stats"]
        t1 = st1["ms_local"] + st1["ms_interface"]
        rate = st1["fallbacks"] / st1["n_sub"]
        ep, ef = rel(sur["p"], ref["p"]), rel(sur["f"], ref["f"])
        say("  gate %.0e: FP64 solve %.3f ms, surrogate solve %.3f ms (inference+gate %.3f ms), "
            "fallbacks %d of %d (%.1f%%), gain %+.3f ms; error vs FP64: p %.2e flux %.2e"
            % (tol, t0, t1, st1["ms_surrogate"], st1["fallbacks"], st1["n_sub"], 100.0 * rate,
               t0 - t1, ep, ef))
        # a looser gate accepts at least what a tighter one did
        if prev is not None:
            assert st1["fallbacks"] <= prev
        prev = st1["fallbacks"]
        if st1["fallbacks"] == st1["n_sub"]:
            # nothing accepted: the FP64 result, bit for bit, reached with
            # strictly more work (inference and gate before the same solve)
            assert np.array_equal(sur["p"], ref["p"])
            assert t1 > t0
        if tol == 1e-6:
            assert ep < 1e-5
    net.close()
