"""GPU tests of the learned warm start: the bf16 matrix-core network against the
FP64 reference (oracle/unet.py) run at the same storage precision, its
gradients, training, and the warm-started Poisson solve."""
import numpy as np
import pytest
import torch

from oracle import unet as OU

pytestmark = pytest.mark.gpu

# Normwise tolerances for random weights. Both sides round the same weights
# and every stored activation to bf16 (and the reference rounds the gradient
# where the GPU's matrix products read it); they differ by the accumulation
# (fp32 against fp64), which moves an activation across a bf16 rounding
# boundary now and then (one ulp, 2^-8 relative) and, near zero, across a
# ReLU kink. The output stays within 1e-2. The weight gradients of the deep
# levels are sums over a few voxels in which such flips do not average out
# (up to 15 % measured on a 2 x 16 x 8 x 16 input); with exact arithmetic
# (test_exact_arithmetic_wiring) every tensor agrees to 1e-7, so the loose
# bound here only guards against gross errors.
TOL_FWD = 1e-2
TOL_GRAD = 0.25


def layer_slices():
    out = []
    o = 0
    for i, (kind, cin, cout) in enumerate(OU.layer_table(16)):
        nw = (27 if kind == "conv3" else 8) * cin * cout
        out.append((f"{i}:{kind}.w", slice(o, o + nw)))
        out.append((f"{i}:{kind}.b", slice(o + nw, o + nw + cout)))
        o += nw + cout
    out.append(("head.w", slice(o, o + 16)))
    out.append(("head.b", slice(o + 16, o + 17)))
    return out


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("shape", [(2, 16, 16, 24), (1, 8, 8, 8)])
def test_forward_parity(shape):
    from paper_2402_08404_amd import pic
    print("forward", shape, flush=True)
    net = pic.UNet(*shape, seed=1)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(shape).astype(np.float32)
    y = net.forward(torch.tensor(x)).cpu().numpy()
    p = net.params.cpu().numpy().astype(np.float64)
    ref = OU.forward_np(p, x.astype(np.float64), bf16=True)
    assert np.all(np.isfinite(y))
    assert relerr(y, ref) < TOL_FWD, relerr(y, ref)
    net.close()


def test_gradient_parity():
    from paper_2402_08404_amd import pic
    shape = (2, 16, 8, 16)
    net = pic.UNet(*shape, seed=3)
    rng = np.random.default_rng(4)
    x = rng.standard_normal(shape).astype(np.float32)
    tg = rng.standard_normal(shape).astype(np.float32)
    loss, g = net.gradients(torch.tensor(x), torch.tensor(tg))
    g = g.cpu().numpy().astype(np.float64)
    p = net.params.cpu().numpy().astype(np.float64)
    rloss, rg, _ = OU.loss_and_grad(p, x.astype(np.float64), tg.astype(np.float64), bf16=True, bf16_grad=True)
    _, rg64, _ = OU.loss_and_grad(p, x.astype(np.float64), tg.astype(np.float64), bf16=True)
    assert loss == pytest.approx(rloss, rel=TOL_FWD)
    bad = []
    for name, sl in layer_slices():
        e = relerr(g[sl], rg[sl])
        print(f"{name:12s} vs rounded-gradient reference {e:.2e}, vs fp64 gradient {relerr(g[sl], rg64[sl]):.2e}, "
              f"reference pair {relerr(rg[sl], rg64[sl]):.2e}")
        if not e < TOL_GRAD:
            bad.append((name, e))
    assert not bad, bad
    net.close()


def sparse_dyadic_params(rng, n_params, density=0.03):
    """Weights in {0, +-1/2, +-1/4} (mostly zero), biases in multiples of
    1/16: with inputs on a 1/16 grid every sum either side forms is exact in
    fp32, so both sides round the same values to bf16 and any difference is a
    wiring or indexing error, not arithmetic."""
    p = np.zeros(n_params)
    o = 0
    for kind, cin, cout in OU.layer_table(16):
        nw = (27 if kind == "conv3" else 8) * cin * cout
        w = rng.choice([0.5, -0.5, 0.25, -0.25], size=nw) * (rng.random(nw) < density)
        p[o:o + nw] = w
        p[o + nw:o + nw + cout] = rng.integers(-4, 5, size=cout) / 16.0
        o += nw + cout
    p[o:o + 16] = rng.choice([0.5, -0.5, 0.25, 1.0], size=16)
    p[o + 16] = 0.125
    return p.astype(np.float32)


@pytest.mark.parametrize("shape", [(2, 16, 8, 16), (1, 32, 16, 8)])
def test_exact_arithmetic_wiring(shape):
    """Forward and every gradient tensor on inputs where the arithmetic is
    exact: agreement to rounding of the final fp32 sums."""
    from paper_2402_08404_amd import pic
    rng = np.random.default_rng(11)
    n = OU.n_params(16)
    p = sparse_dyadic_params(rng, n)
    net = pic.UNet(*shape, params=torch.tensor(p))
    x = (rng.integers(-32, 33, size=shape) / 16.0).astype(np.float32)
    tg = (rng.integers(-32, 33, size=shape) / 16.0).astype(np.float32)
    y = net.forward(torch.tensor(x)).cpu().numpy()
    ref = OU.forward_np(p.astype(np.float64), x.astype(np.float64), bf16=True)
    assert relerr(y, ref) < 1e-6, relerr(y, ref)
    loss, g = net.gradients(torch.tensor(x), torch.tensor(tg))
    g = g.cpu().numpy().astype(np.float64)
    rloss, rg, _ = OU.loss_and_grad(p.astype(np.float64), x.astype(np.float64), tg.astype(np.float64), bf16=True,
                                    bf16_grad=True)
    assert loss == pytest.approx(rloss, rel=1e-6)
    bad = []
    for name, sl in layer_slices():
        e = relerr(g[sl], rg[sl])
        print(f"{name:12s} {e:.2e} |g| {np.linalg.norm(rg[sl]):.3e}")
        if not (e < 1e-4 or np.linalg.norm(rg[sl]) == 0 and np.linalg.norm(g[sl]) == 0):
            bad.append((name, e))
    assert not bad, bad
    net.close()


def test_training_reduces_loss():
    from paper_2402_08404_amd import pic
    shape = (2, 16, 16, 16)
    net = pic.UNet(*shape, seed=5)
    rng = np.random.default_rng(6)
    x = torch.tensor(rng.standard_normal(shape).astype(np.float32))
    # a smooth target the network can fit: a blurred copy of the input
    t = x.clone()
    for ax in (1, 2, 3):
        t = 0.5 * t + 0.25 * (torch.roll(t, 1, ax) + torch.roll(t, -1, ax))
    losses = [net.train_step(x, t, 2e-3) for _ in range(60)]
    assert losses[-1] < 0.3 * losses[0], (losses[0], losses[-1])
    # a second network over the same parameters sees the trained weights
    net2 = pic.UNet(*shape, params=net.params)
    y1 = net.forward(x)
    y2 = net2.forward(x)
    torch.testing.assert_close(y1, y2, rtol=0, atol=0)
    net.close()
    net2.close()


def test_learned_guess_solve():
    """Train on pairs of the small 32 x 32 x 64 workload at several apex
    fields, then solve a held-out state from the learned guess. The raw
    network guess must carry most of the charge response (its error against
    the converged potential well below that of the charge-free guess V0
    phi1); with the energy-norm projection the guess error, measured with the
    oracle's operator, must not exceed that of V0 phi1 or of the raw guess;
    the solve from it must end at the plain solve's result. Iteration counts
    of both solvers from every guess are printed; the gain in iterations is a
    measurement, not asserted."""
    import dataclasses
    from paper_2402_08404_amd import pic, warmstart
    from paper_2402_08404_amd import workloads as W
    base = W.tiny()
    X, Y = warmstart.collect_samples(base, fields=[7e9, 9e9, 11e9, 13e9], per_field=4, steps_between=15,
                                     counts=(20000, 200, 2000))
    print("samples", X.shape, float(X.abs().max()), float(Y.abs().max()), flush=True)
    train_net = pic.UNet(4, base.nz, base.ny, base.nx, seed=7)
    losses = warmstart.train(train_net, X, Y, iters=400, lr=3e-4, lr_final=5e-5)
    print("loss", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.05 * losses[0]
    guess_net = pic.UNet(1, base.nz, base.ny, base.nx, params=train_net.params)
    guess_net.sync()
    cfg = dataclasses.replace(base, apex_field=10e9, seed=123)
    sim = pic.Simulation(cfg, caps=(200000, 20000, 8000), precision=pic.PIC_F64)
    sim.load(W.initial_load(cfg, counts=(20000, 200, 2000), seed=321))
    sim.step(1, pic.STEP_DEPOSIT)
    sim.step(20, pic.STEP_FULL)
    pic.pic_set_learned_guess(sim.ctx, guess_net.net, 0, False)
    sim.solve(solver=pic.PIC_SOLVER_CG, guess=pic.PIC_GUESS_ZERO, rtol=1e-12, maxit=100000)
    exact = sim.grid("phi").copy()
    guesses = {}
    for name, g, proj in (("laplace", pic.PIC_GUESS_LAPLACE, False), ("learned_raw", pic.PIC_GUESS_LEARNED, False),
                          ("learned", pic.PIC_GUESS_LEARNED, True)):
        # the guesses themselves, without the fallback judge
        pic.pic_set_learned_guess(sim.ctx, guess_net.net, 0, proj, fallback=False)
        sim.solve(solver=pic.PIC_SOLVER_CG, guess=g, rtol=1e-12, maxit=0, allow_unconverged=True)
        guesses[name] = sim.grid("phi").copy()
    resp = np.linalg.norm(exact - guesses["laplace"])
    err = np.linalg.norm(guesses["learned_raw"] - exact) / resp
    print("relative error of the learned charge response", err, flush=True)
    assert err < 0.25
    # energy norm of the error from the oracle's operator: the projected
    # weight can only lower it below that of V0 phi1
    from oracle import Oracle
    o = Oracle(cfg, laplace=False)
    free = (o.type == 0)

    def energy(phi):
        e = (phi.ravel() - exact.ravel()) * free
        return float(e @ o.apply_A(e))

    en = {k: energy(v) for k, v in guesses.items()}
    print("energy norm^2 of the guess errors", en, flush=True)
    assert en["learned"] <= en["laplace"] * (1 + 1e-9)
    assert en["learned"] <= en["learned_raw"] * (1 + 1e-9)
    res = {}
    for solver in (pic.PIC_SOLVER_CG, pic.PIC_SOLVER_MGCG):
        for name, g, sm, proj in (("zero", pic.PIC_GUESS_ZERO, 0, True), ("laplace", pic.PIC_GUESS_LAPLACE, 0, True),
                                  ("learned_raw", pic.PIC_GUESS_LEARNED, 0, False),
                                  ("learned", pic.PIC_GUESS_LEARNED, 0, True),
                                  ("learned+2", pic.PIC_GUESS_LEARNED, 2, True)):
            pic.pic_set_learned_guess(sim.ctx, guess_net.net, sm, proj)
            r = sim.solve(solver=solver, guess=g, rtol=1e-8, maxit=100000)
            res[(solver, name)] = (r["iterations"], round(r["relres0"], 4), r["fell_back"])
            phi = sim.grid("phi")
            assert np.linalg.norm(phi - exact) < 1e-5 * np.linalg.norm(exact)
    print("iterations (solver, guess) -> (iterations, initial relative residual)", res, flush=True)
    pic.pic_set_learned_guess(sim.ctx, None)
    sim.close()
    guess_net.close()
    train_net.close()


@pytest.mark.parametrize("fill", ["nan", "zero"])
def test_learned_guess_fallback(fill):
    """Plain CG judges the learned guess: a network whose weights are NaN gives
    a non-finite output, the solve falls back to V0 phi1 (fell_back), starts
    from its residual and converges to the plain tolerance in the iterations of
    the plain solve from V0 phi1; a network with zero weights gives the
    guess V0 phi1 itself, which is not worse, so nothing falls back."""
    from paper_2402_08404_amd import pic
    from paper_2402_08404_amd import workloads as W
    cfg = W.tiny()
    sim = pic.Simulation(cfg, caps=(100000, 10000, 4000), precision=pic.PIC_F64)
    sim.load(W.initial_load(cfg, counts=(20000, 200, 2000), seed=4))
    sim.step(1, pic.STEP_DEPOSIT)
    p = np.full(pic.UNet(1, cfg.nz, cfg.ny, cfg.nx).n_params, np.nan if fill == "nan" else 0.0, np.float32)
    net = pic.UNet(1, cfg.nz, cfg.ny, cfg.nx, params=p)
    net.sync()
    plain = sim.solve(solver=pic.PIC_SOLVER_CG, guess=pic.PIC_GUESS_LAPLACE, rtol=1e-8, maxit=100000)
    phi_plain = sim.grid("phi").copy()
    for project in (True, False):
        pic.pic_set_learned_guess(sim.ctx, net.net, 0, project)
        r = sim.solve(solver=pic.PIC_SOLVER_CG, guess=pic.PIC_GUESS_LEARNED, rtol=1e-8, maxit=100000)
        print(fill, project, r, plain, flush=True)
        assert r["converged"] and r["relres"] <= 1e-8
        assert r["fell_back"] == (fill == "nan")
        assert r["relres0"] == pytest.approx(plain["relres0"], rel=1e-12)
        assert r["iterations"] == plain["iterations"]
        phi = sim.grid("phi")
        assert np.all(np.isfinite(phi))
        assert np.abs(phi - phi_plain).max() <= 1e-12 * np.abs(phi_plain).max()
    pic.pic_set_learned_guess(sim.ctx, None)
    sim.close()
    net.close()
