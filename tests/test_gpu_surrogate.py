"""GPU parity of the surrogate network (BF16 MFMA kernels) against the FP64 CPU reference with the
same BF16 rounding points, training progress, and the surrogate-with-fallback against the solver."""
import time

import numpy as np
import pytest
import torch

from oracle import mlp as M
from paper_2408_00559_amd import inputs as I
from paper_2408_00559_amd import surrogate as S

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _setup(seed=3, B=200):
    net = S.Mlp(n_in=8, width=256, depth=3, max_batch=1024, seed=seed, device=DEV)
    rng = np.random.default_rng(seed)
    mean = rng.normal(size=8).astype(np.float32)
    std = rng.uniform(0.5, 2.0, 8).astype(np.float32)
    net.set_normalization(mean, std, 0.02, 0.01)
    x = (mean + std * rng.normal(size=(B, 8))).astype(np.float32)
    lay = M.Layout(*net.layout())
    return net, lay, x, mean, std


def test_forward_matches_reference():
    net, lay, x, mean, std = _setup()
    out = net.forward(torch.tensor(x)).cpu().numpy()
    p = net.params().cpu().numpy().astype(np.float64)
    y, _ = M.forward(lay, p, x, mean, std, bf16=True)
    price = y[:, 0] * 0.01 + 0.02
    err = np.exp(y[:, 1]) * 0.01 / np.abs(price)
    assert np.max(np.abs(out[:, 0] - price)) < 2e-3 * np.max(np.abs(price))
    assert np.max(np.abs(np.log(out[:, 1]) - np.log(err))) < 2e-2


def test_forward_log_target_matches_reference():
    """Log-price target mode: price = exp(y0 s + m), relative error estimate = exp(y1) s."""
    net, lay, x, mean, std = _setup(seed=4)
    net.set_normalization(mean, std, -4.0, 0.5, out_log=True)
    out = net.forward(torch.tensor(x)).cpu().numpy()
    p = net.params().cpu().numpy().astype(np.float64)
    y, _ = M.forward(lay, p, x, mean, std, bf16=True)
    price = np.exp(y[:, 0] * 0.5 - 4.0)
    err = np.exp(y[:, 1]) * 0.5
    assert np.max(np.abs(out[:, 0] - price) / price) < 2e-3
    assert np.max(np.abs(np.log(out[:, 1]) - np.log(err))) < 2e-2


@pytest.mark.parametrize("out_log", [False, True])
def test_infer_matches_forward_and_reference(out_log):
    """amf_mlp_infer (one launch, activations in LDS, any batch) gives the outputs of the training
    forward pass: the same BF16 rounding points and MFMA accumulation order, so equal to FP32
    rounding; a batch above max_batch and not a multiple of the 64-request workgroup; and it matches
    the FP64 reference as the forward pass does."""
    net, lay, x, mean, std = _setup(seed=6, B=2500)
    if out_log:
        net.set_normalization(mean, std, -4.0, 0.5, out_log=True)
    xt = torch.tensor(x)
    fwd = torch.cat([net.forward(xt[i:i + 1000]) for i in range(0, 2500, 1000)]).cpu().numpy()
    inf = net.infer(xt).cpu().numpy()
    assert np.max(np.abs(inf - fwd) / np.maximum(np.abs(fwd), 1e-30)) < 1e-6
    p = net.params().cpu().numpy().astype(np.float64)
    y, _ = M.forward(lay, p, x[:300], mean, std, bf16=True)
    price = np.exp(y[:, 0] * 0.5 - 4.0) if out_log else y[:, 0] * 0.01 + 0.02
    assert np.max(np.abs(inf[:300, 0] - price)) < 2e-3 * np.max(np.abs(price))


def test_gradients_match_reference():
    net, lay, x, mean, std = _setup(seed=5, B=96)
    rng = np.random.default_rng(7)
    dy = rng.normal(size=(x.shape[0], 2)).astype(np.float32)
    net.forward(torch.tensor(x))
    net.backward(torch.tensor(dy))
    g = net.grads().cpu().numpy().astype(np.float64)
    p = net.params().cpu().numpy().astype(np.float64)
    y, cache = M.forward(lay, p, x, mean, std, bf16=True)
    gr = M.backward(lay, cache, dy, bf16=True)
    # Both sides round the same activations to BF16 (8 significant bits), but from sums taken in a
    # different order (FP32 MFMA vs FP64), so an activation whose value lies near a rounding boundary
    # can round one BF16 ulp (2^-8) apart and move the gradient entries it feeds.  Such flips are
    # rare and isolated: on these inputs the blocks agree to better than 1e-4 in the 2-norm and
    # 2e-4 of the largest entry; the bounds below leave a factor of about ten.
    for l in range(lay.layers):
        for off, size in ((lay.w_off[l], lay.rows[l] * lay.cols[l]), (lay.b_off[l], lay.rows[l])):
            a, b = g[off:off + size], gr[off:off + size]
            scale = np.max(np.abs(b)) + 1e-30
            norm_rel = np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-30)
            print("layer %d block of %d: max %.2e, 2-norm %.2e" % (l, size, np.max(np.abs(a - b)) / scale,
                                                                 norm_rel))
            assert norm_rel < 1e-3, (l, norm_rel)
            assert np.max(np.abs(a - b)) < 2e-3 * scale, (l, np.max(np.abs(a - b)) / scale)


def test_training_reduces_loss():
    net = S.Mlp(n_in=8, width=256, depth=3, max_batch=2048, seed=11, device=DEV)
    rng = np.random.default_rng(11)
    x = rng.uniform(-1, 1, (4096, 8)).astype(np.float32)
    t = (np.sin(x[:, 0] * 2) + x[:, 1] * x[:, 2] + 0.5 * x[:, 3] ** 2).astype(np.float32)
    net.set_normalization(np.zeros(8), np.ones(8), float(t.mean()), float(t.std()))
    xt = torch.tensor(x, device=DEV)
    tt = torch.tensor(t, device=DEV)
    loss = torch.zeros(1, device=DEV)
    first = None
    for k in range(2000):
        i = k % 4
        net.train_step(xt[i * 1024:(i + 1) * 1024].contiguous(), tt[i * 1024:(i + 1) * 1024].contiguous(),
                       2e-3 if k < 1500 else 2e-4, 0.0, loss)
        if first is None:
            first = loss.item()
    pred = net.forward(xt).cpu().numpy()[:, 0]
    rmse = float(np.sqrt(np.mean((pred - t) ** 2)))
    assert loss.item() < 0.05 * first and rmse < 0.05 * t.std(), (first, loss.item(), rmse)


def test_surrogate_gain_with_fallback():
    """Trained on solver prices (d = 4, n = 4, psi = 1, 20 steps), the surrogate serves held-out
    requests much faster than the solver; requests above the error tolerance go to the solver, so
    every returned price is either the solver's or within the tolerance of it."""
    grid, steps = I.combination(4, 1), 20
    train = I.draw_instances(3072, seed=50, d=4, T_range=(0.5, 1.5), lam_range=(0.05, 0.3))
    cal = I.draw_instances(512, seed=52, d=4, T_range=(0.5, 1.5), lam_range=(0.05, 0.3))
    held = I.draw_instances(512, seed=51, d=4, T_range=(0.5, 1.5), lam_range=(0.05, 0.3))
    ytr = S.solver_prices(train, grid, steps)
    sur = S.Surrogate.train(S.features(train), ytr, grid, steps, epochs=300, batch=512, device=DEV)
    sur.calibrate(S.features(cal), S.solver_prices(cal, grid, steps))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    yref = S.solver_prices(held, grid, steps)
    t_solver = time.perf_counter() - t0
    tol = 3e-2
    xh = S.features(held)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pn, est = sur.predict(xh)
    t_net = time.perf_counter() - t0
    p, used, _ = sur.price(held, tol=tol)
    # the library's routing equals the rule written out here, decision for decision (in FP32, the
    # precision the library decides in): inside the training box, finite, calibrated estimate
    # within the relative tolerance
    f32 = np.float32
    inside = np.all((xh.astype(f32) >= sur.box_lo.astype(f32)) & (xh.astype(f32) <= sur.box_hi.astype(f32)), axis=1)
    e32 = f32(sur.calib) * est.astype(f32)
    expect = ~(inside & np.isfinite(pn) & np.isfinite(e32) & (e32 <= f32(tol)))
    assert np.array_equal(used, expect)
    np.testing.assert_allclose(p[~used], pn[~used].astype(np.float32).astype(np.float64), rtol=0, atol=0)
    rel = np.abs(p - yref) / np.abs(yref)
    served = ~used
    assert served.sum() > 0
    # the network alone is far cheaper than the solver on the same requests
    assert t_net < 0.2 * t_solver, (t_net, t_solver)
    # fallback prices are the solver's
    assert np.max(rel[used], initial=0.0) < 1e-6
    # the calibrated error estimate is an honest filter: served prices meet the tolerance up to the
    # calibration quantile
    assert np.quantile(rel[served], 0.9) < tol, np.quantile(rel[served], 0.9)
    # the absolute floor: e |p| <= abs_floor also serves a request (decided in FP32 as above), so at
    # a tight relative tolerance the floor serves more requests, never fewer
    _, used_t, _ = sur.price(held, tol=1e-4)
    _, used_f, _ = sur.price(held, tol=1e-4, abs_floor=3e-4)
    floor_ok = e32 * np.abs(pn.astype(f32)) <= f32(3e-4)
    assert np.array_equal(used_f, ~(inside & np.isfinite(pn) & np.isfinite(e32) & ((e32 <= f32(1e-4)) | floor_ok)))
    assert np.all(used_f <= used_t) and used_f.sum() < used_t.sum()
    # requests outside the training box (maturity beyond its range) always go to the solver
    outside = I.draw_instances(8, seed=53, d=4, T_range=(2.0, 2.5), lam_range=(0.05, 0.3))
    po, used_o, _ = sur.price(outside, tol=1.0)
    assert used_o.all()
    yo = S.solver_prices(outside, grid, steps)
    assert np.max(np.abs(po - yo) / np.abs(yo)) < 1e-6
