"""GPU: the learned stale fill (include/fibar_fill.h, through the C ABI)
against the FP64 reference (oracle/fill.py): forward, loss and the gradient of
every layer at BF16 tolerance, Adam's update, the per-tile fallback, and
training."""
import numpy as np
import pytest

import eventsim
import paper_2510_20071_amd as fb
from oracle import fill as ref
from _harness import torch_dev

pytestmark = pytest.mark.gpu

# BF16 inputs, weights and activations with FP32 accumulation against FP64:
# normwise relative error bound (the reference gets the same FP32 inputs and
# FP32 parameters)
TOL = 2e-2


def bf16_values(a):
    """FP32 values rounded to the nearest BF16 (ties to even), still FP32: the
    device's conversion of them is then exact, and the reference evaluates
    the very network the device runs."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32)


def params_with_biases(seed):
    p = eventsim.fill_init_params(seed, zero_last=False).astype(np.float64)
    rng = np.random.default_rng(seed + 100)
    k = 0
    for ws, bs in ref.layer_shapes():
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        p[k + nw:k + nw + nb] = rng.normal(0, 0.1, nb)
        k += nw + nb
    return p.astype(np.float32)


def make_batch(seed, n, H, W):
    rng = np.random.default_rng(seed)
    L = rng.normal(0, 2.0, (n, H, W)).astype(np.float32)
    stale = (rng.random((n, H, W)) < 0.4).astype(np.uint8)
    age = np.where(stale, rng.uniform(2, 12, (n, H, W)),
                   rng.uniform(0, 3, (n, H, W))).astype(np.float32)
    target = (L + rng.normal(0, 0.5, (n, H, W))).astype(np.float32)
    return L, stale, age, target


def dev(*arrays):
    torch, d = torch_dev()
    return [torch.from_numpy(np.ascontiguousarray(a)).to(d) for a in arrays]


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("shape", [(2, 37, 45), (1, 64, 64), (3, 5, 16)])
def test_forward_matches_reference(shape):
    torch, d = torch_dev()
    n, H, W = shape
    prm = params_with_biases(1)
    L, stale, age, _ = make_batch(2, n, H, W)
    gL, gS, gA = dev(L, stale, age)
    out = torch.empty((n, H, W), dtype=torch.float32, device=d)
    f = fb.Fill(prm)
    assert f.predict(gL, gS, gA, out) == 0
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want, _ = ref.forward(ref.unflatten(prm), ref.make_input(L, stale, age))
    err = rel(got, want)
    print("forward %s: normwise rel err %.3g" % (shape, err))
    assert err < TOL
    f.close()


def test_loss_and_gradient_match_reference():
    """On BF16-representable parameters and inputs (so that both sides
    differentiate the same network; with FP32 weights the device's rounding of
    them shifts every prediction alike, which the nearly cancelling sums of a
    gradient amplify), the remaining difference is the BF16 storage of
    activations and gradients between layers."""
    n, H, W = 2, 40, 48
    prm = bf16_values(params_with_biases(3))
    L, stale, age, target = make_batch(4, n, H, W)
    L, age = bf16_values(L), bf16_values(age)
    f = fb.Fill(prm)
    rc, loss, g = f.loss_grad(*dev(L, stale, age, target))
    assert rc == 0
    want_loss, want_g = ref.loss_and_grad(prm.astype(np.float64), ref.make_input(L, stale, age),
                                          target, stale)
    print("loss %.6g ref %.6g" % (loss, want_loss))
    assert abs(loss - want_loss) <= TOL * want_loss
    k = 0
    errs = []
    for l, (ws, bs) in enumerate(ref.layer_shapes()):
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        ew, eb = rel(g[k:k + nw], want_g[k:k + nw]), rel(g[k + nw:k + nw + nb], want_g[k + nw:k + nw + nb])
        print("layer %d: grad w rel err %.3g, grad b rel err %.3g" % (l, ew, eb))
        errs.append((ew, eb))
        k += nw + nb
    print("whole gradient rel err %.3g" % rel(g, want_g))
    for l, (ew, eb) in enumerate(errs):
        assert ew < TOL and eb < TOL, l
    f.close()


@pytest.mark.parametrize("shape", [(1, 720, 1280), (2, 37, 45), (1, 17, 27)])
def test_fused_inference_equals_layer_by_layer(shape):
    """Inference runs all four layers of a tile in one kernel (activations in
    LDS); training runs them layer by layer through device memory.  Same
    rounding points, so the loss from the layer-by-layer forward equals the
    loss of the fused prediction."""
    torch, d = torch_dev()
    n, H, W = shape
    prm = params_with_biases(17)
    L, stale, age, target = make_batch(18, n, H, W)
    batch = dev(L, stale, age, target)
    f = fb.Fill(prm)
    out = torch.empty((n, H, W), dtype=torch.float32, device=d)
    assert f.predict(*batch[:3], out) == 0
    p = out.cpu().numpy().astype(np.float64)
    m = stale != 0
    want = float(np.mean((p[m] - target[m]) ** 2))
    rc, loss, _ = f.loss_grad(*batch, want_grad=False)
    print("fused-inference loss %.9g, layer-by-layer loss %.9g" % (want, loss))
    assert rc == 0 and abs(loss - want) <= 1e-6 * want
    f.close()


def test_gradient_is_deterministic():
    prm = params_with_biases(5)
    batch = dev(*make_batch(6, 2, 33, 40))
    f = fb.Fill(prm)
    _, l1, g1 = f.loss_grad(*batch)
    _, l2, g2 = f.loss_grad(*batch)
    assert l1 == l2 and np.array_equal(g1, g2)
    f.close()


def test_adam_steps_match_reference_on_the_devices_gradients():
    prm = params_with_biases(7)
    batch = dev(*make_batch(8, 2, 32, 32))
    f = fb.Fill(prm)
    opt = ref.Adam(ref.N_PARAMS, lr=1e-3)
    theta = prm.astype(np.float64)
    for step in range(2):
        rc, loss_g, g = f.loss_grad(*batch)
        assert rc == 0
        rc, loss_t = f.train_step(*batch, lr=1e-3)
        assert rc == 0 and loss_t == loss_g
        theta = opt.step(theta, g.astype(np.float64))
        got = f.get_params()
        assert np.max(np.abs(got - theta)) <= 1e-6, step
        theta = got.astype(np.float64)
    f.close()


def test_set_params_round_trip_and_zero_stale_batch():
    torch, d = torch_dev()
    prm = params_with_biases(9)
    f = fb.Fill(prm)
    assert np.array_equal(f.get_params(), prm)
    L, stale, age, target = make_batch(10, 1, 20, 20)
    stale[:] = 0
    rc, loss, g = f.loss_grad(*dev(L, stale, age, target))
    assert rc == 0 and loss == 0.0 and not np.any(g)
    f.close()


@pytest.mark.parametrize("tile", [16, 8])
def test_apply_uses_prediction_or_falls_back_per_tile(tile):
    torch, d = torch_dev()
    H, W = 37, 45
    prm = params_with_biases(11)
    L, stale, age, _ = make_batch(12, 1, H, W)
    stale[0, :8, :8] = 0                      # one tile without stale pixels
    gL, gS, gA = dev(L[0], stale[0], age[0])
    f = fb.Fill(prm)
    pred = torch.empty((H, W), dtype=torch.float32, device=d)
    out = torch.empty_like(pred)
    assert f.predict(gL, gS, gA, pred) == 0
    p = pred.cpu().numpy()
    tiles = [(ty, tx) for ty in range(0, H, tile) for tx in range(0, W, tile)]
    frac = {t: float(np.mean(stale[0, t[0]:t[0] + tile, t[1]:t[1] + tile] != 0)) for t in tiles}
    with_stale = sum(1 for t in tiles if frac[t] > 0)
    # theta = 0: prediction at every stale pixel, L elsewhere
    rc, nfb = f.apply(gL, gS, gA, out, tile=tile, theta=0.0)
    assert rc == 0 and nfb == 0
    assert np.array_equal(out.cpu().numpy(), np.where(stale[0] != 0, p, L[0]))
    # theta = 1: every tile with a stale pixel keeps L
    rc, nfb = f.apply(gL, gS, gA, out, tile=tile, theta=1.0)
    assert rc == 0 and nfb == with_stale
    assert np.array_equal(out.cpu().numpy(), L[0])
    # a middle theta: exactly the tiles whose stale fraction exceeds it use the net
    theta = float(np.median([v for v in frac.values() if v > 0]))
    rc, nfb = f.apply(gL, gS, gA, out, tile=tile, theta=theta)
    assert rc == 0 and nfb == sum(1 for v in frac.values() if 0 < v <= theta)
    want = L[0].copy()
    for (ty, tx), v in frac.items():
        if v > theta:
            sl = (slice(ty, ty + tile), slice(tx, tx + tile))
            want[sl] = np.where(stale[0][sl] != 0, p[sl], L[0][sl])
    assert np.array_equal(out.cpu().numpy(), want)
    f.close()


def test_apply_falls_back_where_a_prediction_is_not_finite():
    torch, d = torch_dev()
    H, W = 32, 32
    prm = params_with_biases(17)
    L, stale, age, _ = make_batch(18, 1, H, W)
    stale[0] = 1
    Lnan = L[0].copy()
    Lnan[3, 4] = np.nan                       # the net's prediction there is NaN
    gL, gS, gA = dev(Lnan, stale[0], age[0])
    f = fb.Fill(prm)
    out = torch.empty((H, W), dtype=torch.float32, device=d)
    rc, nfb = f.apply(gL, gS, gA, out, tile=16, theta=0.0)
    assert rc == 0
    o = out.cpu().numpy()
    pred = torch.empty_like(out)
    assert f.predict(gL, gS, gA, pred) == 0
    p = pred.cpu().numpy()
    bad_tiles = {(ty, tx) for ty in range(0, H, 16) for tx in range(0, W, 16)
                 if not np.all(np.isfinite(p[ty:ty + 16, tx:tx + 16]))}
    assert bad_tiles and nfb == len(bad_tiles)
    for ty in range(0, H, 16):
        for tx in range(0, W, 16):
            sl = (slice(ty, ty + 16), slice(tx, tx + 16))
            if (ty, tx) in bad_tiles:
                assert np.array_equal(o[sl], Lnan[sl], equal_nan=True)
            else:
                assert np.array_equal(o[sl], p[sl])
    f.close()


def test_training_reduces_the_loss_on_a_learnable_task():
    """Smooth fields; stale pixels show 0 (no information), active pixels the
    truth; the target is the truth, so the network has to inpaint stale
    pixels from their neighbours.  The untrained fill (zero last layer) gives
    back L, so the first loss is the mean square of the truth at stale pixels;
    200 Adam steps must cut it well down."""
    torch, d = torch_dev()
    rng = np.random.default_rng(13)
    n, H, W = 8, 64, 64
    yy, xx = np.mgrid[0:H, 0:W]
    truth = np.zeros((n, H, W))
    for i in range(n):
        for _ in range(12):
            cy, cx, s, a = rng.uniform(0, H), rng.uniform(0, W), rng.uniform(3, 10), rng.normal(0, 2)
            truth[i] += a * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * s * s))
    stale = (rng.random((n, H, W)) < 0.3).astype(np.uint8)
    L = np.where(stale != 0, 0.0, truth).astype(np.float32)
    age = np.where(stale != 0, 8.0, 1.0).astype(np.float32)
    batch = dev(L, stale, age, truth.astype(np.float32))
    f = fb.Fill(eventsim.fill_init_params(14))
    rc, first = f.train_step(*batch, lr=3e-3)
    assert rc == 0
    assert abs(first - np.mean(truth[stale != 0] ** 2)) <= 1e-4 * first
    for _ in range(199):
        assert f.train_step(*batch, lr=3e-3, want_loss=False)[0] == 0
    rc, last, _ = f.loss_grad(*batch, want_grad=False)
    print("loss %.4g -> %.4g" % (first, last))
    assert rc == 0 and last < 0.3 * first
    f.close()


def test_argument_checks():
    torch, d = torch_dev()
    f = fb.Fill(params_with_biases(15))
    gL, gS, gA = dev(*make_batch(16, 1, 8, 8)[:3])
    out = torch.empty((8, 8), dtype=torch.float32, device=d)
    assert fb.fibar_fill_apply(f.handle, gL, gS, gA, 8, 8, 3, 1.0, out)[0] == fb.FIBAR_E_INVALID_ARG
    assert fb.fibar_fill_apply(f.handle, gL, gS, gA, 8, 8, 65, 1.0, out)[0] == fb.FIBAR_E_INVALID_ARG
    assert fb.fibar_fill_predict(f.handle, gL, gS, gA, 0, 8, 8, out) == fb.FIBAR_E_INVALID_ARG
    assert fb.fibar_fill_predict(f.handle, gL, None, gA, 1, 8, 8, out) == fb.FIBAR_E_INVALID_ARG
    assert fb.fibar_fill_train_step(f.handle, gL, gS, gA, out, 1, 8, 8, float("nan"))[0] == \
        fb.FIBAR_E_INVALID_ARG
    f.close()


# Per-pixel bound of the device prediction against the FP64 network.  BF16
# keeps 8 significant bits: the inputs, the weights and every layer's stored
# activations are rounded to it (relative 2^-9 each), sums are FP32.  A
# worst-case bound that adds absolute values through four 3x3 layers of 144
# terms each is ~100x the output itself, so the bound is statistical:
# roundings of independent sign add in quadrature, and after four layers the
# correction's error stays a few 2^-8 of its scale.  Per pixel, |error| <=
# 16 * 2^-8 * the RMS of the network's correction (prediction - L) over the
# band, checked beside the normwise bound.
PIX_BOUND = 16 * 2.0 ** -8


def test_full_frame_forward_matches_reference_on_bands():
    """One 1280x720 frame: the fused kernel's workgroups each loop over many
    tiles with the next tile's loads in flight.  The reference evaluates
    bands of full rows (top edge, interior, bottom edge), each from a crop
    four rows wider on each side, which is exact for a four-layer 3x3
    network; every pixel of the bands is checked."""
    torch, d = torch_dev()
    n, H, W = 1, 720, 1280
    prm = params_with_biases(21)
    L, stale, age, _ = make_batch(22, n, H, W)
    gL, gS, gA = dev(L, stale, age)
    out = torch.empty((n, H, W), dtype=torch.float32, device=d)
    f = fb.Fill(prm)
    assert f.predict(gL, gS, gA, out) == 0
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    f.close()
    params = ref.unflatten(prm)
    worst = 0.0
    for r0, r1 in ((0, 24), (233, 251), (400, 432), (696, 720)):
        c0, c1 = max(0, r0 - 4), min(H, r1 + 4)
        x = ref.make_input(L[:, c0:c1], stale[:, c0:c1], age[:, c0:c1])
        want = ref.forward(params, x)[0][:, r0 - c0:r1 - c0]
        corr = want - L[:, r0:r1]
        bound = PIX_BOUND * float(np.sqrt(np.mean(corr * corr)))
        g = got[:, r0:r1]
        err = rel(g, want)
        d_pix = np.abs(g.astype(np.float64) - want)
        print("rows %d-%d: normwise rel err %.3g, worst pixel error / bound %.3g"
              % (r0, r1, err, float((d_pix / bound).max())))
        assert err < TOL
        assert float(d_pix.max()) <= bound, (r0, r1)
        worst = max(worst, err)


def test_gradient_where_workgroups_take_several_units():
    """24 x 203 x 130: the weight-gradient kernel's units are 8 rows of one
    image by a strip of 128 columns, 24 x 26 x 2 = 1248 of them (the last rows
    of an image and the second strip ragged: 3 rows, 2 columns) over 1024
    workgroups, so some workgroups accumulate two units before the partial
    sums are reduced."""
    n, H, W = 24, 203, 130
    assert n * ((H + 7) // 8) * ((W + 127) // 128) == 1248
    prm = bf16_values(params_with_biases(23))
    L, stale, age, target = make_batch(24, n, H, W)
    L, age = bf16_values(L), bf16_values(age)
    f = fb.Fill(prm)
    rc, loss, g = f.loss_grad(*dev(L, stale, age, target))
    assert rc == 0
    f.close()
    want_loss, want_g = ref.loss_and_grad(prm.astype(np.float64), ref.make_input(L, stale, age),
                                          target, stale)
    print("loss %.6g ref %.6g" % (loss, want_loss))
    assert abs(loss - want_loss) <= TOL * want_loss
    k = 0
    for l, (ws, bs) in enumerate(ref.layer_shapes()):
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        ew = rel(g[k:k + nw], want_g[k:k + nw])
        eb = rel(g[k + nw:k + nw + nb], want_g[k + nw:k + nw + nb])
        print("layer %d: grad w rel err %.3g, grad b rel err %.3g" % (l, ew, eb))
        assert ew < TOL and eb < TOL, l
        k += nw + nb
