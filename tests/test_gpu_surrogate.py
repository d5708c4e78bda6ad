"""HIP surrogate kernels against the FP64 oracle (oracle/surrogate_oracle.py).

Operands: the GPU stores weights and activations in bfloat16 and accumulates
in FP32.  Layer tests feed the oracle the GPU's own bfloat16 layer inputs and
the bfloat16-rounded weights, so the only difference is FP32 accumulation
order over K = 9 C_in terms (relative error ~ sqrt(K) 6e-8): tolerance 1e-5.
The weight gradient sums K = B H W products in FP32: tolerance 1e-4.  The full
backward chain re-rounds every data gradient to bfloat16 on both sides from
FP32 values that differ in their last bits, so isolated one-ulp (2^-8)
differences propagate: normwise tolerance 2e-3 (measured ~2e-4).
"""
import numpy as np
import pytest
import torch

from oracle import surrogate_oracle as S
from paper_2101_03055_amd import sg

pytestmark = pytest.mark.gpu

B, H, W = 2, 16, 64


def setup(seed=0, batch=B):
    rng = np.random.default_rng(seed)
    net = sg.Surrogate(batch, H, W, lr=1e-3)
    w0 = sg.init_weights(seed)
    # non-zero biases so that the bias path is exercised
    layers = sg.unpack(w0)
    for l, (w, b) in enumerate(layers):
        _, cout, _, _ = sg.layer_info(l)
        b[:cout] = rng.uniform(-0.1, 0.1, cout)
    net.set_weights(w0)
    params = torch.tensor(rng.uniform(0, 1, (batch + 3, 5)), dtype=torch.float32, device="cuda")
    fields = torch.tensor(rng.uniform(-1, 1, (batch + 3, 4, H, W)), dtype=torch.float32, device="cuda")
    idx = np.array([3, 1] + list(range(batch - 2)), dtype=np.int32)[:batch]
    return net, w0, params, fields, idx


def relerr(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_features_match_oracle():
    net, w0, params, fields, idx = setup()
    net.gradients(params, fields, idx)
    x0 = net.layer_input(0)
    want = S.bf16(S.features(params.cpu().numpy()[idx].astype(np.float64), H, W))
    got = x0[..., :15]
    diff = np.abs(got - want)
    ulp = np.abs(want) * 2.0 ** -7 + 1e-30
    assert np.all(diff <= ulp)               # at most one bfloat16 ulp (float32 vs float64 sin/cos)
    assert np.mean(diff > 0) < 1e-3
    assert np.all(x0[..., 15:] == 0)


def test_each_layer_forward_matches_oracle():
    net, w0, params, fields, idx = setup()
    net.gradients(params, fields, idx)
    layers = sg.unpack(w0)
    for l, (w, b) in enumerate(layers):
        x = net.layer_input(l).astype(np.float64)
        z = net.layer_output(l).astype(np.float64)
        want = S.conv_forward(x, S.bf16(w), b.astype(np.float32).astype(np.float64))
        e = relerr(z, want)
        print(f"layer {l}: forward rel err {e:.2e}", flush=True)
        assert e < 1e-5, l
        if l + 1 < len(layers):
            nxt = net.layer_input(l + 1).astype(np.float64)
            # the next input is bf16(SiLU(z)) of the GPU's own z
            assert relerr(nxt, S.bf16(S.silu(z))) < 1e-2


def test_last_layer_gradients_match_oracle():
    net, w0, params, fields, idx = setup()
    loss, g = net.gradients(params, fields, idx)
    z5 = net.layer_output(5).astype(np.float64)
    x5 = net.layer_input(5).astype(np.float64)
    tgt = np.transpose(fields.cpu().numpy()[idx], (0, 2, 3, 1)).astype(np.float64)
    l_or, dpred = S.mse(z5[..., :4], tgt)
    assert abs(loss - l_or) / l_or < 1e-5
    dz = np.zeros_like(z5)
    dz[..., :4] = dpred
    dz = S.bf16(dz)
    w5, _ = sg.unpack(w0)[5]
    _, dw, db = S.conv_backward(x5, S.bf16(w5), dz)
    gw, gb = sg.unpack(g)[5]
    print(f"last layer: dW {relerr(gw, dw):.2e} db {relerr(gb, db):.2e}", flush=True)
    assert relerr(gw, dw) < 1e-4 and relerr(gb, db) < 1e-4


def test_all_gradients_match_oracle_chain():
    net, w0, params, fields, idx = setup()
    loss, g = net.gradients(params, fields, idx)
    layers = sg.unpack(w0)
    acts = [net.layer_input(l).astype(np.float64) for l in range(6)]
    zs = [net.layer_output(l).astype(np.float64) for l in range(6)]
    tgt = np.transpose(fields.cpu().numpy()[idx], (0, 2, 3, 1)).astype(np.float64)
    _, dpred = S.mse(zs[-1][..., :4], tgt)
    dz = np.zeros_like(zs[-1])
    dz[..., :4] = dpred
    bl = [(S.bf16(w), b) for w, b in layers]
    want = S.backward(bl, zs, acts, dz, bf16_storage=True)
    got = sg.unpack(g)
    for l in range(6):
        ew, eb = relerr(got[l][0], want[l][0]), relerr(got[l][1], want[l][1])
        print(f"layer {l}: dW {ew:.2e} db {eb:.2e}", flush=True)
        assert ew < 2e-3 and eb < 2e-3, l


def test_adam_step_matches_oracle():
    net, w0, params, fields, idx = setup()
    _, g = net.gradients(params, fields, idx)
    net.train_step(params, fields, idx)
    w1 = net.get_weights()
    want, _, _ = S.adam_step(w0.astype(np.float64), g.astype(np.float64), 0.0, 0.0, 1, lr=1e-3)
    assert np.abs(w1 - want).max() < 1e-6


def test_predict_equals_forward_and_training_reduces_loss():
    torch.manual_seed(0)
    net, w0, params, fields, idx = setup(batch=4)
    n = 16
    rng = np.random.default_rng(3)
    p = rng.uniform(0, 1, (n, 5))
    X, Y = np.meshgrid((np.arange(W) + 0.5) / W, (np.arange(H) + 0.5) / H)
    tg = np.stack([np.stack([p[k, 0] * np.sin(np.pi * X) * np.sin(np.pi * Y),
                             p[k, 1] * np.cos(np.pi * X) * Y,
                             X * (1 - p[k, 2]) + p[k, 3] * Y,
                             np.exp(-p[k, 4] * X)]) for k in range(n)])
    dp = torch.tensor(p, dtype=torch.float32, device="cuda")
    df = torch.tensor(tg, dtype=torch.float32, device="cuda")
    out = torch.empty((n, 4, H, W), dtype=torch.float32, device="cuda")
    net.predict(dp, n, out)
    torch.cuda.synchronize()
    # last chunk of prediction is samples 12..15 in order: compare with the layer output
    z5 = net.layer_output(5)
    assert np.array_equal(out.cpu().numpy()[12:], np.transpose(z5[..., :4], (0, 3, 1, 2)))
    losses = net.train_epochs(dp, df, n, 60, seed=1)
    print("losses", losses[0], losses[-1], flush=True)
    assert np.all(np.isfinite(losses)) and losses[-1] < 0.1 * losses[0]


def test_smooth_matches_oracle():
    rng = np.random.default_rng(11)
    a = rng.standard_normal((3, 4, 37, 29)).astype(np.float32)   # ragged plane
    d_in = torch.tensor(a, device="cuda")
    d_out = torch.empty_like(d_in)
    sg.smooth(d_in, d_out)
    torch.cuda.synchronize()
    want = S.smooth(a.astype(np.float64))
    assert np.abs(d_out.cpu().numpy() - want).max() <= 1e-6 * np.abs(want).max()


def test_destagger_matches_oracle():
    rng = np.random.default_rng(12)
    a = rng.standard_normal((5, 4, 128, 128)).astype(np.float32)
    a[:, 1] += 0.3 * ((-1.0) ** np.arange(128))[:, None]          # a large staggered part
    d = torch.tensor(a, device="cuda")
    sg.destagger(d)
    torch.cuda.synchronize()
    got = d.cpu().numpy().astype(np.float64)
    want = S.destagger(a.astype(np.float64))
    assert np.abs(got - want).max() <= 2e-6
    sy = ((-1.0) ** np.arange(128))[:, None]
    assert np.abs((got[:, 1] * sy).mean(axis=(1, 2))).max() <= 1e-7


@pytest.mark.parametrize("batch, n, epochs, seed", [(4, 12, 2, 5), (1, 300, 1, 6)])
def test_train_epochs_equals_its_steps(batch, n, epochs, seed):
    """sg_train_epochs (steps back to back, indices uploaded per block of 256 steps,
    batch losses summed on the device) against the same steps one sg_train_step call
    at a time in the order its shuffle draws (host copy of its generator): weights and
    epoch losses bitwise equal; 300 steps of one sample cross an index block."""
    from tests.mt64 import shuffled_epochs

    rng = np.random.default_rng(8)
    dp = torch.tensor(rng.uniform(0, 1, (n, 5)), dtype=torch.float32, device="cuda")
    df = torch.tensor(rng.uniform(-1, 1, (n, 4, H, W)), dtype=torch.float32, device="cuda")
    a, w0, _, _, _ = setup(batch=batch)
    la = a.train_epochs(dp, df, n, epochs, seed=seed)
    wa = a.get_weights()
    b = sg.Surrogate(batch, H, W, lr=1e-3)
    b.set_weights(w0)
    lb_ = []
    for order in shuffled_epochs(n, epochs, seed):
        s = 0.0
        for k in range(n // batch):
            s += float(b.train_step(dp, df, np.array(order[k * batch:(k + 1) * batch], dtype=np.int32)))
        lb_.append(np.float32(s / (n // batch)))
    wb = b.get_weights()
    assert np.array_equal(wa, wb)
    assert np.array_equal(la, np.array(lb_, dtype=np.float32))
