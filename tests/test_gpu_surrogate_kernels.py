"""HIP surrogate kernels at the widths the training runs use (W = 128), against
the FP64 oracle (oracle/surrogate_oracle.py).

Layer tests call one convolution or one weight gradient through the C ABI
(sg_conv, sg_weight_grad) on seeded random inputs: bfloat16 operands made on
the host, the same values handed to the oracle, so neither side sees the
other's intermediates.  At width 128 (the training grids) the convolutions and
the weight gradient stream whole image rows per workgroup (runs of 1 to 8 rows
over the shapes below, 8 at the benchmarked 16 x 128^2); other widths that are
multiples of 128 take the 128-pixel workgroup tile and the split-K weight
gradient.

Tolerances:
* forward pre-activation z: FP32 accumulation of K = 9 cin_pad <= 1152 bf16
  products against FP64 (relative error ~ sqrt(K) 2^-24): 1e-5 of max |z|;
* stored bfloat16 outputs (activation, data gradient): one bfloat16 rounding
  (2^-8 relative) of a value that carries the FP32 error above;
* weight and bias gradients: FP32 sums over up to 2.6e5 pixels (partial sums
  per 64-pixel chunk, then fixed-order sums of the split partials): 1e-4 of max.
End to end, the oracle runs forward from the features and the bfloat16 weights
and back through the gradient chain on its own activations.  Every stored
bfloat16 value then differs between the sides wherever the FP32 and FP64 values
round to different neighbours, and those one-ulp flips propagate: an FP32
evaluation of the same network in numpy lands 9e-4 (prediction) and 2e-4
(gradients) relative L2 from the FP64 oracle, so the bounds are 5e-3 and 2e-3.
"""
import numpy as np
import pytest
import torch

from oracle import surrogate_oracle as S
from paper_2101_03055_amd import sg

pytestmark = pytest.mark.gpu


def make_net(batch, H, W, seed):
    rng = np.random.default_rng(seed)
    net = sg.Surrogate(batch, H, W, lr=1e-3)
    w0 = sg.init_weights(seed)
    for l, (w, b) in enumerate(sg.unpack(w0)):
        _, cout, _, _ = sg.layer_info(l)
        b[:cout] = rng.uniform(-0.1, 0.1, cout)
    net.set_weights(w0)
    layers = [(S.bf16(w.astype(np.float64)), b.astype(np.float64)) for w, b in sg.unpack(w0)]
    return net, w0, layers


def bf16_pair(a):
    """(device bfloat16 tensor, the same values as float64) from a float array."""
    t = torch.tensor(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16)
    return t.to("cuda"), t.float().numpy().astype(np.float64)


def to_np(t):
    return t.float().cpu().numpy().astype(np.float64)


def check_bf16_output(got, want, label, rel=1e-5):
    """got = bf16 of a value within rel * max|want| of want."""
    tol = 2.0 ** -8 * np.abs(want) + rel * np.abs(want).max()
    bad = np.abs(got - want) > tol
    exact = np.mean(got == S.bf16(want))
    print(f"{label}: max |got - want| / max|want| {np.abs(got - want).max() / np.abs(want).max():.2e}, "
          f"bf16-identical {exact:.4f}", flush=True)
    assert not bad.any(), label
    assert exact > 0.98, label


# at width 128 the row kernels give each workgroup a run of rows, worked in steps of two
# rows by two groups of wavefronts: 2 x 128 rows over 256 workgroups is one row each (the
# second group idle), 5 x 128 = 640 rows is three (two steps, the last with one row; the
# last workgroup has a single row) or five for the 128-channel outputs, and runs cross
# image boundaries; 7 x 37 = 259 rows gives runs of two rows with an image boundary every
# 37 rows (first and last rows of an image inside a step) and a last workgroup of one row
@pytest.mark.parametrize("B, H, W", [(2, 128, 128), (5, 128, 128), (7, 37, 128), (1, 64, 256)])
def test_forward_convolutions_match_oracle(B, H, W):
    net, _, layers = make_net(B, H, W, seed=1)
    rng = np.random.default_rng(2)
    for l, (w, b) in enumerate(layers):
        _, _, ci, co = sg.layer_info(l)
        dx, x = bf16_pair(rng.uniform(-1.5, 1.5, (B, H, W, ci)))
        dz = torch.empty((B, H, W, co), dtype=torch.float32, device="cuda")
        dy = torch.empty((B, H, W, co), dtype=torch.bfloat16, device="cuda")
        net.conv(l, 0, B, dx, dy, d_z=dz)
        torch.cuda.synchronize()
        want = S.conv_forward(x, w, b)
        z = dz.cpu().numpy().astype(np.float64)
        e = np.abs(z - want).max() / np.abs(want).max()
        print(f"layer {l} ({B}x{H}x{W}): forward z rel err {e:.2e}", flush=True)
        assert e < 1e-5, l
        act = S.silu(want) if l + 1 < len(layers) else want
        check_bf16_output(to_np(dy), act, f"layer {l} activation")
        # without the pre-activation store (the prediction's kernels): the same activation
        dy2 = torch.empty_like(dy)
        net.conv(l, 0, B, dx, dy2)
        torch.cuda.synchronize()
        assert torch.equal(dy, dy2), l


@pytest.mark.parametrize("B, H, W", [(2, 128, 128), (5, 128, 128), (7, 37, 128), (1, 64, 256)])
def test_data_gradient_convolutions_match_oracle(B, H, W):
    net, _, layers = make_net(B, H, W, seed=3)
    rng = np.random.default_rng(4)
    for l in range(1, len(layers)):
        w, _ = layers[l]
        _, _, ci, co = sg.layer_info(l)
        dg, g = bf16_pair(rng.uniform(-1, 1, (B, H, W, co)))
        zprev = rng.uniform(-4, 4, (B, H, W, ci)).astype(np.float32)
        dzp = torch.tensor(zprev, device="cuda")
        dout = torch.empty((B, H, W, ci), dtype=torch.bfloat16, device="cuda")
        net.conv(l, 1, B, dg, dout, d_zprev=dzp)
        torch.cuda.synchronize()
        dxw, _, _ = S.conv_backward(np.zeros((B, H, W, ci)), w, g)
        want = dxw * S.silu_grad(zprev.astype(np.float64))
        check_bf16_output(to_np(dout), want, f"layer {l} data gradient ({B}x{H}x{W})")


@pytest.mark.parametrize("B, H, W", [(1, 128, 128), (2, 128, 128), (1, 5, 128), (3, 37, 128), (1, 64, 256)])
def test_weight_gradients_match_oracle_multichunk(B, H, W):
    # width 128: the row-streaming kernel, runs of 1 (B = 1, 2 at 128^2, and 5 rows) or
    # 1-2 rows (3 x 37 = 111 rows over the workgroups, 37 not a multiple of anything);
    # width 256: the split-K kernel with 128 slices of 2 chunks of 64 pixels
    net, _, layers = make_net(B, H, W, seed=5)
    rng = np.random.default_rng(6)
    for l in range(len(layers)):
        _, _, ci, co = sg.layer_info(l)
        dg, g = bf16_pair(rng.uniform(-1, 1, (B, H, W, co)))
        dx, x = bf16_pair(rng.uniform(-1, 1, (B, H, W, ci)))
        ddw = torch.empty((co, 9, ci), dtype=torch.float32, device="cuda")
        ddb = torch.empty((co,), dtype=torch.float32, device="cuda")
        net.weight_grad(l, B, dg, dx, ddw, ddb)
        torch.cuda.synchronize()
        _, dw, db = S.conv_backward(x, np.zeros((co, 9, ci)), g)
        ew = np.abs(ddw.cpu().numpy() - dw).max() / np.abs(dw).max()
        eb = np.abs(ddb.cpu().numpy() - db).max() / np.abs(db).max()
        print(f"layer {l} (B = {B}): dW rel err {ew:.2e}, db {eb:.2e}", flush=True)
        assert ew < 1e-4 and eb < 1e-4, l
        # fixed-order sums: a second call is bitwise identical
        ddw2 = torch.empty_like(ddw)
        ddb2 = torch.empty_like(ddb)
        net.weight_grad(l, B, dg, dx, ddw2, ddb2)
        torch.cuda.synchronize()
        assert torch.equal(ddw, ddw2) and torch.equal(ddb, ddb2)


def test_benchmark_shape_layers_match_oracle():
    """The benchmarked training shape, 16 x 128 x 128 (32 chunks per split-K
    slice), for the widest-K layer (128 -> 64) and the widest-N layer (64 -> 128):
    forward, data gradient and weight gradient over every output."""
    B = 16
    H = W = 128
    net, _, layers = make_net(B, H, W, seed=7)
    rng = np.random.default_rng(8)
    for l in (1, 2):
        w, b = layers[l]
        _, _, ci, co = sg.layer_info(l)
        dx, x = bf16_pair(rng.uniform(-1, 1, (B, H, W, ci)))
        dz = torch.empty((B, H, W, co), dtype=torch.float32, device="cuda")
        dy = torch.empty((B, H, W, co), dtype=torch.bfloat16, device="cuda")
        net.conv(l, 0, B, dx, dy, d_z=dz)
        dg, g = bf16_pair(rng.uniform(-1, 1, (B, H, W, co)))
        zprev = rng.uniform(-4, 4, (B, H, W, ci)).astype(np.float32)
        dzp = torch.tensor(zprev, device="cuda")
        dgx = torch.empty((B, H, W, ci), dtype=torch.bfloat16, device="cuda")
        net.conv(l, 1, B, dg, dgx, d_zprev=dzp)
        ddw = torch.empty((co, 9, ci), dtype=torch.float32, device="cuda")
        ddb = torch.empty((co,), dtype=torch.float32, device="cuda")
        net.weight_grad(l, B, dg, dx, ddw, ddb)
        torch.cuda.synchronize()
        want = S.conv_forward(x, w, b)
        e = np.abs(dz.cpu().numpy() - want).max() / np.abs(want).max()
        print(f"layer {l} (16x128x128): forward z rel err {e:.2e}", flush=True)
        assert e < 1e-5
        check_bf16_output(to_np(dy), S.silu(want), f"layer {l} activation (16x128x128)")
        del want
        dxw, dw, db = S.conv_backward(x, w, g)
        check_bf16_output(to_np(dgx), dxw * S.silu_grad(zprev.astype(np.float64)),
                          f"layer {l} data gradient (16x128x128)")
        ew = np.abs(ddw.cpu().numpy() - dw).max() / np.abs(dw).max()
        eb = np.abs(ddb.cpu().numpy() - db).max() / np.abs(db).max()
        print(f"layer {l} (16x128x128): dW rel err {ew:.2e}, db {eb:.2e}", flush=True)
        assert ew < 1e-4 and eb < 1e-4


def test_128_channel_forward_beyond_the_partial_buffer():
    """Layer 2's forward (128 K channels) at 128^2 runs as two 64-channel launches through the
    weight gradient's FP32 partial buffer while the partial sums fit (up to 18 samples); a
    batch of 19 takes the 128-pixel tile kernel instead.  Both against the oracle on the first
    and last image (images are independent)."""
    H = W = 128
    for B in (18, 19):
        net, _, layers = make_net(B, H, W, seed=9)
        rng = np.random.default_rng(10 + B)
        w, b = layers[2]
        _, _, ci, co = sg.layer_info(2)
        dx, x = bf16_pair(rng.uniform(-1, 1, (B, H, W, ci)))
        dz = torch.empty((B, H, W, co), dtype=torch.float32, device="cuda")
        dy = torch.empty((B, H, W, co), dtype=torch.bfloat16, device="cuda")
        net.conv(2, 0, B, dx, dy, d_z=dz)
        torch.cuda.synchronize()
        for img in (0, B - 1):
            want = S.conv_forward(x[img:img + 1], w, b)
            z = dz[img:img + 1].cpu().numpy().astype(np.float64)
            e = np.abs(z - want).max() / np.abs(want).max()
            print(f"B = {B}, image {img}: forward z rel err {e:.2e}", flush=True)
            assert e < 1e-5
            check_bf16_output(to_np(dy[img:img + 1]), S.silu(want), f"layer 2 activation (B = {B}, image {img})")
        del net


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_end_to_end_prediction_and_gradients_from_the_oracles_own_forward():
    B, H, W = 2, 128, 128
    net, w0, layers = make_net(B, H, W, seed=9)
    rng = np.random.default_rng(10)
    params = rng.uniform(0, 1, (B, 5)).astype(np.float32)
    fields = rng.uniform(-1, 1, (B, 4, H, W)).astype(np.float32)
    idx = np.arange(B, dtype=np.int32)
    loss, g = net.gradients(torch.tensor(params, device="cuda"), torch.tensor(fields, device="cuda"), idx)
    pred = net.layer_output(5)[..., :4].astype(np.float64)
    # the oracle from the features on: bfloat16 storage of inputs, weights and activations
    x = np.zeros((B, H, W, 32))
    x[..., :15] = S.features(params.astype(np.float64), H, W)
    zs, acts = S.forward(layers, x, bf16_storage=True)
    tgt = np.transpose(fields, (0, 2, 3, 1)).astype(np.float64)
    l_or, dpred = S.mse(zs[-1][..., :4], tgt)
    ep = rel_l2(pred, zs[-1][..., :4])
    print(f"prediction rel L2 {ep:.2e}, loss {loss:.6e} vs {l_or:.6e}", flush=True)
    assert ep < 5e-3
    assert abs(loss - l_or) / l_or < 1e-4
    dz = np.zeros_like(zs[-1])
    dz[..., :4] = dpred
    want = S.backward(layers, zs, acts, dz, bf16_storage=True)
    got = sg.unpack(g)
    for l in range(6):
        ew, eb = rel_l2(got[l][0], want[l][0]), rel_l2(got[l][1], want[l][1])
        print(f"layer {l}: dW rel L2 {ew:.2e}, db {eb:.2e}", flush=True)
        assert ew < 2e-3 and eb < 2e-3, l


def test_conv_entry_points_reject_bad_arguments():
    net, _, _ = make_net(2, 16, 128, seed=0)
    t = torch.zeros((2, 16, 128, 128), dtype=torch.bfloat16, device="cuda")
    z = torch.zeros((2, 16, 128, 128), dtype=torch.float32, device="cuda")
    with pytest.raises(Exception):
        net.conv(0, 1, 2, t, t, d_zprev=z)   # no data gradient below layer 1
    with pytest.raises(Exception):
        net.conv(1, 0, 3, t, t, d_z=z)       # more samples than the batch
    with pytest.raises(Exception):
        net.conv(6, 0, 1, t, t, d_z=z)       # no such layer
