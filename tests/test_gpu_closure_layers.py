"""The closure network's kernels, one C entry point at a time, against the FP64
closure oracle (oracle/nn.py) at the size training runs: 64^3 grid, batch 4.

Each kernel gets the same BF16 operands on both sides (the GPU's own output of the
previous kernel, so differences never compound), and each result is compared
element by element:

- FP32 sums of exact BF16 products (convolutions, weight and bias gradients):
  |gpu - ref| <= 2 (depth + 2) * 2^-24 * A, where A is the same sum over absolute
  values (computed by the oracle) and depth bounds the number of roundings along
  any chain of the GPU's additions.  This is the classical error bound of
  floating-point summation with a full unit (not half) per rounding, which also
  covers an accumulator that truncates, so it holds element by element, whatever
  the data.
- BF16-rounded results: within one BF16 unit in the last place (2^-7 relative) of
  the oracle's value, plus the bound above scaled by the factor applied before
  rounding.
Forward and backward-data results are compared at sampled points (every sample,
tile corners and edges, random interior points) with the oracle's point-by-point
forms; weight and bias gradients, which are sums over every point, in full.
"""
import numpy as np
import pytest

import synth
from oracle import nn

pytestmark = pytest.mark.gpu

N, B = 64, 4
U = 2.0 ** -24            # FP32 unit roundoff
BF16_ULP = 2.0 ** -7      # largest relative spacing of BF16 numbers


def _mods():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a HIP device")
    from paper_1609_01277_amd import closure
    return closure, torch


def bf16(a):
    """Round to bfloat16 (nearest, ties to even), returned as float64."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def planar(a, c):
    """Channel-last [B][P][cpad] (numpy) -> planar [B][c][n][n][n] view, channels < c."""
    return a.reshape(B, N, N, N, -1)[..., :c].transpose(0, 4, 1, 2, 3)


def sample_points(rng):
    pts = []
    edges = (0, 1, 7, 8, 31, 32, 33, 62, 63)
    for b in range(B):
        for z in (0, 31, 63):
            for y in edges:
                for x in edges:
                    pts.append((b, z, y, x))
        pts += [(b,) + tuple(rng.integers(0, N, 3)) for _ in range(300)]
    return np.array(pts, dtype=np.int64)


def at(a_planar, pts):
    """Values of a planar array at the sampled points: [len(pts)][channels]."""
    return a_planar[pts[:, 0], :, pts[:, 1], pts[:, 2], pts[:, 3]]


def to_host(t):
    import torch
    return t.float().cpu().numpy().astype(np.float64) if t.dtype == torch.bfloat16 else \
        t.cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def chain():
    """Runs forward and backward of the 5-32-32-5 network through the per-kernel
    entry points at 64^3, batch 4, and returns every input and output."""
    closure, torch = _mods()
    rng = np.random.default_rng(1609)
    P = N ** 3
    layers = nn.init_params(rng)
    layers = [(W, 0.1 * rng.standard_normal(b.shape)) for W, b in layers]
    ch = [5, 32, 32, 5]
    dev = {}
    # input: standardised state values, already BF16 numbers; padding channels zero
    x = np.zeros((B, P, 8), dtype=np.float32)
    x[..., :5] = bf16(rng.standard_normal((B, P, 5)))
    t = (0.5 * rng.standard_normal((B, 5, N, N, N))).astype(np.float32)
    mean_std = np.array([0.1, -0.2, 0.0, 0.05, 0.3, 0.8, 1.1, 0.9, 1.3, 0.7], dtype=np.float32)
    cu = lambda a, dt=torch.float32: torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()
    dev["x"] = cu(x, torch.bfloat16)
    Wd, Wf, Wb, bd = [], [], [], []
    for li, (W, b) in enumerate(layers):
        cin, cout = ch[li], ch[li + 1]
        Wd.append(cu(W.reshape(cout, cin, 27)))
        bd.append(cu(b))
        Wf.append(torch.zeros((32, closure.sbli_conv3d_packed_width(cin)), dtype=torch.bfloat16, device="cuda"))
        Wb.append(torch.zeros((32, closure.sbli_conv3d_packed_width(cout)), dtype=torch.bfloat16, device="cuda"))
        closure.sbli_conv3d_pack(Wd[li], cin, cout, Wf[li], Wb[li])
    # forward
    pre1 = torch.empty((B, P, 32), device="cuda")
    h1 = torch.empty((B, P, 32), dtype=torch.bfloat16, device="cuda")
    closure.sbli_conv3d_fwd(dev["x"], 5, Wf[0], bd[0], 32, N, B, closure.ACT_GELU, pre1, h1)
    pre2 = torch.empty((B, P, 32), device="cuda")
    h2 = torch.empty((B, P, 32), dtype=torch.bfloat16, device="cuda")
    closure.sbli_conv3d_fwd(h1, 32, Wf[1], bd[1], 32, N, B, closure.ACT_GELU, pre2, h2)
    y = torch.zeros((B, P, 8), device="cuda")
    closure.sbli_conv3d_fwd(h2, 32, Wf[2], bd[2], 5, N, B, closure.ACT_NONE, y)
    # loss and its gradient
    td, msd = cu(t), cu(mean_std)
    dy = torch.empty((B, P, 8), dtype=torch.bfloat16, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    mwork = torch.empty(closure.sbli_mse_grad_work_bytes(N, B) // 8, dtype=torch.float64, device="cuda")
    closure.sbli_mse_grad(y, 8, td, msd, N, B, dy, loss, mwork)
    # backward
    work = torch.empty(closure.sbli_conv3d_bwd_weight_work_bytes(32) // 4, device="cuda")
    grads = []
    for li in range(3):
        cin, cout = ch[li], ch[li + 1]
        grads.append((torch.empty((cout, cin, 27), device="cuda"), torch.empty(cout, device="cuda")))
    closure.sbli_conv3d_bwd_weight(h2, 32, dy, 5, N, B, grads[2][0], grads[2][1], work)
    d2 = torch.empty((B, P, 32), dtype=torch.bfloat16, device="cuda")
    closure.sbli_conv3d_bwd_data(dy, 5, Wb[2], N, B, pre2, d2)
    g2 = torch.empty((B, P, 32), device="cuda")                     # the same without GELU'
    closure.sbli_conv3d_bwd_data(dy, 5, Wb[2], N, B, None, g2)
    d2c = torch.empty((B, P, 32), dtype=torch.bfloat16, device="cuda")
    closure.sbli_gelu_bwd(g2, pre2, B * P * 32, d2c)
    closure.sbli_conv3d_bwd_weight(h1, 32, d2, 32, N, B, grads[1][0], grads[1][1], work)
    d1 = torch.empty((B, P, 32), dtype=torch.bfloat16, device="cuda")
    closure.sbli_conv3d_bwd_data(d2, 32, Wb[1], N, B, pre1, d1)
    closure.sbli_conv3d_bwd_weight(dev["x"], 5, d1, 32, N, B, grads[0][0], grads[0][1], work)
    torch.cuda.synchronize()
    out = dict(layers=layers, x=x.astype(np.float64), t=t, mean_std=mean_std, pts=sample_points(rng),
               Wf=[to_host(w) for w in Wf], Wb=[to_host(w) for w in Wb],
               pre1=to_host(pre1), h1=to_host(h1), pre2=to_host(pre2), h2=to_host(h2), y=to_host(y),
               dy=to_host(dy), loss=float(loss.item()), g2=to_host(g2), d2=to_host(d2), d1=to_host(d1),
               d2_composed_equal=bool(torch.equal(d2, d2c)),
               grads=[(to_host(dW).reshape(-1, ch[li], 3, 3, 3), to_host(db)) for li, (dW, db) in enumerate(grads)])
    out["Wbf"] = [bf16(W) for W, _ in layers]
    out["bf"] = [b.astype(np.float32).astype(np.float64) for _, b in layers]
    return out


def test_pack_is_bf16_of_master_weights(chain):
    """Packed operands hold exactly bf16(W) at the documented positions, zeros elsewhere."""
    ch = [5, 32, 32, 5]
    for li in range(3):
        cin, cout = ch[li], ch[li + 1]
        cp, op = (8 if cin <= 8 else 32), (8 if cout <= 8 else 32)
        Wr = chain["Wbf"][li].reshape(cout, cin, 27)
        ref_f = np.zeros_like(chain["Wf"][li])
        ref_b = np.zeros_like(chain["Wb"][li])
        for tap in range(27):
            ref_f[:cout, tap * cp:tap * cp + cin] = Wr[:, :, tap]
            ref_b[:cin, tap * op:tap * op + cout] = Wr[:, :, 26 - tap].T
        assert np.array_equal(chain["Wf"][li], ref_f), li
        assert np.array_equal(chain["Wb"][li], ref_b), li


def _check_sum(got, ref, absref, depth, what):
    bound = 2 * (depth + 2) * U * absref
    err = np.abs(got - ref)
    worst = np.unravel_index(np.argmax(err - bound), err.shape)
    assert np.all(err <= bound), "%s: |gpu - ref| = %.3e > bound %.3e at %s" % (
        what, err[worst], bound[worst], worst)


def _check_gelu(h, pre, what):
    g = nn.gelu(pre)
    err = np.abs(h - g)
    bound = BF16_ULP * np.abs(g) + 8 * U * (np.abs(pre) + 1.0)
    assert np.all(err <= bound), "%s: GELU output off by %.3e" % (what, (err - bound).max())


def test_forward_layers_match_oracle(chain):
    pts = chain["pts"]
    ins = [planar(chain["x"], 5), planar(chain["h1"], 32), planar(chain["h2"], 32)]
    outs = [chain["pre1"], chain["pre2"], chain["y"]]
    cout = [32, 32, 5]
    for li in range(3):
        W, b = chain["Wbf"][li], chain["bf"][li]
        ref = nn.conv3d_at_points(ins[li], W, b, pts)
        absref = nn.conv3d_at_points(np.abs(ins[li]), np.abs(W), np.abs(b), pts)
        got = at(planar(outs[li], cout[li]), pts)
        _check_sum(got, ref, absref, 27 * ins[li].shape[1], "layer %d pre-activation" % (li + 1))
    # activations: every element, from the GPU's own pre-activations
    _check_gelu(chain["h1"], chain["pre1"], "h1")
    _check_gelu(chain["h2"], chain["pre2"], "h2")
    # the linear layer leaves the padding channels alone
    assert np.all(chain["y"][..., 5:] == 0.0)


def test_mse_loss_and_gradient_match_oracle(chain):
    ms = chain["mean_std"].astype(np.float64)
    y = planar(chain["y"], 5)
    ts = (chain["t"].astype(np.float64) - ms[:5, None, None, None]) / ms[5:, None, None, None]
    loss, g = nn.mse(y, ts)
    assert abs(chain["loss"] - loss) <= 1e-6 * loss
    dy = planar(chain["dy"], 5)
    scale = 2.0 / y.size
    bound = BF16_ULP * np.abs(g) + scale * 4 * U * (np.abs(y) + np.abs(ts))
    assert np.all(np.abs(dy - g) <= bound)
    assert np.all(chain["dy"][..., 5:] == 0.0)


def test_backward_data_matches_oracle(chain):
    pts = chain["pts"]
    # layer 3 -> 2: plain data gradient (FP32), then with GELU' fused (BF16)
    dy = planar(chain["dy"], 5)
    W3 = chain["Wbf"][2]
    ref = nn.conv3d_bwd_data_at_points(dy, W3, pts)
    absref = nn.conv3d_bwd_data_at_points(np.abs(dy), np.abs(W3), pts)
    _check_sum(at(planar(chain["g2"], 32), pts), ref, absref, 27 * 8, "layer 3 data gradient")
    for (dgrad, din, W, pre, name) in (
            (chain["d2"], dy, W3, chain["pre2"], "layer 3 data gradient x GELU'"),
            (chain["d1"], planar(chain["d2"], 32), chain["Wbf"][1], chain["pre1"], "layer 2 data gradient x GELU'")):
        gp = nn.gelu_grad(at(planar(pre, 32), pts))
        ref = nn.conv3d_bwd_data_at_points(din, W, pts)
        absref = nn.conv3d_bwd_data_at_points(np.abs(din), np.abs(W), pts)
        got = at(planar(dgrad, 32), pts)
        # the FP32 sum g (bound as above), times GELU' in FP32 (Phi(v) = (1 + erf)/2 loses
        # up to 2^-24 absolute next to 1 for negative v, so its error is absolute), then
        # rounded to BF16 (one unit, 2^-7 relative, of the value rounded)
        dg = 2 * (27 * 32 + 2) * U * absref
        dgp = 4 * U + 8 * U * np.abs(gp)
        bound = BF16_ULP * (np.abs(ref * gp) + np.abs(ref) * dgp + np.abs(gp) * dg) \
            + np.abs(ref) * dgp + np.abs(gp) * dg + dg * dgp
        err = np.abs(got - ref * gp)
        assert np.all(err <= bound), "%s: off by %.3e" % (name, (err - bound).max())
    # the separate GELU backward on the plain data gradient is bitwise the fused epilogue
    assert chain["d2_composed_equal"]


def test_weight_and_bias_gradients_match_oracle(chain):
    """dW and db of every layer, every element, against the full sums over 4 x 64^3 points.
    Depth of the GPU's sums: 128 MFMA steps of 16 products per workgroup, then 512
    workgroup partials in four interleaved chains (dW); 8192 points per workgroup, at
    most 128 per lane, then at most 256 lanes, then 512 partials in 8 slices (db)."""
    douts = [planar(chain["d1"], 32), planar(chain["d2"], 32), planar(chain["dy"], 5)]
    ins = [planar(chain["x"], 5), planar(chain["h1"], 32), planar(chain["h2"], 32)]
    for li in range(3):
        rW, rb = nn.conv3d_bwd_weight(ins[li], douts[li])
        aW, ab = nn.conv3d_bwd_weight(np.abs(ins[li]), np.abs(douts[li]))
        dW, db = chain["grads"][li]
        _check_sum(dW, rW, aW, 2048 + 130, "layer %d dW" % (li + 1))
        _check_sum(db, rb, ab, 128 + 256 + 64 + 8, "layer %d db" % (li + 1))
        assert np.abs(rW).max() > 0 and np.abs(rb).max() > 0


def test_network_gradients_use_the_same_kernels(chain):
    """sbli_net_gradients at 64^3, batch 4 gives bitwise the per-kernel chain's gradients
    when its standardisation is the identity (mean 0, std 1: the input is already BF16)."""
    closure, torch = _mods()
    net = closure.ClosureNet(N, B)
    net.set_params(closure.join_params(chain["layers"]).astype(np.float32))
    st = np.zeros(closure.N_STATS, dtype=np.float32)
    st[5:10] = 1.0
    st[10:20] = chain["mean_std"]
    st[20:25] = np.inf
    net.set_stats(st)
    q = np.ascontiguousarray(planar(chain["x"], 5)).astype(np.float32)
    loss = net.gradients(torch.from_numpy(q).cuda(), torch.from_numpy(chain["t"]).cuda())
    g = net.get_grads()
    ref = closure.join_params([(dW, db) for dW, db in chain["grads"]]).astype(np.float32)
    assert np.array_equal(g, ref)
    assert loss == chain["loss"]
    net.close()


# The GPU keeps Adam's hyperparameters as FP32 numbers; the oracle is given the same
# values (as doubles), so both apply the same update rule.
BETA1, BETA2 = float(np.float32(0.9)), float(np.float32(0.999))


def _adam_p_bound(rp, lr, t):
    """FP32 evaluation of the update: a few units of p, plus 1 - beta2^t evaluated in
    FP32 next to 1 (cancellation: about 2^-24 / (1 - beta2^t), i.e. 1.5e-5 relative at
    t = 2), which reaches the step through the square root; 1e-4 of lr per step covers it."""
    return 2 * U * np.abs(rp) + 1e-4 * lr * t


def test_adam_three_steps_match_oracle():
    """sbli_adam_step for t = 1, 2, 3 with a different gradient each step (FP32 on the GPU,
    FP64 oracle on the same FP32 gradients): moments and parameters after every step."""
    closure, torch = _mods()
    rng = np.random.default_rng(7)
    n = 36357
    p0 = rng.standard_normal(n).astype(np.float32) * 0.1
    gs = [rng.standard_normal(n).astype(np.float32) * s for s in (1e-2, 3e-3, 5e-2)]
    p, m, v = (torch.from_numpy(p0.copy()).cuda(), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda"))
    rp, rm, rv = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    am = np.zeros(n)          # the first moment's recursion over |g|: bounds its rounding
    lr = 1e-3
    for t, g in enumerate(gs, start=1):
        closure.sbli_adam_step(p, torch.from_numpy(g).cuda(), m, v, n, lr, t)
        g64 = g.astype(np.float64)
        rp, rm, rv = nn.adam_step(rp, g64, rm, rv, t, lr, beta1=BETA1, beta2=BETA2)
        am = BETA1 * am + (1 - BETA1) * np.abs(g64)
        gp, gm, gv = (a.cpu().numpy().astype(np.float64) for a in (p, m, v))
        assert np.all(np.abs(gm - rm) <= 4 * t * U * am), t
        assert np.all(np.abs(gv - rv) <= 6 * t * U * rv), t
        assert np.all(np.abs(gp - rp) <= _adam_p_bound(rp, lr, t)), t
    # the step moved every parameter: bias correction at t = 2, 3 was applied
    assert np.all(np.abs(gp - p0) > 0)


def test_train_step_adam_three_steps_match_oracle():
    """The network's own train_step: parameters after each of three steps equal the oracle's
    Adam applied to the gradients the network computed (bias correction at t = 2, 3)."""
    closure, torch = _mods()
    n = 32
    rng = np.random.default_rng(11)
    layers = [(W, 0.1 * rng.standard_normal(b.shape)) for W, b in nn.init_params(rng)]
    net = closure.ClosureNet(n, 2)
    p = closure.join_params(layers).astype(np.float32)
    net.set_params(p)
    q = torch.from_numpy(synth.random_conservative_state(n, seed=12, mom=0.5).astype(np.float32)[None]
                         .repeat(2, axis=0)).cuda()
    t = torch.from_numpy((0.05 * rng.standard_normal((2, 5, n, n, n))).astype(np.float32)).cuda()
    st = np.zeros(closure.N_STATS, dtype=np.float32)
    st[0:5] = [1.0, 0.0, 0.0, 0.0, 179.0]
    st[5:10] = [0.06, 0.3, 0.3, 0.3, 0.6]
    st[15:20] = 0.05
    st[20:25] = np.inf
    net.set_stats(st)
    rp, rm, rv = p.astype(np.float64), np.zeros(p.size), np.zeros(p.size)
    lr = 1e-3
    for step in (1, 2, 3):
        net.train_step(q, t, lr)
        g = net.get_grads().astype(np.float64)
        rp, rm, rv = nn.adam_step(rp, g, rm, rv, step, lr, beta1=BETA1, beta2=BETA2)
        gp = net.get_params().astype(np.float64)
        assert np.all(np.abs(gp - rp) <= _adam_p_bound(rp, lr, step)), step
    net.close()


def test_box_filter_subtract_mode_matches_oracle():
    """subtract = 1 forms F(fine) - coarse in place (the training target F R_f - R_c)."""
    closure, torch = _mods()
    n = 64
    rng = np.random.default_rng(5)
    f = synth.random_conservative_state(n, seed=6)
    c0 = rng.standard_normal((5, n // 4, n // 4, n // 4)).astype(np.float32)
    for dt in (torch.float64, torch.float32):
        fin = f if dt == torch.float64 else f.astype(np.float32).astype(np.float64)
        ref = nn.box_filter(fin, 4) - c0.astype(np.float64)
        out = torch.from_numpy(c0.copy()).cuda()
        closure.sbli_box_filter(torch.from_numpy(f).to(dt).cuda(), n, 5, 4, out, subtract=True)
        got = out.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - ref) <= U * np.abs(ref) + 1e-13 * np.abs(nn.box_filter(fin, 4)) + 1e-30)


def test_attach_rejects_a_network_on_another_stream():
    closure, torch = _mods()
    import paper_1609_01277_amd as sbli
    s = sbli.Solver(32, order=4, dtype="f32", **synth.TGV)
    other = torch.cuda.Stream()
    net = closure.ClosureNet(32, 1, stream=other)
    with pytest.raises(sbli.SbliError) as ei:
        closure.attach(s, net)
    assert ei.value.code == sbli.SBLI_ERR_ARG and "stream" in str(ei.value)
    net.close()
    net2 = closure.ClosureNet(32, 1)
    closure.attach(s, net2)
    closure.attach(s, None)
    net2.close()
    s.close()


def test_weight_gradient_at_96_cube_matches_oracle():
    """dW and db at 96^3, batch 1, 5 -> 8 channels: a grid that is not a power of
    two, so each of the weight-gradient kernel's 512 workgroups takes 54 blocks of 32
    points (not a whole number of 3-block x-rows), with 8 of the 32 output rows live."""
    closure, torch = _mods()
    n, cin, cout = 96, 5, 8
    P = n ** 3
    rng = np.random.default_rng(96)
    x = np.zeros((1, P, 8), dtype=np.float32)
    x[..., :cin] = bf16(rng.standard_normal((1, P, cin)))
    d = np.zeros((1, P, 8), dtype=np.float32)
    d[..., :cout] = bf16(rng.standard_normal((1, P, cout)))
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(torch.bfloat16).cuda()
    work = torch.empty(closure.sbli_conv3d_bwd_weight_work_bytes(cin) // 4, device="cuda")
    dW = torch.empty((cout, cin, 27), device="cuda")
    db = torch.empty(cout, device="cuda")
    closure.sbli_conv3d_bwd_weight(cu(x), cin, cu(d), cout, n, 1, dW, db, work)
    torch.cuda.synchronize()
    pl = lambda a, c: a.reshape(1, n, n, n, -1)[..., :c].transpose(0, 4, 1, 2, 3).astype(np.float64)
    xs, ds = pl(x, cin), pl(d, cout)
    rW, rb = nn.conv3d_bwd_weight(xs, ds)
    aW, ab = nn.conv3d_bwd_weight(np.abs(xs), np.abs(ds))
    # per workgroup 54 blocks x 2 MFMA steps of 16 products, then 512 partials in four chains
    _check_sum(to_host(dW).reshape(cout, cin, 3, 3, 3), rW, aW, 2 * 54 * 16 + 130, "dW")
    _check_sum(to_host(db), rb, ab, 128 + 256 + 64 + 8, "db")
