"""Learned closure on the GPU against the FP64 closure oracle (oracle/nn.py).

The GPU network computes in BF16 (weights, activations, gradients) with FP32
accumulation.  The oracle is evaluated on the same BF16-rounded operands at the
same points (inputs of every convolution), in FP64; the tolerance (2e-2, relative)
covers FP32 accumulation order and the rare BF16 rounding of an intermediate that
lands on the other side of a rounding boundary.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import nn

pytestmark = pytest.mark.gpu

TOL_BF16 = 2e-2


def _mods():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a HIP device")
    import paper_1609_01277_amd as sbli
    from paper_1609_01277_amd import closure
    return sbli, closure, torch


def bf16(a):
    """Round to bfloat16 (nearest, ties to even), returned as float64."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def rel_norm(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def make_case(n=32, seed=0):
    rng = np.random.default_rng(seed)
    q = synth.random_conservative_state(n, seed=seed + 1, mom=0.5).astype(np.float32)[None]
    t = (0.05 * rng.standard_normal((1, 5, n, n, n))).astype(np.float32)
    layers = nn.init_params(rng)
    layers = [(W, 0.1 * rng.standard_normal(b.shape)) for W, b in layers]
    stats = np.zeros(35, dtype=np.float32)
    stats[0:5] = q[0].reshape(5, -1).mean(axis=1)
    stats[5:10] = q[0].reshape(5, -1).std(axis=1)
    stats[10:15] = 0.01 * np.arange(5)
    stats[15:20] = 0.05
    stats[20:25] = np.inf
    return q, t, layers, stats


def oracle_pass(q, t, layers, stats):
    """FP64 network on BF16-rounded operands, rounding where the GPU rounds."""
    x = bf16((q.astype(np.float64) - stats[0:5, None, None, None]) / stats[5:10, None, None, None])
    Wb = [bf16(W) for W, _ in layers]
    bs = [b.astype(np.float32).astype(np.float64) for _, b in layers]
    pre1 = nn.conv3d(x, Wb[0], bs[0])
    h1 = bf16(nn.gelu(pre1))
    pre2 = nn.conv3d(h1, Wb[1], bs[1])
    h2 = bf16(nn.gelu(pre2))
    y = nn.conv3d(h2, Wb[2], bs[2])
    out = y * stats[15:20, None, None, None] + stats[10:15, None, None, None]
    ts = (t.astype(np.float64) - stats[10:15, None, None, None]) / stats[15:20, None, None, None]
    loss, dy = nn.mse(y, ts)
    dyb = bf16(dy)
    g3 = nn.conv3d_bwd_weight(h2, dyb)
    d2 = bf16(nn.conv3d_bwd_data(dyb, Wb[2]) * nn.gelu_grad(pre2))
    g2 = nn.conv3d_bwd_weight(h1, d2)
    d1 = bf16(nn.conv3d_bwd_data(d2, Wb[1]) * nn.gelu_grad(pre1))
    g1 = nn.conv3d_bwd_weight(x, d1)
    return out, loss, [g1, g2, g3]


def test_box_filter_matches_oracle():
    sbli, closure, torch = _mods()
    n = 64
    f = synth.random_conservative_state(n, seed=3)
    ref = nn.box_filter(f, 4)
    for dt in (torch.float64, torch.float32):
        fd = torch.from_numpy(f).to(dt).cuda()
        out = torch.empty((5, n // 4, n // 4, n // 4), dtype=torch.float32, device="cuda")
        closure.sbli_box_filter(fd, n, 5, 4, out)
        got = out.cpu().numpy()
        for c in range(5):
            assert np.abs(got[c] - ref[c]).max() <= 1e-6 * np.abs(ref[c]).max()


def test_channel_stats_and_guard():
    sbli, closure, torch = _mods()
    n = 32
    net = closure.ClosureNet(n, 1)
    data = torch.from_numpy(synth.random_conservative_state(n, seed=4).astype(np.float32)[None]).cuda()
    net.channel_stats(data, 0)
    st = net.get_stats()
    d = data.cpu().numpy()[0].reshape(5, -1).astype(np.float64)
    assert np.allclose(st[0:5], d.mean(axis=1), rtol=1e-6, atol=1e-7)
    assert np.allclose(st[5:10], d.std(axis=1), rtol=1e-5)
    assert np.array_equal(st[25:30], np.abs(data.cpu().numpy()[0]).reshape(5, -1).max(axis=1))
    st[20:25] = 2.0
    st[15:20] = 1.0
    net.set_stats(st)
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(2, dtype=torch.int32, device="cuda")
    c = torch.ones((5, n, n, n), dtype=torch.float32, device="cuda")
    net.guard(c, flag, cnt)
    assert int(flag) == 1
    c[3, 1, 2, 3] = float("nan")
    net.guard(c, flag, cnt)
    assert int(flag) == 0
    c[3, 1, 2, 3] = 3.0
    net.guard(c, flag, cnt)
    assert int(flag) == 0
    assert cnt.cpu().tolist() == [1, 2]


def test_forward_and_gradients_match_oracle():
    sbli, closure, torch = _mods()
    n = 32
    q, t, layers, stats = make_case(n)
    net = closure.ClosureNet(n, 1)
    net.set_params(closure.join_params(layers).astype(np.float32))
    net.set_stats(stats)
    qd, td = torch.from_numpy(q).cuda(), torch.from_numpy(t).cuda()
    out = net.forward(qd).cpu().numpy()
    loss = net.gradients(qd, td)
    grads = closure.split_params(net.get_grads().astype(np.float64))
    ref_out, ref_loss, ref_grads = oracle_pass(q, t, layers, stats)
    assert np.abs(out - ref_out).max() <= TOL_BF16 * np.abs(ref_out).max()
    assert abs(loss - ref_loss) <= TOL_BF16 * ref_loss
    for li, ((dW, db), (rW, rb)) in enumerate(zip(grads, ref_grads)):
        assert rel_norm(dW, rW) <= TOL_BF16, (li, rel_norm(dW, rW))
        assert rel_norm(db, rb) <= TOL_BF16, (li, rel_norm(db, rb))


def test_conservative_forward_removes_box_means():
    # batch of two different samples: the conservative output is the plain output minus
    # each (sample, field) box mean, against the oracle's output with its box means removed
    sbli, closure, torch = _mods()
    n = 32
    q, t, layers, stats = make_case(n)
    q2 = np.concatenate([q, make_case(n, seed=5)[0]])
    net = closure.ClosureNet(n, 2)
    net.set_params(closure.join_params(layers).astype(np.float32))
    net.set_stats(stats)
    qd = torch.from_numpy(q2).cuda()
    plain = net.forward(qd).cpu().numpy().astype(np.float64)
    net.set_conservative(True)
    cons = net.forward(qd).cpu().numpy().astype(np.float64)
    net.set_conservative(False)
    assert np.array_equal(net.forward(qd).cpu().numpy().astype(np.float64), plain)
    scale = np.abs(plain).max()
    # what the GPU removed is its own output's box mean (FP64 sums, one FP32 rounding)
    assert np.abs(cons - nn.remove_box_mean(plain)).max() <= 1e-6 * scale
    assert np.abs(cons.mean(axis=(2, 3, 4))).max() <= 1e-6 * scale
    for b in range(2):
        ref_out = oracle_pass(q2[b:b + 1], t, layers, stats)[0]
        ref = nn.remove_box_mean(ref_out[None] if ref_out.ndim == 4 else ref_out)
        assert np.abs(cons[b:b + 1] - ref.reshape(cons[b:b + 1].shape)).max() <= TOL_BF16 * np.abs(ref_out).max()
    assert closure._L().sbli_net_set_conservative(net.net, 2) == sbli.SBLI_ERR_ARG


def test_adam_step_matches_oracle():
    sbli, closure, torch = _mods()
    n = 32
    q, t, layers, stats = make_case(n, seed=5)
    net = closure.ClosureNet(n, 1)
    p0 = closure.join_params(layers).astype(np.float32)
    net.set_params(p0)
    net.set_stats(stats)
    qd, td = torch.from_numpy(q).cuda(), torch.from_numpy(t).cuda()
    l0 = net.train_step(qd, td, 1e-3)
    g = net.get_grads().astype(np.float64)
    p1 = net.get_params().astype(np.float64)
    ref, _, _ = nn.adam_step(p0.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, 1e-3)
    assert np.abs(p1 - ref).max() <= 1e-6
    losses = [l0] + [net.train_step(qd, td, 1e-3) for _ in range(8)]
    assert losses[-1] < losses[0]


def _solver_pair(n, torch, sbli):
    s = sbli.Solver(n, order=4, dtype="f32", **synth.TGV)
    return s


def test_closure_attach_constant_term_matches_oracle():
    """Weights zero, output bias b3: the closure is the constant field b3*std + mean,
    so the augmented RK3 equals the oracle's RK3 on R(q) + c."""
    sbli, closure, torch = _mods()
    n, dt, steps = 32, 3.385e-3, 2
    net = closure.ClosureNet(n, 1)
    layers = [(np.zeros_like(W), np.zeros_like(b)) for W, b in nn.init_params(np.random.default_rng(0))]
    b3 = np.array([0.5, -0.3, 0.2, 0.1, -0.4])
    layers[2] = (layers[2][0], b3)
    net.set_params(closure.join_params(layers).astype(np.float32))
    stats = np.zeros(35, dtype=np.float32)
    stats[5:10] = 1.0
    stats[10:15] = [0.1, 0.2, 0.0, -0.1, 0.3]
    stats[15:20] = 2.0
    stats[20:25] = 100.0
    net.set_stats(stats)
    c = b3.astype(np.float32).astype(np.float64) * 2.0 + stats[10:15].astype(np.float64)
    p = oracle.Params(n=(n, n, n), order=4, **synth.TGV)
    q0 = oracle.tgv_init(p)
    ref = oracle.rk3_generic(q0.ravel(), dt, steps,
                             lambda y: (oracle.rhs(y.reshape(q0.shape), p)
                                        + c[:, None, None, None]).ravel()).reshape(q0.shape)
    s = _solver_pair(n, torch, sbli)
    closure.attach(s, net)
    q = torch.from_numpy(q0.astype(np.float32)).cuda()
    s.rk3_step(q, s.empty_state(), s.empty_state(), dt, steps)
    got = q.cpu().numpy()
    mom = np.abs(ref[1:4]).max()
    for f in range(5):
        scale = mom if f in (1, 2, 3) else np.abs(ref[f]).max()
        assert np.abs(got[f] - ref[f]).max() / scale <= 1e-5, f
    acc, rej = closure.counts(s)
    assert (acc, rej) == (3 * steps, 0)


def test_closure_fallback_when_guard_rejects_or_detached():
    sbli, closure, torch = _mods()
    n, dt = 32, 3.385e-3
    net = closure.ClosureNet(n, 1)
    layers = [(np.zeros_like(W), np.zeros_like(b)) for W, b in nn.init_params(np.random.default_rng(0))]
    layers[2] = (layers[2][0], np.full(5, 0.7))
    net.set_params(closure.join_params(layers).astype(np.float32))
    stats = np.zeros(35, dtype=np.float32)
    stats[5:10] = 1.0
    stats[15:20] = 1.0
    stats[20:25] = 0.5            # |C| = 0.7 exceeds every limit: always rejected
    net.set_stats(stats)
    s = sbli.Solver(n, order=4, dtype="f32", **synth.TGV)
    q_plain = s.tgv_init(s.empty_state())
    q_guard = q_plain.clone()
    s.rk3_step(q_plain, s.empty_state(), s.empty_state(), dt, 2)
    closure.attach(s, net)
    s.rk3_step(q_guard, s.empty_state(), s.empty_state(), dt, 2)
    assert torch.equal(q_plain, q_guard)
    assert closure.counts(s) == (0, 6)
    closure.attach(s, None)
    q_det = s.tgv_init(s.empty_state())
    s.rk3_step(q_det, s.empty_state(), s.empty_state(), dt, 2)
    assert torch.equal(q_plain, q_det)


def test_closure_term_same_in_staged_form():
    """With a network attached, the staged form of the stage kernel adds the same closure
    term as the fused variants: bitwise equal states after RK3 steps."""
    sbli, closure, torch = _mods()
    n, dt = 32, 3.385e-3
    net = closure.ClosureNet(n, 1)
    net.set_params(closure.join_params(nn.init_params(np.random.default_rng(4))).astype(np.float32) * 0.05)
    stats = np.zeros(35, dtype=np.float32)
    stats[5:10] = 1.0
    stats[15:20] = 1.0
    stats[20:25] = 1e3            # generous limits: every evaluation accepted
    net.set_stats(stats)
    s = sbli.Solver(n, order=4, dtype="f32", **synth.TGV)
    closure.attach(s, net)
    staged = len(s.variants()) - 1
    out = []
    for v in (0, staged):
        s.set_tuning(v, n)
        q = s.tgv_init(s.empty_state())
        s.rk3_step(q, s.empty_state(), s.empty_state(), dt, 2)
        out.append(q.cpu().numpy())
    accepted, rejected = closure.counts(s)
    assert accepted == 12 and rejected == 0
    assert np.array_equal(out[0], out[1])
    plain = sbli.Solver(n, order=4, dtype="f32", **synth.TGV)
    qp = plain.tgv_init(plain.empty_state())
    plain.rk3_step(qp, plain.empty_state(), plain.empty_state(), dt, 2)
    assert not np.array_equal(out[0], qp.cpu().numpy())   # the term is not zero
