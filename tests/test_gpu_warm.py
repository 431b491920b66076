"""Warm-start network on the GPU against the FP64 reference of the network, plus the objective
check that guards the warm start (a fallback to the cold start y = 0 of Algorithm 2)."""
import numpy as np
import pytest
import torch

from gpu_common import DEV, dev, host, orc, say
from oracle import mlp_ref as M
from paper_1502_01645_amd import nnls as N
from paper_1502_01645_amd import workloads as W

pytestmark = pytest.mark.gpu

LAM = 0.01


def _offsets():
    out, off = {}, 0
    for name, shape in M.SIZES:
        size = int(np.prod(shape))
        out[name] = (off, off + size)
        off += size
    return out


OFF = _offsets()


@pytest.fixture(scope="module")
def params():
    p = W.make_mlp_params(11).astype(np.float64)
    rng = np.random.default_rng(12)
    for name in ("b1", "b2", "b3"):  # nonzero biases so every bias path carries signal
        a, b = OFF[name]
        p[a:b] = 0.05 * rng.standard_normal(b - a)
    return p.astype(np.float32)


def _batch(b, seed):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((b, 256))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    t = np.where(rng.random((b, 256)) < 0.85, 0.0, 0.05 * rng.gamma(1.5, 1.0, (b, 256)))
    return u.astype(np.float32), t.astype(np.float32)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _norm(seed):
    rng = np.random.default_rng(seed)
    shift = (0.05 * rng.standard_normal(256)).astype(np.float32)
    scale = rng.uniform(0.5, 3.0, 256).astype(np.float32)
    return shift, scale


@pytest.mark.parametrize("batch,standardise", [(64, False), (192, True)])
def test_forward_matches_reference(params, batch, standardise):
    say(f"mlp forward batch={batch} standardise={standardise}")
    u, _ = _batch(batch, batch)
    shift, scale = _norm(batch) if standardise else (None, None)
    net = N.WarmStartNet(params, DEV, shift, scale)
    z = host(net.forward(dev(u)))
    z_em, _ = M.forward(params, u, True, shift, scale)
    assert _rel(z, z_em) <= 1e-3, _rel(z, z_em)
    # against exact FP64 arithmetic on the FP32 parameters: BF16 operands cost ~2^-8 relative
    z_ex, _ = M.forward(params, u, False, shift, scale)
    assert _rel(z, z_ex) <= 3e-2, _rel(z, z_ex)


def test_gradients_match_reference(params):
    say("mlp gradients batch=128")
    u, t = _batch(128, 3)
    shift, scale = _norm(3)
    net = N.WarmStartNet(params, DEV, shift, scale)
    loss, g = net.gradients(dev(u), dev(t), LAM)
    loss, g = float(host(loss)[0]), host(g).astype(np.float64)
    loss_ref, g_ref = M.gradients(params, u, t, LAM, True, shift, scale)
    assert abs(loss - loss_ref) <= 1e-4 * abs(loss_ref), (loss, loss_ref)
    for name, (a, b) in OFF.items():
        r = _rel(g[a:b], g_ref[a:b])
        say(f"  grad {name}: rel {r:.2e}")
        assert r <= 1e-3, (name, r)


def test_adam_first_step_and_bf16_copy(params):
    """Adam's bias-corrected first step is lr * g / (|g| + eps) exactly; the BF16 copy follows
    the master weights with round-to-nearest-even."""
    say("mlp adam step")
    u, t = _batch(64, 5)
    net = N.WarmStartNet(params, DEV)
    _, g = net.gradients(dev(u), dev(t), LAM)
    g = host(g).astype(np.float64)
    lr = 1e-3
    net.train_step(dev(u), dev(t), lr, LAM)
    w1 = host(net.master).astype(np.float64)
    w0 = params.astype(np.float64)
    expect = w0 - lr * g / (np.abs(g) + 1e-8)
    err = np.abs(w1 - expect)
    assert np.all(err <= 1e-6 * lr + 2 * 2.0 ** -24 * np.abs(w0) + 1e-12), err.max()
    P = net.P
    copy = host(net.blob[12 * P:14 * P].view(torch.int16)).astype(np.uint16)
    want = M.bf16(host(net.master)).astype(np.float32).view(np.uint32) >> 16
    assert np.array_equal(copy, want.astype(np.uint16))


def test_fit_input_statistics(params):
    """shift and scale are the FP64 mean and 1 / std of each feature; a constant feature gets
    scale 1.  Rows that differ by a tiny fraction of their size keep their spread."""
    rng = np.random.default_rng(8)
    U = (0.0625 + 5e-4 * rng.standard_normal((5000, 256))).astype(np.float32)
    U[:, 7] = 0.25
    net = N.WarmStartNet(params, DEV)
    net.fit_input(dev(U))
    U64 = U.astype(np.float64)
    mu, sd = U64.mean(0), U64.std(0)
    np.testing.assert_allclose(host(net.shift), mu.astype(np.float32), rtol=1e-6)
    sc = host(net.scale)
    assert sc[7] == 1.0
    keep = np.arange(256) != 7
    np.testing.assert_allclose(sc[keep], 1.0 / sd[keep], rtol=1e-5)


def test_reset_state_clears_moments(params):
    net = N.WarmStartNet(params, DEV)
    u, t = _batch(64, 6)
    net.train_step(dev(u), dev(t), 1e-3, LAM)
    assert N.lib().nnls_mlp_reset_state(N._ptr(net.blob), N._stream(DEV)) == 0
    P = net.P
    mv = host(net.blob[4 * P:12 * P].view(torch.float32))
    assert np.all(mv == 0)


def test_checkpoint_resumes_training_exactly(params, tmp_path):
    """Training resumed from a checkpoint (nnls_mlp_save / nnls_mlp_load) takes the same steps,
    bit for bit, as training that never stopped: the file holds the master weights, both Adam
    moments, the BF16 copy, the input standardisation and the step count."""
    say("mlp checkpoint save / load / resume")
    shift, scale = _norm(9)
    net = N.WarmStartNet(params, DEV, shift, scale)
    batches = [_batch(64, 40 + i) for i in range(6)]
    for u, t in batches[:3]:
        net.train_step(dev(u), dev(t), 1e-3, LAM)
    path = tmp_path / "net.ckpt"
    net.save(path)
    saved = host(net.blob).copy()
    for u, t in batches[3:]:
        net.train_step(dev(u), dev(t), 1e-3, LAM)
    torch.cuda.synchronize()
    straight = host(net.blob).copy()

    back = N.WarmStartNet.from_checkpoint(path, DEV)
    assert back.step == 3
    assert np.array_equal(host(back.blob), saved)
    for u, t in batches[3:]:
        back.train_step(dev(u), dev(t), 1e-3, LAM)
    torch.cuda.synchronize()
    assert back.step == 6
    assert np.array_equal(host(back.blob), straight)
    # a damaged file is refused and leaves the blob as it was
    raw = bytearray(path.read_bytes())
    raw[64 + 1000] ^= 0x40
    bad = tmp_path / "bad.ckpt"
    bad.write_bytes(bytes(raw))
    with pytest.raises(N.NNLSError):
        back.load(bad)
    assert np.array_equal(host(back.blob), straight)


def _warm_problem(k, seed):
    A = W.make_warm_matrix()
    B, _ = W.make_warm_rhs(A, k, split=1, start=seed)
    return A, B


def _mixed_problem(k, seed):
    """A general problem whose q has entries of both signs (A, B ~ N(0, 1))."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((600, 256)).astype(np.float32)
    B = rng.standard_normal((600, k)).astype(np.float32)
    return A, B


def _net_with_head(params, z_head):
    """A network whose output is z_head for every input: W3 = 0, b3 = z_head."""
    p = params.copy()
    a, b = OFF["W3"]
    p[a:b] = 0.0
    a, b = OFF["b3"]
    p[a:b] = z_head
    return N.WarmStartNet(p, DEV)


@pytest.mark.parametrize("case", ["descent", "ascent", "zero"])
def test_warm_start_line_search_and_fallback(params, case):
    """Direction v: y0 = c* v with c* = -q'v / v'Qv when q'v < 0; v = max(-q, 0) gives
    c* = ||v||^2 / v'Qv.  v = max(q, 0) has q'v = ||v||^2 > 0 and v = 0 has nothing to scale:
    both fall back to the cold start, which then solves exactly as a cold solve."""
    say(f"warm start {case}")
    A, B = _mixed_problem(1, 21)
    Q, q, s = N.prepare(dev(A), dev(B))
    Qh, qh = host(Q).astype(np.float64), host(q)[:, 0].astype(np.float64)
    v = {"descent": np.maximum(-qh, 0.0), "ascent": np.maximum(qh, 0.0),
         "zero": np.zeros_like(qh)}[case]
    head = v if case != "zero" else -np.ones_like(qh)
    v = v.astype(np.float32).astype(np.float64)  # the head is stored in FP32
    net = _net_with_head(params, head.astype(np.float32))
    Y0, fb = net.warm_start(Q, q)
    Y0, fb = host(Y0)[:, 0], host(fb)
    if case == "descent":
        assert fb[0] == 0
        c = -(qh @ v) / (v @ Qh @ v)
        np.testing.assert_allclose(Y0, c * v, rtol=1e-5, atol=1e-6 * np.abs(c * v).max())
        f0 = 0.5 * Y0 @ Qh @ Y0 + qh @ Y0
        assert f0 < 0
    else:
        assert fb[0] == 1
        assert np.all(Y0 == 0)
        X_w, it_w, _, _ = N.solve(Q, q, s, 1e-5, 0, Y0=torch.zeros_like(q))
        X_c, it_c, _, _ = N.solve(Q, q, s, 1e-5, 0)
        assert np.array_equal(host(X_w), host(X_c))
        assert np.array_equal(host(it_w), host(it_c))


def test_warm_start_many_columns(params):
    """Across many right-hand sides with q of both signs, a column falls back exactly where
    q'v >= 0 for the network's direction v (columns with q'v within rounding of 0 may go either
    way), and elsewhere y0 = c* v."""
    k = 320
    say(f"warm start k={k}")
    A, B = _mixed_problem(k, 22)
    Q, q, s = N.prepare(dev(A), dev(B))
    net = N.WarmStartNet(params, DEV)
    Y0, fb = net.warm_start(Q, q)
    Qh, qh = host(Q).astype(np.float64), host(q).astype(np.float64)
    U, _ = N.mlp_inputs(q)
    z = host(net.forward(U)).astype(np.float64)
    v = np.maximum(z, 0.0).T                       # [256, k]
    a = np.einsum("ik,ij,jk->k", v, Qh, v)
    b = np.einsum("ik,ik->k", qh, v)
    scale = np.abs(qh * v).sum(0)
    fb = host(fb)
    sure = np.abs(b) > 1e-4 * scale
    say(f"  fallbacks {int(fb.sum())} of {k}; undecided {int((~sure).sum())}")
    assert 0 < fb.sum() < k
    assert np.array_equal(fb[sure], (b[sure] >= 0).astype(np.int32))
    Y0 = host(Y0)
    assert np.all(Y0[:, fb == 1] == 0)
    keep = fb == 0
    c = -b[keep] / a[keep]
    np.testing.assert_allclose(Y0[:, keep], c * v[:, keep], rtol=1e-4,
                               atol=1e-6 * np.abs(c * v[:, keep]).max())


def test_mlp_inputs(params):
    A, B = _warm_problem(70, 7)
    Q, q, s = N.prepare(dev(A), dev(B))
    X, _, _, _ = N.solve(Q, q, None, 1e-5, 0)
    U, T = N.mlp_inputs(q, X)
    qh, Yh = host(q).astype(np.float64), host(X).astype(np.float64)
    qn = np.linalg.norm(qh, axis=0)
    np.testing.assert_allclose(host(U), (qh / qn).T, rtol=1e-6, atol=1e-7)
    yn = np.linalg.norm(Yh, axis=0)
    np.testing.assert_allclose(host(T), (Yh / yn).T, rtol=1e-6, atol=1e-7)


def test_trained_network_gains_over_cold_start():
    """What the trained network gains, end to end with the library's own kernels: the network
    is trained on the method's solves of 120000 seeded right-hand sides of the warm-start recipe
    (A 4096 x 256 |N(0,1)|, noiseless b = A x, 85 % zeros), then 8192 held-out right-hand sides
    (more than the resident column slots, so the solve is throughput-bound) are solved from the
    cold start and from the network's start.  Both meet FP64 KKT <= 1e-5 on every column after
    the check; the warm start takes at most 3/4 of the cold start's updates on average and in
    total rows of Q read, and the whole warm step (network included) takes less time than the
    cold step.  (The test data b = A x is formed in FP64 by torch on the device.)"""
    import time
    ntr = 120000
    A_h = W.make_warm_matrix()
    A = dev(A_h)
    A64 = A.double()

    def rhs(count, split):
        X = torch.from_numpy(W.make_warm_codes(256, count, split)).to(DEV)
        return (A64 @ X).float().contiguous()
    Btr = rhs(ntr, 0)
    Bev = rhs(8192, 1)
    say(f"warm gain: {ntr} training solves, 8192 held-out")
    Qt, qt, _ = N.prepare(A, Btr)
    del Btr
    Ytr, _, _, st_tr = N.solve(Qt, qt, None, 3e-6, 20000)
    assert np.all(host(st_tr) == N.CONVERGED)
    U, T = N.mlp_inputs(qt, Ytr)
    net = N.WarmStartNet(W.make_mlp_params(0), DEV)
    net.fit_input(U)
    gen = torch.Generator(device=DEV)
    gen.manual_seed(0)
    loss = torch.zeros(1, device=DEV)
    epochs, bs, steps = 40, 512, ntr // 512
    total, step = epochs * steps, 0
    for ep in range(epochs):
        perm = torch.randperm(ntr, device=DEV, generator=gen)
        for b in range(steps):
            idx = perm[b * bs:(b + 1) * bs]
            lr = 1e-3 * 0.5 * (1.0 + np.cos(np.pi * step / total))
            net.train_step(U[idx].contiguous(), T[idx].contiguous(), lr, 1e-4, loss)
            step += 1
    torch.cuda.synchronize()
    say(f"  final batch loss {float(loss.item()):.5f}")
    k, n = 8192, 256

    def run(warm):
        best = None
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Q, q, s = N.prepare(A, Bev)
            Y0 = net.warm_start(Q, q)[0] if warm else None
            rows = torch.zeros(k, dtype=torch.int64, device=DEV)
            X, it, _, st = N.solve(Q, q, s, 8e-6, 5 * n, Y0=Y0, rows_read=rows)
            kkt64, _ = N.refine(A, Bev, X, objective=False)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            best = t if best is None else min(best, t)
        return best, host(it), host(st), host(kkt64), int(host(rows).sum())

    t_c, it_c, st_c, r_c, rows_c = run(False)
    t_w, it_w, st_w, r_w, rows_w = run(True)
    say(f"  cold: {it_c.mean():.1f} updates, {k / t_c:.0f} solves/s, max KKT {r_c.max():.2e}")
    say(f"  warm: {it_w.mean():.1f} updates, {k / t_w:.0f} solves/s, max KKT {r_w.max():.2e}")
    assert np.all(st_c == N.CONVERGED) and np.all(st_w == N.CONVERGED)
    assert r_c.max() <= 1e-5 and r_w.max() <= 1e-5
    assert it_w.mean() <= 0.75 * it_c.mean()
    assert rows_w <= 0.75 * rows_c
    assert t_w < t_c
