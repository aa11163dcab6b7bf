"""GPU checks of the learned-shrinkage kernels (MFMA, bfloat16 operands,
float32 accumulation) against the FP64 oracle with bfloat16 emulation, and
of the transform adjoint used to back-propagate an image-domain loss.

Tolerances: gains and gradients relative L2 <= 1e-3 (the oracle rounds the
same operands to bfloat16; what remains is float32-vs-float64 accumulation
order, which can flip an occasional bfloat16 rounding of an activation);
adjoint relative L2 <= 1e-5 (float32 transform)."""
import numpy as np
import pytest

from oracle import cnn as OC
from oracle import system as S
from oracle import transform as T
from paper_1402_5670_amd import synthetic as syn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1402_5670_amd import binding as B  # noqa: E402

DEV = torch.device("cuda:0")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def blob(p):
    return np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"], p["W3"].ravel(),
                           p["b3"]])


def unblob(v):
    v = np.asarray(v, dtype=np.float64)
    return {"W1": v[0:576].reshape(32, 2, 3, 3), "b1": v[576:608],
            "W2": v[608:9824].reshape(32, 32, 3, 3), "b2": v[9824:9856],
            "W3": v[9856:10144].reshape(1, 32, 3, 3), "b3": v[10144:10145]}


def _setup(dims=(64, 64), J=2, levels=(1, 1), Bn=2, seed=0):
    sysg = B.System(dims, J, levels)
    sig = np.array([0.05 + 0.05 * b for b in range(Bn)], dtype=np.float32)
    xs = np.stack([syn.noisy_cartoon2d(*dims, 100 + b, float(sig[b]))[1] for b in range(Bn)])
    c, _ = sysg.forward(_gpu(xs))
    torch.cuda.synchronize()
    params = []
    for j in range(J):
        p = OC.init_params(32, seed=seed + j)
        rng = np.random.default_rng(seed + 10 + j)
        for k in ("b1", "b2", "b3"):
            p[k] = rng.standard_normal(p[k].shape) * 0.1
        params.append(p)
    pg = _gpu(np.stack([blob(p) for p in params]))
    return sysg, sig, c, params, pg


def test_inverse_adjoint():
    print("case: adjoint 64x48 J=2 d=[1,1] B=2", flush=True)
    dims = (64, 48)
    sysg = B.System(dims, 2, [1, 1])
    o = S.build_2d(dims, 2, [1, 1])
    rng = np.random.default_rng(4)
    r = rng.standard_normal((2, *dims))
    c = rng.standard_normal((2, sysg.R, *dims))
    a = sysg.inverse_adjoint(_gpu(r))
    x = sysg.inverse(_gpu(c))
    torch.cuda.synchronize()
    an = a.cpu().numpy().astype(np.float64)
    for b in range(2):
        R = np.fft.fft2(r[b]) / o.dual_weight
        ref = np.stack([np.fft.ifft2(R * f).real for f in o.filters])
        assert rel(an[b], ref) < 1e-5
    lhs = np.sum(x.cpu().numpy().astype(np.float64) * r)
    rhs = np.sum(c * an)
    assert abs(lhs - rhs) < 1e-5 * np.linalg.norm(c) * np.linalg.norm(an)


@pytest.mark.parametrize("dims", [(64, 64), (24, 48)])
def test_cnn_forward_matches_oracle(dims):
    # 24 x 48 leaves partial 16 x 32 output tiles in both directions
    print(f"case: cnn apply {dims} J=2 B=2 (32 planes)", flush=True)
    sysg, sig, c, params, pg = _setup(dims=dims)
    net = B.Shrinkage(sysg, pg)
    gains = torch.zeros_like(c)
    out = net.apply(c, _gpu(sig), gains=gains)
    torch.cuda.synchronize()
    cn = c.cpu().numpy().astype(np.float64)
    gn = gains.cpu().numpy()
    on = out.cpu().numpy()
    assert np.array_equal(on[:, 0], c.cpu().numpy()[:, 0])        # lowpass copied
    l2 = np.array([s[4] for s in sysg.subbands], dtype=np.float32)
    num = den = 0.0
    for b in range(c.shape[0]):
        for i in range(1, sysg.R):
            j = sysg.subbands[i][1]
            g, _ = OC.forward(params[j], cn[b, i], float(sig[b]), float(l2[i]), bf16=True)
            num += np.sum((gn[b, i] - g) ** 2)
            den += np.sum(g ** 2)
            assert np.allclose(on[b, i], gn[b, i] * cn[b, i], rtol=1e-6, atol=1e-7)
    assert np.sqrt(num / den) < 1e-3


@pytest.mark.parametrize("dims", [(96, 192), (96, 48)])
def test_fused_and_layerwise_inference_agree(monkeypatch, dims):
    # the fused tile kernel and the layer-by-layer path compute the same network;
    # they differ only in the float32 summation order (layer 1 packs its taps
    # into one product, layer 3 sums per-tap partial products)
    print(f"case: cnn fused vs layerwise {dims} J=2 B=2", flush=True)
    sysg, sig, c, params, pg = _setup(dims=dims)
    net = B.Shrinkage(sysg, pg)
    g1 = torch.zeros_like(c)
    net.apply(c, _gpu(sig), gains=g1)
    monkeypatch.setenv("SL_CNN_LAYERWISE", "1")
    g2 = torch.zeros_like(c)
    net.apply(c, _gpu(sig), gains=g2)
    torch.cuda.synchronize()
    assert rel(g1[:, 1:].cpu().numpy(), g2[:, 1:].cpu().numpy()) < 1e-3


def test_cnn_backward_matches_oracle():
    print("case: cnn backward 64x64 J=2 B=2", flush=True)
    sysg, sig, c, params, pg = _setup(seed=3)
    net = B.Shrinkage(sysg, pg)
    rng = np.random.default_rng(7)
    dc = rng.standard_normal(tuple(c.shape)).astype(np.float32)
    grads = net.backward(c, _gpu(sig), _gpu(dc))
    torch.cuda.synchronize()
    gg = grads.cpu().numpy()
    cn = c.cpu().numpy().astype(np.float64)
    l2 = np.array([s[4] for s in sysg.subbands], dtype=np.float32)
    ref = [{k: np.zeros_like(v) for k, v in params[j].items()} for j in range(sysg.n_scales)]
    absdz = np.zeros(sysg.n_scales)
    for b in range(c.shape[0]):
        for i in range(1, sysg.R):
            j = sysg.subbands[i][1]
            g, cache = OC.forward(params[j], cn[b, i], float(sig[b]), float(l2[i]), bf16=True)
            dg = dc[b, i].astype(np.float64) * cn[b, i]
            gr = OC.backward(cache, dg)
            absdz[j] += np.sum(np.abs(OC.bf16_round(dg * g * (1 - g))))
            for k in gr:
                ref[j][k] += gr[k]
    for j in range(sysg.n_scales):
        got = unblob(gg[j])
        for k in ref[j]:
            if k == "b3":
                # a scalar sum of +- bf16-rounded terms: bound the error by the sum of the
                # terms' magnitudes (cancellation makes the plain relative error ill-posed)
                assert abs(got[k][0] - ref[j][k][0]) < 1e-3 * absdz[j]
            else:
                assert rel(got[k], ref[j][k]) < 1e-3, (j, k, rel(got[k], ref[j][k]))


def test_training_reduces_loss():
    # a few Adam steps on one batch: the image-domain loss must go down
    print("case: cnn training smoke 64x64", flush=True)
    sysg, sig, c, params, pg = _setup(seed=5)
    dims = sysg.dims
    clean = np.stack([syn.cartoon2d(*dims, 100 + b) for b in range(2)])
    cg = _gpu(clean)
    net = B.Shrinkage(sysg, pg)
    m = torch.zeros_like(pg)
    v = torch.zeros_like(pg)
    scratch = torch.zeros(B.SQERR_SCRATCH, dtype=torch.float32, device=DEV)
    sg = _gpu(sig)
    losses = []
    n = clean.size
    for step in range(1, 31):
        shrunk = net.apply(c, sg)
        xh = sysg.inverse(shrunk)
        r = torch.empty_like(xh)
        B.sq_error_grad(xh, cg, 2.0 / n, r, scratch)
        dc = sysg.inverse_adjoint(r)
        grads = net.backward(c, sg, dc)
        B.adam_step(net.params, grads, m, v, 2e-3, step)
        net.pack()
        torch.cuda.synchronize()
        losses.append(float(scratch[0].item()) / n)
    assert losses[-1] < 0.9 * losses[0], losses
    assert np.isfinite(losses).all()


def test_cnn_forward_multi_tile_matches_oracle():
    # 128 x 128 planes hold 8 x 4 output tiles of 16 x 32; B = 2 and R = 17 give
    # 32 detail planes = 1024 tiles on a grid of at most 256 persistent blocks, so
    # each block runs the prefetch / double-buffer loop over several tiles, and
    # block b's tiles (b, b + 256, ...) lie in planes b // 32, b // 32 + 8, ...:
    # the first is a scale-0 plane and the second a scale-1 plane, so the
    # per-scale weights are reloaded inside the loop.
    print("case: cnn apply 128x128 J=2 B=2 (1024 tiles, multi-tile loop)", flush=True)
    sysg, sig, c, params, pg = _setup(dims=(128, 128), seed=11)
    net = B.Shrinkage(sysg, pg)
    gains = torch.zeros_like(c)
    out = net.apply(c, _gpu(sig), gains=gains)
    torch.cuda.synchronize()
    cn = c.cpu().numpy().astype(np.float64)
    gn = gains.cpu().numpy()
    on = out.cpu().numpy()
    l2 = np.array([s[4] for s in sysg.subbands], dtype=np.float32)
    scales_seen = set()
    worst = 0.0
    diffs = []
    for b in range(c.shape[0]):
        for i in range(1, sysg.R):
            j = sysg.subbands[i][1]
            scales_seen.add(j)
            g, _ = OC.forward(params[j], cn[b, i], float(sig[b]), float(l2[i]), bf16=True)
            # each plane within 1e-3 relative L2; element-wise (gains lie in (0, 1))
            # within 5e-3: where float32 and float64 accumulation put an activation
            # on opposite sides of a bfloat16 rounding boundary, it moves by one
            # bfloat16 step (2^-8 relative), which reaches the gain scaled by the
            # next layers' weights and by g (1 - g) <= 1/4
            d = np.abs(gn[b, i] - g)
            worst = max(worst, float(np.max(d)))
            diffs.append(d.ravel())
            assert rel(gn[b, i], g) < 1e-3, (b, i, rel(gn[b, i], g))
            assert np.allclose(on[b, i], gn[b, i] * cn[b, i], rtol=1e-6, atol=1e-7)
    q = np.quantile(np.concatenate(diffs), [0.5, 0.99, 0.999])
    print(f"|gain - oracle|: median {q[0]:.1e}, 99% {q[1]:.1e}, 99.9% {q[2]:.1e}, "
          f"max {worst:.2e}", flush=True)
    assert worst < 5e-3
    assert scales_seen == {0, 1}


def test_adam_matches_oracle_over_steps():
    # sl_cnn_adam against the oracle's Adam (float64) over five steps with
    # changing gradients and learning rates; from step 2 on beta1 and beta2 enter
    # the moments differently, so the comparison covers the recurrences and the
    # bias corrections, not just the first step
    print("case: adam 5 steps, 2 x 10145 parameters", flush=True)
    from oracle import cnn as OCN
    rng = np.random.default_rng(21)
    n = 2 * B.CNN_PARAMS
    p0 = rng.standard_normal(n) * 0.1
    pg = _gpu(p0)
    m = torch.zeros_like(pg)
    v = torch.zeros_like(pg)
    ref = {"w": p0.astype(np.float32).astype(np.float64)}
    st = {}
    for t in range(1, 6):
        g = rng.standard_normal(n) * (0.5 ** t) + 0.01 * t
        lr = 1e-3 * (1.0 + 0.25 * t)
        g32 = g.astype(np.float32)
        B.adam_step(pg, _gpu(g32), m, v, lr, t)
        OCN.adam_step(ref, {"w": g32.astype(np.float64)}, st, lr=np.float32(lr))
        torch.cuda.synchronize()
        got_p = pg.cpu().numpy().astype(np.float64)
        got_m = m.cpu().numpy().astype(np.float64)
        got_v = v.cpu().numpy().astype(np.float64)
        assert rel(got_m, st["m_w"]) < 1e-6, (t, rel(got_m, st["m_w"]))
        assert rel(got_v, st["v_w"]) < 1e-6, (t, rel(got_v, st["v_w"]))
        assert rel(got_p, ref["w"]) < 1e-6, (t, rel(got_p, ref["w"]))
        # the accumulated update itself (not only the parameters, which it barely moves)
        upd_got = got_p - p0.astype(np.float32)
        upd_ref = ref["w"] - p0.astype(np.float32)
        assert rel(upd_got, upd_ref) < 1e-4, (t, rel(upd_got, upd_ref))


@pytest.mark.parametrize("n", [1, 1000, 256 * 1024 + 37])
def test_sq_error_grad_matches_float64(n):
    # out = scale (a - b) and loss = sum (a - b)^2 against float64 sums of the same
    # float32 inputs; n = 1 and a ragged n exercise the grid-stride loop's ends
    print(f"case: sq_error_grad n={n}", flush=True)
    rng = np.random.default_rng(n)
    a = rng.standard_normal(n).astype(np.float32)
    b = (a + rng.standard_normal(n) * 0.1).astype(np.float32)
    scale = 2.0 / n
    out = torch.empty(n, dtype=torch.float32, device=DEV)
    scratch = torch.full((B.SQERR_SCRATCH,), 7.0, dtype=torch.float32, device=DEV)
    B.sq_error_grad(_gpu(a), _gpu(b), scale, out, scratch)
    torch.cuda.synchronize()
    d = a.astype(np.float64) - b.astype(np.float64)
    ref_out = np.float32(scale) * d
    assert rel(out.cpu().numpy(), ref_out) < 1e-6
    loss = float(scratch[0].item())
    ref_loss = float(np.sum(d * d))
    assert abs(loss - ref_loss) < 1e-5 * ref_loss, (loss, ref_loss)
