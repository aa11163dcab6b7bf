"""GPU parity of the wavelet system and of image decomposition (Algorithm 4)
through the C ABI.

The wavelet system's forward and inverse transforms match the FP64 oracle
to relative L2 <= 1e-5.  Decomposition iterations are checked on exact
decision sets, as for inpainting: iteration t is replayed from the GPU's
previous estimates (f0, f1); g0 = f - f1 and g1 = f - f0 are formed in
float32 as the kernel does, their coefficients taken from sl_forward on the
same systems, thresholded at the kernel's float32 thresholds and
reconstructed by the oracle; both estimates must match to <= 1e-5.  Full
runs must equal the chain of single iterations bit for bit (eager, graph,
segments).
"""
import ctypes

import numpy as np
import pytest

from oracle import decompose as D
from oracle import system as S
from oracle import transform as T
from paper_1402_5670_amd import metrics as M
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


@pytest.mark.parametrize("dims,J,Bn,dtype,tol", [
    ((64, 64), 3, 2, "f32", 1e-5), ((24, 96), 2, 3, "f32", 1e-5), ((512, 512), 4, 1, "f32", 1e-5),
    ((128, 128), 3, 2, "f16", 2e-3), ((128, 128), 3, 2, "bf16", 2e-3)])
def test_wavelet_system_parity(dims, J, Bn, dtype, tol):
    print(f"case: wavelet system {dims} J={J} B={Bn} {dtype}", flush=True)
    x = np.random.default_rng(51).standard_normal((Bn, *dims))
    sw = B.System(dims, J, wavelet=True, dtype=dtype)
    o = D.build_wavelet_2d(dims, J)
    assert sw.R == 3 * J + 1
    c, sc = sw.forward(_gpu(x))
    xr = sw.inverse(c, sc)
    torch.cuda.synchronize()
    cg = c.float().cpu().numpy().astype(np.float64)
    if dtype != "f32":
        cg = cg * sc.cpu().numpy().astype(np.float64)[:, :, None, None]
    # coefficients within tol; the reconstruction within tol, or for BF16 within
    # the coefficient error times sqrt(B / A) (frame bounds A = min Psi_hat,
    # B = max Psi_hat: the dual-frame inverse has norm 1 / sqrt(A), ||c|| <=
    # sqrt(B) ||x||)
    amp = np.sqrt(o.dual_weight.max() / o.dual_weight.min())
    for b in range(Bn):
        ec = rel(cg[b], T.forward(x[b], o.filters))
        ex = rel(xr[b].cpu().numpy(), x[b])
        assert ec < tol
        assert ex < (amp * ec + 1e-5 if dtype == "bf16" else tol), (ec, ex, amp)


def _sigma32(dinit, delta_min, iterations, t):
    lam = delta_min ** (1.0 / (iterations - 1)) if iterations > 1 else 1.0
    fac = np.float32(lam ** t) if t > 0 else np.float32(1.0)
    return np.float32(dinit) * fac


def _expected(sysg, o, g, dinit, delta_min, iterations, t):
    """Oracle reconstruction of T_delta T g on the GPU's own decisions."""
    cg, _ = sysg.forward(_gpu(g))
    cg = cg.cpu().numpy()
    l2 = np.array([sb[4] for sb in sysg.subbands], dtype=np.float32)
    out = []
    for b in range(g.shape[0]):
        assert rel(cg[b], T.forward(g[b], o.filters)) < 1e-5
        sig = _sigma32(dinit[b], delta_min, iterations, t)
        ct = cg[b].astype(np.float64)
        for i in range(1, sysg.R):
            ct[i] = np.where(np.abs(cg[b, i]) >= np.float32(sig * l2[i]), ct[i], 0.0)
        out.append(T.inverse(ct, o.filters, o.dual_weight))
    return np.stack(out)


def _check_step(s0, s1, o0, o1, f, prev, new, dinit, dmin, its, t):
    f32 = f.astype(np.float32)
    if t == 0:
        g0 = g1 = f32
    else:
        g0 = f32 - prev[1].astype(np.float32)
        g1 = f32 - prev[0].astype(np.float32)
    e0 = rel(new[0], _expected(s0, o0, g0, dinit, dmin, its, t))
    e1 = rel(new[1], _expected(s1, o1, g1, dinit, dmin, its, t))
    assert e0 < 1e-5 and e1 < 1e-5, (t, e0, e1)
    return max(e0, e1)


@pytest.mark.parametrize("dims,J,levels,Bn", [((64, 64), 3, [1, 1, 2], 2),
                                              ((48, 96), 2, [0, 1], 1)])
def test_decompose_iterations_exact_decisions(dims, J, levels, Bn):
    print(f"case: decompose {dims} J={J} B={Bn}", flush=True)
    pairs = [syn.points_and_curves(*dims, 60 + b) for b in range(Bn)]
    f = np.stack([c + p for c, p in pairs])
    dinit = np.array([2.0, 3.0][:Bn], dtype=np.float32)
    its, dmin = 4, 0.05
    s0 = B.System(dims, J, levels)
    s1 = B.System(dims, J, wavelet=True)
    o0, o1 = S.build_2d(dims, J, levels), D.build_wavelet_2d(dims, J)
    fg, dg = _gpu(f), _gpu(dinit)
    f0 = torch.full_like(fg, 5.0)           # not read at t_begin = 0
    f1 = torch.full_like(fg, -5.0)
    prev = None
    for t in range(its):
        s0.decompose(s1, fg, dg, dmin, its, t_begin=t, t_end=t + 1, f0=f0, f1=f1)
        torch.cuda.synchronize()
        cur = (f0.cpu().numpy(), f1.cpu().numpy())
        err = _check_step(s0, s1, o0, o1, f, prev, cur, dinit, dmin, its, t)
        print(f"iteration {t}: relL2 vs oracle on GPU decisions {err:.2e}", flush=True)
        prev = cur
    a0, a1 = s0.decompose(s1, fg, dg, dmin, its)
    torch.cuda.synchronize()
    assert np.array_equal(a0.cpu().numpy(), prev[0]) and np.array_equal(a1.cpu().numpy(), prev[1])
    g0, g1 = torch.zeros_like(fg), torch.zeros_like(fg)
    for rep in range(3):
        g0.fill_(7.0)
        g1.fill_(7.0)
        s0.decompose(s1, fg, dg, dmin, its, f0=g0, f1=g1, use_graph=True)
        torch.cuda.synchronize()
        assert np.array_equal(g0.cpu().numpy(), prev[0]), rep
        assert np.array_equal(g1.cpu().numpy(), prev[1]), rep
        s1.forward(fg)                             # eager work between replays
        torch.cuda.synchronize()
    h0, h1 = torch.zeros_like(fg), torch.zeros_like(fg)
    s0.decompose(s1, fg, dg, dmin, its, t_end=2, f0=h0, f1=h1, use_graph=True)
    s0.decompose(s1, fg, dg, dmin, its, t_begin=2, f0=h0, f1=h1, use_graph=True)
    torch.cuda.synchronize()
    assert np.array_equal(h0.cpu().numpy(), prev[0]) and np.array_equal(h1.cpu().numpy(), prev[1])


def test_decompose_full_run_matches_oracle():
    print("case: decompose 64x64 30 iterations vs oracle run", flush=True)
    dims, J, levels = (64, 64), 3, [1, 1, 2]
    c, p = syn.points_and_curves(64, 64, 7)
    f = (c + p)[None]
    s0, s1 = B.System(dims, J, levels), B.System(dims, J, wavelet=True)
    o0, o1 = S.build_2d(dims, J, levels), D.build_wavelet_2d(dims, J)
    a0, a1 = s0.decompose(s1, _gpu(f), _gpu(np.array([2.0])), 0.05, 30, use_graph=True)
    torch.cuda.synchronize()
    r0, r1 = D.decompose(f[0], o0, o1, 2.0, 0.05, 30)
    e0, e1 = rel(a0.cpu().numpy()[0], r0), rel(a1.cpu().numpy()[0], r1)
    print(f"relL2 vs oracle run: f0 {e0:.2e}, f1 {e1:.2e}", flush=True)
    assert e0 < 1e-4 and e1 < 1e-4


def test_decompose_512_points_and_curves():
    # SL2D_2-type system (4 scales, shear levels [1, 1, 2, 2], R = 49) with the
    # 4-scale wavelet bank, 100 iterations on a 512^2 points-and-curves image;
    # the last iteration on exact decisions, the separation by Q
    print("case: decompose 512x512 R=49 + wavelets, 100 iterations", flush=True)
    dims, J, levels = (512, 512), 4, [1, 1, 2, 2]
    c, p = syn.points_and_curves(512, 512, 900300)
    f = (c + p)[None]
    dinit = np.array([2.0], dtype=np.float32)
    its, dmin = 100, 0.05
    s0, s1 = B.System(dims, J, levels), B.System(dims, J, wavelet=True)
    fg, dg = _gpu(f), _gpu(dinit)
    f0, f1 = s0.decompose(s1, fg, dg, dmin, its, t_end=its - 1, use_graph=True)
    torch.cuda.synchronize()
    prev = (f0.cpu().numpy(), f1.cpu().numpy())
    s0.decompose(s1, fg, dg, dmin, its, t_begin=its - 1, f0=f0, f1=f1)
    torch.cuda.synchronize()
    cur = (f0.cpu().numpy(), f1.cpu().numpy())
    o0, o1 = S.build_2d(dims, J, levels), D.build_wavelet_2d(dims, J)
    err = _check_step(s0, s1, o0, o1, f, prev, cur, dinit, dmin, its, its - 1)
    qc, qp = M.q_opt(c, cur[0][0])[0], M.q_opt(p, cur[1][0])[0]
    print(f"last iteration relL2 {err:.2e}; Q_opt curves {qc:.4f} (unseparated "
          f"{M.q_opt(c, f[0])[0]:.4f}), points {qp:.4f}", flush=True)
    assert qc < 0.25 and qp < 0.5


def test_decompose_error_paths():
    print("case: decompose error paths", flush=True)
    s0 = B.System((64, 64), 2, [1, 1])
    s1 = B.System((64, 64), 2, wavelet=True)
    s2 = B.System((64, 128), 2, wavelet=True)
    f = torch.zeros((1, 64, 64), device=DEV)
    d = torch.ones(1, device=DEV)
    with pytest.raises(B.ShearletError):
        B.check(B.lib().sl_decompose_workspace_size(s0._h, s2._h, 1, ctypes.byref(ctypes.c_size_t())))
    ws = torch.empty(s0.decompose_workspace_bytes(s1, 1), dtype=torch.uint8, device=DEV)
    f0 = torch.zeros_like(f)
    with pytest.raises(B.ShearletError):      # f0 and f1 alias
        B.check(B.lib().sl_decompose(s0._h, s1._h, B._ptr(f), 1, B._ptr(d), 0.1, 5, 0, 5,
                                     B._ptr(f0), B._ptr(f0), 0, B._ptr(ws), ws.numel(), None))
    with pytest.raises(B.ShearletError):      # different dims
        B.check(B.lib().sl_decompose(s0._h, s2._h, B._ptr(f), 1, B._ptr(d), 0.1, 5, 0, 5,
                                     B._ptr(f0), B._ptr(torch.zeros_like(f)), 0, B._ptr(ws),
                                     ws.numel(), None))
    with pytest.raises(B.ShearletError):
        s0.decompose(s1, f, d, 0.1, 5, t_begin=4, t_end=6)
    with pytest.raises(B.ShearletError):
        s0.decompose(s1, f, d, 0.1, 5, workspace=torch.empty(64, dtype=torch.uint8, device=DEV))
