"""GPU parity of inpainting by iterative hard thresholding (Algorithm 3)
through the C ABI.

Every iteration is checked on an exact decision set: the test replays one
iteration t from the GPU's previous estimate, takes the GPU's own float32
coefficients of the iteration's input (sl_forward on the same system) and
its float32 threshold float32(delta_init * float32(lambda^t)) * ||psi_i||_2,
and reconstructs the thresholded coefficients with the FP64 oracle; the GPU
estimate must match that to relative L2 <= 1e-5, and the coefficients must
match the oracle's forward transform to 1e-5.  A full run must equal the
chain of its single iterations bit for bit, eagerly, in segments and
replayed from a HIP graph.  A short full run is also compared with the
oracle's own run (its threshold decisions in FP64).
"""
import ctypes

import numpy as np
import pytest

from oracle import inpaint as I
from oracle import system as S
from oracle import transform as T
from paper_1402_5670_amd import synthetic as syn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1402_5670_amd import binding as B  # noqa: E402

DEV = torch.device("cuda:0")
KINDS = ("random", "squares", "text")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def _gpu(x, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dtype)).to(DEV)


def _cases_2d(dims, Bn, seed):
    clean, masks = [], []
    for b in range(Bn):
        c, m = syn.inpainting_case(dims[0], dims[1], seed + b, KINDS[b % 3])
        clean.append(c)
        masks.append(m)
    return np.stack(clean), np.stack(masks)


def _sigma32(dinit, delta_min, iterations, t):
    lam = delta_min ** (1.0 / (iterations - 1)) if iterations > 1 else 1.0
    fac = np.float32(lam ** t) if t > 0 else np.float32(1.0)
    return np.float32(dinit) * fac


def _check_step(sysg, o, fm, m, f_prev, f_new, dinit, delta_min, iterations, t):
    """Iteration t of the GPU against the oracle on the GPU's decisions."""
    g = np.where(m != 0, fm.astype(np.float32), f_prev.astype(np.float32))
    cg, _ = sysg.forward(_gpu(g))
    cg = cg.cpu().numpy()
    l2 = np.array([sb[4] for sb in sysg.subbands], dtype=np.float32)
    worst = 0.0
    for b in range(g.shape[0]):
        assert rel(cg[b], T.forward(g[b], o.filters)) < 1e-5
        sig = _sigma32(dinit[b], delta_min, iterations, t)
        ct = cg[b].astype(np.float64)
        for i in range(1, sysg.R):
            keep = np.abs(cg[b, i]) >= np.float32(sig * l2[i])
            ct[i] = np.where(keep, ct[i], 0.0)
        ref = T.inverse(ct, o.filters, o.dual_weight)
        err = rel(f_new[b], ref)
        worst = max(worst, err)
        assert err < 1e-5, (t, b, err)
    return worst


@pytest.mark.parametrize("dims,J,levels,Bn,chunk_mb", [
    ((64, 64), 2, [1, 1], 3, None),
    ((64, 64), 2, [1, 1], 3, 1),            # pair planes split over chunks
    ((24, 96), 3, [1, 1, 2], 2, None),      # ragged row tiles
])
def test_inpaint_iterations_exact_decisions(monkeypatch, dims, J, levels, Bn, chunk_mb):
    print(f"case: inpaint {dims} J={J} B={Bn} chunk={chunk_mb}", flush=True)
    if chunk_mb:
        monkeypatch.setenv("SL_CHUNK_MB", str(chunk_mb))
    clean, masks = _cases_2d(dims, Bn, 70)
    fm = clean * masks
    dinit = np.array([4.0, 2.0, 1.0][:Bn], dtype=np.float32)
    its, dmin = 4, 0.01
    sysg = B.System(dims, J, levels)
    o = S.build_2d(dims, J, levels)
    fmg, mg, dg = _gpu(fm), _gpu(masks, np.uint8), _gpu(dinit)
    f = torch.full_like(fmg, 123.0)           # not read at t_begin = 0
    states = []
    for t in range(its):
        prev = f.cpu().numpy() if t else np.zeros(fm.shape, np.float32)
        sysg.inpaint(fmg, mg, dg, dmin, its, t_begin=t, t_end=t + 1, f=f)
        torch.cuda.synchronize()
        cur = f.cpu().numpy()
        err = _check_step(sysg, o, fm, masks, prev, cur, dinit, dmin, its, t)
        print(f"iteration {t}: relL2 vs oracle on GPU decisions {err:.2e}", flush=True)
        states.append(cur)
    # the whole run in one call, eagerly and from a graph, equals the chain
    full = sysg.inpaint(fmg, mg, dg, dmin, its)
    torch.cuda.synchronize()
    assert np.array_equal(full.cpu().numpy(), states[-1])
    fg = torch.zeros_like(fmg)
    for rep in range(3):
        fg.fill_(-1.0)
        sysg.inpaint(fmg, mg, dg, dmin, its, f=fg, use_graph=True)
        torch.cuda.synchronize()
        assert np.array_equal(fg.cpu().numpy(), states[-1]), rep
        sysg.denoise_fused(fmg, dg, [1.0] * J)     # eager work between replays
        torch.cuda.synchronize()
    seg = torch.zeros_like(fmg)
    sysg.inpaint(fmg, mg, dg, dmin, its, t_end=1, f=seg, use_graph=True)
    sysg.inpaint(fmg, mg, dg, dmin, its, t_begin=1, f=seg, use_graph=True)
    torch.cuda.synchronize()
    assert np.array_equal(seg.cpu().numpy(), states[-1])


def test_inpaint_full_run_matches_oracle():
    # 40 iterations at 64 x 64 against the oracle's own run (FP64 decisions)
    print("case: inpaint 64x64 40 iterations vs oracle run", flush=True)
    dims, J, levels = (64, 64), 2, [1, 1]
    clean, masks = _cases_2d(dims, 3, 12)
    fm = clean * masks
    sysg = B.System(dims, J, levels)
    o = S.build_2d(dims, J, levels)
    out = sysg.inpaint(_gpu(fm), _gpu(masks, np.uint8), _gpu(np.full(3, 4.0)), 0.005, 40,
                       use_graph=True)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    for b in range(3):
        ref = I.inpaint(fm[b], masks[b], o, 4.0, 0.005, 40)
        e = rel(out[b], ref)
        dp = abs(T.psnr(clean[b], out[b]) - T.psnr(clean[b], ref))
        print(f"{KINDS[b]}: relL2 vs oracle run {e:.2e}, PSNR difference {dp:.2e} dB", flush=True)
        assert e < 1e-4 and dp < 0.01


def test_inpaint_3d_exact_decisions():
    print("case: inpaint 3D (16, 24, 32) J=2", flush=True)
    dims, J, levels = (16, 24, 32), 2, [1, 1]
    clean = np.stack([syn.cartoon3d(*dims, 31), syn.cartoon3d(*dims, 32)])
    masks = np.stack([syn.random_mask(dims, 31), syn.squares_mask(dims, 32, 0.05)])
    fm = clean * masks
    dinit = np.array([4.0, 3.0], dtype=np.float32)
    its, dmin = 3, 0.05
    sysg = B.System(dims, J, levels)
    o = S.build_3d(dims, J, levels)
    fmg, mg, dg = _gpu(fm), _gpu(masks, np.uint8), _gpu(dinit)
    f = torch.zeros_like(fmg)
    prev = np.zeros(fm.shape, np.float32)
    for t in range(its):
        sysg.inpaint(fmg, mg, dg, dmin, its, t_begin=t, t_end=t + 1, f=f)
        torch.cuda.synchronize()
        cur = f.cpu().numpy()
        err = _check_step(sysg, o, fm, masks, prev, cur, dinit, dmin, its, t)
        print(f"iteration {t}: relL2 {err:.2e}", flush=True)
        prev = cur
    full = sysg.inpaint(fmg, mg, dg, dmin, its, use_graph=True)
    torch.cuda.synchronize()
    assert np.array_equal(full.cpu().numpy(), prev)


def test_inpaint_512_paper_schedule():
    # the paper's setting: 512^2, four scales with shear levels [1, 1, 2, 2]
    # (R = 49), 300 iterations, the three mask types; the last iteration is
    # checked on exact decisions, the result for quality
    print("case: inpaint 512x512 R=49 300 iterations, three masks", flush=True)
    dims, J, levels = (512, 512), 4, [1, 1, 2, 2]
    clean, masks = _cases_2d(dims, 3, 900000)
    fm = clean * masks
    dinit = np.full(3, 4.0, dtype=np.float32)
    its, dmin = 300, 0.005
    sysg = B.System(dims, J, levels)
    fmg, mg, dg = _gpu(fm), _gpu(masks, np.uint8), _gpu(dinit)
    f = sysg.inpaint(fmg, mg, dg, dmin, its, t_end=its - 1, use_graph=True)
    torch.cuda.synchronize()
    prev = f.cpu().numpy()
    sysg.inpaint(fmg, mg, dg, dmin, its, t_begin=its - 1, f=f)
    full = sysg.inpaint(fmg, mg, dg, dmin, its, use_graph=True)
    torch.cuda.synchronize()
    cur = f.cpu().numpy()
    assert np.array_equal(full.cpu().numpy(), cur)
    o = S.build_2d(dims, J, levels)
    err = _check_step(sysg, o, fm, masks, prev, cur, dinit, dmin, its, its - 1)
    print(f"last iteration relL2 vs oracle on GPU decisions {err:.2e}", flush=True)
    for b in range(3):
        p0, p1 = T.psnr(clean[b], fm[b]), T.psnr(clean[b], cur[b])
        known = masks[b] == 1
        rms = np.sqrt(np.mean((cur[b] - clean[b])[known] ** 2))
        print(f"{KINDS[b]}: PSNR occluded {p0:.2f} -> inpainted {p1:.2f} dB, "
              f"known-sample RMS {rms:.4f}", flush=True)
        assert p1 > p0 + 8.0 and rms < 0.01


def test_inpaint_error_paths():
    print("case: inpaint error paths", flush=True)
    sysg = B.System((64, 64), 2, [1, 1])
    fm = torch.zeros((2, 64, 64), device=DEV)
    m = torch.ones((2, 64, 64), dtype=torch.uint8, device=DEV)
    d = torch.ones(2, device=DEV)
    with pytest.raises(B.ShearletError):
        sysg.inpaint(fm, m, d, 0.1, 5, t_begin=2, t_end=6)
    with pytest.raises(B.ShearletError):
        sysg.inpaint(fm, m, d, -0.1, 5)
    with pytest.raises(B.ShearletError):
        sysg.inpaint(fm, m, d, 0.1, 0)
    ws = torch.empty(16, dtype=torch.uint8, device=DEV)
    with pytest.raises(B.ShearletError):
        sysg.inpaint(fm, m, d, 0.1, 5, workspace=ws)
    big = torch.zeros(2 * 64 * 64 + 1, device=DEV)
    wsok = torch.empty(sysg.inpaint_workspace_bytes(2), dtype=torch.uint8, device=DEV)
    with pytest.raises(B.ShearletError):     # f misaligned by one float
        B.check(B.lib().sl_inpaint(sysg._h, B._ptr(fm), B._ptr(m), 2, B._ptr(d), 0.1, 5, 0, 5,
                                   ctypes.c_void_p(big.data_ptr() + 4), 0, B._ptr(wsok), wsok.numel(), None))
    # t_begin == t_end is a no-op
    f = torch.full_like(fm, 7.0)
    sysg.inpaint(fm, m, d, 0.1, 5, t_begin=3, t_end=3, f=f)
    torch.cuda.synchronize()
    assert bool((f == 7.0).all())
