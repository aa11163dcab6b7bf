"""Uneven batches: several image sizes in one schedule, eager and replayed
from a HIP graph, against the FP64 oracle (FP16 coefficient storage,
relative L2 <= 2e-3 per image) and the autotuner's cache."""
import os

import numpy as np
import pytest

from oracle import system as S
from oracle import transform as T
from paper_1402_5670_amd import synthetic as syn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1402_5670_amd import binding as B  # noqa: E402

DEV = torch.device("cuda:0")
SIZES = [(64, 3), (96, 2), (128, 2), (256, 1)]
J, LEVELS = 3, [1, 1, 2]


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def _setup(dtype="f16"):
    systems, xs, coeffs, scales, outs, host = [], [], [], [], [], []
    seed = 4001
    for n, count in SIZES:
        s = B.System((n, n), J, LEVELS, dtype=dtype)
        imgs = np.stack([syn.noisy_cartoon2d(n, n, seed + k, 0.1)[1] for k in range(count)])
        seed += count
        host.append(imgs)
        systems.append(s)
        xs.append(torch.from_numpy(imgs.astype(np.float32)).to(DEV))
        c, sc = s.alloc_coeffs(count, DEV)
        coeffs.append(c)
        scales.append(sc)
        outs.append(torch.empty((count, n, n), device=DEV))
    m = B.Multi(systems, [c for _, c in SIZES])
    ws = torch.empty(m.workspace_bytes(), dtype=torch.uint8, device=DEV)
    return m, systems, host, xs, coeffs, scales, outs, ws


def _check(systems, host, coeffs, scales, outs, tol):
    for s, imgs, c, sc, o in zip(systems, host, coeffs, scales, outs):
        orc = S.build_2d(s.dims, J, LEVELS)
        cd = c.float().cpu().numpy().astype(np.float64)
        if c.dtype != torch.float32:
            cd = cd * sc.cpu().numpy()[:, :, None, None]
        for k in range(imgs.shape[0]):
            assert rel(cd[k], T.forward(imgs[k], orc.filters)) < tol
            assert rel(o[k].cpu().numpy(), imgs[k]) < tol


def test_uneven_eager_and_graph():
    print("case: uneven sizes 64x3 96x2 128x2 256x1, f16", flush=True)
    m, systems, host, xs, coeffs, scales, outs, ws = _setup()
    m.run(3, xs, coeffs, scales, outs=outs, workspace=ws)
    torch.cuda.synchronize()
    _check(systems, host, coeffs, scales, outs, 2e-3)
    ref_c = [c.clone() for c in coeffs]
    ref_o = [o.clone() for o in outs]
    m.graph_build(3, xs, coeffs, scales, outs=outs, workspace=ws)
    for rep in range(3):
        for c in coeffs:
            c.zero_()
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        m.graph_launch()
        torch.cuda.synchronize()
        for a, b in zip(coeffs, ref_c):
            assert torch.equal(a, b), rep
        for a, b in zip(outs, ref_o):
            assert torch.equal(a, b), rep
        # eager work between replays
        m.run(1, xs, coeffs, scales, workspace=ws)
        torch.cuda.synchronize()


def test_uneven_graph_build_with_timing_on():
    # building the multi-batch graph while per-pass timing is on records no
    # timing events into the graph: after replays the timing queries return the
    # eager launches only, and the replayed results are unchanged
    print("case: uneven graph build with pass timing enabled", flush=True)
    m, systems, host, xs, coeffs, scales, outs, ws = _setup()
    B.timing_reset()
    B.timing_enable(True)
    try:
        m.graph_build(3, xs, coeffs, scales, outs=outs, workspace=ws)
        for _ in range(2):
            m.graph_launch()
        torch.cuda.synchronize()
        assert B.timing_report() == {}
        m.run(1, xs, coeffs, scales, workspace=ws)
        torch.cuda.synchronize()
        rep = B.timing_report()
        assert rep and all(n > 0 and ms >= 0 for ms, n in rep.values())
    finally:
        B.timing_enable(False)
        B.timing_reset()
    m.graph_launch()
    torch.cuda.synchronize()
    _check(systems, host, coeffs, scales, outs, 2e-3)


def test_uneven_autotune(tmp_path):
    print("case: uneven autotune", flush=True)
    m, systems, host, xs, coeffs, scales, outs, ws = _setup()
    cache = str(tmp_path / "tune.txt")
    m.autotune(xs, coeffs, scales, outs, ws, cache_path=cache)
    assert os.path.exists(cache)
    lines = [ln.split() for ln in open(cache).read().split("\n") if ln.strip()]
    sched = [ln for ln in lines if ln[0].startswith("schedule;")]
    lines = [ln for ln in lines if not ln[0].startswith("schedule;")]
    assert len(lines) == len(SIZES) and len(sched) == 1
    # key, chunk bytes, images per inverse block (1 or 2), pair-loop split (0 or 1),
    # line plan (1 or 2)
    for ln in lines:
        assert len(ln) == 5 and int(ln[1]) >= 1 << 20
        assert int(ln[2]) in (1, 2) and int(ln[3]) in (0, 1) and int(ln[4]) in (1, 2)
    # the schedule across classes: 0 multi-class row launches, 1 per class
    assert int(sched[0][3]) in (0, 1)
    assert m.multi_class_rows() == (int(sched[0][3]) == 0)
    m.run(3, xs, coeffs, scales, outs=outs, workspace=ws)
    torch.cuda.synchronize()
    _check(systems, host, coeffs, scales, outs, 2e-3)
    # a second autotune reads the cache
    m.autotune(xs, coeffs, scales, outs, ws, cache_path=cache)


def test_c4_uneven_64_images():
    # 64 images, sizes drawn uniformly from {256, 384, 512, 1024}^2 (seed 4000), 3 scales
    # [1, 1, 2] (R = 33), FP16 storage, autotuned and replayed from one graph; every
    # image's coefficients and reconstruction against the FP64 oracle
    print("case: C4 uneven batch, 64 images", flush=True)
    sizes = syn.uneven_sizes(64, 4000)
    classes = sorted(set(sizes))
    systems, xs, coeffs, scales, outs, host, seeds = [], [], [], [], [], [], []
    for n in classes:
        idx = [k for k, s in enumerate(sizes) if s == n]
        imgs = np.stack([syn.noisy_cartoon2d(n, n, 4001 + k, 0.1)[1] for k in idx])
        s = B.System((n, n), J, LEVELS, dtype="f16")
        systems.append(s)
        host.append(imgs)
        xs.append(torch.from_numpy(imgs.astype(np.float32)).to(DEV))
        c, sc = s.alloc_coeffs(len(idx), DEV)
        coeffs.append(c)
        scales.append(sc)
        outs.append(torch.empty((len(idx), n, n), device=DEV))
    m = B.Multi(systems, [h.shape[0] for h in host])
    ws = torch.empty(m.workspace_bytes(), dtype=torch.uint8, device=DEV)
    m.autotune(xs, coeffs, scales, outs, ws)
    m.graph_build(3, xs, coeffs, scales, outs=outs, workspace=ws)
    m.graph_launch()
    torch.cuda.synchronize()
    # every image: coefficients (FP16 storage) and reconstruction against the
    # FP64 oracle, reported per image
    worst = 0.0
    for s, imgs, c, sc, o in zip(systems, host, coeffs, scales, outs):
        orc = S.build_2d(s.dims, J, LEVELS)
        og = o.cpu().numpy()
        errs = []
        for k in range(imgs.shape[0]):
            cd = c[k].float().cpu().numpy().astype(np.float64) * sc[k].cpu().numpy()[:, None, None]
            ec = rel(cd, T.forward(imgs[k], orc.filters))
            er = rel(og[k], imgs[k])
            errs.append((ec, er))
            assert ec < 2e-3 and er < 2e-3, (s.dims, k, ec, er)
        line = " ".join(f"{ec:.1e}/{er:.1e}" for ec, er in errs)
        print(f"size {s.dims[0]}: {imgs.shape[0]} images, coefficient/reconstruction relL2: {line}",
              flush=True)
        worst = max(worst, max(max(e) for e in errs))
    print(f"worst relL2 over the 64 images: {worst:.2e}", flush=True)


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_line_plan_1024(dtype):
    # the second line plan of 1024-point lines (one wavefront per row, 512-thread
    # inverse accumulation blocks) against the default plan and the oracle
    # three images: the two-image column blocks of 1024-point lines get an
    # odd tail (a block whose second image does not exist)
    print(f"case: 1024^2 line plans, B=3, J=2, {dtype}", flush=True)
    dims = (1024, 1024)
    s = B.System(dims, 2, [1, 1], dtype=dtype)
    xs = np.stack([syn.noisy_cartoon2d(*dims, 4200 + b, 0.1)[1] for b in range(3)])
    xg = torch.from_numpy(xs.astype(np.float32)).to(DEV)
    sg = torch.tensor([0.1, 0.1, 0.1], dtype=torch.float32, device=DEV)
    K = [3.0, 4.0]
    outs = {}
    for em in (1, 2):
        s.set_line_plan(em)
        assert s.line_plan() == em
        c, sc = s.forward(xg)
        r = s.inverse(c, sc)
        d = s.inverse(c, sc, sigma=sg, K=K)
        torch.cuda.synchronize()
        outs[em] = (c.float().cpu().numpy() * (sc.cpu().numpy()[:, :, None, None]
                                               if dtype != "f32" else 1.0),
                    r.cpu().numpy(), d.cpu().numpy())
    s.set_line_plan(1)
    tol_gpu = 1e-6 if dtype == "f32" else 1e-3
    for k in range(3):
        assert rel(outs[2][k], outs[1][k]) < tol_gpu, k
    tol = 1e-5 if dtype == "f32" else 2e-3
    o = S.build_2d(dims, 2, [1, 1])
    for b in (0, 2):
        for em in (1, 2):
            assert rel(outs[em][0][b], T.forward(xs[b], o.filters)) < tol, (b, em)
    assert rel(outs[2][1], xs) < tol
    assert rel(outs[1][1], xs) < tol


@pytest.mark.parametrize("dtype", ["f16", "f32"])
def test_multi_class_row_schedule(dtype):
    # the multi-class schedule (one coefficient row launch over the row blocks
    # of all classes per step) computes every row with the same plan and line
    # FFT as the per-class launches: with 16-bit storage (the same prefetching
    # row kernels) results equal bit for bit; with float32 storage the
    # per-class launches use the single-group row kernels, which the compiler
    # contracts differently, so they agree to float32 rounding (<= 1e-6).  The
    # graph replays equal the eager multi-class run bit for bit, and the
    # results match the oracle.
    def same(a, b):
        if dtype == "f16":
            return torch.equal(a, b)
        return rel(a.cpu().numpy(), b.cpu().numpy()) <= 1e-6
    print(f"case: multi-class row schedule, {dtype}", flush=True)
    m, systems, host, xs, coeffs, scales, outs, ws = _setup(dtype)
    assert m.multi_class_rows()
    m.run(3, xs, coeffs, scales, outs=outs, workspace=ws)
    torch.cuda.synchronize()
    ref_c = [c.clone() for c in coeffs]
    ref_o = [o.clone() for o in outs]
    m.set_schedule(True)
    assert not m.multi_class_rows()
    m.run(3, xs, coeffs, scales, outs=outs, workspace=ws)
    torch.cuda.synchronize()
    for a, b in zip(coeffs, ref_c):
        assert same(a, b)
    for a, b in zip(outs, ref_o):
        assert same(a, b)
    m.set_schedule(False)
    assert m.multi_class_rows()
    m.graph_build(3, xs, coeffs, scales, outs=outs, workspace=ws)
    for rep in range(2):
        for c in coeffs:
            c.zero_()
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        m.graph_launch()
        torch.cuda.synchronize()
        for a, b in zip(coeffs, ref_c):
            assert torch.equal(a, b), rep
        for a, b in zip(outs, ref_o):
            assert torch.equal(a, b), rep
    _check(systems, host, coeffs, scales, outs, 2e-3 if dtype == "f16" else 1e-5)
