"""The no-allocation fused denoiser (sl_denoise_fused_noalloc, workspace in
the library's static device array) against sl_denoise_fused with a caller
workspace, through the C ABI: two calls in a row, the second on a smaller
input (the array then holds the first call's data), and the size limit."""
import numpy as np
import pytest

from paper_1402_5670_amd import synthetic as syn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1402_5670_amd import binding as B  # noqa: E402

DEV = torch.device("cuda:0")
SCRATCH = 128 << 20


def _case(dims, J, levels, K, seeds, sigmas):
    sysg = B.System(dims, J, levels)
    xs = np.stack([syn.noisy_cartoon2d(*dims, s, sg)[1] for s, sg in zip(seeds, sigmas)])
    x = torch.from_numpy(xs.astype(np.float32)).to(DEV)
    sg = torch.tensor(sigmas, dtype=torch.float32, device=DEV)
    return sysg, x, sg


def _rel(a, b):
    a = a.double().cpu()
    b = b.double().cpu()
    return float((a - b).norm() / b.norm())


def test_noalloc_matches_workspace_call_twice():
    # first call: 2 images of 256^2, R = 33 (needs well under the array's size)
    print("case: noalloc fused denoise 2x256^2 J=3 then 1x128x96 J=2", flush=True)
    s1, x1, g1 = _case((256, 256), 3, [1, 1, 2], [3.0, 3.0, 4.0], [700, 701], [0.05, 0.1])
    assert s1.workspace_bytes(2) <= SCRATCH
    ref1 = s1.denoise_fused(x1, g1, [3.0, 3.0, 4.0])
    got1 = s1.denoise_fused_noalloc(x1, g1, [3.0, 3.0, 4.0])
    torch.cuda.synchronize()
    assert _rel(got1, ref1) <= 1e-6
    # second call: a smaller input on another system; the array still holds the
    # first call's planes, which nothing may read
    s2, x2, g2 = _case((128, 96), 2, [1, 1], [3.0, 4.0], [702], [0.08])
    ref2 = s2.denoise_fused(x2, g2, [3.0, 4.0])
    got2 = s2.denoise_fused_noalloc(x2, g2, [3.0, 4.0])
    torch.cuda.synchronize()
    assert _rel(got2, ref2) <= 1e-6
    # and the first system again, after the smaller call
    got1b = s1.denoise_fused_noalloc(x1, g1, [3.0, 3.0, 4.0])
    torch.cuda.synchronize()
    assert _rel(got1b, ref1) <= 1e-6


def test_noalloc_one_512_image_fits():
    print("case: noalloc fused denoise 1x512^2 J=4 R=49", flush=True)
    s, x, g = _case((512, 512), 4, [1, 1, 2, 2], [3.0, 3.0, 3.0, 4.0], [703], [0.1])
    assert s.workspace_bytes(1) <= SCRATCH
    ref = s.denoise_fused(x, g, [3.0, 3.0, 3.0, 4.0])
    got = s.denoise_fused_noalloc(x, g, [3.0, 3.0, 3.0, 4.0])
    torch.cuda.synchronize()
    assert _rel(got, ref) <= 1e-6


def test_noalloc_rejects_inputs_beyond_the_array():
    # 4 images of 512^2 need more than 128 MiB: SL_ENOMEM before any GPU work,
    # the output untouched
    print("case: noalloc size limit 4x512^2", flush=True)
    s = B.System((512, 512), 4, [1, 1, 2, 2])
    assert s.workspace_bytes(4) > SCRATCH
    x = torch.zeros((4, 512, 512), dtype=torch.float32, device=DEV)
    g = torch.full((4,), 0.1, dtype=torch.float32, device=DEV)
    out = torch.full_like(x, 7.0)
    with pytest.raises(B.ShearletError) as e:
        s.denoise_fused_noalloc(x, g, [3.0, 3.0, 3.0, 4.0], out=out)
    assert e.value.code == -2
    assert b"static array" in B.lib().sl_last_error()
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
