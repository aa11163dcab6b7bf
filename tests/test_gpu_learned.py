"""The trained shrinkage network against hard thresholding at equal sigma
(held-out cartoons), and the rasteriser against the host cartoon generator."""
import numpy as np
import pytest

from paper_1402_5670_amd import synthetic as syn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1402_5670_amd import binding as B  # noqa: E402
from paper_1402_5670_amd import train as TR  # noqa: E402

DEV = torch.device("cuda:0")


def test_rasteriser_matches_host_generator():
    # the same shape draws rendered on the GPU (float32 geometry) and on the host
    # (float64): identical except for pixels whose centre lies on a shape edge
    seeds = [11, 12, 13]
    shapes = torch.from_numpy(syn.shape_table(96, 128, seeds)).to(DEV)
    clean = torch.empty((3, 96, 128), device=DEV)
    B.render_cartoons(shapes, 96, 128, None, 0, clean)
    torch.cuda.synchronize()
    for n, s in enumerate(seeds):
        ref = syn.cartoon2d(96, 128, s)
        diff = np.abs(clean[n].cpu().numpy() - ref) > 1e-6
        assert diff.mean() < 2e-3


def test_learned_beats_hard_threshold():
    # What training adds: the network starts as a sigmoid-smoothed hard
    # threshold (init_params), so the trained weights must beat that starting
    # point at every sigma, the starting point must beat the noisy input, and the
    # trained network must beat plain hard thresholding (Section 5.3's operator,
    # the yardstick) on average over sigma.
    print("case: train 128x128 J=3 d=[1,1,2], 2000 images", flush=True)
    K = (3.0, 3.0, 4.0)
    state, hist = TR.train(images=2000, batch=8, size=128, n_scales=3, shear_levels=(1, 1, 2),
                           lr=1e-3, lr_min=5e-5, seed=123, log_every=25, quiet=True, K=K)
    print(hist, flush=True)
    kw = dict(size=128, n_scales=3, shear_levels=(1, 1, 2), K=K, n_images=12, reps=2)
    res = TR.evaluate(state["params"], **kw)
    init = TR.evaluate(TR.init_params(3, seed=0, K=K), **kw)
    print({"trained": res, "init": init}, flush=True)
    assert res["psnr_learned"] > res["psnr_hard"]
    for s in (20, 30, 40):
        assert res[f"psnr_learned_{s}"] > init[f"psnr_learned_{s}"], s
        assert init[f"psnr_learned_{s}"] > init[f"psnr_noisy_{s}"], s
