"""Training of the learned shrinkage network on the GPU.

Every step renders a batch of cartoon images and their noisy versions
(sigma ~ U[10, 50]/255), transforms the noisy images, applies the per-scale
CNN gains, reconstructs, and minimises the image-domain squared error to the
clean images.  The gradient flows back through the reconstruction with
sl_inverse_adjoint (the forward transform with the dual filters) and through
the network with sl_cnn_backward; Adam updates the FP32 master weights and
sl_cnn_pack refreshes the bfloat16 operand copies.  All arithmetic runs in
libshearlet's kernels; this module only orchestrates the calls.

    python -m paper_1402_5670_amd.train --images 10000 --out weights.npz

Checkpoints (.npz) hold the weights, the Adam moments, the step and the
configuration; --resume continues a run exactly.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1402_5670_amd import binding as B          # noqa: E402
from paper_1402_5670_amd import synthetic as syn      # noqa: E402

PARAMS = B.CNN_PARAMS


def default_K(J):
    """Per-scale threshold constants: 3 on every scale, 4 on the finest."""
    return [3.0] * (J - 1) + [4.0]


def init_params(J, C=32, seed=0, K=None, alpha=6.0, noise=0.1):
    """Initial weights per scale that start as a smooth hard threshold.

    Channel 0 carries the normalised magnitude x0 = |c| / (sigma ||psi||)
    through the two hidden layers (centre taps 1, biases 0) and the output
    is alpha * (x0 - K_j), so the initial gain sigmoid(alpha (x0 - K_j))
    approximates thresholding at K_j sigma ||psi||.  All other weights are
    He-initialised and scaled by noise, leaving room to learn context."""
    rng = np.random.default_rng(seed)
    K = default_K(J) if K is None else list(K)
    out = np.zeros((J, PARAMS), dtype=np.float32)
    for j in range(J):
        w1 = rng.standard_normal((C, 2, 3, 3)) * np.sqrt(2.0 / 18) * noise
        w2 = rng.standard_normal((C, C, 3, 3)) * np.sqrt(2.0 / (9 * C)) * noise
        w3 = rng.standard_normal((1, C, 3, 3)) * np.sqrt(1.0 / (9 * C)) * noise
        w1[0] = 0.0
        w1[0, 0, 1, 1] = 1.0
        w2[0] = 0.0
        w2[0, 0, 1, 1] = 1.0
        w3[0, 0] = 0.0
        w3[0, 0, 1, 1] = alpha
        blob = np.concatenate([w1.ravel(), np.zeros(C), w2.ravel(), np.zeros(C), w3.ravel(),
                               [-alpha * K[j]]])
        out[j] = blob
    return out


def sigmas_for(seed, idx):
    """sigma ~ U[10, 50] / 255 for training image idx."""
    return np.array([np.random.default_rng([seed + i, 2]).uniform(10.0, 50.0) / 255.0
                     for i in idx], dtype=np.float32)


def train(images=10000, batch=4, size=512, n_scales=4, shear_levels=(1, 1, 2, 2), lr=1e-3,
          lr_min=5e-5, seed=0, init_seed=0, resume=None, out=None, log_every=50, device="cuda:0",
          quiet=False, K=None):
    import torch
    dev = torch.device(device)
    sysg = B.System((size, size), n_scales, shear_levels)
    J = n_scales
    start_step = 0
    if resume:
        ck = np.load(resume)
        params = torch.from_numpy(ck["params"]).to(dev)
        m = torch.from_numpy(ck["m"]).to(dev)
        v = torch.from_numpy(ck["v"]).to(dev)
        start_step = int(ck["step"])
    else:
        params = torch.from_numpy(init_params(J, seed=init_seed, K=K)).to(dev)
        m = torch.zeros_like(params)
        v = torch.zeros_like(params)
    net = B.Shrinkage(sysg, params)
    steps = images // batch
    scratch = torch.zeros(B.SQERR_SCRATCH, dtype=torch.float32, device=dev)
    clean = torch.empty((batch, size, size), dtype=torch.float32, device=dev)
    noisy = torch.empty_like(clean)
    resid = torch.empty_like(clean)
    coeffs, _ = sysg.alloc_coeffs(batch, dev)
    shrunk = torch.empty_like(coeffs)
    recon = torch.empty_like(clean)
    dco = torch.empty_like(coeffs)
    npx = batch * size * size
    hist = []
    t0 = time.perf_counter()
    for step in range(start_step, steps):
        idx = list(range(step * batch, (step + 1) * batch))
        shapes = torch.from_numpy(syn.shape_table(size, size, [seed + i for i in idx])).to(dev)
        sig = torch.from_numpy(sigmas_for(seed, idx)).to(dev)
        B.render_cartoons(shapes, size, size, sig, seed * 1000003 + step, clean, noisy)
        sysg.forward(noisy, coeffs)
        net.apply(coeffs, sig, out=shrunk)
        sysg.inverse(shrunk, out=recon)
        B.sq_error_grad(recon, clean, 2.0 / npx, resid, scratch)
        sysg.inverse_adjoint(resid, coeffs=dco)
        grads = net.backward(coeffs, sig, dco)
        frac = step / max(1, steps - 1)
        lr_t = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * frac))
        B.adam_step(net.params, grads, m, v, lr_t, step + 1)
        net.pack()
        if (step + 1) % log_every == 0 or step + 1 == steps:
            mse = float(scratch[0].item()) / npx
            hist.append((step + 1, mse))
            if not quiet:
                print(json.dumps({"step": step + 1, "images": (step + 1) * batch,
                                  "mse": mse, "psnr_db": -10 * math.log10(max(mse, 1e-30)),
                                  "lr": lr_t, "s": round(time.perf_counter() - t0, 1)}),
                      flush=True)
    torch.cuda.synchronize()
    state = dict(params=net.params.cpu().numpy(), m=m.cpu().numpy(), v=v.cpu().numpy(),
                 step=np.int64(steps), size=size, n_scales=n_scales,
                 shear_levels=np.array(shear_levels), images=images, batch=batch, seed=seed)
    if out:
        np.savez(out, **state)
    return state, hist


def psnr(ref, est):
    """20 log10(sqrt(N) / ||ref - est||) for images in [0, 1] (eq. PSNR, peak 1)."""
    err = np.linalg.norm((np.asarray(ref, np.float64) - np.asarray(est, np.float64)).ravel())
    return 20.0 * np.log10(np.sqrt(np.asarray(ref).size) / err)


def evaluate(params, size=512, n_scales=4, shear_levels=(1, 1, 2, 2), K=(3.0, 3.0, 3.0, 4.0),
             n_images=32, seed0=900000, sigmas255=(20.0, 30.0, 40.0), reps=5, device="cuda:0"):
    """Held-out comparison of learned shrinkage and hard thresholding at equal
    sigma on CPU-rendered cartoons; returns PSNRs per sigma and images/s of
    both paths (forward + shrinkage + inverse, timed with device events)."""
    import torch
    dev = torch.device(device)
    sysg = B.System((size, size), n_scales, shear_levels)
    net = B.Shrinkage(sysg, torch.as_tensor(np.asarray(params, np.float32)).to(dev))
    sig = np.array([sigmas255[b % len(sigmas255)] / 255.0 for b in range(n_images)],
                   dtype=np.float32)
    pairs = [syn.noisy_cartoon2d(size, size, seed0 + b, float(sig[b])) for b in range(n_images)]
    x = torch.from_numpy(np.stack([p[1] for p in pairs]).astype(np.float32)).to(dev)
    sg = torch.from_numpy(sig).to(dev)
    coeffs, scales = sysg.alloc_coeffs(n_images, dev)
    shrunk = torch.empty_like(coeffs)
    out_h = torch.empty_like(x)
    out_l = torch.empty_like(x)

    def hard():
        sysg.denoise(x, sg, K, coeffs=coeffs, scales=scales, out=out_h)

    def learned():
        sysg.forward(x, coeffs)
        net.apply(coeffs, sg, out=shrunk)
        sysg.inverse(shrunk, out=out_l)

    res = {}
    for name, fn in (("hard", hard), ("learned", learned)):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        res[name + "_images_per_s"] = n_images * reps / (a.elapsed_time(b) / 1000.0)
    oh, ol = out_h.cpu().numpy(), out_l.cpu().numpy()
    for s255 in sigmas255:
        sel = [b for b in range(n_images) if abs(sig[b] * 255.0 - s255) < 1e-3]
        res[f"psnr_noisy_{int(s255)}"] = float(np.mean([psnr(pairs[b][0], pairs[b][1]) for b in sel]))
        res[f"psnr_hard_{int(s255)}"] = float(np.mean([psnr(pairs[b][0], oh[b]) for b in sel]))
        res[f"psnr_learned_{int(s255)}"] = float(np.mean([psnr(pairs[b][0], ol[b]) for b in sel]))
    res["psnr_hard"] = float(np.mean([psnr(pairs[b][0], oh[b]) for b in range(n_images)]))
    res["psnr_learned"] = float(np.mean([psnr(pairs[b][0], ol[b]) for b in range(n_images)]))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--images", type=int, default=10000)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--resume", default=None)
    ap.add_argument("--out", default="shrinkage_weights.npz")
    args = ap.parse_args()
    state, _ = train(images=args.images, batch=args.batch, size=args.size, lr=args.lr,
                     seed=args.seed, resume=args.resume, out=args.out)
    if args.size == 512:
        print(json.dumps({"eval": evaluate(state["params"])}), flush=True)


if __name__ == "__main__":
    main()
