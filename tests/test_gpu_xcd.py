"""The XCD-cooperative 512 x 512 passes (each XCD's workgroups exchange the
subband-pair planes through its L2) against the line passes and the FP64
oracle, through the C ABI; and the bounded waits: a wait forced to give up
makes the kernel drain and the next call report SL_EHIP.

Tolerances: the two GPU paths compute the same float32 products and FFTs
(in another grouping of the column FFTs' threads), relative L2 <= 1e-6
between them; against the oracle 1e-5 (coefficients, reconstruction) and,
for the hard threshold, the exact-mask check of the other 2D tests."""
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
J, LEVELS, K = 4, [1, 1, 2, 2], [3.0, 3.0, 3.0, 4.0]


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def _batch(n, seed0):
    sig = np.array([(20.0, 30.0, 40.0)[b % 3] / 255.0 for b in range(n)], dtype=np.float32)
    xs = np.stack([syn.noisy_cartoon2d(512, 512, seed0 + b, float(sig[b]))[1] for b in range(n)])
    return xs, sig


@pytest.fixture(scope="module")
def system():
    s = B.System((512, 512), J, LEVELS)
    s.set_xcd(True)
    if not s.xcd_active(8):
        pytest.skip("the device is not 8 XCDs of 32 compute units")
    return s


@pytest.fixture(scope="module")
def oracle_system():
    return S.build_2d((512, 512), J, LEVELS)


@pytest.mark.parametrize("n", [8, 11])
def test_xcd_forward_inverse_against_line_passes_and_oracle(system, oracle_system, n):
    # 11 images: XCDs 0..2 transform two images, the others one
    print(f"case: xcd 512^2 B={n} R=49", flush=True)
    xs, sig = _batch(n, 7100 + n)
    xg = torch.from_numpy(xs.astype(np.float32)).to(DEV)
    sg = torch.from_numpy(sig).to(DEV)
    assert system.xcd_active(n)
    c1, _ = system.forward(xg)
    r1 = system.inverse(c1)
    d1 = system.inverse(c1, sigma=sg, K=K)
    torch.cuda.synchronize()
    system.set_xcd(False)
    try:
        assert not system.xcd_active(n)
        c2, _ = system.forward(xg)
        r2 = system.inverse(c2)
        d2 = system.inverse(c1, sigma=sg, K=K)
        torch.cuda.synchronize()
    finally:
        system.set_xcd(True)
    cn1, cn2 = c1.cpu().numpy(), c2.cpu().numpy()
    assert rel(cn1, cn2) < 1e-6
    assert rel(r1.cpu().numpy(), r2.cpu().numpy()) < 1e-6
    assert rel(d1.cpu().numpy(), d2.cpu().numpy()) < 1e-6
    assert rel(r1.cpu().numpy(), xs) < 1e-5
    o = oracle_system
    l2 = np.array([sb[4] for sb in system.subbands], dtype=np.float32)
    js = [sb[1] for sb in system.subbands]
    dn1 = d1.cpu().numpy()
    for b in (0, n - 1):
        assert rel(cn1[b], T.forward(xs[b], o.filters)) < 1e-5, b
        # hard threshold: the oracle decides on the GPU's float32 coefficients
        ct = cn1[b].astype(np.float64)
        for i in range(1, system.R):
            delta = np.float32(np.float32(K[js[i]]) * sig[b]) * l2[i]
            ct[i] = np.where(np.abs(cn1[b, i]) >= delta, ct[i], 0.0)
        assert rel(dn1[b], T.inverse(ct, o.filters, o.dual_weight)) < 1e-5, b


def test_xcd_wait_gives_up_and_reports(system):
    # a spin limit of one poll makes the first waits give up: every workgroup
    # leaves the kernel, the stream completes, and the next call on the system
    # returns SL_EHIP; with the default limit the passes are correct again
    print("case: xcd bounded wait forced to give up (spin limit 1)", flush=True)
    xs, sig = _batch(8, 7300)
    xg = torch.from_numpy(xs.astype(np.float32)).to(DEV)
    c, _ = system.alloc_coeffs(8, DEV)
    system.set_xcd(True, spin_limit=1)
    try:
        system.forward(xg, c)
        torch.cuda.synchronize()
    finally:
        system.set_xcd(True, spin_limit=0)
    with pytest.raises(B.ShearletError) as e:
        system.forward(xg, c)
    assert e.value.code == -5
    assert b"gave up" in B.lib().sl_last_error()
    # the flag is cleared once reported: the passes run normally again
    system.forward(xg, c)
    r = system.inverse(c)
    torch.cuda.synchronize()
    assert rel(r.cpu().numpy(), xs) < 1e-5
