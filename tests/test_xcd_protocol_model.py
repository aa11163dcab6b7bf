"""Host-thread model of the arrival-counter protocol that the XCD-cooperative
passes use to exchange a pair plane through one XCD's L2 (the kernels in
csrc/xcd2d.hip): every value a workgroup reads is the one the current phase
wrote, under randomised interleavings, and a wait that cannot complete gives
up, flags the error and lets every workgroup return.  Runs on the CPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "xcd_protocol_model.cpp")


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("xcd") / "xcd_protocol_model")
    subprocess.run([gxx, "-O2", "-std=c++17", "-pthread", SRC, "-o", exe], check=True)
    return exe


def run(exe, G, images, pairs, seed, dead=-1, spin=1 << 30):
    r = subprocess.run([exe, str(G), str(images), str(pairs), str(seed), str(dead), str(spin)],
                       capture_output=True, text=True, timeout=120)
    return r.returncode, r.stdout.strip()


@pytest.mark.parametrize("G,images,pairs,seed", [(8, 3, 5, 1), (32, 2, 4, 2), (13, 2, 3, 3)])
def test_every_read_sees_its_phase(model, G, images, pairs, seed):
    rc, out = run(model, G, images, pairs, seed)
    assert rc == 0, out
    n = G * 4
    # per image: one column read of the plane, then one row read per pair
    assert out == f"ok {images * (1 + pairs) * n * n}", out


def test_missing_arrival_gives_up_and_drains(model):
    # one workgroup never arrives after writing its rows: the others' bounded
    # waits give up, set the flag and return (the process exits, nothing hangs)
    rc, out = run(model, 8, 2, 3, 4, dead=5, spin=20000)
    assert rc == 0 and out == "gave-up", out


def test_protocol_without_the_b_wait_is_caught(model, tmp_path):
    # the model is sensitive: dropping the wait on B before the column writes
    # of a pair (writers may then overwrite rows still being read) must make
    # some read see another phase's value for at least one seed
    src = open(SRC).read()
    broken = src.replace(
        "    for (int p = 0; p < pairs; ++p) {\n"
        "      if (!wait_for(s, s.B, (unsigned)G * nB, spin)) return;\n",
        "    for (int p = 0; p < pairs; ++p) {\n", 1)
    assert broken != src
    path = tmp_path / "broken.cpp"
    path.write_text(broken)
    exe = str(tmp_path / "broken")
    subprocess.run([shutil.which("g++"), "-O2", "-std=c++17", "-pthread", str(path), "-o", exe],
                   check=True)
    caught = any(run(exe, 8, 2, 6, seed)[0] == 1 for seed in range(1, 13))
    assert caught
