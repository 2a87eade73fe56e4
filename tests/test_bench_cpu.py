"""The benchmark script's host-side contract, checked without a GPU.

* more than one GPU is refused with a message and exit status 2 (single-GPU
  build), and so is a run where no GPU is visible: no CPU fallback;
* the five-pass byte model B(n) that fixes `effective_GBps` is the sum of its
  terms (S read, Phi written, 12 complex n^2 (n+1) of workspace traffic, the
  (n+1)^3 spectrum octant read once), written out here per pass;
* the source hash that ties the committed counters to a build covers the
  kernel sources and the build script, and changes when one of them does.
"""
import json
import os
import shutil
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=300, env=env, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "single-GPU" in line["error"]


@pytest.mark.skipif(shutil.which("rocm-smi") is not None and os.path.exists("/dev/kfd"), reason="a GPU may be visible")
def test_no_visible_gpu_is_an_error_not_a_fallback():
    r = _run(["--steps", "1", "--warmup", "0"], {"HIP_VISIBLE_DEVICES": "-1"})
    assert r.returncode == 2
    assert json.loads(r.stdout.strip().splitlines()[-1]) == {"error": "no GPU visible"}


@pytest.mark.parametrize("n,real", [(16, 4), (128, 4), (128, 8), (512, 4)])
def test_five_pass_byte_model(n, real):
    c = 2 * real
    half = c * n * n * (n + 1)  # complex values of n z planes x n y rows x (n+1) kx: the stored half
    passes = {
        "x_fwd": real * n**3 + half,             # read S, write the stored half
        "y_fwd": half + 2 * half,                # read the stored half, write all 2n ky rows
        "z_conv": 2 * half + 2 * half + real * (n + 1) ** 3,  # read and write the 2n rows, spectrum octant once
        "y_inv": 2 * half + half,                # read all rows, keep the first n
        "x_inv": half + real * n**3,             # read the stored half, write Phi
    }
    assert bench.algorithmic_bytes(n, real) == sum(passes.values())


def test_n128_fp32_byte_model_value():
    # 2*4*128^3 + 12*8*128^2*129 + 4*129^3
    assert bench.algorithmic_bytes(128, 4) == 16777216 + 202899456 + 8586756


def test_source_hash_tracks_the_kernel_sources(tmp_path, monkeypatch):
    h0 = bench.source_hash()
    assert len(h0) == 16 and int(h0, 16) >= 0
    # a copy of the tree's sources with one byte changed hashes differently
    src = os.path.join(ROOT, "paper_1106_0557_amd")
    dst = tmp_path / "paper_1106_0557_amd"
    shutil.copytree(os.path.join(src, "csrc"), dst / "csrc")
    shutil.copy(os.path.join(src, "build.py"), dst / "build.py")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.source_hash() == h0
    p = dst / "csrc" / "internal.h"
    p.write_text(p.read_text() + "\n")
    assert bench.source_hash() != h0
