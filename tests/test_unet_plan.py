"""CPU check of the U-Net training launch plan (csrc/ct_unet_plan.hpp): over batch shapes from 1 x 8 x 8
to 8 x 512 x 512, every weight-, bias-, input- and output-layer gradient launch fits the partial-sum
buffer sized for the maximum batch, and its pixel splits cover the pixels with no empty split. Run as a
separate executable: an arithmetic fault in the plan (a split count divided by zero for a deep level
with fewer than 64 pixels, as the 2 x 24 x 40 batch once produced) fails the test instead of the run."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_training_plan_fits_and_covers(tmp_path):
    exe = str(tmp_path / "unet_plan_check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "paper_1512_04564_amd", "csrc"),
                    os.path.join(ROOT, "tests", "emu", "unet_plan_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert " 0 failed" in r.stdout
