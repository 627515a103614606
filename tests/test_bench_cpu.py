"""Host-side checks of bench.py that need no GPU."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(HERE, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_work_model():
    """The per-launch work figures the roofline divides by: about 25 VALU
    operations per evaluated pair for the blends, a tile evaluating 256 x its
    longest walk (so `walked` = sum over tiles of the longest walk), bytes for
    the HBM-bound kernels, and the rasterizer's algorithmic bytes."""
    sys.path.insert(0, HERE)
    import bench
    st = dict(n=1000, pixels=64 * 64, walked=10, evals=5000, sh_floats=48, K=20000, contribs=8 * 16 * 1000,
              table_bytes=4096, table_entries=1024)
    bound, amount, unit = bench.algorithmic_work("blend_bwd", st)
    assert bound == "alu" and amount == 256 * 10 * 25
    bound, amount, unit = bench.algorithmic_work("blend_fwd", st)
    assert bound == "alu" and amount == 256 * 10 * 25
    bound, amount, unit = bench.algorithmic_work("preprocess_fwd", st)
    assert bound == "hbm" and amount == 1000 * (12 + 16 + 12 + 4 + 4 * 48 + 12 + 16 + 48 + 4 + 8 + 4)
    # rasterizer: per Gaussian 304 + 8 S bytes, 52 per pair, 40 per pixel
    assert bench.raster_bytes(1000, 20000, 4096, 48) == 1000 * (304 + 8 * 48) + 20000 * 52 + 4096 * 40
