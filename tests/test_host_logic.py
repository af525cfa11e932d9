"""Host-side logic without a GPU: the autotuner's candidate sets and the benchmark's refusal of
more than one GPU."""
import os
import subprocess
import sys

from paper_2202_08612_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_autotune_candidates():
    from paper_2202_08612_amd.autotune import CANDIDATES, cache_key, candidates
    # the contravariant form that is not the size rule's default is the one tried
    assert candidates(I.Dims(12, 60, 30, 250, 600), 1)["contra_form"] == [0, 2]   # default per sub-cube
    assert candidates(I.Dims(4, 32, 6, 47, 19), 1)["contra_form"] == [0, 1]       # 16 | n_v: default orbit
    assert candidates(I.Dims(8, 136, 13, 217, 690), 1)["contra_form"] == [0, 1]   # n_v > 64: default orbit
    # vector groups only below the vector count (0 = library default stays)
    assert candidates(I.Dims(4, 12, 6, 20, 60), 1)["vec_group"] == [0]
    assert candidates(I.Dims(4, 12, 6, 20, 60), 8)["vec_group"] == [0, 1, 2, 4]
    c = candidates(I.Dims(4, 12, 6, 20, 60), 4)
    assert set(c) == set(CANDIDATES) and all(v[0] == 0 for v in c.values())
    k1 = cache_key(I.Dims(4, 12, 6, 20, 60), 4, "fp64", "gfx950")
    assert k1 != cache_key(I.Dims(4, 12, 6, 20, 60), 4, "bf16x6", "gfx950")
    assert k1 != cache_key(I.Dims(4, 12, 6, 20, 61), 4, "fp64", "gfx950")


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
