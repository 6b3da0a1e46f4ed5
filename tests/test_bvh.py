"""Host BVH builder (CPU only): structure and closest-hit agreement with a
brute-force search, through a small C++ checker compiled against the
builder's source."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2309_15676_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2309_15676_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path_factory.mktemp("bvh") / "bvh_check")
    subprocess.run([gxx, "-std=c++17", "-O2", "-I", CSRC, os.path.join(HERE, "bvh_check.cpp"),
                    os.path.join(CSRC, "bvh.cpp"), "-o", exe], check=True)
    return exe


def _run(checker, tmp_path, v, t):
    f = tmp_path / "mesh.bin"
    v = np.ascontiguousarray(np.asarray(v, np.float32).reshape(-1, 3))
    t = np.ascontiguousarray(np.asarray(t, np.int32).reshape(-1, 3))
    with open(f, "wb") as fh:
        fh.write(np.array([v.shape[0], t.shape[0]], np.int32).tobytes())
        fh.write(v.tobytes())
        fh.write(t.tobytes())
    r = subprocess.run([checker, str(f)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout.split()


@pytest.mark.parametrize("mesh", ["one", "two", "fan", "ico8", "height24", "ico40", "soup"])
def test_bvh_structure_and_closest_hit(checker, tmp_path, mesh):
    if mesh == "one":
        v, t = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]]), np.array([[0, 1, 2]])
    elif mesh == "two":
        v, t = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]]), np.array([[0, 1, 2], [1, 3, 2]])
    elif mesh == "fan":
        v = np.array([[0, 0, 0], [-1, 0, -1], [1, 0, -1], [1, 0, 1], [-1, 0, 1]])
        t = np.array([[0, 2, 1], [0, 3, 2], [0, 4, 3], [0, 1, 4]])
    elif mesh == "ico8":
        v, t = I.icosphere(8, seed=1)
    elif mesh == "height24":
        v, t = I.heightfield(24, seed=2)
    elif mesh == "ico40":
        v, t = I.icosphere(40, seed=3, disp=0.3)
    else:
        # random triangle soup, many overlaps
        g = I.rng(5)
        v = g.uniform(-1, 1, (3000, 3))
        t = np.arange(3000).reshape(-1, 3)
    out = _run(checker, tmp_path, v, t)
    assert out[0] == "ok", out
    depth, nodes, hits = int(out[1]), int(out[2]), int(out[3])
    assert 1 <= depth <= 48 and nodes >= 1
    if mesh not in ("one", "two"):
        assert hits > 100


def test_bvh_flat_mesh_is_not_degenerate(checker, tmp_path):
    # many triangles with identical centroids are still split (by index)
    v = np.tile(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32), (200, 1))
    t = np.arange(600).reshape(-1, 3)
    out = _run(checker, tmp_path, v, t)
    assert out[0] == "ok", out
