"""CPU check of the product's BVH builder (host code of libgrwave) before any kernel uses it."""

import os
import subprocess

import numpy as np
import pytest

from workloads import scenes as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("bvh") / "grwave_bvh_check")
    srcs = [os.path.join(ROOT, "tests", "bvh_check.cpp"),
            os.path.join(ROOT, "paper_2303_15762_amd", "csrc", "bvh_build.cpp")]
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-o", exe] + srcs)
    return exe


def _run(exe, verts, tris, rays):
    lines = [f"{len(verts)} {len(tris)}"]
    lines += [" ".join(f"{v:.9g}" for v in p) for p in verts]
    lines += [" ".join(str(int(i)) for i in t) for t in tris]
    lines.append(str(len(rays)))
    lines += [" ".join(f"{v:.9g}" for v in r) for r in rays]
    r = subprocess.run([exe], input="\n".join(lines), capture_output=True, text=True)
    return r.returncode, r.stdout.strip()


def _rays(n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    o = rng.uniform(lo, hi, (n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return np.concatenate([o, d], 1)


@pytest.mark.parametrize("case", ["terrain", "tiny", "boxes", "degenerate"])
def test_bvh_structure_and_traversal(checker, case):
    if case == "terrain":
        sc = W.terrain_scene(nx=64, ny=32, seed=3, tiles=4)
        verts, tris = sc.verts.astype(np.float32), sc.tris
        rays = _rays(2000, [-0.01, -0.01, -0.01], [0.11, 0.11, 0.02], 1)
    elif case == "tiny":
        wl = W.tiny_grating()
        verts, tris = wl.scene.verts.astype(np.float32), wl.scene.tris
        rays = _rays(500, -1e-3, 1e-3, 2)
    elif case == "boxes":
        sc = W.large_scene(n_inst_x=1, n_inst_y=1, n_boxes=300, seed=4, tile_nx=16, tile_ny=8)
        verts, tris = sc.verts.astype(np.float32), sc.tris
        rays = _rays(2000, [0, 0, -0.01], [0.1, 0.1, 0.04], 3)
    else:
        # many identical triangles (coincident centroids) force the median fallback
        base = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
        verts = np.concatenate([base] * 200)
        tris = np.arange(600).reshape(200, 3)
        rays = _rays(200, -0.5, 1.5, 4)
    rc, out = _run(checker, verts, tris, rays)
    assert rc == 0 and out.startswith("OK"), out
    depth, max_sp, nodes = map(int, out.split()[1:])
    assert max_sp <= 3 * (depth + 1) + 1


# --------------------------------------------------------------------------------------
# Material-boundary lists of composite interactions (host code of libgrwave)
# --------------------------------------------------------------------------------------

@pytest.fixture(scope="module")
def bchecker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("boundary") / "grwave_boundary_check")
    srcs = [os.path.join(ROOT, "tests", "boundary_check.cpp"),
            os.path.join(ROOT, "paper_2303_15762_amd", "csrc", "boundary.cpp")]
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-o", exe] + srcs)
    return exe


@pytest.mark.parametrize("case", ["terrain", "instances", "split"])
@pytest.mark.parametrize("reach", [2e-3, 0.3e-3])
def test_boundary_lists_complete(bchecker, case, reach):
    """Every boundary edge of a hit's material within the reach is in its triangle's list, so
    the nearest found through the list is the nearest of all (brute force over every edge)."""
    if case == "terrain":
        sc = W.terrain_scene()
    elif case == "instances":
        sc = W.large_scene(n_inst_x=2, n_inst_y=1, n_boxes=50, seed=4, tile_nx=64, tile_ny=32)
    else:
        sc = W.split_mirror().scene
    verts, tris, mats = sc.verts.astype(np.float32), sc.tris, sc.tri_mat
    rng = np.random.default_rng(5)
    ts = rng.integers(0, len(tris), 3000)
    bc = rng.dirichlet([1, 1, 1], 3000)
    lines = [f"{len(verts)} {len(tris)} {reach:.9g}"]
    lines += [" ".join(f"{v:.9g}" for v in p) for p in verts]
    lines += [f"{a} {b} {c} {m}" for (a, b, c), m in zip(tris, mats)]
    lines.append(str(len(ts)))
    lines += [f"{t} {u:.17g} {w:.17g}" for t, (_, u, w) in zip(ts, bc)]
    r = subprocess.run([bchecker], input="\n".join(lines), capture_output=True, text=True)
    out = r.stdout.strip()
    assert r.returncode == 0 and out.startswith("OK"), out
    n_edges, found, entries = map(int, out.split()[1:])
    print(case, reach, "edges", n_edges, "queries with a boundary", found, "list entries", entries)
    assert n_edges > 0 and found > 0
