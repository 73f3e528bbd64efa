"""Host-side logic of bench.py: the algorithmic byte count of the five-colour box sweep against a brute-force
count over Python sets, and the refusal of multi-GPU runs."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def brute_bytes(cls, N, elem):
    W = N + 2
    flat = [cls[g].ravel() for g in range(3)]
    vals = set()  # (field, index) of every value read
    clsb = set()
    rows = set()  # internal unknowns: right-hand side read and value written
    for j in range(N):
        for i in range(N):
            c = (j + 1) * W + (i + 1)
            box = [(0, c), (0, c + 1), (1, c), (1, c + W), (2, c)]
            if not any(flat[g][k] == 1 for g, k in box):
                continue
            for g, k in box:
                clsb.add((g, k))
                if flat[g][k] != 1:
                    continue
                rows.add((g, k))
                if g == 0:  # momentum x: -Laplacian of u and the pressure difference across the face
                    vals.update((0, k + o) for o in (0, -1, 1, -W, W))
                    vals.update([(2, k), (2, k - 1)])
                elif g == 1:
                    vals.update((1, k + o) for o in (0, -1, 1, -W, W))
                    vals.update([(2, k), (2, k - W)])
                else:  # continuity: the four faces of the cell
                    vals.update([(0, k), (0, k + 1), (1, k), (1, k + W)])
    return len(clsb) + len(rows) * 2 * elem + len(vals) * elem


def test_box_sweep_bytes_matches_brute_force():
    rng = np.random.default_rng(5)
    for N in (7, 12):
        W = N + 2
        cls = rng.choice([0, 1, 2, 3], size=(3, W, W), p=[0.2, 0.6, 0.1, 0.1]).astype(np.uint8)
        cls[:, 0, :] = cls[:, -1, :] = cls[:, :, 0] = cls[:, :, -1] = 3  # the border ring holds no unknown
        for elem in (8, 4):
            assert bench.box_sweep_bytes(cls, N, elem) == brute_bytes(cls, N, elem)


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_native_oracle_builds_with_openmp_and_matches_portable_build(tmp_path):
    """the CPU-baseline library (-O3 -march=native -fopenmp) runs the same iteration: a cycle of the petal body
    at N = 64 agrees with the portable single-thread build to rounding"""
    import oracle as O
    from paper_1911_00994_amd import workloads as wl
    from tests.common import make_linear_problem
    shape = wl.Shape(wl.PETALS, (0.35, 0.07, 0.0, 5.0))
    N = 64
    out = []
    for path in (None, O.build_native(str(tmp_path / "libnative.so"), openmp=True)):
        O.lib(path or O.build_oracle())
        o, _, _ = make_linear_problem(N, shape, 0.64 * (2.0 / N) ** 2)
        o.cycle()
        out.append(np.concatenate([a.ravel() for a in o.get_x()[:3]]))
        threads = O.lib().or_threads()
        del o
    O.lib(O.build_oracle())
    assert threads >= 1
    assert np.abs(out[0] - out[1]).max() < 1e-9 * max(1.0, np.abs(out[0]).max())
