"""The sound-wave workload against the linear-wave configurations the paper prints
(Sec. 4, linear waves: the table of N and n and Eq. wave_angle, in
tests/golden/linear_wave_configurations.txt): its wave travels along the direction the
paper's rotation gives, the in-plane diagonal in 2D and the body diagonal in 3D."""
import math
import os

import numpy as np

from paper_2205_00095_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                out.append(line.split())
    return out


def _rotation(axis, theta):
    """R = cos(theta) I + (1 - cos(theta)) a a^T + sin(theta) [a]_x about the unit axis a."""
    a = np.asarray(axis, dtype=float)
    a = a / np.linalg.norm(a)
    ax = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    return math.cos(theta) * np.eye(3) + (1 - math.cos(theta)) * np.outer(a, a) + math.sin(theta) * ax


def _paper_direction(test_type, N, n):
    theta = math.atan(math.sqrt(N / (N - n) - 1.0))
    axis = (0.0, -1.0, 1.0) if test_type.startswith("3D") else (0.0, 1.0, 0.0)
    return _rotation(axis, theta) @ np.array([1.0, 0.0, 0.0]), theta


def _workload_direction(dim):
    cfg = wl.make_config("sound", dim=dim, p=2, n_elem=tuple([4] * dim + [1] * (3 - dim)))
    rho, v, P = wl.sound_primitives(cfg)
    flat = v.reshape(dim, -1)
    i = int(np.argmax(np.linalg.norm(flat, axis=0)))
    d = flat[:, i] / np.linalg.norm(flat[:, i])
    return d * np.sign(d[0])


def test_table_angles():
    rows = {r[0]: (int(r[1]), int(r[2])) for r in _rows("linear_wave_configurations.txt")}
    assert set(rows) == {"1D", "2D_grid_aligned", "2D_non_grid_aligned", "3D_grid_aligned", "3D_non_grid_aligned"}
    for name, (N, n) in rows.items():
        k, theta = _paper_direction(name, N, n)
        assert abs(np.linalg.norm(k) - 1.0) < 1e-15
        if n == 0:
            assert theta == 0.0 and np.allclose(k, [1.0, 0.0, 0.0], atol=1e-15)
    assert abs(_paper_direction("2D_non_grid_aligned", *rows["2D_non_grid_aligned"])[1] - math.pi / 4) < 1e-15


def test_sound_workload_follows_the_paper_directions():
    rows = {r[0]: (int(r[1]), int(r[2])) for r in _rows("linear_wave_configurations.txt")}
    # 3D: the rotation about (0, -1, 1) by the tabulated angle takes x to the body diagonal
    k3, _ = _paper_direction("3D_non_grid_aligned", *rows["3D_non_grid_aligned"])
    assert np.allclose(k3, np.ones(3) / math.sqrt(3.0), atol=1e-15)
    assert np.allclose(_workload_direction(3), k3, atol=1e-12)
    # 2D: 45 degrees; the rotation about y leaves the x-y plane, read as the in-plane
    # diagonal (equal components along the two axes of the simulated plane)
    k2, _ = _paper_direction("2D_non_grid_aligned", *rows["2D_non_grid_aligned"])
    comps = np.sort(np.abs(k2[np.abs(k2) > 1e-12]))
    assert np.allclose(comps, [1 / math.sqrt(2.0)] * 2, atol=1e-15)
    assert np.allclose(np.abs(_workload_direction(2)), comps, atol=1e-12)
