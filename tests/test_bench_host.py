"""Host logic of bench.py: the boundary edges the grid roofline counts."""
import numpy as np

import bench
from paper_2605_01536_amd import workloads as W


def test_boundary_vertex_z_counts():
    V = np.array([[0, 0, 0], [1, 0, 1], [0, 1, 2], [1, 1, 3]], np.float32)
    # one triangle: three boundary edges, starting at each vertex once
    assert sorted(bench.boundary_vertex_z(V, np.array([[0, 1, 2]]))) == [0, 1, 2]
    # two consistently oriented triangles sharing 1-2: the four outer edges
    z = bench.boundary_vertex_z(V, np.array([[0, 1, 2], [2, 1, 3]]))
    assert sorted(z) == [0, 1, 2, 3]
    # the same pair with the second flipped: edge 1->2 counts twice
    z = bench.boundary_vertex_z(V, np.array([[0, 1, 2], [1, 2, 3]]))
    assert sorted(z) == [0, 1, 1, 2, 2, 3]
    # a closed surface has none
    s = W.icosphere(2)
    assert bench.boundary_vertex_z(s.V, s.F).size == 0


def test_grid_slots_bounds():
    s = W.opened_spheres(seed=3, n_surf=2, tris_per_surf=200)
    g = W.GridSpec(origin=(-1, -1, -1), spacing=(2 / 8, 2 / 8, 2 / 200), dims=(8, 8, 200))
    for prec in ("fp32", "fp64"):
        slots, above, below = bench.grid_slots(s, g, prec)
        dense = bench.I_MIN_GRID_FP64 if prec == "fp64" else bench.I_MIN_GRID
        assert 0.0 < above < 1.0 and 0.0 < below < 1.0 and above + below < 1.0
        assert slots == dense - bench.SKIP_SLOTS[prec] * above - bench.SKIP_SEL_SLOTS[prec] * below
    # a grid wholly above every vertex skips every block's reciprocal; wholly
    # below, every block's select
    hi = W.GridSpec(origin=(-1, -1, 5), spacing=(0.1, 0.1, 0.1), dims=(2, 2, 100))
    lo = W.GridSpec(origin=(-1, -1, -50), spacing=(0.1, 0.1, 0.1), dims=(2, 2, 100))
    assert bench.grid_slots(s, hi, "fp32")[1:] == (1.0, 0.0)
    # blocks of 64 and 36 samples: the first drops the select, the last keeps it
    assert bench.grid_slots(s, lo, "fp32")[1:] == (0.0, 0.64)


def test_cpu_model_is_reported():
    import bench
    s = bench.cpu_model()
    assert isinstance(s, str) and s
