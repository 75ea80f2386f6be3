"""Dynamic regridding of a two-level problem: tag, cluster, move the fine level.

The paper's grids adapt to the flow: cells are tagged for refinement and new
fine boxes are built around them (sections 2 and 3; figure 1 shows fine boxes
over separate parts of the coarse level).  Tags come from the GPU
(``Solver.tag``: relative density jump across a cell), clusters from the
library's Berger-Rigoutsos clustering on the host (``ctuppm.cluster``), and
the fine level moves on the GPU (``Solver.regrid``: old fine data where a new
box overlaps the old fine level, conservative interpolation from the coarse
level elsewhere).  Every cluster becomes a fine patch of its own: the tags
are first grown by a buffer of cells, so the clusters cover the buffered
tags and stay disjoint, and each is kept at least 3 coarse cells inside the
domain.
"""
from __future__ import annotations

from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import ctuppm
from . import workloads as W

MARGIN = 3  # coarse cells between a fine patch and the domain boundary

CBox = Tuple[Tuple[int, int, int], Tuple[int, int, int]]  # coarse cells lo..hi, inclusive


def dilate(tags: np.ndarray, cells: int) -> np.ndarray:
    """Tags (nz, ny, nx) grown by `cells` cells in every direction (a cube)."""
    out = np.asarray(tags, dtype=bool).copy()
    for axis in range(3):
        cur = out.copy()
        for s in range(1, cells + 1):
            lo = [slice(None)] * 3
            hi = [slice(None)] * 3
            lo[axis], hi[axis] = slice(s, None), slice(None, -s)
            out[tuple(lo)] |= cur[tuple(hi)]
            out[tuple(hi)] |= cur[tuple(lo)]
    return out


def patches_from_tags(tags: np.ndarray, buffer: int = 2, blocking: int = 4, efficiency: float = 0.7,
                      max_edge: int = 64) -> List[CBox]:
    """Coarse patches (lo, hi inclusive) for level-0 tags (nz, ny, nx): the
    Berger-Rigoutsos clusters of the tags grown by `buffer` cells, each clipped
    to MARGIN cells inside the domain (clusters left empty are dropped).  The
    patches are disjoint and cover every buffered tag inside the margin."""
    boxes = ctuppm.cluster(dilate(tags, buffer), blocking, efficiency, max_edge)
    n = tags.shape[::-1]
    out = []
    for lo, hi in boxes:
        lo = tuple(max(MARGIN, lo[d]) for d in range(3))
        hi = tuple(min(n[d] - 1 - MARGIN, hi[d]) for d in range(3))
        if all(hi[d] >= lo[d] for d in range(3)):
            out.append((lo, hi))
    return out


def fine_boxes(patch: CBox, fine_box: int = 32) -> List[W.Box]:
    """Fine boxes (at most fine_box cells per edge) tiling the fine cells of a
    coarse patch (ratio 2)."""
    clo, chi = patch
    flo = tuple(2 * c for c in clo)
    fn = tuple(2 * (chi[d] - clo[d] + 1) for d in range(3))
    return W.regular_boxes(fn, (fine_box,) * 3, origin=flo)


def fine_level(patches: Sequence[CBox], fine_box: int = 32):
    """Fine boxes tiling every coarse patch, and the patches as fine rectangles
    (fine index lo, extent)."""
    boxes, rects = [], []
    for p in patches:
        boxes += fine_boxes(p, fine_box)
        rects.append((tuple(2 * c for c in p[0]), tuple(2 * (p[1][d] - p[0][d] + 1) for d in range(3))))
    return boxes, rects


def current_patches(solver: ctuppm.Solver) -> List[CBox]:
    """The solver's fine patches as coarse cell ranges."""
    return [(tuple(lo[d] // 2 for d in range(3)), tuple((lo[d] + n[d]) // 2 - 1 for d in range(3)))
            for lo, n in solver.patches]


def adapt(solver: ctuppm.Solver, threshold: float, buffer: int = 2, fine_box: int = 32, blocking: int = 4,
          efficiency: float = 0.7) -> Optional[List[CBox]]:
    """Tag the solver's coarse level and, if the patches of the tags differ
    from the current ones, regrid onto them.  Returns the new coarse patches
    (None if nothing was tagged or the patches did not change)."""
    tags = solver.tag(threshold)
    patches = patches_from_tags(tags, buffer, blocking, efficiency)
    if not patches or sorted(patches) == sorted(current_patches(solver)):
        return None
    boxes, rects = fine_level(patches, fine_box)
    solver.regrid(boxes, rects)
    return patches
