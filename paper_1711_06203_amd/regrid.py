"""Dynamic regridding of a two-level problem: tag, cluster, move the fine level.

The paper's grids adapt to the flow: cells are tagged for refinement and new
fine boxes are built around them (sections 2 and 3).  Tags come from the GPU
(``Solver.tag``: relative density jump across a cell), clusters from the
library's Berger-Rigoutsos clustering on the host (``ctuppm.cluster``), and
the fine level moves on the GPU (``Solver.regrid``: old fine data where the
new patch overlaps the old one, conservative interpolation from the coarse
level elsewhere).  The solver's fine level is one rectangle, so the patch is
the bounding rectangle of the clusters, grown by a buffer and kept at least 3
coarse cells inside the domain.
"""
from __future__ import annotations

from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import ctuppm
from . import workloads as W

MARGIN = 3  # coarse cells between the fine patch and the domain boundary


def patch_from_tags(tags: np.ndarray, buffer: int = 2, blocking: int = 4, efficiency: float = 0.7,
                    max_edge: int = 64) -> Optional[Tuple[Tuple[int, int, int], Tuple[int, int, int]]]:
    """Coarse cell range (lo, hi) of the fine patch for level-0 tags (nz, ny, nx):
    the bounding rectangle of the Berger-Rigoutsos clusters, grown by `buffer`
    cells and clipped to MARGIN cells inside the domain; None without tags."""
    boxes = ctuppm.cluster(tags, blocking, efficiency, max_edge)
    if not boxes:
        return None
    n = tags.shape[::-1]
    lo = [max(MARGIN, min(b[0][d] for b in boxes) - buffer) for d in range(3)]
    hi = [min(n[d] - 1 - MARGIN, max(b[1][d] for b in boxes) + buffer) for d in range(3)]
    if any(hi[d] < lo[d] for d in range(3)):
        return None
    return tuple(lo), tuple(hi)


def fine_boxes(patch, fine_box: int = 32) -> List[W.Box]:
    """Fine boxes (at most fine_box cells per edge) tiling the fine cells of a
    coarse patch (ratio 2)."""
    clo, chi = patch
    flo = tuple(2 * c for c in clo)
    fn = tuple(2 * (chi[d] - clo[d] + 1) for d in range(3))
    return W.regular_boxes(fn, (fine_box,) * 3, origin=flo)


def adapt(solver: ctuppm.Solver, threshold: float, buffer: int = 2, fine_box: int = 32, blocking: int = 4,
          efficiency: float = 0.7) -> Optional[List[W.Box]]:
    """Tag the solver's coarse level, and if the resulting patch differs from
    the current one, regrid onto it.  Returns the new fine boxes (None if the
    patch did not change or nothing was tagged)."""
    tags = solver.tag(threshold)
    patch = patch_from_tags(tags, buffer, blocking, efficiency)
    if patch is None:
        return None
    cur = (tuple(v // 2 for v in solver.fine_lo),
           tuple((solver.fine_lo[d] + solver.fine_n[d]) // 2 - 1 for d in range(3)))
    if patch == cur:
        return None
    boxes = fine_boxes(patch, fine_box)
    solver.regrid(boxes)
    return boxes
