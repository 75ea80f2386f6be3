"""Host-side regridding: the library's Berger-Rigoutsos clustering (host code,
no GPU) against the invariants a clustering must satisfy, and the oracle's
tagging and regrid pinned by closed forms and conservation."""
import math
import os

import numpy as np
import pytest

import oracle
from paper_1711_06203_amd import workloads as W


def _lib_or_skip():
    from paper_1711_06203_amd import ctuppm
    if not os.path.exists(ctuppm.LIB_PATH):
        pytest.skip("library not built")
    return ctuppm


def _blobs(n, seed, count):
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(*[np.arange(v) for v in n[::-1]], indexing="ij")
    t = np.zeros(n[::-1], dtype=bool)
    for _ in range(count):
        c = rng.uniform(0, 1, 3) * np.array(n)
        r = rng.uniform(2, 6, 3)
        t |= ((x - c[0]) / r[0]) ** 2 + ((y - c[1]) / r[1]) ** 2 + ((z - c[2]) / r[2]) ** 2 < 1.0
    return t


@pytest.mark.parametrize("seed,blocking,eff", [(1, 4, 0.7), (2, 2, 0.8), (3, 8, 0.5), (4, 4, 0.9), (5, 1, 0.7)])
def test_cluster_invariants(seed, blocking, eff):
    ctuppm = _lib_or_skip()
    n = (48, 40, 32)
    tags = _blobs(n, seed, 5)
    boxes = ctuppm.cluster(tags, blocking, eff, max_edge=32)
    cover = np.zeros_like(tags, dtype=int)
    for lo, hi in boxes:
        for d in range(3):
            assert 0 <= lo[d] <= hi[d] < n[d]
            assert lo[d] % blocking == 0                                   # aligned
            assert (hi[d] + 1) % blocking == 0 or hi[d] == n[d] - 1        # aligned or clipped
            assert hi[d] - lo[d] + 1 <= 32                                 # edge limit
        cover[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] += 1
        # efficiency in blocks: tagged blocks / blocks of the box
        sub = tags[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1]
        nb = [-(-s // blocking) for s in sub.shape]
        tb = 0
        for k in range(nb[0]):
            for j in range(nb[1]):
                for i in range(nb[2]):
                    tb += sub[k * blocking:(k + 1) * blocking, j * blocking:(j + 1) * blocking,
                              i * blocking:(i + 1) * blocking].any()
        assert tb / (nb[0] * nb[1] * nb[2]) >= eff - 1e-12
    assert cover.max() <= 1                  # disjoint
    assert np.all(cover[tags] == 1)          # every tagged cell covered


def test_cluster_separates_two_blobs():
    ctuppm = _lib_or_skip()
    tags = np.zeros((32, 32, 32), dtype=bool)
    tags[4:8, 4:8, 4:8] = True
    tags[20:28, 20:24, 16:28] = True
    boxes = sorted(ctuppm.cluster(tags, 4, 0.7, 64))
    assert boxes == [((4, 4, 4), (7, 7, 7)), ((16, 20, 20), (27, 23, 27))]


def test_cluster_empty_and_bad_arguments():
    ctuppm = _lib_or_skip()
    assert ctuppm.cluster(np.zeros((8, 8, 8), dtype=bool)) == []
    with pytest.raises(ctuppm.CtuError):
        ctuppm.cluster(np.ones((8, 8, 8), dtype=bool), blocking=0)


def test_patches_from_tags_cover_the_buffered_tags_disjointly():
    _lib_or_skip()
    from paper_1711_06203_amd import regrid
    tags = np.zeros((32, 32, 32), dtype=bool)
    tags[10:12, 8:9, 12:20] = True    # (z, y, x)
    tags[14:16, 20:22, 12:14] = True
    tags[2, 2, 2] = True              # near the corner: clipped to the margin
    patches = regrid.patches_from_tags(tags, buffer=2, blocking=4)
    assert len(patches) >= 2          # the two blobs are not merged into one rectangle
    grown = regrid.dilate(tags, 2)
    cover = np.zeros_like(tags)
    for q, (lo, hi) in enumerate(patches):
        for d in range(3):
            assert regrid.MARGIN <= lo[d] <= hi[d] <= 31 - regrid.MARGIN
        box = cover[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1]
        assert not box.any()          # disjoint
        box[...] = True
    inner = np.zeros_like(tags)
    m = regrid.MARGIN
    inner[m:32 - m, m:32 - m, m:32 - m] = True
    assert not (grown & inner & ~cover).any()
    # dilation by a cube of half-width 2
    one = np.zeros((9, 9, 9), dtype=bool)
    one[4, 4, 4] = True
    assert np.array_equal(np.argwhere(regrid.dilate(one, 2)).min(0), [2, 2, 2])
    assert regrid.dilate(one, 2).sum() == 125
    fb, rects = regrid.fine_level(patches, fine_box=16)
    vol = sum(np.prod([b[1][d] - b[0][d] + 1 for d in range(3)]) for b in fb)
    assert vol == 8 * sum(np.prod([hi[d] - lo[d] + 1 for d in range(3)]) for lo, hi in patches)


def test_oracle_regrid_patches_copies_every_old_patch():
    n = (16, 16, 16)
    x, y, z = W.cell_centres(n)
    Uc = np.stack([1.0 - 0.2 * x + 0.3 * y + 0.05 * z] * 5)
    rng = np.random.default_rng(1)
    old = [((8, 8, 8), rng.uniform(0.5, 1.5, (5, 4, 4, 4))), ((16, 8, 8), rng.uniform(0.5, 1.5, (5, 4, 4, 6)))]
    new = [((6, 6, 8), (16, 8, 4))]   # fine x 6..21, y 6..13, z 8..11
    (Uf,) = oracle.regrid_patches(Uc, old, new)
    np.testing.assert_array_equal(Uf[:, 0:4, 2:6, 2:6], old[0][1])
    np.testing.assert_array_equal(Uf[:, 0:4, 2:6, 10:16], old[1][1][:, :, :, 0:6])
    fx, fy, fz = W.cell_centres((32, 32, 32))
    exact = (1.0 - 0.2 * fx + 0.3 * fy + 0.05 * fz)[8:12, 6:14, 6:22]
    mask = np.ones(exact.shape, dtype=bool)
    mask[0:4, 2:6, 2:6] = False
    mask[0:4, 2:6, 10:16] = False
    np.testing.assert_allclose(Uf[0][mask], exact[mask], rtol=0, atol=1e-14)


def test_oracle_tags_the_cells_beside_a_jump():
    prob = W.sod(n=(16, 4, 4))
    tags = oracle.tag_cells(prob.U0, oracle.params_of(prob), 0.1)
    want = np.zeros(tags.shape, dtype=bool)
    want[:, :, 7:9] = True                     # the two cells on either side of x = 0.5
    assert np.array_equal(tags, want)
    uni = W.uniform(n=(8, 8, 8))
    assert not oracle.tag_cells(uni.U0, oracle.params_of(uni), 1e-12).any()


def test_oracle_regrid_interpolates_linear_fields_exactly_and_copies_overlap():
    n = (16, 16, 16)
    x, y, z = W.cell_centres(n)
    Uc = np.stack([1.0 + 0.3 * x - 0.2 * y + 0.1 * z] * 5)
    old_lo, old_n = (12, 12, 12), (8, 8, 8)
    Uf_old = np.random.default_rng(0).uniform(0.5, 1.5, (5, 8, 8, 8))
    new_lo, new_n = (8, 10, 14), (12, 10, 8)
    Uf = oracle.regrid_fine(Uc, Uf_old, old_lo, new_lo, new_n)
    fx, fy, fz = W.cell_centres((32, 32, 32))
    sl = (slice(new_lo[2], new_lo[2] + new_n[2]), slice(new_lo[1], new_lo[1] + new_n[1]),
          slice(new_lo[0], new_lo[0] + new_n[0]))
    exact = (1.0 + 0.3 * fx - 0.2 * fy + 0.1 * fz)[sl]
    # overlap with the old patch: fine x 12..19 -> new 4..11, y 12..19 -> 2..9, z 14..19 -> 0..5
    ov = (slice(None), slice(0, 6), slice(2, 10), slice(4, 12))
    np.testing.assert_array_equal(Uf[ov], Uf_old[:, 2:8, 0:8, 0:8])
    mask = np.ones(exact.shape, dtype=bool)
    mask[0:6, 2:10, 4:12] = False
    np.testing.assert_allclose(Uf[0][mask], exact[mask], rtol=0, atol=1e-14)


def test_oracle_regrid_conserves_the_composite_state():
    """Regridding a consistent two-level state (coarse cells under the fine
    patch equal to the average of their children) keeps the composite totals."""
    prob = W.cloud_wind(n=16, box=16, fine_box=16, fine_region=((4, 4, 4), (12, 12, 12)))
    rc, rf, _, _ = oracle.run_two_level(prob, 2)

    def composite(Uc, Uf, flo):
        c = np.array(flo) // 2
        nf = np.array(Uf.shape[1:][::-1])
        mask = np.ones(Uc.shape[1:], dtype=bool)
        mask[c[2]:c[2] + nf[2] // 2, c[1]:c[1] + nf[1] // 2, c[0]:c[0] + nf[0] // 2] = False
        return [math.fsum(Uc[m][mask].ravel()) + math.fsum(Uf[m].ravel()) / 8.0 for m in range(Uc.shape[0])]

    before = composite(rc, rf, prob.fine_lo)
    new_lo, new_n = (10, 8, 8), (16, 18, 16)
    Uf = oracle.regrid_fine(rc, rf, prob.fine_lo, new_lo, new_n)
    after = composite(rc, Uf, new_lo)
    for m in range(len(before)):
        assert abs(after[m] - before[m]) <= 1e-13 * max(1.0, abs(before[m]))
