"""Parity at the full benchmark sizes, in the launch configuration bench.py times.

The GPU takes one step of the whole 256^3 (64 boxes) and 384^3 (uneven
boxes) workloads in the graph form; the oracle computes sampled cells one by
one from their 9^3 neighbourhoods of the same initial state (ghosts filled by
the oracle), with the dt it computes itself from the whole initial state."""
import numpy as np
import pytest

import oracle
from paper_1711_06203_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1711_06203_amd import ctuppm
    c = ctuppm.Context()
    yield c
    c.close()


def _sampled(ctx, prob, nsamp, seed):
    from paper_1711_06203_amd import ctuppm
    s = ctuppm.Solver(ctx, prob, form="graph")
    s.step(1)
    got = s.state()
    dt_gpu = s.dt()
    s.close()
    ctx.torch.cuda.empty_cache()
    P = oracle.params_of(prob)
    G = oracle.fill_domain(oracle.grow(prob.U0), P)
    dt = P.cfl / oracle.signal_speed(G, P)
    assert dt_gpu == dt
    rng = np.random.default_rng(seed)
    n = prob.n
    cells = [tuple(int(rng.integers(n[d])) for d in range(3)) for _ in range(nsamp)]
    # always include box corners and domain faces
    for (lo, hi) in prob.boxes[:8]:
        cells.append(tuple(lo))
        cells.append(tuple(hi))
    cells += [(0, 0, 0), (n[0] - 1, n[1] - 1, n[2] - 1), (0, n[1] - 1, 0)]
    want = oracle.sample_step(G, P, dt, cells)
    for c, w in zip(cells, want):
        g = got[:, c[2], c[1], c[0]]
        assert np.array_equal(g, w), (c, g, w)


@pytest.mark.slow
def test_kh256_one_step_sampled(ctx):
    _sampled(ctx, W.kelvin_helmholtz(n=256, box=64), 400, 1)


@pytest.mark.slow
def test_largest_box_edge_one_box_256_sampled(ctx):
    """The whole 256^3 KH domain as one box, the largest edge accepted."""
    prob = W.kelvin_helmholtz(n=256, box=256)
    assert len(prob.boxes) == 1
    _sampled(ctx, prob, 200, 11)


def _fullsize_digests():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_sha256.txt")
    out = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            out[k.strip()] = v.split()
    return out


@pytest.mark.slow
@pytest.mark.parametrize("name", ["kh256_10", "kh256_13species_1", "kh256_mol2_2", "cloud256_1", "two_clouds256_1"])
def test_fullsize_states_bitwise(ctx, name):
    """The whole state after a few steps of a full-size workload (KH 256^3 ten
    steps, with 13 species, with MOL-RK2; the two-level cloud 256^3 + 256^3 one
    coarse step; two clouds with a fine patch each, 2 x 128^3 fine cells, one
    coarse step) bit for bit the oracle's, compared through the SHA-256 digests
    of the oracle's runs (tests/golden/make_fullsize_digests.py writes them)."""
    import hashlib
    import os
    import sys
    from paper_1711_06203_amd import ctuppm
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import make_fullsize_digests as G
    want = _fullsize_digests()[name]
    prob, steps = G.cases()[name]
    s = ctuppm.Solver(ctx, prob, form="graph")
    s.step(steps)
    states = [s.state()] + (s.state_patches() if prob.fine_boxes else [])
    dt = s.dt()
    cnt = s.counters()
    s.close()
    ctx.torch.cuda.empty_cache()
    assert not cnt[:5].any()
    assert dt == float.fromhex(want[0])
    got = [hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest() for a in states]
    assert got == want[1:], name


@pytest.mark.slow
def test_rt384_uneven_one_step_sampled(ctx):
    prob = W.rayleigh_taylor(n=384)
    assert len(prob.boxes) > 500
    _sampled(ctx, prob, 400, 2)


@pytest.mark.slow
@pytest.mark.parametrize("n", [32, 48, 64, 96, 128])
def test_serving_sizes_ten_steps(ctx, n):
    from paper_1711_06203_amd import ctuppm
    from gpu_helpers import max_rel, totals_rel
    prob = W.serving_request(seed=40 + n, n=n, steps=10)
    ref, _, _ = oracle.run_problem(prob, 10)
    s = ctuppm.Solver(ctx, prob, form="graph")
    s.step(10)
    got = s.state()
    s.close()
    print(f"serving N={n}: bitwise={np.array_equal(got, ref)}", flush=True)
    assert max(max_rel(got, ref)) <= 1e-10 and max(totals_rel(got, ref)) <= 1e-13


@pytest.mark.slow
def test_kh256_ten_steps_full(ctx):
    from paper_1711_06203_amd import ctuppm
    from gpu_helpers import l1_rel, totals_rel
    prob = W.kelvin_helmholtz(n=256, box=64)
    s = ctuppm.Solver(ctx, prob, form="graph")
    s.step(10)
    got = s.state()
    s.close()
    ctx.torch.cuda.empty_cache()
    ref, _, cnt = oracle.run_problem(prob, 10)
    print(f"kh256 10 steps: bitwise={np.array_equal(got, ref)}", flush=True)
    assert max(l1_rel(got, ref)) <= 1e-8 and max(totals_rel(got, ref)) <= 1e-13
    assert not cnt.any()


@pytest.mark.slow
def test_rt384_two_steps_full(ctx):
    """The batched uneven-box workload at full size (RT 384^3, 1436 boxes,
    gravity, reflecting walls): the whole state after two graph steps bitwise
    the oracle's."""
    from paper_1711_06203_amd import ctuppm
    prob = W.rayleigh_taylor(n=384)
    s = ctuppm.Solver(ctx, prob, form="graph")
    s.step(2)
    got = s.state()
    cnt = s.counters()
    s.close()
    ctx.torch.cuda.empty_cache()
    ref, _, rcnt = oracle.run_problem(prob, 2)
    print(f"rt384 2 steps: bitwise={np.array_equal(got, ref)}", flush=True)
    assert np.array_equal(got, ref)
    assert not cnt[:5].any() and not rcnt.any()


@pytest.mark.slow
@pytest.mark.parametrize("variant", [dict(riemann=1), dict(limiter=1), dict(steepen=1), dict(scheme=2)],
                         ids=["twoshock", "cs", "steepen", "mol3"])
def test_kh256_variants_one_step_full(ctx, variant):
    """Each scheme variant at the full KH 256^3 size: the whole state after
    one graph step bitwise the oracle's, run beside it."""
    from paper_1711_06203_amd import ctuppm
    prob = W.kelvin_helmholtz(n=256, box=64)
    for k, v in variant.items():
        setattr(prob, k, v)
    s = ctuppm.Solver(ctx, prob, form="graph")
    s.step(1)
    got = s.state()
    s.close()
    ctx.torch.cuda.empty_cache()
    ref, _, rcnt = oracle.run_problem(prob, 1)
    assert np.array_equal(got, ref), variant
    assert not rcnt.any()


@pytest.mark.slow
def test_rt96_twenty_steps(ctx):
    from paper_1711_06203_amd import ctuppm
    from gpu_helpers import l1_rel
    prob = W.rayleigh_taylor(n=96, seed=6)
    ref, _, _ = oracle.run_problem(prob, 20)
    s = ctuppm.Solver(ctx, prob, form="graph")
    s.step(20)
    got = s.state()
    s.close()
    assert max(l1_rel(got, ref)) <= 1e-8


@pytest.mark.slow
def test_cloud_two_level_64_twenty_steps(ctx):
    from paper_1711_06203_amd import ctuppm
    from gpu_helpers import l1_rel
    prob = W.cloud_wind(n=64, box=32, fine_box=32)
    rc, rf, _, _ = oracle.run_two_level(prob, 20)
    s = ctuppm.Solver(ctx, prob, form="graph")
    s.step(20)
    gc, gf = s.state(), s.state_fine()
    s.close()
    print(f"cloud64 20 steps: bitwise coarse={np.array_equal(gc, rc)} fine={np.array_equal(gf, rf)}", flush=True)
    assert max(l1_rel(gc, rc)) <= 1e-8 and max(l1_rel(gf, rf)) <= 1e-8


@pytest.mark.slow
def test_kh256_13species_one_step_sampled(ctx):
    prob = W.kelvin_helmholtz(n=256, box=64, nspec=13)
    assert prob.U0.shape[0] == 18
    _sampled(ctx, prob, 200, 3)


@pytest.mark.slow
def test_kh256_mol_rk2_one_step_sampled(ctx):
    """The method-of-lines (SSP-RK2) step of the full 256^3 KH workload in the
    graph form, sampled cells against the oracle's two stages computed from
    each sample's periodic neighbourhood."""
    from paper_1711_06203_amd import ctuppm
    prob = W.kelvin_helmholtz(n=256, box=64)
    prob.scheme = 1
    s = ctuppm.Solver(ctx, prob, form="graph")
    s.step(1)
    got = s.state()
    dt_gpu = s.dt()
    s.close()
    ctx.torch.cuda.empty_cache()
    P = oracle.params_of(prob)
    G = oracle.fill_domain(oracle.grow(prob.U0), P)
    dt = P.cfl / oracle.signal_speed(G, P)
    assert dt_gpu == dt
    rng = np.random.default_rng(4)
    cells = [tuple(int(rng.integers(256)) for _ in range(3)) for _ in range(150)]
    cells += [(0, 0, 0), (255, 255, 255), (63, 64, 0), (64, 63, 255)]
    want = oracle.sample_step_mol(prob.U0, P, dt, cells)
    for c, w in zip(cells, want):
        g = got[:, c[2], c[1], c[0]]
        assert np.array_equal(g, w), (c, g, w)


@pytest.mark.slow
def test_kh256_twoshock_one_step_sampled(ctx):
    prob = W.kelvin_helmholtz(n=256, box=64)
    prob.riemann = 1
    _sampled(ctx, prob, 150, 5)


@pytest.mark.slow
def test_kh256_cs_limiter_one_step_sampled(ctx):
    prob = W.kelvin_helmholtz(n=256, box=64)
    prob.limiter = 1
    _sampled(ctx, prob, 150, 6)


@pytest.mark.slow
def test_kh256_steepened_one_step_sampled(ctx):
    prob = W.kelvin_helmholtz(n=256, box=64)
    prob.steepen = 1
    _sampled(ctx, prob, 150, 7)


@pytest.mark.slow
def test_cloud256_tags_and_regrid_sampled(ctx):
    """Full-size two-level cloud: tags of the initial coarse state equal the
    oracle's, and a regrid onto a larger patch gives, at sampled fine cells,
    the old fine value inside the old patch and the oracle's coarse-to-fine
    interpolation outside it."""
    from paper_1711_06203_amd import ctuppm, regrid
    prob = W.cloud_wind(n=256, box=64, fine_box=32)
    s = ctuppm.Solver(ctx, prob, form="graph")
    P = oracle.params_of(prob)
    tg = s.tag(0.05)
    assert np.array_equal(tg, oracle.tag_cells(prob.U0, P, 0.05))
    patch = ((70, 60, 64), (185, 190, 170))
    s.regrid(regrid.fine_boxes(patch, 32))
    got = s.state_fine()
    s.step(1)
    cnt = s.counters()
    s.close()
    ctx.torch.cuda.empty_cache()
    assert not cnt[:5].any()
    flo = np.array([2 * v for v in patch[0]])
    fn = np.array([2 * (patch[1][d] - patch[0][d] + 1) for d in range(3)])
    olo = np.array(prob.fine_lo)
    on = np.array(prob.U0_fine.shape[1:][::-1])
    rng = np.random.default_rng(9)
    cells = [flo + rng.integers(fn) for _ in range(300)] + [flo, flo + fn - 1, olo, olo + on - 1, olo - 1, olo + on]
    cells = [I for I in cells if np.all(I >= flo) and np.all(I < flo + fn)]  # inside the new patch
    assert len(cells) >= 300
    for I in cells:
        g = got[:, I[2] - flo[2], I[1] - flo[1], I[0] - flo[0]]
        if np.all(I >= olo) and np.all(I < olo + on):
            w = prob.U0_fine[:, I[2] - olo[2], I[1] - olo[1], I[0] - olo[0]]
        else:
            w = oracle.cf_interp(prob.U0, (0, 0, 0), I[None, :])[:, 0]
        assert np.array_equal(g, w), (I, g, w)
