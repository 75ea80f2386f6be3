"""Seeded synthetic inputs shared by the HIP path, the tests and the bench.

This module holds no step of the hydro scheme.  It evaluates initial
conditions at cell centres, turns the primitive initial fields into the
conserved state with the ideal-gas energy relation (E = p/(gamma-1) + kinetic
energy), and cuts index-space domains into boxes.  Random numbers come from
numpy's PCG64 (``numpy.random.default_rng(seed)``) and are drawn over the global
index space in C order (k, j, i), so a box decomposition never changes an
initial condition.

The workloads stand in for the paper's own problems (Sedov with a stellar
equation of state, white-dwarf mergers, X-ray bursts; section 4), whose inputs
are not available: their shapes follow the paper's description of block
structured grids (boxes of unequal size, a refined patch over several coarse
boxes; section 3, Figure 1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

NVAR = 5
NGHOST = 4

BC_PERIODIC, BC_OUTFLOW, BC_REFLECT, BC_INFLOW = 0, 1, 2, 3

Box = Tuple[Tuple[int, int, int], Tuple[int, int, int]]  # (lo, hi) inclusive, (i, j, k)


@dataclasses.dataclass
class Problem:
    """One hydro problem on a level-0 index space [0, n) with its boxes."""

    name: str
    n: Tuple[int, int, int]                 # cells (nx, ny, nz)
    gamma: float
    U0: np.ndarray                          # conserved state, shape (5, nz, ny, nx)
    boxes: List[Box]
    bc_lo: Tuple[int, int, int] = (BC_PERIODIC,) * 3
    bc_hi: Tuple[int, int, int] = (BC_PERIODIC,) * 3
    cfl: float = 0.5
    grav_z: float = 0.0
    inflow: Tuple[float, float, float, float, float] = (1.0, 0.0, 0.0, 0.0, 1.0)
    prob_lo: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    prob_hi: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    steps: int = 10
    small_dens: float = 1e-12
    small_pres: float = 1e-12
    nspec: int = 0                          # passive species (rho X_s after rho E)
    inflow_X: Tuple[float, ...] = ()        # species mass fractions written by inflow
    scheme: int = 0                         # 0 CTU/PPM, 1 MOL + SSP-RK2, 2 MOL + SSP-RK3
    riemann: int = 0                        # 0 HLLC, 1 two-shock approximate solver
    limiter: int = 0                        # 0 CW84, 1 Colella-Sekora extremum-preserving
    steepen: int = 0                        # 1: CW84 contact steepening of the density
    # two-level problems only
    fine_boxes: Optional[List[Box]] = None   # fine-level index space
    U0_fine: Optional[np.ndarray] = None     # (5, nzf, nyf, nxf) over the fine bounding region
    fine_lo: Optional[Tuple[int, int, int]] = None  # fine index of U0_fine[..., 0, 0, 0]
    # a fine level of several rectangular patches: (fine index lo, state); when
    # set, fine_boxes tile every patch and U0_fine / fine_lo are not used
    fine_patches: Optional[List[Tuple[Tuple[int, int, int], np.ndarray]]] = None

    @property
    def dx(self) -> Tuple[float, float, float]:
        return tuple((self.prob_hi[d] - self.prob_lo[d]) / self.n[d] for d in range(3))

    @property
    def zones(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


# ----------------------------------------------------------------------------
# geometry helpers
# ----------------------------------------------------------------------------

def cell_centres(n: Sequence[int], lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), offset=(0, 0, 0)):
    """Cell-centre coordinates (x, y, z), each shaped (nz, ny, nx)."""
    axes = []
    for d in range(3):
        dx = (hi[d] - lo[d]) / n[d]
        axes.append(lo[d] + (np.arange(offset[d], offset[d] + n[d], dtype=np.float64) + 0.5) * dx)
    z, y, x = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return x, y, z


def conserved(gamma, rho, u, v, w, p, X=None) -> np.ndarray:
    """Ideal-gas conserved state (rho, rho u, rho v, rho w, rho E[, rho X_s]) of
    primitive fields; X is an optional sequence of species mass fractions."""
    rho = np.asarray(rho, dtype=np.float64)
    ns = 0 if X is None else len(X)
    shape = np.broadcast_shapes(np.shape(rho), np.shape(u), np.shape(v), np.shape(w), np.shape(p),
                                *[np.shape(x) for x in (X or [])])
    U = np.empty((NVAR + ns,) + shape, dtype=np.float64)
    rho = np.broadcast_to(rho, shape)
    u = np.broadcast_to(np.asarray(u, np.float64), shape)
    v = np.broadcast_to(np.asarray(v, np.float64), shape)
    w = np.broadcast_to(np.asarray(w, np.float64), shape)
    p = np.broadcast_to(np.asarray(p, np.float64), shape)
    U[0] = rho
    U[1] = rho * u
    U[2] = rho * v
    U[3] = rho * w
    U[4] = p / (gamma - 1.0) + 0.5 * rho * ((u * u + v * v) + w * w)
    for s_ in range(ns):
        U[NVAR + s_] = rho * np.broadcast_to(np.asarray(X[s_], np.float64), shape)
    return U


def regular_boxes(n: Sequence[int], edge: Sequence[int], origin=(0, 0, 0)) -> List[Box]:
    """Cut [origin, origin+n) into boxes of the given edge; the last box along a
    direction keeps the remainder (a ragged tail) when the edge does not divide n."""
    out = []
    for k in range(0, n[2], edge[2]):
        for j in range(0, n[1], edge[1]):
            for i in range(0, n[0], edge[0]):
                lo = (origin[0] + i, origin[1] + j, origin[2] + k)
                hi = (origin[0] + min(i + edge[0], n[0]) - 1, origin[1] + min(j + edge[1], n[1]) - 1,
                      origin[2] + min(k + edge[2], n[2]) - 1)
                out.append((lo, hi))
    return out


EDGE_SET = (16, 24, 32, 48, 64)


def _composition(rng: np.random.Generator, total: int, edges=EDGE_SET) -> List[int]:
    """Split ``total`` into edges from ``edges``; every draw leaves 0 or >= 16."""
    out = []
    rem = total
    while rem > 0:
        allowed = [e for e in edges if e <= rem and (rem - e == 0 or rem - e >= min(edges))]
        if not allowed:
            raise ValueError(f"cannot compose {total} from {edges}")
        e = allowed[int(rng.integers(len(allowed)))]
        out.append(e)
        rem -= e
    return out


def uneven_boxes(n: Sequence[int], seed: int, edges=EDGE_SET) -> List[Box]:
    """Hierarchical compositions: z slabs, then per slab y rows, then per row x boxes."""
    rng = np.random.default_rng(seed)
    out = []
    z0 = 0
    for ez in _composition(rng, n[2], edges):
        y0 = 0
        for ey in _composition(rng, n[1], edges):
            x0 = 0
            for ex in _composition(rng, n[0], edges):
                out.append(((x0, y0, z0), (x0 + ex - 1, y0 + ey - 1, z0 + ez - 1)))
                x0 += ex
            y0 += ey
        z0 += ez
    return out


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

def sod(n=32, axis=0, gamma=1.4, boxes_edge=None, steps=20, flip=False) -> Problem:
    """Sod shock tube along ``axis``: left (rho, p) = (1, 1), right (0.125, 0.1)."""
    nn = [n, n, n] if np.isscalar(n) else list(n)
    x = cell_centres(nn)[axis]
    left = x < 0.5
    if flip:
        left = ~left
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    U = conserved(gamma, rho, 0.0, 0.0, 0.0, p)
    bc = [BC_PERIODIC] * 3
    bc[axis] = BC_OUTFLOW
    edge = boxes_edge or nn
    if np.isscalar(edge):
        edge = [edge] * 3
    return Problem("sod", tuple(nn), gamma, U, regular_boxes(nn, edge), tuple(bc), tuple(bc),
                   cfl=0.5, steps=steps)


def species_bands(y, nspec: int, width: float = 0.05):
    """nspec smooth mass fractions summing to 1: normalised Gaussian bands centred
    at (s + 1/2) / nspec across y (periodic images included)."""
    raw = []
    for s_ in range(nspec):
        c = (s_ + 0.5) / nspec
        b = sum(np.exp(-((y - c + sh) / width) ** 2) for sh in (-1.0, 0.0, 1.0))
        raw.append(b + 1e-3)
    tot = sum(raw)
    return [r / tot for r in raw]


def kelvin_helmholtz(n=256, box=64, seed=20260102, gamma=5.0 / 3.0, steps=100, nspec=0) -> Problem:
    """Periodic shear layer: rho=2, u_x=+0.5 in |y-0.5|<0.25; rho=1, u_x=-0.5 outside;
    p=2.5; u_y = 0.01 (2r-1) with r ~ U[0,1) per cell; optionally nspec passive
    species in smooth bands across y (mass fractions summing to 1)."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    x, y, z = cell_centres(nn)
    rng = np.random.default_rng(seed)
    r = rng.random((nn[2], nn[1], nn[0]))
    inside = np.abs(y - 0.5) < 0.25
    rho = np.where(inside, 2.0, 1.0)
    u = np.where(inside, 0.5, -0.5)
    v = 0.01 * (2.0 * r - 1.0)
    U = conserved(gamma, rho, u, v, 0.0, 2.5, species_bands(y, nspec) if nspec else None)
    be = (box, box, box) if np.isscalar(box) else tuple(box)
    return Problem("kh", nn, gamma, U, regular_boxes(nn, be), cfl=0.5, steps=steps, nspec=nspec)


def material_species(mask, y, nspec: int):
    """nspec mass fractions for a two-material problem: species 0 marks the
    material where ``mask`` holds, species 1 the other one (sharp interfaces,
    carried by the contact), any further species smooth bands across y; they
    sum to 1."""
    if nspec <= 0:
        return None
    m = np.asarray(mask, dtype=np.float64)
    if nspec == 1:
        return [m]
    if nspec == 2:
        return [m, 1.0 - m]
    bands = species_bands(y, nspec - 2)
    return [0.8 * m, 0.8 * (1.0 - m)] + [0.2 * b for b in bands]


def rayleigh_taylor(n=384, seed=20260103, box_seed=None, gamma=1.4, steps=200, boxes=None, nspec=0) -> Problem:
    """Heavy over light in g_z = -1: rho=2 for z>0.5 else 1, p = 2.5 - rho (z-0.5),
    u_z = 0.01 (2r-1) (1+cos(4 pi (z-0.5)))/2 for |z-0.5| < 0.25; periodic x, y,
    reflecting z; boxes from seeded hierarchical compositions; optionally
    nspec passive species marking the two fluids (material_species)."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    x, y, z = cell_centres(nn)
    rng = np.random.default_rng(seed)
    r = rng.random((nn[2], nn[1], nn[0]))
    rho = np.where(z > 0.5, 2.0, 1.0)
    p = 2.5 - rho * (z - 0.5)
    window = np.abs(z - 0.5) < 0.25
    w = np.where(window, 0.01 * (2.0 * r - 1.0) * 0.5 * (1.0 + np.cos(4.0 * np.pi * (z - 0.5))), 0.0)
    U = conserved(gamma, rho, 0.0, 0.0, w, p, material_species(z > 0.5, y, nspec))
    if boxes is None:
        boxes = uneven_boxes(nn, seed if box_seed is None else box_seed)
    return Problem("rt", nn, gamma, U, boxes, (BC_PERIODIC, BC_PERIODIC, BC_REFLECT),
                   (BC_PERIODIC, BC_PERIODIC, BC_REFLECT), cfl=0.5, grav_z=-1.0, steps=steps, nspec=nspec)


def _fourier_field(rng: np.random.Generator, x, y, z, modes=8):
    """Sum of `modes` seeded modes a_m sin(2 pi k_m . x + phase_m), k_m in
    {-2..2}^3 without 0, normalised by the sum of the amplitudes."""
    ks = [k for k in np.ndindex(5, 5, 5) if k != (2, 2, 2)]
    amps = rng.uniform(0.5, 1.0, size=modes)
    phases = rng.uniform(0.0, 2.0 * np.pi, size=modes)
    picks = rng.integers(len(ks), size=modes)
    # sin(a + b + c) = Im(e^{ia} e^{ib} e^{ic}): each mode is a (z, y) plane
    # pattern times an x profile, so the sum is one matrix product (x, y, z
    # are the cell-centre grids of cell_centres, each varying along one axis)
    x1, y1, z1 = x[0, 0, :], y[0, :, 0], z[:, 0, 0]
    zy = np.empty((z1.size * y1.size, 2 * modes))
    xp = np.empty((2 * modes, x1.size))
    for m in range(modes):
        kx, ky, kz = (c - 2 for c in ks[int(picks[m])])
        ex = np.exp(1j * (2.0 * np.pi * kx * x1 + phases[m]))
        p = amps[m] * (np.exp(1j * (2.0 * np.pi * kz * z1))[:, None] * np.exp(1j * (2.0 * np.pi * ky * y1))[None, :])
        zy[:, 2 * m] = p.real.ravel()
        zy[:, 2 * m + 1] = p.imag.ravel()
        xp[2 * m] = ex.imag
        xp[2 * m + 1] = ex.real
    f = (zy @ xp).reshape(z1.size, y1.size, x1.size)
    return f / amps.sum()


SERVING_SIZES = (32, 48, 64, 96, 128)


def serving_request(seed: int, n: Optional[int] = None, gamma=1.4, steps=50, nspec=0) -> Problem:
    """One serving request: a periodic N^3 box with a smooth random state
    (rho = 1 + 0.1 f, p = 1 + 0.1 f, u_d = 0.3 sqrt(gamma) f; 8 Fourier modes
    each), optionally with nspec smooth species bands across y."""
    rng = np.random.default_rng(seed)
    if n is None:
        n = SERVING_SIZES[int(rng.integers(len(SERVING_SIZES)))]
    nn = (n, n, n)
    x, y, z = cell_centres(nn)
    rho = 1.0 + 0.1 * _fourier_field(rng, x, y, z)
    p = 1.0 + 0.1 * _fourier_field(rng, x, y, z)
    a = 0.3 * math.sqrt(gamma)
    u = a * _fourier_field(rng, x, y, z)
    v = a * _fourier_field(rng, x, y, z)
    w = a * _fourier_field(rng, x, y, z)
    U = conserved(gamma, rho, u, v, w, p, species_bands(y, nspec) if nspec else None)
    return Problem(f"serve{n}", nn, gamma, U, [((0, 0, 0), (n - 1, n - 1, n - 1))], cfl=0.5, steps=steps,
                   nspec=nspec)


def smooth_wave(n=32, gamma=1.4, box=None, amp=0.2) -> Problem:
    """rho = 1 + amp sin(2 pi (x+y+z)), u=v=w=1, p=1, periodic (advected entropy wave)."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    x, y, z = cell_centres(nn)
    rho = 1.0 + amp * np.sin(2.0 * np.pi * (x + y + z))
    U = conserved(gamma, rho, 1.0, 1.0, 1.0, 1.0)
    be = box or nn
    if np.isscalar(be):
        be = (be, be, be)
    return Problem("wave", nn, gamma, U, regular_boxes(nn, be), cfl=0.5)


def uniform(n=16, gamma=1.4, rho=1.3, vel=(0.3, -0.2, 0.1), p=0.9, box=None, bc=BC_PERIODIC,
            grav_z=0.0) -> Problem:
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    U = conserved(gamma, np.full((nn[2], nn[1], nn[0]), rho), vel[0], vel[1], vel[2], p)
    be = box or nn
    if np.isscalar(be):
        be = (be, be, be)
    return Problem("uniform", nn, gamma, U, regular_boxes(nn, be), (bc,) * 3, (bc,) * 3, grav_z=grav_z)


def cloud_wind(n=256, box=64, fine_box=32, fine_region=None, gamma=5.0 / 3.0, steps=100, nspec=0) -> Problem:
    """Dense cloud (rho 10, radius 0.1, at rest, pressure-matched p=1) in a Mach-2
    wind (rho 1, p 1, u_x = 2 sqrt(gamma)); inflow x-lo, outflow x-hi, periodic y, z.
    Two levels: the fine level (ratio 2) covers coarse cells ``fine_region``
    (default: the central half of the domain).  Optionally nspec passive
    species mark cloud and wind material (material_species); the inflow
    carries the wind's mass fractions."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    wind = 2.0 * math.sqrt(gamma)

    def state(x, y, z):
        r2 = (x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2
        inc = r2 < 0.01
        rho = np.where(inc, 10.0, 1.0)
        u = np.where(inc, 0.0, wind)
        return conserved(gamma, rho, u, 0.0, 0.0, 1.0, material_species(inc, y, nspec))

    x, y, z = cell_centres(nn)
    U = state(x, y, z)
    if fine_region is None:
        fine_region = (tuple(v // 4 for v in nn), tuple(3 * v // 4 for v in nn))
    clo, chi = fine_region
    flo = tuple(2 * c for c in clo)
    fn = tuple(2 * (chi[d] - clo[d]) for d in range(3))
    nf = tuple(2 * v for v in nn)
    # fine cell centres: (i + 0.5) / (2 n)
    axes = [(np.arange(flo[d], flo[d] + fn[d], dtype=np.float64) + 0.5) / nf[d] for d in range(3)]
    zf, yf, xf = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    Uf = state(xf, yf, zf)
    be = (box, box, box) if np.isscalar(box) else tuple(box)
    fbe = (fine_box,) * 3 if np.isscalar(fine_box) else tuple(fine_box)
    prob = Problem("cloud", nn, gamma, U, regular_boxes(nn, be),
                   (BC_INFLOW, BC_PERIODIC, BC_PERIODIC), (BC_OUTFLOW, BC_PERIODIC, BC_PERIODIC),
                   cfl=0.5, inflow=(1.0, wind, 0.0, 0.0, 1.0), steps=steps, nspec=nspec)
    if nspec:
        # the wind's fractions at the inflow face (y = 0.5 for the bands)
        prob.inflow_X = tuple(float(np.asarray(a).ravel()[0])
                              for a in material_species(np.zeros(1, bool), np.full(1, 0.5), nspec))
    prob.fine_boxes = regular_boxes(fn, fbe, origin=flo)
    prob.U0_fine = Uf
    prob.fine_lo = flo
    return prob


def two_clouds(n=256, box=64, fine_box=32, patches=None, gamma=5.0 / 3.0, steps=100, nspec=0) -> Problem:
    """Two dense clouds (rho 10, radius 0.1, at rest, p = 1) at x = 0.3 and
    x = 0.7 of a Mach-2 wind along x (the cloud problem's physics), each
    refined by its own fine patch: a fine level of two rectangles (section 3,
    figure 1: fine boxes over separate regions of the coarse level).
    ``patches``: coarse cell ranges ((lo), (hi)) half-open, default two cubes
    of n/4 cells around the clouds."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    wind = 2.0 * math.sqrt(gamma)
    centres = ((0.3, 0.5, 0.5), (0.7, 0.5, 0.5))

    def state(x, y, z):
        inc = np.zeros(np.shape(x), dtype=bool)
        for cx, cy, cz in centres:
            inc |= (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 < 0.01
        rho = np.where(inc, 10.0, 1.0)
        u = np.where(inc, 0.0, wind)
        return conserved(gamma, rho, u, 0.0, 0.0, 1.0, material_species(inc, y, nspec))

    x, y, z = cell_centres(nn)
    be = (box, box, box) if np.isscalar(box) else tuple(box)
    fbe = (fine_box,) * 3 if np.isscalar(fine_box) else tuple(fine_box)
    prob = Problem("two_clouds", nn, gamma, state(x, y, z), regular_boxes(nn, be),
                   (BC_INFLOW, BC_PERIODIC, BC_PERIODIC), (BC_OUTFLOW, BC_PERIODIC, BC_PERIODIC),
                   cfl=0.5, inflow=(1.0, wind, 0.0, 0.0, 1.0), steps=steps, nspec=nspec)
    if nspec:
        prob.inflow_X = tuple(float(np.asarray(a).ravel()[0])
                              for a in material_species(np.zeros(1, bool), np.full(1, 0.5), nspec))
    if patches is None:
        q = nn[0] // 4
        patches = []
        for cx, cy, cz in centres:
            c = (int(round(cx * nn[0])), int(round(cy * nn[1])), int(round(cz * nn[2])))
            patches.append((tuple(c[d] - q // 2 for d in range(3)), tuple(c[d] + q // 2 for d in range(3))))
    prob.fine_patches, prob.fine_boxes = refine_patches(patches, nn, fbe, state)
    return prob


def refine_patches(patches, n, fine_edge, state):
    """Fine patches (ratio 2) over half-open coarse ranges, their initial states
    from ``state(x, y, z)`` at fine cell centres, and the fine boxes tiling them."""
    nf = tuple(2 * v for v in n)
    pats, boxes = [], []
    for clo, chi in patches:
        flo = tuple(2 * c for c in clo)
        fn = tuple(2 * (chi[d] - clo[d]) for d in range(3))
        axes = [(np.arange(flo[d], flo[d] + fn[d], dtype=np.float64) + 0.5) / nf[d] for d in range(3)]
        zf, yf, xf = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        pats.append((flo, state(xf, yf, zf)))
        boxes += regular_boxes(fn, fine_edge, origin=flo)
    return pats, boxes


def patch_list(prob: Problem):
    """The fine patches of a two-level problem as (fine index lo, state)."""
    if prob.fine_patches:
        return [(tuple(lo), U) for lo, U in prob.fine_patches]
    return [(tuple(prob.fine_lo), prob.U0_fine)]


def patch_of_box(patches, box: Box) -> int:
    """Index of the patch whose cells hold a fine box."""
    lo, hi = box
    for q, (plo, U) in enumerate(patches):
        pn = U.shape[1:][::-1]
        if all(plo[d] <= lo[d] and hi[d] < plo[d] + pn[d] for d in range(3)):
            return q
    raise ValueError(f"fine box {box} lies in no patch")


# ----------------------------------------------------------------------------
# per-box views
# ----------------------------------------------------------------------------

def box_shape(box: Box) -> Tuple[int, int, int]:
    lo, hi = box
    return tuple(hi[d] - lo[d] + 1 for d in range(3))


def grown_fab(U: np.ndarray, box: Box, origin=(0, 0, 0), fill=np.nan) -> np.ndarray:
    """Grown (5, nz+8, ny+8, nx+8) array of one box with valid cells copied from the
    level array ``U`` (whose [..., 0, 0, 0] is index ``origin``); ghosts = ``fill``."""
    lo, hi = box
    nx, ny, nz = box_shape(box)
    g = NGHOST
    out = np.full((U.shape[0], nz + 2 * g, ny + 2 * g, nx + 2 * g), fill, dtype=np.float64)
    sl = (slice(None),
          slice(lo[2] - origin[2], hi[2] + 1 - origin[2]),
          slice(lo[1] - origin[1], hi[1] + 1 - origin[1]),
          slice(lo[0] - origin[0], hi[0] + 1 - origin[0]))
    out[:, g:g + nz, g:g + ny, g:g + nx] = U[sl]
    return out


def gather_valid(fabs: Sequence[np.ndarray], boxes: Sequence[Box], n, origin=(0, 0, 0)) -> np.ndarray:
    """Inverse of grown_fab over a box list: assemble the level's valid cells."""
    out = np.full((np.asarray(fabs[0]).shape[0], n[2], n[1], n[0]), np.nan, dtype=np.float64)
    g = NGHOST
    for f, b in zip(fabs, boxes):
        lo, hi = b
        nx, ny, nz = box_shape(b)
        out[:, lo[2] - origin[2]:hi[2] + 1 - origin[2], lo[1] - origin[1]:hi[1] + 1 - origin[1],
            lo[0] - origin[0]:hi[0] + 1 - origin[0]] = np.asarray(f)[:, g:g + nz, g:g + ny, g:g + nx]
    return out
