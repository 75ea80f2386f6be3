// gfx950 kernels of the unsplit CTU/PPM advance, one kernel per stage.
//
// Work decomposition: the cell and face stages run over "march" units: 256
// consecutive items (cells or faces, i fastest) of one (x, y) plane of a box's
// region, visited for a run of consecutive z planes.  Lanes touch consecutive
// doubles of every SoA array, and a z neighbour a stencil reads was read by
// the same block one or two planes earlier, so it comes from cache rather than
// HBM.  The same kernels serve the per-box form (one launch per box over that
// box's units) and the batched form (one persistent launch over the units of
// all boxes of all problems in a step).  Blocks walk their units with an
// XCD-aware mapping: workgroups are dispatched round-robin over the 8 XCDs, so
// block b runs on XCD b%8 and takes a contiguous eighth of the unit list, which
// keeps the y neighbours of a unit (the adjacent units) in the same XCD's L2.
// Ghost fills run over 256-item chunks of their copy tags.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ctuppm_internal.h"
#include "hydro_device.h"

namespace ctu {

namespace {

// Device arrays are accessed through global-address-space pointers, so loads
// and stores compile to global (not flat) memory instructions: their
// completion is tracked by the vector-memory counter alone and a uniform base
// goes in scalar registers.
using gdbl = __attribute__((address_space(1))) double;
CTU_DEV gdbl* gp(double* p) { return (gdbl*)p; }
// LDS doubles, volatile: values a thread parks there are re-read from LDS
// (not kept in registers), through ds_* instructions.
using ldbl = __attribute__((address_space(3))) volatile double;
// The problem record as the stage kernels read it: through the constant
// address space, since it is the same for a whole block and no kernel writes
// the fields it reads this way (counters and the signal-speed maxima are
// updated through the ordinary pointer).  The reads become scalar loads into
// scalar registers; as flat loads they would also make a wave wait for its
// earlier stores.
using CProb = __attribute__((address_space(4))) const ProbDev;
CTU_DEV CProb* cprob(const ProbDev* P) { return (CProb*)P; }

template <class F>
CTU_DEV void for_each_chunk(int nchunks, F&& f) {
  const int per = gridDim.x >> 3;
  const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3;
  const int span = (nchunks + 7) >> 3;
  const int beg = xcd * span;
  const int end = beg + span < nchunks ? beg + span : nchunks;
  for (int c = beg + local; c < end; c += per) f(c);
}

// Segment of launch item c (block-uniform: a scalar scan over the kernel
// argument).
CTU_DEV int seg_of(const Segs& L, int c) {
  int s = 0;
  while (s + 1 < L.n && c >= L.beg[s + 1]) ++s;
  return s;
}

// The unit's record and box through restrict-qualified pointers: the
// kernels' stores then cannot alias them, so their fields stay in registers
// (without it the transverse kernel needs 30-40 more VGPRs).
template <class F>
CTU_DEV void unit_body(const March* __restrict__ w, const BoxRec* __restrict__ bx, int i, F&& f) {
  const March M = w[i];
  f(M, bx[M.box]);
}

// Visit the march units of a launch: f(unit, its box).
template <class F>
CTU_DEV void for_each_unit(const Segs& L, F&& f) {
  for_each_chunk(L.beg[L.n], [&](int c) {
    const int s = seg_of(L, c);
    unit_body((const March*)L.s[s].work, L.s[s].boxes, c - L.beg[s], f);
  });
}

// Visit the tag chunks of a launch: f(chunk, its segment).
template <class F>
CTU_DEV void for_each_tag_chunk(const Segs& L, F&& f) {
  for_each_chunk(L.beg[L.n], [&](int c) {
    const int s = seg_of(L, c);
    f(((const Chunk*)L.s[s].work)[c - L.beg[s]], L.s[s]);
  });
}

// Visit the (i, j, k) items of a march unit in region `kind`; f(i, j, k) is
// called for the lane's (i, j) at every plane of the unit.  Lanes past the
// plane's end skip all planes (no barrier inside f).
template <class F>
CTU_DEV void march(int kind, const BoxRec& B, const March& M, F&& f) {
  int org[3], ext[3];
  region_of(kind, B.n, org, ext);
  const int t = M.start + threadIdx.x;
  if (t >= M.end) return;
  const int i = t % ext[0] + org[0];
  const int j = t / ext[0] + org[1];
  for (int k = M.z0; k < M.z1; ++k) f(i, j, k);
}

// Geometry of one box: grown arrays (ghosts -4..n+3) and halo-1 arrays (-1..n);
// ns passive species follow the five hydro components of every array.
struct Geo {
  int gx, gplane, gcomp;
  int hx, hplane, hcomp;
  int ns, nv;
  CTU_DEV Geo(const int n[3], int nspec) {
    ns = nspec;
    nv = kNV + nspec;
    gx = n[0] + 2 * kNG;
    gplane = gx * (n[1] + 2 * kNG);
    gcomp = gplane * (n[2] + 2 * kNG);
    hx = n[0] + 2;
    hplane = h1_plane(n);
    hcomp = hplane * (n[2] + 2);
  }
  CTU_DEV int g(int i, int j, int k) const { return (k + kNG) * gplane + (j + kNG) * gx + (i + kNG); }
  CTU_DEV int h(int i, int j, int k) const { return (k + 1) * hplane + (j + 1) * hx + (i + 1); }
  CTU_DEV int gstride(int d) const { return d == 0 ? 1 : (d == 1 ? gx : gplane); }
  CTU_DEV int hstride(int d) const { return d == 0 ? 1 : (d == 1 ? hx : hplane); }
  // scratch sub-arrays: q, phi, then 18 arrays of nv components (ql[3], qr[3],
  // fn[3], f1[6], ff[3]); offsets in 64 bits (a 256^3 box with 16 species
  // spans more than 2^31 doubles)
  CTU_DEV gdbl* h1arr(double* s, int a) const {
    return gp(s) + (long long)(kNV + 1 + ns) * gcomp + (1 + (long long)nv * a) * hcomp;
  }
  CTU_DEV gdbl* q(double* s) const { return gp(s); }
  CTU_DEV gdbl* phi(double* s) const { return gp(s) + (long long)(kNV + 1 + ns) * gcomp; }
  // ql(d) is indexed by face (element f: the left state of face f along d)
  // but stored at the cell below the face, f - 1, so the tracing of a cell
  // writes its own, line-aligned index; the pointer is offset accordingly.
  CTU_DEV gdbl* ql(double* s, int d) const { return h1arr(s, d) - hstride(d); }
  CTU_DEV gdbl* qr(double* s, int d) const { return h1arr(s, 3 + d); }
  CTU_DEV gdbl* fn(double* s, int d) const { return h1arr(s, 6 + d); }
  CTU_DEV gdbl* f1(double* s, int p) const { return h1arr(s, 9 + p); }
  CTU_DEV gdbl* ff(double* s, int d) const { return h1arr(s, 15 + d); }
};

CTU_DEV void count(unsigned long long* c, unsigned long long v) {
  if (v) atomicAdd(c, v);
}

// Interface flux of the Riemann solver RS (0 HLLC, 1 two-shock), permuted order.
template <int RS>
CTU_DEV void rflux(const double L[5], const double R[5], CProb* P, double F[5], Wave& W) {
  if (RS == 1) twoshock(L, R, P->gamma, P->rgm1, P->small_dens, P->small_pres, F, W);
  else hllc(L, R, P->gamma, P->rgm1, F, W);
}

// The state array `arr` of a box (current fab, Runge-Kutta stage fab, or the
// fab that receives the new state).
CTU_DEV double* state_arr(const BoxRec& B, int arr) {
  const int cur = cprob(B.P)->cur;
  switch (arr) {
    case kArrW0: return B.W[0];
    case kArrW1: return B.W[1];
    case kArrNext: return B.U[cur ^ 1];
    default: return B.U[cur];
  }
}

// ---------------------------------------------------------------- ghost fill

__global__ __launch_bounds__(kBlock) void k_fill(const Segs L, int arr) {
  for_each_tag_chunk(L, [&](const Chunk& ch, const Seg& S) {
    const FillTag T = ((const FillTag*)S.tags)[ch.box];
    const int t = ch.start + threadIdx.x;
    if (t >= T.ext[0] * T.ext[1] * T.ext[2]) return;
    const int i = T.lo[0] + t % T.ext[0];
    const int r = t / T.ext[0];
    const int j = T.lo[1] + r % T.ext[1];
    const int k = T.lo[2] + r / T.ext[1];
    const BoxRec& D = S.boxes[T.dst];
    const BoxRec& Sb = S.boxes[T.src];
    const Geo gd(D.n, D.ns), gs(Sb.n, Sb.ns);
    const gdbl* __restrict__ src = gp(state_arr(Sb, arr));
    gdbl* __restrict__ dst = gp(state_arr(D, arr));
    const int si = gs.g(i + T.off[0], j + T.off[1], k + T.off[2]);
    const int di = gd.g(i, j, k);
#pragma unroll
    for (int m = 0; m < kNV; ++m) dst[m * gd.gcomp + di] = src[m * gs.gcomp + si];
    for (int m = kNV; m < gd.nv; ++m) dst[m * gd.gcomp + di] = src[m * gs.gcomp + si];
  });
}

// Physical boundary of one direction D: outflow copies the edge cell, reflect
// mirrors with the normal momentum negated, inflow writes a fixed state.
template <int D>
__global__ __launch_bounds__(kBlock) void k_bc(const Segs L, int arr) {
  for_each_tag_chunk(L, [&](const Chunk& ch, const Seg& S) {
    const BcTag& T = ((const BcTag*)S.tags)[ch.box];  // by reference: the inflow state is indexed at run time
    const int t = ch.start + threadIdx.x;
    if (t >= T.ext[0] * T.ext[1] * T.ext[2]) return;
    int x[3];
    x[0] = T.lo[0] + t % T.ext[0];
    const int r = t / T.ext[0];
    x[1] = T.lo[1] + r % T.ext[1];
    x[2] = T.lo[2] + r / T.ext[1];
    const BoxRec& B = S.boxes[T.box];
    const Geo g(B.n, B.ns);
    gdbl* __restrict__ U = gp(state_arr(B, arr));
    const int di = g.g(x[0], x[1], x[2]);
    if (T.bc == 3) {
      for (int m = 0; m < g.nv; ++m) U[m * g.gcomp + di] = T.inflow[m];
      return;
    }
    const int X = B.lo[D] + x[D];  // level index of the ghost cell
    int Xs;
    if (T.bc == 1) Xs = T.side == 0 ? T.dom_lo : T.dom_hi;
    else Xs = T.side == 0 ? 2 * T.dom_lo - X - 1 : 2 * T.dom_hi + 1 - X;
    int s[3] = {x[0], x[1], x[2]};
    s[D] = Xs - B.lo[D];
    const int si = g.g(s[0], s[1], s[2]);
#pragma unroll
    for (int m = 0; m < kNV; ++m) {
      double v = U[m * g.gcomp + si];
      if (T.bc == 2 && m == 1 + D) v = -v;
      U[m * g.gcomp + di] = v;
    }
    for (int m = kNV; m < g.nv; ++m) U[m * g.gcomp + di] = U[m * g.gcomp + si];
  });
}

// ------------------------------------------------------- cons -> prim + CFL

CTU_DEV double block_max(double v, double* lds) {
  for (int off = 32; off > 0; off >>= 1) v = dmax(v, __shfl_xor(v, off, 64));
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double r = lds[0];
  for (int q = 1; q < kBlock / 64; ++q) r = dmax(r, lds[q]);
  __syncthreads();
  return r;
}

CTU_DEV void flush_max(ProbDev* P, double m, double* lds) {
  const double bm = block_max(m, lds);
  if (threadIdx.x == 0) atomicMax(&P->smax[blockIdx.x % kSlots][0], (unsigned long long)__double_as_longlong(bm));
}

// Primitive state (rho, u, v, w, p, c) with floors (WQ: stored for every
// grown cell) and the signal speed max_d (|u_d| + c) / dx_d of the valid
// cells (CFL: reduced per problem by wave shuffles, LDS and a 64-bit atomic
// max on the bit pattern; non-negative doubles order like unsigned integers,
// so the max is exact and order-free).  The batched forms do both in one pass;
// the per-box form, whose boxes share one scratch, reduces first (CFL only)
// and stores q box by box after dt is known.
template <bool WQ, bool CFL>
__global__ __launch_bounds__(kBlock) void k_c2p(const Segs L, int arr) {
  __shared__ double lds[kBlock / 64];
  double smax = 0.0;
  ProbDev* curP = nullptr;
  for_each_unit(L, [&](const March& M, const BoxRec& B) {
    ProbDev* P = B.P;
    if (P != curP) {  // block-uniform: flush the running max of the previous problem
      if (CFL && curP) flush_max(curP, smax, lds);
      smax = 0.0;
      curP = P;
    }
    const Geo g(B.n, B.ns);
    const gdbl* __restrict__ U = gp(state_arr(B, arr));
    gdbl* __restrict__ q = g.q(B.scr);
    CProb* Pc = cprob(P);
    const bool summed = Pc->scheme != 0;
    const double gamma = Pc->gamma, gm1 = Pc->gm1, sd = Pc->small_dens, sp = Pc->small_pres;
    const double rdx = Pc->rdx[0], rdy = Pc->rdx[1], rdz = Pc->rdx[2];
    unsigned long long hd = 0, hp = 0;
    march(WQ ? kGrown : kValid, B, M, [&](int i, int j, int k) {
      const int o = g.g(i, j, k);
      double rho = U[o];
      if (rho < sd) { rho = sd; ++hd; }
      const double u = U[g.gcomp + o] / rho, v = U[2 * g.gcomp + o] / rho, w = U[3 * g.gcomp + o] / rho;
      const double ke = 0.5 * rho * ((u * u + v * v) + w * w);
      double p = gm1 * (U[4 * g.gcomp + o] - ke);
      if (p < sp) { p = sp; ++hp; }
      const double cs = sqrt(gamma * p / rho);
      if (WQ) {
        q[o] = rho;
        q[g.gcomp + o] = u;
        q[2 * g.gcomp + o] = v;
        q[3 * g.gcomp + o] = w;
        q[4 * g.gcomp + o] = p;
        q[5 * g.gcomp + o] = cs;
        for (int is = 0; is < g.ns; ++is) q[(6 + is) * g.gcomp + o] = U[(kNV + is) * g.gcomp + o] / rho;
      }
      if (CFL && i >= 0 && i < B.n[0] && j >= 0 && j < B.n[1] && k >= 0 && k < B.n[2]) {
        const double sx = (fabs(u) + cs) * rdx;
        const double sy = (fabs(v) + cs) * rdy;
        const double sz = (fabs(w) + cs) * rdz;
        smax = dmax(smax, summed ? (sx + sy) + sz : dmax(sx, dmax(sy, sz)));
      }
    });
    if (WQ) {
      count(&P->cnt[0], hd);
      count(&P->cnt[1], hp);
    }
  });
  if (CFL && curP) flush_max(curP, smax, lds);
}

// The step's dt and its per-direction factors (the same roundings as writing
// them out where they are used).
CTU_DEV void set_dt(ProbDev* P, double dt) {
  P->dt = dt;
  for (int d = 0; d < 3; ++d) {
    const double r = dt / P->dx[d];
    P->dtdx[d] = r;
    P->dt3dx[d] = r / 3.0;
    P->dt2dx[d] = 0.5 * r;
  }
}

__global__ void k_dt(const Segs L) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L.n) return;
  ProbDev* P = L.s[t].P;
  unsigned long long bits = 0ull;
  for (int q = 0; q < kSlots; ++q) {
    bits = P->smax[q][0] > bits ? P->smax[q][0] : bits;
    P->smax[q][0] = 0ull;
  }
  const double s = __longlong_as_double((long long)bits);
  set_dt(P, P->fixed_dt > 0.0 ? P->fixed_dt : P->cfl / s);
}

// A caller's dt (a device double) for the next advance of a problem: the
// coarse level takes it, a fine level half of it.
__global__ void k_set_dt(ProbDev* Pc, ProbDev* Pf, const double* dt) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double v = *dt;
  set_dt(Pc, v);
  if (Pf) set_dt(Pf, 0.5 * v);
}

// Commit a step (flip the current fab, count it).  A guarded step whose
// failure count grew is not committed: the old state stays current (it is
// intact in the other fab), the rejection is counted and mirrored to the
// host-mapped flag the host reads without synchronising.
__global__ void k_flip(const Segs L, int guard) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L.n) return;
  ProbDev* P = L.s[t].P;
  const unsigned long long nf = P->cnt[4];
  if (guard && nf != P->fail_mark) {
    P->rejected += 1;
    if (P->fail_step == P->nsteps) P->fail_step = -1;  // the test hook fires once
    if (P->hflag) __hip_atomic_store(P->hflag, P->rejected, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  } else {
    P->cur ^= 1;
    P->nsteps += 1;
  }
  P->fail_mark = nf;
}

// ---------------------------------------------------------------- flattening

// CW84 shock indicator of a cell from the pressures two cells either side of
// it (pm2, pm1, pp1, pp2) and the normal velocities of its neighbours.
CTU_DEV double shock_ind(double pm2, double pm1, double pp1, double pp2, double um1, double up1) {
  const double dp1 = pp1 - pm1;
  const double dp2 = pp2 - pm2;
  double f = 0.0;
  if (fabs(dp1) > 0.33 * dmin(pp1, pm1) && um1 - up1 > 0.0)
    f = dmin(1.0, dmax(0.0, 10.0 * (fabs(dp1) / dmax(fabs(dp2), 1e-300) - 0.75)));
  return f;
}

// Flattening coefficient of the cell at grown offset o: the minimum over the
// directions of 1 - max(shock indicator here, at the neighbour on the side of
// lower pressure).  Every pressure and velocity either neighbour's indicator
// could need is loaded before any arithmetic, so a wave waits for memory once.
CTU_DEV double flatten_cell(const Geo& g, const gdbl* __restrict__ q, int o) {
  const gdbl* __restrict__ p = q + 4 * g.gcomp;
  double pv[3][7], uv[3][5];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int st = g.gstride(d);
    const gdbl* __restrict__ un = q + (1 + d) * g.gcomp;
#pragma unroll
    for (int t = 0; t < 7; ++t) pv[d][t] = p[o + (t - 3) * st];
#pragma unroll
    for (int t = 0; t < 5; ++t) uv[d][t] = un[o + (t - 2) * st];
  }
  double phi = 1.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double* v = pv[d];
    const double* u = uv[d];
    const int c = (v[4] - v[2]) > 0.0 ? 2 : 4;  // the neighbour on the side of lower pressure
    const double f0 = shock_ind(v[1], v[2], v[4], v[5], u[1], u[3]);
    const double f1 = shock_ind(v[c - 2], v[c - 1], v[c + 1], v[c + 2], u[c - 2], u[c]);
    const double fd = dmax(f0, f1);
    const double w = 1.0 - fd;
    phi = d == 0 ? w : dmin(phi, w);
  }
  return phi;
}

__global__ __launch_bounds__(kBlock) void k_flatten(const Segs L) {
  for_each_unit(L, [&](const March& M, const BoxRec& B) {
    const Geo g(B.n, B.ns);
    const gdbl* __restrict__ q = g.q(B.scr);
    gdbl* __restrict__ phiout = g.phi(B.scr);
    march(kCells1, B, M, [&](int i, int j, int k) { phiout[g.h(i, j, k)] = flatten_cell(g, q, g.g(i, j, k)); });
  });
}

// ------------------------------------------------------ PPM + tracing along D

// The same with streaming (non-temporal) stores, for fluxes that only a later
// launch reads: they do not displace lines the current launch reads again.
template <int D>
CTU_DEV void store_flux_nt(gdbl* __restrict__ F, int hcomp, int o, const double f[5]) {
  __builtin_nontemporal_store(f[0], &F[o]);
  __builtin_nontemporal_store(f[1], &F[(1 + D) * hcomp + o]);
  __builtin_nontemporal_store(f[2], &F[(1 + (D + 1) % 3) * hcomp + o]);
  __builtin_nontemporal_store(f[3], &F[(1 + (D + 2) % 3) * hcomp + o]);
  __builtin_nontemporal_store(f[4], &F[4 * hcomp + o]);
}
template <int D>
CTU_DEV void store_flux(gdbl* __restrict__ F, int hcomp, int o, const double f[5]) {
  F[o] = f[0];
  F[(1 + D) * hcomp + o] = f[1];
  F[(1 + (D + 1) % 3) * hcomp + o] = f[2];
  F[(1 + (D + 2) % 3) * hcomp + o] = f[3];
  F[4 * hcomp + o] = f[4];
}

// Tracing of one cell (of -1..n) along D: parabolas of the five permuted
// primitives, tracing to both faces, floors and the gravity predictor; the
// left state of the upper face and the right state of the lower face are
// stored for faces 0..n.  It comes in pieces -- the loads of the stencils,
// the parabolas, the two traced states, the stores -- so that a kernel
// tracing several directions can order them: a wave with stores in flight
// that waits for a later load waits for those stores as well (one counter
// covers both), so the merged kernel issues all its global stores after its
// last load.
struct Stencil {
  double sv[5][5];  // the five permuted primitives at offsets -2..2 along D
  double cs;        // the sound speed of the cell
};

template <int D, bool CS = true>
CTU_DEV void trace_load(const Geo& g, const gdbl* __restrict__ q, int o, Stencil& S) {
  constexpr int comp[5] = {0, 1 + D, 1 + (D + 1) % 3, 1 + (D + 2) % 3, 4};
  const int st = g.gstride(D);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const gdbl* a = q + comp[m] * g.gcomp + o;
#pragma unroll
    for (int t = 0; t < 5; ++t) S.sv[m][t] = a[(t - 2) * st];
  }
  if (CS) S.cs = q[5 * g.gcomp + o];
}

// The parabolas of the five permuted primitives of a cell along D.
template <int D, int LIM>
CTU_DEV void trace_parab(CProb* P, const Stencil& S, double phi, Parab par[5]) {
  double eta = 0.0;
  if (LIM & 2)  // contact steepening weight from the density and the neighbours' pressures
    eta = steep_eta(S.sv[0][0], S.sv[0][1], S.sv[0][2], S.sv[0][3], S.sv[0][4], S.sv[4][1], S.sv[4][3], P->gamma);
#pragma unroll
  for (int m = 0; m < 5; ++m)
    par[m] = ppm_l<LIM>(S.sv[m][0], S.sv[m][1], S.sv[m][2], S.sv[m][3], S.sv[m][4], phi, m == 0 ? eta : 0.0);
}

// The left state of the upper face (UP) or the right state of the lower face,
// floors and gravity predictor applied.  Both are computed for every cell of
// -1..n; floors are counted only on the states of faces 0..n (xd is the
// cell's index along D, nd the box's extent).
template <int D, bool UP>
CTU_DEV void trace_face(CProb* P, const Parab par[5], double rho, double un, double cs, int xd, int nd,
                        double v[5], unsigned long long& floors) {
  constexpr int zpos = 1 + (2 - D + 3) % 3;  // permuted slot of the z velocity
  const double dtdx = P->dtdx[D];
  const unsigned long long f = UP ? xd <= nd - 1 : xd >= 0;
  if (UP) trace_up(par, rho, un, cs, dtdx, v);
  else trace_dn(par, rho, un, cs, dtdx, v);
  if (v[0] < P->small_dens) { v[0] = P->small_dens; floors += f; }
  if (v[4] < P->small_pres) { v[4] = P->small_pres; floors += f; }
  if (P->grav_z != 0.0) v[zpos] = v[zpos] + 0.5 * P->dt * P->grav_z;
}

// Stores of the cell's two traced states, unconditionally: the upper state
// of cell n (a face n + 1) and the lower state of cell -1 (a face -1) land in
// their own slots of the halo-1 arrays and are never read; storing them
// lets a wave write whole, line-aligned runs of every array.  The stores
// stream (non-temporal): only later launches read the states.
template <int D>
CTU_DEV void trace_store(const BoxRec& B, const Geo& g, int oh, const double up[5], const double dn[5]) {
  gdbl* __restrict__ ql = g.ql(B.scr, D);
  gdbl* __restrict__ qr = g.qr(B.scr, D);
  const int sth = g.hstride(D);
#pragma unroll
  for (int m = 0; m < 5; ++m) __builtin_nontemporal_store(up[m], &ql[m * g.hcomp + oh + sth]);
#pragma unroll
  for (int m = 0; m < 5; ++m) __builtin_nontemporal_store(dn[m], &qr[m * g.hcomp + oh]);
}

// The species of the cell along D: parabolas with the hydro flattening,
// traced with the hydro wave speeds of the cell.  Stored unconditionally, as
// the hydro states (the unread slots of cells n and -1 keep the runs whole).
template <int D, int LIM>
CTU_DEV void trace_species(const BoxRec& B, const Geo& g, CProb* P, int o, int oh, double phi) {
  const gdbl* __restrict__ q = g.q(B.scr);
  gdbl* __restrict__ ql = g.ql(B.scr, D);
  gdbl* __restrict__ qr = g.qr(B.scr, D);
  const int st = g.gstride(D), sth = g.hstride(D);
  const double dtdx = P->dtdx[D];
  const double un = q[(1 + D) * g.gcomp + o], cs = q[5 * g.gcomp + o];
  const double lm = un - cs, l0 = un, lp = un + cs;
  const double sm = fabs(lm) * dtdx, s0 = fabs(l0) * dtdx, spp = fabs(lp) * dtdx;
  for (int is = 0; is < g.ns; ++is) {
    const gdbl* a = q + (6 + is) * g.gcomp + o;
    const Parab px = ppm_l<LIM>(a[-2 * st], a[-st], a[0], a[st], a[2 * st], phi);
    __builtin_nontemporal_store(species_up(px, lp, l0, spp, s0), &ql[(kNV + is) * g.hcomp + oh + sth]);
    __builtin_nontemporal_store(species_dn(px, lm, l0, sm, s0), &qr[(kNV + is) * g.hcomp + oh]);
  }
}

// The species of the cell along x, y and z at once (the merged kernels):
// TRACE = characteristic tracing with the hydro wave speeds of the cell, else
// the method-of-lines edge values.  A species' 13 stencil values are loaded
// before the stores of the previous species are issued, so no wave waits
// for its own stores to read the next species; every store is unconditional.
template <int LIM, bool TRACE>
CTU_DEV void species3(const BoxRec& B, const Geo& g, CProb* P, int o, int oh, double phi) {
  const gdbl* __restrict__ q = g.q(B.scr);
  const int st[3] = {g.gstride(0), g.gstride(1), g.gstride(2)};
  double un[3], cs = 0.0;
  if (TRACE) {
    cs = q[5 * g.gcomp + o];
#pragma unroll
    for (int d = 0; d < 3; ++d) un[d] = q[(1 + d) * g.gcomp + o];
  }
  // v[0] the cell; v[1 + 4d ..] the stencil neighbours -2, -1, +1, +2 along d
  auto load = [&](int is, double v[13]) {
    const gdbl* a = q + (6 + is) * g.gcomp + o;
    v[0] = a[0];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      v[1 + 4 * d] = a[-2 * st[d]]; v[2 + 4 * d] = a[-st[d]];
      v[3 + 4 * d] = a[st[d]]; v[4 + 4 * d] = a[2 * st[d]];
    }
  };
  double cur[13], nxt[13];
  load(0, cur);
#pragma unroll 1
  for (int is = 0; is < g.ns; ++is) {
    if (is + 1 < g.ns) load(is + 1, nxt);
    double up[3], dn[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const Parab px = ppm_l<LIM>(cur[1 + 4 * d], cur[2 + 4 * d], cur[0], cur[3 + 4 * d], cur[4 + 4 * d], phi);
      if (TRACE) {
        // the wave speeds of the cell along d, as the single-direction tracing
        const double dtdx = P->dtdx[d];
        const double lm = un[d] - cs, l0 = un[d], lp = un[d] + cs;
        up[d] = species_up(px, lp, l0, fabs(lp) * dtdx, fabs(l0) * dtdx);
        dn[d] = species_dn(px, lm, l0, fabs(lm) * dtdx, fabs(l0) * dtdx);
      } else {
        up[d] = px.aR;
        dn[d] = px.aL;
      }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      gdbl* __restrict__ ql = g.ql(B.scr, d);
      gdbl* __restrict__ qr = g.qr(B.scr, d);
      __builtin_nontemporal_store(up[d], &ql[(kNV + is) * g.hcomp + oh + g.hstride(d)]);
      __builtin_nontemporal_store(dn[d], &qr[(kNV + is) * g.hcomp + oh]);
    }
    if (is + 1 < g.ns) {
#pragma unroll
      for (int m = 0; m < 13; ++m) cur[m] = nxt[m];
    }
  }
}

template <int D, int LIM>
CTU_DEV void trace_cell(const BoxRec& B, const Geo& g, CProb* P, int i, int j, int k, double phi,
                        unsigned long long& floors) {
  const int x[3] = {i, j, k};
  const int o = g.g(i, j, k), oh = g.h(i, j, k);
  Stencil S;
  Parab par[5];
  double up[5], dn[5];
  trace_load<D>(g, g.q(B.scr), o, S);
  trace_parab<D, LIM>(P, S, phi, par);
  trace_face<D, true>(P, par, S.sv[0][2], S.sv[1][2], S.cs, x[D], B.n[D], up, floors);
  trace_face<D, false>(P, par, S.sv[0][2], S.sv[1][2], S.cs, x[D], B.n[D], dn, floors);
  trace_store<D>(B, g, oh, up, dn);
  if (g.ns > 0) trace_species<D, LIM>(B, g, P, o, oh, phi);
}

// One thread per cell of -1..n, tracing along D.
template <int D, int LIM>
__global__ __launch_bounds__(kBlock) void k_trace(const Segs L) {
  for_each_unit(L, [&](const March& M, const BoxRec& B) {
    const Geo g(B.n, B.ns);
    unsigned long long floors = 0;
    const gdbl* __restrict__ phiv = g.phi(B.scr);
    march(kCells1, B, M, [&](int i, int j, int k) {
      trace_cell<D, LIM>(B, g, cprob(B.P), i, j, k, phiv[g.h(i, j, k)], floors);
    });
    count(&B.P->cnt[2], floors);
  });
}

// One thread per cell of -1..n: the flattening coefficient (also stored, for
// stage dumps), then tracing along x, then y, then z, so the cell's
// primitives are read once for the flattening and the three directions (the
// separate kernels read them four times).  The traced states of x and y wait
// in LDS (each thread its own slots) until the loads of z have returned: a
// wave whose stores are still in flight waits for them as well when it waits
// for a later load, so every global store of the cell is issued after its
// last load.  Three waves per SIMD (the LDS allows four): the register
// budget that keeps the species loop from lowering the occupancy to two.
// spec = 0: the species are left to k_spec3.
template <int LIM>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_trace3(const Segs L, int spec) {
  // 40 KB: the up and dn states of x and y, [direction][component][thread];
  // volatile, so the compiler keeps them in LDS rather than in registers
  __shared__ double held_lds[2 * 10 * kBlock];
  ldbl* held = (ldbl*)held_lds;
  for_each_unit(L, [&](const March& M, const BoxRec& B) {
    const Geo g(B.n, B.ns);
    CProb* P = cprob(B.P);
    const gdbl* __restrict__ q = g.q(B.scr);
    gdbl* __restrict__ phiout = g.phi(B.scr);
    unsigned long long floors = 0;
    const int t = threadIdx.x;
    march(kCells1, B, M, [&](int i, int j, int k) {
      const int o = g.g(i, j, k), oh = g.h(i, j, k);
      const double phi = flatten_cell(g, q, o);
      Stencil S;
      Parab par[5];
      double v[5];
      // x, then y: both traced states parked in LDS
      trace_load<0>(g, q, o, S);
      trace_parab<0, LIM>(P, S, phi, par);
      trace_face<0, true>(P, par, S.sv[0][2], S.sv[1][2], S.cs, i, B.n[0], v, floors);
#pragma unroll
      for (int m = 0; m < 5; ++m) held[m * kBlock + t] = v[m];
      trace_face<0, false>(P, par, S.sv[0][2], S.sv[1][2], S.cs, i, B.n[0], v, floors);
#pragma unroll
      for (int m = 0; m < 5; ++m) held[(5 + m) * kBlock + t] = v[m];
      trace_load<1>(g, q, o, S);
      trace_parab<1, LIM>(P, S, phi, par);
      trace_face<1, true>(P, par, S.sv[0][2], S.sv[1][2], S.cs, j, B.n[1], v, floors);
#pragma unroll
      for (int m = 0; m < 5; ++m) held[(10 + m) * kBlock + t] = v[m];
      trace_face<1, false>(P, par, S.sv[0][2], S.sv[1][2], S.cs, j, B.n[1], v, floors);
#pragma unroll
      for (int m = 0; m < 5; ++m) held[(15 + m) * kBlock + t] = v[m];
      // z, the last loads: from here on the cell only stores
      trace_load<2>(g, q, o, S);
      trace_parab<2, LIM>(P, S, phi, par);
      double up[5], dn[5];
      trace_face<2, true>(P, par, S.sv[0][2], S.sv[1][2], S.cs, k, B.n[2], up, floors);
      trace_face<2, false>(P, par, S.sv[0][2], S.sv[1][2], S.cs, k, B.n[2], dn, floors);
      trace_store<2>(B, g, oh, up, dn);
      phiout[oh] = phi;
#pragma unroll
      for (int d = 0; d < 2; ++d) {
#pragma unroll
        for (int m = 0; m < 5; ++m) { up[m] = held[(10 * d + m) * kBlock + t]; dn[m] = held[(10 * d + 5 + m) * kBlock + t]; }
        if (d == 0) trace_store<0>(B, g, oh, up, dn);
        else trace_store<1>(B, g, oh, up, dn);
      }
      if (spec && g.ns > 0) species3<LIM, true>(B, g, P, o, oh, phi);
    });
    count(&B.P->cnt[2], floors);
  });
}

// The passive species of the merged tracing (TRACE) or of the merged
// method-of-lines face states in a kernel of their own (after k_trace3 or
// k_recon3, which stored the flattening coefficient): a thread takes its cell
// column through the unit's planes, kSpecPlanes at a time, species by
// species.  Along z it keeps the column's five stencil values in registers
// and shifts them by one plane per step (a rolling window), so each species
// value is loaded once per kSpecPlanes planes plus four halo planes, not
// once for every cell whose z stencil holds it; the flattening coefficient,
// velocities and sound speed of the planes are loaded once for all species.
// The arithmetic is species3's, value for value.
constexpr int kSpecPlanes = 4;
template <int LIM, bool TRACE>
__global__ __launch_bounds__(kBlock) void k_spec3(const Segs L) {
  // phi, u, v, w, c of each plane of a chunk, [plane][quantity][thread]
  __shared__ double hyd_lds[kSpecPlanes * 5 * kBlock];
  ldbl* hyd = (ldbl*)hyd_lds;
  for_each_unit(L, [&](const March& M, const BoxRec& B) {
    const Geo g(B.n, B.ns);
    if (g.ns == 0) return;
    CProb* P = cprob(B.P);
    int org[3], ext[3];
    region_of(kCells1, B.n, org, ext);
    const int t = threadIdx.x, it = M.start + t;
    if (it >= M.end) return;
    const int i = it % ext[0] + org[0];
    const int j = it / ext[0] + org[1];
    const gdbl* __restrict__ q = g.q(B.scr);
    const gdbl* __restrict__ phiv = g.phi(B.scr);
    const int gx = g.gx, gpl = g.gplane;
    for (int z0 = M.z0; z0 < M.z1; z0 += kSpecPlanes) {
      const int nz = min(kSpecPlanes, M.z1 - z0);
      const int o0 = g.g(i, j, z0), oh0 = g.h(i, j, z0);
      for (int p = 0; p < nz; ++p) {
        const int o = o0 + p * gpl;
        hyd[(5 * p) * kBlock + t] = phiv[oh0 + p * g.hplane];
        if (TRACE) {
#pragma unroll
          for (int d = 0; d < 3; ++d) hyd[(5 * p + 1 + d) * kBlock + t] = q[(1 + d) * g.gcomp + o];
          hyd[(5 * p + 4) * kBlock + t] = q[5 * g.gcomp + o];
        }
      }
      // a plane's loads: v[0] the value two planes up, v[1..4] the x
      // neighbours -2, -1, +1, +2, v[5..8] the y neighbours
      auto plane_loads = [&](const gdbl* a, int o, double v[9]) {
        v[0] = a[o + 2 * gpl];
        v[1] = a[o - 2]; v[2] = a[o - 1]; v[3] = a[o + 1]; v[4] = a[o + 2];
        v[5] = a[o - 2 * gx]; v[6] = a[o - gx]; v[7] = a[o + gx]; v[8] = a[o + 2 * gx];
      };
#pragma unroll 1
      for (int is = 0; is < g.ns; ++is) {
        const gdbl* a = q + (6 + is) * g.gcomp;
        // the z window at the first plane: values at z0-2, z0-1, z0, z0+1
        double w0 = a[o0 - 2 * gpl], w1 = a[o0 - gpl], w2 = a[o0], w3 = a[o0 + gpl];
        double cur[9], nxt[9];
        plane_loads(a, o0, cur);
#pragma unroll 1
        for (int p = 0; p < nz; ++p) {
          // the next plane's loads go out before this plane's stores
          if (p + 1 < nz) plane_loads(a, o0 + (p + 1) * gpl, nxt);
          const double phi = hyd[(5 * p) * kBlock + t], cs = TRACE ? hyd[(5 * p + 4) * kBlock + t] : 0.0;
          const Parab pr[3] = {ppm_l<LIM>(cur[1], cur[2], w2, cur[3], cur[4], phi),
                               ppm_l<LIM>(cur[5], cur[6], w2, cur[7], cur[8], phi),
                               ppm_l<LIM>(w0, w1, w2, w3, cur[0], phi)};
          const int oh = oh0 + p * g.hplane;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            double up = pr[d].aR, dn = pr[d].aL;  // method-of-lines edge values
            if (TRACE) {
              const double un = hyd[(5 * p + 1 + d) * kBlock + t], dtdx = P->dtdx[d];
              const double lm = un - cs, l0 = un, lp = un + cs;
              up = species_up(pr[d], lp, l0, fabs(lp) * dtdx, fabs(l0) * dtdx);
              dn = species_dn(pr[d], lm, l0, fabs(lm) * dtdx, fabs(l0) * dtdx);
            }
            gdbl* __restrict__ ql = g.ql(B.scr, d);
            gdbl* __restrict__ qr = g.qr(B.scr, d);
            __builtin_nontemporal_store(up, &ql[(kNV + is) * g.hcomp + oh + g.hstride(d)]);
            __builtin_nontemporal_store(dn, &qr[(kNV + is) * g.hcomp + oh]);
          }
          // shift the window one plane up
          w0 = w1; w1 = w2; w2 = w3; w3 = cur[0];
          if (p + 1 < nz) {
#pragma unroll
            for (int m = 0; m < 9; ++m) cur[m] = nxt[m];
          }
        }
      }
    }
  });
}

// Reflecting walls: the Riemann problem on a face that lies on a reflecting
// domain boundary takes the mirror image of the inside state as the outside
// one (normal velocity negated), so the wall lets no mass through.  Side of
// face fa along d of box B: 1 low wall (the left state is outside), 2 high
// wall (the right state is outside), 0 none.
CTU_DEV int wall_side(const BoxRec& B, int d, int fa) {
  if (fa == 0 && (B.wall[d] & 1)) return 1;
  if (fa == B.n[d] && (B.wall[d] & 2)) return 2;
  return 0;
}

// Permuted primitive states (slot 1 the normal velocity).
CTU_DEV void wall_mirror(int side, double L[5], double R[5]) {
  const bool lo = side == 1, hi = side == 2;
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const double l = L[m], r = R[m];
    L[m] = lo ? (m == 1 ? -r : r) : l;
    R[m] = hi ? (m == 1 ? -l : l) : r;
  }
}

// Normal flux of every face 0..n along D (cells -1..n across).  Along x and
// y the threads cover cells -1..n, so a wave writes whole rows (x) and whole
// planes (y): the slot of face -1, which nothing reads, takes zeros instead
// of leaving a partly written line in every row.
template <int D, int RS>
__global__ __launch_bounds__(kBlock) void k_riemann(const Segs L) {
  for_each_unit(L, [&](const March& M, const BoxRec& B) {
    CProb* P = cprob(B.P);
    const Geo g(B.n, B.ns);
    const gdbl* __restrict__ ql = g.ql(B.scr, D);
    const gdbl* __restrict__ qr = g.qr(B.scr, D);
    gdbl* __restrict__ fn = g.fn(B.scr, D);
    march(D == 2 ? kFace2 : kCells1, B, M, [&](int i, int j, int k) {
      const int o = g.h(i, j, k);
      const int fa = D == 0 ? i : (D == 1 ? j : k);
      if (fa < 0) {
        for (int m = 0; m < g.nv; ++m) fn[m * g.hcomp + o] = 0.0;
        return;
      }
      const int side = wall_side(B, D, fa);
      double L[5], R[5], f[5];
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        L[m] = ql[m * g.hcomp + o];
        R[m] = qr[m * g.hcomp + o];
      }
      wall_mirror(side, L, R);
      Wave W;
      rflux<RS>(L, R, P, f, W);
      store_flux<D>(fn, g.hcomp, o, f);
      for (int is = 0; is < g.ns; ++is) {
        const int mo = (kNV + is) * g.hcomp + o;
        const double xl = ql[mo], xr = qr[mo];
        fn[mo] = species_flux(W, side == 1 ? xr : xl, side == 2 ? xl : xr);
      }
    });
  });
}

// Permuted primitive (sweep along A) -> conserved, global component order.
template <int A>
CTU_DEV void to_cons(const double s[5], double rgm1, double U[5]) {
  const double rho = s[0];
  U[0] = rho;
  U[1 + A] = rho * s[1];
  U[1 + (A + 1) % 3] = rho * s[2];
  U[1 + (A + 2) % 3] = rho * s[3];
  U[4] = s[4] * rgm1 + 0.5 * rho * ((s[1] * s[1] + s[2] * s[2]) + s[3] * s[3]);
}

// Conserved -> permuted primitive of a sweep along A; keeps s0 (and returns 1)
// when the result has rho < small_dens or p < small_pres.
template <int A>
CTU_DEV int to_prim_or_keep(const double U[5], const double s0[5], double gm1, double sd, double sp,
                            double s[5]) {
  const double rho = U[0];
  const double un = U[1 + A] / rho, ut1 = U[1 + (A + 1) % 3] / rho, ut2 = U[1 + (A + 2) % 3] / rho;
  const double ke = 0.5 * rho * ((un * un + ut1 * ut1) + ut2 * ut2);
  const double p = gm1 * (U[4] - ke);
  if (rho < sd || p < sp) {
#pragma unroll
    for (int m = 0; m < 5; ++m) s[m] = s0[m];
    return 1;
  }
  s[0] = rho; s[1] = un; s[2] = ut1; s[3] = ut2; s[4] = p;
  return 0;
}

// Stage 1 at one face along A: the face states corrected by dt/(3 dx_B)
// times the normal B-flux difference across their owner cell, for B = the
// two other directions, then the Riemann flux -> F^{A|B}.  fb counts states
// that fell back to the uncorrected ones.  SP: the launch holds problems with
// species, whose face states are read once for both directions B after the
// hydro fluxes of both (without SP every problem of the launch has none).
template <int A, int RS, bool SP>
CTU_DEV void trans1_face(const BoxRec& B, const Geo& g, CProb* P, int i, int j, int k,
                         unsigned long long& fb) {
  const int sa = g.hstride(A);
  const gdbl* __restrict__ ql = g.ql(B.scr, A);
  const gdbl* __restrict__ qr = g.qr(B.scr, A);
  const int x[3] = {i, j, k};
  const int o = g.h(i, j, k);
  double sL[5], sR[5], UL[5], UR[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    // read once: streaming loads leave the L2 to the normal fluxes, which
    // the faces of the neighbouring plane read again
    sL[m] = __builtin_nontemporal_load(&ql[m * g.hcomp + o]);
    sR[m] = __builtin_nontemporal_load(&qr[m * g.hcomp + o]);
  }
  to_cons<A>(sL, P->rgm1, UL);
  to_cons<A>(sR, P->rgm1, UR);
  const int side = wall_side(B, A, x[A]);
  // what the species correction of each direction B needs from the hydro one
  bool on[2];
  Wave Ws[2];
  double rL[2], rR[2];
  int keepL[2], keepR[2];
#pragma unroll
  for (int which = 0; which < 2; ++which) {
    const int Bd = which == 0 ? (A + 1) % 3 : (A + 2) % 3;
    on[which] = x[Bd] >= 0 && x[Bd] < B.n[Bd];
    if (!on[which]) continue;
    const double c3 = P->dt3dx[Bd];
    const int sb = g.hstride(Bd);
    const gdbl* __restrict__ Fb = g.fn(B.scr, Bd);
    double VL[5], VR[5], tL[5], tR[5], f[5];
    const int oL = o - sa, oR = o;  // owner cells of the left and right states
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const gdbl* Fm = Fb + m * g.hcomp;
      VL[m] = UL[m] - c3 * (Fm[oL + sb] - Fm[oL]);
      VR[m] = UR[m] - c3 * (Fm[oR + sb] - Fm[oR]);
    }
    const int kL = to_prim_or_keep<A>(VL, sL, P->gm1, P->small_dens, P->small_pres, tL);
    const int kR = to_prim_or_keep<A>(VR, sR, P->gm1, P->small_dens, P->small_pres, tR);
    fb += kL + kR;
    wall_mirror(side, tL, tR);
    Wave W;
    rflux<RS>(tL, tR, P, f, W);
    gdbl* __restrict__ F1 = g.f1(B.scr, 2 * A + which);
    store_flux_nt<A>(F1, g.hcomp, o, f);
    if (SP) {
      Ws[which] = W;
      rL[which] = VL[0]; rR[which] = VR[0];
      keepL[which] = kL; keepR[which] = kR;
    }
  }
  if (!SP) return;
  // species: rho X corrected by the same flux differences as the density,
  // back to X with the corrected density (or the traced X where the state
  // fell back)
  const int oL = o - sa, oR = o;
  for (int is = 0; is < g.ns; ++is) {
    const int c = (kNV + is) * g.hcomp;
    const double xL = __builtin_nontemporal_load(&ql[c + o]), xR = __builtin_nontemporal_load(&qr[c + o]);
#pragma unroll
    for (int which = 0; which < 2; ++which) {
      if (!on[which]) continue;
      const int Bd = which == 0 ? (A + 1) % 3 : (A + 2) % 3;
      const double c3 = P->dt3dx[Bd];
      const int sb = g.hstride(Bd);
      const gdbl* Fm = g.fn(B.scr, Bd) + c;
      const double wL = sL[0] * xL - c3 * (Fm[oL + sb] - Fm[oL]);
      const double wR = sR[0] * xR - c3 * (Fm[oR + sb] - Fm[oR]);
      const double yL = keepL[which] ? xL : wL / rL[which], yR = keepR[which] ? xR : wR / rR[which];
      gdbl* __restrict__ F1 = g.f1(B.scr, 2 * A + which);
      __builtin_nontemporal_store(species_flux(Ws[which], side == 1 ? yR : yL, side == 2 ? yL : yR), &F1[c + o]);
    }
  }
}

// Stage 1 along A over faces 0..n (cells -1..n across).
template <int A, int RS>
__global__ __launch_bounds__(kBlock) void k_trans1(const Segs L) {
  for_each_unit(L, [&](const March& M, const BoxRec& B) {
    const Geo g(B.n, B.ns);
    unsigned long long fb = 0;
    march(kFace0 + A, B, M, [&](int i, int j, int k) { trans1_face<A, RS, true>(B, g, cprob(B.P), i, j, k, fb); });
    count(&B.P->cnt[3], fb);
  });
}

// Stage 1 along x, then y, then z, one thread per cell of -1..n (the lower
// A-face of the cell, where the cell is not at -1 along A): each normal flux
// array is read once instead of by two of the per-direction kernels.  SP as
// for trans1_face.
template <int RS, bool SP>
__global__ __launch_bounds__(kBlock) void k_trans1_all(const Segs L) {
  for_each_unit(L, [&](const March& M, const BoxRec& B) {
    const Geo g(B.n, B.ns);
    unsigned long long fb = 0;
    march(kCells1, B, M, [&](int i, int j, int k) {
      if (i >= 0) trans1_face<0, RS, SP>(B, g, cprob(B.P), i, j, k, fb);
      if (j >= 0) trans1_face<1, RS, SP>(B, g, cprob(B.P), i, j, k, fb);
      if (k >= 0) trans1_face<2, RS, SP>(B, g, cprob(B.P), i, j, k, fb);
    });
    count(&B.P->cnt[3], fb);
  });
}

// Stage 2 at one face along A: the face states corrected by dt/(2 dx_B)
// dF^{B|C} and then dt/(2 dx_C) dF^{C|B}, with (B, C) the cyclic successors of
// A, then the final HLLC flux (global component order).  fb counts states that
// fell back to the uncorrected ones.  Threads whose slot holds no face (on
// false) store zeros with the same store instructions.
template <int A, int RS>
CTU_DEV void final_flux(const BoxRec& B, const Geo& g, CProb* P, int o, int fa, bool on, gdbl* __restrict__ ff,
                        int& fb) {
  constexpr int Bd = (A + 1) % 3, Cd = (A + 2) % 3;
  // F^{B|C}: pair index 2B + (C == B+1 ? 0 : 1); F^{C|B}: 2C + (B == C+1 ? 0 : 1)
  constexpr int pbc = 2 * Bd + (Cd == (Bd + 1) % 3 ? 0 : 1);
  constexpr int pcb = 2 * Cd + (Bd == (Cd + 1) % 3 ? 0 : 1);
  const int sa = g.hstride(A), sb = g.hstride(Bd), sc = g.hstride(Cd);
  const gdbl* __restrict__ ql = g.ql(B.scr, A);
  const gdbl* __restrict__ qr = g.qr(B.scr, A);
  const gdbl* __restrict__ Fbc = g.f1(B.scr, pbc);
  const gdbl* __restrict__ Fcb = g.f1(B.scr, pcb);
  const double c2b = P->dt2dx[Bd];
  const double c2c = P->dt2dx[Cd];
  const int oL = o - sa, oR = o;
  const int side = wall_side(B, A, fa);
  double sL0 = 0.0, sR0 = 0.0, rL = 1.0, rR = 1.0, f[5] = {};
  int kL = 0, kR = 0;
  Wave W{};
  if (on) {
    double sL[5], sR[5], UL[5], UR[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      sL[m] = ql[m * g.hcomp + o];
      sR[m] = qr[m * g.hcomp + o];
    }
    to_cons<A>(sL, P->rgm1, UL);
    to_cons<A>(sR, P->rgm1, UR);
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const gdbl* F1 = Fbc + m * g.hcomp;
      const gdbl* F2 = Fcb + m * g.hcomp;
      UL[m] = UL[m] - c2b * (F1[oL + sb] - F1[oL]);
      UR[m] = UR[m] - c2b * (F1[oR + sb] - F1[oR]);
      UL[m] = UL[m] - c2c * (F2[oL + sc] - F2[oL]);
      UR[m] = UR[m] - c2c * (F2[oR + sc] - F2[oR]);
    }
    double tL[5], tR[5];
    kL = to_prim_or_keep<A>(UL, sL, P->gm1, P->small_dens, P->small_pres, tL);
    kR = to_prim_or_keep<A>(UR, sR, P->gm1, P->small_dens, P->small_pres, tR);
    fb += kL + kR;
    wall_mirror(side, tL, tR);
    rflux<RS>(tL, tR, P, f, W);
    sL0 = sL[0]; sR0 = sR[0]; rL = UL[0]; rR = UR[0];
  }
  store_flux<A>(ff, g.hcomp, o, f);
  for (int is = 0; is < g.ns; ++is) {
    const int c = (kNV + is) * g.hcomp;
    double v = 0.0;
    if (on) {
      const gdbl* F1 = Fbc + c;
      const gdbl* F2 = Fcb + c;
      const double xL = ql[c + o], xR = qr[c + o];
      double wL = sL0 * xL, wR = sR0 * xR;
      wL = wL - c2b * (F1[oL + sb] - F1[oL]);
      wR = wR - c2b * (F1[oR + sb] - F1[oR]);
      wL = wL - c2c * (F2[oL + sc] - F2[oL]);
      wR = wR - c2c * (F2[oR + sc] - F2[oR]);
      const double yL = kL ? xL : wL / rL, yR = kR ? xR : wR / rR;
      v = species_flux(W, side == 1 ? yR : yL, side == 2 ? yL : yR);
    }
    ff[c + o] = v;
  }
}

// Stage 2 along A over faces 0..n (cells 0..n-1 across): final fluxes; the
// threads cover whole rows (x over -1..n) and store zeros off the faces.
template <int A, int RS>
__global__ __launch_bounds__(kBlock) void k_trans2(const Segs L) {
  for_each_unit(L, [&](const March& M, const BoxRec& B) {
    CProb* P = cprob(B.P);
    const Geo g(B.n, B.ns);
    gdbl* __restrict__ ff = g.ff(B.scr, A);
    int fb = 0;
    const int ilast = A == 0 ? B.n[0] : B.n[0] - 1;  // last x index holding a face
    march(kFin0 + A, B, M, [&](int i, int j, int k) {
      final_flux<A, RS>(B, g, P, g.h(i, j, k), A == 0 ? i : (A == 1 ? j : k), i >= 0 && i <= ilast, ff, fb);
    });
    count(&B.P->cnt[3], (unsigned long long)fb);
  });
}

// Conservative update U^{n+1} = U^n + sum_d dt/dx_d (F_lo - F_hi) in the order
// x, y, z, the trapezoid gravity corrector on rho w then rho E, and the
// failure check (rho < small_dens, p < small_pres or a non-finite value).
__global__ __launch_bounds__(kBlock) void k_update(const Segs L) {
  for_each_unit(L, [&](const March& M, const BoxRec& B) {
    CProb* P = cprob(B.P);
    const Geo g(B.n, B.ns);
    const gdbl* __restrict__ U = gp(B.U[P->cur]);
    gdbl* __restrict__ Un = gp(B.U[P->cur ^ 1]);
    const gdbl* __restrict__ Fx = g.ff(B.scr, 0);
    const gdbl* __restrict__ Fy = g.ff(B.scr, 1);
    const gdbl* __restrict__ Fz = g.ff(B.scr, 2);
    const double dtdx = P->dtdx[0], dtdy = P->dtdx[1], dtdz = P->dtdx[2];
    const bool grav = P->grav_z != 0.0;
    const double hdtg = 0.5 * P->dt * P->grav_z;
    const bool forced = P->fail_step == P->nsteps;
    unsigned long long nbad = 0;
    march(kValid, B, M, [&](int i, int j, int k) {
      const int o = g.h(i, j, k), og = g.g(i, j, k);
      double un[5];
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        const int mo = m * g.hcomp + o;
        double du = dtdx * (Fx[mo] - Fx[mo + 1]);
        du = du + dtdy * (Fy[mo] - Fy[mo + g.hx]);
        du = du + dtdz * (Fz[mo] - Fz[mo + g.hplane]);
        un[m] = __builtin_nontemporal_load(&U[m * g.gcomp + og]) + du;  // read once here
      }
      if (grav) {
        un[3] = un[3] + hdtg * (U[og] + un[0]);
        un[4] = un[4] + hdtg * (U[3 * g.gcomp + og] + un[3]);
      }
      bool bad = false;
#pragma unroll
      for (int m = 0; m < 5; ++m) bad = bad || !isfinite(un[m]);
      if (un[0] < P->small_dens) bad = true;
      if (!bad) {
        const double uu = un[1] / un[0], vv = un[2] / un[0], ww = un[3] / un[0];
        const double ke = 0.5 * un[0] * ((uu * uu + vv * vv) + ww * ww);
        if (P->gm1 * (un[4] - ke) < P->small_pres) bad = true;
      }
      if (forced && i == 0 && j == 0 && k == 0) bad = true;  // host-set test hook
#pragma unroll
      for (int m = 0; m < 5; ++m) __builtin_nontemporal_store(un[m], &Un[m * g.gcomp + og]);  // read next step
      for (int m = kNV; m < g.nv; ++m) {
        const int mo = m * g.hcomp + o;
        double du = dtdx * (Fx[mo] - Fx[mo + 1]);
        du = du + dtdy * (Fy[mo] - Fy[mo + g.hx]);
        du = du + dtdz * (Fz[mo] - Fz[mo + g.hplane]);
        const double v = __builtin_nontemporal_load(&U[m * g.gcomp + og]) + du;
        bad = bad || !isfinite(v);
        __builtin_nontemporal_store(v, &Un[m * g.gcomp + og]);
      }
      nbad += bad ? 1ull : 0ull;
    });
    count(&B.P->cnt[4], nbad);
  });
}

// ------------------------------------------------------- method of lines
//
// The method-of-lines variant (the formulation of the paper's GPU proxy,
// section 4): the face states are the edge values of the same PPM parabolas,
// with no characteristic tracing and no transverse corrections; the normal
// HLLC fluxes (k_riemann) give the flux divergence, and a strong-stability-
// preserving Runge-Kutta method (Shu & Osher 1988) of order 2 or 3 advances
// the state, with a ghost fill before every stage.

// Method-of-lines face states of a cell along D: the edge values of its
// parabolas (the upper one the left state of the face above, the lower one
// the right state of the face below), floored; floors are counted only on
// the states of faces 0..n (xd the cell's index along D, nd the extent).
template <int D, int LIM>
CTU_DEV void recon_eval(CProb* P, const Stencil& S, double phi, int xd, int nd, double up[5], double dn[5],
                        unsigned long long& floors) {
  Parab par[5];
  trace_parab<D, LIM>(P, S, phi, par);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    up[m] = par[m].aR;
    dn[m] = par[m].aL;
  }
  const double sd = P->small_dens, sp = P->small_pres;
  const unsigned long long fu = xd <= nd - 1, fd = xd >= 0;
  if (up[0] < sd) { up[0] = sd; floors += fu; }
  if (up[4] < sp) { up[4] = sp; floors += fu; }
  if (dn[0] < sd) { dn[0] = sd; floors += fd; }
  if (dn[4] < sp) { dn[4] = sp; floors += fd; }
}

// The species edge values of a cell along D (the hydro flattening), stored
// unconditionally as the hydro states.
template <int D, int LIM>
CTU_DEV void recon_species(const BoxRec& B, const Geo& g, int o, int oh, double phi) {
  const gdbl* __restrict__ q = g.q(B.scr);
  gdbl* __restrict__ ql = g.ql(B.scr, D);
  gdbl* __restrict__ qr = g.qr(B.scr, D);
  const int st = g.gstride(D), sth = g.hstride(D);
  for (int is = 0; is < g.ns; ++is) {
    const gdbl* a = q + (6 + is) * g.gcomp + o;
    const Parab par = ppm_l<LIM>(a[-2 * st], a[-st], a[0], a[st], a[2 * st], phi);
    __builtin_nontemporal_store(par.aR, &ql[(kNV + is) * g.hcomp + oh + sth]);
    __builtin_nontemporal_store(par.aL, &qr[(kNV + is) * g.hcomp + oh]);
  }
}

// One thread per cell of -1..n: method-of-lines face states along D (the
// flattening coefficient from the flattening launch).  The loads come before
// the arithmetic and every store after it, unconditionally and streaming (the
// upper state of cell n and the lower state of cell -1 are never read).
template <int D, int LIM>
__global__ __launch_bounds__(kBlock) void k_recon(const Segs L) {
  for_each_unit(L, [&](const March& M, const BoxRec& B) {
    CProb* P = cprob(B.P);
    const Geo g(B.n, B.ns);
    const gdbl* __restrict__ q = g.q(B.scr);
    const gdbl* __restrict__ phiv = g.phi(B.scr);
    unsigned long long floors = 0;
    march(kCells1, B, M, [&](int i, int j, int k) {
      const int x[3] = {i, j, k};
      const int o = g.g(i, j, k), oh = g.h(i, j, k);
      const double phi = phiv[oh];
      Stencil S;
      double up[5], dn[5];
      trace_load<D, false>(g, q, o, S);
      recon_eval<D, LIM>(P, S, phi, x[D], B.n[D], up, dn, floors);
      trace_store<D>(B, g, oh, up, dn);
      if (g.ns > 0) recon_species<D, LIM>(B, g, o, oh, phi);
    });
    count(&B.P->cnt[2], floors);
  });
}

// One thread per cell of -1..n: the flattening coefficient (also stored, for
// stage dumps), then the method-of-lines face states along x, y and z from
// the same primitives, read once; the states of x and y wait in LDS until the
// loads of z have returned, as in the merged tracing.  spec = 0: the species
// are left to k_spec3.
template <int LIM>
__global__ __launch_bounds__(kBlock) void k_recon3(const Segs L, int spec) {
  __shared__ double held_lds[2 * 10 * kBlock];
  ldbl* held = (ldbl*)held_lds;
  for_each_unit(L, [&](const March& M, const BoxRec& B) {
    CProb* P = cprob(B.P);
    const Geo g(B.n, B.ns);
    const gdbl* __restrict__ q = g.q(B.scr);
    gdbl* __restrict__ phiout = g.phi(B.scr);
    unsigned long long floors = 0;
    const int t = threadIdx.x;
    march(kCells1, B, M, [&](int i, int j, int k) {
      const int o = g.g(i, j, k), oh = g.h(i, j, k);
      const double phi = flatten_cell(g, q, o);
      Stencil S;
      double up[5], dn[5];
      trace_load<0, false>(g, q, o, S);
      recon_eval<0, LIM>(P, S, phi, i, B.n[0], up, dn, floors);
#pragma unroll
      for (int m = 0; m < 5; ++m) { held[m * kBlock + t] = up[m]; held[(5 + m) * kBlock + t] = dn[m]; }
      trace_load<1, false>(g, q, o, S);
      recon_eval<1, LIM>(P, S, phi, j, B.n[1], up, dn, floors);
#pragma unroll
      for (int m = 0; m < 5; ++m) { held[(10 + m) * kBlock + t] = up[m]; held[(15 + m) * kBlock + t] = dn[m]; }
      trace_load<2, false>(g, q, o, S);
      recon_eval<2, LIM>(P, S, phi, k, B.n[2], up, dn, floors);
      trace_store<2>(B, g, oh, up, dn);
      phiout[oh] = phi;
#pragma unroll
      for (int d = 0; d < 2; ++d) {
#pragma unroll
        for (int m = 0; m < 5; ++m) { up[m] = held[(10 * d + m) * kBlock + t]; dn[m] = held[(10 * d + 5 + m) * kBlock + t]; }
        if (d == 0) trace_store<0>(B, g, oh, up, dn);
        else trace_store<1>(B, g, oh, up, dn);
      }
      if (spec && g.ns > 0) species3<LIM, false>(B, g, P, o, oh, phi);
    });
    count(&B.P->cnt[2], floors);
  });
}

// One Runge-Kutta stage: T = Us + dt L(Us), L(Us) the flux divergence of the
// normal fluxes (x, then y, then z) plus the gravity source g (0, 0, 0, rho,
// rho w) of Us; written as T, or as U0 + c (T - U0) with U0 the current fab
// (the convex combinations of the SSP methods, in a form that keeps a
// constant state exactly constant).  Failures are counted as in k_update.
__global__ __launch_bounds__(kBlock) void k_mol_update(const Segs L, int arr,
                                                       int out, int comb, double c, int last) {
  for_each_unit(L, [&](const March& M, const BoxRec& B) {
    CProb* P = cprob(B.P);
    const Geo g(B.n, B.ns);
    const gdbl* __restrict__ Us = gp(state_arr(B, arr));
    const gdbl* __restrict__ U0 = gp(B.U[P->cur]);
    gdbl* __restrict__ Un = gp(state_arr(B, out));
    const gdbl* __restrict__ Fx = g.fn(B.scr, 0);
    const gdbl* __restrict__ Fy = g.fn(B.scr, 1);
    const gdbl* __restrict__ Fz = g.fn(B.scr, 2);
    const double dtdx = P->dtdx[0], dtdy = P->dtdx[1], dtdz = P->dtdx[2];
    const bool grav = P->grav_z != 0.0;
    const double dtg = P->dt * P->grav_z;
    const bool forced = last && P->fail_step == P->nsteps;
    unsigned long long nbad = 0;
    march(kValid, B, M, [&](int i, int j, int k) {
      const int o = g.h(i, j, k), og = g.g(i, j, k);
      double t[5];
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        const int mo = m * g.hcomp + o;
        double du = dtdx * (Fx[mo] - Fx[mo + 1]);
        du = du + dtdy * (Fy[mo] - Fy[mo + g.hx]);
        du = du + dtdz * (Fz[mo] - Fz[mo + g.hplane]);
        t[m] = Us[m * g.gcomp + og] + du;
      }
      if (grav) {
        t[3] = t[3] + dtg * Us[og];
        t[4] = t[4] + dtg * Us[3 * g.gcomp + og];
      }
      if (comb) {
#pragma unroll
        for (int m = 0; m < 5; ++m) {
          const double a = U0[m * g.gcomp + og];
          t[m] = a + c * (t[m] - a);
        }
      }
      bool bad = false;
#pragma unroll
      for (int m = 0; m < 5; ++m) bad = bad || !isfinite(t[m]);
      if (t[0] < P->small_dens) bad = true;
      if (!bad) {
        const double uu = t[1] / t[0], vv = t[2] / t[0], ww = t[3] / t[0];
        const double ke = 0.5 * t[0] * ((uu * uu + vv * vv) + ww * ww);
        if (P->gm1 * (t[4] - ke) < P->small_pres) bad = true;
      }
      if (forced && i == 0 && j == 0 && k == 0) bad = true;  // host-set test hook
#pragma unroll
      for (int m = 0; m < 5; ++m) __builtin_nontemporal_store(t[m], &Un[m * g.gcomp + og]);
      for (int m = kNV; m < g.nv; ++m) {
        const int mo = m * g.hcomp + o;
        double du = dtdx * (Fx[mo] - Fx[mo + 1]);
        du = du + dtdy * (Fy[mo] - Fy[mo + g.hx]);
        du = du + dtdz * (Fz[mo] - Fz[mo + g.hplane]);
        double v = Us[m * g.gcomp + og] + du;
        if (comb) {
          const double a = U0[m * g.gcomp + og];
          v = a + c * (v - a);
        }
        bad = bad || !isfinite(v);
        __builtin_nontemporal_store(v, &Un[m * g.gcomp + og]);
      }
      nbad += bad ? 1ull : 0ull;
    });
    count(&B.P->cnt[4], nbad);
  });
}

// ------------------------------------------------------------- two levels
//
// Subcycled two-level advance (section 3.2: coarse advanced, fine advanced in
// steps to the same time, levels then synchronised), synchronised as in
// Berger & Colella (1989): a flux register replaces the coarse fluxes at the
// coarse-fine faces by the fine ones, covered coarse cells take the average of
// their eight children, and fine ghost cells come from the coarse state
// interpolated linearly in time and MC-linearly in space.

// Box-local item of a 3-D tag range.
CTU_DEV bool tag_item(const int ext[3], int t, int& a, int& b, int& c) {
  if (t >= ext[0] * ext[1] * ext[2]) return false;
  a = t % ext[0];
  const int r = t / ext[0];
  b = r % ext[1];
  c = r / ext[1];
  return true;
}

__global__ __launch_bounds__(kBlock) void k_gather(TwoLevelArgs A, const GatherTag* __restrict__ tags,
                                                   const Chunk* __restrict__ chunks, int n, int which) {
  const int rplane = A.rext[0] * A.rext[1], rcomp = rplane * A.rext[2];
  gdbl* __restrict__ dst = gp(which ? A.ct1 : A.ct0);
  for_each_chunk(n, [&](int c) {
    const Chunk ch = chunks[c];
    const GatherTag T = tags[ch.box];
    int a, b, cc;
    if (!tag_item(T.ext, ch.start + threadIdx.x, a, b, cc)) return;
    const BoxRec& B = A.cboxes[T.box];
    const Geo g(B.n, B.ns);
    const gdbl* __restrict__ U = gp(B.U[which ? (B.P->cur ^ 1) : B.P->cur]);
    const int so = g.g(T.lo[0] + a, T.lo[1] + b, T.lo[2] + cc);
    const int ro = (T.roff[2] + cc) * rplane + (T.roff[1] + b) * A.rext[0] + (T.roff[0] + a);
    for (int m = 0; m < g.nv; ++m) dst[m * rcomp + ro] = U[m * g.gcomp + so];
  });
}

__global__ __launch_bounds__(kBlock) void k_cfinterp(TwoLevelArgs A, const CfTag* __restrict__ tags,
                                                     const Chunk* __restrict__ chunks, int n, double theta) {
  const int rplane = A.rext[0] * A.rext[1], rcomp = rplane * A.rext[2];
  const double w0 = 1.0 - theta;
  for_each_chunk(n, [&](int c) {
    const Chunk ch = chunks[c];
    const CfTag T = tags[ch.box];
    int x[3];
    if (!tag_item(T.ext, ch.start + threadIdx.x, x[0], x[1], x[2])) return;
    const BoxRec& B = A.fboxes[T.box];
    const Geo g(B.n, B.ns);
    gdbl* __restrict__ U = gp(B.U[B.P->cur]);
    int I[3], rp[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      x[d] += T.lo[d];
      I[d] = B.lo[d] + x[d];          // global fine index (>= 0: the patch is interior)
      rp[d] = (I[d] >> 1) - A.rlo[d];  // parent's region index
    }
    const int po = (rp[2] * A.rext[1] + rp[1]) * A.rext[0] + rp[0];
    const int st[3] = {1, A.rext[0], rplane};
    const int go = g.g(x[0], x[1], x[2]);
    for (int m = 0; m < g.nv; ++m) {
      const gdbl* __restrict__ a0 = gp(A.ct0) + m * rcomp;
      const gdbl* __restrict__ a1 = gp(A.ct1) + m * rcomp;
      const double cpar = w0 * a0[po] + theta * a1[po];
      double val = cpar;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double um = w0 * a0[po - st[d]] + theta * a1[po - st[d]];
        const double up = w0 * a0[po + st[d]] + theta * a1[po + st[d]];
        const double sl = mc_slope(um, cpar, up);
        const double sgn = (I[d] & 1) ? 0.25 : -0.25;
        val = val + sgn * sl;
      }
      U[m * g.gcomp + go] = val;
    }
  });
}

__global__ void k_reg_coarse(TwoLevelArgs A, const RegFace* __restrict__ faces, int n) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n) return;
  const RegFace F = faces[f];
  const BoxRec& B = A.cboxes[F.cbox];
  const Geo g(B.n, B.ns);
  const gdbl* __restrict__ Ff = g.ff(B.scr, F.d);
  const int o = g.h(F.cface[0], F.cface[1], F.cface[2]);
  const double dt = A.Pc->dt;
  gdbl* r = gp(A.reg) + 2 * g.nv * f;
  for (int m = 0; m < g.nv; ++m) {
    r[m] = dt * Ff[m * g.hcomp + o];
    r[g.nv + m] = 0.0;
  }
}

__global__ void k_reg_fine(TwoLevelArgs A, const RegFace* __restrict__ faces, int n) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n) return;
  const RegFace F = faces[f];
  const BoxRec& B = A.fboxes[F.fbox];
  const Geo g(B.n, B.ns);
  const gdbl* __restrict__ Ff = g.ff(B.scr, F.d);
  const int t1 = F.d == 0 ? 1 : 0, t2 = F.d == 2 ? 1 : 2;  // transverse directions, increasing
  const int s1 = g.hstride(t1), s2 = g.hstride(t2);
  const int o = g.h(F.fface[0], F.fface[1], F.fface[2]);
  const double dt = A.Pf->dt;
  gdbl* r = gp(A.reg) + 2 * g.nv * f;
  for (int m = 0; m < g.nv; ++m) {
    const gdbl* Fm = Ff + m * g.hcomp;
    const double t00 = dt * Fm[o], t10 = dt * Fm[o + s1], t01 = dt * Fm[o + s2], t11 = dt * Fm[o + s1 + s2];
    r[g.nv + m] = r[g.nv + m] + ((t00 + t10) + (t01 + t11));
  }
}

__global__ __launch_bounds__(kBlock) void k_avgdown(TwoLevelArgs A, const AvgTag* __restrict__ tags,
                                                    const Chunk* __restrict__ chunks, int n) {
  for_each_chunk(n, [&](int c) {
    const Chunk ch = chunks[c];
    const AvgTag T = tags[ch.box];
    int a, b, cc;
    if (!tag_item(T.ext, ch.start + threadIdx.x, a, b, cc)) return;
    const BoxRec& C = A.cboxes[T.cbox];
    const BoxRec& Fb = A.fboxes[T.fbox];
    const Geo gc(C.n, C.ns), gf(Fb.n, Fb.ns);
    gdbl* __restrict__ Uc = gp(C.U[C.P->cur ^ 1]);
    const gdbl* __restrict__ Uf = gp(Fb.U[Fb.P->cur]);
    const int co = gc.g(T.clo[0] + a, T.clo[1] + b, T.clo[2] + cc);
    const int fo = gf.g(T.flo[0] + 2 * a, T.flo[1] + 2 * b, T.flo[2] + 2 * cc);
    const int sx = 1, sy = gf.gx, sz = gf.gplane;
    for (int m = 0; m < gc.nv; ++m) {
      const gdbl* f = Uf + m * gf.gcomp + fo;
      const double s0 = (f[0] + f[sx]) + (f[sy] + f[sx + sy]);
      const double s1 = (f[sz] + f[sx + sz]) + (f[sy + sz] + f[sx + sy + sz]);
      Uc[m * gc.gcomp + co] = 0.125 * (s0 + s1);
    }
  });
}

__global__ void k_reflux(TwoLevelArgs A, const RegFace* __restrict__ faces, int n) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n) return;
  const RegFace F = faces[f];
  const BoxRec& B = A.cboxes[F.cbox];
  const Geo g(B.n, B.ns);
  gdbl* __restrict__ U = gp(B.U[B.P->cur ^ 1]);
  const int o = g.g(F.ucell[0], F.ucell[1], F.ucell[2]);
  const double rdx = A.Pc->rdx[F.d];
  const gdbl* r = gp(A.reg) + 2 * g.nv * f;
  for (int m = 0; m < g.nv; ++m) {
    const double R = r[m] - 0.25 * r[g.nv + m];
    const double u = U[m * g.gcomp + o];
    U[m * g.gcomp + o] = F.side == 0 ? u + R * rdx : u - R * rdx;
  }
}

// ------------------------------------------------------------- regridding

// Tag a level-0 valid cell when its density jumps across it along some
// direction by more than `thr` relative to the two neighbours (ghosts filled).
__global__ __launch_bounds__(kBlock) void k_tag(const Segs L, double thr, unsigned char* __restrict__ tags, int dnx,
                                                int dny, int dlx, int dly, int dlz) {
  for_each_unit(L, [&](const March& M, const BoxRec& B) {
    const Geo g(B.n, B.ns);
    const gdbl* __restrict__ U = gp(B.U[B.P->cur]);
    march(kValid, B, M, [&](int i, int j, int k) {
      const int o = g.g(i, j, k);
      bool t = false;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int st = g.gstride(d);
        const double rp = U[o + st], rm = U[o - st];
        if (fabs(rp - rm) > thr * (rp + rm)) t = true;
      }
      const long long I = B.lo[0] + i - dlx, J = B.lo[1] + j - dly, K = B.lo[2] + k - dlz;
      tags[(K * dny + J) * dnx + I] = t ? 1 : 0;
    });
  });
}

// New fine state of a regrid: copy from the old fine level, or MC-linear
// interpolation from the gathered coarse region (the coarse-fine rule).
__global__ __launch_bounds__(kBlock) void k_prolong(TwoLevelArgs A, const BoxRec* __restrict__ newf,
                                                    const BoxRec* __restrict__ oldf,
                                                    const ProlongTag* __restrict__ tags,
                                                    const Chunk* __restrict__ chunks, int n) {
  const int rplane = A.rext[0] * A.rext[1], rcomp = rplane * A.rext[2];
  for_each_chunk(n, [&](int c) {
    const Chunk ch = chunks[c];
    const ProlongTag T = tags[ch.box];
    int x[3];
    if (!tag_item(T.ext, ch.start + threadIdx.x, x[0], x[1], x[2])) return;
    const BoxRec& B = newf[T.box];
    const Geo g(B.n, B.ns);
    gdbl* __restrict__ U = gp(B.U[0]);
    int I[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      x[d] += T.lo[d];
      I[d] = B.lo[d] + x[d];
    }
    const int go = g.g(x[0], x[1], x[2]);
    if (T.src >= 0) {
      const BoxRec& S = oldf[T.src];
      const Geo gs(S.n, S.ns);
      const gdbl* __restrict__ V = gp(S.U[S.P->cur]);
      const int so = gs.g(I[0] - S.lo[0], I[1] - S.lo[1], I[2] - S.lo[2]);
      for (int m = 0; m < g.nv; ++m) U[m * g.gcomp + go] = V[m * gs.gcomp + so];
      return;
    }
    int rp[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) rp[d] = (I[d] >> 1) - A.rlo[d];
    const int po = (rp[2] * A.rext[1] + rp[1]) * A.rext[0] + rp[0];
    const int st[3] = {1, A.rext[0], rplane};
    for (int m = 0; m < g.nv; ++m) {
      const gdbl* __restrict__ a0 = gp(A.ct0) + m * rcomp;
      const double cpar = a0[po];
      double val = cpar;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double sl = mc_slope(a0[po - st[d]], cpar, a0[po + st[d]]);
        const double sgn = (I[d] & 1) ? 0.25 : -0.25;
        val = val + sgn * sl;
      }
      U[m * g.gcomp + go] = val;
    }
  });
}

__global__ void k_dt2(ProbDev* Pc, ProbDev* Pf) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  unsigned long long bc = 0ull, bf = 0ull;
  for (int q = 0; q < kSlots; ++q) {
    bc = Pc->smax[q][0] > bc ? Pc->smax[q][0] : bc;
    bf = Pf->smax[q][0] > bf ? Pf->smax[q][0] : bf;
    Pc->smax[q][0] = 0ull;
    Pf->smax[q][0] = 0ull;
  }
  const double a = Pc->cfl / __longlong_as_double((long long)bc);
  const double b = 2.0 * (Pc->cfl / __longlong_as_double((long long)bf));
  const double dt = Pc->fixed_dt > 0.0 ? Pc->fixed_dt : (a < b ? a : b);
  set_dt(Pc, dt);
  set_dt(Pf, 0.5 * dt);
}

}  // namespace

// ---------------------------------------------------------------- launchers

const char* stage_name(int s) {
  static const char* names[kNumStages] = {
      "fill", "bc_x", "bc_y", "bc_z", "cons2prim_cfl", "cfl", "cons2prim", "dt", "flatten",
      "trace_x", "trace_y", "trace_z", "riemann_x", "riemann_y", "riemann_z",
      "trans1_x", "trans1_y", "trans1_z", "trans2_x", "trans2_y", "trans2_z", "update", "flip",
      "recon_x", "recon_y", "recon_z", "mol_update", "trace_xyz", "trans1_xyz", "recon_xyz", "species_xyz"};
  return (s >= 0 && s < kNumStages) ? names[s] : "?";
}

hipError_t launch_stage(int stage, const Launch& L) {
  const Segs& G = L.segs;
  if (G.n <= 0 || G.beg[G.n] <= 0) return hipSuccess;
  const dim3 grid(L.grid), block(kBlock);
  hipStream_t s = L.stream;
#define CTU_LIM(K, D)                                                        \
  (L.lim == 1   ? K<D, 1><<<grid, block, 0, s>>>(G)                          \
   : L.lim == 2 ? K<D, 2><<<grid, block, 0, s>>>(G)                          \
                : K<D, 0><<<grid, block, 0, s>>>(G))
  switch (stage) {
    case kStFill: k_fill<<<grid, block, 0, s>>>(G, L.arr); break;
    case kStBcX: k_bc<0><<<grid, block, 0, s>>>(G, L.arr); break;
    case kStBcY: k_bc<1><<<grid, block, 0, s>>>(G, L.arr); break;
    case kStBcZ: k_bc<2><<<grid, block, 0, s>>>(G, L.arr); break;
    case kStC2P: k_c2p<true, true><<<grid, block, 0, s>>>(G, L.arr); break;
    case kStCfl: k_c2p<false, true><<<grid, block, 0, s>>>(G, L.arr); break;
    case kStC2POnly: k_c2p<true, false><<<grid, block, 0, s>>>(G, L.arr); break;
    case kStReconX: CTU_LIM(k_recon, 0); break;
    case kStReconY: CTU_LIM(k_recon, 1); break;
    case kStReconZ: CTU_LIM(k_recon, 2); break;
    case kStMolUpdate: k_mol_update<<<grid, block, 0, s>>>(G, L.arr, L.out, L.comb, L.c, L.last); break;
#define CTU_LIM3(K)                                                         \
  (L.lim == 1   ? K<1><<<grid, block, 0, s>>>(G)                            \
   : L.lim == 2 ? K<2><<<grid, block, 0, s>>>(G)                            \
                : K<0><<<grid, block, 0, s>>>(G))
    case kStRecon3: {
      const int spec = L.spstage ? 0 : 1;
      if (L.lim == 1) k_recon3<1><<<grid, block, 0, s>>>(G, spec);
      else if (L.lim == 2) k_recon3<2><<<grid, block, 0, s>>>(G, spec);
      else k_recon3<0><<<grid, block, 0, s>>>(G, spec);
      break;
    }
    case kStFlatten: k_flatten<<<grid, block, 0, s>>>(G); break;
    case kStTraceX: CTU_LIM(k_trace, 0); break;
    case kStTraceY: CTU_LIM(k_trace, 1); break;
    case kStTraceZ: CTU_LIM(k_trace, 2); break;
    case kStTrace3: {
      // species go to k_spec3 when the species stage runs
      const int spec = L.spstage ? 0 : 1;
      if (L.lim == 1) k_trace3<1><<<grid, block, 0, s>>>(G, spec);
      else if (L.lim == 2) k_trace3<2><<<grid, block, 0, s>>>(G, spec);
      else k_trace3<0><<<grid, block, 0, s>>>(G, spec);
      break;
    }
    case kStSpec3:
      if (L.mol) {
        if (L.lim == 1) k_spec3<1, false><<<grid, block, 0, s>>>(G);
        else if (L.lim == 2) k_spec3<2, false><<<grid, block, 0, s>>>(G);
        else k_spec3<0, false><<<grid, block, 0, s>>>(G);
      } else {
        if (L.lim == 1) k_spec3<1, true><<<grid, block, 0, s>>>(G);
        else if (L.lim == 2) k_spec3<2, true><<<grid, block, 0, s>>>(G);
        else k_spec3<0, true><<<grid, block, 0, s>>>(G);
      }
      break;
#undef CTU_LIM3
    case kStT1All:
      if (L.sp) {
        if (L.rs) k_trans1_all<1, true><<<grid, block, 0, s>>>(G);
        else k_trans1_all<0, true><<<grid, block, 0, s>>>(G);
      } else {
        if (L.rs) k_trans1_all<1, false><<<grid, block, 0, s>>>(G);
        else k_trans1_all<0, false><<<grid, block, 0, s>>>(G);
      }
      break;
#define CTU_RS(K, D) (L.rs ? K<D, 1><<<grid, block, 0, s>>>(G) : K<D, 0><<<grid, block, 0, s>>>(G))
    case kStRiemX: CTU_RS(k_riemann, 0); break;
    case kStRiemY: CTU_RS(k_riemann, 1); break;
    case kStRiemZ: CTU_RS(k_riemann, 2); break;
    case kStT1X: CTU_RS(k_trans1, 0); break;
    case kStT1Y: CTU_RS(k_trans1, 1); break;
    case kStT1Z: CTU_RS(k_trans1, 2); break;
    case kStT2X: CTU_RS(k_trans2, 0); break;
    case kStT2Y: CTU_RS(k_trans2, 1); break;
    case kStT2Z: CTU_RS(k_trans2, 2); break;
#undef CTU_RS
    case kStUpdate: k_update<<<grid, block, 0, s>>>(G); break;
    default: return hipErrorInvalidValue;
  }
#undef CTU_LIM
  return hipGetLastError();
}

hipError_t launch_gather(const TwoLevelArgs& A, const GatherTag* tags, const Chunk* chunks, int n, int which,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_gather<<<(n + 7) / 8 * 8, kBlock, 0, s>>>(A, tags, chunks, n, which);
  return hipGetLastError();
}

hipError_t launch_cfinterp(const TwoLevelArgs& A, const CfTag* tags, const Chunk* chunks, int n, double theta,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_cfinterp<<<(n + 7) / 8 * 8, kBlock, 0, s>>>(A, tags, chunks, n, theta);
  return hipGetLastError();
}

hipError_t launch_reg_coarse(const TwoLevelArgs& A, const RegFace* faces, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_reg_coarse<<<(n + 255) / 256, 256, 0, s>>>(A, faces, n);
  return hipGetLastError();
}

hipError_t launch_reg_fine(const TwoLevelArgs& A, const RegFace* faces, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_reg_fine<<<(n + 255) / 256, 256, 0, s>>>(A, faces, n);
  return hipGetLastError();
}

hipError_t launch_avgdown(const TwoLevelArgs& A, const AvgTag* tags, const Chunk* chunks, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_avgdown<<<(n + 7) / 8 * 8, kBlock, 0, s>>>(A, tags, chunks, n);
  return hipGetLastError();
}

hipError_t launch_reflux(const TwoLevelArgs& A, const RegFace* faces, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_reflux<<<(n + 255) / 256, 256, 0, s>>>(A, faces, n);
  return hipGetLastError();
}

hipError_t launch_tag(const Segs& L, int grid, double threshold, unsigned char* tags, const int dn[3],
                      const int dlo[3], hipStream_t s) {
  if (L.n <= 0 || L.beg[L.n] <= 0) return hipSuccess;
  k_tag<<<grid, kBlock, 0, s>>>(L, threshold, tags, dn[0], dn[1], dlo[0], dlo[1], dlo[2]);
  return hipGetLastError();
}

hipError_t launch_prolong(const TwoLevelArgs& A, const BoxRec* newf, const BoxRec* oldf, const ProlongTag* tags,
                          const Chunk* chunks, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_prolong<<<(n + 7) / 8 * 8, kBlock, 0, s>>>(A, newf, oldf, tags, chunks, n);
  return hipGetLastError();
}

hipError_t launch_dt2(ProbDev* Pc, ProbDev* Pf, hipStream_t s) {
  k_dt2<<<1, 64, 0, s>>>(Pc, Pf);
  return hipGetLastError();
}

hipError_t launch_set_dt(ProbDev* Pc, ProbDev* Pf, const double* dt, hipStream_t s) {
  k_set_dt<<<1, 64, 0, s>>>(Pc, Pf, dt);
  return hipGetLastError();
}

hipError_t launch_dt(const Segs& L, hipStream_t s) {
  if (L.n <= 0) return hipSuccess;
  k_dt<<<1, 64, 0, s>>>(L);
  return hipGetLastError();
}

hipError_t launch_flip(const Segs& L, int guard, hipStream_t s) {
  if (L.n <= 0) return hipSuccess;
  k_flip<<<1, 64, 0, s>>>(L, guard);
  return hipGetLastError();
}

// ------------------------------------------------------ bandwidth probes
//
// What plain streaming reaches on this GPU, as the ceiling the stage kernels
// are measured against: grid-stride loops of 16-byte accesses (two doubles
// per lane), a copy (read + write), a read (summed per lane; the sum is stored
// only if it equals a value it never takes, so the loads stay) and a write.
namespace {
using v2 = double __attribute__((ext_vector_type(2)));
using gv2 = __attribute__((address_space(1))) v2;

__global__ __launch_bounds__(kBlock) void k_probe(int kind, const void* __restrict__ a, void* __restrict__ b,
                                                  long long n, double never) {
  const gv2* __restrict__ src = (const gv2*)a;
  gv2* __restrict__ dst = (gv2*)b;
  const long long stride = (long long)gridDim.x * blockDim.x;
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    if (kind == 0) {
      dst[i] = src[i];
    } else if (kind == 1) {
      const v2 v = src[i];
      acc += v.x + v.y;
    } else {
      dst[i] = v2{never, never};
    }
  }
  if (kind == 1 && acc == never) dst[0] = v2{acc, acc};
}
}  // namespace

hipError_t launch_probe(int kind, const void* src, void* dst, size_t bytes, int blocks, hipStream_t s) {
  k_probe<<<blocks, kBlock, 0, s>>>(kind, src, dst, (long long)(bytes / 16), -1.25e300);
  return hipGetLastError();
}

// ------------------------------------------------------ static stage scratch
//
// Stage scratch of ctuppm_step_static, for callers that cannot allocate: a
// file-scope device array every GPU the library runs on holds until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in for the symbol); the address hipGetSymbolAddress
// gives for the current device, taken once per device, is what the box
// records hold.
namespace {
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(int dev, void** ptr) {
  *ptr = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_static_ptr[dev] = p;
  }
  *ptr = g_static_ptr[dev];
  return hipSuccess;
}

}  // namespace ctu
